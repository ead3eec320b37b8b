// sans_host_math.hpp -- FP64 host set-up routines of the tracer.
#pragma once

namespace sans {
namespace host {

double normal_quantile(double u);
void gauss_legendre(int n, double* x, double* w);
void py_series(double phi, int nterms, double* c, double* abg);
double schulz_moment(double p, int k);
double positive_normal_quantile(double u, double p);
double positive_normal_moment(double p, int k);
double size_moment(int poly_kind, double p, int k);
double mean_volume(int kind, const double size[3], double shell, double poly, int mask, int poly_kind);

}  // namespace host
}  // namespace sans
