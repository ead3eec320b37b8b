// sans_host_math.hpp -- FP64 host set-up routines of the tracer.
#pragma once

namespace sans {
namespace host {

double normal_quantile(double u);
void schulz_table(double p, int M, double* out);
void gauss_legendre(int n, double* x, double* w);
void py_series(double phi, int nterms, double* c, double* abg);
double schulz_moment(double p, int k);
double mean_volume(int kind, const double size[3], double shell, double poly, int mask);

}  // namespace host
}  // namespace sans
