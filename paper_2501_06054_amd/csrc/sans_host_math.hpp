// sans_host_math.hpp -- FP64 host set-up routines of the tracer.
#pragma once

namespace sans {
namespace host {

double normal_quantile(double u);
void gauss_legendre(int n, double* x, double* w);
void py_series(double phi, int nterms, double* c, double* abg);
// Baxter's adhesive hard spheres (volume fraction eta, stickiness tau): his
// factor function on [0, 1] (units of the diameter) is the quadratic
// h x^2 + b x + c0; hbc[0..2] = h, b, c0.  ca[m], cb[m]: coefficients of k^(2m)
// in A(k) = 1 - 12 eta int Q cos(kx) and in B(k)/k = -12 eta int Q sin(kx)/k.
// False when the adhesion parameter has no real solution.
bool sticky_constants(double eta, double tau, int nterms, double* ca, double* cb, double* hbc);
double schulz_moment(double p, int k);
double positive_normal_quantile(double u, double p);
// Chebyshev coefficients (n of them, FP64) of the Percus-Yevick G(x)/x over
// x in [0, xmax] in the variable z = 2 (x/xmax)^2 - 1 (G/x is even in x).
void py_chebyshev(double phi, double xmax, int n, double* out);
// Inverse-CDF tables of the sizes, M knots (M even), equally spaced in
// t = -ln(2 min(u, 1 - u)) with step 32 ln 2 / (M/2 - 1): knot j < M/2 at
// u = e^(-j dt)/2, knot M/2 + j at u = 1 - e^(-j dt)/2 (the upper tail from
// its own probability).  table_tail(j, M) = e^(-j dt)/2.
double table_tail(int j, int M);
void positive_normal_table(int M, double p, double* out);
// The orientation's standard normal table: knots at u = (k + 1/2)/M.
void normal_table(int M, double* out);
double positive_normal_moment(double p, int k);
double size_moment(int poly_kind, double p, int k);
// Number-averaged particle volume; extra: the micelle's N and volumes.
double mean_volume(int kind, const double size[3], double shell, double poly, int mask, int poly_kind,
                   const double extra[4]);
// End caps of a barbell (barbell = true) or capped cylinder of radius R,
// length L, cap radius r >= R: the cap centre's distance from the particle
// centre, the lowest point t0 (in units of r, from the cap centre) where a cap
// meets the cylinder, and the volume of the two caps beyond the cylinder.
void cap_geometry(bool barbell, double R, double L, double r, double* zc, double* t0, double* vcaps);
// The caps' n-point Gauss-Legendre rule at unit size as FP32 arrays [3][n]:
// t_i in [t0, 1], r sqrt(1 - t_i^2) and 2 pi r^3 (1 - t_i^2) w_i (1 - t0)/2.
void cap_rule(bool barbell, double R, double L, double r, int n, float* out);
// The superball's nested n-point Gauss-Legendre rule at unit size, FP32
// [n + 3 n^2]: x_i in [0, 1]; then per (i, j) y_ij in [0, ym(x_i)], the
// half-height zm(x_i, y_ij) and the weight 8 (w_i/2)(ym(x_i) w_j/2).
void superball_rule(double p, int n, float* out);
inline int superball_rule_size(int n) { return n + 3 * n * n; }
double superball_volume(double R, double p);
// Hayter-Penfold structure factor: hard spheres of diameter sigma with
// beta U = uc (sigma/r) exp(-ks (r/sigma - 1)) outside the core, in the mean
// spherical approximation.  msa_solve: the direct correlation c(x) inside
// the core at x = i/1024, i = 0..1024 (cin, 1025 values; x in units of
// sigma); false when the iteration does not reach a physical solution
// (1 - rho c^ > 0 everywhere).  Solutions are cached by (eta, uc, ks).
constexpr int kMsaCin = 1025;
bool msa_solve(double eta, double uc, double ks, double* cin);
// S(K) and dK S'(K) at the n knots K_j = j dK, dK = kmax/(n - 1)
// (K = q sigma), interleaved (out: 2n floats), for cubic Hermite
// interpolation.
void msa_knots(const double* cin, double eta, double uc, double ks, double kmax, int n, float* out);

}  // namespace host
}  // namespace sans
