// sans_host_math.cpp -- FP64 host-side set-up of the tracer: inverse-CDF
// tables, Gauss-Legendre nodes, the Percus-Yevick power series and the mean
// particle volume.  Runs once per model (not per neutron); the results are
// rounded to FP32 for the device.
#include "sans_host_math.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace sans {
namespace host {

static const double kPiH = 3.141592653589793238462643383;

// Standard normal quantile.  Start: Abramowitz & Stegun 26.2.23 (rational
// approximation, |error| < 4.5e-4); then Halley steps on
// Phi(y) - u = 0 with Phi(y) = erfc(-y/sqrt 2)/2, which converge cubically to
// full double precision.
double normal_quantile(double u)
{
    if (!(u > 0.0 && u < 1.0)) return std::nan("");
    const double m = u < 0.5 ? u : 1.0 - u;
    const double t = std::sqrt(-2.0 * std::log(m));
    double y = t - (2.515517 + 0.802853 * t + 0.010328 * t * t)
                 / (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t);
    if (u < 0.5) y = -y;
    for (int it = 0; it < 8; ++it) {
        const double e = 0.5 * std::erfc(-y / std::sqrt(2.0)) - u;
        const double d = e * std::sqrt(2.0 * kPiH) * std::exp(0.5 * y * y);
        const double step = d / (1.0 + 0.5 * y * d);
        y -= step;
        if (std::fabs(step) <= 1e-16 * std::max(1.0, std::fabs(y))) break;
    }
    return y;
}

// Schulz (Gamma, mean 1, relative width p) density.
static double schulz_pdf(double y, double a, double lnorm)
{
    if (y <= 0.0) return 0.0;
    return std::exp(lnorm + (a - 1.0) * std::log(y) - a * y);
}

// 16-point Gauss-Legendre rule on [-1, 1], built once.
static void gl16(double* x, double* w)
{
    static double sx[16], sw[16];
    static bool done = false;
    if (!done) {
        gauss_legendre(16, sx, sw);
        done = true;
    }
    for (int i = 0; i < 16; ++i) {
        x[i] = sx[i];
        w[i] = sw[i];
    }
}

static double integrate_pdf(double lo, double hi, double a, double lnorm)
{
    double x[16], w[16];
    gl16(x, w);
    const double h = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += w[i] * schulz_pdf(c + h * x[i], a, lnorm);
    return h * s;
}

// Schulz quantiles at (k + 1/2)/M.  The CDF is tabulated by integrating the
// density panel by panel (16-point Gauss-Legendre per panel) and each quantile
// is then refined inside its panel by safeguarded Newton steps on
// C(y_j) + int_{y_j}^{y} pdf - u = 0.
void schulz_table(double p, int M, double* out)
{
    const double a = 1.0 / (p * p);
    const double lnorm = a * std::log(a) - std::lgamma(a);
    const double ymax = 1.0 + 60.0 * p + 10.0 * p * p;
    const int P = 8192;
    const double dy = ymax / P;
    std::vector<double> cdf(P + 1, 0.0);
    for (int j = 0; j < P; ++j) cdf[j + 1] = cdf[j] + integrate_pdf(j * dy, (j + 1) * dy, a, lnorm);
    const double total = cdf[P];
    for (int k = 0; k < M; ++k) {
        const double u = (k + 0.5) / M * total;
        int j = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin()) - 1;
        j = std::min(std::max(j, 0), P - 1);
        double lo = j * dy, hi = (j + 1) * dy;
        double y = lo + (u - cdf[j]) / std::max(cdf[j + 1] - cdf[j], 1e-300) * dy;
        for (int it = 0; it < 60; ++it) {
            const double g = cdf[j] + integrate_pdf(j * dy, y, a, lnorm) - u;
            if (g > 0.0) hi = y; else lo = y;
            const double f = schulz_pdf(y, a, lnorm);
            double yn = (f > 0.0) ? y - g / f : 0.5 * (lo + hi);
            if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
            if (std::fabs(yn - y) <= 1e-16 * y) {
                y = yn;
                break;
            }
            y = yn;
        }
        out[k] = y;
    }
}

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton's method on
// P_n, evaluated by the Bonnet recurrence, from Tricomi's initial estimate.
void gauss_legendre(int n, double* x, double* w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        // i-th largest root
        const double th = kPiH * (4.0 * i + 3.0) / (4.0 * n + 2.0);
        double z = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th);
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double pm1 = 1.0, p = z;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2 * k - 1) * z * p - (k - 1) * pm1) / k;
                pm1 = p;
                p = pk;
            }
            if (n == 1) {
                p = z;
                pm1 = 1.0;
            }
            dp = n * (pm1 - z * p) / (1.0 - z * z);
            const double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16) break;
        }
        double pm1 = 1.0, p = z;
        for (int k = 2; k <= n; ++k) {
            const double pk = ((2 * k - 1) * z * p - (k - 1) * pm1) / k;
            pm1 = p;
            p = pk;
        }
        if (n == 1) pm1 = 1.0;
        dp = n * (pm1 - z * p) / (1.0 - z * z);
        const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        x[n - 1 - i] = z;
        w[n - 1 - i] = wt;
        x[i] = -z;
        w[i] = wt;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// G(x)/x of the Percus-Yevick solution as a power series.  G(x) is the sine
// transform int_0^1 (alpha s + beta s^2 + gamma s^4) sin(x s) ds of the
// direct correlation function; expanding sin termwise gives
//   G(x)/x = sum_m (-1)^m x^(2m) / (2m+1)! [alpha/(2m+3) + beta/(2m+4) + gamma/(2m+6)].
void py_series(double phi, int nterms, double* c, double* abg)
{
    const double om = 1.0 - phi;
    const double om4 = om * om * om * om;
    const double alpha = (1.0 + 2.0 * phi) * (1.0 + 2.0 * phi) / om4;
    const double beta = -6.0 * phi * (1.0 + 0.5 * phi) * (1.0 + 0.5 * phi) / om4;
    const double gamma = 0.5 * phi * alpha;
    abg[0] = alpha;
    abg[1] = beta;
    abg[2] = gamma;
    double f = 1.0;  // (2m+1)!
    for (int m = 0; m < nterms; ++m) {
        if (m > 0) f *= (2.0 * m) * (2.0 * m + 1.0);
        const double sgn = (m % 2) ? -1.0 : 1.0;
        c[m] = sgn / f * (alpha / (2 * m + 3) + beta / (2 * m + 4) + gamma / (2 * m + 6));
    }
}

// E[y^k] of the Schulz distribution: Gamma(a + k) / (Gamma(a) a^k), a = 1/p^2.
double schulz_moment(double p, int k)
{
    if (p <= 0.0 || k == 0) return 1.0;
    const double a = 1.0 / (p * p);
    return std::exp(std::lgamma(a + k) - std::lgamma(a) - k * std::log(a));
}

// Number-averaged volume of the particle population.
double mean_volume(int kind, const double size[3], double shell, double poly, int mask)
{
    const bool b0 = mask & 1, b1 = mask & 2, b2 = mask & 4;
    const double c43 = 4.0 / 3.0 * kPiH;
    switch (kind) {
    case 0:
        return c43 * size[0] * size[0] * size[0] * schulz_moment(poly, b0 ? 3 : 0);
    case 1: {
        // (y R + t)^3 expanded in powers of y
        const double r = size[0], t = shell;
        if (!b0) return c43 * (r + t) * (r + t) * (r + t);
        double v = 0.0;
        const double binom[4] = {1.0, 3.0, 3.0, 1.0};
        for (int j = 0; j <= 3; ++j)
            v += binom[j] * std::pow(r, j) * std::pow(t, 3 - j) * schulz_moment(poly, j);
        return c43 * v;
    }
    case 2:
        return kPiH * size[0] * size[0] * size[1] * schulz_moment(poly, (b0 ? 2 : 0) + (b1 ? 1 : 0));
    case 3:
        return c43 * size[0] * size[1] * size[2]
             * schulz_moment(poly, (b0 ? 1 : 0) + (b1 ? 1 : 0) + (b2 ? 1 : 0));
    case 4:
        return size[0] * size[1] * size[2]
             * schulz_moment(poly, (b0 ? 1 : 0) + (b1 ? 1 : 0) + (b2 ? 1 : 0));
    }
    return 0.0;
}

}  // namespace host
}  // namespace sans
