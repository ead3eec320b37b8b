// sans_host_math.cpp -- FP64 host-side set-up of the tracer: inverse-CDF
// tables, Gauss-Legendre nodes, the Percus-Yevick power series and the mean
// particle volume.  Runs once per model (not per neutron); the results are
// rounded to FP32 for the device.
#include "sans_host_math.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <tuple>
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

// G(x)/x from its power series (40 terms: at x = 12 the largest term is about
// 1.4e3 and the last below 1e-40, so FP64 keeps 1e-13), at Chebyshev-Gauss
// nodes in z, then the discrete Chebyshev transform.
void py_chebyshev(double phi, double xmax, int n, double* out)
{
    constexpr int kTerms = 40, kNodes = 64, kTab = 16;
    // cos(k theta_j) at the fixed nodes theta_j = pi (j + 1/2) / kNodes, for
    // k < kTab: computed once per process (a batch fits thousands of sets)
    struct CosTable {
        double c[kTab][kNodes];
        CosTable()
        {
            for (int k = 0; k < kTab; ++k)
                for (int j = 0; j < kNodes; ++j) c[k][j] = std::cos(k * (kPiH * (j + 0.5) / kNodes));
        }
    };
    static const CosTable tab;
    double c[kTerms], abg[3];
    py_series(phi, kTerms, c, abg);
    // the series at every node (Horner, all nodes in step)
    double f[kNodes], x2[kNodes];
    for (int j = 0; j < kNodes; ++j) {
        x2[j] = xmax * xmax * 0.5 * (tab.c[1][j] + 1.0);
        f[j] = 0.0;
    }
    for (int m = kTerms - 1; m >= 0; --m)
        for (int j = 0; j < kNodes; ++j) f[j] = f[j] * x2[j] + c[m];
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < kNodes; ++j) s += f[j] * (k < kTab ? tab.c[k][j] : std::cos(k * (kPiH * (j + 0.5) / kNodes)));
        out[k] = (k == 0 ? 1.0 : 2.0) * s / kNodes;
    }
}

// Adhesive hard spheres in the Percus-Yevick closure (Baxter): the adhesion
// parameter lambda is the smaller root of
// (eta/12) l^2 - (tau + eta/(1 - eta)) l + (1 + eta/2)/(1 - eta)^2 = 0; with
// mu = lambda eta (1 - eta) the factor function is
// Q(x) = a/2 (x^2 - 1) + b (x - 1) + lambda/12, a = (1 + 2 eta - mu)/(1 - eta)^2,
// b = (mu - 3 eta)/(2 (1 - eta)^2).  Its moments m_n = int_0^1 Q x^n dx give
// the power series of the transform's real and imaginary parts.
bool sticky_constants(double eta, double tau, int nterms, double* ca, double* cb, double* hbc)
{
    const double om = 1.0 - eta;
    const double qa = eta / 12.0, qb = tau + eta / om, qc = (1.0 + 0.5 * eta) / (om * om);
    const double disc = qb * qb - 4.0 * qa * qc;
    if (!(disc >= 0.0)) return false;
    // the smaller root, written without cancellation
    const double lam = 2.0 * qc / (qb + std::sqrt(disc));
    const double mu = lam * eta * om;
    const double a = (1.0 + 2.0 * eta - mu) / (om * om), b = (mu - 3.0 * eta) / (2.0 * om * om);
    const double h = 0.5 * a, c0 = lam / 12.0 - h - b;
    hbc[0] = h;
    hbc[1] = b;
    hbc[2] = c0;
    const double e = 12.0 * eta;
    double f = 1.0;  // n!
    for (int n = 0; n < 2 * nterms; ++n) {
        if (n > 0) f *= n;
        const double mom = h / (n + 3) + b / (n + 2) + c0 / (n + 1);
        const double sgn = ((n / 2) % 2) ? -1.0 : 1.0;
        if (n % 2 == 0) ca[n / 2] = (n == 0 ? 1.0 : 0.0) - e * sgn * mom / f;
        else cb[n / 2] = -e * sgn * mom / f;
    }
    return true;
}

// Superball |x|^2p + |y|^2p + |z|^2p <= 1: the transform is even in each
// coordinate, so 8 times the octant's; z is integrated exactly
// (sin(Q_C zm)/Q_C), x and y by Gauss-Legendre on [0, 1] and [0, ym(x)].
void superball_rule(double p, int n, float* out)
{
    std::vector<double> gx(n), gw(n);
    gauss_legendre(n, gx.data(), gw.data());
    const double e = 2.0 * p, ie = 1.0 / e;
    float* xs = out;
    float* ys = out + n;
    float* zs = ys + (size_t)n * n;
    float* ws = zs + (size_t)n * n;
    for (int i = 0; i < n; ++i) {
        const double x = 0.5 * (gx[i] + 1.0);
        const double xe = std::pow(x, e);
        const double ym = std::pow(1.0 - xe, ie);
        xs[i] = (float)x;
        for (int j = 0; j < n; ++j) {
            const double y = 0.5 * ym * (gx[j] + 1.0);
            const double rest = 1.0 - xe - std::pow(y, e);
            const size_t k = (size_t)i * n + j;
            ys[k] = (float)y;
            zs[k] = (float)(rest > 0.0 ? std::pow(rest, ie) : 0.0);
            ws[k] = (float)(8.0 * 0.5 * gw[i] * 0.5 * ym * gw[j]);
        }
    }
}

double superball_volume(double R, double p)
{
    const double g = std::tgamma(1.0 + 0.5 / p);
    return 8.0 * R * R * R * g * g * g / std::tgamma(1.0 + 1.5 / p);
}

// E[y^k] of the Schulz distribution: Gamma(a + k) / (Gamma(a) a^k), a = 1/p^2.
double schulz_moment(double p, int k)
{
    if (p <= 0.0 || k == 0) return 1.0;
    const double a = 1.0 / (p * p);
    return std::exp(std::lgamma(a + k) - std::lgamma(a) - k * std::log(a));
}

// The paper's size distribution (Methods, "Polydispersity and orientational
// distributions", Eq. (8)) restricted to positive sizes: N(1, p^2) on y > 0.
// Quantile: 1 + p Phi^-1(Phi(-1/p) + u (1 - Phi(-1/p))).
double positive_normal_quantile(double u, double p)
{
    const double c0 = 0.5 * std::erfc(1.0 / (p * std::sqrt(2.0)));
    return 1.0 + p * normal_quantile(c0 + u * (1.0 - c0));
}

double table_tail(int j, int M) { return 0.5 * std::exp(-j * (32.0 * std::log(2.0) / (M / 2 - 1))); }

void normal_table(int M, double* out)
{
    for (int k = 0; k < M; ++k) out[k] = normal_quantile((k + 0.5) / M);
}

// Upper half: 1 - u = v, so c0 + u (1 - c0) = 1 - v (1 - c0) and, the normal
// being symmetric, y = 1 - p Phi^-1(v (1 - c0)).
void positive_normal_table(int M, double p, double* out)
{
    const int H = M / 2;
    const double c0 = 0.5 * std::erfc(1.0 / (p * std::sqrt(2.0)));
    for (int j = 0; j < H; ++j) {
        const double v = table_tail(j, M);
        out[j] = positive_normal_quantile(v, p);
        out[H + j] = 1.0 - p * normal_quantile(v * (1.0 - c0));
    }
}

// E[y^k] of that distribution by composite Gauss-Legendre quadrature of
// y^k exp(-(y-1)^2 / 2p^2) over [max(0, 1 - 12p), 1 + 12p] (8 panels of 16
// nodes), divided by the same quadrature of the density.
double positive_normal_moment(double p, int k)
{
    if (p <= 0.0 || k == 0) return 1.0;
    double gx[16], gw[16];
    gauss_legendre(16, gx, gw);
    const double lo = std::max(0.0, 1.0 - 12.0 * p), hi = 1.0 + 12.0 * p;
    const int panels = 8;
    const double h = (hi - lo) / panels;
    double num = 0.0, den = 0.0;
    for (int j = 0; j < panels; ++j)
        for (int i = 0; i < 16; ++i) {
            const double y = lo + h * (j + 0.5 * (gx[i] + 1.0));
            const double d = (y - 1.0) / p;
            const double f = 0.5 * h * gw[i] * std::exp(-0.5 * d * d);
            num += f * std::pow(y, k);
            den += f;
        }
    return num / den;
}

double size_moment(int poly_kind, double p, int k)
{
    return poly_kind == 1 ? positive_normal_moment(p, k) : schulz_moment(p, k);
}

// E[prod_i (f[i][0] y^k_i + f[i][1])] for three factors: each product term
// of the expansion takes the moment of its total power of y.
static double expand_moment(const double f[3][2], const int k[3], int poly_kind, double poly)
{
    double total = 0.0;
    for (int pick = 0; pick < 8; ++pick) {
        double c = 1.0;
        int power = 0;
        for (int i = 0; i < 3; ++i) {
            const bool scaled = pick >> i & 1;
            c *= f[i][scaled ? 0 : 1];
            power += scaled ? k[i] : 0;
        }
        total += c * size_moment(poly_kind, poly, power);
    }
    return total;
}

// Number-averaged volume of the particle population.
double mean_volume(int kind, const double size[3], double shell, double poly, int mask, int poly_kind,
                   const double extra[4])
{
    const bool b0 = mask & 1, b1 = mask & 2, b2 = mask & 4;
    const double c43 = 4.0 / 3.0 * kPiH;
    switch (kind) {
    case 0:
        return c43 * size[0] * size[0] * size[0] * size_moment(poly_kind, poly, b0 ? 3 : 0);
    case 1: {
        // (y R + t)^3 expanded in powers of y
        const double r = size[0], t = shell;
        if (!b0) return c43 * (r + t) * (r + t) * (r + t);
        double v = 0.0;
        const double binom[4] = {1.0, 3.0, 3.0, 1.0};
        for (int j = 0; j <= 3; ++j)
            v += binom[j] * std::pow(r, j) * std::pow(t, 3 - j) * size_moment(poly_kind, poly, j);
        return c43 * v;
    }
    case 2:
        return kPiH * size[0] * size[0] * size[1] * size_moment(poly_kind, poly, (b0 ? 2 : 0) + (b1 ? 1 : 0));
    case 3:
        return c43 * size[0] * size[1] * size[2]
             * size_moment(poly_kind, poly, (b0 ? 1 : 0) + (b1 ? 1 : 0) + (b2 ? 1 : 0));
    case 4:
        return size[0] * size[1] * size[2]
             * size_moment(poly_kind, poly, (b0 ? 1 : 0) + (b1 ? 1 : 0) + (b2 ? 1 : 0));
    case 5:
    case 6: {
        // every length scales with y (mask 7), so V(y) = y^3 V(1)
        double zc, t0, vcaps;
        cap_geometry(kind == 5, size[0], size[1], size[2], &zc, &t0, &vcaps);
        const double v1 = kPiH * size[0] * size[0] * size[1] + vcaps;
        return v1 * size_moment(poly_kind, poly, mask == 7 ? 3 : 0);
    }
    case 7: {
        // wall thickness times the surface 2 (AB + BC + AC); face areas scale
        // with the product of their two edges' draws
        const int k0 = b0 ? 1 : 0, k1 = b1 ? 1 : 0, k2 = b2 ? 1 : 0;
        return 2.0 * shell
             * (size[0] * size[1] * size_moment(poly_kind, poly, k0 + k1)
                + size[1] * size[2] * size_moment(poly_kind, poly, k1 + k2)
                + size[0] * size[2] * size_moment(poly_kind, poly, k0 + k2));
    }
    case 8:
        // N chains, each a core block and a corona chain (not scaled by y)
        return extra[0] * (extra[1] + extra[2]);
    case 9: {
        // pi L ((R + t)^2 - R^2) = pi (L y^b1) (2 R t y^b0 + t^2)
        const int k0 = b0 ? 1 : 0, k1 = b1 ? 1 : 0;
        return kPiH * size[1]
             * (2.0 * size[0] * shell * size_moment(poly_kind, poly, k0 + k1)
                + shell * shell * size_moment(poly_kind, poly, k1));
    }
    case 10: {
        // the outer cylinder pi (R y^b0 + t)^2 (L y^b1 + 2 t_face)
        const double f[3][2] = {{size[0], shell}, {size[0], shell}, {size[1], 2.0 * extra[0]}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * expand_moment(f, k, poly_kind, poly);
    }
    case 11: {
        // the outer ellipsoid 4/3 pi prod (s_i y^b_i + t)
        const double f[3][2] = {{size[0], shell}, {size[1], shell}, {size[2], shell}};
        const int k[3] = {b0 ? 1 : 0, b1 ? 1 : 0, b2 ? 1 : 0};
        return c43 * expand_moment(f, k, poly_kind, poly);
    }
    case 41:
        return kPiH * size[0] * size[1] * size[2]
             * size_moment(poly_kind, poly, (b0 ? 1 : 0) + (b1 ? 1 : 0) + (b2 ? 1 : 0));
    case 42: {
        // the outer cylinder pi (R y^b0 + rim)^2 (L y^b1 + 2 t_face)
        const double f[3][2] = {{size[0], shell}, {size[0], shell}, {size[1], 2.0 * extra[0]}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * expand_moment(f, k, poly_kind, poly);
    }
    case 43: {
        // the core box and the six face slabs
        const int k0 = b0 ? 1 : 0, k1 = b1 ? 1 : 0, k2 = b2 ? 1 : 0;
        return size[0] * size[1] * size[2] * size_moment(poly_kind, poly, k0 + k1 + k2)
             + 2.0 * (extra[0] * size[1] * size[2] * size_moment(poly_kind, poly, k1 + k2)
                      + extra[1] * size[0] * size[2] * size_moment(poly_kind, poly, k0 + k2)
                      + extra[2] * size[0] * size[1] * size_moment(poly_kind, poly, k0 + k1));
    }
    case 44: {
        // the outer elliptic cylinder pi (R y^b0 + t)(x R y^b0 + t)(L y^b1 + 2 t_f)
        const double f[3][2] = {{size[0], shell}, {extra[2] * size[0], shell}, {size[1], 2.0 * extra[0]}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * expand_moment(f, k, poly_kind, poly);
    }
    case 56: {
        // core and belt pi (R y^b0 + t)(x R y^b0 + t) L y^b1, faces 2 pi x (R y^b0)^2 t_f
        const double f[3][2] = {{size[0], shell}, {extra[2] * size[0], shell}, {size[1], 0.0}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        const double g[3][2] = {{size[0], 0.0}, {extra[2] * size[0], 0.0}, {1.0, 0.0}};
        const int kg[3] = {b0 ? 1 : 0, b0 ? 1 : 0, 0};
        return kPiH * expand_moment(f, k, poly_kind, poly) + 2.0 * kPiH * extra[0] * expand_moment(g, kg, poly_kind, poly);
    }
    case 62: {
        // flexible elliptical cylinder: pi eps (R y^b0)^2 (L y^b1)
        const double f[3][2] = {{size[0], 0.0}, {size[0], 0.0}, {size[1], 0.0}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * extra[1] * expand_moment(f, k, poly_kind, poly);
    }
    case 63: {
        // flexible cylinder: pi (R y^b0)^2 (L y^b1)
        const double f[3][2] = {{size[0], 0.0}, {size[0], 0.0}, {size[1], 0.0}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * expand_moment(f, k, poly_kind, poly);
    }
    case 61: {
        // pringle: pi (R y^b0)^2 (t y^b1)
        const double f[3][2] = {{size[0], 0.0}, {size[0], 0.0}, {size[1], 0.0}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * expand_moment(f, k, poly_kind, poly);
    }
    case 45: {
        // one disk: pi R^2 (core + two layers)
        const double f[3][2] = {{size[0], 0.0}, {size[0], 0.0}, {size[1], 2.0 * shell}};
        const int k[3] = {b0 ? 1 : 0, b0 ? 1 : 0, b1 ? 1 : 0};
        return kPiH * expand_moment(f, k, poly_kind, poly);
    }
    case 46:
    case 47:
    case 48:
        return mean_volume(0, size, shell, poly, mask, poly_kind, extra);
    case 38:
        return mean_volume(0, size, shell, poly, mask, poly_kind, extra);
    case 39:
        return mean_volume(1, size, shell, poly, mask, poly_kind, extra);
    case 58:
        // pearl necklace: N pearls and N - 1 rods
        return extra[0] * c43 * size[0] * size[0] * size[0] * size_moment(poly_kind, poly, b0 ? 3 : 0)
             + (extra[0] - 1.0) * 0.25 * kPiH * size[2] * size[2] * size[1];
    case 57:
        // raspberry: the large sphere and its small ones
        return c43 * size[0] * size[0] * size[0] * size_moment(poly_kind, poly, b0 ? 3 : 0)
             + extra[0] * c43 * size[1] * size[1] * size[1];
    case 25:
    case 28:
        // fuzzy sphere: the sphere; linear pearls: n spheres
        return (kind == 28 ? extra[0] : 1.0) * c43 * size[0] * size[0] * size[0]
             * size_moment(poly_kind, poly, b0 ? 3 : 0);
    case 26: {
        // the shell (R y + t)^3 - (R y)^3 = 3 R^2 t y^2 + 3 R t^2 y + t^3
        const double r = size[0], t = shell;
        if (!b0) return c43 * ((r + t) * (r + t) * (r + t) - r * r * r);
        return c43 * (3.0 * r * r * t * size_moment(poly_kind, poly, 2) + 3.0 * r * t * t * size_moment(poly_kind, poly, 1)
                      + t * t * t);
    }
    case 27: {
        // n shells, one every shell + gap (monodisperse)
        double v = 0.0, ri = size[0];
        for (int k = 0; k < (int)extra[0]; ++k) {
            const double ro = ri + shell;
            v += c43 * (ro * ro * ro - ri * ri * ri);
            ri = ro + size[1];
        }
        return v;
    }
    case 13: case 14: case 15: case 16: case 17: case 18: case 19: case 20: case 21: case 22: case 23:
    case 24: case 29: case 30: case 31: case 32: case 33: case 34: case 35: case 36: case 37: case 40: case 49: case 50:
        return 1.0;  // shape-independent: no particles (the weight uses the cross-section)
    case 51:
        return superball_volume(size[0], extra[0]) * size_moment(poly_kind, poly, b0 ? 3 : 0);
    case 52: case 53: case 54: case 55: case 60:
        return 1.0;  // lamellae, adsorbed layers: the weight is per unit volume fraction
    case 12: {
        // the box minus its cavity (monodisperse)
        const double t2 = 2.0 * shell;
        return size[0] * size[1] * size[2] - (size[0] - t2) * (size[1] - t2) * (size[2] - t2);
    }
    }
    return 0.0;
}

void cap_geometry(bool barbell, double R, double L, double r, double* zc, double* t0, double* vcaps)
{
    // the cap sphere cuts the cylinder's end circle at height h = +-sqrt(r^2 - R^2)
    // below its centre: outside the cylinder for the barbell, inside otherwise
    const double h = std::sqrt(std::max(r * r - R * R, 0.0)) * (barbell ? 1.0 : -1.0);
    *zc = 0.5 * L + h;
    *t0 = -h / r;
    // each cap: pi r^3 times the integral of (1 - t^2) over [t0, 1]
    *vcaps = 2.0 * kPiH * r * r * r * ((1.0 - *t0) - (1.0 - *t0 * *t0 * *t0) / 3.0);
}

void cap_rule(bool barbell, double R, double L, double r, int n, float* out)
{
    double zc, t0, vcaps;
    cap_geometry(barbell, R, L, r, &zc, &t0, &vcaps);
    std::vector<double> gx(n), gw(n);
    gauss_legendre(n, gx.data(), gw.data());
    for (int i = 0; i < n; ++i) {
        const double t = 0.5 * (1.0 - t0) * gx[i] + 0.5 * (1.0 + t0);
        const double one_t2 = std::max(1.0 - t * t, 0.0);
        out[i] = (float)t;
        out[n + i] = (float)(r * std::sqrt(one_t2));
        out[2 * n + i] = (float)(2.0 * kPiH * r * r * r * one_t2 * gw[i] * 0.5 * (1.0 - t0));
    }
}

}  // namespace host
}  // namespace sans

namespace sans {
namespace host {

// ------------------------------------------------------------------ MSA
// Ornstein-Zernike with the mean spherical closure on a radial grid (units
// of sigma): x_i = i h, h = 1/1024, 0 < i < 65536; gamma = h - c iterated
// through c = -1 - gamma inside the core, -beta U outside (the mean of the
// two one-sided values at x = 1), its three-dimensional transform as a sine
// transform, gamma^ = rho c^2/(1 - rho c^), and back.  The sine transforms
// by a complex radix-2 FFT of the odd extension (length 2N).

namespace {

constexpr int kMsaIn = 1024;           // grid intervals inside the core
constexpr int kMsaN = 65536;           // grid points (to x = 64)

// In-place iterative radix-2 FFT (forward, e^{-2 pi i jk/n}), n a power of 2.
void fft_inplace(std::vector<std::complex<double>>& a, const std::vector<std::complex<double>>& tw)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const size_t step = n / len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * tw[k * step];
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

// out[j] = sum_{i=1}^{N-1} in[i] sin(pi i j / N), j = 1..N-1 (index j - 1).
struct Dst {
    int N;
    std::vector<std::complex<double>> tw, buf;
    explicit Dst(int n) : N(n), tw(n), buf(2 * (size_t)n)
    {
        for (int k = 0; k < n; ++k) tw[k] = std::polar(1.0, -M_PI * k / n);
    }
    void operator()(const std::vector<double>& in, std::vector<double>& out)
    {
        const size_t n2 = 2 * (size_t)N;
        buf[0] = buf[N] = 0.0;
        for (int i = 1; i < N; ++i) {
            buf[i] = in[i - 1];
            buf[n2 - i] = -in[i - 1];
        }
        fft_inplace(buf, tw);
        for (int j = 1; j < N; ++j) out[j - 1] = -0.5 * buf[j].imag();
    }
};

bool msa_solve_uncached(double eta, double uc, double ks, double* cin)
{
    const int N = kMsaN, M = N - 1;
    const double h = 1.0 / kMsaIn, L = N * h, rho = 6.0 * eta / M_PI, dk = M_PI / L;
    std::vector<double> x(M), K(M), u(M);
    for (int i = 0; i < M; ++i) {
        x[i] = (i + 1) * h;
        K[i] = (i + 1) * dk;
        u[i] = x[i] > 1.0 ? uc * std::exp(-ks * (x[i] - 1.0)) / x[i] : 0.0;
    }
    const int i1 = kMsaIn - 1;   // x = 1
    Dst dst(N);
    std::vector<double> c(M), t(M), ch(M), gh(M), gn(M);
    bool physical = true;
    // one pass gamma -> next gamma at the contact potential us * U_c; clears
    // `physical` when 1 - rho c^ <= 0 at some K
    auto step = [&](const std::vector<double>& g, double us, std::vector<double>& res) {
        for (int i = 0; i < M; ++i) c[i] = x[i] < 1.0 - 0.5 * h ? -1.0 - g[i] : -us * u[i];
        c[i1] = 0.5 * ((-1.0 - g[i1]) - us * uc);
        for (int i = 0; i < M; ++i) t[i] = x[i] * c[i];
        dst(t, ch);
        physical = true;
        for (int j = 0; j < M; ++j) {
            ch[j] *= 4.0 * M_PI * h / K[j];
            const double d = 1.0 - rho * ch[j];
            physical = physical && d > 0.0;
            gh[j] = K[j] * rho * ch[j] * ch[j] / d;
        }
        dst(gh, res);
        for (int i = 0; i < M; ++i) res[i] *= dk / (2.0 * M_PI * M_PI * x[i]);
    };
    // Anderson mixing over the last 6 differences (mixing 0.3) at one stage,
    // from the gamma in g; true once gamma moves by less than tol
    std::vector<double> f(M);
    auto anderson = [&](std::vector<double>& g, double us, double tol) {
        std::vector<std::vector<double>> hg, hf;
        const int m = 6;
        const double beta = 0.3;
        for (int it = 0; it < 400; ++it) {
            step(g, us, gn);
            if (!physical) return false;
            double err = 0.0;
            for (int i = 0; i < M; ++i) {
                f[i] = gn[i] - g[i];
                err = std::max(err, std::fabs(f[i]));
            }
            if (!std::isfinite(err)) return false;
            if (err < tol) {
                g = gn;
                return true;
            }
            hg.push_back(g);
            hf.push_back(f);
            if ((int)hg.size() > m) {
                hg.erase(hg.begin());
                hf.erase(hf.begin());
            }
            // least squares min |f - dF coef| over the differences of the
            // history, by modified Gram-Schmidt on the columns of dF (columns
            // nearly dependent on the earlier ones are dropped)
            const int nd = (int)hf.size() - 1;
            std::vector<std::vector<double>> Q;
            std::vector<int> col;
            std::vector<double> R((size_t)std::max(nd, 1) * std::max(nd, 1), 0.0);
            double r00 = 0.0;
            for (int a = 0; a < nd; ++a) {
                std::vector<double> v(M);
                for (int i = 0; i < M; ++i) v[i] = hf[a + 1][i] - hf[a][i];
                double n0 = 0.0;
                for (int i = 0; i < M; ++i) n0 += v[i] * v[i];
                r00 = std::max(r00, std::sqrt(n0));
                for (size_t b = 0; b < Q.size(); ++b) {
                    double d = 0.0;
                    for (int i = 0; i < M; ++i) d += Q[b][i] * v[i];
                    R[b * nd + a] = d;
                    for (int i = 0; i < M; ++i) v[i] -= d * Q[b][i];
                }
                double nv = 0.0;
                for (int i = 0; i < M; ++i) nv += v[i] * v[i];
                nv = std::sqrt(nv);
                if (!(nv > 1e-12 * r00)) continue;
                for (int i = 0; i < M; ++i) v[i] /= nv;
                R[Q.size() * nd + a] = nv;
                Q.push_back(std::move(v));
                col.push_back(a);
            }
            const int nk = (int)Q.size();
            std::vector<double> coef(std::max(nd, 1), 0.0);
            for (int b = 0; b < nk; ++b) {
                double d = 0.0;
                for (int i = 0; i < M; ++i) d += Q[b][i] * f[i];
                coef[col[b]] = d;
            }
            // R restricted to the kept columns is upper triangular
            for (int b = nk - 1; b >= 0; --b) {
                double v = coef[col[b]];
                for (int c2 = b + 1; c2 < nk; ++c2) v -= R[b * nd + col[c2]] * coef[col[c2]];
                coef[col[b]] = v / R[b * nd + col[b]];
            }
            for (int i = 0; i < M; ++i) {
                double v = g[i] + beta * f[i];
                for (int a = 0; a < nd; ++a)
                    v -= ((hg[a + 1][i] - hg[a][i]) + beta * (hf[a + 1][i] - hf[a][i])) * coef[a];
                g[i] = v;
            }
        }
        return false;
    };
    // continuation in the contact potential from the uncharged spheres:
    // stages U_c s / S, S = max(1, ceil U_c), to 1e-8 on the way and 1e-12
    // at the end
    std::vector<double> g(M, 0.0);
    const int stages = std::max(1, (int)std::ceil(uc));
    for (int s = 1; s <= stages; ++s)
        if (!anderson(g, (double)s / stages, s == stages ? 1e-12 : 1e-8)) return false;
    step(g, 1.0, gn);                 // c^ of the solution
    if (!physical) return false;
    // gamma(0) from its transform, the inside c on x = i/1024
    double g0 = 0.0;
    for (int j = 0; j < M; ++j) g0 += K[j] * gh[j];
    g0 *= dk / (2.0 * M_PI * M_PI);
    cin[0] = -1.0 - g0;
    for (int i = 1; i <= kMsaIn; ++i) cin[i] = -1.0 - g[i - 1];
    return true;
}

}  // namespace

bool msa_solve(double eta, double uc, double ks, double* cin)
{
    // solutions by (eta, U_c, kappa sigma): one solve serves every model
    // and experiment that shares them (at most 64 kept, then all dropped)
    static std::mutex mu;
    static std::map<std::tuple<double, double, double>, std::vector<double>> cache;
    const auto key = std::make_tuple(eta, uc, ks);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            if (it->second.empty()) return false;
            std::copy(it->second.begin(), it->second.end(), cin);
            return true;
        }
    }
    std::vector<double> v(kMsaIn + 1);
    const bool ok = msa_solve_uncached(eta, uc, ks, v.data());
    std::lock_guard<std::mutex> lock(mu);
    if (cache.size() >= 64) cache.clear();
    if (ok) {
        std::copy(v.begin(), v.end(), cin);
        cache[key] = std::move(v);
    } else {
        cache[key] = std::vector<double>();
    }
    return ok;
}

void msa_knots(const double* cin, double eta, double uc, double ks, double kmax, int n, float* out)
{
    // c^(K) = 4 pi / K int_0^1 x c(x) sin(K x) dx (Simpson) + the tail's
    // closed form T(K) = -4 pi U_c N / D, N = ks sin K + K cos K,
    // D = K (ks^2 + K^2); S = 1 / (1 - rho c^), S' = rho S^2 c^'
    const double h = 1.0 / kMsaIn, rho = 6.0 * eta / M_PI, dK = kmax / (n - 1);
    std::vector<double> wxc(kMsaIn + 1);
    for (int i = 0; i <= kMsaIn; ++i) {
        const double w = (i == 0 || i == kMsaIn) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        wxc[i] = w * h / 3.0 * (i * h) * cin[i];
    }
    for (int j = 0; j < n; ++j) {
        const double Kq = dK * j;
        double ch, dch;
        if (j == 0) {
            double m2 = 0.0;
            for (int i = 0; i <= kMsaIn; ++i) m2 += wxc[i] * (i * h);
            ch = 4.0 * M_PI * m2 - 4.0 * M_PI * uc * (1.0 / ks + 1.0 / (ks * ks));
            dch = 0.0;                 // c^ is even in K
        } else {
            double I = 0.0, J = 0.0;
            for (int i = 0; i <= kMsaIn; ++i) {
                const double xi = i * h;
                I += wxc[i] * std::sin(Kq * xi);
                J += wxc[i] * xi * std::cos(Kq * xi);
            }
            const double sK = std::sin(Kq), cK = std::cos(Kq);
            const double N = ks * sK + Kq * cK, dN = (ks + 1.0) * cK - Kq * sK;
            const double D = Kq * (ks * ks + Kq * Kq), dD = ks * ks + 3.0 * Kq * Kq;
            ch = 4.0 * M_PI * I / Kq - 4.0 * M_PI * uc * N / D;
            dch = 4.0 * M_PI * (J / Kq - I / (Kq * Kq)) - 4.0 * M_PI * uc * (dN * D - N * dD) / (D * D);
        }
        const double S = 1.0 / (1.0 - rho * ch);
        out[2 * j] = (float)S;
        out[2 * j + 1] = (float)(dK * rho * S * S * dch);
    }
}

}  // namespace host
}  // namespace sans
