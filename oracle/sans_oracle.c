/*
 * sans_oracle.c -- plain FP64 CPU oracle of the SANS sample tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, nowhere else.  The
 * product (the HIP library) never links, loads or calls it, and the two share
 * no code, header, table or constant generator: everything here is written
 * out again from the paper and from textbook definitions.
 *
 * What it computes (arXiv 2501.06054, "Small Angle Neutron Scattering in
 * McStas: optimization for high throughput virtual experiments"):
 *   - each neutron is independent and scatters at most once inside the sample
 *     (Introduction; Methods, "Acceleration schemes": the problem is
 *     embarrassingly parallel and split scatter-gather over workers);
 *   - the per-event intensity is I = n (drho)^2 V^2 P(Q) S(Q), Eq. (3), built
 *     from the scattering amplitude A(Q) of Eq. (1) with |A|^2 as in Eqs. (2)
 *     and (4); the amplitude depends on |Q| (Eq. (5)), on (Q_A, Q_B, Q_C)
 *     (Eq. (6)) or on (Q_AB, Q_C) (Eq. (7)); cylinder amplitude Eq. (9);
 *   - size and orientation are redrawn at every scattering event from the
 *     configured distributions (Methods, "Polydispersity and orientational
 *     distributions");
 *   - detector tallies are summed in FP64 (atomic, thread-locked updates in
 *     the paper's GPU scheme; here: one private detector per thread merged in
 *     a fixed order, the paper's scatter-gather).
 * Where the paper is silent (instrument, weight, random generator, tables,
 * Schulz distribution, hard-sphere S(Q)) the readings are the ones recorded in
 * the design notes of the repository; each function says which one it takes.
 *
 * Precision: FP64 throughout, compiled with -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_MAX_QUAD 512

/* ------------------------------------------------------------------------ */
/* Parameters.  Own layout (not the product's).  Geometry in metres, sample
 * in Angstrom; angles in radians.                                          */
typedef struct {
    int32_t kind;          /* 0 sphere, 1 core-shell sphere, 2 cylinder,
                              3 triaxial ellipsoid, 4 parallelepiped,
                              5 barbell, 6 capped cylinder,
                              7 hollow rectangular prism with thin walls,
                              8 polymer micelle (isotropic), 9 hollow
                              cylinder, 10 core-shell cylinder, 11 core-shell
                              ellipsoid, 12 hollow prism with thick walls;
                              shape-independent (isotropic, I(q) in 1/cm
                              with I(0) = extra[0]): 13 Guinier, 14
                              Ornstein-Zernike, 15 Debye-Anderson-Brumberger,
                              16 Gaussian coil, 17 polydisperse Gaussian
                              coil, 18 Teubner-Strey, 19 power law, 20
                              Gaussian peak, 21 Lorentzian peak, 22 mass
                              fractal, 23 star polymer, 24 Gauss-Lorentz gel;
                              isotropic particles: 25 fuzzy sphere, 26
                              vesicle, 27 multilayer vesicle, 28 linear
                              pearls; shape-independent: 29 surface fractal,
                              30 two power law, 31 Guinier-Porod, 32
                              spinodal, 33 Porod, 34 line, 35 two
                              Lorentzians, 36 correlation length, 37 broad
                              peak, 40 polymer with excluded volume;
                              fractal aggregates of spheres: 38 homogeneous,
                              39 core-shell; oriented: 41 elliptical
                              cylinder, 42 core-shell bicelle, 43 core-shell
                              parallelepiped, 44 elliptical core-shell
                              bicelle, 45 stacked disks, 46 simple cubic,
                              47 body-centred, 48 face-centred cubic
                              paracrystals of spheres; shape-independent:
                              49 mass-surface fractal, 50 gel (fractal
                              network plus frozen inhomogeneities);
                              oriented: 51 superball; randomly oriented
                              lamellae: 52 bilayers with head and tail
                              groups, 53 stacks with Caille fluctuations,
                              54 head-tail bilayers in Caille stacks, 55
                              paracrystalline stacks; oriented: 56
                              elliptical bicelle with a belt and rough
                              interfaces; 57 raspberry, 58 pearl necklace
                              (isotropic); 59 binary hard spheres (two
                              sizes with their Percus-Yevick partial
                              structure factors); 60 adsorbed layers on
                              large particles; oriented: 61 pringle (a
                              saddle-shaped plate)                          */
    int32_t mode;          /* 0 Monte Carlo draws, 1 exact quadrature average */
    double size[3];        /* sphere R | core R | cyl R,L | ell a,b,c | par A,B,C |
                              barbell / capped cylinder: R, L, cap radius r >= R |
                              hollow prism: outer edges A, B, C |
                              micelle: core radius, corona chain Rg |
                              hollow cylinder: bore radius, length |
                              core-shell cylinder: core R, core length |
                              core-shell ellipsoid: core semi-axes |
                              thick hollow prism: outer edges              */
    double shell;          /* core-shell shell thickness; hollow prism wall   */
    double sld[3];         /* particle (core), shell, solvent                */
    double phi;            /* particle volume fraction, n = phi/<V>          */
    double sq_phi;         /* hard-sphere volume fraction; 0 -> S = 1        */
    double sq_radius;      /* hard-sphere radius                             */
    double poly;           /* relative width sigma/mean; 0 -> none           */
    int32_t poly_mask;     /* bit k: size[k] is scaled by the size draw      */
    int32_t orient_kind;   /* 0 fixed, 1 gaussian, 2 isotropic, 3 uniform angles */
    double orient_mean[3]; /* theta, phi, Psi                                */
    double orient_sigma[3];
    double src_w, src_h, src_z;
    double slit_w, slit_h, slit_z;
    double lambda0, dlambda_rel, cone_alpha;
    double sample_w, sample_h, sample_d;
    double det_w, det_h, det_z;
    int32_t nx, ny;
    int32_t table_size;    /* inverse-CDF knots (M)                          */
    int32_t quad_n;        /* Gauss-Legendre order of the exact average      */
    int32_t poly_kind;     /* size distribution: 0 Schulz, 1 Gaussian kept
                              only where the size is positive                */
    int32_t sq_kind;       /* structure factor when sq_phi > 0: 0 hard
                              spheres (Percus-Yevick), 1 adhesive hard spheres
                              (Baxter), 2 square-well (mean spherical)     */
    double extra[4];       /* micelle: aggregation number N, core-block and
                              corona-chain volumes (A^3), penetration d;
                              core-shell cylinder: extra[0] = end-face shell */
    double sq_extra[2];    /* adhesive spheres: stickiness tau; square well:
                              depth (kT) and width (in diameters)           */
    double mu_att;         /* attenuation coefficient of the sample (1/m);
                              0 -> none                                     */
    double poly_sep[3];    /* independent relative widths (Methods,
                              "Polydispersity ...", Eq. (8)): size[k] times
                              its own draw y_k ~ N(1, poly_sep[k]^2) kept
                              where positive; 0 -> size[k] fixed            */
    double guide[9];       /* straight guide upstream of the source aperture:
                              length (m; 0 -> none), width, height, gap from
                              its exit to the aperture (m), supermirror m,
                              R0, Qc (1/A), alpha (A), W (1/A)              */
} orc_params;

/* Surrogate mode (mode 2): a network replaces the exact average; set with
 * orc_set_surrogate.  Defined at the end of the file. */
static double surrogate_f2(const orc_params* p, double q, int* in_domain);

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box; the two key
 * words are advanced by the Weyl constants before every round but the first. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The random block b of neutron i in experiment e: counter (lo i, hi i, b, e),
 * key (lo seed, hi seed). */
static void neutron_block(uint64_t seed, uint64_t i, uint32_t b, uint32_t e, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), b, e};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Raw streams for tests: out[(j*nblocks + b)*4 + w] for neutron first+j. */
void orc_philox_stream(uint64_t seed, uint64_t first, uint64_t n, uint32_t nblocks,
                       uint32_t exp_id, uint32_t* out)
{
    for (uint64_t j = 0; j < n; ++j)
        for (uint32_t b = 0; b < nblocks; ++b)
            neutron_block(seed, first + j, b, exp_id, out + (j * nblocks + b) * 4);
}

/* u = (x + 1/2) 2^-32, an exact FP64 value strictly inside (0, 1). */
double orc_uniform(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

/* ------------------------------------------------------------------------ */
/* Inverse cumulative distributions. */

/* Standard normal CDF from the complementary error function. */
static double normal_cdf(double y) { return 0.5 * erfc(-y / sqrt(2.0)); }

/* Standard normal quantile: bisection of normal_cdf(y) = u (slow, plain). */
double orc_normal_quantile(double u)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (normal_cdf(mid) < u) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Regularised lower incomplete gamma P(a, x).  Series (Abramowitz & Stegun
 * 6.5.29) below x = a + 1, otherwise 1 - Q with Q from Legendre's continued
 * fraction (A&S 6.5.31) evaluated by the modified Lentz method. */
double orc_gamma_p(double a, double x)
{
    if (x <= 0.0) return 0.0;
    double lpre = a * log(x) - x - lgamma(a);
    if (x < a + 1.0) {
        double term = 1.0 / a, sum = term;
        for (int n = 1; n < 1000000; ++n) {
            term *= x / (a + n);
            sum += term;
            if (fabs(term) < fabs(sum) * 1e-17) break;
        }
        return sum * exp(lpre);
    }
    const double tiny = 1e-300;
    double b = x + 1.0 - a;
    double c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int n = 1; n < 1000000; ++n) {
        double an = -n * (n - a);
        b += 2.0;
        d = an * d + b;
        if (fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return 1.0 - exp(lpre) * h;
}

/* Regularised upper incomplete gamma Q(a, x) = 1 - P(a, x), computed
 * directly (Legendre's continued fraction) where it is small, so that the
 * far upper tail keeps its relative precision. */
double orc_gamma_q(double a, double x)
{
    if (x <= 0.0) return 1.0;
    if (x < a + 1.0) return 1.0 - orc_gamma_p(a, x);
    double lpre = a * log(x) - x - lgamma(a);
    const double tiny = 1e-300;
    double b = x + 1.0 - a;
    double c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int n = 1; n < 1000000; ++n) {
        double an = -n * (n - a);
        b += 2.0;
        d = an * d + b;
        if (fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return exp(lpre) * h;
}

/* Schulz distribution of the relative size y (mean 1, relative width p):
 * y ~ Gamma(shape a = 1/p^2, scale 1/a), i.e. z = 1/p^2 - 1 in the usual
 * Schulz notation.  Quantile by bisection of P(a, a*y) = u. */
double orc_schulz_quantile(double u, double p)
{
    double a = 1.0 / (p * p);
    double lo = 0.0, hi = 1.0;
    while (orc_gamma_p(a, a * hi) < u) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (orc_gamma_p(a, a * mid) < u) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* The Schulz size whose upper tail holds probability v: bisection of
 * Q(a, a*y) = v. */
double orc_schulz_quantile_upper(double v, double p)
{
    double a = 1.0 / (p * p);
    double lo = 0.0, hi = 1.0;
    while (orc_gamma_q(a, a * hi) > v) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (orc_gamma_q(a, a * mid) > v) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* The paper's size distribution (Methods, "Polydispersity and orientational
 * distributions", Eq. (8)): y ~ N(1, p^2), redrawn until positive, i.e. the
 * normal distribution restricted to y > 0.  Its quantile maps u into the
 * part of the normal CDF above y = 0: y = 1 + p Phi^-1(Phi(-1/p) + u (1 -
 * Phi(-1/p))). */
double orc_truncnorm_quantile(double u, double p)
{
    double c0 = normal_cdf(-1.0 / p);
    return 1.0 + p * orc_normal_quantile(c0 + u * (1.0 - c0));
}

/* Inverse-CDF tables of the sizes.  The knots are equally spaced in
 * t = -ln(2 min(u, 1 - u)), which places them densely in both tails: with
 * H = M/2 and dt = 32 ln 2 / (H - 1) (t = 32 ln 2 is the farthest tail a
 * 32-bit uniform reaches, u = 2^-33), knot j < H is F^-1(e^(-j dt)/2) (the
 * lower half, from the median down) and knot H + j is F^-1(1 - e^(-j dt)/2)
 * (the upper half, from the median up); the upper half is computed from the
 * upper tail's probability, so the far tail keeps its precision. */
static double table_dt(int32_t M) { return 32.0 * log(2.0) / (M / 2 - 1); }

/* The orientation's normal table keeps knots at u = (k + 1/2)/M, linear in
 * u: its far tails carry no moment the weight divides by, and this lookup
 * needs no logarithm. */
void orc_table_normal(int32_t M, double* knots)
{
    for (int k = 0; k < M; ++k) knots[k] = orc_normal_quantile((k + 0.5) / M);
}

void orc_table_schulz(int32_t M, double p, double* knots)
{
    const int H = M / 2;
    for (int j = 0; j < H; ++j) {
        double v = 0.5 * exp(-j * table_dt(M));
        knots[j] = orc_schulz_quantile(v, p);
        knots[H + j] = orc_schulz_quantile_upper(v, p);
    }
}

void orc_table_truncnorm(int32_t M, double p, double* knots)
{
    /* upper tail: 1 - u = v, so c0 + u (1 - c0) = 1 - v (1 - c0) and, by the
       symmetry of the normal, y = 1 - p Phi^-1(v (1 - c0)) */
    const int H = M / 2;
    double c0 = normal_cdf(-1.0 / p);
    for (int j = 0; j < H; ++j) {
        double v = 0.5 * exp(-j * table_dt(M));
        knots[j] = orc_truncnorm_quantile(v, p);
        knots[H + j] = 1.0 - p * orc_normal_quantile(v * (1.0 - c0));
    }
}

/* The size table of a parameter set (Schulz or positive Gaussian). */
static void size_table(const orc_params* p, double* knots)
{
    if (p->poly_kind == 1) orc_table_truncnorm(p->table_size, p->poly, knots);
    else orc_table_schulz(p->table_size, p->poly, knots);
}

/* Lookup in the normal table: s = u M - 1/2, k = clamp(floor(s), 0, M - 2),
 * linear interpolation between knots k and k + 1 (linear extrapolation in
 * the two end half-cells). */
double orc_table_lookup_u(const double* knots, int32_t M, double u)
{
    double s = u * M - 0.5;
    double fk = floor(s);
    if (fk < 0.0) fk = 0.0;
    if (fk > M - 2) fk = M - 2;
    int k = (int)fk;
    double f = s - fk;
    return knots[k] + f * (knots[k + 1] - knots[k]);
}

/* Table lookup: t = -ln(2 min(u, 1 - u)), s = t/dt, j = min(floor(s),
 * H - 2), linear interpolation in t between knots j and j + 1 of the half
 * that u falls in (u < 1/2 the lower half, else the upper one). */
double orc_table_lookup(const double* knots, int32_t M, double u)
{
    const int H = M / 2;
    const double* half = u < 0.5 ? knots : knots + H;
    double t = -log(2.0 * (u < 0.5 ? u : 1.0 - u));
    double s = t / table_dt(M);
    double fj = floor(s);
    if (fj > H - 2) fj = H - 2;
    int j = (int)fj;
    double f = s - fj;
    return half[j] + f * (half[j + 1] - half[j]);
}

/* ------------------------------------------------------------------------ */
/* Shape functions. */

/* 3 j1(x)/x = 3 (sin x - x cos x)/x^3, the normalised sphere amplitude
 * (-> 1 as x -> 0).  Below x = 0.1 its Taylor series
 * sum_m (-1)^m 6 (m+1) x^(2m) / (2m+3)! is summed instead. */
double orc_sph(double x)
{
    x = fabs(x);
    if (x < 0.1) {
        double s = 0.0, x2 = x * x, xp = 1.0, fact = 6.0; /* (2m+3)! at m=0 */
        for (int m = 0; m < 8; ++m) {
            double term = 6.0 * (m + 1) * xp / fact;
            s += (m % 2 == 0) ? term : -term;
            xp *= x2;
            fact *= (2.0 * m + 4.0) * (2.0 * m + 5.0);
        }
        return s;
    }
    return 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
}

/* Lambda1(x) = 2 J1(x)/x (-> 1 as x -> 0), J1 from the C library; below
 * 1e-3 the series 1 - x^2/8 + x^4/192. */
double orc_lambda1(double x)
{
    x = fabs(x);
    if (x < 1e-3) {
        double x2 = x * x;
        return 1.0 - x2 / 8.0 + x2 * x2 / 192.0;
    }
    return 2.0 * j1(x) / x;
}

/* sinc(x) = sin(x)/x. */
double orc_sinc(double x)
{
    if (fabs(x) < 1e-4) return 1.0 - x * x / 6.0;
    return sin(x) / x;
}

/* ------------------------------------------------------------------------ */
/* Hard-sphere structure factor in the Percus-Yevick closure (Wertheim 1963;
 * Kinning & Thomas 1984), the "hard sphere" model of the isotropic table:
 *   x = 2 q R,  S = 1 / (1 + 24 phi G(x)/x),
 *   G(x) = alpha (sin x - x cos x)/x^2
 *        + beta (2x sin x + (2 - x^2) cos x - 2)/x^3
 *        + gamma (-x^4 cos x + 4[(3x^2 - 6) cos x + (x^3 - 6x) sin x + 6])/x^5,
 *   alpha = (1+2phi)^2/(1-phi)^4, beta = -6 phi (1+phi/2)^2/(1-phi)^4,
 *   gamma = phi alpha / 2.
 * The closed form cancels catastrophically at small x, so below x = 1 the
 * Taylor series of G(x)/x is used; its coefficients are the x^(2m) terms of
 * the three brackets expanded with the power series of sin and cos.        */
static double fact(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}
static double sgn(int n) { return (n % 2 == 0) ? 1.0 : -1.0; }

/* c[m] = coefficient of x^(2m) in G(x)/x, m = 0 .. nterms-1. */
void orc_py_series(double phi, int32_t nterms, double* c)
{
    double om = 1.0 - phi;
    double om4 = om * om * om * om;
    double alpha = (1.0 + 2.0 * phi) * (1.0 + 2.0 * phi) / om4;
    double beta = -6.0 * phi * (1.0 + 0.5 * phi) * (1.0 + 0.5 * phi) / om4;
    double gamma = 0.5 * phi * alpha;
    for (int m = 0; m < nterms; ++m) {
        /* (sin x - x cos x)/x^3: x^(2m) coefficient */
        double am = sgn(m) * 2.0 * (m + 1) / fact(2 * m + 3);
        /* (2x sin x + (2 - x^2) cos x - 2)/x^4: x^(2M) of the numerator, M = m+2 */
        int M = m + 2;
        double bm = 2.0 * sgn(M - 1) / fact(2 * M - 1) + 2.0 * sgn(M) / fact(2 * M)
                  - sgn(M - 1) / fact(2 * M - 2);
        /* gamma bracket / x^6: x^(2K) of the numerator, K = m+3 */
        int K = m + 3;
        double gm = -sgn(K - 2) / fact(2 * K - 4) + 12.0 * sgn(K - 1) / fact(2 * K - 2)
                  - 24.0 * sgn(K) / fact(2 * K) + 4.0 * sgn(K - 2) / fact(2 * K - 3)
                  - 24.0 * sgn(K - 1) / fact(2 * K - 1);
        c[m] = alpha * am + beta * bm + gamma * gm;
    }
}

/* G(x)/x by the closed form (valid, but inaccurate for small x). */
double orc_py_g_over_x_direct(double x, double phi)
{
    double om = 1.0 - phi;
    double om4 = om * om * om * om;
    double alpha = (1.0 + 2.0 * phi) * (1.0 + 2.0 * phi) / om4;
    double beta = -6.0 * phi * (1.0 + 0.5 * phi) * (1.0 + 0.5 * phi) / om4;
    double gamma = 0.5 * phi * alpha;
    double s = sin(x), c = cos(x);
    double x2 = x * x, x3 = x2 * x, x4 = x2 * x2, x5 = x4 * x;
    double G = alpha * (s - x * c) / x2
             + beta * (2.0 * x * s + (2.0 - x2) * c - 2.0) / x3
             + gamma * (-x4 * c + 4.0 * ((3.0 * x2 - 6.0) * c + (x3 - 6.0 * x) * s + 6.0)) / x5;
    return G / x;
}

double orc_py_sq(double q, double radius, double phi)
{
    if (phi <= 0.0) return 1.0;
    double x = 2.0 * q * radius;
    double gx;
    if (x < 1.0) {
        double c[14];
        orc_py_series(phi, 14, c);
        double x2 = x * x, xp = 1.0;
        gx = 0.0;
        for (int m = 0; m < 14; ++m) { gx += c[m] * xp; xp *= x2; }
    } else {
        gx = orc_py_g_over_x_direct(x, phi);
    }
    return 1.0 / (1.0 + 24.0 * phi * gx);
}

void orc_gauss_legendre(int32_t n, double* x, double* w);

/* Adhesive hard spheres in the Percus-Yevick closure (Baxter's model:
 * diameter sigma, volume fraction eta, stickiness tau).  lambda is the
 * smaller root of (eta/12) l^2 - (tau + eta/(1 - eta)) l + (1 + eta/2)/(1 - eta)^2;
 * NaN when the roots are complex (inside the model's two-phase region). */
double orc_sticky_lambda(double eta, double tau)
{
    double a = eta / 12.0, b = -(tau + eta / (1.0 - eta));
    double c = (1.0 + 0.5 * eta) / ((1.0 - eta) * (1.0 - eta));
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return NAN;
    if (a == 0.0) return c / -b;
    return (-b - sqrt(disc)) / (2.0 * a);
}

/* S(q) = 1 / |Qhat(k)|^2 with Baxter's factor function: in units of sigma,
 * Q(x) = (a/2)(x^2 - 1) + b (x - 1) + lambda/12 on 0 <= x <= 1, with
 * mu = lambda eta (1 - eta), a = (1 + 2 eta - mu)/(1 - eta)^2,
 * b = (mu - 3 eta)/(2 (1 - eta)^2), and Qhat(k) = 1 - 12 eta int_0^1 Q(x)
 * exp(i k x) dx, k = q sigma.  The integral by composite Gauss-Legendre
 * (32 nodes on each of 1 + k/4 panels: Q is a quadratic, the panels follow
 * the oscillation of exp(i k x)). */
double orc_sticky_sq(double q, double radius, double eta, double tau)
{
    if (eta <= 0.0) return 1.0;
    double lam = orc_sticky_lambda(eta, tau);
    double mu = lam * eta * (1.0 - eta);
    double om2 = (1.0 - eta) * (1.0 - eta);
    double a = (1.0 + 2.0 * eta - mu) / om2, b = (mu - 3.0 * eta) / (2.0 * om2);
    double k = 2.0 * q * radius;
    double gx[32], gw[32];
    orc_gauss_legendre(32, gx, gw);
    int npan = 1 + (int)(k / 4.0);
    double h = 1.0 / npan, re = 0.0, im = 0.0;
    for (int j = 0; j < npan; ++j) {
        for (int i = 0; i < 32; ++i) {
            double x = h * (j + 0.5 * (gx[i] + 1.0)), w = 0.5 * h * gw[i];
            double qx = 0.5 * a * (x * x - 1.0) + b * (x - 1.0) + lam / 12.0;
            re += w * qx * cos(k * x);
            im += w * qx * sin(k * x);
        }
    }
    double A = 1.0 - 12.0 * eta * re, B = -12.0 * eta * im;
    return 1.0 / (A * A + B * B);
}

/* Square-well fluid in the mean spherical approximation (Sharma and Sharma):
 * the hard-sphere (Percus-Yevick) direct correlation plus, between sigma and
 * width * sigma, c(r) = depth (the well's depth in kT, attractive when
 * positive), so 1/S = 1/S_PY - rho c_well(q) with
 * rho c_well(q) = 24 eta depth int_1^width x^2 sin(k x)/(k x) dx, k = q sigma
 * (composite Gauss-Legendre, 32 nodes on each of 1 + k (width - 1)/4 panels). */
double orc_square_well_sq(double q, double radius, double eta, double depth, double width)
{
    if (eta <= 0.0) return 1.0;
    double k = 2.0 * q * radius;
    double gx[32], gw[32];
    orc_gauss_legendre(32, gx, gw);
    int npan = 1 + (int)(k * (width - 1.0) / 4.0);
    double h = (width - 1.0) / npan, integral = 0.0;
    for (int j = 0; j < npan; ++j) {
        for (int i = 0; i < 32; ++i) {
            double x = 1.0 + h * (j + 0.5 * (gx[i] + 1.0));
            double kx = k * x;
            double sinc = kx < 1e-8 ? 1.0 : sin(kx) / kx;
            integral += 0.5 * h * gw[i] * x * x * sinc;
        }
    }
    return 1.0 / (1.0 / orc_py_sq(q, radius, eta) - 24.0 * eta * depth * integral);
}

/* The structure factor selected by sq_kind (1 when sq_phi = 0). */
/* Hayter-Penfold structure factor (sq_kind 3): charged hard spheres of
 * diameter sigma = 2 sq_radius with beta U = U_c (sigma/r) exp(-kappa (r -
 * sigma)) outside the core (U_c = sq_extra[0], kappa sigma = sq_extra[1]) in
 * the mean spherical approximation.  The direct correlation function inside
 * the core, c(x) at x = i/ORC_MSA_N (i = 0..ORC_MSA_N, units of sigma), comes
 * from the oracle's Ornstein-Zernike solver (oracle/msa.py) through
 * orc_set_msa; here S = 1/(1 - rho c^(K)), K = q sigma, rho = 6 eta/pi, with
 * c^ = 4 pi/K int_0^1 x c sin(K x) dx by Simpson on the grid plus the tail's
 * closed form -4 pi U_c (k sin K + K cos K)/(K (k^2 + K^2)), k = kappa sigma. */
#define ORC_MSA_N 1024
static double g_msa_c[ORC_MSA_N + 1];
static double g_msa_key[3] = {-1.0, -1.0, -1.0};

void orc_set_msa(const double* c_in, double eta, double uc, double ks)
{
    memcpy(g_msa_c, c_in, sizeof(double) * (ORC_MSA_N + 1));
    g_msa_key[0] = eta;
    g_msa_key[1] = uc;
    g_msa_key[2] = ks;
}

double orc_msa_sq(double q, double radius, double eta, double uc, double ks)
{
    if (g_msa_key[0] != eta || g_msa_key[1] != uc || g_msa_key[2] != ks) return NAN;  /* not set up */
    const double K = 2.0 * radius * q, h = 1.0 / ORC_MSA_N;
    double inner = 0.0;
    for (int i = 0; i <= ORC_MSA_N; ++i) {
        const double w = (i == 0 || i == ORC_MSA_N) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        const double x = i * h;
        inner += w * x * g_msa_c[i] * sin(K * x);
    }
    inner *= h / 3.0 * 4.0 * ORC_PI / K;
    const double tail = -4.0 * ORC_PI * uc * (ks * sin(K) + K * cos(K)) / (K * (ks * ks + K * K));
    return 1.0 / (1.0 - 6.0 * eta / ORC_PI * (inner + tail));
}

static double struct_factor(const orc_params* p, double q)
{
    if (!(p->sq_phi > 0.0)) return 1.0;
    if (p->sq_kind == 3) return orc_msa_sq(q, p->sq_radius, p->sq_phi, p->sq_extra[0], p->sq_extra[1]);
    if (p->sq_kind == 1) return orc_sticky_sq(q, p->sq_radius, p->sq_phi, p->sq_extra[0]);
    if (p->sq_kind == 2) return orc_square_well_sq(q, p->sq_radius, p->sq_phi, p->sq_extra[0], p->sq_extra[1]);
    return orc_py_sq(q, p->sq_radius, p->sq_phi);
}

/* ------------------------------------------------------------------------ */
/* Particle amplitudes F (the Fourier transform of the excess scattering
 * length density, Eq. (1)), in Angstrom: F^2 = (drho V)^2 P.  The particle
 * axes A, B, C are given in the laboratory frame; Q_A = Q.A etc.           */

static double vol_sphere(double r) { return 4.0 / 3.0 * ORC_PI * r * r * r; }

/* Gauss-Legendre nodes on [-1, 1] for the caps' integral, computed once per
 * order (under a lock; read-only afterwards). */
static pthread_mutex_t g_cap_lock = PTHREAD_MUTEX_INITIALIZER;
static double g_cap_x[ORC_MAX_QUAD + 1][ORC_MAX_QUAD], g_cap_w[ORC_MAX_QUAD + 1][ORC_MAX_QUAD];
static int g_cap_ready[ORC_MAX_QUAD + 1];

void orc_gauss_legendre(int32_t n, double* x, double* w);

static void cap_nodes(int n, const double** x, const double** w)
{
    pthread_mutex_lock(&g_cap_lock);
    if (!g_cap_ready[n]) {
        orc_gauss_legendre(n, g_cap_x[n], g_cap_w[n]);
        g_cap_ready[n] = 1;
    }
    pthread_mutex_unlock(&g_cap_lock);
    *x = g_cap_x[n];
    *w = g_cap_w[n];
}

/* Bodies of revolution about C made of a cylinder (radius R, length L,
 * |z| <= L/2) and two spherical caps of radius r >= R that meet the end
 * faces in the circle of radius R (Tables I-II, group A: Barbell, Capped
 * cylinder).  The cap sphere's centre sits at z_c = L/2 + h: h = +sqrt(r^2 -
 * R^2) beyond the end face (barbell: the cap is most of a sphere) or h =
 * -sqrt(r^2 - R^2) inside the cylinder (capped cylinder: a dome).  The
 * amplitude is the Fourier transform of the body: slicing it into discs of
 * radius rho(z) normal to C, a disc contributes pi rho^2 2J1(Q_AB rho)/(Q_AB
 * rho) e^{i Q_C z}; the cylinder gives pi R^2 L sinc(Q_C L/2) 2J1(Q_AB
 * R)/(Q_AB R), and the caps (z = z_c + r t, rho = r sqrt(1 - t^2), t from
 * t0 = -h/r to 1, both ends adding the complex conjugates)
 *   2 pi r^3 int_{t0}^{1} cos(Q_C (z_c + r t)) (1 - t^2)
 *                         2J1(Q_AB r sqrt(1-t^2))/(Q_AB r sqrt(1-t^2)) dt,
 * here by n-point Gauss-Legendre.  Volume: pi R^2 L + 2 pi (r^3 (1 - t0)
 * - r^3 (1 - t0^3)/3). */
static double caps_amplitude(const double s[3], int barbell, double qab, double qc, int n)
{
    double R = s[0], L = s[1], r = s[2];
    double h = sqrt(r * r - R * R) * (barbell ? 1.0 : -1.0);
    double zc = 0.5 * L + h, t0 = -h / r;
    const double *gx, *gw;
    cap_nodes(n, &gx, &gw);
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        double t = 0.5 * (1.0 - t0) * gx[i] + 0.5 * (1.0 + t0);
        double rho = r * sqrt(1.0 - t * t);
        sum += gw[i] * cos(qc * (zc + r * t)) * (1.0 - t * t) * orc_lambda1(qab * rho);
    }
    return 2.0 * ORC_PI * r * r * r * 0.5 * (1.0 - t0) * sum;
}

static double caps_volume(const double s[3], int barbell)
{
    double R = s[0], r = s[2];
    double h = sqrt(r * r - R * R) * (barbell ? 1.0 : -1.0);
    double t0 = -h / r;
    /* pi r^3 int_{t0}^{1} (1 - t^2) dt, twice */
    return 2.0 * ORC_PI * r * r * r * ((1.0 - t0) - (1.0 - t0 * t0 * t0) / 3.0);
}

/* Superball |x|^(2p) + |y|^(2p) + |z|^(2p) <= R^(2p) (Tables I-II, group F;
 * p = 1/2 octahedron, 1 sphere, p -> infinity the cube of edge 2R), axes
 * x, y, z along A, B, C.  Its transform, even in each coordinate, is
 *   8 int_0^R dx cos(Q_A x) int_0^ym(x) dy cos(Q_B y) sin(Q_C zm)/Q_C,
 * ym(x) = (R^2p - x^2p)^(1/2p), zm(x, y) = (R^2p - x^2p - y^2p)^(1/2p): the z
 * integral exact, x and y by n-point Gauss-Legendre on [0, R] and
 * [0, ym(x)].  Volume 8 R^3 Gamma(1 + 1/2p)^3 / Gamma(1 + 3/2p). */
static double superball_amplitude(double R, double p, double qa, double qb, double qc, int n)
{
    const double *gx, *gw;
    cap_nodes(n, &gx, &gw);
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        double x = 0.5 * R * (gx[i] + 1.0);
        double ym = R * pow(1.0 - pow(x / R, 2.0 * p), 1.0 / (2.0 * p));
        double inner = 0.0;
        for (int j = 0; j < n; ++j) {
            double y = 0.5 * ym * (gx[j] + 1.0);
            double rest = 1.0 - pow(x / R, 2.0 * p) - pow(y / R, 2.0 * p);
            double zm = rest > 0.0 ? R * pow(rest, 1.0 / (2.0 * p)) : 0.0;
            double zint = zm * orc_sinc(qc * zm); /* sin(Q_C zm)/Q_C */
            inner += 0.5 * ym * gw[j] * cos(qb * y) * zint;
        }
        sum += 0.5 * R * gw[i] * cos(qa * x) * inner;
    }
    return 8.0 * sum;
}

static double superball_volume(double R, double p)
{
    double g1 = tgamma(1.0 + 1.0 / (2.0 * p));
    return 8.0 * R * R * R * g1 * g1 * g1 / tgamma(1.0 + 3.0 / (2.0 * p));
}

/* Unit-contrast amplitudes of the homogeneous bodies the layered models are
 * built from: a cylinder (radius r, length len, axis C), an ellipsoid
 * (semi-axes a, b, c along A, B, C) and a box (edges a, b, c). */
static double cyl_amp(double r, double len, double qab, double qc)
{
    return ORC_PI * r * r * len * orc_sinc(0.5 * qc * len) * orc_lambda1(qab * r);
}

static double ell_amp(double a, double b, double c, double qa, double qb, double qc)
{
    double x = sqrt((a * qa) * (a * qa) + (b * qb) * (b * qb) + (c * qc) * (c * qc));
    return 4.0 / 3.0 * ORC_PI * a * b * c * orc_sph(x);
}

static double box_amp(double a, double b, double c, double qa, double qb, double qc)
{
    return a * b * c * orc_sinc(0.5 * qa * a) * orc_sinc(0.5 * qb * b) * orc_sinc(0.5 * qc * c);
}

/* Amplitude for one set of (possibly scaled) sizes; cap_n is the
 * Gauss-Legendre order of the caps' integral (barbell, capped cylinder). */
static double amplitude(int kind, const double s[3], double shell, const double sld[3],
                        const double extra[4], double q, double qa, double qb, double qc, int cap_n)
{
    double drho = sld[0] - sld[2];
    switch (kind) {
    case 0: /* sphere, isotropic, Eq. (5) */
        return drho * vol_sphere(s[0]) * orc_sph(q * s[0]);
    case 1: { /* core-shell sphere: core minus shell contrast plus shell minus solvent */
        double rc = s[0], ro = s[0] + shell;
        return (sld[0] - sld[1]) * vol_sphere(rc) * orc_sph(q * rc)
             + (sld[1] - sld[2]) * vol_sphere(ro) * orc_sph(q * ro);
    }
    case 2: { /* cylinder, one symmetry axis C, Eqs. (7) and (9): the sinc factor
                 takes the projection on the axis and half the length, the
                 Bessel factor the projection on the AB plane and the radius */
        double r = s[0], len = s[1];
        double qab2 = q * q - qc * qc;
        double qab = qab2 > 0.0 ? sqrt(qab2) : 0.0;
        return drho * ORC_PI * r * r * len * orc_sinc(0.5 * qc * len) * orc_lambda1(qab * r);
    }
    case 3: { /* triaxial ellipsoid, semi-axes a, b, c along A, B, C, Eq. (6) */
        double a = s[0], b = s[1], c = s[2];
        double x = sqrt((a * qa) * (a * qa) + (b * qb) * (b * qb) + (c * qc) * (c * qc));
        return drho * 4.0 / 3.0 * ORC_PI * a * b * c * orc_sph(x);
    }
    case 4: { /* parallelepiped, edges A, B, C, Eq. (6) */
        double a = s[0], b = s[1], c = s[2];
        return drho * a * b * c * orc_sinc(0.5 * qa * a) * orc_sinc(0.5 * qb * b)
             * orc_sinc(0.5 * qc * c);
    }
    case 5:   /* barbell */
    case 6: { /* capped cylinder */
        double r = s[0], len = s[1];
        double qab2 = q * q - qc * qc;
        double qab = qab2 > 0.0 ? sqrt(qab2) : 0.0;
        double cyl = ORC_PI * r * r * len * orc_sinc(0.5 * qc * len) * orc_lambda1(qab * r);
        return drho * (cyl + caps_amplitude(s, kind == 5, qab, qc, cap_n));
    }
    case 7: { /* hollow rectangular prism, walls of thickness shell -> 0: the
                 six faces as sheets of areal density shell; the two faces
                 normal to an axis sit at +-half that edge, so their sum is
                 2 cos(half phase) times the face's own transform (the two
                 in-plane sinc factors times its area) */
        double a = s[0], b = s[1], c = s[2];
        double xa = 0.5 * qa * a, xb = 0.5 * qb * b, xc = 0.5 * qc * c;
        double sa = orc_sinc(xa), sb = orc_sinc(xb), sc = orc_sinc(xc);
        return drho * 2.0 * shell
             * (b * c * cos(xa) * sb * sc + a * c * sa * cos(xb) * sc + a * b * sa * sb * cos(xc));
    }
    case 9: { /* hollow cylinder: the cylinder of radius bore + shell minus the bore */
        double qab2 = q * q - qc * qc;
        double qab = qab2 > 0.0 ? sqrt(qab2) : 0.0;
        return drho * (cyl_amp(s[0] + shell, s[1], qab, qc) - cyl_amp(s[0], s[1], qab, qc));
    }
    case 10: { /* core-shell cylinder: the core (R, L) in a shell of radial thickness
                  shell and end-face thickness extra[0]; contrasts as for the
                  core-shell sphere */
        double qab2 = q * q - qc * qc;
        double qab = qab2 > 0.0 ? sqrt(qab2) : 0.0;
        return (sld[0] - sld[1]) * cyl_amp(s[0], s[1], qab, qc)
             + (sld[1] - sld[2]) * cyl_amp(s[0] + shell, s[1] + 2.0 * extra[0], qab, qc);
    }
    case 11: /* core-shell ellipsoid: the core's semi-axes each grown by shell */
        return (sld[0] - sld[1]) * ell_amp(s[0], s[1], s[2], qa, qb, qc)
             + (sld[1] - sld[2]) * ell_amp(s[0] + shell, s[1] + shell, s[2] + shell, qa, qb, qc);
    case 12: /* hollow prism, walls of thickness shell: the box minus its cavity */
        return drho * (box_amp(s[0], s[1], s[2], qa, qb, qc)
                       - box_amp(s[0] - 2.0 * shell, s[1] - 2.0 * shell, s[2] - 2.0 * shell, qa, qb, qc));
    case 51: /* superball: half-edge s0, exponent parameter p = extra[0] */
        return drho * superball_amplitude(s[0], extra[0], qa, qb, qc, cap_n);
    case 41: { /* elliptical cylinder: semi-axes s0 along A, s1 along B, length s2
                  along C; the ellipse's transform is the disc's at the scaled
                  projection sqrt((s0 Q_A)^2 + (s1 Q_B)^2) */
        double x = sqrt((s[0] * qa) * (s[0] * qa) + (s[1] * qb) * (s[1] * qb));
        return drho * ORC_PI * s[0] * s[1] * s[2] * orc_sinc(0.5 * qc * s[2]) * orc_lambda1(x);
    }
    case 42: { /* core-shell bicelle: core (R, L), face layers of thickness extra[0]
                  on the ends (SLD extra[1]), a rim of thickness shell around the
                  whole (SLD sld[1]): core, core + faces, and the outer cylinder
                  with their contrast steps */
        double qab2 = q * q - qc * qc;
        double qab = qab2 > 0.0 ? sqrt(qab2) : 0.0;
        double tf = extra[0], rf = extra[1];
        return (sld[0] - rf) * cyl_amp(s[0], s[1], qab, qc)
             + (rf - sld[1]) * cyl_amp(s[0], s[1] + 2.0 * tf, qab, qc)
             + (sld[1] - sld[2]) * cyl_amp(s[0] + shell, s[1] + 2.0 * tf, qab, qc);
    }
    case 44: { /* elliptical core-shell bicelle: the bicelle with its cross
                  sections stretched by extra[2] along B (the core's semi-axes
                  R and x R; the rim adds shell to both) */
        double xr = extra[2], tf = extra[0], rf = extra[1], rr = s[0] + shell;
        double a1 = sqrt((s[0] * qa) * (s[0] * qa) + (xr * s[0] * qb) * (xr * s[0] * qb));
        double a2 = sqrt((rr * qa) * (rr * qa) + ((xr * s[0] + shell) * qb) * ((xr * s[0] + shell) * qb));
        double lf = s[1] + 2.0 * tf;
        double core = ORC_PI * s[0] * xr * s[0] * s[1] * orc_sinc(0.5 * qc * s[1]) * orc_lambda1(a1);
        double faces = ORC_PI * s[0] * xr * s[0] * lf * orc_sinc(0.5 * qc * lf) * orc_lambda1(a1);
        double outer = ORC_PI * rr * (xr * s[0] + shell) * lf * orc_sinc(0.5 * qc * lf) * orc_lambda1(a2);
        return (sld[0] - rf) * core + (rf - sld[1]) * faces + (sld[1] - sld[2]) * outer;
    }
    case 56: { /* elliptical bicelle with a belt: an elliptic core (semi-axes R,
                  x R; length L), face layers of thickness t_f = extra[0] (SLD
                  extra[1]) over the core's cross-section at both ends, a belt
                  of thickness shell (SLD sld[1]) around the core only (length
                  L); rough interfaces damp the amplitude by exp(-(q sigma)^2/2),
                  sigma = extra[3] */
        double xr = extra[2], tf = extra[0], rf = extra[1], t = shell;
        double ra = s[0], rb = xr * s[0], len = s[1], lf = len + 2.0 * tf;
        double a1 = sqrt((ra * qa) * (ra * qa) + (rb * qb) * (rb * qb));
        double a2 = sqrt(((ra + t) * qa) * ((ra + t) * qa) + ((rb + t) * qb) * ((rb + t) * qb));
        double core = ORC_PI * ra * rb * len * orc_sinc(0.5 * qc * len) * orc_lambda1(a1);
        double faces = ORC_PI * ra * rb * lf * orc_sinc(0.5 * qc * lf) * orc_lambda1(a1);
        double belt = ORC_PI * (ra + t) * (rb + t) * len * orc_sinc(0.5 * qc * len) * orc_lambda1(a2);
        double amp = (sld[0] - rf - sld[1] + sld[2]) * core + (rf - sld[2]) * faces + (sld[1] - sld[2]) * belt;
        return amp * exp(-0.5 * q * q * extra[3] * extra[3]);
    }
    case 45: { /* one disk of the stack: a core of radius R, thickness s1, with
                  layers of thickness shell on both faces */
        double qab2 = q * q - qc * qc;
        double qab = qab2 > 0.0 ? sqrt(qab2) : 0.0;
        return (sld[0] - sld[1]) * cyl_amp(s[0], s[1], qab, qc)
             + (sld[1] - sld[2]) * cyl_amp(s[0], s[1] + 2.0 * shell, qab, qc);
    }
    case 46:
    case 47:
    case 48: /* the lattice's sphere, radius s0 */
        return drho * vol_sphere(s[0]) * orc_sph(q * s[0]);
    case 43: { /* core-shell parallelepiped: the core box and, on each pair of
                  faces, a slab of thickness extra[k] covering just that face
                  (SLD sld[1]); the two slabs normal to an axis sit at +-(edge +
                  t)/2, so their sum is 2 cos(Q (edge + t)/2) times one slab */
        double core = box_amp(s[0], s[1], s[2], qa, qb, qc);
        double ta = extra[0], tb = extra[1], tc = extra[2];
        double sa = 2.0 * cos(0.5 * qa * (s[0] + ta)) * box_amp(ta, s[1], s[2], qa, qb, qc);
        double sb = 2.0 * cos(0.5 * qb * (s[1] + tb)) * box_amp(s[0], tb, s[2], qa, qb, qc);
        double sc = 2.0 * cos(0.5 * qc * (s[2] + tc)) * box_amp(s[0], s[1], tc, qa, qb, qc);
        return (sld[0] - sld[2]) * core + (sld[1] - sld[2]) * (sa + sb + sc);
    }
    }
    return 0.0;
}

/* Polymer micelle (Pedersen and Gerstenberg, Macromolecules 29 (1996) 1363):
 * a homogeneous spherical core of radius R carrying N Gaussian chains of
 * radius of gyration Rg that start at its surface.  With the excess
 * scattering lengths of one core block and one chain, b_s and b_c, and
 * x = (q Rg)^2, the scattering per micelle is the sum of the core's self term,
 * the chains' self terms (Debye function), core-chain and chain-chain
 * interference; the chain amplitude is the average of exp(-x t) along the
 * chain and the chains' centres sit at R + d Rg (spherical average: sinc). */
static double debye_chain(double x)
{
    /* 2 (exp(-x) - 1 + x) / x^2: the double average of exp(-x |t - u|) */
    if (x < 1e-3) return 1.0 - x / 3.0 + x * x / 12.0 - x * x * x / 60.0;
    return 2.0 * (expm1(-x) + x) / (x * x);
}

static double chain_amplitude(double x)
{
    /* (1 - exp(-x)) / x: the average of exp(-x t) over t in [0, 1] */
    if (x < 1e-3) return 1.0 - x / 2.0 + x * x / 6.0 - x * x * x / 24.0;
    return -expm1(-x) / x;
}

static double micelle_f2(const double s[3], const double sld[3], const double extra[4], double q)
{
    double R = s[0], rg = s[1];
    double n = extra[0], bs = extra[1] * (sld[0] - sld[2]), bc = extra[2] * (sld[1] - sld[2]);
    double x = q * rg * q * rg;
    double core = orc_sph(q * R);
    double pc = debye_chain(x), ac = chain_amplitude(x);
    double shell = orc_sinc(q * (R + extra[3] * rg));
    return n * n * bs * bs * core * core + n * bc * bc * pc + 2.0 * n * n * bs * bc * core * ac * shell
         + n * (n - 1.0) * bc * bc * ac * ac * shell * shell;
}

/* Shape-independent models: the macroscopic cross-section dSigma/dOmega(q)
 * in 1/cm, scale = its value at q = 0 (extra[0]); the length is size[0]. */
static int shape_independent(int kind)
{
    return (kind >= 13 && kind <= 24) || (kind >= 29 && kind <= 37) || kind == 40 || kind == 49 || kind == 50;
}

/* Fractal aggregates of spherical blocks (radius R0): Teixeira's structure
 * factor of a mass fractal of dimension D with cut-off length xi, 1 plus the
 * blocks' number density times the transform of the pair correlation
 * (D / (4 pi R0^D)) r^(D - 3) exp(-r/xi). */
static double teixeira_sq(double q, double r0, double xi, double d)
{
    if (q * xi < 1e-6) return 1.0 + tgamma(d + 1.0) * pow(xi / r0, d);
    double qx = q * xi;
    return 1.0 + d * tgamma(d - 1.0) * sin((d - 1.0) * atan(qx))
                 / (pow(q * r0, d) * pow(1.0 + 1.0 / (qx * qx), 0.5 * (d - 1.0)));
}

static double shape_independent_iq(const orc_params* p, const double s[3], double q)
{
    double scale = p->extra[0], l = s[0];
    double x = q * l * q * l;
    switch (p->kind) {
    case 13: /* Guinier: exp(-(q Rg)^2 / 3) */
        return scale * exp(-x / 3.0);
    case 14: /* Ornstein-Zernike (Lorentzian), correlation length xi */
        return scale / (1.0 + x);
    case 15: /* Debye-Anderson-Brumberger, random two-phase, correlation length */
        return scale / ((1.0 + x) * (1.0 + x));
    case 16: /* Gaussian coil: the Debye function of (q Rg)^2 */
        return scale * debye_chain(x);
    case 17: { /* Gaussian coils whose masses follow a Schulz-Zimm distribution
                  (U = Mw/Mn - 1 = extra[1]): the mass-squared weighted average
                  of the Debye function, 2 ((1 + U z)^(-1/U) - 1 + z) / ((1 + U) z^2)
                  with z = (q Rg_n)^2 and Rg_n^2 = Rg_z^2 / (1 + 2U), Rg_z the
                  Guinier (z-average) radius of gyration given in size[0] */
        double u = p->extra[1];
        double z = x / (1.0 + 2.0 * u);
        if (u <= 0.0) return scale * debye_chain(z);
        if (z < 1e-4) /* series: 1 - z (1 + 2U)/3 + z^2 (1 + 2U)(1 + 3U)/12 */
            return scale * (1.0 - z * (1.0 + 2.0 * u) / 3.0 + z * z * (1.0 + 2.0 * u) * (1.0 + 3.0 * u) / 12.0);
        return scale * 2.0 * (pow(1.0 + u * z, -1.0 / u) - 1.0 + z) / ((1.0 + u) * z * z);
    }
    case 18: { /* Teubner-Strey: period d = size[1], correlation length xi = size[0];
                  1/I is a quadratic in q^2 with its minimum at q = 2 pi/d
                  when d << xi, normalised to I(0) = scale */
        double k = 2.0 * ORC_PI / s[1], ixi2 = 1.0 / (l * l);
        double a = (k * k + ixi2) * (k * k + ixi2);
        return scale * a / (a + 2.0 * (ixi2 - k * k) * q * q + q * q * q * q);
    }
    case 19: /* power law scale q^-m, m = extra[1] (q in 1/A) */
        return scale * pow(q, -p->extra[1]);
    case 20: { /* Gaussian peak at q0 = extra[1], standard deviation extra[2] */
        double d = (q - p->extra[1]) / p->extra[2];
        return scale * exp(-0.5 * d * d);
    }
    case 21: { /* Lorentzian peak at q0 = extra[1], half width extra[2] */
        double d = (q - p->extra[1]) / p->extra[2];
        return scale / (1.0 + d * d);
    }
    case 22: { /* mass fractal of dimension D = extra[1] with cut-off length xi:
                  the transform of r^(D - 3) exp(-r/xi), normalised at q = 0:
                  sin((D - 1) atan(q xi)) / ((D - 1) q xi (1 + (q xi)^2)^((D - 1)/2)) */
        double dm1 = p->extra[1] - 1.0, qx = q * l;
        if (qx < 1e-6) return scale * (1.0 - (dm1 + 1.0) * (dm1 + 2.0) / 6.0 * qx * qx); /* Guinier term */
        return scale * sin(dm1 * atan(qx)) / (dm1 * qx * pow(1.0 + qx * qx, 0.5 * dm1));
    }
    case 23: { /* star polymer of f = extra[1] Gaussian arms (Benoit), Rg of the
                  star: pairs on one arm give the chain's double average, pairs
                  on two arms the square of its single average, v = f (q Rg)^2 / (3f - 2) */
        double f = p->extra[1];
        double v = f * x / (3.0 * f - 2.0);
        double a = chain_amplitude(v);
        return scale * (debye_chain(v) + (f - 1.0) * a * a) / f;
    }
    case 24: /* Gauss-Lorentz gel: a Gaussian (length size[0], I(0) = extra[0]) plus
                an Ornstein-Zernike term (length size[1], I(0) = extra[1]) */
        return scale * exp(-0.5 * x) + p->extra[1] / (1.0 + q * s[1] * q * s[1]);
    case 29: { /* surface fractal of dimension Ds = extra[1] in (2, 3): the
                  transform of r^(3 - Ds) exp(-r/xi), a = 5 - Ds, normalised at 0:
                  sin(a atan(q xi)) / (a q xi (1 + (q xi)^2)^(a/2)) */
        double am = 5.0 - p->extra[1], qx = q * l;
        if (qx < 1e-6) return scale * (1.0 - (am + 1.0) * (am + 2.0) / 6.0 * qx * qx); /* Guinier term */
        return scale * sin(am * atan(qx)) / (am * qx * pow(1.0 + qx * qx, 0.5 * am));
    }
    case 30: { /* two power laws joined at qc = extra[2]: A q^-m1 below, the
                  continuous A qc^(m2 - m1) q^-m2 above; A = extra[0], m1 =
                  extra[1], m2 = extra[3] */
        double qc = p->extra[2];
        if (q <= qc) return scale * pow(q, -p->extra[1]);
        return scale * pow(qc, p->extra[3] - p->extra[1]) * pow(q, -p->extra[3]);
    }
    case 31: { /* Guinier-Porod (Hammouda): G q^-s exp(-(q Rg)^2/(3 - s)) up to q1,
                  D q^-m beyond, with q1 and D fixed by the continuity of the
                  intensity and of its slope; G = extra[0], s = extra[1], m = extra[2] */
        double sd = p->extra[1], m = p->extra[2];
        double q1 = sqrt((m - sd) * (3.0 - sd) / 2.0) / l;
        if (q <= q1) return scale * pow(q, -sd) * exp(-x / (3.0 - sd));
        double d = scale * exp(-(m - sd) / 2.0) * pow(q1, m - sd);
        return d * pow(q, -m);
    }
    case 32: { /* spinodal decomposition (Furukawa's scaling form): peak I_max =
                  extra[0] at q_max = extra[1], exponent gamma = extra[2]:
                  (1 + g/2) x^2 / (g/2 + x^(2 + g)), x = q / q_max */
        double g = p->extra[2], xx = q / p->extra[1];
        return scale * (1.0 + 0.5 * g) * xx * xx / (0.5 * g + pow(xx, 2.0 + g));
    }
    case 33: /* Porod: extra[0] q^-4 */
        return scale * pow(q, -4.0);
    case 34: /* line: extra[0] + extra[1] q */
        return scale + p->extra[1] * q;
    case 35: /* two generalised Lorentzians: extra[0] / (1 + (q xi1)^n1) +
                extra[2] / (1 + (q xi2)^n2); xi1, xi2 = size[0], size[1];
                n1 = extra[1], n2 = extra[3] */
        return scale / (1.0 + pow(q * s[0], p->extra[1])) + p->extra[2] / (1.0 + pow(q * s[1], p->extra[3]));
    case 36: /* correlation length: extra[0] q^-n + extra[2] / (1 + (q xi)^m);
                n = extra[1], m = extra[3], xi = size[0] */
        return scale * pow(q, -p->extra[1]) + p->extra[2] / (1.0 + pow(q * s[0], p->extra[3]));
    case 37: /* broad peak: extra[0] q^-n + extra[2] / (1 + (|q - q0| xi)^m);
                q0 = size[1], xi = size[0], n = extra[1], m = extra[3] */
        return scale * pow(q, -p->extra[1]) + p->extra[2] / (1.0 + pow(fabs(q - s[1]) * s[0], p->extra[3]));
    case 40: { /* polymer with excluded volume (Flory exponent nu = extra[1],
                  radius of gyration size[0]): the chain's double average of
                  exp(-U |t - u|^(2 nu)), U = (q Rg)^2 (2nu + 1)(2nu + 2)/6, through
                  lower incomplete gamma functions; a series below U = 1e-3 */
        double nu = p->extra[1];
        double u = x * (2.0 * nu + 1.0) * (2.0 * nu + 2.0) / 6.0;
        double s1 = 1.0 / (2.0 * nu), s2 = 1.0 / nu;
        if (u < 1e-3) {
            double a = 0.0, b = 0.0, t = 1.0;
            for (int k = 0; k < 4; ++k) {
                a += t / (s1 + k);
                b += t / (s2 + k);
                t *= -u / (k + 1.0);
            }
            return scale * (a - b) / nu;
        }
        double g1 = tgamma(s1) * orc_gamma_p(s1, u), g2 = tgamma(s2) * orc_gamma_p(s2, u);
        return scale * (g1 / pow(u, s1) - g2 / pow(u, s2)) / nu;
    }
    case 49: { /* mass-surface fractal (Hurd, Schaefer and Martin): clusters of
                  mass dimension Dm = extra[1] and radius of gyration
                  Rc = size[0] built of primary particles with fractal
                  surfaces of dimension Ds = extra[2] and radius of gyration
                  Rp = size[1]; two generalised Lorentzians, each with the
                  Guinier radius of its level:
                  (1 + (q Rc)^2/(3 pm))^-pm (1 + (q Rp)^2/(3 ps))^-ps,
                  pm = Dm/2, ps = (6 - Ds - Dm)/2 (so q^-(6-Ds) at large q) */
        double pm = 0.5 * p->extra[1], ps = 0.5 * (6.0 - p->extra[2] - p->extra[1]);
        double qp = q * s[1];
        return scale * pow(1.0 + x / (3.0 * pm), -pm) * pow(1.0 + qp * qp / (3.0 * ps), -ps);
    }
    case 50: { /* gel: a fractal network of mesh size xi = size[0] and dimension
                  D = extra[2], extra[0] (1 + (D + 1)/3 (q xi)^2)^(-D/2), plus
                  frozen inhomogeneities of radius of gyration Rg = size[1] as a
                  Guinier term extra[1] exp(-(q Rg)^2 / 3) */
        double d = p->extra[2], qg = q * s[1];
        return scale * pow(1.0 + (d + 1.0) / 3.0 * x, -0.5 * d) + p->extra[1] * exp(-qg * qg / 3.0);
    }
    }
    return 0.0;
}

/* Isotropic sphere-based particles (Tables I-II, group F), their squared
 * amplitude averaged over orientations:
 * fuzzy sphere: the sphere convolved with a Gaussian of width sigma = shell
 *   (its amplitude times exp(-(q sigma)^2 / 2));
 * vesicle: a solvent-filled shell, bore R = size[0], thickness shell;
 * multilayer vesicle: n = extra[0] shells of thickness shell, separated by
 *   solvent layers of size[1], the first around a solvent core of radius R;
 * linear pearls: n = extra[0] spheres of radius R in a straight line with
 *   gaps size[1] between them, orientation averaged (Debye's pair sum). */
static double sphere_family_f2(const orc_params* p, const double s[3], double q)
{
    double drho = p->sld[0] - p->sld[2], sh = p->sld[1] - p->sld[2];
    switch (p->kind) {
    case 25: {
        double f = drho * vol_sphere(s[0]) * orc_sph(q * s[0]) * exp(-0.5 * q * q * p->shell * p->shell);
        return f * f;
    }
    case 26: {
        double ri = s[0], ro = s[0] + p->shell;
        double f = sh * (vol_sphere(ro) * orc_sph(q * ro) - vol_sphere(ri) * orc_sph(q * ri));
        return f * f;
    }
    case 27: {
        int n = (int)p->extra[0];
        double f = 0.0;
        for (int k = 0; k < n; ++k) {
            double ri = s[0] + k * (p->shell + s[1]), ro = ri + p->shell;
            f += sh * (vol_sphere(ro) * orc_sph(q * ro) - vol_sphere(ri) * orc_sph(q * ri));
        }
        return f * f;
    }
    case 28: {
        int n = (int)p->extra[0];
        double f = drho * vol_sphere(s[0]) * orc_sph(q * s[0]);
        double d = 2.0 * s[0] + s[1], pairs = n;
        for (int k = 1; k < n; ++k) pairs += 2.0 * (n - k) * orc_sinc(q * k * d);
        return f * f * pairs;
    }
    case 58: {
        /* pearl necklace: N = extra[0] pearls (radius s0, sld[0]) joined by
           N - 1 thin rods (length l = s1 between pearl surfaces, diameter s2,
           sld[1]) into a freely jointed chain: each pearl-rod-pearl unit
           points in an independent uniform direction, so the phase between
           units d apart averages to x^d, x = sinc(q A), A = 2 R + l.  A rod
           seen from the centre of either pearl it joins averages to beta =
           int_R^{R+l} sinc(q s) ds / l; its own average is the thin rod's
           P = (2/l^2) int_0^l (l - t) sinc(q t) dt.  Pair sums:
             pearls: N + 2 sum_{d=1}^{N-1} (N - d) x^d
             rods:   (N - 1) P + 2 beta^2 sum_{d=1}^{N-2} (N - 1 - d) x^(d-1)
             pearl-rod (each pair once): 2 sum_{d=0}^{N-2} (N - 1 - d) x^d beta
           weighted by the pearls' and rods' excess lengths (drho V).  The
           two integrals by quad_n-point Gauss-Legendre (in every mode). */
        int n = (int)p->extra[0];
        double R = s[0], l = s[1], ms = drho * vol_sphere(R);
        double mr = sh * ORC_PI * 0.25 * s[2] * s[2] * l;
        double psi = orc_sph(q * R), x = orc_sinc(q * (2.0 * R + l));
        const double *gx, *gw;
        cap_nodes(p->quad_n, &gx, &gw);
        double beta = 0.0, prod = 0.0;
        for (int i = 0; i < p->quad_n; ++i) {
            double t = 0.5 * l * (gx[i] + 1.0), w = 0.5 * l * gw[i];
            beta += w * orc_sinc(q * (R + t));
            prod += w * (l - t) * orc_sinc(q * t);
        }
        beta /= l;
        double prod_rod = 2.0 * prod / (l * l);
        double spp = n, srr = (n - 1) * prod_rod, spr = 0.0;
        for (int d = 1; d < n; ++d) spp += 2.0 * (n - d) * pow(x, d);
        for (int d = 1; d <= n - 2; ++d) srr += 2.0 * beta * beta * (n - 1 - d) * pow(x, d - 1);
        for (int d = 0; d <= n - 2; ++d) spr += 2.0 * (n - 1 - d) * pow(x, d) * beta;
        return ms * ms * psi * psi * spp + mr * mr * srr + 2.0 * ms * mr * psi * spr;
    }
    case 57: {
        /* raspberry: a large sphere (radius s0, sld[0]) carrying N = extra[0]
           small spheres (radius s1, sld[1]) whose centres sit at D = s0 + s1
           (1 - 2 delta) from its centre (delta = extra[1] in [0, 1], the depth
           of penetration in small-sphere diameters), at independent uniform
           positions on that sphere.  Averaged over orientations and positions
           (Debye's pair sum): F_L^2 + N F_S^2 + 2 N F_L F_S <sinc> + N (N - 1)
           F_S^2 <sinc>^2 with <sinc> = sin(qD)/(qD), the average of exp(i Q.r)
           over a sphere of radius D */
        double n = p->extra[0];
        double fl = drho * vol_sphere(s[0]) * orc_sph(q * s[0]);
        double fs = sh * vol_sphere(s[1]) * orc_sph(q * s[1]);
        double dd = s[0] + s[1] * (1.0 - 2.0 * p->extra[1]);
        double c = orc_sinc(q * dd);
        return fl * fl + n * fs * fs + 2.0 * n * fl * fs * c + n * (n - 1.0) * fs * fs * c * c;
    }
    }
    return 0.0;
}

/* Randomly oriented lamellae (Tables I-II, group C).  A flat sheet of area
 * A with the transverse contrast profile drho(z) scatters
 * |F1(Q_z)|^2 |S_A(Q_par)|^2; averaged over the directions of its normal,
 * the in-plane factor, whose integral over Q_par is (2 pi)^2 A, is picked up
 * at the two poles, giving 2 pi A |F1(q)|^2 / q^2.  Sheets of thickness
 * delta at volume fraction phi have phi/delta of area per volume, so
 *   dSigma/dOmega = phi (2 pi / delta) |F1(q)|^2 S(q) / q^2,
 * S the stacking factor per sheet (1 for isolated sheets).  Profiles are
 * symmetric: F1(q) = int drho(z) cos(q z) dz.  Here f2 is returned per unit
 * phi (the weight's phi / <V> with <V> = 1). */
static int lamellar(int kind) { return (kind >= 52 && kind <= 55) || kind == 60; }

/* Caille stacking of N sheets, repeat distance d, Caille parameter eta: the
 * mean-square displacement of sheets n apart grows as (eta d^2 / 2 pi^2)
 * (ln(pi n) + gamma), so S = 1 + 2 sum_{n<N} (1 - n/N) cos(q d n)
 * exp(-eta (q d / 2 pi)^2 (ln(pi n) + gamma)). */
static double caille_sq(double q, double d, int n, double eta)
{
    const double euler_gamma = 0.57721566490153286061;
    double a = eta * (q * d / (2.0 * ORC_PI)) * (q * d / (2.0 * ORC_PI)), st = 1.0;
    for (int k = 1; k < n; ++k)
        st += 2.0 * (1.0 - (double)k / n) * cos(q * d * k) * exp(-a * (log(ORC_PI * k) + euler_gamma));
    return st;
}

static double lamellar_iq(const orc_params* p, const double s[3], double q)
{
    double rt = p->sld[0] - p->sld[2], rh = p->sld[1] - p->sld[2];
    double f1, delta, st = 1.0;
    if (p->kind == 60) {
        /* a layer adsorbed on large particles (radius R = s0, contrast-matched
           cores; volume fraction phi): locally a flat sheet of excess
           thickness t = shell (the adsorbed amount over the layer's bulk
           density) with 3 phi / R of area per volume, smeared by a Gaussian of
           width sigma = extra[0]: phi (3 / R) 2 pi (drho t)^2 exp(-(q sigma)^2) / q^2 */
        double t = p->shell, sg = p->extra[0];
        return 3.0 / s[0] * 2.0 * ORC_PI * (rt * t) * (rt * t) * exp(-q * q * sg * sg) / (q * q);
    }
    if (p->kind == 52 || p->kind == 54) {
        /* tails over |z| < L_T (sld[0]), heads over L_T < |z| < L_T + L_H (sld[1]) */
        double lt = s[0], lh = s[1];
        delta = 2.0 * (lt + lh);
        f1 = 2.0 * ((rt - rh) * sin(q * lt) + rh * sin(q * (lt + lh))) / q;
    } else {
        /* one slab of thickness delta = size[0] (sld[0]) */
        delta = s[0];
        f1 = 2.0 * rt * sin(0.5 * q * delta) / q;
    }
    int n = (int)p->extra[0];
    if (p->kind == 53) st = caille_sq(q, s[1], n, p->extra[1]);
    if (p->kind == 54) st = caille_sq(q, s[2], n, p->extra[1]);
    if (p->kind == 55) {
        /* paracrystal: spacings independent Gaussians (mean d = size[1], width
           extra[1]), so sheets n apart are n d +- sqrt(n) sigma */
        double d = s[1], sg = p->extra[1];
        for (int k = 1; k < n; ++k)
            st += 2.0 * (1.0 - (double)k / n) * cos(q * d * k) * exp(-0.5 * k * q * q * sg * sg);
    }
    return 2.0 * ORC_PI / delta * f1 * f1 * st / (q * q);
}

/* Binary hard spheres (Tables I-II, group F): species 1 (radius s0,
 * sld[0]) and 2 (radius s1, sld[1]) at volume fractions phi - extra[0] and
 * extra[0]; number densities n_i = phi_i / V_i.  Their Percus-Yevick
 * partial structure factors from Baxter's factorisation for mixtures:
 * with diameters d_i, xi_m = (pi/6) sum_i n_i d_i^m and D = 1 - xi_3,
 *   Q_ij(r) = a_i/2 (r^2 - d_ij^2) + b_i (r - d_ij) on (d_i - d_j)/2 < r < d_ij,
 *   d_ij = (d_i + d_j)/2, a_i = (1 - xi_3 + 3 d_i xi_2)/D^2,
 *   b_i = -(3/2) d_i^2 xi_2 / D^2,
 *   Qhat_ij(q) = delta_ij - 2 pi sqrt(n_i n_j) int Q_ij(r) exp(i q r) dr,
 * and I - C(q) = Qhat(q)^H Qhat(q) (C_ij = sqrt(n_i n_j) c_ij), S = (I - C)^-1.
 * The cross-section sum_ij sqrt(n_i n_j) F_i F_j S_ij = v^T S v with
 * v_i = sqrt(n_i) F_i; returned per unit total number density (the weight's
 * phi / <V> is n_1 + n_2).  Integrals by composite Gauss-Legendre. */
static void bhs_qhat(const double d[2], const double n[2], double q, double re[2][2], double im[2][2])
{
    double xi2 = ORC_PI / 6.0 * (n[0] * d[0] * d[0] + n[1] * d[1] * d[1]);
    double xi3 = ORC_PI / 6.0 * (n[0] * d[0] * d[0] * d[0] + n[1] * d[1] * d[1] * d[1]);
    double dd = 1.0 - xi3;
    double gx[32], gw[32];
    orc_gauss_legendre(32, gx, gw);
    for (int i = 0; i < 2; ++i) {
        double a = (1.0 - xi3 + 3.0 * d[i] * xi2) / (dd * dd), b = -1.5 * d[i] * d[i] * xi2 / (dd * dd);
        for (int j = 0; j < 2; ++j) {
            double dij = 0.5 * (d[i] + d[j]), lo = 0.5 * (d[i] - d[j]);
            int npan = 1 + (int)(q * (dij - lo) / 2.0);
            double h = (dij - lo) / npan, cr = 0.0, ci = 0.0;
            for (int pnl = 0; pnl < npan; ++pnl) {
                for (int k = 0; k < 32; ++k) {
                    double r = lo + h * (pnl + 0.5 * (gx[k] + 1.0)), w = 0.5 * h * gw[k];
                    double qq = 0.5 * a * (r * r - dij * dij) + b * (r - dij);
                    cr += w * qq * cos(q * r);
                    ci += w * qq * sin(q * r);
                }
            }
            double f = 2.0 * ORC_PI * sqrt(n[i] * n[j]);
            re[i][j] = (i == j ? 1.0 : 0.0) - f * cr;
            im[i][j] = -f * ci;
        }
    }
}

/* I - C = Qhat^H Qhat, as a 2x2 complex matrix (re, im). */
void orc_bhs_inverse_s(double r1, double r2, double phi1, double phi2, double q, double re[4], double im[4])
{
    double d[2] = {2.0 * r1, 2.0 * r2};
    double n[2] = {phi1 / vol_sphere(r1), phi2 / vol_sphere(r2)};
    double qr[2][2], qi[2][2];
    bhs_qhat(d, n, q, qr, qi);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double sr = 0.0, si = 0.0;
            for (int l = 0; l < 2; ++l) { /* conj(Q_li) Q_lj */
                sr += qr[l][i] * qr[l][j] + qi[l][i] * qi[l][j];
                si += qr[l][i] * qi[l][j] - qi[l][i] * qr[l][j];
            }
            re[2 * i + j] = sr;
            im[2 * i + j] = si;
        }
}

static double binary_hs_f2(const orc_params* p, const double s[3], double q)
{
    double phi2 = p->extra[0], phi1 = p->phi - phi2;
    double n1 = phi1 / vol_sphere(s[0]), n2 = phi2 / vol_sphere(s[1]), nt = n1 + n2;
    double f1 = (p->sld[0] - p->sld[2]) * vol_sphere(s[0]) * orc_sph(q * s[0]);
    double f2 = (p->sld[1] - p->sld[2]) * vol_sphere(s[1]) * orc_sph(q * s[1]);
    double re[4], im[4];
    orc_bhs_inverse_s(s[0], s[1], phi1, phi2, q, re, im);
    /* S = (I - C)^-1 is real symmetric: invert the real part (the imaginary
       part vanishes, pinned in the tests) */
    double det = re[0] * re[3] - re[1] * re[2];
    double s11 = re[3] / det, s22 = re[0] / det, s12 = -re[1] / det;
    double v1 = sqrt(n1) * f1, v2 = sqrt(n2) * f2;
    return (v1 * v1 * s11 + 2.0 * v1 * v2 * s12 + v2 * v2 * s22) / nt;
}

/* Pringle (Tables I-II, group A): a plate of thickness t = s1 over the disc
 * x^2 + y^2 <= R^2 (R = s0; x, y along A, B) bent into the saddle
 * z = alpha x^2 - beta y^2 (alpha, beta = extra[0], extra[1] in 1/A):
 *   F = drho t sinc(Q_C t / 2) int_disc exp(i (Q_A x + Q_B y + Q_C z(x, y))) dA,
 * |F|^2 returned (the saddle is not centrosymmetric, F is complex).  The
 * disc integral in polar coordinates: r by n-point Gauss-Legendre on [0, R],
 * the angle by the 2n-point midpoint rule on [0, pi) (periodic), pairing
 * (x, y) with (-x, -y), which share z: 2 cos(Q_A x + Q_B y) exp(i Q_C z). */
static double pringle_f2(const orc_params* p, const double s[3], double qa, double qb, double qc)
{
    int n = p->quad_n, m = 2 * p->quad_n;
    double R = s[0], t = s[1], al = p->extra[0], be = p->extra[1];
    const double *gx, *gw;
    cap_nodes(n, &gx, &gw);
    double re = 0.0, im = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.5 * R * (gx[i] + 1.0), wr = 0.5 * R * gw[i] * r;
        for (int j = 0; j < m; ++j) {
            double ph = ORC_PI * (j + 0.5) / m, c = cos(ph), sn = sin(ph);
            double x = r * c, y = r * sn, z = al * x * x - be * y * y;
            double w = wr * ORC_PI / m * 2.0 * cos(qa * x + qb * y);
            re += w * cos(qc * z);
            im += w * sin(qc * z);
        }
    }
    double pre = (p->sld[0] - p->sld[2]) * t * orc_sinc(0.5 * qc * t);
    return pre * pre * (re * re + im * im);
}

/* Flexible cylinder with an elliptical cross-section (kind 62; named in
 * Table II of the paper, no formula given there).  The reading: a
 * semiflexible (wormlike) chain of contour length L = size[1] and Kuhn
 * length b = extra[0] whose local cross-section is an ellipse of semi-axes
 * R = size[0] and eps R (eps = extra[1]), uniform contrast drho; the chain
 * and the cross-section decouple,
 *   F^2 = (drho pi eps R^2 L)^2 P_chain(q) P_cs(q),
 * P_chain by Kholodenko's closed form for the wormlike chain (Macromolecules
 * 26, 4179 (1993)): with x = 3L/b,
 *   P_chain = (2/x) (I_1 - I_2/x),  I_n = int_0^x f(z) z^(n-1) dz,
 *   f(z) = sinh(E z)/(E sinh z), E = sqrt(1 - (q b/3)^2) for q b < 3, and
 *   f(z) = sin(F z)/(F sinh z), F = sqrt((q b/3)^2 - 1) above;
 * the integrals by n-point Gauss-Legendre on [0, x_e], x_e = min(x, 40/(1 -
 * E)) or min(x, 40) (the integrands fall as exp(-(1 - E) z) and exp(-z);
 * what is cut is below e^-40), with f written as exp((E - 1) z) (1 -
 * e^(-2Ez))/(E (1 - e^(-2z))) so that nothing overflows; P_cs the average of
 * [2 J1(q r)/(q r)]^2 over the angle psi in [0, pi/2] between q and the
 * ellipse's axes, r = R sqrt(sin^2 psi + eps^2 cos^2 psi), by the same
 * n-point rule; n = quad_n in every mode. */
static double flexcyl_chain(double q, double L, double b, int n)
{
    double gx[ORC_MAX_QUAD], gw[ORC_MAX_QUAD];
    orc_gauss_legendre(n, gx, gw);
    const double x = 3.0 * L / b, v = q * b / 3.0;
    const int below = v < 1.0;
    const double E = below ? sqrt(1.0 - v * v) : 0.0, F = below ? 0.0 : sqrt(v * v - 1.0);
    double xe = x;
    if (below && 1.0 - E > 0.0 && 40.0 / (1.0 - E) < xe) xe = 40.0 / (1.0 - E);
    if (!below && xe > 40.0) xe = 40.0;
    double i1 = 0.0, i2 = 0.0;
    for (int k = 0; k < n; ++k) {
        const double z = 0.5 * xe * (gx[k] + 1.0), wz = 0.5 * xe * gw[k];
        double f;
        if (below) {
            /* sinh(Ez)/(E sinh z) */
            const double num = E > 0.0 ? -expm1(-2.0 * E * z) / E : 2.0 * z;
            f = exp((E - 1.0) * z) * num / (-expm1(-2.0 * z));
        } else {
            /* sin(Fz)/F -> z at q b = 3 */
            f = 2.0 * (F > 0.0 ? sin(F * z) / F : z) * exp(-z) / (-expm1(-2.0 * z));
        }
        i1 += wz * f;
        i2 += wz * f * z;
    }
    return 2.0 / x * (i1 - i2 / x);
}

static double flexcyl_section(double q, double R, double eps, int n)
{
    double gx[ORC_MAX_QUAD], gw[ORC_MAX_QUAD];
    orc_gauss_legendre(n, gx, gw);
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        const double psi = 0.25 * ORC_PI * (gx[k] + 1.0);
        const double r = R * sqrt(sin(psi) * sin(psi) + eps * eps * cos(psi) * cos(psi));
        const double l = orc_lambda1(q * r);
        s += 0.5 * gw[k] * l * l;   /* (pi/4) w / (pi/2) */
    }
    return s;
}

double orc_flexcyl_chain(double q, double L, double b, int32_t n) { return flexcyl_chain(q, L, b, n); }
double orc_flexcyl_section(double q, double R, double eps, int32_t n) { return flexcyl_section(q, R, eps, n); }

static double flexcyl_f2(const orc_params* p, const double s[3], double q)
{
    const double R = s[0], L = s[1], b = p->extra[0], eps = p->extra[1];
    const double v = (p->sld[0] - p->sld[2]) * ORC_PI * eps * R * R * L;
    return v * v * flexcyl_chain(q, L, b, p->quad_n) * flexcyl_section(q, R, eps, p->quad_n);
}

/* Flexible cylinder (kind 63; named in Table I of the paper, no formula
 * given there): the same chain with a circular cross-section of radius
 * R = size[0], F^2 = (drho pi R^2 L)^2 P_chain(q) [2 J1(q R)/(q R)]^2. */
static double flexcyl_round_f2(const orc_params* p, const double s[3], double q)
{
    const double R = s[0], L = s[1], l = orc_lambda1(q * R);
    const double v = (p->sld[0] - p->sld[2]) * ORC_PI * R * R * L;
    return v * v * flexcyl_chain(q, L, p->extra[0], p->quad_n) * l * l;
}

/* The squared amplitude of one particle, or for the micelle its scattering
 * per particle (it has incoherent chain terms); for the shape-independent
 * models their cross-section in 1/cm. */
static double form_f2(const orc_params* p, const double s[3], double q, double qa, double qb, double qc)
{
    if (shape_independent(p->kind)) return shape_independent_iq(p, s, q);
    if (lamellar(p->kind)) return lamellar_iq(p, s, q);
    if (p->kind == 59) return binary_hs_f2(p, s, q);
    if (p->kind == 61) return pringle_f2(p, s, qa, qb, qc);
    if (p->kind == 62) return flexcyl_f2(p, s, q);
    if (p->kind == 63) return flexcyl_round_f2(p, s, q);
    if (p->kind == 8) return micelle_f2(s, p->sld, p->extra, q);
    if ((p->kind >= 25 && p->kind <= 28) || p->kind == 57 || p->kind == 58) return sphere_family_f2(p, s, q);
    if (p->kind == 45) {
        /* stacked disks: N = extra[0] disks, spacing d = s1 + 2 shell along C with
           Gaussian spread extra[1]: F^2 times 1 + (2/N) sum_k (N - k) cos(k d Q_C)
           exp(-k (Q_C sigma)^2 / 2) */
        double f = amplitude(p->kind, s, p->shell, p->sld, p->extra, q, qa, qb, qc, p->quad_n);
        int n = (int)p->extra[0];
        double d = s[1] + 2.0 * p->shell, sg = p->extra[1], st = 1.0;
        for (int k = 1; k < n; ++k)
            st += 2.0 / n * (n - k) * cos(k * d * qc) * exp(-0.5 * k * qc * qc * sg * sg);
        return f * f * st;
    }
    if (p->kind >= 46 && p->kind <= 48) {
        /* paracrystals (Matsuoka): spheres on a cubic lattice whose primitive
           vectors a_k (nearest-neighbour distance D = s1) are the particle axes'
           combinations; each direction a one-dimensional paracrystal with
           Gaussian distortion g D: Z_k = (1 - e^2) / (1 - 2 e cos(Q.a_k) + e^2),
           e = exp(-(q g D)^2 / 2); the lattice factor is the product */
        double f = amplitude(p->kind, s, p->shell, p->sld, p->extra, q, qa, qb, qc, p->quad_n);
        double dd = s[1], e = exp(-0.5 * q * q * p->extra[0] * p->extra[0] * dd * dd);
        double v[3][3];
        if (p->kind == 46) {          /* simple cubic: a = D */
            double b[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
            memcpy(v, b, sizeof(v));
            for (int k = 0; k < 3; ++k) for (int j = 0; j < 3; ++j) v[k][j] *= dd;
        } else if (p->kind == 47) {   /* bcc: a = 2 D / sqrt 3, vectors (a/2)(-1,1,1) ... */
            double b[3][3] = {{-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
            memcpy(v, b, sizeof(v));
            for (int k = 0; k < 3; ++k) for (int j = 0; j < 3; ++j) v[k][j] *= dd / sqrt(3.0);
        } else {                      /* fcc: a = sqrt 2 D, vectors (a/2)(0,1,1) ... */
            double b[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
            memcpy(v, b, sizeof(v));
            for (int k = 0; k < 3; ++k) for (int j = 0; j < 3; ++j) v[k][j] *= dd / sqrt(2.0);
        }
        double z = 1.0;
        for (int k = 0; k < 3; ++k) {
            double x = qa * v[k][0] + qb * v[k][1] + qc * v[k][2];
            z *= (1.0 - e * e) / (1.0 - 2.0 * e * cos(x) + e * e);
        }
        return f * f * z;
    }
    if (p->kind == 38 || p->kind == 39) {
        /* blocks: a sphere (38) or a core-shell sphere (39) of radius size[0]
           (core), shell; fractal: xi = size[1], D = extra[1] */
        double f = p->kind == 38 ? (p->sld[0] - p->sld[2]) * vol_sphere(s[0]) * orc_sph(q * s[0])
                                 : amplitude(1, s, p->shell, p->sld, p->extra, q, 0.0, 0.0, 0.0, p->quad_n);
        double r0 = p->kind == 38 ? s[0] : s[0] + p->shell;
        return f * f * teixeira_sq(q, r0, s[1], p->extra[1]);
    }
    double f = amplitude(p->kind, s, p->shell, p->sld, p->extra, q, qa, qb, qc, p->quad_n);
    return f * f;
}

/* Orientation matters (the particles from 2 to 12 but the micelle). */
static int anisotropic(int kind) { return (kind >= 2 && kind != 8 && kind <= 12) || (kind >= 41 && kind <= 48) || kind == 51 || kind == 56 || kind == 61; }

/* Sizes scaled by the relative size draw y according to the mask. */
static void scaled_sizes(const orc_params* p, double y, double s[3])
{
    for (int k = 0; k < 3; ++k) s[k] = (p->poly_mask >> k & 1) ? p->size[k] * y : p->size[k];
}

/* Schulz moments <y^k> = prod_{j=0}^{k-1} (a + j)/a with a = 1/p^2. */
static double schulz_moment(double p, int k)
{
    if (p <= 0.0) return 1.0;
    double a = 1.0 / (p * p), m = 1.0;
    for (int j = 0; j < k; ++j) m *= (a + j) / a;
    return m;
}

/* Moments <y^k> of N(1, p^2) restricted to y > 0 (mean mu = 1, sd s = p,
 * alpha = -1/p, Z = 1 - Phi(alpha)): m_0 = 1, m_1 = mu + s phi(alpha)/Z and,
 * the lower bound being 0, m_k = mu m_{k-1} + (k - 1) s^2 m_{k-2} (k >= 2). */
static double truncnorm_moment(double p, int k)
{
    if (p <= 0.0) return 1.0;
    double alpha = -1.0 / p;
    double z = 1.0 - normal_cdf(alpha);
    double dens = exp(-0.5 * alpha * alpha) / sqrt(2.0 * ORC_PI);
    double m0 = 1.0, m1 = 1.0 + p * dens / z;
    if (k == 0) return m0;
    for (int j = 2; j <= k; ++j) {
        double m2 = m1 + (j - 1) * p * p * m0;
        m0 = m1;
        m1 = m2;
    }
    return m1;
}

static double size_moment(const orc_params* p, int k)
{
    return p->poly_kind == 1 ? truncnorm_moment(p->poly, k) : schulz_moment(p->poly, k);
}

double orc_size_moment(const orc_params* p, int32_t k) { return size_moment(p, k); }

/* E[prod_{i<n} (alpha_i y^b_i + beta_i)] over the size draw y, expanded into
 * the moments <y^k> term by term (one term per subset of the factors). */
static double prod_moment(const orc_params* p, const double* alpha, const double* beta, const int* b, int n)
{
    double total = 0.0;
    for (int mask = 0; mask < (1 << n); ++mask) {
        double c = 1.0;
        int k = 0;
        for (int i = 0; i < n; ++i) {
            if (mask >> i & 1) {
                c *= alpha[i];
                k += b[i];
            } else {
                c *= beta[i];
            }
        }
        total += c * size_moment(p, k);
    }
    return total;
}

/* Any independent width set. */
static int sep_on(const orc_params* p)
{
    return p->poly_sep[0] > 0.0 || p->poly_sep[1] > 0.0 || p->poly_sep[2] > 0.0;
}

/* Number-averaged particle volume <V> (n = phi/<V>). */
double orc_mean_volume(const orc_params* p)
{
    const double* s = p->size;
    if (sep_on(p)) {
        /* independent draws of the sizes: V is a product of powers of the
           sizes for the models that take them, so <V> is V times the
           moments <y_k^e_k>, e_k the power of size k in V */
        int e[3] = {0, 0, 0};
        double v;
        switch (p->kind) {
        case 0: v = vol_sphere(s[0]); e[0] = 3; break;
        case 2: v = ORC_PI * s[0] * s[0] * s[1]; e[0] = 2; e[1] = 1; break;
        case 3: v = 4.0 / 3.0 * ORC_PI * s[0] * s[1] * s[2]; e[0] = e[1] = e[2] = 1; break;
        case 4: v = s[0] * s[1] * s[2]; e[0] = e[1] = e[2] = 1; break;
        case 41: v = ORC_PI * s[0] * s[1] * s[2]; e[0] = e[1] = e[2] = 1; break;
        default: return NAN;
        }
        for (int k = 0; k < 3; ++k) v *= truncnorm_moment(p->poly_sep[k], e[k]);
        return v;
    }
    int b0 = p->poly_mask & 1, b1 = p->poly_mask >> 1 & 1, b2 = p->poly_mask >> 2 & 1;
    switch (p->kind) {
    case 0:
        return vol_sphere(s[0]) * size_moment(p, b0 ? 3 : 0);
    case 1: {
        double r = s[0], t = p->shell;
        if (!b0) return vol_sphere(r + t);
        return 4.0 / 3.0 * ORC_PI * (r * r * r * size_moment(p, 3)
                                      + 3.0 * r * r * t * size_moment(p, 2)
                                      + 3.0 * r * t * t * size_moment(p, 1) + t * t * t);
    }
    case 2:
        return ORC_PI * s[0] * s[0] * s[1] * size_moment(p, 2 * b0 + b1);
    case 3:
        return 4.0 / 3.0 * ORC_PI * s[0] * s[1] * s[2] * size_moment(p, b0 + b1 + b2);
    case 4:
        return s[0] * s[1] * s[2] * size_moment(p, b0 + b1 + b2);
    case 5:
    case 6: /* all three sizes scale together (or none): V(y) = V(1) y^3 */
        return (ORC_PI * s[0] * s[0] * s[1] + caps_volume(s, p->kind == 5))
             * size_moment(p, p->poly_mask == 7 ? 3 : 0);
    case 51:
        return superball_volume(s[0], p->extra[0]) * size_moment(p, b0 ? 3 : 0);
    case 52: case 53: case 54: case 55: case 60: /* lamellae, adsorbed layers: f2 is per unit volume fraction */
        return 1.0;
    case 25: /* fuzzy sphere: the sphere's volume */
        return vol_sphere(s[0]) * size_moment(p, b0 ? 3 : 0);
    case 26: { /* vesicle: the shell, 4/3 pi ((R y + t)^3 - (R y)^3) */
        double al[3] = {s[0], s[0], s[0]}, be[3] = {p->shell, p->shell, p->shell}, z[3] = {0.0, 0.0, 0.0};
        int bb[3] = {b0, b0, b0};
        return 4.0 / 3.0 * ORC_PI * (prod_moment(p, al, be, bb, 3) - prod_moment(p, al, z, bb, 3));
    }
    case 27: { /* multilayer vesicle: the n shells (monodisperse) */
        double v = 0.0;
        for (int k = 0; k < (int)p->extra[0]; ++k) {
            double ri = s[0] + k * (p->shell + s[1]);
            v += vol_sphere(ri + p->shell) - vol_sphere(ri);
        }
        return v;
    }
    case 38: /* fractal aggregate: the blocks' volume */
        return vol_sphere(s[0]) * size_moment(p, b0 ? 3 : 0);
    case 39: {
        double r = s[0], t = p->shell;
        if (!b0) return vol_sphere(r + t);
        return 4.0 / 3.0 * ORC_PI * (r * r * r * size_moment(p, 3) + 3.0 * r * r * t * size_moment(p, 2)
                                      + 3.0 * r * t * t * size_moment(p, 1) + t * t * t);
    }
    case 59: { /* binary hard spheres: total volume fraction over total number density */
        double phi2 = p->extra[0], phi1 = p->phi - phi2;
        return p->phi / (phi1 / vol_sphere(s[0]) + phi2 / vol_sphere(s[1]));
    }
    case 62: /* flexible elliptical cylinder: pi eps R^2 L */
        return ORC_PI * p->extra[1] * s[0] * s[0] * s[1]
             * size_moment(p, (p->poly_mask & 1 ? 2 : 0) + (p->poly_mask & 2 ? 1 : 0));
    case 63: /* flexible cylinder: pi R^2 L */
        return ORC_PI * s[0] * s[0] * s[1]
             * size_moment(p, (p->poly_mask & 1 ? 2 : 0) + (p->poly_mask & 2 ? 1 : 0));
    case 61: /* pringle: the plate's area times its thickness */
        return ORC_PI * s[0] * s[0] * s[1] * size_moment(p, (p->poly_mask & 1 ? 2 : 0) + (p->poly_mask & 2 ? 1 : 0));
    case 58: /* pearl necklace: N pearls and N - 1 rods */
        return p->extra[0] * vol_sphere(s[0]) * size_moment(p, (p->poly_mask & 1) ? 3 : 0)
             + (p->extra[0] - 1.0) * ORC_PI * 0.25 * s[2] * s[2] * s[1];
    case 57: /* raspberry: the large sphere and its N small ones */
        return vol_sphere(s[0]) * size_moment(p, (p->poly_mask & 1) ? 3 : 0) + p->extra[0] * vol_sphere(s[1]);
    case 28: /* linear pearls: n spheres */
        return p->extra[0] * vol_sphere(s[0]) * size_moment(p, b0 ? 3 : 0);
    case 8: /* N chains, each a core block and a corona chain */
        return p->extra[0] * (p->extra[1] + p->extra[2]);
    case 9: { /* pi L ((R + t)^2 - R^2) = pi (L y^b1)(2 R t y^b0 + t^2) */
        double al[2] = {s[1], 2.0 * s[0] * p->shell}, be[2] = {0.0, p->shell * p->shell};
        int bb[2] = {b1, b0};
        return ORC_PI * prod_moment(p, al, be, bb, 2);
    }
    case 10: { /* the outer cylinder: pi (R + t)^2 (L + 2 t_face) */
        double al[3] = {s[0], s[0], s[1]}, be[3] = {p->shell, p->shell, 2.0 * p->extra[0]};
        int bb[3] = {b0, b0, b1};
        return ORC_PI * prod_moment(p, al, be, bb, 3);
    }
    case 11: { /* the outer ellipsoid: 4/3 pi (a + t)(b + t)(c + t) */
        double be[3] = {p->shell, p->shell, p->shell};
        int bb[3] = {b0, b1, b2};
        return 4.0 / 3.0 * ORC_PI * prod_moment(p, s, be, bb, 3);
    }
    case 44: { /* the outer elliptic cylinder pi (R + t)(x R + t)(L + 2 t_f) */
        double xr = p->extra[2];
        double al[3] = {s[0], xr * s[0], s[1]}, be[3] = {p->shell, p->shell, 2.0 * p->extra[0]};
        int bb[3] = {b0, b0, b1};
        return ORC_PI * prod_moment(p, al, be, bb, 3);
    }
    case 56: { /* core and belt pi (R + t)(x R + t) L plus the two faces 2 pi x R^2 t_f */
        double xr = p->extra[2];
        double al[3] = {s[0], xr * s[0], s[1]}, be[3] = {p->shell, p->shell, 0.0};
        int bb[3] = {b0, b0, b1};
        double af[2] = {s[0], xr * s[0]}, bf[2] = {0.0, 0.0};
        int cf[2] = {b0, b0};
        return ORC_PI * prod_moment(p, al, be, bb, 3) + 2.0 * ORC_PI * p->extra[0] * prod_moment(p, af, bf, cf, 2);
    }
    case 45: { /* one disk: pi R^2 (core + two layers) */
        double al[3] = {s[0], s[0], s[1]}, be[3] = {0.0, 0.0, 2.0 * p->shell};
        int bb[3] = {b0, b0, b1};
        return ORC_PI * prod_moment(p, al, be, bb, 3);
    }
    case 46:
    case 47:
    case 48:
        return vol_sphere(s[0]) * size_moment(p, b0 ? 3 : 0);
    case 41: /* pi a b L */
        return ORC_PI * s[0] * s[1] * s[2] * size_moment(p, b0 + b1 + b2);
    case 42: { /* the outer cylinder pi (R y^b0 + t)^2 (L y^b1 + 2 t_f) */
        double al[3] = {s[0], s[0], s[1]}, be[3] = {p->shell, p->shell, 2.0 * p->extra[0]};
        int bb[3] = {b0, b0, b1};
        return ORC_PI * prod_moment(p, al, be, bb, 3);
    }
    case 43: { /* core plus the six face slabs */
        double z[3] = {0.0, 0.0, 0.0};
        double a0[3] = {s[0], s[1], s[2]};
        int bb[3] = {b0, b1, b2};
        double v = prod_moment(p, a0, z, bb, 3);
        double pa[2] = {s[1], s[2]}, pb[2] = {s[0], s[2]}, pc[2] = {s[0], s[1]};
        int ba[2] = {b1, b2}, bbb[2] = {b0, b2}, bc[2] = {b0, b1};
        v += 2.0 * p->extra[0] * prod_moment(p, pa, z, ba, 2) + 2.0 * p->extra[1] * prod_moment(p, pb, z, bbb, 2)
           + 2.0 * p->extra[2] * prod_moment(p, pc, z, bc, 2);
        return v;
    }
    case 12: { /* box minus cavity (monodisperse) */
        double t2 = 2.0 * p->shell;
        return s[0] * s[1] * s[2] - (s[0] - t2) * (s[1] - t2) * (s[2] - t2);
    }
    case 7: /* wall volume: thickness times the surface 2 (AB + BC + AC) */
        return 2.0 * p->shell
             * (s[0] * s[1] * size_moment(p, b0 + b1) + s[1] * s[2] * size_moment(p, b1 + b2)
                + s[0] * s[2] * size_moment(p, b0 + b2));
    }
    return 0.0;
}

/* Particle axes from the angles (theta, phi, Psi): R = Rz(phi) Ry(theta)
 * Rz(Psi); C = R z (theta, phi give the C axis), A = R x, B = R y (Psi turns
 * A, B about C), as the orientation angles are defined with Eq. (6).       */
static void particle_axes(const double ang[3], double A[3], double B[3], double C[3])
{
    double ct = cos(ang[0]), st = sin(ang[0]);
    double cp = cos(ang[1]), sp = sin(ang[1]);
    double cs = cos(ang[2]), ss = sin(ang[2]);
    A[0] = cp * ct * cs - sp * ss;
    A[1] = sp * ct * cs + cp * ss;
    A[2] = -st * cs;
    B[0] = -cp * ct * ss - sp * cs;
    B[1] = -sp * ct * ss + cp * cs;
    B[2] = st * ss;
    C[0] = cp * st;
    C[1] = sp * st;
    C[2] = ct;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_n with
 * the three-term recurrence (n P_n = (2n-1) x P_{n-1} - (n-1) P_{n-2}).     */
void orc_gauss_legendre(int32_t n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute the derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Schulz probability density of y (mean 1, relative width p). */
static double schulz_pdf(double y, double p)
{
    double a = 1.0 / (p * p);
    if (y <= 0.0) return 0.0;
    return exp(a * log(a) + (a - 1.0) * log(y) - a * y - lgamma(a));
}

/* Density of the positive Gaussian (up to its constant normalisation: the
 * quadrature weights are normalised to sum 1). */
static double truncnorm_pdf(double y, double p)
{
    if (y <= 0.0) return 0.0;
    double d = (y - 1.0) / p;
    return exp(-0.5 * d * d);
}

static double size_pdf(const orc_params* p, double y)
{
    return p->poly_kind == 1 ? truncnorm_pdf(y, p->poly) : schulz_pdf(y, p->poly);
}

/* Exact average <F^2>(q) that replaces the per-event size and orientation
 * draws in quadrature mode: Schulz size average by quad_n Gauss-Legendre
 * nodes on y in [max(0, 1-6p), 1+8p] (weights normalised to the quadrature
 * of the density) and, for isotropic orientation, the orientation average
 *   <g> = int_0^1 dmu g(mu)                     (one symmetry axis, Eq. (7))
 *   <g> = (2/pi) int_0^1 dmu int_0^(pi/2) dbeta g(mu, beta)   (Eq. (6))
 * with Q_C = q mu, Q_A = q sqrt(1-mu^2) cos beta, Q_B = q sqrt(1-mu^2) sin beta.
 * Fixed orientation evaluates the amplitude at the given Q vector.          */
static double pq_avg_nodes(const orc_params* p, double q, const double qvec[3],
                           const double* gx, const double* gw)
{
    int n = p->quad_n;

    /* size nodes */
    int ny = 1;
    double ys[ORC_MAX_QUAD], yw[ORC_MAX_QUAD];
    ys[0] = 1.0;
    yw[0] = 1.0;
    if (p->poly > 0.0) {
        /* Schulz: [1 - 6p, 1 + 8p] (right-skewed); Gaussian: 1 -+ 6p */
        double lo = 1.0 - 6.0 * p->poly, hi = 1.0 + (p->poly_kind == 1 ? 6.0 : 8.0) * p->poly;
        if (lo < 0.0) lo = 0.0;
        double norm = 0.0;
        ny = n;
        for (int j = 0; j < n; ++j) {
            ys[j] = 0.5 * (hi - lo) * gx[j] + 0.5 * (hi + lo);
            yw[j] = 0.5 * (hi - lo) * gw[j] * size_pdf(p, ys[j]);
            norm += yw[j];
        }
        for (int j = 0; j < n; ++j) yw[j] /= norm;
    }

    int aniso = anisotropic(p->kind);
    int iso = aniso && p->orient_kind == 2;
    /* a spheroid (a = b, scaled alike) needs only the angle to its C axis */
    int one_axis = (p->kind == 2 || p->kind == 5 || p->kind == 6 || p->kind == 9 || p->kind == 10
                    || p->kind == 42 || p->kind == 45)
                || ((p->kind == 3 || p->kind == 11) && p->size[0] == p->size[1]
                    && (p->poly_mask & 1) == (p->poly_mask >> 1 & 1));
    double A[3], B[3], C[3];
    particle_axes(p->orient_mean, A, B, C);

    double total = 0.0;
    for (int j = 0; j < ny; ++j) {
        double s[3];
        scaled_sizes(p, ys[j], s);
        double avg = 0.0;
        if (!aniso) {
            avg = form_f2(p, s, q, 0.0, 0.0, 0.0);
        } else if (!iso) {
            double qa = qvec[0] * A[0] + qvec[1] * A[1] + qvec[2] * A[2];
            double qb = qvec[0] * B[0] + qvec[1] * B[1] + qvec[2] * B[2];
            double qc = qvec[0] * C[0] + qvec[1] * C[1] + qvec[2] * C[2];
            avg = form_f2(p, s, q, qa, qb, qc);
        } else if (one_axis) {
            for (int i = 0; i < n; ++i) {
                double mu = 0.5 * (gx[i] + 1.0);
                double st = sqrt(1.0 - mu * mu);
                /* A-B plane direction is irrelevant for a symmetric particle */
                avg += 0.5 * gw[i] * form_f2(p, s, q, q * st, 0.0, q * mu);
            }
        } else {
            for (int i = 0; i < n; ++i) {
                double mu = 0.5 * (gx[i] + 1.0);
                double st = sqrt(1.0 - mu * mu);
                for (int k = 0; k < n; ++k) {
                    double beta = 0.25 * ORC_PI * (gx[k] + 1.0);
                    double qa = q * st * cos(beta), qb = q * st * sin(beta), qc = q * mu;
                    avg += 0.25 * gw[i] * gw[k] * form_f2(p, s, q, qa, qb, qc);
                }
            }
        }
        total += yw[j] * avg;
    }
    return total;
}

double orc_pq_avg(const orc_params* p, double q, const double qvec[3])
{
    if (p->quad_n < 1 || p->quad_n > ORC_MAX_QUAD) return NAN;
    double gx[ORC_MAX_QUAD], gw[ORC_MAX_QUAD];
    orc_gauss_legendre(p->quad_n, gx, gw);
    return pq_avg_nodes(p, q, qvec, gx, gw);
}

/* Amplitude at a single explicit event, for tests: sizes scaled by y,
 * orientation angles ang, scattering vector qvec (|qvec| = q). */
double orc_amplitude(const orc_params* p, double q, const double qvec[3], double y,
                     const double ang[3])
{
    double s[3], A[3], B[3], C[3];
    scaled_sizes(p, y, s);
    particle_axes(ang, A, B, C);
    double qa = qvec[0] * A[0] + qvec[1] * A[1] + qvec[2] * A[2];
    double qb = qvec[0] * B[0] + qvec[1] * B[1] + qvec[2] * B[2];
    double qc = qvec[0] * C[0] + qvec[1] * C[1] + qvec[2] * C[2];
    return amplitude(p->kind, s, p->shell, p->sld, p->extra, q, qa, qb, qc, p->quad_n);
}

/* The squared amplitude at one event with the particle's sizes given. */
static double form_f2_sizes(const orc_params* p, const double s[3], double q, const double qvec[3],
                            const double ang[3])
{
    double A[3], B[3], C[3];
    particle_axes(ang, A, B, C);
    double qa = qvec[0] * A[0] + qvec[1] * A[1] + qvec[2] * A[2];
    double qb = qvec[0] * B[0] + qvec[1] * B[1] + qvec[2] * B[2];
    double qc = qvec[0] * C[0] + qvec[1] * C[1] + qvec[2] * C[2];
    return form_f2(p, s, q, qa, qb, qc);
}

/* The squared amplitude (micelle: scattering per particle) at one explicit
 * event, as orc_amplitude. */
double orc_form_f2(const orc_params* p, double q, const double qvec[3], double y, const double ang[3])
{
    double s[3], A[3], B[3], C[3];
    scaled_sizes(p, y, s);
    particle_axes(ang, A, B, C);
    double qa = qvec[0] * A[0] + qvec[1] * A[1] + qvec[2] * A[2];
    double qb = qvec[0] * B[0] + qvec[1] * B[1] + qvec[2] * B[2];
    double qc = qvec[0] * C[0] + qvec[1] * C[1] + qvec[2] * C[2];
    return form_f2(p, s, q, qa, qb, qc);
}

/* ------------------------------------------------------------------------ */
/* The tracer. */

typedef struct {
    const orc_params* p;
    double* tab_size;   /* Schulz knots (or NULL) */
    double* tab_norm;   /* normal knots (or NULL) */
    double one_minus_cos; /* 1 - cos(alpha) */
    double prefactor;   /* solid angle * phi / <V> */
    int third_block;    /* block 2 is used */
    int fourth_block;   /* block 3 is used (independent draws of sizes 1, 2) */
    double* tab_sep[3]; /* positive-Gaussian knots per independent width */
    double gx[ORC_MAX_QUAD], gw[ORC_MAX_QUAD]; /* quadrature nodes (mode 1) */
} orc_ctx;


typedef struct {
    int32_t pixel; /* -1: no tally */
    double w;
    double q;
    /* intermediate values, for diagnostics: the independent size factors
       ysep (1 where a size has no width of its own) */
    double qv[3], y, ang[3], len, ysep[3];
} orc_event;

static int ctx_init(orc_ctx* cx, const orc_params* p)
{
    memset(cx, 0, sizeof(*cx));
    cx->p = p;
    int M = p->table_size;
    if (p->mode == 0 && p->poly > 0.0) {
        cx->tab_size = (double*)malloc(sizeof(double) * M);
        size_table(p, cx->tab_size);
    }
    if (p->mode == 0 && p->orient_kind == 1) {
        cx->tab_norm = (double*)malloc(sizeof(double) * M);
        orc_table_normal(M, cx->tab_norm);
    }
    for (int k = 0; k < 3; ++k) {
        if (p->mode == 0 && p->poly_sep[k] > 0.0) {
            cx->tab_sep[k] = (double*)malloc(sizeof(double) * M);
            orc_table_truncnorm(M, p->poly_sep[k], cx->tab_sep[k]);
        }
    }
    double sh = sin(0.5 * p->cone_alpha);
    cx->one_minus_cos = 2.0 * sh * sh;
    /* n F^2 in 1/Angstrom; a shape-independent model gives dSigma/dOmega in
     * 1/cm directly (1e-8 per Angstrom) */
    cx->prefactor = 2.0 * ORC_PI * cx->one_minus_cos
                  * (shape_independent(p->kind) ? 1e-8 : p->phi / orc_mean_volume(p));
    cx->third_block = (p->mode == 0) && (p->poly > 0.0 || p->orient_kind != 0 || sep_on(p));
    cx->fourth_block = (p->mode == 0) && (p->poly_sep[1] > 0.0 || p->poly_sep[2] > 0.0);
    if (p->mode >= 1) {
        if (p->quad_n < 1 || p->quad_n > ORC_MAX_QUAD) return -1;
        orc_gauss_legendre(p->quad_n, cx->gx, cx->gw);
    }
    return 0;
}

static void ctx_free(orc_ctx* cx)
{
    free(cx->tab_size);
    free(cx->tab_norm);
    for (int k = 0; k < 3; ++k) free(cx->tab_sep[k]);
}

/* The neutron guide (an upstream instrument component of the paper's
 * KWS-1 simulation, Methods): a straight rectangular channel of length L,
 * width w and height h whose exit lies a gap g upstream of the source
 * aperture, its walls supermirrors of reflectivity (the usual form for
 * them)
 *   R(Q) = R0                                                  Q <= Qc,
 *   R(Q) = R0/2 (1 - tanh((Q - m Qc)/W)) (1 - alpha (Q - Qc))  Q > Qc,
 * (0 where that is negative), Q = 4 pi sin(theta)/lambda for the grazing
 * angle theta.  The moderator fills the guide's entrance.  A neutron that
 * reaches the source aperture at src flying along ki is followed back: to
 * the exit plane (it must pass inside the exit, else nothing feeds it:
 * weight 0), then inside the guide wall by wall, reflecting off each wall
 * it meets, until it reaches the entrance plane; its weight is the product
 * of the reflectivities met. */
static double guide_reflectivity(const orc_params* p, double q)
{
    const double r0 = p->guide[5], qc = p->guide[6], alpha = p->guide[7], wc = p->guide[8], m = p->guide[4];
    if (q <= qc) return r0;
    double r = 0.5 * r0 * (1.0 - tanh((q - m * qc) / wc)) * (1.0 - alpha * (q - qc));
    return r > 0.0 ? r : 0.0;
}

static double guide_weight(const orc_params* p, const double src[3], const double ki[3], double lambda)
{
    if (!(p->guide[0] > 0.0)) return 1.0;
    const double len = p->guide[0], hw = 0.5 * p->guide[1], hh = 0.5 * p->guide[2], gap = p->guide[3];
    /* back along -ki from the aperture to the exit plane z_src - gap */
    double t = gap / ki[2];
    double x = src[0] - t * ki[0], y = src[1] - t * ki[1], z = src[2] - gap;
    if (fabs(x) > hw || fabs(y) > hh) return 0.0;
    double dx = -ki[0], dy = -ki[1], dz = -ki[2];
    const double z_in = src[2] - gap - len;
    const double qx = 4.0 * ORC_PI * fabs(ki[0]) / lambda, qy = 4.0 * ORC_PI * fabs(ki[1]) / lambda;
    const double rx = guide_reflectivity(p, qx), ry = guide_reflectivity(p, qy);
    double w = 1.0;
    for (int step = 0; step < 1000000; ++step) {
        double tz = (z_in - z) / dz;
        double tx = dx > 0.0 ? (hw - x) / dx : dx < 0.0 ? (-hw - x) / dx : INFINITY;
        double ty = dy > 0.0 ? (hh - y) / dy : dy < 0.0 ? (-hh - y) / dy : INFINITY;
        if (tz <= tx && tz <= ty) return w;       /* the entrance */
        if (tx <= ty) {
            x += tx * dx; y += tx * dy; z += tx * dz;
            x = dx > 0.0 ? hw : -hw;
            dx = -dx;
            w *= rx;
        } else {
            x += ty * dx; y += ty * dy; z += ty * dz;
            y = dy > 0.0 ? hh : -hh;
            dy = -dy;
            w *= ry;
        }
    }
    return w;
}

double orc_guide_weight(const orc_params* p, const double src[3], const double ki[3], double lambda)
{
    return guide_weight(p, src, ki, lambda);
}

static orc_event trace_one(const orc_ctx* cx, uint64_t i, uint64_t seed, uint32_t e)
{
    const orc_params* p = cx->p;
    orc_event ev;
    memset(&ev, 0, sizeof(ev));
    ev.pixel = -1;
    ev.ysep[0] = ev.ysep[1] = ev.ysep[2] = 1.0;
    uint32_t r0[4], r1[4], r2[4] = {0, 0, 0, 0}, r3[4] = {0, 0, 0, 0};
    neutron_block(seed, i, 0, e, r0);
    neutron_block(seed, i, 1, e, r1);
    if (cx->third_block) neutron_block(seed, i, 2, e, r2);
    if (cx->fourth_block) neutron_block(seed, i, 3, e, r3);
    double u[16];
    for (int k = 0; k < 4; ++k) {
        u[k] = orc_uniform(r0[k]);
        u[4 + k] = orc_uniform(r1[k]);
        u[8 + k] = orc_uniform(r2[k]);
        u[12 + k] = orc_uniform(r3[k]);
    }

    /* source point and slit point; the neutron flies from one to the other */
    double src[3] = {(u[0] - 0.5) * p->src_w, (u[1] - 0.5) * p->src_h, p->src_z};
    double slt[3] = {(u[2] - 0.5) * p->slit_w, (u[3] - 0.5) * p->slit_h, p->slit_z};
    double d[3] = {slt[0] - src[0], slt[1] - src[1], slt[2] - src[2]};
    double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double ki[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
    double lambda = p->lambda0 * (1.0 + p->dlambda_rel * (2.0 * u[4] - 1.0));
    double k = 2.0 * ORC_PI / lambda; /* 1/Angstrom */

    /* the slab sample, centred at the origin: entry and exit along the ray */
    double half[3] = {0.5 * p->sample_w, 0.5 * p->sample_h, 0.5 * p->sample_d};
    double s_in = 0.0, s_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (ki[a] != 0.0) {
            double t1 = (-half[a] - src[a]) / ki[a];
            double t2 = (half[a] - src[a]) / ki[a];
            double tl = t1 < t2 ? t1 : t2, th = t1 < t2 ? t2 : t1;
            if (tl > s_in) s_in = tl;
            if (th < s_out) s_out = th;
        } else if (fabs(src[a]) > half[a]) {
            s_out = -1.0;
        }
    }
    ev.q = 0.0;
    if (!(s_out > s_in)) return ev;
    double len = s_out - s_in; /* metres */
    double s = s_in + u[5] * len;
    double rs[3] = {src[0] + s * ki[0], src[1] + s * ki[1], src[2] + s * ki[2]};

    /* outgoing direction uniform in solid angle inside the cone of half-angle
     * alpha about ki; basis orthogonal to ki after Duff et al., "Building an
     * Orthonormal Basis, Revisited", JCGT 6(1), 2017 */
    double t = u[6] * cx->one_minus_cos;
    double c2 = 1.0 - t;
    double s2 = sqrt(t * (2.0 - t));
    double psi = 2.0 * ORC_PI * u[7];
    double cps = cos(psi), sps = sin(psi);
    double sg = copysign(1.0, ki[2]);
    double aa = -1.0 / (sg + ki[2]);
    double bb = ki[0] * ki[1] * aa;
    double e1[3] = {1.0 + sg * ki[0] * ki[0] * aa, sg * bb, -sg * ki[0]};
    double e2[3] = {bb, sg + ki[1] * ki[1] * aa, -ki[1]};
    double perp[3], kf[3], qv[3];
    for (int a = 0; a < 3; ++a) {
        perp[a] = cps * e1[a] + sps * e2[a];
        kf[a] = c2 * ki[a] + s2 * perp[a];
        qv[a] = k * (-t * ki[a] + s2 * perp[a]);
    }
    double q = k * sqrt(2.0 * t);
    ev.q = q;

    /* size and orientation of the particle met by this neutron */
    double y = 1.0;
    double ang[3] = {p->orient_mean[0], p->orient_mean[1], p->orient_mean[2]};
    double f2;
    if (p->mode == 0) {
        if (p->poly > 0.0) {
            y = orc_table_lookup(cx->tab_size, p->table_size, u[8]);
            if (y < 0.0) y = 0.0;
        }
        if (p->orient_kind == 1) {
            for (int a = 0; a < 3; ++a)
                ang[a] = p->orient_mean[a]
                       + p->orient_sigma[a] * orc_table_lookup_u(cx->tab_norm, p->table_size, u[9 + a]);
        } else if (p->orient_kind == 2) {
            ang[0] = acos(2.0 * u[9] - 1.0);
            ang[1] = 2.0 * ORC_PI * u[10];
            ang[2] = 2.0 * ORC_PI * u[11];
        } else if (p->orient_kind == 3) {
            ang[0] = ORC_PI * u[9];
            ang[1] = 2.0 * ORC_PI * u[10];
            ang[2] = 2.0 * ORC_PI * u[11];
        }
        if (sep_on(p)) {
            /* independent draws: size k from word (block 2, x) for k = 0 and
               (block 3, x), (block 3, y) for k = 1, 2 */
            const double uk[3] = {u[8], u[12], u[13]};
            double s[3];
            scaled_sizes(p, y, s);
            for (int k2 = 0; k2 < 3; ++k2) {
                if (p->poly_sep[k2] > 0.0) {
                    double yk = orc_table_lookup(cx->tab_sep[k2], p->table_size, uk[k2]);
                    ev.ysep[k2] = yk < 0.0 ? 0.0 : yk;
                    s[k2] *= ev.ysep[k2];
                }
            }
            f2 = form_f2_sizes(p, s, q, qv, ang);
        } else {
            f2 = orc_form_f2(p, q, qv, y, ang);
        }
    } else if (p->mode == 1) {
        f2 = pq_avg_nodes(p, q, qv, cx->gx, cx->gw);
    } else {
        int in_domain = 0;
        f2 = surrogate_f2(p, q, &in_domain);
        if (!in_domain) f2 = pq_avg_nodes(p, q, qv, cx->gx, cx->gw);
    }
    double sq = struct_factor(p, q);
    double w = len * 1e10 * cx->prefactor * f2 * sq * guide_weight(p, src, ki, lambda);
    /* attenuation: exp(-mu (path before the scattering point + path after it
       along kf to where the slab is left)) */
    if (p->mu_att > 0.0) {
        double tout = INFINITY;
        for (int a = 0; a < 3; ++a) {
            double tt = INFINITY;
            if (kf[a] > 0.0) tt = (half[a] - rs[a]) / kf[a];
            if (kf[a] < 0.0) tt = (-half[a] - rs[a]) / kf[a];
            if (tt < tout) tout = tt;
        }
        w *= exp(-p->mu_att * ((s - s_in) + tout));
    }
    for (int a = 0; a < 3; ++a) {
        ev.qv[a] = qv[a];
        ev.ang[a] = ang[a];
    }
    ev.y = y;
    ev.len = len;

    /* straight flight to the detector plane and the pixel hit */
    if (!(kf[2] > 0.0)) return ev;
    double sd = (p->det_z - rs[2]) / kf[2];
    double xd = rs[0] + sd * kf[0];
    double yd = rs[1] + sd * kf[1];
    double fx = floor((xd + 0.5 * p->det_w) / (p->det_w / p->nx));
    double fy = floor((yd + 0.5 * p->det_h) / (p->det_h / p->ny));
    if (fx < 0.0 || fx >= p->nx || fy < 0.0 || fy >= p->ny) return ev;
    ev.pixel = (int32_t)fy * p->nx + (int32_t)fx;
    ev.w = w;
    return ev;
}

int orc_trace_debug(const orc_params* p, uint64_t first, uint64_t n, uint64_t seed,
                    uint32_t exp_id, int32_t* pixel, double* w, double* q)
{
    orc_ctx cx;
    if (ctx_init(&cx, p) != 0) return -1;
    for (uint64_t j = 0; j < n; ++j) {
        orc_event ev = trace_one(&cx, first + j, seed, exp_id);
        if (pixel) pixel[j] = ev.pixel;
        if (w) w[j] = ev.w;
        if (q) q[j] = ev.q;
    }
    ctx_free(&cx);
    return 0;
}

/* Per-neutron intermediate values (diagnostics): out[j*11 + k], k = pixel,
 * w, q, Q_x, Q_y, Q_z, y, theta, phi, Psi, path length (m). */
int orc_trace_debug_ex(const orc_params* p, uint64_t first, uint64_t n, uint64_t seed,
                       uint32_t exp_id, double* out)
{
    orc_ctx cx;
    if (ctx_init(&cx, p) != 0) return -1;
    for (uint64_t j = 0; j < n; ++j) {
        orc_event ev = trace_one(&cx, first + j, seed, exp_id);
        double* o = out + j * 14;
        o[0] = ev.pixel;
        o[1] = ev.w;
        o[2] = ev.q;
        o[3] = ev.qv[0];
        o[4] = ev.qv[1];
        o[5] = ev.qv[2];
        o[6] = ev.y;
        o[7] = ev.ang[0];
        o[8] = ev.ang[1];
        o[9] = ev.ang[2];
        o[10] = ev.len;
        o[11] = ev.ysep[0];
        o[12] = ev.ysep[1];
        o[13] = ev.ysep[2];
    }
    ctx_free(&cx);
    return 0;
}

typedef struct {
    const orc_ctx* cx;
    uint64_t first, n, seed;
    uint32_t exp_id;
    double* det;
    double* det_w2;
    uint64_t* det_count;
} orc_job;

static void* run_job(void* arg)
{
    orc_job* jb = (orc_job*)arg;
    for (uint64_t j = 0; j < jb->n; ++j) {
        orc_event ev = trace_one(jb->cx, jb->first + j, jb->seed, jb->exp_id);
        if (ev.pixel >= 0) {
            jb->det[ev.pixel] += ev.w;
            if (jb->det_w2) jb->det_w2[ev.pixel] += ev.w * ev.w;
            if (jb->det_count) jb->det_count[ev.pixel] += 1;
        }
    }
    return NULL;
}

/* Traces neutrons first .. first+n-1 and writes the summed detector (ny*nx,
 * row-major, FP64) into det; det_w2 (sum of w^2) and det_count (hits) are
 * optional.  The range is split into nthreads contiguous parts with private
 * detectors that are merged in thread order. */
int orc_trace(const orc_params* p, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
              int32_t nthreads, double* det, double* det_w2, uint64_t* det_count)
{
    if (nthreads < 1) nthreads = 1;
    size_t npix = (size_t)p->nx * (size_t)p->ny;
    orc_ctx cx;
    if (ctx_init(&cx, p) != 0) return -1;
    orc_job* jobs = (orc_job*)calloc(nthreads, sizeof(orc_job));
    pthread_t* th = (pthread_t*)calloc(nthreads, sizeof(pthread_t));
    uint64_t start = first;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t cnt = n / nthreads + ((uint64_t)t < n % nthreads ? 1 : 0);
        jobs[t].cx = &cx;
        jobs[t].first = start;
        jobs[t].n = cnt;
        jobs[t].seed = seed;
        jobs[t].exp_id = exp_id;
        jobs[t].det = (double*)calloc(npix, sizeof(double));
        jobs[t].det_w2 = det_w2 ? (double*)calloc(npix, sizeof(double)) : NULL;
        jobs[t].det_count = det_count ? (uint64_t*)calloc(npix, sizeof(uint64_t)) : NULL;
        start += cnt;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
    run_job(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    memset(det, 0, npix * sizeof(double));
    if (det_w2) memset(det_w2, 0, npix * sizeof(double));
    if (det_count) memset(det_count, 0, npix * sizeof(uint64_t));
    for (int t = 0; t < nthreads; ++t) {
        for (size_t k = 0; k < npix; ++k) {
            det[k] += jobs[t].det[k];
            if (det_w2) det_w2[k] += jobs[t].det_w2[k];
            if (det_count) det_count[k] += jobs[t].det_count[k];
        }
        free(jobs[t].det);
        free(jobs[t].det_w2);
        free(jobs[t].det_count);
    }
    free(jobs);
    free(th);
    ctx_free(&cx);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The transmitted (unscattered) beam: the neutron that does not scatter
 * keeps its straight flight from the source point through the slit point
 * to the detector plane; the slab removes it with probability 1 -
 * exp(-mu_att chord), so its weight is exp(-mu_att chord), the chord being
 * its path inside the slab (zero when it misses the slab: weight 1).  Its
 * random numbers are the first block of the neutron's stream, the same
 * source and slit points as its scattered flight. */
static int transmitted_one(const orc_params* p, uint64_t i, uint64_t seed, uint32_t e, double* w)
{
    uint32_t r0[4];
    neutron_block(seed, i, 0, e, r0);
    double src[3] = {(orc_uniform(r0[0]) - 0.5) * p->src_w, (orc_uniform(r0[1]) - 0.5) * p->src_h, p->src_z};
    double slt[3] = {(orc_uniform(r0[2]) - 0.5) * p->slit_w, (orc_uniform(r0[3]) - 0.5) * p->slit_h, p->slit_z};
    double d[3] = {slt[0] - src[0], slt[1] - src[1], slt[2] - src[2]};
    double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double ki[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
    double half[3] = {0.5 * p->sample_w, 0.5 * p->sample_h, 0.5 * p->sample_d};
    double s_in = 0.0, s_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (ki[a] != 0.0) {
            double t1 = (-half[a] - src[a]) / ki[a];
            double t2 = (half[a] - src[a]) / ki[a];
            double tl = t1 < t2 ? t1 : t2, th = t1 < t2 ? t2 : t1;
            if (tl > s_in) s_in = tl;
            if (th < s_out) s_out = th;
        } else if (fabs(src[a]) > half[a]) {
            s_out = -1.0;
        }
    }
    double chord = s_out > s_in ? s_out - s_in : 0.0;
    *w = exp(-p->mu_att * chord);
    if (p->guide[0] > 0.0) {
        uint32_t r1[4];
        neutron_block(seed, i, 1, e, r1);
        double lambda = p->lambda0 * (1.0 + p->dlambda_rel * (2.0 * orc_uniform(r1[0]) - 1.0));
        *w *= guide_weight(p, src, ki, lambda);
    }
    if (!(ki[2] > 0.0)) return -1;
    double sd = (p->det_z - src[2]) / ki[2];
    double xd = src[0] + sd * ki[0], yd = src[1] + sd * ki[1];
    double fx = floor((xd + 0.5 * p->det_w) / (p->det_w / p->nx));
    double fy = floor((yd + 0.5 * p->det_h) / (p->det_h / p->ny));
    if (fx < 0.0 || fx >= p->nx || fy < 0.0 || fy >= p->ny) return -1;
    return (int)fy * p->nx + (int)fx;
}

/* Per-neutron transmitted events: pixel (-1 off the detector) and weight
 * (0 off the detector). */
int orc_transmitted_debug(const orc_params* p, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                          int32_t* pixel, double* w)
{
    for (uint64_t j = 0; j < n; ++j) {
        double wj;
        int32_t px = transmitted_one(p, first + j, seed, exp_id, &wj);
        pixel[j] = px;
        w[j] = px >= 0 ? wj : 0.0;
    }
    return 0;
}

/* Adds the transmitted beam of neutrons first .. first+n-1 to det (and to
 * det_w2 / det_count when given). */
int orc_transmitted_add(const orc_params* p, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                        double* det, double* det_w2, uint64_t* det_count)
{
    for (uint64_t j = 0; j < n; ++j) {
        double wj;
        int32_t px = transmitted_one(p, first + j, seed, exp_id, &wj);
        if (px < 0) continue;
        det[px] += wj;
        if (det_w2) det_w2[px] += wj * wj;
        if (det_count) det_count[px] += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The surrogate network, plainly: 8 -> 256 -> 256 -> 256 -> 256 -> 1 with
 * SiLU hidden units, parameters flat in the order W0[8][256] b0 W1[256][256]
 * b1 W2 b2 W3 b3 W4[256] b4 (W stored [in][out]).  FP64 arithmetic; with
 * round_bf16 set, every operand of a matrix product is first rounded to
 * FP32 and then to BF16 (round to nearest even), the operand precision the
 * device uses, so that the comparison isolates the accumulation; the two
 * exceptions follow the network's definition: each input enters as the sum
 * of its two BF16 parts, and the output layer takes the last activations
 * unrounded.                                                               */
#define ORC_NIN 8
#define ORC_NH 256
#define ORC_NP 199937

static long orc_offw(int l) { return l == 0 ? 0 : ORC_NIN * ORC_NH + ORC_NH + (long)(l - 1) * (ORC_NH * ORC_NH + ORC_NH); }
static long orc_offb(int l) { return l == 0 ? ORC_NIN * ORC_NH : orc_offw(l) + (long)ORC_NH * ORC_NH; }
static const long ORC_OFFW4 = ORC_NIN * ORC_NH + ORC_NH + 3L * (ORC_NH * ORC_NH + ORC_NH);

double orc_bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double op(double v, int r) { return r ? orc_bf16_round(v) : v; }
static double orc_silu(double z) { return z / (1.0 + exp(-z)); }
static double orc_silu_grad(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

int64_t orc_mlp_param_count(void) { return ORC_NP; }

/* Forward for n samples; z (optional, [4][n][256]) receives the
 * pre-activations, h (optional, [4][n][256]) the activations. */
void orc_mlp_forward(const double* w, const double* x, int32_t n, double* y, int32_t round_bf16,
                     double* z, double* h)
{
    double* a = (double*)malloc(sizeof(double) * ORC_NH);
    double* b = (double*)malloc(sizeof(double) * ORC_NH);
    for (int i = 0; i < n; ++i) {
        /* layer 0: with operand rounding, each input enters as the sum of
         * its two BF16 parts, hi = bf16(x) and lo = bf16(x - hi) */
        for (int o = 0; o < ORC_NH; ++o) {
            double s = 0.0;
            for (int k = 0; k < ORC_NIN; ++k) {
                const double xv = x[(long)i * ORC_NIN + k];
                const double xin = round_bf16 ? orc_bf16_round(xv) + orc_bf16_round(xv - orc_bf16_round(xv)) : xv;
                s += xin * op(w[orc_offw(0) + (long)k * ORC_NH + o], round_bf16);
            }
            double zz = s + op(w[orc_offb(0) + o], round_bf16);
            if (z) z[(long)i * ORC_NH + o] = zz;
            a[o] = orc_silu(zz);
            if (h) h[(long)i * ORC_NH + o] = a[o];
        }
        for (int l = 1; l < 4; ++l) {
            for (int o = 0; o < ORC_NH; ++o) {
                double s = 0.0;
                for (int k = 0; k < ORC_NH; ++k)
                    s += op(a[k], round_bf16) * op(w[orc_offw(l) + (long)k * ORC_NH + o], round_bf16);
                double zz = s + op(w[orc_offb(l) + o], round_bf16);
                if (z) z[((long)l * n + i) * ORC_NH + o] = zz;
                b[o] = orc_silu(zz);
                if (h) h[((long)l * n + i) * ORC_NH + o] = b[o];
            }
            memcpy(a, b, sizeof(double) * ORC_NH);
        }
        /* output layer: the last activations enter unrounded */
        double s = 0.0;
        for (int k = 0; k < ORC_NH; ++k) s += a[k] * op(w[ORC_OFFW4 + k], round_bf16);
        y[i] = s + op(w[ORC_OFFW4 + ORC_NH], round_bf16);
    }
    free(a);
    free(b);
}

/* dw = gradient of sum_i dy_i y_i over the parameters (chain rule written
 * out layer by layer).  dw_abs (optional, [ORC_NP]) receives, for each
 * element, the sum of the absolute values of the terms that form it (the
 * scale of its rounding error). */
void orc_mlp_backward(const double* w, const double* x, const double* dy, int32_t n, double* dw,
                      int32_t round_bf16, double* dw_abs)
{
    double* z = (double*)malloc(sizeof(double) * 4L * n * ORC_NH);
    double* h = (double*)malloc(sizeof(double) * 4L * n * ORC_NH);
    double* y = (double*)malloc(sizeof(double) * n);
    double* g = (double*)malloc(sizeof(double) * (long)n * ORC_NH);
    double* gn = (double*)malloc(sizeof(double) * (long)n * ORC_NH);
    orc_mlp_forward(w, x, n, y, round_bf16, z, h);
    memset(dw, 0, sizeof(double) * ORC_NP);
    if (dw_abs) memset(dw_abs, 0, sizeof(double) * ORC_NP);
    /* output layer */
    for (int k = 0; k < ORC_NH; ++k) {
        double s = 0.0, sa = 0.0;
        for (int i = 0; i < n; ++i) {
            const double t = op(h[(3L * n + i) * ORC_NH + k], round_bf16) * op(dy[i], round_bf16);
            s += t;
            sa += fabs(t);
        }
        dw[ORC_OFFW4 + k] = s;
        if (dw_abs) dw_abs[ORC_OFFW4 + k] = sa;
    }
    {
        double s = 0.0, sa = 0.0;
        for (int i = 0; i < n; ++i) {
            s += dy[i];
            sa += fabs(dy[i]);
        }
        dw[ORC_OFFW4 + ORC_NH] = s;
        if (dw_abs) dw_abs[ORC_OFFW4 + ORC_NH] = sa;
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < ORC_NH; ++k)
            g[(long)i * ORC_NH + k] = op(dy[i], round_bf16) * op(w[ORC_OFFW4 + k], round_bf16)
                                    * orc_silu_grad(z[(3L * n + i) * ORC_NH + k]);
    for (int l = 3; l >= 0; --l) {
        int kin = l == 0 ? ORC_NIN : ORC_NH;
        for (int k = 0; k < kin; ++k)
            for (int o = 0; o < ORC_NH; ++o) {
                double s = 0.0, sa = 0.0;
                for (int i = 0; i < n; ++i) {
                    double hin = l == 0 ? x[(long)i * ORC_NIN + k] : h[((long)(l - 1) * n + i) * ORC_NH + k];
                    const double t = op(hin, round_bf16) * op(g[(long)i * ORC_NH + o], round_bf16);
                    s += t;
                    sa += fabs(t);
                }
                dw[orc_offw(l) + (long)k * ORC_NH + o] = s;
                if (dw_abs) dw_abs[orc_offw(l) + (long)k * ORC_NH + o] = sa;
            }
        for (int o = 0; o < ORC_NH; ++o) {
            double s = 0.0, sa = 0.0;
            for (int i = 0; i < n; ++i) {
                s += g[(long)i * ORC_NH + o];
                sa += fabs(g[(long)i * ORC_NH + o]);
            }
            dw[orc_offb(l) + o] = s;
            if (dw_abs) dw_abs[orc_offb(l) + o] = sa;
        }
        if (l == 0) break;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < ORC_NH; ++k) {
                double s = 0.0;
                for (int o = 0; o < ORC_NH; ++o)
                    s += op(g[(long)i * ORC_NH + o], round_bf16) * op(w[orc_offw(l) + (long)k * ORC_NH + o], round_bf16);
                gn[(long)i * ORC_NH + k] = s * orc_silu_grad(z[((long)(l - 1) * n + i) * ORC_NH + k]);
            }
        memcpy(g, gn, sizeof(double) * (long)n * ORC_NH);
    }
    free(z);
    free(h);
    free(y);
    free(g);
    free(gn);
}

/* ------------------------------------------------------------------------ */
/* Surrogate mode: the weight uses <F^2>(0) P_ref(q) exp(net(u)) with the
 * network's inputs u_k = (2 x_k - lo_k - hi_k)/(hi_k - lo_k) (0 where lo_k =
 * hi_k) of x = (ln(q s0), ln(s1/s0), ln(s2/s0), p) and the reference
 * P_ref = (1 + q^2 Rg^2/6)^-2, Rg^2 = (s0^2 + s1^2 + s2^2)/12 for the
 * parallelepiped and /5 for the ellipsoid (its Guinier and Porod limits);
 * outside the box the exact average is used.  The network runs with BF16
 * operand rounding (the device's operand precision).  <F^2>(0) is the exact
 * average at q = 0.                                                       */
static double g_sur_w[ORC_NP];
static double g_sur_lo[4], g_sur_hi[4];
static int g_sur_set = 0;
/* the in-domain judge: bins of ln(q s0) over [lo_0, hi_0] in which the
   network was found more than the tolerance away from the exact average;
   neutrons in them take the exact average */
#define ORC_MAX_JUDGE_BINS 65536
static unsigned char g_judge_flag[ORC_MAX_JUDGE_BINS];
static int g_judge_bins = 0;

void orc_set_surrogate(const double* w, const double* lo, const double* hi)
{
    memcpy(g_sur_w, w, sizeof(double) * ORC_NP);
    for (int k = 0; k < 4; ++k) {
        g_sur_lo[k] = lo[k];
        g_sur_hi[k] = hi[k];
    }
    g_sur_set = 1;
    g_judge_bins = 0;
}

/* The network's inputs for this parameter set at x0 = ln(q s0) (u as in
   surrogate_f2); 0 when the model's own shape lies outside the box. */
static int surrogate_u(const orc_params* p, double x0, double u[8])
{
    double x[4] = {x0, log(p->size[1] / p->size[0]), log(p->size[2] / p->size[0]), p->poly};
    for (int k = 0; k < 8; ++k) u[k] = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (!(x[k] >= g_sur_lo[k] - (k ? 1e-6 : 0.0) && x[k] <= g_sur_hi[k] + (k ? 1e-6 : 0.0))) return 0;
        u[k] = g_sur_hi[k] > g_sur_lo[k] ? (2.0 * x[k] - g_sur_lo[k] - g_sur_hi[k]) / (g_sur_hi[k] - g_sur_lo[k]) : 0.0;
    }
    return 1;
}

/* ln of the surrogate's <F^2>(q) over the exact one at x0 = ln(q s0). */
static double surrogate_log_error(const orc_params* p, double x0, const double* gx, const double* gw)
{
    double u[8], y;
    if (!surrogate_u(p, x0, u)) return 0.0;
    orc_mlp_forward(g_sur_w, u, 1, &y, 1, NULL, NULL);
    const double q = exp(x0) / p->size[0];
    orc_params p1 = *p;
    p1.mode = 1;
    double qv0[3] = {0.0, 0.0, 0.0};
    const double f2_0 = pq_avg_nodes(&p1, 0.0, qv0, gx, gw);
    const double rg2 = (p->size[0] * p->size[0] + p->size[1] * p->size[1] + p->size[2] * p->size[2])
                     / (p->kind == 4 ? 12.0 : 5.0);
    const double t = 1.0 + q * q * rg2 / 6.0;
    const double sur = f2_0 * exp(y) / (t * t);
    return log(sur / pq_avg_nodes(&p1, q, qv0, gx, gw));
}

/* The judge for parameter set p: the surrogate's ln-error at the edges and
   midpoints of nbins bins of x0 over [lo_0, hi_0] (err [2 nbins + 1],
   optional); a bin is flagged when the error at any of its three points
   exceeds tol, and its neutrons then take the exact average.  Returns the
   number of flagged bins (-1 on bad arguments). */
int32_t orc_surrogate_judge(const orc_params* p, double tol, int32_t nbins, double* err)
{
    if (!g_sur_set || nbins < 1 || nbins > ORC_MAX_JUDGE_BINS || p->quad_n < 1 || p->quad_n > ORC_MAX_QUAD)
        return -1;
    double gx[ORC_MAX_QUAD], gw[ORC_MAX_QUAD];
    orc_gauss_legendre(p->quad_n, gx, gw);
    const double lo = g_sur_lo[0], hi = g_sur_hi[0];
    double prev = fabs(surrogate_log_error(p, lo, gx, gw));
    if (err) err[0] = prev;
    int32_t flagged = 0;
    for (int b = 0; b < nbins; ++b) {
        const double xm = lo + (hi - lo) * (b + 0.5) / nbins, xe = lo + (hi - lo) * (b + 1.0) / nbins;
        const double em = fabs(surrogate_log_error(p, xm, gx, gw)), ee = fabs(surrogate_log_error(p, xe, gx, gw));
        if (err) {
            err[2 * b + 1] = em;
            err[2 * b + 2] = ee;
        }
        g_judge_flag[b] = prev > tol || em > tol || ee > tol;
        flagged += g_judge_flag[b];
        prev = ee;
    }
    g_judge_bins = nbins;
    return flagged;
}

static double surrogate_f2(const orc_params* p, double q, int* in_domain)
{
    const double x0 = log(q * p->size[0]);
    *in_domain = 0;
    if (!g_sur_set) return 0.0;
    /* trained on Schulz sizes that scale all three axes together only */
    if (p->poly > 0.0 && (p->poly_kind != 0 || (p->poly_mask & 7) != 7)) return 0.0;
    double u[8];
    if (!surrogate_u(p, x0, u)) return 0.0;
    if (g_judge_bins > 0) {
        /* the judge's bin of x0 */
        double fb = floor((x0 - g_sur_lo[0]) / (g_sur_hi[0] - g_sur_lo[0]) * g_judge_bins);
        if (fb < 0.0) fb = 0.0;
        if (fb > g_judge_bins - 1) fb = g_judge_bins - 1;
        if (g_judge_flag[(int)fb]) return 0.0;
    }
    *in_domain = 1;
    double y;
    orc_mlp_forward(g_sur_w, u, 1, &y, 1, NULL, NULL);
    double qv0[3] = {0.0, 0.0, 0.0};
    double gx[ORC_MAX_QUAD], gw[ORC_MAX_QUAD];
    orc_gauss_legendre(p->quad_n, gx, gw);
    orc_params p0 = *p;
    p0.mode = 1;
    double f2_0 = pq_avg_nodes(&p0, 0.0, qv0, gx, gw);
    const double rg2 = (p->size[0] * p->size[0] + p->size[1] * p->size[1] + p->size[2] * p->size[2])
                     / (p->kind == 4 ? 12.0 : 5.0);
    const double t = 1.0 + q * q * rg2 / 6.0;
    return f2_0 * exp(y) / (t * t);
}
