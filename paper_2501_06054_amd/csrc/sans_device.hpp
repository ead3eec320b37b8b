// sans_device.hpp -- device code of the gfx950 SANS sample tracer.
//
// One neutron per lane.  The per-neutron steps:
//   1. Philox4x32-10 blocks of the neutron's counter (Salmon et al., SC'11);
//   2. source and slit points, wavelength, flight direction (FP64);
//   3. slab-sample entry and exit, scattering point (FP64);
//   4. outgoing direction uniform in the cone, scattering vector Q (FP64);
//   5. particle size and orientation from inverse-CDF tables staged in LDS
//      (Methods, "Polydispersity and orientational distributions");
//   6. amplitude F of the model (Eqs. (5)-(7), (9)) and the hard-sphere
//      Percus-Yevick S(Q);
//   7. weight w = l dOmega n F^2 S (Eq. (3) with n = phi/<V>), FP32;
//   8. straight flight to the detector plane and the pixel index (FP64).
//
// Precision split.  Everything that is geometry -- positions, directions, Q,
// the particle axes, the dimensionless phases x = Q.r that enter the shape
// functions, and their reduction modulo pi/2 -- is FP64, so that a neutron's
// pixel and the distance of its phase to a zero of F are exact to FP64
// rounding.  The transcendentals (sin/cos polynomials on the reduced phase,
// J1, the series) and the weight itself are FP32 VALU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sans {

// ---------------------------------------------------------------- constants
constexpr double kPi = 3.141592653589793238462643383;
// pi/2 split for Cody-Waite reduction (FP64 head + tail)
constexpr double kPio2Hi = 1.5707963267948966;
constexpr double kPio2Lo = 6.123233995736766e-17;
constexpr double k2oPi = 0.6366197723675814;

constexpr double cfact(int n) { return n <= 1 ? 1.0 : n * cfact(n - 1); }
constexpr double cpow4(int m) { return m == 0 ? 1.0 : 4.0 * cpow4(m - 1); }

// Taylor coefficients in x^2 of 3 j1(x)/x: 3 (-1)^m 2(m+1) / (2m+3)!
constexpr double sph_coef(int m) { return (m % 2 ? -1.0 : 1.0) * 6.0 * (m + 1) / cfact(2 * m + 3); }
// Taylor coefficients in x^2 of 2 J1(x)/x: (-1)^m / (4^m m! (m+1)!)
constexpr double lam_coef(int m) { return (m % 2 ? -1.0 : 1.0) / (cpow4(m) * cfact(m) * cfact(m + 1)); }
// Taylor coefficients of sin and cos
constexpr double sin_coef(int m) { return (m % 2 ? -1.0 : 1.0) / cfact(2 * m + 1); }
constexpr double cos_coef(int m) { return (m % 2 ? -1.0 : 1.0) / cfact(2 * m); }

// Forced compile-time evaluation of the coefficients (no run-time calls).
template <int M> struct SphC { static constexpr float v = (float)sph_coef(M); };
template <int M> struct LamC { static constexpr float v = (float)lam_coef(M); };
template <int M> struct SinC { static constexpr float v = (float)sin_coef(M); };
template <int M> struct CosC { static constexpr float v = (float)cos_coef(M); };
template <int M> struct SinD { static constexpr double v = sin_coef(M); };
template <int M> struct CosD { static constexpr double v = cos_coef(M); };

constexpr int kPySeriesTerms = 12;
constexpr int kPyCheb = 12;      // Chebyshev terms of the Percus-Yevick G(x)/x
constexpr int kMaxQuad = 256;
// Structure-factor constants in device memory: the adhesive spheres' series
// of A(k) and B(k)/k in k^2 [kPySeriesTerms each], then 12 eta and the factor
// function's coefficients h, b, c0 (h x^2 + b x + c0); the square well's
// 8 eta depth, width, width^3.
constexpr int kSqA = 0, kSqB = kPySeriesTerms, kSqE = 2 * kPySeriesTerms, kSqH = kSqE + 1, kSqBb = kSqE + 2,
              kSqC0 = kSqE + 3, kSqW8 = kSqE + 4, kSqW = kSqE + 5, kSqW3 = kSqE + 6, kSqCoef = kSqE + 7;
// Hayter-Penfold table: 1/dK, the last knot's index, two unused floats,
// then (S, dK dS/dK) at K_j = j dK
constexpr int kMsaHead = 4;

// orientation node arrays of the exact average: mu, w_mu, cos beta, sin beta,
// w_beta, sqrt(1 - mu^2)
constexpr int kQuadArrays = 6;

// ---------------------------------------------------------------- arguments
// Everything a trace kernel needs, passed by value as the kernel argument.
struct TraceArgs {
    int32_t kind;                 // model (the batched kernel switches on it per tile)
    // instrument, FP64
    double src_w, src_h, src_z;
    double slit_w, slit_h, slit_z;
    double lambda0, lambda_span;  // lambda = lambda0 + lambda_span (2u - 1)
    double half_x, half_y, half_z;
    double clear_x, clear_y;      // the half-widths less 1e-9 of themselves
    double omc;                   // 1 - cos(alpha)
    double mu_att;                // attenuation coefficient (1/m)
    // the guide upstream of the source aperture (guide_on: length > 0):
    // half-width, half-height, length, gap to the aperture, reflectivity
    int32_t guide_on;
    double guide_hw, guide_hh, guide_len, guide_gap, guide_m, guide_r0, guide_qc, guide_alpha, guide_wc;
    int32_t att_on;               // mu_att > 0 (an integer: the branch stays scalar)
    double det_z, det_hw, det_hh;
    double inv_px, inv_py;        // nx / det_w, ny / det_h
    double wscale;                // 1e10 * dOmega * phi / <V>  (per metre of path)
    int32_t nx, ny;
    // FP32 geometry of isotropic models (fast_geom: the source lies upstream
    // of the slab and the detector downstream of it): source and slit widths,
    // 1/(slit_z - src_z), the distances from the source plane to the slab's
    // faces, the depth, the faces' half-widths less 1e-5 of themselves,
    // 1 - cos alpha, the detector plane, its half-widths and pixels per metre,
    // the margins (pixels) inside which a pixel edge is decided in FP64
    // instead, the smallest direction cosine along z taken in FP32, and the
    // weight's scale per metre
    int32_t fast_geom;
    float f_src_w, f_src_h, f_slit_w, f_slit_h, f_inv_dz, f_lz_in, f_lz_out, f_depth, f_half_z;
    float f_clear_x, f_clear_y, f_omc;
    float f_det_z, f_det_hw, f_det_hh, f_inv_px, f_inv_py, f_eps_x, f_eps_y, f_fz_min, f_wscale;
    // sample
    double size[3];               // sizes (phases are formed in FP64)
    double shell;
    double ang_sin[3], ang_cos[3];// sin, cos of the mean angles
    double ang_sigma[3];
    float contrast;               // drho = sld[0] - sld[2]
    float cs_core, cs_shell;      // core-shell: sld0 - sld1, sld1 - sld2
    int32_t poly_on, poly_mask, orient_kind, third_block;
    // independent size draws: sep_on[k] for size k (its table in tab_sep +
    // k M, global memory), sep_block3 when sizes 1 or 2 draw (fourth block)
    int32_t sep_any, sep_on[3], sep_block3;
    const double* tab_sep;
    int32_t sq_on, sq_kind;       // sq_kind: 0 hard spheres, 1 adhesive, 2 square well, 3 Hayter-Penfold
    float sq_2r, sq_24phi;
    float py_alpha, py_beta, py_gamma;
    float py_c[kPySeriesTerms];
    // G(x)/x as a Chebyshev sum in z = x^2 py_cheb_s - 1 over x <= py_cheb_xmax
    // (the instrument's largest q sigma); py_cheb_xmax < 0: none
    float py_cheb[kPyCheb];
    float py_cheb_s, py_cheb_xmax;
    // adhesive and square-well constants (kSqCoef floats) or the Hayter-
    // Penfold table (device memory; read only on their branch, so they hold
    // no registers in the other kernels)
    const float* sq_coef;
    // tables (device global memory, FP64 knots; kernels stage them in LDS)
    int32_t M;                    // knots per table
    const double* tab_size;       // Schulz quantiles or nullptr
    const double* tab_norm;       // normal quantiles or nullptr
    // exact-average quadrature (QUAD mode), FP32 nodes
    int32_t quad_n, quad_ny, quad_dims;   // orientation nodes, size nodes, 0/1/2-D orientation
    const float* quad_nodes;      // mu[n] wmu[n] cb[n] sb[n] wb[n] st[n] y[ny] wy[ny] (global)
    float fsize[3], fshell;       // FP32 copies for the quadrature loop
    float fA[3], fB[3], fC[3];    // fixed-orientation particle axes (FP32)
    // barbell / capped cylinder: the caps' Gauss-Legendre rule at y = 1, FP32
    // [3][cap_n] in global memory: t in [t0, 1], s = r sqrt(1 - t^2) (A) and
    // w = 2 pi r^3 (1 - t^2) w_t (1 - t0)/2 (A^3); the cap centre's distance
    // z_c from the particle centre and the cap radius r (A)
    int32_t cap_n;
    const float* cap_nodes;
    double cap_zc, cap_r;
    float fcap_zc, fcap_r;
    // polymer micelle: N, excess lengths of a core block and a chain (A), the
    // chains' penetration factor d
    float mic_n, mic_bs, mic_bc;
    double mic_d;
    // shape-independent models: I(0) in 1/cm; the polydisperse coil's U and
    // 1/(1 + 2U); Teubner-Strey's c = 1/xi^2 - k^2, e = 4 k^2/xi^2 and
    // n = (k^2 + 1/xi^2)^2 (k = 2 pi/d)
    float si_scale;
    double si_u, si_z;
    float ts_c, ts_e, ts_n;
    // further model constants: power law m; peaks q0, 1/width; mass fractal
    // D - 1, D (D + 1)/6; star f/(3f - 2), f - 1, 1/f; gel Lorentz scale and
    // length
    double si_a, si_b, si_c, si_d, si_e, si_f, si_g;
    // sphere family: shells or pearls (n), the step between shells or the gap
    // between pearls (A)
    int32_t sf_n;
    double sf_gap;
    // core-shell cylinder and bicelle: thickness of the shell on each end face
    // (A); bicelle: contrasts core - face, face - rim, rim - solvent;
    // core-shell parallelepiped: the face slabs' thicknesses (A)
    double cs_face;
    float fcs_face;
    float bi_c[3];
    double csp_t[3];
    float fcsp_t[3];
    // elliptical bicelle: cross-section ratio; stacked disks: spacing d, spread
    // sigma, count (sf_n); paracrystals: primitive vectors (A), (g D)^2 / 2
    double bi_x, sd_d, sd_sig, pc_v[3][3], pc_b;
    // belt bicelle: -sigma^2 / 2 of the interface roughness; raspberry: the
    // number of small spheres (their centres' offset beyond R in sf_gap);
    // pearl necklace: a rod's excess length drho pi th^2 l / 4
    double bi_rough;
    float rb_n;
    // binary hard spheres: sqrt(n_1), sqrt(n_2) and 1 / (n_1 + n_2) (number
    // densities in 1/A^3, the nodes of Baxter's integrals in cap_nodes)
    float bhs_sn[2], bhs_int;
    // lamellae: 2 pi / delta and the Caille parameter (the repeat distance,
    // spacing spread and count in sd_d, sd_sig, sf_n; the Caille exponents'
    // gamma + ln(pi n) in cap_nodes)
    float lam_c, lam_eta;
    // flexible elliptical cylinder: Kuhn length (A) and the section's axis ratio
    float fc_b, fc_eps;
    // run
    uint64_t first, n;
    uint32_t seed_lo, seed_hi, exp_id;
};

// ---------------------------------------------------------------- Philox
struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10: ten rounds of the 4x32 S-box; the key gets the Weyl
// increments before every round after the first.
__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
    // The key is uniform across the wave (one seed per launch or per batch
    // tile), so it can live in scalar registers.  Its value is hidden here
    // so that the nine round-key
    // increments are recomputed with scalar adds at every call instead of
    // being hoisted out of the neutron loop, where twenty loop-invariant
    // round keys overflow the scalar registers and come back through VALU
    // lane reads.
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply per word (v_mad_u64_u32 gives both halves)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input xor in one instruction (truth table 0x96 of v_bitop3_b32)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// FP64 reciprocal, quotient and square root for finite, normal operands of
// the geometry: the hardware estimates (v_rcp_f64, v_rsq_f64) refined by
// Newton steps to about one ulp, without the scaling and special-case
// handling of the IEEE sequences (none of these operands is zero, denormal
// or infinite; a zero divisor gives a NaN, which fails every comparison).
__device__ __forceinline__ double rcp_d(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double div_d(double a, double b)
{
    const double r = rcp_d(b);
    const double q = a * r;
    return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
// x > 0
__device__ __forceinline__ double sqrt_d(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double e = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, e, g);
    h = __builtin_fma(h, e, h);
    const double d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}

// (x + 1/2) 2^-32 - 1/2 and (x + 1/2) 2^-32, exact in FP64.
__device__ __forceinline__ double centred_u(uint32_t x)
{
    return __builtin_fma((double)x, 0x1p-32, 0x1p-33 - 0.5);
}
__device__ __forceinline__ double u64(uint32_t x) { return __builtin_fma((double)x, 0x1p-32, 0x1p-33); }
// The same in FP32 (x rounded to 24 bits: absolute error below 2^-25).
__device__ __forceinline__ float centred_uf(uint32_t x) { return __builtin_fmaf((float)x, 0x1p-32f, -0.5f); }
__device__ __forceinline__ float uf(uint32_t x) { return __builtin_fmaf((float)x, 0x1p-32f, 0x1p-33f); }

// ---------------------------------------------------------------- FP32 math
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// sin r and cos r for |r| <= pi/4 by their Taylor polynomials (degree 11 and
// 12; truncation below 1e-11).
__device__ __forceinline__ void sincos_poly(float r, float& s, float& c)
{
    const float r2 = r * r;
    float ps = SinC<5>::v;
    ps = __builtin_fmaf(ps, r2, SinC<4>::v);
    ps = __builtin_fmaf(ps, r2, SinC<3>::v);
    ps = __builtin_fmaf(ps, r2, SinC<2>::v);
    ps = __builtin_fmaf(ps, r2, SinC<1>::v);
    s = __builtin_fmaf(ps * r2, r, r);
    float pc = CosC<6>::v;
    pc = __builtin_fmaf(pc, r2, CosC<5>::v);
    pc = __builtin_fmaf(pc, r2, CosC<4>::v);
    pc = __builtin_fmaf(pc, r2, CosC<3>::v);
    pc = __builtin_fmaf(pc, r2, CosC<2>::v);
    pc = __builtin_fmaf(pc, r2, CosC<1>::v);
    c = __builtin_fmaf(pc, r2, 1.0f);
}

// Quadrant rotation: (sin, cos) of n pi/2 + r from those of r.
__device__ __forceinline__ void quadrant(int n, float sr, float cr, float& s, float& c)
{
    const bool odd = n & 1;
    const float a = odd ? cr : sr, b = odd ? sr : cr;
    s = (n & 2) ? -a : a;
    c = ((n + 1) & 2) ? -b : b;
}

// sin and cos of an FP64 phase: Cody-Waite reduction by pi/2 in FP64, then
// the FP32 polynomials.  Exact quadrant and remainder for |x| < 2^40.
__device__ __forceinline__ void sincos_phase(double x, float& s, float& c)
{
    const double n = rint(x * k2oPi);
    double r = __builtin_fma(-n, kPio2Hi, x);
    r = __builtin_fma(-n, kPio2Lo, r);
    float sr, cr;
    sincos_poly((float)r, sr, cr);
    quadrant((int)(int64_t)n, sr, cr, s, c);
}

// The same for an FP32 argument (quadrature loops): FP32 Cody-Waite.
__device__ __forceinline__ void sincos_f(float x, float& s, float& c)
{
    const float n = rintf(x * (float)k2oPi);
    float r = __builtin_fmaf(-n, 1.5707963705062866f, x);   // pi/2 rounded to FP32
    r = __builtin_fmaf(-n, -4.3711388286737929e-08f, r);     // pi/2 minus that
    float sr, cr;
    sincos_poly(r, sr, cr);
    quadrant((int)n, sr, cr, s, c);
}

// 3 j1(x)/x, the normalised sphere amplitude: series below 2, else from the
// reduced phase.
__device__ __forceinline__ float sph3j_series(float x)
{
    const float x2 = x * x;
    float r = SphC<8>::v;
    r = __builtin_fmaf(r, x2, SphC<7>::v);
    r = __builtin_fmaf(r, x2, SphC<6>::v);
    r = __builtin_fmaf(r, x2, SphC<5>::v);
    r = __builtin_fmaf(r, x2, SphC<4>::v);
    r = __builtin_fmaf(r, x2, SphC<3>::v);
    r = __builtin_fmaf(r, x2, SphC<2>::v);
    r = __builtin_fmaf(r, x2, SphC<1>::v);
    return __builtin_fmaf(r, x2, 1.0f);
}

// 3 j1(x)/x from its Taylor series to x^30, given x^2, for x <= kSphLongMax:
// no branch and no square root.  FP32 Horner: absolute error below 1.4e-6
// there (1 at x = 0), set by the cancellation of the alternating terms.
constexpr float kSphLongMax = 8.0f;
template <int M>
__device__ __forceinline__ float sph_horner(float x2, float r)
{
    if constexpr (M < 0) {
        return r;
    } else {
        return sph_horner<M - 1>(x2, __builtin_fmaf(r, x2, SphC<M>::v));
    }
}
__device__ __forceinline__ float sph3j_long(float x2) { return sph_horner<14>(x2, SphC<15>::v); }

// 3 j1(x)/x at an FP64 phase: the short series below 2, else the closed form
// on the FP64 phase.  LONG: the long series up to x = kSphLongTo instead of
// the short one up to 2, so that the lanes of a wave, which mostly lie below
// it, seldom split between the series and the closed form (both of which a
// split wave runs).  Its absolute error there is below 1.3e-7, against 1e-8
// for the other two forms; the bound stays below the first zero of j1
// (4.493), so its relative error stays below 5e-6 (F(4.3) = 0.030).  Where
// an amplitude is a difference of nearly equal spheres (vesicles, the shells
// of fractal aggregates) the absolute error would grow relative to it, so
// only the single sphere and the core-shell sphere take it.  The choice is
// the lane's own, so a neutron's weight does not depend on which neutrons
// share its wave.
constexpr float kSphLongTo = 4.3f;
template <bool LONG = false>
__device__ __forceinline__ float sph3j_d(double xd)
{
    xd = fabs(xd);
    const float x = (float)xd;
    if constexpr (LONG)
        if (x <= kSphLongTo) return sph3j_long(x * x);
    if (x < 2.0f) return sph3j_series(x);
    float s, c;
    sincos_phase(xd, s, c);
    const float ix = rcpf(x);
    return 3.0f * __builtin_fmaf(-x, c, s) * (ix * ix * ix);
}

__device__ __forceinline__ float sph3j_f(float x)
{
    x = fabsf(x);
    if (x < 2.0f) return sph3j_series(x);
    float s, c;
    sincos_f(x, s, c);
    const float ix = rcpf(x);
    return 3.0f * __builtin_fmaf(-x, c, s) * (ix * ix * ix);
}


// 2 J1(x)/x (the cylinder's cross-section factor, Eq. (9)): Taylor series
// below 3, the device library's j1f above.
__device__ __forceinline__ float lambda1_f(float x)
{
    x = fabsf(x);
    if (x < 3.0f) {
        const float x2 = x * x;
        float r = LamC<10>::v;
        r = __builtin_fmaf(r, x2, LamC<9>::v);
        r = __builtin_fmaf(r, x2, LamC<8>::v);
        r = __builtin_fmaf(r, x2, LamC<7>::v);
        r = __builtin_fmaf(r, x2, LamC<6>::v);
        r = __builtin_fmaf(r, x2, LamC<5>::v);
        r = __builtin_fmaf(r, x2, LamC<4>::v);
        r = __builtin_fmaf(r, x2, LamC<3>::v);
        r = __builtin_fmaf(r, x2, LamC<2>::v);
        r = __builtin_fmaf(r, x2, LamC<1>::v);
        return __builtin_fmaf(r, x2, 1.0f);
    }
    return 2.0f * j1f(x) * rcpf(x);
}

// sin(x)/x: Taylor series to x^16 below 2 (truncation below 2e-10 there;
// the sums of the quadrature stay on this branch for the small-angle
// workloads, so a wave rarely takes both), else from the reduced phase.
constexpr float kSincSeriesMax = 2.0f;
__device__ __forceinline__ float sinc_series(float x)
{
    const float x2 = x * x;
    float r = SinC<8>::v;
    r = __builtin_fmaf(r, x2, SinC<7>::v);
    r = __builtin_fmaf(r, x2, SinC<6>::v);
    r = __builtin_fmaf(r, x2, SinC<5>::v);
    r = __builtin_fmaf(r, x2, SinC<4>::v);
    r = __builtin_fmaf(r, x2, SinC<3>::v);
    r = __builtin_fmaf(r, x2, SinC<2>::v);
    r = __builtin_fmaf(r, x2, SinC<1>::v);
    return __builtin_fmaf(r, x2, 1.0f);
}

__device__ __forceinline__ float sinc_d(double xd)
{
    xd = fabs(xd);
    const float x = (float)xd;
    if (x < kSincSeriesMax) return sinc_series(x);
    float s, c;
    sincos_phase(xd, s, c);
    return s * rcpf(x);
}

// sin(x)/x by its Taylor series to x^10 for |x| <= kSincShortMax (truncation
// below 6e-10 there): the exact average's inner loops when a whole wave's
// arguments are known to stay that small.
constexpr float kSincShortMax = 1.1f;
__device__ __forceinline__ float sinc_short(float x)
{
    const float x2 = x * x;
    float r = SinC<5>::v;
    r = __builtin_fmaf(r, x2, SinC<4>::v);
    r = __builtin_fmaf(r, x2, SinC<3>::v);
    r = __builtin_fmaf(r, x2, SinC<2>::v);
    r = __builtin_fmaf(r, x2, SinC<1>::v);
    return __builtin_fmaf(r, x2, 1.0f);
}

__device__ __forceinline__ float sinc_f(float x)
{
    x = fabsf(x);
    if (x < kSincSeriesMax) return sinc_series(x);
    float s, c;
    sincos_f(x, s, c);
    return s * rcpf(x);
}

// Percus-Yevick hard spheres: 1/S(q) = 1 + 24 phi G(x)/x, x = 2 q R.  Below
// x = 2.5 G(x)/x comes from its power series (coefficients computed on the
// host); above, from the closed form.
__device__ __forceinline__ float py_inv_sq(const TraceArgs& a, float x)
{
    float gx;
    if (x <= a.py_cheb_xmax) {
        // Clenshaw's recurrence of the Chebyshev sum: one branch-free form for
        // every q of the instrument (relative error of 1/S below 5e-7 for
        // volume fractions up to 0.2, 4e-6 at 0.45), so a wave never runs
        // both the series and the closed form below
        const float z = __builtin_fmaf(x * x, a.py_cheb_s, -1.0f), z2 = z + z;
        float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
        for (int k = kPyCheb - 1; k >= 1; --k) {
            const float t = __builtin_fmaf(z2, b1, a.py_cheb[k]) - b2;
            b2 = b1;
            b1 = t;
        }
        gx = __builtin_fmaf(z, b1, a.py_cheb[0]) - b2;
    } else if (x < 2.5f) {
        const float x2 = x * x;
        float r = a.py_c[kPySeriesTerms - 1];
#pragma unroll
        for (int m = kPySeriesTerms - 2; m >= 0; --m) r = __builtin_fmaf(r, x2, a.py_c[m]);
        gx = r;
    } else {
        float s, c;
        sincos_f(x, s, c);
        const float ix = rcpf(x);
        const float ix2 = ix * ix;
        const float x2 = x * x;
        const float ta = (s - x * c) * ix2;
        const float tb = (2.0f * x * s + (2.0f - x2) * c - 2.0f) * ix2 * ix;
        const float tg = (-x2 * x2 * c + 4.0f * ((3.0f * x2 - 6.0f) * c + (x2 * x - 6.0f * x) * s + 6.0f))
                       * ix2 * ix2 * ix;
        gx = (a.py_alpha * ta + a.py_beta * tb + a.py_gamma * tg) * ix;
    }
    return __builtin_fmaf(a.sq_24phi, gx, 1.0f);
}

// Adhesive hard spheres (Baxter): S = 1/(A^2 + B^2) with A, B the real and
// imaginary parts of 1 - 12 eta int_0^1 Q(x) exp(i k x) dx, k = q sigma, Q
// the quadratic factor function; power series in k^2 below k = 2.5, above
// the closed forms of int x^n cos(kx) and int x^n sin(kx) (n = 0, 1, 2).
__device__ __forceinline__ float sticky_sq(const float* __restrict__ c, float k)
{
    float A, B;
    if (k < 2.5f) {
        const float k2 = k * k;
        float ra = c[kSqA + kPySeriesTerms - 1], rb = c[kSqB + kPySeriesTerms - 1];
#pragma unroll
        for (int m = kPySeriesTerms - 2; m >= 0; --m) {
            ra = __builtin_fmaf(ra, k2, c[kSqA + m]);
            rb = __builtin_fmaf(rb, k2, c[kSqB + m]);
        }
        A = ra;
        B = rb * k;
    } else {
        float s, cs;
        sincos_f(k, s, cs);
        const float ik = rcpf(k);
        const float ks = k * s, kc = k * cs;
        const float c0 = s * ik;
        const float c1 = (ks + cs - 1.0f) * ik * ik;
        const float c2 = __builtin_fmaf(k, ks, 2.0f * (kc - s)) * ik * ik * ik;
        const float s0 = (1.0f - cs) * ik;
        const float s1 = (s - kc) * ik * ik;
        const float s2 = (__builtin_fmaf(-k, kc, 2.0f * (ks + cs)) - 2.0f) * ik * ik * ik;
        const float h = c[kSqH], b = c[kSqBb], q0 = c[kSqC0];
        A = __builtin_fmaf(-c[kSqE], __builtin_fmaf(h, c2, __builtin_fmaf(b, c1, q0 * c0)), 1.0f);
        B = c[kSqE] * __builtin_fmaf(h, s2, __builtin_fmaf(b, s1, q0 * s0));
    }
    return rcpf(__builtin_fmaf(A, A, B * B));
}

// Hayter-Penfold S at K = q sigma: cubic Hermite between the two knots
// around K from their values and slopes (clamped to the table's span).
__device__ __forceinline__ float msa_sq(const float* __restrict__ c, float K)
{
    const float t = fminf(fmaxf(K * c[0], 0.0f), c[1]);
    const float fk = fminf(floorf(t), c[1] - 1.0f);
    const int k = (int)fk;
    const float f = t - fk;
    const float* __restrict__ e = c + kMsaHead + 2 * k;
    const float s0 = e[0], d0 = e[1], s1 = e[2], d1 = e[3];
    const float ds = s1 - s0;
    const float c3 = __builtin_fmaf(-2.0f, ds, d0 + d1);
    const float c2 = __builtin_fmaf(3.0f, ds, -__builtin_fmaf(2.0f, d0, d1));
    return __builtin_fmaf(f, __builtin_fmaf(f, __builtin_fmaf(f, c3, c2), d0), s0);
}

// The structure factor of the model (the kind is the same for every lane):
// hard spheres; adhesive spheres; the square well, whose mean-spherical
// direct correlation adds 8 eta depth (w^3 Phi(w x) - Phi(x)) to the
// hard-sphere one (Phi the sphere's 3 j1(y)/y); Hayter-Penfold's charged
// spheres from their table.
__device__ __forceinline__ float struct_factor(const TraceArgs& a, float q)
{
    const float x = q * a.sq_2r;
    if (a.sq_kind == 1) return sticky_sq(a.sq_coef, x);
    if (a.sq_kind == 3) return msa_sq(a.sq_coef, x);
    float inv = py_inv_sq(a, x);
    if (a.sq_kind == 2) {
        const float* __restrict__ c = a.sq_coef;
        inv = __builtin_fmaf(-c[kSqW8], __builtin_fmaf(c[kSqW3], sph3j_f(c[kSqW] * x), -sph3j_f(x)), inv);
    }
    return rcpf(inv);
}

// Lookup in the orientation's FP64 normal table (knots at (k + 1/2)/M),
// linear in u with linear extrapolation in the end half-cells.
__device__ __forceinline__ double table_lerp_u(const double* tab, int M, double u)
{
    const double s = __builtin_fma(u, (double)M, -0.5);
    double fk = floor(s);
    fk = fmin(fmax(fk, 0.0), (double)(M - 2));
    const int k = (int)fk;
    const double f = s - fk;
    const double y0 = tab[k], y1 = tab[k + 1];
    return __builtin_fma(f, y1 - y0, y0);
}

// Inverse-CDF lookup in an FP64 size table whose knots are equally spaced in
// t = -ln(2 min(u, 1 - u)) with step 32 ln 2 / (M/2 - 1): the lower half
// (knots 0 .. M/2 - 1, from the median down) for u < 1/2, else the upper half
// (from the median up), linear in t.  t and the interpolation fraction are
// formed in FP32: the lookup is continuous across knots, so their rounding
// moves y by parts in 1e7 of one knot interval.
__device__ __forceinline__ double table_lerp(const double* tab, int M, double u)
{
    const int H = M >> 1;
    const bool up = u >= 0.5;
    const double v = up ? 1.0 - u : u;
    const float t = -0.693147181f * log2f((float)(2.0 * v));
    const float s = t * ((float)(H - 1) * 0.0450842200f);   // t / dt
    const float fj = fminf(fmaxf(floorf(s), 0.0f), (float)(H - 2));
    const int j = (int)fj;
    const double f = (double)(s - fj);
    const double* half = up ? tab + H : tab;
    const double y0 = half[j], y1 = half[j + 1];
    return __builtin_fma(f, y1 - y0, y0);
}

// ---------------------------------------------------------------- orientation (FP64)
// sin and cos of a small FP64 angle (|d| < 0.8: Taylor, degree 15/16),
// otherwise the device library's FP64 sincos.
__device__ __forceinline__ void sincos_small(double d, double& s, double& c)
{
    if (fabs(d) < 0.8) {
        const double d2 = d * d;
        double ps = SinD<7>::v;
        ps = __builtin_fma(ps, d2, SinD<6>::v);
        ps = __builtin_fma(ps, d2, SinD<5>::v);
        ps = __builtin_fma(ps, d2, SinD<4>::v);
        ps = __builtin_fma(ps, d2, SinD<3>::v);
        ps = __builtin_fma(ps, d2, SinD<2>::v);
        ps = __builtin_fma(ps, d2, SinD<1>::v);
        s = __builtin_fma(ps * d2, d, d);
        double pc = CosD<8>::v;
        pc = __builtin_fma(pc, d2, CosD<7>::v);
        pc = __builtin_fma(pc, d2, CosD<6>::v);
        pc = __builtin_fma(pc, d2, CosD<5>::v);
        pc = __builtin_fma(pc, d2, CosD<4>::v);
        pc = __builtin_fma(pc, d2, CosD<3>::v);
        pc = __builtin_fma(pc, d2, CosD<2>::v);
        pc = __builtin_fma(pc, d2, CosD<1>::v);
        c = __builtin_fma(pc, d2, 1.0);
    } else {
        sincos(d, &s, &c);
    }
}

// sin, cos of (mean + d) from those of the mean (host, exact) and of d.
__device__ __forceinline__ void rotate_by(double sm, double cm, double d, double& s, double& c)
{
    double sd, cd;
    sincos_small(d, sd, cd);
    s = __builtin_fma(sm, cd, cm * sd);
    c = __builtin_fma(cm, cd, -sm * sd);
}

// Particle axes A = R x, B = R y, C = R z with R = Rz(phi) Ry(theta) Rz(Psi),
// from the sines and cosines of (theta, phi, Psi).
struct Trig3 {
    double st, ct, sp, cp, ss, cs;
};

// Projections of Q on the particle axes (Eq. (6)); C only when WANT_AB is false.
template <bool WANT_AB>
__device__ __forceinline__ void project(const Trig3& g, const double qv[3], double& qa, double& qb,
                                        double& qc)
{
    const double cx = g.cp * g.st, cy = g.sp * g.st, cz = g.ct;
    qc = qv[0] * cx + qv[1] * cy + qv[2] * cz;
    if constexpr (WANT_AB) {
        const double ax = g.cp * g.ct * g.cs - g.sp * g.ss;
        const double ay = g.sp * g.ct * g.cs + g.cp * g.ss;
        const double az = -g.st * g.cs;
        const double bx = -g.cp * g.ct * g.ss - g.sp * g.cs;
        const double by = -g.sp * g.ct * g.ss + g.cp * g.cs;
        const double bz = g.st * g.ss;
        qa = qv[0] * ax + qv[1] * ay + qv[2] * az;
        qb = qv[0] * bx + qv[1] * by + qv[2] * bz;
    } else {
        qa = qb = 0.0;
    }
}

// ---------------------------------------------------------------- models
enum : int { kSphere = 0, kCoreShell = 1, kCylinder = 2, kEllipsoid = 3, kParallelepiped = 4,
              kBarbell = 5, kCappedCylinder = 6, kHollowPrism = 7, kMicelle = 8,
              kHollowCylinder = 9, kCoreShellCylinder = 10, kCoreShellEllipsoid = 11,
              kHollowPrismThick = 12, kGuinier = 13, kOrnsteinZernike = 14, kDab = 15, kGaussCoil = 16,
              kPolyGaussCoil = 17, kTeubnerStrey = 18, kPowerLaw = 19, kGaussianPeak = 20,
              kLorentzPeak = 21, kMassFractal = 22, kStarPolymer = 23, kGaussLorentzGel = 24,
              kFuzzySphere = 25, kVesicle = 26, kMultilayerVesicle = 27, kLinearPearls = 28,
              kSurfaceFractal = 29, kTwoPowerLaw = 30, kGuinierPorod = 31, kSpinodal = 32, kPorod = 33,
              kLine = 34, kTwoLorentzian = 35, kCorrelationLength = 36, kBroadPeak = 37, kFractal = 38,
              kFractalCoreShell = 39, kPolymerExclVolume = 40, kEllipticalCylinder = 41,
              kCoreShellBicelle = 42, kCoreShellParallelepiped = 43, kCoreShellBicelleElliptical = 44,
              kStackedDisks = 45, kScParacrystal = 46, kBccParacrystal = 47, kFccParacrystal = 48,
              kMassSurfaceFractal = 49, kGelFit = 50, kSuperball = 51, kLamellarHg = 52,
              kLamellarStackCaille = 53, kLamellarHgStackCaille = 54, kLamellarStackParacrystal = 55,
              kBicelleBeltRough = 56, kRaspberry = 57, kPearlNecklace = 58, kBinaryHardSphere = 59,
              kAdsorbedLayer = 60, kPringle = 61, kFlexCylEll = 62, kFlexCyl = 63 };

// Randomly oriented lamellae: the weight per unit volume fraction.
template <int KIND>
constexpr bool kLamellar = (KIND >= kLamellarHg && KIND <= kLamellarStackParacrystal) || KIND == kAdsorbedLayer;

// F^2 multiplied by an orientation-dependent interference factor (stacked
// disks, paracrystals).
template <int KIND>
constexpr bool kLattice = KIND >= kStackedDisks && KIND <= kFccParacrystal;

// Shape-independent models: the weight is a cross-section in 1/cm of |Q|.
template <int KIND>
constexpr bool kShapeIndependent = (KIND >= kGuinier && KIND <= kGaussLorentzGel)
                                   || (KIND >= kSurfaceFractal && KIND <= kBroadPeak)
                                   || KIND == kPolymerExclVolume || KIND == kMassSurfaceFractal
                                   || KIND == kGelFit;

// Isotropic sphere-based particles (fuzzy sphere, vesicles, pearl strings,
// fractal aggregates of spheres).
template <int KIND>
constexpr bool kSphereFamily = (KIND >= kFuzzySphere && KIND <= kLinearPearls) || KIND == kFractal
                               || KIND == kFractalCoreShell || KIND == kRaspberry || KIND == kPearlNecklace
                               || KIND == kBinaryHardSphere;

// Orientation enters the weight (the particles from the cylinder to the
// thick hollow prism, but the micelle).
template <int KIND>
constexpr bool kAniso = (KIND >= kCylinder && KIND <= kHollowPrismThick && KIND != kMicelle)
                        || (KIND >= kEllipticalCylinder && KIND <= kFccParacrystal) || KIND == kSuperball
                        || KIND == kBicelleBeltRough || KIND == kPringle;

// Bodies of revolution about C: cylinders (plain, hollow, core-shell),
// barbell, capped cylinder (only the axis projection Q.C and Q_AB enter, the
// third angle does not).
template <int KIND>
constexpr bool kOneAxis = KIND == kCylinder || KIND == kBarbell || KIND == kCappedCylinder
                          || KIND == kHollowCylinder || KIND == kCoreShellCylinder || KIND == kCoreShellBicelle
                          || KIND == kStackedDisks;

// Models that take independent size draws (volumes that are products of
// powers of the sizes): sphere, cylinder, ellipsoid, parallelepiped,
// elliptical cylinder.
template <int KIND>
constexpr bool kSepKind = KIND == kSphere || KIND == kCylinder || KIND == kEllipsoid || KIND == kParallelepiped
                          || KIND == kEllipticalCylinder;

// The caps' part of the barbell / capped-cylinder amplitude (Tables I-II,
// group A), in FP32: sum_i w_i cos(P + B t_i) 2J1(X s_i)/(X s_i) over the
// Gauss-Legendre nodes t_i of the cap integral at unit size, where P = y Q_C
// z_c is the phase of the cap centre (its sine and cosine come in as sP, cP,
// reduced by the caller), B = y Q_C r and X = y Q_AB.  Splitting the phase
// keeps the per-node argument B t_i within |y Q_C r|, so it needs no
// precision beyond FP32.  The caller multiplies by y^3.  The node arrays are
// read with uniform indices (scalar loads).
__device__ __forceinline__ float caps_sum(const TraceArgs& a, float sP, float cP, float B, float X)
{
    const float* __restrict__ tn = a.cap_nodes;
    const float* __restrict__ sn = a.cap_nodes + a.cap_n;
    const float* __restrict__ wn = a.cap_nodes + 2 * a.cap_n;
    float sum = 0.0f;
#pragma unroll 4
    for (int i = 0; i < a.cap_n; ++i) {
        float sv, cv;
        sincos_f(B * tn[i], sv, cv);
        const float c = __builtin_fmaf(cP, cv, -(sP * sv));
        sum = __builtin_fmaf(wn[i] * c, lambda1_f(X * sn[i]), sum);
    }
    return sum;
}

// The superball's transform at unit size and contrast, given the phases per
// unit length times the size, ta = Q_A R, tb = Q_B R, tc = Q_C R: the nested
// Gauss-Legendre rule over the octant's x and y (host nodes, [n + 3 n^2]
// floats: x_i, then y_ij, zm_ij and the weights), the z integral
// sin(tc zm)/tc exact (its series below |tc| = 1e-2).
__device__ __forceinline__ float superball_sum(const TraceArgs& a, float ta, float tb, float tc)
{
    const int n = a.cap_n;
    const float* __restrict__ xs = a.cap_nodes;
    const float* __restrict__ ys = xs + n;
    const float* __restrict__ zs = ys + n * n;
    const float* __restrict__ ws = zs + n * n;
    const bool small = fabsf(tc) < 1e-2f;
    const float itc = small ? 0.0f : rcpf(tc);
    const float tc2 = tc * tc * (-1.0f / 6.0f);
    float sum = 0.0f;
    for (int i = 0; i < n; ++i) {
        float sx, cx;
        sincos_f(ta * xs[i], sx, cx);
        float inner = 0.0f;
        const int base = i * n;
#pragma unroll 4
        for (int j = 0; j < n; ++j) {
            float sy, cy, sz, cz;
            sincos_f(tb * ys[base + j], sy, cy);
            const float z = zs[base + j];
            sincos_f(tc * z, sz, cz);
            const float zi = small ? z * __builtin_fmaf(tc2 * z, z, 1.0f) : sz * itc;
            inner = __builtin_fmaf(ws[base + j] * cy, zi, inner);
        }
        sum = __builtin_fmaf(cx, inner, sum);
    }
    return sum;
}

// The pringle's |F|^2: the saddle-bent plate's disc integral over the host's
// polar rule (cap_nodes: 2 n^2 nodes of x, then y, then z = alpha x^2 - beta
// y^2, then the weights with the (x, y) <-> (-x, -y) pairing folded in),
// exp(i (Q_A x + Q_B y + Q_C z)) summed into its real and imaginary parts;
// the thickness factor t sinc(Q_C t / 2).  y_s scales the plate's radius and
// y_t its thickness.
__device__ __forceinline__ float pringle_f2(const TraceArgs& a, double ys, double yt, double qa, double qb,
                                            double qc)
{
    const int m = 2 * a.cap_n * a.cap_n;
    const float* __restrict__ xs = a.cap_nodes;
    const float* __restrict__ yv = xs + m;
    const float* __restrict__ zs = yv + m;
    const float* __restrict__ ws = zs + m;
    const float ta = (float)(qa * ys), tb = (float)(qb * ys), tc = (float)(qc * ys * ys);
    float re = 0.0f, im = 0.0f;
#pragma unroll 4
    for (int k = 0; k < m; ++k) {
        float s1, c1, s2, c2;
        sincos_f(__builtin_fmaf(ta, xs[k], tb * yv[k]), s1, c1);
        sincos_f(tc * zs[k], s2, c2);
        const float w = ws[k] * c1;
        re = __builtin_fmaf(w, c2, re);
        im = __builtin_fmaf(w, s2, im);
    }
    const double t = a.size[1] * yt;
    const float pre = a.contrast * (float)t * sinc_d(0.5 * qc * t) * (float)(ys * ys);
    return pre * pre * __builtin_fmaf(re, re, im * im);
}

// sin(x)/x and cos x together (thin-walled prism): both from one reduction;
// the quotient is taken directly (sin x keeps its relative precision down to
// small x), with 1 at x = 0.
__device__ __forceinline__ void sinc_cos_d(double xd, float& sn, float& cs)
{
    float s, c;
    sincos_phase(xd, s, c);
    const float x = (float)xd;
    sn = x == 0.0f ? 1.0f : s * rcpf(x);
    cs = c;
}

__device__ __forceinline__ void sinc_cos_f(float x, float& sn, float& cs)
{
    float s, c;
    sincos_f(x, s, c);
    sn = x == 0.0f ? 1.0f : s * rcpf(x);
    cs = c;
}

// The thin-walled hollow prism's amplitude per unit contrast and wall: each
// pair of faces normal to an axis contributes 2 cos(half phase) times the
// face's area and its two in-plane sinc factors (Tables I-II).
__device__ __forceinline__ float hollow_faces(float a, float b, float c, float sa, float ca, float sb,
                                              float cb, float sc, float cc)
{
    const float sab = sa * sb;
    return 2.0f * (sc * __builtin_fmaf(b * c * ca, sb, a * c * sa * cb) + a * b * sab * cc);
}

// Polymer micelle (Tables I-II; the model of Pedersen and Gerstenberg): a
// homogeneous core of radius R with N Gaussian chains (radius of gyration Rg)
// starting at its surface.  Scattering per micelle, with the excess lengths
// b_s (core block) and b_c (chain), x = (q Rg)^2, the chain's double average
// P(x) = 2 (e^-x - 1 + x)/x^2 and single average psi(x) = (1 - e^-x)/x, the
// core amplitude Phi = 3 j1(qR)/(qR) and sigma = sinc(q (R + d Rg)):
//   (N (b_s Phi + b_c psi sigma))^2 + N b_c^2 (P - (psi sigma)^2),
// the coherent micelle plus what the chains' self terms add beyond it.  The
// phases in FP64, the chain functions in FP32 (series below x = 1).
template <int K> struct DebyeC {   // 2 (-1)^k / (k + 2)!
    static constexpr double f(int k) { return k == 0 ? 0.5 : f(k - 1) * (-1.0) / (k + 2); }
    static constexpr float v = (float)(2.0 * f(K));
};
template <int K> struct ChainC {   // (-1)^k / (k + 1)!
    static constexpr double f(int k) { return k == 0 ? 1.0 : f(k - 1) * (-1.0) / (k + 1); }
    static constexpr float v = (float)f(K);
};

__device__ __forceinline__ void chain_functions(float x, float& pdebye, float& psi)
{
    if (x < 1.0f) {
        float p = DebyeC<10>::v, c = ChainC<10>::v;
        p = __builtin_fmaf(p, x, DebyeC<9>::v);  c = __builtin_fmaf(c, x, ChainC<9>::v);
        p = __builtin_fmaf(p, x, DebyeC<8>::v);  c = __builtin_fmaf(c, x, ChainC<8>::v);
        p = __builtin_fmaf(p, x, DebyeC<7>::v);  c = __builtin_fmaf(c, x, ChainC<7>::v);
        p = __builtin_fmaf(p, x, DebyeC<6>::v);  c = __builtin_fmaf(c, x, ChainC<6>::v);
        p = __builtin_fmaf(p, x, DebyeC<5>::v);  c = __builtin_fmaf(c, x, ChainC<5>::v);
        p = __builtin_fmaf(p, x, DebyeC<4>::v);  c = __builtin_fmaf(c, x, ChainC<4>::v);
        p = __builtin_fmaf(p, x, DebyeC<3>::v);  c = __builtin_fmaf(c, x, ChainC<3>::v);
        p = __builtin_fmaf(p, x, DebyeC<2>::v);  c = __builtin_fmaf(c, x, ChainC<2>::v);
        p = __builtin_fmaf(p, x, DebyeC<1>::v);  c = __builtin_fmaf(c, x, ChainC<1>::v);
        pdebye = __builtin_fmaf(p, x, 1.0f);
        psi = __builtin_fmaf(c, x, 1.0f);
    } else {
        const float e = __expf(-x);
        const float ix = rcpf(x);
        psi = (1.0f - e) * ix;
        pdebye = 2.0f * (e - 1.0f + x) * ix * ix;
    }
}

__device__ __forceinline__ float micelle_f2(const TraceArgs& a, double R, double rg, double q)
{
    const float core = sph3j_d(q * R);
    const float sigma = sinc_d(q * __builtin_fma(a.mic_d, rg, R));
    const float qr = (float)(q * rg);
    float pc, psi;
    chain_functions(qr * qr, pc, psi);
    const float ps = psi * sigma;
    const float amp = a.mic_n * __builtin_fmaf(a.mic_bs, core, a.mic_bc * ps);
    return __builtin_fmaf(amp, amp, a.mic_n * a.mic_bc * a.mic_bc * __builtin_fmaf(-ps, ps, pc));
}

// The excluded-volume chain's rule: nodes per integral and the largest U it serves.
constexpr int kPevRuleNodes = 32;
constexpr double kPevRuleMaxU = 40.0;

// Lower incomplete gamma g(s, x) = Gamma(s) P(s, x), FP64: its power series
// below x = s + 1, else Gamma(s) less Legendre's continued fraction for the
// upper one (modified Lentz); gs = Gamma(s).
__device__ __forceinline__ double lower_gamma_d(double s, double x, double gs)
{
    const double pre = exp(s * log(x) - x);
    if (x < s + 1.0) {
        double term = 1.0 / s, sum = term;
        for (int n = 1; n < 400; ++n) {
            term *= x / (s + n);
            sum += term;
            if (fabs(term) < 1e-17 * sum) break;
        }
        return sum * pre;
    }
    const double tiny = 1e-300;
    double b = x + 1.0 - s, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int n = 1; n < 400; ++n) {
        const double an = -n * (n - s);
        b += 2.0;
        d = __builtin_fma(an, d, b);
        d = fabs(d) < tiny ? tiny : d;
        c = b + an / c;
        c = fabs(c) < tiny ? tiny : c;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return gs - pre * h;
}

// Shape-independent models (Tables I-II): dSigma/dOmega(q) in 1/cm with the
// length L = size[0]: Guinier exp(-(qL)^2/3), Ornstein-Zernike 1/(1 + (qL)^2),
// Debye-Anderson-Brumberger 1/(1 + (qL)^2)^2, the Gaussian coil's Debye
// function, coils with Schulz-Zimm masses (the M^2-weighted Debye function,
// 2 ((1 + U z)^(-1/U) - 1 + z)/((1 + U) z^2), z = (qL)^2/(1 + 2U), the
// power in FP64 with a series below z = 1e-3), and Teubner-Strey, written as
// (k^2 + 1/xi^2)^2 / ((q^2 + c)^2 + e) (no cancellation near its peak); all
// normalised to I(0) = scale.
template <int KIND>
__device__ __forceinline__ float shape_iq(const TraceArgs& a, double len, double q)
{
    const float ql = (float)(q * len);
    const float x = ql * ql;
    if constexpr (KIND == kGuinier) {
        return a.si_scale * __expf(x * (-1.0f / 3.0f));
    } else if constexpr (KIND == kOrnsteinZernike) {
        return a.si_scale * rcpf(1.0f + x);
    } else if constexpr (KIND == kDab) {
        const float r = rcpf(1.0f + x);
        return a.si_scale * r * r;
    } else if constexpr (KIND == kGaussCoil) {
        float pc, psi;
        chain_functions(x, pc, psi);
        return a.si_scale * pc;
    } else if constexpr (KIND == kPolyGaussCoil) {
        const double qld = q * len;
        const double z = qld * qld * a.si_z, u = a.si_u;
        double f;
        if (z < 1e-3) {
            f = 1.0 - z * (1.0 + 2.0 * u) / 3.0 + z * z * (1.0 + 2.0 * u) * (1.0 + 3.0 * u) / 12.0;
        } else if (u > 0.0) {
            f = 2.0 * (pow(1.0 + u * z, -1.0 / u) - 1.0 + z) / ((1.0 + u) * z * z);
        } else {
            f = 2.0 * (expm1(-z) + z) / (z * z);
        }
        return a.si_scale * (float)f;
    } else if constexpr (KIND == kTeubnerStrey) {
        const float d = (float)(q * q) + a.ts_c;
        return a.si_scale * a.ts_n * rcpf(__builtin_fmaf(d, d, a.ts_e));
    } else if constexpr (KIND == kPowerLaw) {
        // in FP64: the few smallest-q neutrons carry the total, and an FP32
        // exponent of magnitude m |log2 q| would cost them about 1e-6
        return a.si_scale * (float)exp2(-a.si_a * log2(q));
    } else if constexpr (KIND == kGaussianPeak) {
        const float d = (float)((q - a.si_a) * a.si_b);
        return a.si_scale * __expf(-0.5f * d * d);
    } else if constexpr (KIND == kLorentzPeak) {
        const float d = (float)((q - a.si_a) * a.si_b);
        return a.si_scale * rcpf(__builtin_fmaf(d, d, 1.0f));
    } else if constexpr (KIND == kMassFractal || KIND == kSurfaceFractal) {
        // sin(a atan(q xi)) / (a q xi (1 + (q xi)^2)^(a/2)), a = D - 1 (mass)
        // or 5 - Ds (surface), its Guinier term below q xi = 1e-3
        if (ql < 1e-3f) return a.si_scale * __builtin_fmaf(-(float)a.si_b, x, 1.0f);
        const float dm1 = (float)a.si_a;
        return a.si_scale * sinf(dm1 * atanf(ql)) * rcpf(dm1 * ql * exp2f(0.5f * dm1 * log2f(1.0f + x)));
    } else if constexpr (KIND == kStarPolymer) {
        float pc, psi;
        chain_functions(x * (float)a.si_a, pc, psi);
        return a.si_scale * (float)a.si_c * __builtin_fmaf((float)a.si_b * psi, psi, pc);
    } else if constexpr (KIND == kGaussLorentzGel) {
        // Gauss-Lorentz gel: exp(-(q L)^2 / 2) plus an Ornstein-Zernike term
        const float q2 = (float)(q * a.si_b);
        return __builtin_fmaf(a.si_scale, __expf(-0.5f * x), (float)a.si_a * rcpf(__builtin_fmaf(q2, q2, 1.0f)));
    } else if constexpr (KIND == kTwoPowerLaw) {
        // q^-m1 up to qc, qc^(m2 - m1) q^-m2 beyond (FP64 powers)
        const double v = q <= a.si_b ? exp2(-a.si_a * log2(q)) : a.si_d * exp2(-a.si_c * log2(q));
        return a.si_scale * (float)v;
    } else if constexpr (KIND == kGuinierPorod) {
        // q^-s exp(-(q Rg)^2 / (3 - s)) up to q1, (D/G) q^-m beyond
        if (q <= a.si_c) return a.si_scale * (float)exp2(-a.si_a * log2(q)) * __expf(-x * (float)a.si_e);
        return a.si_scale * (float)(a.si_d * exp2(-a.si_b * log2(q)));
    } else if constexpr (KIND == kSpinodal) {
        // spinodal: (1 + g/2) x^2 / (g/2 + x^(2 + g)), x = q / q_max (FP64 power)
        const double xs = q * a.si_a;
        const double v = a.si_c * xs * xs / (0.5 * a.si_b + exp2((2.0 + a.si_b) * log2(xs)));
        return a.si_scale * (float)v;
    } else if constexpr (KIND == kPorod) {
        const double iq2 = 1.0 / (q * q);
        return a.si_scale * (float)(iq2 * iq2);
    } else if constexpr (KIND == kLine) {
        return (float)(__builtin_fma(a.si_a, q, (double)a.si_scale));
    } else if constexpr (KIND == kTwoLorentzian) {
        // two generalised Lorentzians (FP64 powers)
        const double v = (double)a.si_scale / (1.0 + exp2(a.si_a * log2(q * a.si_d)))
                       + a.si_b / (1.0 + exp2(a.si_c * log2(q * a.si_e)));
        return (float)v;
    } else if constexpr (KIND == kCorrelationLength || KIND == kBroadPeak) {
        // a power law plus a generalised Lorentzian about 0 or about q0 (FP64)
        const double dq = KIND == kBroadPeak ? fabs(q - a.si_e) : q;
        const double v = (double)a.si_scale * exp2(-a.si_a * log2(q))
                       + a.si_b / (1.0 + exp2(a.si_c * log2(dq * a.si_d)));
        return (float)v;
    } else if constexpr (KIND == kMassSurfaceFractal) {
        // (1 + x/(3 pm))^-pm (1 + (q Rp)^2/(3 ps))^-ps: si_a = 1/(3 pm),
        // si_b = pm, si_c = Rp^2/(3 ps), si_d = ps
        const float xp = (float)(q * q * a.si_c);
        const float l2 = __builtin_fmaf((float)a.si_b, log2f(__builtin_fmaf(x, (float)a.si_a, 1.0f)),
                                        (float)a.si_d * log2f(1.0f + xp));
        return a.si_scale * exp2f(-l2);
    } else if constexpr (KIND == kGelFit) {
        // extra[0] (1 + (D + 1)/3 x)^(-D/2) + extra[1] exp(-(q Rg)^2/3):
        // si_a = (D + 1)/3, si_b = D/2, si_c = extra[1], si_d = Rg^2/3
        const float net = exp2f(-(float)a.si_b * log2f(__builtin_fmaf(x, (float)a.si_a, 1.0f)));
        return __builtin_fmaf(a.si_scale, net, (float)a.si_c * __expf(-(float)(q * q * a.si_d)));
    } else {
        // polymer with excluded volume: (g(s1, U)/U^s1 - g(s2, U)/U^s2)/nu with
        // the lower incomplete gamma g, s1 = 1/(2 nu), s2 = 1/nu, i.e.
        // int_0^1 t^(s-1) exp(-U t) dt for each s: a series below U = 1e-3; up to
        // U = 40 the host's rule (t = w^6 makes the integrands smooth in w;
        // 32 Gauss-Legendre nodes, relative error below 1e-9 there) in FP32;
        // beyond, FP64 incomplete gammas
        const double qr = q * len;
        const double u = qr * qr * a.si_a, s1 = a.si_c, s2 = a.si_d;
        double v;
        if (u >= 1e-3 && u <= kPevRuleMaxU) {
            const float uf = (float)u;
            const float* __restrict__ nd = a.cap_nodes;
            float x1 = 0.0f, x2 = 0.0f;
#pragma unroll 8
            for (int k = 0; k < kPevRuleNodes; ++k) {
                x1 = __builtin_fmaf(nd[kPevRuleNodes + k], __expf(-uf * nd[k]), x1);
                x2 = __builtin_fmaf(nd[3 * kPevRuleNodes + k], __expf(-uf * nd[2 * kPevRuleNodes + k]), x2);
            }
            return a.si_scale * (x1 - x2) * (float)(1.0 / a.si_b);
        }
        if (u < 1e-3) {
            double x1 = 0.0, x2 = 0.0, t = 1.0;
            for (int k = 0; k < 4; ++k) {
                x1 += t / (s1 + k);
                x2 += t / (s2 + k);
                t *= -u / (k + 1.0);
            }
            v = x1 - x2;
        } else {
            v = lower_gamma_d(s1, u, a.si_f) * exp(-s1 * log(u)) - lower_gamma_d(s2, u, a.si_g) * exp(-s2 * log(u));
        }
        return a.si_scale * (float)(v / a.si_b);
    }
}

// Randomly oriented lamellae (Tables I-II, group C), per unit volume fraction:
// (2 pi / delta) F1(q)^2 S(q) / q^2 with the sheet's transverse transform F1
// (head-tail bilayer: tails |z| < L_T, heads out to L_T + L_H; else one slab of
// thickness delta) and the stacking factor S of N sheets: Caille,
// 1 + 2 sum_n (1 - n/N) cos(q d n) exp(-eta (q d/2 pi)^2 (gamma + ln(pi n))),
// or a paracrystal with independent Gaussian spacings,
// 1 + 2 sum_n (1 - n/N) cos(q d n) exp(-n (q sigma)^2 / 2); phases in FP64.
template <int KIND>
__device__ __forceinline__ float lamellar_f2(const TraceArgs& a, double q)
{
    if constexpr (KIND == kAdsorbedLayer) {
        // a layer of excess thickness t on large particles, locally flat: 3 phi / R
        // of sheet per volume (in lam_c = 6 pi / R), smeared by sigma (sd_sig)
        const float f1 = a.contrast * a.fshell;
        const float iq = (float)(1.0 / q);
        return a.lam_c * f1 * f1 * __expf(-(float)(q * q * a.sd_sig * a.sd_sig)) * iq * iq;
    }
    float f1;
    if constexpr (KIND == kLamellarHg || KIND == kLamellarHgStackCaille) {
        const double lt = a.size[0], lo = a.size[0] + a.size[1];
        f1 = 2.0f * __builtin_fmaf(a.cs_core * (float)lt, sinc_d(q * lt), a.cs_shell * (float)lo * sinc_d(q * lo));
    } else {
        f1 = a.contrast * (float)a.size[0] * sinc_d(0.5 * q * a.size[0]);
    }
    float st = 1.0f;
    if constexpr (KIND != kLamellarHg) {
        const int n = a.sf_n;
        const float inv_n = 1.0f / (float)n;
        const double qd = q * a.sd_d;
        float s = 0.0f;
        if constexpr (KIND == kLamellarStackParacrystal) {
            const float damp = (float)exp(-0.5 * q * q * a.sd_sig * a.sd_sig);
            float dk = 1.0f;
            for (int k = 1; k < n; ++k) {
                float sv, cv;
                sincos_phase(qd * k, sv, cv);
                dk *= damp;
                s = __builtin_fmaf(__builtin_fmaf(-(float)k, inv_n, 1.0f) * dk, cv, s);
            }
        } else {
            const float x = (float)(qd * (0.5 / kPi));
            const float al = -a.lam_eta * x * x;
            const float* __restrict__ ln = a.cap_nodes;
            for (int k = 1; k < n; ++k) {
                float sv, cv;
                sincos_phase(qd * k, sv, cv);
                s = __builtin_fmaf(__builtin_fmaf(-(float)k, inv_n, 1.0f) * __expf(al * ln[k]), cv, s);
            }
        }
        st = __builtin_fmaf(2.0f, s, 1.0f);
    }
    const float iq = (float)(1.0 / q);
    return a.lam_c * f1 * f1 * st * iq * iq;
}

// Isotropic sphere-based particles (Tables I-II, group F), F^2 averaged over
// orientations; R the (drawn) sphere or bore radius, the phases in FP64:
// fuzzy sphere: the sphere smeared by a Gaussian of width shell, its
// amplitude times exp(-(q shell)^2 / 2); vesicle: a solvent-filled shell of
// thickness shell; multilayer vesicle: n such shells, one every shell + gap;
// linear pearls: n spheres in a line, centre spacing 2R + gap, with the
// orientation average sum_jk sinc(q r_jk) of the pair phases.
template <int KIND>
__device__ __forceinline__ float sphere_family_f2(const TraceArgs& a, double R, double q)
{
    constexpr float k43pi = (float)(4.0 / 3.0 * kPi);
    if constexpr (KIND == kFuzzySphere) {
        const float r = (float)R, qs = (float)(q * a.shell);
        const float f = a.contrast * k43pi * r * r * r * sph3j_d(q * R) * __expf(-0.5f * qs * qs);
        return f * f;
    } else if constexpr (KIND == kVesicle || KIND == kMultilayerVesicle) {
        const int n = KIND == kVesicle ? 1 : a.sf_n;
        float f = 0.0f;
        double ri = R;
        for (int k = 0; k < n; ++k) {
            const double ro = ri + a.shell;
            const float fi = (float)ri, fo = (float)ro;
            f += fo * fo * fo * sph3j_d(q * ro) - fi * fi * fi * sph3j_d(q * ri);
            ri = ro + a.sf_gap;
        }
        f *= a.cs_shell * k43pi;
        return f * f;
    } else if constexpr (KIND == kFractal || KIND == kFractalCoreShell) {
        // the blocks' F^2 times Teixeira's mass-fractal structure factor:
        // 1 + D Gamma(D - 1) sin((D - 1) atan(q xi)) / ((q R0)^D (1 + 1/(q xi)^2)^((D - 1)/2)),
        // its q -> 0 limit 1 + Gamma(D + 1) (xi/R0)^D below q xi = 1e-3 (FP64)
        const float r = (float)R;
        float f;
        double r0 = R;
        if constexpr (KIND == kFractal) {
            f = a.contrast * k43pi * r * r * r * sph3j_d(q * R);
        } else {
            r0 = R + a.shell;
            const float ro = (float)r0;
            f = a.cs_core * k43pi * r * r * r * sph3j_d(q * R) + a.cs_shell * k43pi * ro * ro * ro * sph3j_d(q * r0);
        }
        // in FP64: the powers' arguments reach tens, where FP32 exponents
        // would carry 1e-6 of relative error
        const double qx = q * a.si_d, d = a.si_c;
        double sq;
        if (qx < 1e-3) {
            sq = 1.0 + a.si_e * exp(d * log(a.si_d / r0));
        } else {
            const double num = a.si_a * sin((d - 1.0) * atan(qx));
            sq = 1.0 + num * exp(-d * log(q * r0) - 0.5 * (d - 1.0) * log1p(1.0 / (qx * qx)));
        }
        return f * f * (float)sq;
    } else if constexpr (KIND == kPearlNecklace) {
        // freely jointed chain of N pearls and N - 1 rods: x = sinc(q A) per unit,
        // beta (a rod seen from its pearls) and P (the rod itself) by the host's
        // Gauss-Legendre rule on [0, 1] (cap_nodes: t_i, then w_i summing to 1)
        const int n = a.sf_n, m = a.cap_n;
        const float r = (float)R;
        const float fs = a.contrast * k43pi * r * r * r * sph3j_d(q * R);   // a pearl's amplitude
        const double l = a.size[1];
        const float x = sinc_d(q * __builtin_fma(2.0, R, l));
        const float* __restrict__ tn = a.cap_nodes;
        const float* __restrict__ wn = a.cap_nodes + m;
        const float ql = (float)(q * l);
        float beta = 0.0f, prod = 0.0f;
        for (int i = 0; i < m; ++i) {
            beta = __builtin_fmaf(wn[i], sinc_d(__builtin_fma(l, (double)tn[i], R) * q), beta);
            prod = __builtin_fmaf(wn[i] * (1.0f - tn[i]), sinc_f(ql * tn[i]), prod);
        }
        const float nf = (float)n;
        float spp = nf, srr_sum = 0.0f, spr_sum = nf - 1.0f, xp = 1.0f;
        for (int d = 1; d < n; ++d) {
            const float xd = xp * x;                      // x^d
            spp = __builtin_fmaf(2.0f * (nf - (float)d), xd, spp);
            if (d <= n - 2) {
                srr_sum = __builtin_fmaf(nf - 1.0f - (float)d, xp, srr_sum);   // x^(d-1)
                spr_sum = __builtin_fmaf(nf - 1.0f - (float)d, xd, spr_sum);
            }
            xp = xd;
        }
        const float mr = a.rb_n;
        const float srr = __builtin_fmaf(2.0f * beta * beta, srr_sum, (nf - 1.0f) * 2.0f * prod);
        const float spr = 2.0f * beta * spr_sum;
        return __builtin_fmaf(fs * fs, spp, __builtin_fmaf(mr * mr, srr, 2.0f * fs * mr * spr));
    } else if constexpr (KIND == kBinaryHardSphere) {
        // Qhat_ij = delta_ij - sum_k W_k exp(i q r_k) over the host's rule
        // (cap_nodes: per (i, j) in row order 16 r_k, then 16 W_k, the factor
        // 2 pi sqrt(n_i n_j) Q_ij(r_k) and the weight folded into W_k); I - C =
        // Qhat^H Qhat (real), S its inverse; v^T S v / (n_1 + n_2), v_i = sqrt(n_i) F_i
        const float* __restrict__ nd = a.cap_nodes;
        const float qf = (float)q;
        float qr[4], qi[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float cr = 0.0f, ci = 0.0f;
#pragma unroll 4
            for (int k = 0; k < 16; ++k) {
                float sv, cv;
                sincos_f(qf * nd[32 * e + k], sv, cv);
                const float w = nd[32 * e + 16 + k];
                cr = __builtin_fmaf(w, cv, cr);
                ci = __builtin_fmaf(w, sv, ci);
            }
            qr[e] = ((e == 0 || e == 3) ? 1.0f : 0.0f) - cr;
            qi[e] = -ci;
        }
        const float m00 = qr[0] * qr[0] + qi[0] * qi[0] + qr[2] * qr[2] + qi[2] * qi[2];
        const float m11 = qr[1] * qr[1] + qi[1] * qi[1] + qr[3] * qr[3] + qi[3] * qi[3];
        const float m01 = qr[0] * qr[1] + qi[0] * qi[1] + qr[2] * qr[3] + qi[2] * qi[3];
        const float idet = rcpf(__builtin_fmaf(m00, m11, -m01 * m01));
        const float r1 = (float)R, r2 = (float)a.size[1];
        const float v1 = a.bhs_sn[0] * a.contrast * k43pi * r1 * r1 * r1 * sph3j_d(q * R);
        const float v2 = a.bhs_sn[1] * a.cs_shell * k43pi * r2 * r2 * r2 * sph3j_d(q * a.size[1]);
        const float quad = __builtin_fmaf(v1 * v1, m11, __builtin_fmaf(-2.0f * v1 * v2, m01, v2 * v2 * m00));
        return quad * idet * a.bhs_int;
    } else if constexpr (KIND == kRaspberry) {
        // (F_L + N F_S c)^2 + N F_S^2 (1 - c^2), c = sinc(q D), D = R + offset:
        // the pair sum averaged over independent positions on the sphere of radius D
        const float r = (float)R, rs = (float)a.size[1], n = a.rb_n;
        const float fl = a.contrast * k43pi * r * r * r * sph3j_d(q * R);
        const float fs = a.cs_shell * k43pi * rs * rs * rs * sph3j_d(q * a.size[1]);
        const float c = sinc_d(q * (R + a.sf_gap));
        const float t = __builtin_fmaf(n * fs, c, fl);
        return __builtin_fmaf(t, t, n * fs * fs * __builtin_fmaf(-c, c, 1.0f));
    } else {
        const float r = (float)R;
        const float fs = a.contrast * k43pi * r * r * r * sph3j_d(q * R);
        const double d = __builtin_fma(2.0, R, a.sf_gap);
        float pairs = (float)a.sf_n;
        for (int k = 1; k < a.sf_n; ++k) pairs += 2.0f * (float)(a.sf_n - k) * sinc_d(q * (k * d));
        return fs * fs * pairs;
    }
}

// Interference factors multiplying F^2 (FP64 phases):
// stacked disks: 1 + (2/N) sum_k (N - k) cos(k d Q_C) exp(-k (Q_C sigma)^2 / 2)
// (spacings scattering as N(d, sigma^2) each, the disorder accumulating);
// paracrystals (Matsuoka): the product over the three primitive vectors v_k
// of (1 - e^2) / ((1 - e)^2 + 4 e sin^2(Q.v_k / 2)), e = exp(-(q g D)^2 / 2)
// (the same as (1 - e^2)/(1 - 2e cos + e^2), without its cancellation).
template <int KIND>
__device__ __forceinline__ float lattice_factor(const TraceArgs& a, double q, double qa, double qb, double qc)
{
    if constexpr (KIND == kStackedDisks) {
        const int n = a.sf_n;
        const float damp = (float)exp(-0.5 * qc * qc * a.sd_sig * a.sd_sig);
        float s = 0.0f, dk = 1.0f;
        for (int k = 1; k < n; ++k) {
            float sv, cv;
            sincos_phase(qc * (k * a.sd_d), sv, cv);
            dk *= damp;
            s = __builtin_fmaf((float)(n - k) * dk, cv, s);
        }
        return 1.0f + 2.0f * s / (float)n;
    } else {
        const double b = q * q * a.pc_b;
        const double ome = -expm1(-b), e = exp(-b);
        float z = 1.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = qa * a.pc_v[k][0] + qb * a.pc_v[k][1] + qc * a.pc_v[k][2];
            float sh, ch;
            sincos_phase(0.5 * x, sh, ch);
            const double den = __builtin_fma(4.0 * e, (double)sh * (double)sh, ome * ome);
            z *= (float)(ome * (1.0 + e) / den);
        }
        return z;
    }
}

// F of one drawn particle (MC mode).  y scales the sizes selected by the
// polydispersity mask, ys[k] size k (independent draws; 1 when off); q, qa,
// qb, qc are |Q| and its projections (FP64).
template <int KIND>
__device__ __forceinline__ float amplitude_mc(const TraceArgs& a, double y, const double ys[3], double q,
                                              double qa, double qb, double qc)
{
    double s[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = ((a.poly_mask >> c & 1) ? a.size[c] * y : a.size[c]) * ys[c];
    constexpr float k43pi = (float)(4.0 / 3.0 * kPi);
    if constexpr (KIND == kSphere) {
        const float r = (float)s[0];
        return a.contrast * k43pi * r * r * r * sph3j_d<true>(q * s[0]);
    } else if constexpr (KIND == kCoreShell) {
        const double ro_d = s[0] + a.shell;
        const float rc = (float)s[0], ro = (float)ro_d;
        return a.cs_core * k43pi * rc * rc * rc * sph3j_d<true>(q * s[0])
             + a.cs_shell * k43pi * ro * ro * ro * sph3j_d<true>(q * ro_d);
    } else if constexpr (KIND == kCylinder) {
        const double qab = sqrt(fmax(__builtin_fma(q, q, -qc * qc), 0.0));
        const float r = (float)s[0], len = (float)s[1];
        return a.contrast * (float)kPi * r * r * len * sinc_d(0.5 * qc * s[1])
             * lambda1_f((float)(qab * s[0]));
    } else if constexpr (KIND == kEllipsoid) {
        const double xa = qa * s[0], xb = qb * s[1], xc = qc * s[2];
        const double x = sqrt(xa * xa + xb * xb + xc * xc);
        return a.contrast * k43pi * (float)s[0] * (float)s[1] * (float)s[2] * sph3j_d(x);
    } else if constexpr (KIND == kBarbell || KIND == kCappedCylinder) {
        const double qab = sqrt(fmax(__builtin_fma(q, q, -qc * qc), 0.0));
        const float r = (float)s[0], len = (float)s[1];
        const float cyl = (float)kPi * r * r * len * sinc_d(0.5 * qc * s[1]) * lambda1_f((float)(qab * s[0]));
        const double qcy = qc * y;
        float sP, cP;
        sincos_phase(qcy * a.cap_zc, sP, cP);
        const float yf = (float)y;
        const float caps = caps_sum(a, sP, cP, (float)(qcy * a.cap_r), (float)(qab * y));
        return a.contrast * __builtin_fmaf(yf * yf * yf, caps, cyl);
    } else if constexpr (KIND == kHollowPrism) {
        float sa, ca, sb, cb, sc, cc;
        sinc_cos_d(0.5 * qa * s[0], sa, ca);
        sinc_cos_d(0.5 * qb * s[1], sb, cb);
        sinc_cos_d(0.5 * qc * s[2], sc, cc);
        return a.contrast * a.fshell * hollow_faces((float)s[0], (float)s[1], (float)s[2], sa, ca, sb, cb, sc, cc);
    } else if constexpr (KIND == kHollowCylinder) {
        // the cylinder of radius bore + wall minus the bore
        const double qab = sqrt(fmax(__builtin_fma(q, q, -qc * qc), 0.0));
        const double ro_d = s[0] + a.shell;
        const float ri = (float)s[0], ro = (float)ro_d;
        const float ring = ro * ro * lambda1_f((float)(qab * ro_d)) - ri * ri * lambda1_f((float)(qab * s[0]));
        return a.contrast * (float)kPi * (float)s[1] * sinc_d(0.5 * qc * s[1]) * ring;
    } else if constexpr (KIND == kCoreShellCylinder) {
        // core (R, L) and the outer cylinder (R + shell, L + 2 face)
        const double qab = sqrt(fmax(__builtin_fma(q, q, -qc * qc), 0.0));
        const double ro_d = s[0] + a.shell, lo_d = __builtin_fma(2.0, a.cs_face, s[1]);
        const float r = (float)s[0], len = (float)s[1], ro = (float)ro_d, lo = (float)lo_d;
        const float core = r * r * len * sinc_d(0.5 * qc * s[1]) * lambda1_f((float)(qab * s[0]));
        const float outer = ro * ro * lo * sinc_d(0.5 * qc * lo_d) * lambda1_f((float)(qab * ro_d));
        return (float)kPi * __builtin_fmaf(a.cs_core, core, a.cs_shell * outer);
    } else if constexpr (KIND == kCoreShellEllipsoid) {
        // the core's semi-axes and the same grown by the shell
        const double oa = s[0] + a.shell, ob = s[1] + a.shell, oc = s[2] + a.shell;
        const double xa = qa * s[0], xb = qb * s[1], xc = qc * s[2];
        const double ya = qa * oa, yb = qb * ob, yc = qc * oc;
        const float core = (float)s[0] * (float)s[1] * (float)s[2] * sph3j_d(sqrt(xa * xa + xb * xb + xc * xc));
        const float outer = (float)oa * (float)ob * (float)oc * sph3j_d(sqrt(ya * ya + yb * yb + yc * yc));
        return k43pi * __builtin_fmaf(a.cs_core, core, a.cs_shell * outer);
    } else if constexpr (KIND == kHollowPrismThick) {
        // the box minus its cavity (edges less twice the wall)
        const double t2 = 2.0 * a.shell;
        const double ia = s[0] - t2, ib = s[1] - t2, ic = s[2] - t2;
        const float box = (float)s[0] * (float)s[1] * (float)s[2] * sinc_d(0.5 * qa * s[0])
                        * sinc_d(0.5 * qb * s[1]) * sinc_d(0.5 * qc * s[2]);
        const float cav = (float)ia * (float)ib * (float)ic * sinc_d(0.5 * qa * ia) * sinc_d(0.5 * qb * ib)
                        * sinc_d(0.5 * qc * ic);
        return a.contrast * (box - cav);
    } else if constexpr (KIND == kEllipticalCylinder) {
        // the ellipse's transform is the disc's at sqrt((a Q_A)^2 + (b Q_B)^2)
        const double xa = qa * s[0], xb = qb * s[1];
        const float x = (float)sqrt(xa * xa + xb * xb);
        return a.contrast * (float)kPi * (float)s[0] * (float)s[1] * (float)s[2] * sinc_d(0.5 * qc * s[2])
             * lambda1_f(x);
    } else if constexpr (KIND == kCoreShellBicelle) {
        // core (R, L), core + faces (R, L + 2 t_f), outer (R + rim, L + 2 t_f)
        const double qab = sqrt(fmax(__builtin_fma(q, q, -qc * qc), 0.0));
        const double lf = __builtin_fma(2.0, a.cs_face, s[1]), ro = s[0] + a.shell;
        const float r = (float)s[0], len = (float)s[1], flf = (float)lf, fro = (float)ro;
        const float disc = lambda1_f((float)(qab * s[0]));
        const float core = r * r * len * sinc_d(0.5 * qc * s[1]) * disc;
        const float ends = sinc_d(0.5 * qc * lf);
        const float faces = r * r * flf * ends * disc;
        const float outer = fro * fro * flf * ends * lambda1_f((float)(qab * ro));
        return (float)kPi * (a.bi_c[0] * core + a.bi_c[1] * faces + a.bi_c[2] * outer);
    } else if constexpr (KIND == kCoreShellBicelleElliptical) {
        // cross sections R x xR (core, faces) and (R + rim) x (xR + rim) (outer)
        const double ra = s[0], rb = a.bi_x * s[0], oa = ra + a.shell, ob = rb + a.shell;
        const double lf = __builtin_fma(2.0, a.cs_face, s[1]);
        const float d1 = lambda1_f((float)sqrt((ra * qa) * (ra * qa) + (rb * qb) * (rb * qb)));
        const float d2 = lambda1_f((float)sqrt((oa * qa) * (oa * qa) + (ob * qb) * (ob * qb)));
        const float ends = sinc_d(0.5 * qc * lf);
        const float core = (float)ra * (float)rb * (float)s[1] * sinc_d(0.5 * qc * s[1]) * d1;
        const float faces = (float)ra * (float)rb * (float)lf * ends * d1;
        const float outer = (float)oa * (float)ob * (float)lf * ends * d2;
        return (float)kPi * (a.bi_c[0] * core + a.bi_c[1] * faces + a.bi_c[2] * outer);
    } else if constexpr (KIND == kBicelleBeltRough) {
        // core R x xR x L, faces over the core's cross-section (L + 2 t_f), the
        // belt (R + t) x (xR + t) x L; roughness exp(-(q sigma)^2 / 2)
        const double ra = s[0], rb = a.bi_x * s[0], oa = ra + a.shell, ob = rb + a.shell;
        const double lf = __builtin_fma(2.0, a.cs_face, s[1]);
        const float d1 = lambda1_f((float)sqrt((ra * qa) * (ra * qa) + (rb * qb) * (rb * qb)));
        const float d2 = lambda1_f((float)sqrt((oa * qa) * (oa * qa) + (ob * qb) * (ob * qb)));
        const float mid = sinc_d(0.5 * qc * s[1]);
        const float core = (float)ra * (float)rb * (float)s[1] * mid * d1;
        const float faces = (float)ra * (float)rb * (float)lf * sinc_d(0.5 * qc * lf) * d1;
        const float belt = (float)oa * (float)ob * (float)s[1] * mid * d2;
        const float rough = __expf((float)(q * q * a.bi_rough));
        return (float)kPi * rough * (a.bi_c[0] * core + a.bi_c[1] * faces + a.bi_c[2] * belt);
    } else if constexpr (KIND == kStackedDisks) {
        // one disk: core (R, s1) and core + face layers (R, s1 + 2 shell)
        const double qab = sqrt(fmax(__builtin_fma(q, q, -qc * qc), 0.0));
        const double lo = __builtin_fma(2.0, a.shell, s[1]);
        const float r = (float)s[0], disc = lambda1_f((float)(qab * s[0]));
        const float core = r * r * (float)s[1] * sinc_d(0.5 * qc * s[1]) * disc;
        const float outer = r * r * (float)lo * sinc_d(0.5 * qc * lo) * disc;
        return (float)kPi * __builtin_fmaf(a.cs_core, core, a.cs_shell * outer);
    } else if constexpr (KIND == kScParacrystal || KIND == kBccParacrystal || KIND == kFccParacrystal) {
        const float r = (float)s[0];
        return a.contrast * k43pi * r * r * r * sph3j_d(q * s[0]);
    } else if constexpr (KIND == kPringle || KIND == kFlexCylEll || KIND == kFlexCyl) {
        return 0.0f;   // F^2 comes from pringle_f2 / flexcyl_f2
    } else if constexpr (KIND == kSuperball) {
        const float r = (float)s[0];
        return a.contrast * r * r * r * superball_sum(a, (float)(qa * s[0]), (float)(qb * s[0]), (float)(qc * s[0]));
    } else if constexpr (KIND == kCoreShellParallelepiped) {
        // the core box and the face slabs, each pair 2 cos(Q (edge + t)/2) times one slab
        const float A = (float)s[0], B = (float)s[1], C = (float)s[2];
        const float sa = sinc_d(0.5 * qa * s[0]), sb = sinc_d(0.5 * qb * s[1]), sc = sinc_d(0.5 * qc * s[2]);
        float sn, ca, cb, cc;
        sincos_phase(0.5 * qa * (s[0] + a.csp_t[0]), sn, ca);
        sincos_phase(0.5 * qb * (s[1] + a.csp_t[1]), sn, cb);
        sincos_phase(0.5 * qc * (s[2] + a.csp_t[2]), sn, cc);
        const float ta = a.fcsp_t[0], tb = a.fcsp_t[1], tc = a.fcsp_t[2];
        const float slabs = 2.0f * (ca * ta * B * C * sinc_d(0.5 * qa * a.csp_t[0]) * sb * sc
                                    + cb * A * tb * C * sa * sinc_d(0.5 * qb * a.csp_t[1]) * sc
                                    + cc * A * B * tc * sa * sb * sinc_d(0.5 * qc * a.csp_t[2]));
        return a.contrast * A * B * C * sa * sb * sc + a.cs_shell * slabs;
    } else {
        return a.contrast * (float)s[0] * (float)s[1] * (float)s[2] * sinc_d(0.5 * qa * s[0])
             * sinc_d(0.5 * qb * s[1]) * sinc_d(0.5 * qc * s[2]);
    }
}

// F in FP32 throughout (quadrature loops; sizes s and projections FP32).
template <int KIND>
__device__ __forceinline__ float amplitude_f(const TraceArgs& a, const float s[3], float q, float qa,
                                             float qb, float qc, float y)
{
    constexpr float k43pi = (float)(4.0 / 3.0 * kPi);
    if constexpr (KIND == kSphere) {
        const float r = s[0];
        return a.contrast * k43pi * r * r * r * sph3j_f(q * r);
    } else if constexpr (KIND == kCoreShell) {
        const float rc = s[0], ro = s[0] + a.fshell;
        return a.cs_core * k43pi * rc * rc * rc * sph3j_f(q * rc)
             + a.cs_shell * k43pi * ro * ro * ro * sph3j_f(q * ro);
    } else if constexpr (KIND == kCylinder) {
        const float r = s[0], len = s[1];
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        return a.contrast * (float)kPi * r * r * len * sinc_f(0.5f * qc * len) * lambda1_f(qab * r);
    } else if constexpr (KIND == kEllipsoid) {
        const float xa = qa * s[0], xb = qb * s[1], xc = qc * s[2];
        const float x = sqrtf(xa * xa + xb * xb + xc * xc);
        return a.contrast * k43pi * s[0] * s[1] * s[2] * sph3j_f(x);
    } else if constexpr (KIND == kBarbell || KIND == kCappedCylinder) {
        const float r = s[0], len = s[1];
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        const float cyl = (float)kPi * r * r * len * sinc_f(0.5f * qc * len) * lambda1_f(qab * r);
        const float qcy = qc * y;
        float sP, cP;
        sincos_f(qcy * a.fcap_zc, sP, cP);
        const float caps = caps_sum(a, sP, cP, qcy * a.fcap_r, qab * y);
        return a.contrast * __builtin_fmaf(y * y * y, caps, cyl);
    } else if constexpr (KIND == kHollowPrism) {
        float sa, ca, sb, cb, sc, cc;
        sinc_cos_f(0.5f * qa * s[0], sa, ca);
        sinc_cos_f(0.5f * qb * s[1], sb, cb);
        sinc_cos_f(0.5f * qc * s[2], sc, cc);
        return a.contrast * a.fshell * hollow_faces(s[0], s[1], s[2], sa, ca, sb, cb, sc, cc);
    } else if constexpr (KIND == kHollowCylinder) {
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        const float ri = s[0], ro = s[0] + a.fshell, len = s[1];
        const float ring = ro * ro * lambda1_f(qab * ro) - ri * ri * lambda1_f(qab * ri);
        return a.contrast * (float)kPi * len * sinc_f(0.5f * qc * len) * ring;
    } else if constexpr (KIND == kCoreShellCylinder) {
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        const float r = s[0], len = s[1], ro = s[0] + a.fshell, lo = __builtin_fmaf(2.0f, a.fcs_face, s[1]);
        const float core = r * r * len * sinc_f(0.5f * qc * len) * lambda1_f(qab * r);
        const float outer = ro * ro * lo * sinc_f(0.5f * qc * lo) * lambda1_f(qab * ro);
        return (float)kPi * __builtin_fmaf(a.cs_core, core, a.cs_shell * outer);
    } else if constexpr (KIND == kCoreShellEllipsoid) {
        const float oa = s[0] + a.fshell, ob = s[1] + a.fshell, oc = s[2] + a.fshell;
        const float xa = qa * s[0], xb = qb * s[1], xc = qc * s[2];
        const float ya = qa * oa, yb = qb * ob, yc = qc * oc;
        const float core = s[0] * s[1] * s[2] * sph3j_f(sqrtf(xa * xa + xb * xb + xc * xc));
        const float outer = oa * ob * oc * sph3j_f(sqrtf(ya * ya + yb * yb + yc * yc));
        return k43pi * __builtin_fmaf(a.cs_core, core, a.cs_shell * outer);
    } else if constexpr (KIND == kHollowPrismThick) {
        const float t2 = 2.0f * a.fshell;
        const float ia = s[0] - t2, ib = s[1] - t2, ic = s[2] - t2;
        const float box = s[0] * s[1] * s[2] * sinc_f(0.5f * qa * s[0]) * sinc_f(0.5f * qb * s[1])
                        * sinc_f(0.5f * qc * s[2]);
        const float cav = ia * ib * ic * sinc_f(0.5f * qa * ia) * sinc_f(0.5f * qb * ib) * sinc_f(0.5f * qc * ic);
        return a.contrast * (box - cav);
    } else if constexpr (KIND == kEllipticalCylinder) {
        const float xa = qa * s[0], xb = qb * s[1];
        return a.contrast * (float)kPi * s[0] * s[1] * s[2] * sinc_f(0.5f * qc * s[2])
             * lambda1_f(sqrtf(__builtin_fmaf(xa, xa, xb * xb)));
    } else if constexpr (KIND == kCoreShellBicelle) {
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        const float r = s[0], len = s[1], lf = __builtin_fmaf(2.0f, a.fcs_face, s[1]), ro = s[0] + a.fshell;
        const float disc = lambda1_f(qab * r), ends = sinc_f(0.5f * qc * lf);
        const float core = r * r * len * sinc_f(0.5f * qc * len) * disc;
        const float faces = r * r * lf * ends * disc;
        const float outer = ro * ro * lf * ends * lambda1_f(qab * ro);
        return (float)kPi * (a.bi_c[0] * core + a.bi_c[1] * faces + a.bi_c[2] * outer);
    } else if constexpr (KIND == kCoreShellBicelleElliptical) {
        const float ra = s[0], rb = (float)a.bi_x * s[0], oa = ra + a.fshell, ob = rb + a.fshell;
        const float lf = __builtin_fmaf(2.0f, a.fcs_face, s[1]);
        const float xa1 = ra * qa, xb1 = rb * qb, xa2 = oa * qa, xb2 = ob * qb;
        const float d1 = lambda1_f(sqrtf(__builtin_fmaf(xa1, xa1, xb1 * xb1)));
        const float d2 = lambda1_f(sqrtf(__builtin_fmaf(xa2, xa2, xb2 * xb2)));
        const float ends = sinc_f(0.5f * qc * lf);
        const float core = ra * rb * s[1] * sinc_f(0.5f * qc * s[1]) * d1;
        const float faces = ra * rb * lf * ends * d1;
        const float outer = oa * ob * lf * ends * d2;
        return (float)kPi * (a.bi_c[0] * core + a.bi_c[1] * faces + a.bi_c[2] * outer);
    } else if constexpr (KIND == kBicelleBeltRough) {
        const float ra = s[0], rb = (float)a.bi_x * s[0], oa = ra + a.fshell, ob = rb + a.fshell;
        const float lf = __builtin_fmaf(2.0f, a.fcs_face, s[1]);
        const float xa1 = ra * qa, xb1 = rb * qb, xa2 = oa * qa, xb2 = ob * qb;
        const float d1 = lambda1_f(sqrtf(__builtin_fmaf(xa1, xa1, xb1 * xb1)));
        const float d2 = lambda1_f(sqrtf(__builtin_fmaf(xa2, xa2, xb2 * xb2)));
        const float mid = sinc_f(0.5f * qc * s[1]);
        const float core = ra * rb * s[1] * mid * d1;
        const float faces = ra * rb * lf * sinc_f(0.5f * qc * lf) * d1;
        const float belt = oa * ob * s[1] * mid * d2;
        const float rough = __expf(q * q * (float)a.bi_rough);
        return (float)kPi * rough * (a.bi_c[0] * core + a.bi_c[1] * faces + a.bi_c[2] * belt);
    } else if constexpr (KIND == kStackedDisks) {
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        const float r = s[0], lo = __builtin_fmaf(2.0f, a.fshell, s[1]), disc = lambda1_f(qab * r);
        const float core = r * r * s[1] * sinc_f(0.5f * qc * s[1]) * disc;
        const float outer = r * r * lo * sinc_f(0.5f * qc * lo) * disc;
        return (float)kPi * __builtin_fmaf(a.cs_core, core, a.cs_shell * outer);
    } else if constexpr (KIND == kScParacrystal || KIND == kBccParacrystal || KIND == kFccParacrystal) {
        return a.contrast * k43pi * s[0] * s[0] * s[0] * sph3j_f(q * s[0]);
    } else if constexpr (KIND == kPringle || KIND == kFlexCylEll || KIND == kFlexCyl) {
        return 0.0f;   // no quadrature mode for these (refused at validation)
    } else if constexpr (KIND == kSuperball) {
        return a.contrast * s[0] * s[0] * s[0] * superball_sum(a, qa * s[0], qb * s[0], qc * s[0]);
    } else if constexpr (KIND == kCoreShellParallelepiped) {
        const float A = s[0], B = s[1], C = s[2];
        const float ta = a.fcsp_t[0], tb = a.fcsp_t[1], tc = a.fcsp_t[2];
        const float sa = sinc_f(0.5f * qa * A), sb = sinc_f(0.5f * qb * B), sc = sinc_f(0.5f * qc * C);
        float sn, ca, cb, cc;
        sincos_f(0.5f * qa * (A + ta), sn, ca);
        sincos_f(0.5f * qb * (B + tb), sn, cb);
        sincos_f(0.5f * qc * (C + tc), sn, cc);
        const float slabs = 2.0f * (ca * ta * B * C * sinc_f(0.5f * qa * ta) * sb * sc
                                    + cb * A * tb * C * sa * sinc_f(0.5f * qb * tb) * sc
                                    + cc * A * B * tc * sa * sb * sinc_f(0.5f * qc * tc));
        return a.contrast * A * B * C * sa * sb * sc + a.cs_shell * slabs;
    } else {
        return a.contrast * s[0] * s[1] * s[2] * sinc_f(0.5f * qa * s[0]) * sinc_f(0.5f * qb * s[1])
             * sinc_f(0.5f * qc * s[2]);
    }
}

// ---------------------------------------------------------------- exact average
// <F^2>(q) over the Schulz size nodes and (isotropic) the orientation nodes
// lq = mu[n] wmu[n] cb[n] sb[n] wb[n] st[n] y[ny] wy[ny], with st =
// sqrt(1 - mu^2), read from global memory: every lane of a wave reads the
// same node at the same time, so the reads go through the scalar data cache
// into scalar registers (no LDS traffic, no vector registers for them).  The parallelepiped's amplitude is a product of one
// factor per axis, so its C factor (which depends on mu only) leaves the
// inner beta sum: <F^2> = sum_i w_i F_C(mu_i)^2 sum_l w_l F_A^2 F_B^2.
// part/nparts: this call sums only every nparts-th node of the outermost
// loop with more than one node (sizes if there are several, else mu),
// starting at part; the nparts partial sums add up to the average.
template <int KIND>
__device__ __forceinline__ float quad_average(const TraceArgs& a, const float* __restrict__ lq, float q,
                                              const float qv[3], int part = 0, int nparts = 1)
{
    const int n = a.quad_n, ny = a.quad_ny;
    const float* mu = lq;
    const float* wmu = lq + n;
    const float* cb = lq + 2 * n;
    const float* sb = lq + 3 * n;
    const float* wb = lq + 4 * n;
    const float* stt = lq + 5 * n;
    const float* ys = lq + kQuadArrays * n;
    const float* wy = lq + kQuadArrays * n + ny;
    float qa0 = 0.0f, qb0 = 0.0f, qc0 = 0.0f;
    if (a.quad_dims == 0 && kAniso<KIND>) {
        qa0 = qv[0] * a.fA[0] + qv[1] * a.fA[1] + qv[2] * a.fA[2];
        qb0 = qv[0] * a.fB[0] + qv[1] * a.fB[1] + qv[2] * a.fB[2];
        qc0 = qv[0] * a.fC[0] + qv[1] * a.fC[1] + qv[2] * a.fC[2];
    }
    const bool split_sizes = ny > 1;
    const int j0 = split_sizes ? part : 0, jstep = split_sizes ? nparts : 1;
    const int i0 = split_sizes ? 0 : part, istep = split_sizes ? 1 : nparts;
    float total = 0.0f;
    for (int j = j0; j < ny; j += jstep) {
        const float y = ys[j];
        float s[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] = (a.poly_mask >> c & 1) ? a.fsize[c] * y : a.fsize[c];
        float avg = 0.0f;
        if (a.quad_dims == 0) {
            float f2;
            if constexpr (KIND == kMicelle) {
                f2 = micelle_f2(a, s[0], s[1], (double)q);
            } else if constexpr (kShapeIndependent<KIND>) {
                f2 = shape_iq<KIND>(a, a.size[0], (double)q);
            } else if constexpr (kLamellar<KIND>) {
                f2 = lamellar_f2<KIND>(a, (double)q);
            } else if constexpr (kSphereFamily<KIND>) {
                f2 = sphere_family_f2<KIND>(a, s[0], (double)q);
            } else {
                const float f = amplitude_f<KIND>(a, s, q, qa0, qb0, qc0, y);
                f2 = f * f;
                if constexpr (kLattice<KIND>) f2 *= lattice_factor<KIND>(a, q, qa0, qb0, qc0);
            }
            avg = i0 == 0 ? f2 : 0.0f;
        } else if (a.quad_dims == 1) {
            bool done = false;
            if constexpr (KIND == kEllipsoid) {
                // spheroid (a = b): x^2 = (q a sin)^2 + (q c mu)^2; when every
                // lane's x stays within the long series' range, no branch
                const float qa = q * s[0], qc = q * s[2];
                if (__all(fmaxf(qa, qc) <= kSphLongMax)) {
                    float sum = 0.0f;
#pragma unroll 4
                    for (int i = i0; i < n; i += istep) {
                        const float xa = qa * stt[i], xc = qc * mu[i];
                        const float p = sph3j_long(__builtin_fmaf(xa, xa, xc * xc));
                        sum = __builtin_fmaf(wmu[i], p * p, sum);
                    }
                    const float f0 = a.contrast * (float)(4.0 / 3.0 * kPi) * s[0] * s[1] * s[2];
                    avg = f0 * f0 * sum;
                    done = true;
                }
            }
            if (!done) {
#pragma unroll 4
                for (int i = i0; i < n; i += istep) {
                    const float f = amplitude_f<KIND>(a, s, q, q * stt[i], 0.0f, q * mu[i], y);
                    float f2 = f * f;
                    if constexpr (kLattice<KIND>) f2 *= lattice_factor<KIND>(a, q, q * stt[i], 0.0f, q * mu[i]);
                    avg = __builtin_fmaf(wmu[i], f2, avg);
                }
            }
        } else if constexpr (KIND == kParallelepiped) {
            const float f0 = a.contrast * s[0] * s[1] * s[2];
            const float ha = 0.5f * q * s[0], hb = 0.5f * q * s[1], hc = 0.5f * q * s[2];
            // the A and B arguments never exceed ha and hb (|st cb|, |st sb| <= 1):
            // when they stay within the short series' range across the wave,
            // every inner node takes it, without a branch
            if (__all(fmaxf(ha, hb) <= kSincShortMax)) {
                for (int i = i0; i < n; i += istep) {
                    const float fc = sinc_f(hc * mu[i]);
                    const float xa = ha * stt[i], xb = hb * stt[i];
                    float inner = 0.0f;
#pragma unroll 4
                    for (int l = 0; l < n; ++l) {
                        const float g = sinc_short(xa * cb[l]) * sinc_short(xb * sb[l]);
                        inner = __builtin_fmaf(wb[l], g * g, inner);
                    }
                    avg = __builtin_fmaf(wmu[i] * fc * fc, inner, avg);
                }
            } else {
                for (int i = i0; i < n; i += istep) {
                    const float fc = sinc_f(hc * mu[i]);
                    const float xa = ha * stt[i], xb = hb * stt[i];
                    float inner = 0.0f;
#pragma unroll 4
                    for (int l = 0; l < n; ++l) {
                        const float g = sinc_f(xa * cb[l]) * sinc_f(xb * sb[l]);
                        inner = __builtin_fmaf(wb[l], g * g, inner);
                    }
                    avg = __builtin_fmaf(wmu[i] * fc * fc, inner, avg);
                }
            }
            avg *= f0 * f0;
        } else if constexpr (KIND == kHollowPrism) {
            // the C axis' sinc and cos depend on mu only
            const float f0 = a.contrast * a.fshell;
            const float ha = 0.5f * q * s[0], hb = 0.5f * q * s[1], hc = 0.5f * q * s[2];
            for (int i = i0; i < n; i += istep) {
                float sc, cc;
                sinc_cos_f(hc * mu[i], sc, cc);
                const float xa = ha * stt[i], xb = hb * stt[i];
                float inner = 0.0f;
#pragma unroll 2
                for (int l = 0; l < n; ++l) {
                    float s_a, c_a, s_b, c_b;
                    sinc_cos_f(xa * cb[l], s_a, c_a);
                    sinc_cos_f(xb * sb[l], s_b, c_b);
                    const float g = hollow_faces(s[0], s[1], s[2], s_a, c_a, s_b, c_b, sc, cc);
                    inner = __builtin_fmaf(wb[l], g * g, inner);
                }
                avg = __builtin_fmaf(wmu[i], inner, avg);
            }
            avg *= f0 * f0;
        } else {
            for (int i = i0; i < n; i += istep) {
                const float qst = q * stt[i];
                const float qc = q * mu[i];
                float inner = 0.0f;
                for (int l = 0; l < n; ++l) {
                    const float f = amplitude_f<KIND>(a, s, q, qst * cb[l], qst * sb[l], qc, y);
                    float f2 = f * f;
                    if constexpr (kLattice<KIND>) f2 *= lattice_factor<KIND>(a, q, qst * cb[l], qst * sb[l], qc);
                    inner = __builtin_fmaf(wb[l], f2, inner);
                }
                avg = __builtin_fmaf(wmu[i], inner, avg);
            }
        }
        total = __builtin_fmaf(wy[j], avg, total);
    }
    return total;
}

// ---------------------------------------------------------------- one neutron
// Flexible cylinder with an elliptical cross-section: (drho V)^2 P_chain
// P_cs with V = pi eps R^2 L.  P_chain by Kholodenko's closed form for the
// wormlike chain: x = 3 L/b, (2/x)(I_1 - I_2/x), I_n = int_0^x f(z) z^(n-1)
// dz, f = sinh(E z)/(E sinh z), E = sqrt(1 - (q b/3)^2), below q b = 3 and
// sin(F z)/(F sinh z), F = sqrt((q b/3)^2 - 1), above, both integrals by the
// n-point Gauss-Legendre rule on [0, x_e] (x_e = min(x, 40/(1 - E)) or
// min(x, 40): the integrands fall as exp(-(1 - E) z) and exp(-z)), f written
// without overflow as exp((E - 1) z) (1 - e^(-2 E z))/(E (1 - e^(-2 z)));
// P_cs the average of [2 J1(q r)/(q r)]^2 over the in-plane angle psi,
// r = R sqrt(sin^2 psi + eps^2 cos^2 psi), by the same rule.  cap_nodes:
// [t_k, w_k] on [0, 1] (n each), then [sin^2 psi_k, cos^2 psi_k, w_k/...]
// with the section's weights summing to 1.  ELL false: the circular
// section, [2 J1(q R)/(q R)]^2 itself (eps = 1, no average).
template <bool ELL>
__device__ __forceinline__ float flexcyl_f2(const TraceArgs& a, double Rd, double Ld, double qd)
{
    const int n = a.cap_n;
    const float* __restrict__ t = a.cap_nodes;
    const float* __restrict__ tw = a.cap_nodes + n;
    const float* __restrict__ s2 = a.cap_nodes + 2 * n;
    const float* __restrict__ c2 = a.cap_nodes + 3 * n;
    const float* __restrict__ sw = a.cap_nodes + 4 * n;
    const float R = (float)Rd, L = (float)Ld, q = (float)qd, b = a.fc_b, eps = a.fc_eps;
    const float x = 3.0f * L / b, v = q * b * (1.0f / 3.0f);
    const bool below = v < 1.0f;
    const float E = below ? sqrtf(1.0f - v * v) : 0.0f, F = below ? 0.0f : sqrtf(v * v - 1.0f);
    const float em1 = -v * v / (1.0f + E);           // E - 1 without cancellation
    float xe = x;
    if (below && em1 < 0.0f) xe = fminf(xe, -40.0f / em1);
    if (!below) xe = fminf(xe, 40.0f);
    float i1 = 0.0f, i2 = 0.0f;
    for (int k = 0; k < n; ++k) {
        const float z = xe * t[k], wz = xe * tw[k];
        const float den = -expm1f(-2.0f * z);
        float f;
        if (below) {
            const float num = E > 0.0f ? -expm1f(-2.0f * E * z) / E : 2.0f * z;
            f = expf(em1 * z) * num / den;
        } else {
            f = 2.0f * (F > 0.0f ? sinf(F * z) / F : z) * expf(-z) / den;
        }
        i1 = __builtin_fmaf(wz, f, i1);
        i2 = __builtin_fmaf(wz * f, z, i2);
    }
    const float chain = 2.0f / x * (i1 - i2 / x);
    float sec = 0.0f;
    if constexpr (ELL) {
        for (int k = 0; k < n; ++k) {
            const float r = R * sqrtf(__builtin_fmaf(eps * eps, c2[k], s2[k]));
            const float l = lambda1_f(q * r);
            sec = __builtin_fmaf(sw[k], l * l, sec);
        }
    } else {
        const float l = lambda1_f(q * R);
        sec = l * l;
    }
    const float fv = a.contrast * (float)kPi * eps * R * R * L;
    return fv * fv * chain * sec;
}

// ---------------------------------------------------------------- geometry
// One neutron's flight (A3-A6, A12): the chord through the slab, |Q|, the
// pixel, and what the weight and the attenuation need.
struct Geom {
    bool in_sample, on_det;
    int32_t pixel;
    float len;            // chord through the slab (m)
    double qd;            // |Q| (1/A), FP64: the amplitudes' phases are formed from it
    double qv[3];         // Q in the lab frame (anisotropic models)
    float path_in;        // path inside the slab before the scattering point (m)
    float px, py, pz;     // scattering point (m; attenuation)
    float fx, fy, fz;     // outgoing direction (attenuation)
};

// The flight in FP64 (the reference arithmetic of the pixel): source and
// slit points, the slab by the z faces when the path stays clear of the side
// faces (else the three-axis intersection), the cone about the flight
// direction with the basis of Duff et al. (JCGT 2017), the detector plane.
template <bool ANISO, bool ATT>
__device__ __forceinline__ void geom_f64(const TraceArgs& a, const U4& r0, const U4& r1, Geom& g)
{
    const double sx = centred_u(r0.x) * a.src_w, sy = centred_u(r0.y) * a.src_h;
    const double tx = centred_u(r0.z) * a.slit_w, ty = centred_u(r0.w) * a.slit_h;
    const double dx = tx - sx, dy = ty - sy, dz = a.slit_z - a.src_z;
    const double dl = sqrt_d(dx * dx + dy * dy + dz * dz);
    const double idl = rcp_d(dl);
    const double kx = dx * idl, ky = dy * idl, kz = dz * idl;
    const double lambda = __builtin_fma(a.lambda_span, 2.0 * u64(r1.x) - 1.0, a.lambda0);
    const double k = div_d(2.0 * kPi, lambda);

    // slab entry/exit along src + s k, s >= 0.  The beam axis first: when
    // the path between the two z faces stays clear of the x and y faces at
    // both ends (by a margin of 1e-9 of the half-widths, far above the
    // rounding of the crossing points), those faces cannot cut it, and the
    // three-axis intersection below would select exactly the z crossings.
    double s_in = 0.0, s_out = 1e300;
    bool clear = false;
    if (kz != 0.0) {
        const double inv = rcp_d(kz);
        const double t1 = (-a.half_z - a.src_z) * inv, t2 = (a.half_z - a.src_z) * inv;
        const double zin = fmax(0.0, fmin(t1, t2)), zout = fmax(t1, t2);
        const double xa = __builtin_fma(zin, kx, sx), xb = __builtin_fma(zout, kx, sx);
        const double ya = __builtin_fma(zin, ky, sy), yb = __builtin_fma(zout, ky, sy);
        clear = fmax(fabs(xa), fabs(xb)) < a.clear_x && fmax(fabs(ya), fabs(yb)) < a.clear_y;
        s_in = zin;
        s_out = zout;
    }
    if (!clear) {
        s_in = 0.0;
        s_out = 1e300;
        const double o[3] = {sx, sy, a.src_z};
        const double dv[3] = {kx, ky, kz};
        const double h[3] = {a.half_x, a.half_y, a.half_z};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (dv[c] != 0.0) {
                const double inv = rcp_d(dv[c]);
                const double t1 = (-h[c] - o[c]) * inv, t2 = (h[c] - o[c]) * inv;
                s_in = fmax(s_in, fmin(t1, t2));
                s_out = fmin(s_out, fmax(t1, t2));
            } else if (fabs(o[c]) > h[c]) {
                s_out = -1.0;
            }
        }
    }
    // no early exit: a miss is carried as a flag
    const bool in_sample = s_out > s_in;
    const double len = in_sample ? s_out - s_in : 0.0;
    const double sp = __builtin_fma(u64(r1.y), len, s_in);
    const double rx = __builtin_fma(sp, kx, sx), ry = __builtin_fma(sp, ky, sy),
                 rz = __builtin_fma(sp, kz, a.src_z);

    // cone sampling about the flight direction
    const double t = u64(r1.z) * a.omc;
    const double c2 = 1.0 - t;
    const double s2 = sqrt_d(t * (2.0 - t));
    double sps, cps;
    sincospi(2.0 * u64(r1.w), &sps, &cps);
    const double sg = kz >= 0.0 ? 1.0 : -1.0;
    const double aa = -rcp_d(sg + kz);
    const double bb = kx * ky * aa;
    const double px = cps * (1.0 + sg * kx * kx * aa) + sps * bb;
    const double py = cps * (sg * bb) + sps * (sg + ky * ky * aa);
    const double pz = cps * (-sg * kx) + sps * (-ky);
    const double fx = c2 * kx + s2 * px, fy = c2 * ky + s2 * py, fz = c2 * kz + s2 * pz;
    const double qd = k * sqrt_d(2.0 * t);

    // detector plane and pixel
    const bool forward = fz > 0.0;
    const double sd = div_d(a.det_z - rz, fz);
    const double xd = __builtin_fma(sd, fx, rx), yd = __builtin_fma(sd, fy, ry);
    const double fxp = floor((xd + a.det_hw) * a.inv_px);
    const double fyp = floor((yd + a.det_hh) * a.inv_py);
    g.in_sample = in_sample;
    g.on_det = in_sample && forward && fxp >= 0.0 && fxp < (double)a.nx && fyp >= 0.0 && fyp < (double)a.ny;
    g.pixel = g.on_det ? (int32_t)fyp * a.nx + (int32_t)fxp : -1;
    g.len = (float)len;
    g.qd = qd;
    if constexpr (ANISO) {
        g.qv[0] = k * __builtin_fma(s2, px, -t * kx);
        g.qv[1] = k * __builtin_fma(s2, py, -t * ky);
        g.qv[2] = k * __builtin_fma(s2, pz, -t * kz);
    }
    if constexpr (ATT) {
        g.path_in = (float)(sp - s_in);
        g.px = (float)rx;
        g.py = (float)ry;
        g.pz = (float)rz;
        g.fx = (float)fx;
        g.fy = (float)fy;
        g.fz = (float)fz;
    }
}

// ---------------------------------------------------------------- guide
// Supermirror reflectivity: R0 up to Qc, then R0/2 (1 - tanh((Q - m Qc)/W))
// (1 - alpha (Q - Qc)), 0 where negative.
__device__ __forceinline__ double guide_reflectivity(const TraceArgs& a, double q)
{
    if (q <= a.guide_qc) return a.guide_r0;
    const double r = 0.5 * a.guide_r0 * (1.0 - tanh((q - a.guide_m * a.guide_qc) / a.guide_wc))
                     * (1.0 - a.guide_alpha * (q - a.guide_qc));
    return fmax(r, 0.0);
}

// The guide's weight of a neutron that reaches the source aperture at
// (sx, sy) flying along the unit vector k with wavelength lambda: back to the
// exit plane (outside the exit: 0), then through the guide as the straight
// line unfolded across the walls -- a wall plane crossed is a reflection at
// the same grazing angle, |floor((x_entrance + w/2)/w)| of them across x
// (likewise y) -- R(Q_x)^n_x R(Q_y)^n_y, Q = 4 pi |k_x| / lambda.
__device__ __forceinline__ double guide_weight(const TraceArgs& a, double sx, double sy, const double k[3],
                                               double lambda)
{
    const double ikz = rcp_d(k[2]);
    const double ex = sx - a.guide_gap * k[0] * ikz, ey = sy - a.guide_gap * k[1] * ikz;
    if (fabs(ex) > a.guide_hw || fabs(ey) > a.guide_hh) return 0.0;
    const double xu = ex - a.guide_len * k[0] * ikz, yu = ey - a.guide_len * k[1] * ikz;
    const double nx = fabs(floor((xu + a.guide_hw) / (2.0 * a.guide_hw)));
    const double ny = fabs(floor((yu + a.guide_hh) / (2.0 * a.guide_hh)));
    const double fq = 4.0 * kPi / lambda;
    double w = 1.0;
    if (nx > 0.0) w *= pow(guide_reflectivity(a, fq * fabs(k[0])), nx);
    if (ny > 0.0) w *= pow(guide_reflectivity(a, fq * fabs(k[1])), ny);
    return w;
}

// The guide's weight of neutron (r0, r1): its source and slit points and
// wavelength as in its flight (FP64).
__device__ __forceinline__ double guide_weight_of(const TraceArgs& a, const U4& r0, const U4& r1)
{
    const double sx = centred_u(r0.x) * a.src_w, sy = centred_u(r0.y) * a.src_h;
    const double tx = centred_u(r0.z) * a.slit_w, ty = centred_u(r0.w) * a.slit_h;
    const double dx = tx - sx, dy = ty - sy, dz = a.slit_z - a.src_z;
    const double idl = rcp_d(sqrt_d(dx * dx + dy * dy + dz * dz));
    const double k[3] = {dx * idl, dy * idl, dz * idl};
    const double lambda = __builtin_fma(a.lambda_span, 2.0 * u64(r1.x) - 1.0, a.lambda0);
    return guide_weight(a, sx, sy, k, lambda);
}

// ---------------------------------------------------------------- transmitted beam
// The unscattered neutron: its straight flight from the source point through
// the slit point (the first Philox block, as in its scattered flight), the
// chord through the slab along it and the pixel where it meets the detector
// plane; weight exp(-mu_att chord), 1 when it misses the slab.
struct Straight {
    int32_t pixel;   // -1: off the detector
    double w;
};

__device__ __forceinline__ Straight straight_flight(const TraceArgs& a, uint64_t i)
{
    const U4 r0 = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), 0u, a.exp_id, a.seed_lo, a.seed_hi);
    const double sx = centred_u(r0.x) * a.src_w, sy = centred_u(r0.y) * a.src_h;
    const double tx = centred_u(r0.z) * a.slit_w, ty = centred_u(r0.w) * a.slit_h;
    const double dx = tx - sx, dy = ty - sy, dz = a.slit_z - a.src_z;
    const double idl = rcp_d(sqrt_d(dx * dx + dy * dy + dz * dz));
    const double dv[3] = {dx * idl, dy * idl, dz * idl};
    const double o[3] = {sx, sy, a.src_z};
    const double h[3] = {a.half_x, a.half_y, a.half_z};
    double s_in = 0.0, s_out = 1e300;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (dv[c] != 0.0) {
            const double inv = rcp_d(dv[c]);
            const double t1 = (-h[c] - o[c]) * inv, t2 = (h[c] - o[c]) * inv;
            s_in = fmax(s_in, fmin(t1, t2));
            s_out = fmin(s_out, fmax(t1, t2));
        } else if (fabs(o[c]) > h[c]) {
            s_out = -1.0;
        }
    }
    const double chord = s_out > s_in ? s_out - s_in : 0.0;
    Straight st{-1, 0.0};
    if (!(dv[2] > 0.0)) return st;
    const double sd = div_d(a.det_z - a.src_z, dv[2]);
    const double xd = __builtin_fma(sd, dv[0], sx), yd = __builtin_fma(sd, dv[1], sy);
    const double fxp = floor((xd + a.det_hw) * a.inv_px);
    const double fyp = floor((yd + a.det_hh) * a.inv_py);
    if (fxp >= 0.0 && fxp < (double)a.nx && fyp >= 0.0 && fyp < (double)a.ny) {
        st.pixel = (int32_t)fyp * a.nx + (int32_t)fxp;
        st.w = exp(-a.mu_att * chord);
        if (a.guide_on) {
            const U4 r1 = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), 1u, a.exp_id, a.seed_lo, a.seed_hi);
            const double lambda = __builtin_fma(a.lambda_span, 2.0 * u64(r1.x) - 1.0, a.lambda0);
            st.w *= guide_weight(a, sx, sy, dv, lambda);
        }
    }
    return st;
}

// The same flight in FP32 for isotropic models, measured from the slab rather
// than the source (the entry point through the slopes dx/dz, dy/dz; the chord
// as depth x |k|/k_z), which leaves no cancellation.  |Q| = k sqrt(2t) needs
// only the wavelength and the cone draw and stays FP64 (the amplitudes' phases
// reach tens of radians, where FP32 would lose the pixel bar's 1e-4 in
// sparse pixels); an anisotropic model's Q vector also needs the direction to
// better than FP32, so those models take geom_f64 throughout.  Its pixel coordinates carry an
// error below 2e-7 m (rounding of the ~0.3 m lever arm to the detector and of
// the direction); a neutron whose coordinates lie within the margin f_eps_x,
// f_eps_y (6e-7 m) of a pixel edge, whose path comes near a side face of the
// slab or whose outgoing direction is far from the beam axis is not decided
// here (false): the caller takes geom_f64.  Every neutron decided here lands
// in the pixel geom_f64 gives it.
template <bool ATT>
__device__ __forceinline__ bool geom_f32(const TraceArgs& a, const U4& r0, const U4& r1, Geom& g)
{
    const float sx = centred_uf(r0.x) * a.f_src_w, sy = centred_uf(r0.y) * a.f_src_h;
    const float tx = centred_uf(r0.z) * a.f_slit_w, ty = centred_uf(r0.w) * a.f_slit_h;
    const float mx = (tx - sx) * a.f_inv_dz, my = (ty - sy) * a.f_inv_dz;
    // entry and exit points on the z faces
    const float xa = __builtin_fmaf(a.f_lz_in, mx, sx), xb = __builtin_fmaf(a.f_lz_out, mx, sx);
    const float ya = __builtin_fmaf(a.f_lz_in, my, sy), yb = __builtin_fmaf(a.f_lz_out, my, sy);
    const bool clear = fmaxf(fabsf(xa), fabsf(xb)) < a.f_clear_x && fmaxf(fabsf(ya), fabsf(yb)) < a.f_clear_y;
    const float g2 = __builtin_fmaf(mx, mx, __builtin_fmaf(my, my, 1.0f));
    const float rn = __builtin_amdgcn_rsqf(g2);
    const float kz = rn, kx = mx * rn, ky = my * rn;
    const float len = a.f_depth * g2 * rn;                     // depth sqrt(1 + mx^2 + my^2)
    const float u5 = uf(r1.y);
    const float ud = u5 * a.f_depth;
    const float rx = __builtin_fmaf(ud, mx, xa), ry = __builtin_fmaf(ud, my, ya);
    const float rz = ud - a.f_half_z;

    // cone about k: psi = 2 pi u from the quarter turns of u
    const float t = uf(r1.z) * a.f_omc;
    const float c2 = 1.0f - t;
    const float s2 = __builtin_amdgcn_sqrtf(t * (2.0f - t));
    const float u7 = 4.0f * uf(r1.w);
    const float nq = rintf(u7);
    float sr, cr, sps, cps;
    sincos_poly((u7 - nq) * (float)(0.5 * kPi), sr, cr);
    quadrant((int)nq, sr, cr, sps, cps);
    const float aa = -rcpf(1.0f + kz);
    const float bb = kx * ky * aa;
    const float px = cps * __builtin_fmaf(kx * kx, aa, 1.0f) + sps * bb;
    const float py = cps * bb + sps * __builtin_fmaf(ky * ky, aa, 1.0f);
    const float pz = -(cps * kx + sps * ky);
    const float fx = __builtin_fmaf(c2, kx, s2 * px), fy = __builtin_fmaf(c2, ky, s2 * py);
    const float fz = __builtin_fmaf(c2, kz, s2 * pz);

    // detector plane, pixel coordinates
    const float sd = (a.f_det_z - rz) * rcpf(fz);
    const float X = (__builtin_fmaf(sd, fx, rx) + a.f_det_hw) * a.f_inv_px;
    const float Y = (__builtin_fmaf(sd, fy, ry) + a.f_det_hh) * a.f_inv_py;
    const bool near = fabsf(X - rintf(X)) < a.f_eps_x || fabsf(Y - rintf(Y)) < a.f_eps_y;
    const float fxp = floorf(X), fyp = floorf(Y);
    g.in_sample = true;
    g.on_det = fxp >= 0.0f && fxp < (float)a.nx && fyp >= 0.0f && fyp < (float)a.ny;
    g.pixel = g.on_det ? (int32_t)fyp * a.nx + (int32_t)fxp : -1;
    g.len = len;
    const double lambda = __builtin_fma(a.lambda_span, 2.0 * u64(r1.x) - 1.0, a.lambda0);
    g.qd = div_d(2.0 * kPi, lambda) * sqrt_d(2.0 * (u64(r1.z) * a.omc));
    if constexpr (ATT) {
        g.path_in = u5 * len;
        g.px = rx;
        g.py = ry;
        g.pz = rz;
        g.fx = fx;
        g.fy = fy;
        g.fz = fz;
    }
    return clear && !near && fz > a.f_fz_min;
}

struct Event {
    int32_t pixel;  // -1: not tallied
    float w;
    float q;        // 0 when the sample is missed
    float qlo;      // surrogate mode: |Q| - q, so that q + qlo carries |Q| in FP64
};

// Traces neutron i.  tab_size/tab_norm point to the LDS copies of the
// tables; lq to the LDS copy of the quadrature nodes (QUAD mode; with
// nparts > 1 the weight is this part's share of the exact average).
// ATT: the sample's attenuation is compiled in (the atomic-tally and
// per-neutron kernels; the others leave it out and the host routes attenuated
// runs to the atomic tallies)
template <int KIND, int MODE, bool ATT = false>
__device__ __forceinline__ Event trace_neutron(const TraceArgs& a, uint64_t i,
                                               const double* tab_size, const double* tab_norm,
                                               const float* lq, int part = 0, int nparts = 1)
{
    Event ev{-1, 0.0f, 0.0f, 0.0f};
    const uint32_t ilo = (uint32_t)i, ihi = (uint32_t)(i >> 32);
    const U4 r0 = philox4x32_10(ilo, ihi, 0u, a.exp_id, a.seed_lo, a.seed_hi);
    const U4 r1 = philox4x32_10(ilo, ihi, 1u, a.exp_id, a.seed_lo, a.seed_hi);

    Geom geo;
    bool exact = true;
    if constexpr (!kAniso<KIND>)
        if (a.fast_geom) exact = !geom_f32<ATT>(a, r0, r1, geo);
    if (exact) geom_f64<kAniso<KIND>, ATT>(a, r0, r1, geo);
    const bool in_sample = geo.in_sample, on_det = geo.on_det;
    const double qd = geo.qd;
    const float q = (float)qd;
    ev.q = in_sample ? q : 0.0f;
    if constexpr (MODE == 2) ev.qlo = in_sample ? (float)(qd - (double)q) : 0.0f;

    // attenuation along the path inside the slab, before the scattering point
    // and after it along k_f to the face where it leaves (when asked for)
    float att = 1.0f;
    if (ATT && a.att_on) {
        const float o[3] = {geo.px, geo.py, geo.pz}, dv[3] = {geo.fx, geo.fy, geo.fz};
        const float hw[3] = {(float)a.half_x, (float)a.half_y, (float)a.half_z};
        float tout = 3.0e38f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (dv[c] != 0.0f) tout = fminf(tout, ((dv[c] > 0.0f ? hw[c] : -hw[c]) - o[c]) * rcpf(dv[c]));
        att = expf(-(float)a.mu_att * (geo.path_in + tout));
    }

    // scattering vector in the lab frame (anisotropic models)
    double qvd[3] = {0.0, 0.0, 0.0};
    if constexpr (kAniso<KIND>) {
        qvd[0] = geo.qv[0];
        qvd[1] = geo.qv[1];
        qvd[2] = geo.qv[2];
    }
    // the weight (computed for every lane: the wave runs it anyway)
    float f2;
    if constexpr (MODE == 0) {
        double y = 1.0;
        double ys[3] = {1.0, 1.0, 1.0};   // independent size draws (1 when off)
        Trig3 g{a.ang_sin[0], a.ang_cos[0], a.ang_sin[1], a.ang_cos[1], a.ang_sin[2], a.ang_cos[2]};
        if (a.third_block) {
            const U4 r2 = philox4x32_10(ilo, ihi, 2u, a.exp_id, a.seed_lo, a.seed_hi);
            if (a.poly_on) y = fmax(table_lerp(tab_size, a.M, u64(r2.x)), 0.0);
            // independent size draws: size 0 from (block 2, x), sizes 1 and 2
            // from (block 3, x) and (block 3, y)
            if constexpr (kSepKind<KIND>) {
                if (a.sep_any) {
                    if (a.sep_on[0]) ys[0] = fmax(table_lerp(a.tab_sep, a.M, u64(r2.x)), 0.0);
                    if (a.sep_block3) {
                        const U4 r3 = philox4x32_10(ilo, ihi, 3u, a.exp_id, a.seed_lo, a.seed_hi);
                        if (a.sep_on[1]) ys[1] = fmax(table_lerp(a.tab_sep + a.M, a.M, u64(r3.x)), 0.0);
                        if (a.sep_on[2]) ys[2] = fmax(table_lerp(a.tab_sep + 2 * a.M, a.M, u64(r3.y)), 0.0);
                    }
                }
            }
            if constexpr (kAniso<KIND>) {
                if (a.orient_kind == 1) {
                    rotate_by(a.ang_sin[0], a.ang_cos[0],
                              a.ang_sigma[0] * table_lerp_u(tab_norm, a.M, u64(r2.y)), g.st, g.ct);
                    rotate_by(a.ang_sin[1], a.ang_cos[1],
                              a.ang_sigma[1] * table_lerp_u(tab_norm, a.M, u64(r2.z)), g.sp, g.cp);
                    if constexpr (!kOneAxis<KIND>)
                        rotate_by(a.ang_sin[2], a.ang_cos[2],
                                  a.ang_sigma[2] * table_lerp_u(tab_norm, a.M, u64(r2.w)), g.ss, g.cs);
                } else if (a.orient_kind == 2) {
                    // cos(theta) uniform in [-1, 1]; phi, Psi uniform in [0, 2 pi)
                    g.ct = __builtin_fma(2.0, u64(r2.y), -1.0);
                    g.st = sqrt(fmax(__builtin_fma(-g.ct, g.ct, 1.0), 0.0));
                    sincospi(2.0 * u64(r2.z), &g.sp, &g.cp);
                    if constexpr (!kOneAxis<KIND>) sincospi(2.0 * u64(r2.w), &g.ss, &g.cs);
                } else if (a.orient_kind == 3) {
                    // the literal rule: theta uniform in [0, pi)
                    sincospi(u64(r2.y), &g.st, &g.ct);
                    sincospi(2.0 * u64(r2.z), &g.sp, &g.cp);
                    if constexpr (!kOneAxis<KIND>) sincospi(2.0 * u64(r2.w), &g.ss, &g.cs);
                }
            }
        }
        double qa = 0.0, qb = 0.0, qc = 0.0;
        if constexpr (kAniso<KIND>) project<!kOneAxis<KIND>>(g, qvd, qa, qb, qc);
        if constexpr (KIND == kMicelle) {
            f2 = micelle_f2(a, (a.poly_mask & 1) ? a.size[0] * y : a.size[0],
                            (a.poly_mask & 2) ? a.size[1] * y : a.size[1], qd);
        } else if constexpr (kShapeIndependent<KIND>) {
            f2 = shape_iq<KIND>(a, a.size[0], qd);
        } else if constexpr (kLamellar<KIND>) {
            f2 = lamellar_f2<KIND>(a, qd);
        } else if constexpr (KIND == kPringle) {
            f2 = pringle_f2(a, (a.poly_mask & 1) ? y : 1.0, (a.poly_mask & 2) ? y : 1.0, qa, qb, qc);
        } else if constexpr (KIND == kFlexCylEll || KIND == kFlexCyl) {
            f2 = flexcyl_f2<KIND == kFlexCylEll>(a, (a.poly_mask & 1) ? a.size[0] * y : a.size[0],
                                                 (a.poly_mask & 2) ? a.size[1] * y : a.size[1], qd);
        } else if constexpr (kSphereFamily<KIND>) {
            f2 = sphere_family_f2<KIND>(a, (a.poly_mask & 1) ? a.size[0] * y : a.size[0], qd);
        } else {
            const float f = amplitude_mc<KIND>(a, y, ys, qd, qa, qb, qc);
            f2 = f * f;
            if constexpr (kLattice<KIND>) f2 *= lattice_factor<KIND>(a, qd, qa, qb, qc);
        }
    } else if constexpr (MODE == 1) {
        const float qv[3] = {(float)qvd[0], (float)qvd[1], (float)qvd[2]};
        f2 = quad_average<KIND>(a, a.quad_nodes, q, qv, part, nparts);
    } else {
        // MODE 2 (surrogate): the caller multiplies by the network's <F^2>
        f2 = 1.0f;
    }
    float w = geo.len * a.f_wscale * f2;
    if (a.sq_on) w *= struct_factor(a, q);
    if constexpr (ATT) {
        w *= att;
        if (a.guide_on) w *= (float)guide_weight_of(a, r0, r1);
    }
    if (on_det) {
        ev.pixel = geo.pixel;
        ev.w = w;
    }
    return ev;
}

}  // namespace sans
