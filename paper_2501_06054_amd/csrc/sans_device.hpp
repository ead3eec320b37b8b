// sans_device.hpp -- device code of the gfx950 SANS sample tracer.
//
// One neutron per lane.  The per-neutron steps:
//   1. Philox4x32-10 blocks of the neutron's counter (Salmon et al., SC'11);
//   2. source and slit points, wavelength, flight direction (FP64);
//   3. slab-sample entry and exit, scattering point (FP64);
//   4. outgoing direction uniform in the cone, scattering vector Q (FP64);
//   5. particle size and orientation from inverse-CDF tables staged in LDS
//      (Methods, "Polydispersity and orientational distributions"), FP32;
//   6. amplitude F of the model (Eqs. (5)-(7), (9)) and the hard-sphere
//      Percus-Yevick S(Q), FP32 VALU;
//   7. weight w = l dOmega n F^2 S (Eq. (3) with n = phi/<V>), FP32;
//   8. straight flight to the detector plane and the pixel index (FP64).
// Geometry stays FP64 so that the pixel a neutron lands in does not depend
// on rounding; the physics of the weight is FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sans {

// ---------------------------------------------------------------- constants
constexpr double kPi = 3.141592653589793238462643383;

constexpr double cfact(int n) { return n <= 1 ? 1.0 : n * cfact(n - 1); }
constexpr double cpow4(int m) { return m == 0 ? 1.0 : 4.0 * cpow4(m - 1); }

// Taylor coefficients in x^2 of 3 j1(x)/x: 3 (-1)^m 2(m+1) / (2m+3)!
constexpr double sph_coef(int m) { return (m % 2 ? -1.0 : 1.0) * 6.0 * (m + 1) / cfact(2 * m + 3); }
// Taylor coefficients in x^2 of 2 J1(x)/x: (-1)^m / (4^m m! (m+1)!)
constexpr double lam_coef(int m) { return (m % 2 ? -1.0 : 1.0) / (cpow4(m) * cfact(m) * cfact(m + 1)); }
// Taylor coefficients in x^2 of sin(x)/x: (-1)^m / (2m+1)!
constexpr double sinc_coef(int m) { return (m % 2 ? -1.0 : 1.0) / cfact(2 * m + 1); }

// Forced compile-time evaluation of the coefficients (no run-time calls).
template <int M> struct SphC { static constexpr float v = (float)sph_coef(M); };
template <int M> struct LamC { static constexpr float v = (float)lam_coef(M); };
template <int M> struct SincC { static constexpr float v = (float)sinc_coef(M); };

constexpr int kPySeriesTerms = 12;
constexpr int kMaxQuad = 256;

// ---------------------------------------------------------------- arguments
// Everything a trace kernel needs, passed by value as the kernel argument.
struct TraceArgs {
    // instrument, FP64
    double src_w, src_h, src_z;
    double slit_w, slit_h, slit_z;
    double lambda0, lambda_span;  // lambda = lambda0 + lambda_span (2u - 1)
    double half_x, half_y, half_z;
    double omc;                   // 1 - cos(alpha)
    double det_z, det_hw, det_hh;
    double inv_px, inv_py;        // nx / det_w, ny / det_h
    double wscale;                // 1e10 * dOmega * phi / <V>  (per metre of path)
    int32_t nx, ny;
    // sample, FP32
    float size[3];
    float shell;
    float contrast;               // drho = sld[0] - sld[2]
    float cs_core, cs_shell;      // core-shell: sld0 - sld1, sld1 - sld2
    int32_t poly_on, poly_mask, orient_kind, third_block;
    float ang_sin[3], ang_cos[3];  // sin, cos of the mean angles (FP64 on the host)
    float ang_sigma[3];
    int32_t sq_on;
    float sq_2r, sq_24phi;
    float py_alpha, py_beta, py_gamma;
    float py_c[kPySeriesTerms];
    // tables (device global memory; kernels stage them in LDS)
    int32_t M;                    // knots per table
    const float* tab_size;        // Schulz quantiles or nullptr
    const float* tab_norm;        // normal quantiles or nullptr
    // exact-average quadrature (QUAD mode)
    int32_t quad_n, quad_ny, quad_dims;   // orientation nodes, size nodes, 0/1/2-D orientation
    const float* quad_mu;         // [quad_n] mu nodes
    const float* quad_wmu;        // [quad_n]
    const float* quad_cb;         // [quad_n] cos(beta) nodes
    const float* quad_sb;         // [quad_n] sin(beta)
    const float* quad_wb;         // [quad_n]
    const float* quad_y;          // [quad_ny] size nodes
    const float* quad_wy;         // [quad_ny] normalised Schulz weights
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
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// (x + 1/2) 2^-32 - 1/2, exact in FP64 (both steps are exact).
__device__ __forceinline__ double centred_u(uint32_t x)
{
    return __builtin_fma((double)x, 0x1p-32, 0x1p-33 - 0.5);
}
__device__ __forceinline__ double u64(uint32_t x) { return __builtin_fma((double)x, 0x1p-32, 0x1p-33); }
__device__ __forceinline__ float u32f(uint32_t x) { return __builtin_fmaf((float)x, 0x1p-32f, 0x1p-33f); }

// ---------------------------------------------------------------- FP32 math
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// 3 j1(x)/x, the normalised sphere amplitude (Eq. (5) for a sphere).
__device__ __forceinline__ float sph3j(float x)
{
    x = fabsf(x);
    if (x < 2.0f) {
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
    float s, c;
    sincosf(x, &s, &c);
    const float ix = rcpf(x);
    return 3.0f * (s - x * c) * (ix * ix * ix);
}

// 2 J1(x)/x (the cylinder's cross-section factor, Eq. (9)).
__device__ __forceinline__ float lambda1(float x)
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

// sin(x)/x (parallelepiped faces, cylinder length factor).
__device__ __forceinline__ float sincf(float x)
{
    const float ax = fabsf(x);
    if (ax < 0.5f) {
        const float x2 = x * x;
        float r = SincC<4>::v;
        r = __builtin_fmaf(r, x2, SincC<3>::v);
        r = __builtin_fmaf(r, x2, SincC<2>::v);
        r = __builtin_fmaf(r, x2, SincC<1>::v);
        return __builtin_fmaf(r, x2, 1.0f);
    }
    return sinf(ax) * rcpf(ax);
}

// Percus-Yevick hard-sphere S(q): x = 2 q R, S = 1/(1 + 24 phi G(x)/x).
// Below x = 2.5 G(x)/x comes from its power series (coefficients computed on
// the host); above, from the closed form.
__device__ __forceinline__ float py_sq(const TraceArgs& a, float q)
{
    const float x = q * a.sq_2r;
    float gx;
    if (x < 2.5f) {
        const float x2 = x * x;
        float r = a.py_c[kPySeriesTerms - 1];
#pragma unroll
        for (int m = kPySeriesTerms - 2; m >= 0; --m) r = __builtin_fmaf(r, x2, a.py_c[m]);
        gx = r;
    } else {
        float s, c;
        sincosf(x, &s, &c);
        const float ix = rcpf(x);
        const float ix2 = ix * ix;
        const float x2 = x * x;
        const float ta = (s - x * c) * ix2;
        const float tb = (2.0f * x * s + (2.0f - x2) * c - 2.0f) * ix2 * ix;
        const float tg = (-x2 * x2 * c + 4.0f * ((3.0f * x2 - 6.0f) * c + (x2 * x - 6.0f * x) * s + 6.0f))
                       * ix2 * ix2 * ix;
        gx = (a.py_alpha * ta + a.py_beta * tb + a.py_gamma * tg) * ix;
    }
    return rcpf(__builtin_fmaf(a.sq_24phi, gx, 1.0f));
}

// Linear interpolation in an inverse-CDF table (knots at (k + 1/2)/M).
__device__ __forceinline__ float table_lerp(const float* tab, int M, float u)
{
    const float s = __builtin_fmaf(u, (float)M, -0.5f);
    float fk = floorf(s);
    fk = fminf(fmaxf(fk, 0.0f), (float)(M - 2));
    const int k = (int)fk;
    const float f = s - fk;
    const float y0 = tab[k], y1 = tab[k + 1];
    return __builtin_fmaf(f, y1 - y0, y0);
}

// ---------------------------------------------------------------- models
enum : int { kSphere = 0, kCoreShell = 1, kCylinder = 2, kEllipsoid = 3, kParallelepiped = 4 };

// F of one particle with sizes s and lab-frame projections (qa, qb, qc) of Q.
template <int KIND>
__device__ __forceinline__ float amplitude(const TraceArgs& a, const float s[3], float q, float qa,
                                           float qb, float qc)
{
    constexpr float k43pi = (float)(4.0 / 3.0 * kPi);
    if constexpr (KIND == kSphere) {
        const float r = s[0];
        return a.contrast * k43pi * r * r * r * sph3j(q * r);
    } else if constexpr (KIND == kCoreShell) {
        const float rc = s[0], ro = s[0] + a.shell;
        return a.cs_core * k43pi * rc * rc * rc * sph3j(q * rc)
             + a.cs_shell * k43pi * ro * ro * ro * sph3j(q * ro);
    } else if constexpr (KIND == kCylinder) {
        const float r = s[0], len = s[1];
        const float qab = sqrtf(fmaxf(__builtin_fmaf(q, q, -qc * qc), 0.0f));
        return a.contrast * (float)kPi * r * r * len * sincf(0.5f * qc * len) * lambda1(qab * r);
    } else if constexpr (KIND == kEllipsoid) {
        const float xa = qa * s[0], xb = qb * s[1], xc = qc * s[2];
        const float x = sqrtf(xa * xa + xb * xb + xc * xc);
        return a.contrast * k43pi * s[0] * s[1] * s[2] * sph3j(x);
    } else {
        return a.contrast * s[0] * s[1] * s[2] * sincf(0.5f * qa * s[0]) * sincf(0.5f * qb * s[1])
             * sincf(0.5f * qc * s[2]);
    }
}

// Particle axes A = R x, B = R y, C = R z with R = Rz(phi) Ry(theta) Rz(Psi),
// from the sines and cosines of (theta, phi, Psi).
struct Trig3 {
    float st, ct, sp, cp, ss, cs;
};

__device__ __forceinline__ void particle_axes(const Trig3& g, float A[3], float B[3], float C[3])
{
    A[0] = g.cp * g.ct * g.cs - g.sp * g.ss;
    A[1] = g.sp * g.ct * g.cs + g.cp * g.ss;
    A[2] = -g.st * g.cs;
    B[0] = -g.cp * g.ct * g.ss - g.sp * g.cs;
    B[1] = -g.sp * g.ct * g.ss + g.cp * g.cs;
    B[2] = g.st * g.ss;
    C[0] = g.cp * g.st;
    C[1] = g.sp * g.st;
    C[2] = g.ct;
}

// sin and cos of (mean + d) from those of the mean (exact on the host) and of
// the small offset d: keeps the rounding of the mean angle out of FP32.
__device__ __forceinline__ void rotate_by(float sm, float cm, float d, float& s, float& c)
{
    float sd, cd;
    sincosf(d, &sd, &cd);
    s = __builtin_fmaf(sm, cd, cm * sd);
    c = __builtin_fmaf(cm, cd, -sm * sd);
}

// ---------------------------------------------------------------- one neutron
struct Event {
    int32_t pixel;  // -1: not tallied
    float w;
    float q;        // 0 when the sample is missed
};

// Exact average <F^2>(q) over the Schulz size nodes and (isotropic) the
// orientation nodes held in LDS.
template <int KIND>
__device__ __forceinline__ float quad_average(const TraceArgs& a, const float* lq, float q,
                                              const float qv[3]);

// Traces neutron i.  tab_size/tab_norm point to the LDS copies of the
// tables; lq to the LDS copy of the quadrature nodes (QUAD mode).
template <int KIND, int MODE>
__device__ __forceinline__ Event trace_neutron(const TraceArgs& a, uint64_t i,
                                               const float* tab_size, const float* tab_norm,
                                               const float* lq)
{
    Event ev{-1, 0.0f, 0.0f};
    const uint32_t ilo = (uint32_t)i, ihi = (uint32_t)(i >> 32);
    const U4 r0 = philox4x32_10(ilo, ihi, 0u, a.exp_id, a.seed_lo, a.seed_hi);
    const U4 r1 = philox4x32_10(ilo, ihi, 1u, a.exp_id, a.seed_lo, a.seed_hi);

    // source -> slit flight
    const double sx = centred_u(r0.x) * a.src_w, sy = centred_u(r0.y) * a.src_h;
    const double tx = centred_u(r0.z) * a.slit_w, ty = centred_u(r0.w) * a.slit_h;
    const double dx = tx - sx, dy = ty - sy, dz = a.slit_z - a.src_z;
    const double dl = sqrt(dx * dx + dy * dy + dz * dz);
    const double idl = 1.0 / dl;
    const double kx = dx * idl, ky = dy * idl, kz = dz * idl;
    const double lambda = __builtin_fma(a.lambda_span, 2.0 * u64(r1.x) - 1.0, a.lambda0);
    const double k = 2.0 * kPi / lambda;

    // slab entry/exit along src + s k, s >= 0
    double s_in = 0.0, s_out = 1e300;
    {
        const double o[3] = {sx, sy, a.src_z};
        const double dv[3] = {kx, ky, kz};
        const double h[3] = {a.half_x, a.half_y, a.half_z};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (dv[c] != 0.0) {
                const double inv = 1.0 / dv[c];
                const double t1 = (-h[c] - o[c]) * inv, t2 = (h[c] - o[c]) * inv;
                s_in = fmax(s_in, fmin(t1, t2));
                s_out = fmin(s_out, fmax(t1, t2));
            } else if (fabs(o[c]) > h[c]) {
                s_out = -1.0;
            }
        }
    }
    if (!(s_out > s_in)) return ev;
    const double len = s_out - s_in;
    const double sp = __builtin_fma(u64(r1.y), len, s_in);
    const double rx = __builtin_fma(sp, kx, sx), ry = __builtin_fma(sp, ky, sy),
                 rz = __builtin_fma(sp, kz, a.src_z);

    // cone sampling about the flight direction; basis of Duff et al. (JCGT 2017)
    const double t = u64(r1.z) * a.omc;
    const double c2 = 1.0 - t;
    const double s2 = sqrt(t * (2.0 - t));
    double sps, cps;
    sincospi(2.0 * u64(r1.w), &sps, &cps);
    const double sg = kz >= 0.0 ? 1.0 : -1.0;
    const double aa = -1.0 / (sg + kz);
    const double bb = kx * ky * aa;
    const double px = cps * (1.0 + sg * kx * kx * aa) + sps * bb;
    const double py = cps * (sg * bb) + sps * (sg + ky * ky * aa);
    const double pz = cps * (-sg * kx) + sps * (-ky);
    const double fx = c2 * kx + s2 * px, fy = c2 * ky + s2 * py, fz = c2 * kz + s2 * pz;
    const double qd = k * sqrt(2.0 * t);
    const float q = (float)qd;
    ev.q = q;

    // detector plane and pixel
    if (!(fz > 0.0)) return ev;
    const double sd = (a.det_z - rz) / fz;
    const double xd = __builtin_fma(sd, fx, rx), yd = __builtin_fma(sd, fy, ry);
    const double fxp = floor((xd + a.det_hw) * a.inv_px);
    const double fyp = floor((yd + a.det_hh) * a.inv_py);
    const bool on_det = fxp >= 0.0 && fxp < (double)a.nx && fyp >= 0.0 && fyp < (double)a.ny;

    // the weight (computed for every lane: the wave runs it anyway)
    float qv[3];
    if constexpr (KIND >= kCylinder) {
        qv[0] = (float)(k * __builtin_fma(s2, px, -t * kx));
        qv[1] = (float)(k * __builtin_fma(s2, py, -t * ky));
        qv[2] = (float)(k * __builtin_fma(s2, pz, -t * kz));
    }
    float f2;
    if constexpr (MODE == 0) {
        float y = 1.0f;
        Trig3 g{a.ang_sin[0], a.ang_cos[0], a.ang_sin[1], a.ang_cos[1], a.ang_sin[2], a.ang_cos[2]};
        if (a.third_block) {
            const U4 r2 = philox4x32_10(ilo, ihi, 2u, a.exp_id, a.seed_lo, a.seed_hi);
            if (a.poly_on) y = fmaxf(table_lerp(tab_size, a.M, u32f(r2.x)), 0.0f);
            if constexpr (KIND >= kCylinder) {
                if (a.orient_kind == 1) {
                    rotate_by(a.ang_sin[0], a.ang_cos[0],
                              a.ang_sigma[0] * table_lerp(tab_norm, a.M, u32f(r2.y)), g.st, g.ct);
                    rotate_by(a.ang_sin[1], a.ang_cos[1],
                              a.ang_sigma[1] * table_lerp(tab_norm, a.M, u32f(r2.z)), g.sp, g.cp);
                    rotate_by(a.ang_sin[2], a.ang_cos[2],
                              a.ang_sigma[2] * table_lerp(tab_norm, a.M, u32f(r2.w)), g.ss, g.cs);
                } else if (a.orient_kind == 2) {
                    // cos(theta) uniform in [-1, 1]; phi, Psi uniform in [0, 2 pi)
                    g.ct = __builtin_fmaf(2.0f, u32f(r2.y), -1.0f);
                    g.st = sqrtf(fmaxf(__builtin_fmaf(-g.ct, g.ct, 1.0f), 0.0f));
                    sincospif(2.0f * u32f(r2.z), &g.sp, &g.cp);
                    sincospif(2.0f * u32f(r2.w), &g.ss, &g.cs);
                } else if (a.orient_kind == 3) {
                    // the literal rule: theta uniform in [0, pi)
                    sincospif(u32f(r2.y), &g.st, &g.ct);
                    sincospif(2.0f * u32f(r2.z), &g.sp, &g.cp);
                    sincospif(2.0f * u32f(r2.w), &g.ss, &g.cs);
                }
            }
        }
        float s[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] = (a.poly_mask >> c & 1) ? a.size[c] * y : a.size[c];
        float qa = 0.0f, qb = 0.0f, qc = 0.0f;
        if constexpr (KIND >= kCylinder) {
            float A[3], B[3], C[3];
            particle_axes(g, A, B, C);
            qc = qv[0] * C[0] + qv[1] * C[1] + qv[2] * C[2];
            if constexpr (KIND != kCylinder) {
                qa = qv[0] * A[0] + qv[1] * A[1] + qv[2] * A[2];
                qb = qv[0] * B[0] + qv[1] * B[1] + qv[2] * B[2];
            }
        }
        const float f = amplitude<KIND>(a, s, q, qa, qb, qc);
        f2 = f * f;
    } else {
        f2 = quad_average<KIND>(a, lq, q, qv);
    }
    float w = (float)(len * a.wscale) * f2;
    if (a.sq_on) w *= py_sq(a, q);
    if (on_det) {
        ev.pixel = (int32_t)fyp * a.nx + (int32_t)fxp;
        ev.w = w;
    }
    return ev;
}

// LDS layout of the quadrature nodes: mu[n], wmu[n], cb[n], sb[n], wb[n],
// y[ny], wy[ny].
template <int KIND>
__device__ __forceinline__ float quad_average(const TraceArgs& a, const float* lq, float q,
                                              const float qv[3])
{
    const int n = a.quad_n, ny = a.quad_ny;
    const float* mu = lq;
    const float* wmu = lq + n;
    const float* cb = lq + 2 * n;
    const float* sb = lq + 3 * n;
    const float* wb = lq + 4 * n;
    const float* ys = lq + 5 * n;
    const float* wy = lq + 5 * n + ny;
    float total = 0.0f;
    for (int j = 0; j < ny; ++j) {
        const float y = ys[j];
        float s[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] = (a.poly_mask >> c & 1) ? a.size[c] * y : a.size[c];
        float avg = 0.0f;
        if (a.quad_dims == 0) {
            float qa = 0.0f, qb = 0.0f, qc = 0.0f;
            if constexpr (KIND >= kCylinder) {
                float A[3], B[3], C[3];
                const Trig3 g{a.ang_sin[0], a.ang_cos[0], a.ang_sin[1], a.ang_cos[1], a.ang_sin[2],
                              a.ang_cos[2]};
                particle_axes(g, A, B, C);
                qa = qv[0] * A[0] + qv[1] * A[1] + qv[2] * A[2];
                qb = qv[0] * B[0] + qv[1] * B[1] + qv[2] * B[2];
                qc = qv[0] * C[0] + qv[1] * C[1] + qv[2] * C[2];
            }
            const float f = amplitude<KIND>(a, s, q, qa, qb, qc);
            avg = f * f;
        } else if (a.quad_dims == 1) {
            for (int i = 0; i < n; ++i) {
                const float m = mu[i];
                const float st = sqrtf(fmaxf(1.0f - m * m, 0.0f));
                const float f = amplitude<KIND>(a, s, q, q * st, 0.0f, q * m);
                avg = __builtin_fmaf(wmu[i], f * f, avg);
            }
        } else {
            for (int i = 0; i < n; ++i) {
                const float m = mu[i];
                const float qst = q * sqrtf(fmaxf(1.0f - m * m, 0.0f));
                const float qc = q * m;
                float inner = 0.0f;
                for (int l = 0; l < n; ++l) {
                    const float f = amplitude<KIND>(a, s, q, qst * cb[l], qst * sb[l], qc);
                    inner = __builtin_fmaf(wb[l], f * f, inner);
                }
                avg = __builtin_fmaf(wmu[i], inner, avg);
            }
        }
        total = __builtin_fmaf(wy[j], avg, total);
    }
    return total;
}

}  // namespace sans
