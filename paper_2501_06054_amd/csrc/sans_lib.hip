// sans_lib.hip -- host side of the C ABI of libsans (gfx950), and the small
// kernels around the per-model ones (sans_kernels.hpp):
//   k_reduce_partials           sum of the LDS-tally partial histograms
//   k_bin_accumulate,           binned tally, pass 2: each detector band summed
//   k_reduce_binned             in LDS, then the bands' slices summed
//   k_philox                    raw Philox words for stream tests
//   k_fill, k_sum_replicas      detector clearing / XCD replica reduction
//   k_schulz_tables             FP64 Schulz quantile tables
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "../../include/sans.h"
#include "sans_device.hpp"
#include "sans_host_math.hpp"
#include "sans_kernels.hpp"
#include "sans_surrogate.hpp"

using namespace sans;

namespace {

constexpr size_t kLdsMax = 160 * 1024;
// the surrogate's default in-domain judge: tolerance on ln <F^2>, bins of ln(q s0)
constexpr double kSurJudgeTol = 1e-3;
constexpr int kSurJudgeBins = 2048;

thread_local std::string g_last_error;

int fail(int status, const std::string& msg)
{
    g_last_error = msg;
    return status;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(SANS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)


// The partial sums of a detector pixel are read by kRedWaves waves of one
// workgroup, each over every kRedWaves-th partial (a wave loads 64
// consecutive pixels of one partial at a time: 512 B, coalesced), and added
// in a fixed order: the result does not depend on the launch.  Workgroup b
// takes pixels [64 b, 64 b + 64).
constexpr int kRedWaves = 4;
static_assert(kRedWaves == 4, "the final sums below add four wave sums");

// det[p] (+)= sum over g < G of partial[g][p]  (p < npix)
__global__ __launch_bounds__(64 * kRedWaves) void k_reduce_partials(double* det, const double* partial, int G,
                                                                    int npix, int accumulate)
{
    __shared__ double part[kRedWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (p < npix) {
#pragma unroll 8
        for (int g = w; g < G; g += kRedWaves) s += partial[(size_t)g * npix + p];
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && p < npix) {
        const double t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        det[p] = accumulate ? det[p] + t : t;
    }
}

// Binned tally, pass 2: workgroup (t, s) sums the segments of waves
// [s W/S, (s+1) W/S) of tile t in an LDS histogram of the tile (each of its
// waves takes every 16th segment) and writes it to its own partial slot (the
// first chunk of a call) or adds it there.  A
// wave first reads the counts of up to 64 of its segments at once (one per
// lane), then streams each segment with kAccUnroll loads in flight per lane
// before their LDS atomics.
constexpr int kAccUnroll = 8;

__global__ __launch_bounds__(kHistBlock) void k_bin_accumulate(const uint2* buckets, const unsigned* seg_count,
                                                               unsigned capw, unsigned nwaves, int tile_pixels,
                                                               int slices, double* partial, int overwrite)
{
    extern __shared__ double hist[];
    const int t = blockIdx.x / slices, sl = blockIdx.x % slices;
    for (int i = threadIdx.x; i < tile_pixels; i += blockDim.x) hist[i] = 0.0;
    __syncthreads();
    const unsigned w0 = (unsigned)((uint64_t)nwaves * sl / slices);
    const unsigned w1 = (unsigned)((uint64_t)nwaves * (sl + 1) / slices);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr unsigned kWaves = kHistBlock / 64;
    for (unsigned g0 = w0 + wave; g0 < w1; g0 += 64 * kWaves) {
        // lane k: count of segment g0 + k * kWaves
        const unsigned wl = g0 + (unsigned)lane * kWaves;
        const unsigned mycnt = wl < w1 ? seg_count[(size_t)t * nwaves + wl] : 0u;
        const int nseg = (int)std::min<unsigned>(64u, (w1 - g0 + kWaves - 1) / kWaves);
        for (int k = 0; k < nseg; ++k) {
            const unsigned cnt = (unsigned)__builtin_amdgcn_readlane((int)mycnt, k);
            const uint2* b = buckets + ((size_t)t * nwaves + g0 + (unsigned)k * kWaves) * capw;
            for (unsigned i0 = 0; i0 < cnt; i0 += 64 * kAccUnroll) {
                uint2 e[kAccUnroll];
#pragma unroll
                for (int u = 0; u < kAccUnroll; ++u) {
                    const unsigned i = i0 + (unsigned)(u * 64 + lane);
                    e[u] = i < cnt ? b[i] : make_uint2(0u, 0u);
                }
#pragma unroll
                for (int u = 0; u < kAccUnroll; ++u)
                    if (e[u].y != 0u)
                        __hip_atomic_fetch_add(hist + e[u].x, (double)__uint_as_float(e[u].y), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    double* out = partial + (size_t)blockIdx.x * tile_pixels;
    if (overwrite)
        for (int i = threadIdx.x; i < tile_pixels; i += blockDim.x) out[i] = hist[i];
    else
        for (int i = threadIdx.x; i < tile_pixels; i += blockDim.x) out[i] += hist[i];
}

// det[p] (+)= sum over the slices of tile t(p) of partial[t][s][p - t*tile]
// (the same split over kRedWaves waves)
__global__ __launch_bounds__(64 * kRedWaves) void k_reduce_binned(double* det, const double* partial,
                                                                  int tile_pixels, int slices, int npix,
                                                                  int accumulate)
{
    __shared__ double part[kRedWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (p < npix) {
        const int t = p / tile_pixels, q = p - t * tile_pixels;
        const double* src = partial + (size_t)t * slices * tile_pixels + q;
#pragma unroll 8
        for (int k = w; k < slices; k += kRedWaves) s += src[(size_t)k * tile_pixels];
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && p < npix) {
        const double t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        det[p] = accumulate ? det[p] + t : t;
    }
}


__global__ void k_philox(uint32_t seed_lo, uint32_t seed_hi, uint64_t first, uint64_t n,
                         uint32_t nblocks, uint32_t exp_id, uint32_t* out)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint64_t i = first + j;
    for (uint32_t b = 0; b < nblocks; ++b) {
        const U4 r = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), b, exp_id, seed_lo, seed_hi);
        uint32_t* o = out + (j * nblocks + b) * 4;
        o[0] = r.x;
        o[1] = r.y;
        o[2] = r.z;
        o[3] = r.w;
    }
}

__global__ void k_fill(double* p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_fill_u32(unsigned* p, int n)
{
    const int i = threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_fill_u64(unsigned long long* p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// The transmitted beam of neutrons a.first .. a.first + a.n - 1, added to
// det (and det_w2 / det_count when given).  One lane per neutron, the grid
// striding in whole waves; the direct beam falls on a few pixels, so each
// wave first merges its lanes' events pixel by pixel and issues one atomic
// per distinct pixel.
__global__ __launch_bounds__(256) void k_transmit(const TraceArgs a, double* det, double* det_w2,
                                                  unsigned long long* det_count)
{
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t base = wave * 64; base < a.n; base += nwaves * 64) {
        const uint64_t j = base + (uint64_t)lane;
        Straight st{-1, 0.0};
        if (j < a.n) st = straight_flight(a, a.first + j);
        int32_t pix = st.pixel;
        unsigned long long pending = __ballot(pix >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int32_t lp = __shfl(pix, leader);
            const bool mine = pix == lp;
            const unsigned long long same = __ballot(mine);
            double sw = mine ? st.w : 0.0, sw2 = sw * sw;
            for (int off = 32; off > 0; off >>= 1) {
                sw += __shfl_xor(sw, off);
                sw2 += __shfl_xor(sw2, off);
            }
            if (lane == leader) {
                atomicAdd(det + lp, sw);
                if (det_w2) atomicAdd(det_w2 + lp, sw2);
                if (det_count) atomicAdd(det_count + lp, (unsigned long long)__popcll(same));
            }
            if (mine) pix = -1;
            pending &= ~same;
        }
    }
}

// Per-neutron transmitted events: pixel (-1 off the detector) and weight.
__global__ __launch_bounds__(256) void k_debug_transmit(const TraceArgs a, int32_t* pixel, double* w)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const Straight st = straight_flight(a, a.first + j);
    pixel[j] = st.pixel;
    w[j] = st.pixel >= 0 ? st.w : 0.0;
}

// det[i] (+)= sum over the XCD replicas, which are cleared for the next run.
__global__ void k_sum_replicas(double* det, double* rep, int npix, int accumulate)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    double s = accumulate ? det[i] : 0.0;
#pragma unroll
    for (int x = 0; x < kXcds; ++x) {
        s += rep[(size_t)x * npix + i];
        rep[(size_t)x * npix + i] = 0.0;
    }
    det[i] = s;
}


// ------------------------------------------------------------------ Schulz tables (FP64)
// Knots of the Schulz distribution (Gamma with shape a = 1/p^2 and mean 1)
// in the tables' layout: knot j < M/2 at the lower-tail probability
// v_j = e^(-j dt)/2, knot M/2 + j at the upper-tail probability v_j.  The
// density is integrated over kSchulzPanels panels (16-point Gauss-Legendre
// each) and summed in LDS from the bottom (the CDF) and from the top (the
// upper tail, so that tail probabilities down to 1e-10 keep their relative
// precision); each knot is then refined inside its panel by safeguarded
// Newton steps.  One workgroup per table.
constexpr int kSchulzPanels = 2048;
constexpr int kSchulzBlock = 256;

struct SchulzJob {
    double a, lnorm, ymax;   // shape, log normaliser a ln a - lgamma(a), upper limit
    unsigned long long out;  // offset of the table in the output array
};

// Gauss-Legendre nodes on [-1, 1]: 16 points for the panels of the CDF, 4
// for the Newton steps inside one panel (a panel is about 1/2048 of the
// support: the 4-point rule is exact to rounding there).
struct GL16 {
    double x[16], w[16];
    double x4[4], w4[4];
};

__device__ __forceinline__ double schulz_pdf_d(double y, double a, double lnorm)
{
    return y > 0.0 ? exp(lnorm + (a - 1.0) * log(y) - a * y) : 0.0;
}

__device__ __forceinline__ double pdf_integral(double lo, double hi, double a, double lnorm,
                                               const GL16& g)
{
    const double h = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s = __builtin_fma(g.w[i], schulz_pdf_d(__builtin_fma(h, g.x[i], c), a, lnorm), s);
    return h * s;
}

__device__ __forceinline__ double pdf_integral4(double lo, double hi, double a, double lnorm, const GL16& g)
{
    const double h = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) s = __builtin_fma(g.w4[i], schulz_pdf_d(__builtin_fma(h, g.x4[i], c), a, lnorm), s);
    return h * s;
}

// Exclusive scan of one value per thread across the block (in part[]).
__device__ __forceinline__ void block_offsets(double* part)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int t = 0; t < kSchulzBlock; ++t) {
            const double v = part[t];
            part[t] = r;
            r += v;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kSchulzBlock) void k_schulz_tables(const SchulzJob* jobs, int M,
                                                                double* tables, const GL16 g)
{
    __shared__ double cdf[kSchulzPanels + 1];   // integral over [0, j dy]
    __shared__ double sdf[kSchulzPanels + 1];   // integral over [j dy, ymax]
    __shared__ double part[kSchulzBlock];
    const SchulzJob jb = jobs[blockIdx.x];
    const double dy = jb.ymax / kSchulzPanels;
    constexpr int per = kSchulzPanels / kSchulzBlock;
    const int j0 = threadIdx.x * per;
    double pan[per];
    double acc = 0.0;
    for (int k = 0; k < per; ++k) {
        pan[k] = pdf_integral((j0 + k) * dy, (j0 + k + 1) * dy, jb.a, jb.lnorm, g);
        acc += pan[k];
        cdf[j0 + k + 1] = acc;
    }
    part[threadIdx.x] = acc;
    block_offsets(part);
    for (int k = 0; k < per; ++k) cdf[j0 + k + 1] += part[threadIdx.x];
    if (threadIdx.x == 0) cdf[0] = 0.0;
    // the same from the top: thread t holds panels j0 .. j0 + per - 1, whose
    // tails are summed downwards, offset by the threads above it
    __syncthreads();
    double up = 0.0;
    for (int k = per - 1; k >= 0; --k) {
        up += pan[k];
        sdf[j0 + k] = up;
    }
    part[kSchulzBlock - 1 - threadIdx.x] = up;
    block_offsets(part);
    for (int k = 0; k < per; ++k) sdf[j0 + k] += part[kSchulzBlock - 1 - threadIdx.x];
    if (threadIdx.x == 0) sdf[kSchulzPanels] = 0.0;
    __syncthreads();
    const double total = cdf[kSchulzPanels];
    const int H = M / 2;
    const double dt = 32.0 * 0.69314718055994530942 / (H - 1);
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        const bool upper = k >= H;
        const double v = 0.5 * exp(-(upper ? k - H : k) * dt) * total;
        // the panel holding the knot: cdf[j] <= v < cdf[j+1] (lower), or
        // sdf[j+1] <= v < sdf[j] (upper)
        int lo = 0, hi = kSchulzPanels;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (upper ? sdf[mid] > v : cdf[mid] <= v) lo = mid; else hi = mid;
        }
        const int j = lo;
        double ylo = j * dy, yhi = (j + 1) * dy;
        double y = upper ? ylo + (sdf[j] - v) / fmax(sdf[j] - sdf[j + 1], 1e-300) * dy
                         : ylo + (v - cdf[j]) / fmax(cdf[j + 1] - cdf[j], 1e-300) * dy;
        for (int it = 0; it < 60; ++it) {
            // increasing in y for both halves: the mass below y minus its target
            const double gval = upper ? v - (sdf[j + 1] + pdf_integral4(y, (j + 1) * dy, jb.a, jb.lnorm, g))
                                      : cdf[j] + pdf_integral4(j * dy, y, jb.a, jb.lnorm, g) - v;
            if (gval > 0.0) yhi = y; else ylo = y;
            const double f = schulz_pdf_d(y, jb.a, jb.lnorm);
            double yn = f > 0.0 ? y - gval / f : 0.5 * (ylo + yhi);
            if (!(yn > ylo && yn < yhi)) yn = 0.5 * (ylo + yhi);
            const bool done = fabs(yn - y) <= 1e-16 * y;
            y = yn;
            if (done) break;
        }
        tables[jb.out + k] = y;
    }
}


// ------------------------------------------------------------------ dispatch table
// Kernel pointers of every model, filled once by the kind-group translation
// units.  Callers have validated kind (0 .. kNumKinds - 1); mode 0 selects the
// Monte Carlo kernels, any other mode the exact-average ones.
const KindFns* kind_table()
{
    static KindFns table[kNumKinds];
    static std::once_flag once;
    std::call_once(once, [] {
        fill_kinds_0(table);
        fill_kinds_1(table);
        fill_kinds_2(table);
        fill_kinds_3(table);
        fill_kinds_4(table);
        fill_kinds_5(table);
        fill_kinds_6(table);
        fill_kinds_7(table);
    });
    return table;
}

bool known_kind(int kind) { return kind >= 0 && kind < kNumKinds; }

TraceFn pick_trace(int kind, int mode, int tally)
{
    return known_kind(kind) ? kind_table()[kind].trace[mode == 0 ? 0 : 1][tally == SANS_TALLY_XCD ? 1 : 0]
                            : nullptr;
}

// att: the Monte Carlo instance with the attenuation and the guide compiled in
HistFn pick_hist(int kind, int mode, bool att)
{
    return known_kind(kind) ? kind_table()[kind].hist[mode != 0 ? 1 : att ? 2 : 0] : nullptr;
}

EmitFn pick_emit(int kind, int mode, bool att)
{
    return known_kind(kind) ? kind_table()[kind].emit[mode != 0 ? 1 : att ? 2 : 0] : nullptr;
}

// Runs that need the attenuation or the guide (only some kernel instances
// carry them).
bool needs_instrument(const sans_params& p) { return p.mu_att > 0.0 || p.guide[0] > 0.0; }

DebugFn pick_debug(int kind, int mode, bool att)
{
    return known_kind(kind) ? kind_table()[kind].debug[mode == 0 ? 0 : 1][att ? 1 : 0] : nullptr;
}

PqFn pick_pq(int kind) { return known_kind(kind) ? kind_table()[kind].pq : nullptr; }

}  // namespace

// ------------------------------------------------------------------ model handle
struct sans_model_s {
    sans_params p;
    TraceArgs args;            // constants; per-call fields are filled at launch
    double mean_v = 0.0, wscale = 0.0, omc = 0.0;
    std::vector<double> h_tab_size, h_tab_norm;
    std::vector<float> h_quad;
    double* d_tab_size = nullptr;
    double* d_tab_norm = nullptr;
    std::vector<double> h_tab_sep;
    double* d_tab_sep = nullptr;   // independent size widths' tables [3][M]
    float* d_quad = nullptr;
    float* d_caps = nullptr;   // node rule (capped bodies, superball) and structure-factor constants
    double* d_replicas = nullptr;
    size_t replica_pix = 0;
    // tally workspaces (grown on demand, freed with the model)
    double* d_partial = nullptr;
    size_t partial_cap = 0;     // doubles
    uint2* d_buckets = nullptr;
    size_t bucket_cap = 0;      // events
    unsigned* d_bucket_count = nullptr;  // [tile][wave] event counts
    size_t bucket_count_cap = 0;
    // surrogate network (SANS_MODE_SURROGATE)
    double sur_f2_0 = 0.0;      // <F^2>(q = 0) from the size nodes (normalisation of the target)
    __bf16* d_sur_w = nullptr;  // flat BF16 parameters
    mlp::bf16x8* d_sur_pack = nullptr;
    float sur_lo[4] = {0, 0, 0, 0}, sur_hi[4] = {0, 0, 0, 0};
    bool sur_attached = false;
    unsigned long long* d_queue = nullptr;
    size_t queue_cap = 0;
    unsigned* d_qcount = nullptr;
    // the surrogate's in-domain judge: flags per bin of ln(q s0) (device), the
    // bin count (0 = none) and the tolerance it was run with
    unsigned char* d_sur_flags = nullptr;
    int sur_nbins = 0;
    double sur_tol = 0.0;
    int device = 0;
    int num_cu = 256;
};

namespace {

bool finite(double x) { return std::isfinite(x); }

// Shape-independent models: a cross-section in 1/cm of |Q| only.
bool is_shape_independent(int kind)
{
    return (kind >= SANS_GUINIER && kind <= SANS_GAUSS_LORENTZ_GEL)
           || (kind >= SANS_SURFACE_FRACTAL && kind <= SANS_BROAD_PEAK) || kind == SANS_POLYMER_EXCL_VOLUME
           || kind == SANS_MASS_SURFACE_FRACTAL || kind == SANS_GEL_FIT;
}

// Isotropic sphere-based particles.
bool is_sphere_family(int kind)
{
    return (kind >= SANS_FUZZY_SPHERE && kind <= SANS_LINEAR_PEARLS) || kind == SANS_FRACTAL
           || kind == SANS_FRACTAL_CORE_SHELL || kind == SANS_RASPBERRY || kind == SANS_PEARL_NECKLACE
           || kind == SANS_BINARY_HARD_SPHERE;
}

// Orientation enters the weight (the particles from the cylinder to the thick
// hollow prism, but the micelle).
bool is_aniso(int kind)
{
    return (kind >= SANS_CYLINDER && kind <= SANS_HOLLOW_PRISM_THICK && kind != SANS_POLYMER_MICELLE)
           || (kind >= SANS_ELLIPTICAL_CYLINDER && kind <= SANS_FCC_PARACRYSTAL) || kind == SANS_SUPERBALL
           || kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH || kind == SANS_PRINGLE;
}

// Floats of the per-model node rule in device memory: the end caps' rule
// [3][quad_n] (barbell, capped cylinder), the superball's nested rule, else 0.
size_t rule_floats(const sans_params& p)
{
    if (p.kind == SANS_BARBELL || p.kind == SANS_CAPPED_CYLINDER) return 3 * (size_t)p.quad_n;
    if (p.kind == SANS_SUPERBALL) return (size_t)host::superball_rule_size(p.quad_n);
    if (p.kind == SANS_LAMELLAR_STACK_CAILLE || p.kind == SANS_LAMELLAR_HG_STACK_CAILLE) return (size_t)p.extra[0];
    if (p.kind == SANS_PEARL_NECKLACE) return 2 * (size_t)p.quad_n;
    if (p.kind == SANS_BINARY_HARD_SPHERE) return 4 * 32;
    if (p.kind == SANS_PRINGLE) return 8 * (size_t)p.quad_n * p.quad_n;
    if (p.kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL) return 5 * (size_t)p.quad_n;
    if (p.kind == SANS_FLEXIBLE_CYLINDER) return 2 * (size_t)p.quad_n;
    if (p.kind == SANS_POLYMER_EXCL_VOLUME) return 4 * (size_t)kPevRuleNodes;
    return 0;
}

// The Hayter-Penfold table spans K = q sigma from 0 to 1.01 sigma q_max (the
// largest q of the cone) with knots at most 0.01 apart (256 to 65536 knots).
double msa_kmax(const sans_params& p)
{
    const double lmin = p.lambda0 * (1.0 - p.dlambda_rel);
    return 2.0 * p.sq_radius * 4.0 * kPi / lmin * std::sin(0.5 * p.cone_alpha) * 1.01;
}
int msa_knot_count(const sans_params& p)
{
    const double n = std::ceil(msa_kmax(p) / 0.01) + 1.0;
    return (int)std::min(65536.0, std::max(256.0, n));
}

// The rule, then the constants of an adhesive or square-well structure
// factor, or the Hayter-Penfold knots.
bool needs_sq_coef(const sans_params& p) { return p.sq_phi > 0.0 && p.sq_kind != SANS_SQ_HARD_SPHERE; }
size_t sq_floats(const sans_params& p)
{
    if (!needs_sq_coef(p)) return 0;
    return p.sq_kind == SANS_SQ_HAYTER_MSA ? kMsaHead + 2 * (size_t)msa_knot_count(p) : (size_t)kSqCoef;
}
size_t node_floats(const sans_params& p) { return rule_floats(p) + sq_floats(p); }

// Fills the node buffer of one parameter set (node_floats(p) floats) and
// points the kernel arguments at it (base: its device address).  False
// when the Hayter-Penfold solve (done first in validation) fails.
bool fill_nodes(const sans_params& p, float* out, const float* base, TraceArgs& a)
{
    const size_t nr = rule_floats(p);
    if (p.kind == SANS_SUPERBALL) {
        host::superball_rule(p.extra[0], p.quad_n, out);
    } else if (p.kind == SANS_LAMELLAR_STACK_CAILLE || p.kind == SANS_LAMELLAR_HG_STACK_CAILLE) {
        // the Caille exponents' gamma + ln(pi n), n = 0 .. N - 1 (n = 0 unused)
        const double euler_gamma = 0.57721566490153286061;
        out[0] = 0.0f;
        for (size_t k = 1; k < nr; ++k) out[k] = (float)(euler_gamma + std::log(kPi * (double)k));
    } else if (p.kind == SANS_POLYMER_EXCL_VOLUME) {
        // int_0^1 t^(s-1) exp(-U t) dt with t = w^6: 6 w^(6 s - 1) exp(-U w^6) dw,
        // smooth in w, by 32-point Gauss-Legendre on [0, 1]; s = 1/(2 nu), 1/nu
        const int n = kPevRuleNodes;
        double gx[kPevRuleNodes], gw[kPevRuleNodes];
        host::gauss_legendre(n, gx, gw);
        const double nu = p.extra[1], sv[2] = {0.5 / nu, 1.0 / nu};
        for (int h = 0; h < 2; ++h)
            for (int k = 0; k < n; ++k) {
                const double w = 0.5 * (gx[k] + 1.0);
                out[2 * h * n + k] = (float)std::pow(w, 6.0);
                out[(2 * h + 1) * n + k] = (float)(6.0 * 0.5 * gw[k] * std::pow(w, 6.0 * sv[h] - 1.0));
            }
    } else if (p.kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL || p.kind == SANS_FLEXIBLE_CYLINDER) {
        // the chain's rule on [0, 1] (scaled to [0, x_e] per event) and, for
        // the ellipse, the section's angle psi in [0, pi/2] (weights of the
        // average, sum 1)
        const int n = p.quad_n;
        const bool ell = p.kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL;
        std::vector<double> gx(n), gw(n);
        host::gauss_legendre(n, gx.data(), gw.data());
        for (int k = 0; k < n; ++k) {
            out[k] = (float)(0.5 * (gx[k] + 1.0));
            out[n + k] = (float)(0.5 * gw[k]);
            if (!ell) continue;
            const double psi = 0.25 * kPi * (gx[k] + 1.0);
            out[2 * n + k] = (float)(std::sin(psi) * std::sin(psi));
            out[3 * n + k] = (float)(std::cos(psi) * std::cos(psi));
            out[4 * n + k] = (float)(0.5 * gw[k]);
        }
    } else if (p.kind == SANS_PRINGLE) {
        // polar rule on the disc: r by n-point Gauss-Legendre on [0, R], the
        // angle by the 2n-point midpoint rule on [0, pi); (x, y) pairs with
        // (-x, -y) (same z), so the weight carries 2 cos(Q_A x + Q_B y)'s 2
        const int n = p.quad_n, m = 2 * n, tot = n * m;
        std::vector<double> gx(n), gw(n);
        host::gauss_legendre(n, gx.data(), gw.data());
        const double R = p.size[0], al = p.extra[0], be = p.extra[1];
        for (int i = 0; i < n; ++i) {
            const double r = 0.5 * R * (gx[i] + 1.0), wr = 0.5 * R * gw[i] * r;
            for (int j = 0; j < m; ++j) {
                const double ph = kPi * (j + 0.5) / m, x = r * std::cos(ph), y = r * std::sin(ph);
                const int k = i * m + j;
                out[k] = (float)x;
                out[tot + k] = (float)y;
                out[2 * tot + k] = (float)(al * x * x - be * y * y);
                out[3 * tot + k] = (float)(2.0 * wr * kPi / m);
            }
        }
    } else if (p.kind == SANS_BINARY_HARD_SPHERE) {
        // Baxter's factor functions for the mixture, Q_ij(r) = a_i/2 (r^2 - d_ij^2)
        // + b_i (r - d_ij) on (d_i - d_j)/2 < r < d_ij: 16 Gauss-Legendre nodes
        // per (i, j), weights times 2 pi sqrt(n_i n_j) Q_ij(r_k)
        const double d[2] = {2.0 * p.size[0], 2.0 * p.size[1]};
        const double v1 = 4.0 / 3.0 * kPi * p.size[0] * p.size[0] * p.size[0];
        const double v2 = 4.0 / 3.0 * kPi * p.size[1] * p.size[1] * p.size[1];
        const double n[2] = {(p.phi - p.extra[0]) / v1, p.extra[0] / v2};
        const double xi2 = kPi / 6.0 * (n[0] * d[0] * d[0] + n[1] * d[1] * d[1]);
        const double xi3 = kPi / 6.0 * (n[0] * d[0] * d[0] * d[0] + n[1] * d[1] * d[1] * d[1]);
        const double dd = 1.0 - xi3;
        double gx[16], gw[16];
        host::gauss_legendre(16, gx, gw);
        for (int i = 0; i < 2; ++i) {
            const double ai = (1.0 - xi3 + 3.0 * d[i] * xi2) / (dd * dd), bi = -1.5 * d[i] * d[i] * xi2 / (dd * dd);
            for (int j = 0; j < 2; ++j) {
                const double dij = 0.5 * (d[i] + d[j]), lo = 0.5 * (d[i] - d[j]), h = 0.5 * (dij - lo);
                const double f = 2.0 * kPi * std::sqrt(n[i] * n[j]);
                float* blk = out + 32 * (2 * i + j);
                for (int k = 0; k < 16; ++k) {
                    const double r = lo + h * (gx[k] + 1.0);
                    blk[k] = (float)r;
                    blk[16 + k] = (float)(f * h * gw[k] * (0.5 * ai * (r * r - dij * dij) + bi * (r - dij)));
                }
            }
        }
    } else if (p.kind == SANS_PEARL_NECKLACE) {
        // Gauss-Legendre on [0, 1]: nodes, then weights summing to 1
        const int n = p.quad_n;
        std::vector<double> gx(n), gw(n);
        host::gauss_legendre(n, gx.data(), gw.data());
        for (int i = 0; i < n; ++i) {
            out[i] = (float)(0.5 * (gx[i] + 1.0));
            out[n + i] = (float)(0.5 * gw[i]);
        }
    } else if (nr) {
        host::cap_rule(p.kind == SANS_BARBELL, p.size[0], p.size[1], p.size[2], p.quad_n, out);
    }
    if (nr) a.cap_nodes = base;
    if (!needs_sq_coef(p)) return true;
    float* c = out + nr;
    a.sq_coef = base + nr;
    if (p.sq_kind == SANS_SQ_HAYTER_MSA) {
        // head: 1/dK, n - 1; then (S, dK S') at K_j = j dK (the solve is
        // cached from validation)
        const int n = msa_knot_count(p);
        const double kmax = msa_kmax(p);
        std::vector<double> cin(host::kMsaCin);
        if (!host::msa_solve(p.sq_phi, p.sq_extra[0], p.sq_extra[1], cin.data())) return false;
        for (int k = 0; k < kMsaHead; ++k) c[k] = 0.0f;
        c[0] = (float)((n - 1) / kmax);
        c[1] = (float)(n - 1);
        host::msa_knots(cin.data(), p.sq_phi, p.sq_extra[0], p.sq_extra[1], kmax, n, c + kMsaHead);
        return true;
    }
    for (int k = 0; k < kSqCoef; ++k) c[k] = 0.0f;
    if (p.sq_kind == SANS_SQ_STICKY_HARD_SPHERE) {
        double ca[kPySeriesTerms], cb[kPySeriesTerms], hbc[3];
        host::sticky_constants(p.sq_phi, p.sq_extra[0], kPySeriesTerms, ca, cb, hbc);
        for (int k = 0; k < kPySeriesTerms; ++k) {
            c[kSqA + k] = (float)ca[k];
            c[kSqB + k] = (float)cb[k];
        }
        c[kSqE] = (float)(12.0 * p.sq_phi);
        c[kSqH] = (float)hbc[0];
        c[kSqBb] = (float)hbc[1];
        c[kSqC0] = (float)hbc[2];
    } else {
        const double w = p.sq_extra[1];
        c[kSqW8] = (float)(8.0 * p.sq_phi * p.sq_extra[0]);
        c[kSqW] = (float)w;
        c[kSqW3] = (float)(w * w * w);
    }
    return true;
}

int validate(const sans_params* p)
{
    if (!p) return fail(SANS_E_INVALID_ARG, "params is NULL");
    if (p->abi_version != SANS_ABI_VERSION) return fail(SANS_E_INVALID_ARG, "abi_version mismatch");
    if (!known_kind(p->kind)) return fail(SANS_E_UNSUPPORTED, "unknown model kind");
    if (p->mode < 0 || p->mode > 2) return fail(SANS_E_UNSUPPORTED, "unknown mode");
    if (p->mode == SANS_MODE_SURROGATE) {
        if (p->kind != SANS_ELLIPSOID && p->kind != SANS_PARALLELEPIPED)
            return fail(SANS_E_UNSUPPORTED, "surrogate mode: ellipsoid or parallelepiped only");
        if (p->orient_kind != SANS_ORIENT_ISOTROPIC)
            return fail(SANS_E_UNSUPPORTED, "surrogate mode: isotropic orientation only");
        if (p->kind == SANS_ELLIPSOID && p->size[0] != p->size[1])
            return fail(SANS_E_UNSUPPORTED, "surrogate mode: ellipsoids of revolution (a = b) only");
        if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
    }
    if (p->orient_kind < 0 || p->orient_kind > 3) return fail(SANS_E_UNSUPPORTED, "unknown orientation kind");
    if (p->tally < 0 || p->tally > 4) return fail(SANS_E_UNSUPPORTED, "unknown tally strategy");
    const bool two_sizes = p->kind == SANS_CYLINDER || p->kind == SANS_POLYMER_MICELLE
                           || p->kind == SANS_HOLLOW_CYLINDER || p->kind == SANS_CORE_SHELL_CYLINDER
                           || p->kind == SANS_CORE_SHELL_BICELLE || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL
                           || p->kind == SANS_STACKED_DISKS || p->kind == SANS_SC_PARACRYSTAL
                           || p->kind == SANS_BCC_PARACRYSTAL || p->kind == SANS_FCC_PARACRYSTAL
                           || p->kind == SANS_LAMELLAR_HG || p->kind == SANS_LAMELLAR_STACK_CAILLE
                           || p->kind == SANS_LAMELLAR_STACK_PARACRYSTAL
                           || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH || p->kind == SANS_PRINGLE
                           || p->kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL || p->kind == SANS_FLEXIBLE_CYLINDER;
    int nsize = (p->kind <= 1 || p->kind == SANS_SUPERBALL || p->kind == SANS_ADSORBED_LAYER) ? 1 : (two_sizes ? 2 : 3);
    if (is_shape_independent(p->kind))
        nsize = (p->kind == SANS_POWER_LAW || p->kind == SANS_GAUSSIAN_PEAK || p->kind == SANS_LORENTZ_PEAK
                 || p->kind == SANS_TWO_POWER_LAW || p->kind == SANS_SPINODAL || p->kind == SANS_POROD
                 || p->kind == SANS_LINE)
                    ? 0
                : (p->kind == SANS_TEUBNER_STREY || p->kind == SANS_GAUSS_LORENTZ_GEL
                   || p->kind == SANS_TWO_LORENTZIAN)
                    ? 2
                    : 1;
    if (is_sphere_family(p->kind))
        nsize = (p->kind == SANS_FRACTAL || p->kind == SANS_FRACTAL_CORE_SHELL || p->kind == SANS_RASPBERRY
                 || p->kind == SANS_PEARL_NECKLACE || p->kind == SANS_BINARY_HARD_SPHERE) ? 2 : 1;
    for (int k = 0; k < nsize; ++k)
        if (!(p->size[k] > 0.0) || !finite(p->size[k])) return fail(SANS_E_INVALID_ARG, "size must be > 0");
    if (p->kind == SANS_BARBELL || p->kind == SANS_CAPPED_CYLINDER) {
        if (!(p->size[2] >= p->size[0]))
            return fail(SANS_E_INVALID_ARG, "cap radius size[2] must be >= the cylinder radius size[0]");
        if (p->poly > 0.0 && p->poly_mask != 7)
            return fail(SANS_E_UNSUPPORTED, "barbell / capped cylinder: poly_mask must be 7 (all sizes)");
        if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
    }
    if (p->kind == SANS_PRINGLE) {
        if (!(finite(p->extra[0]) && finite(p->extra[1])))
            return fail(SANS_E_INVALID_ARG, "pringle: curvatures extra[0], extra[1] must be finite");
        if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
        if (p->mode == SANS_MODE_QUAD)
            return fail(SANS_E_UNSUPPORTED, "pringle: no quadrature mode (2 quad_n^2 nodes per orientation node)");
        if (p->poly > 0.0 && (p->poly_mask & 4))
            return fail(SANS_E_UNSUPPORTED, "pringle: poly_mask bits 0 (radius) and 1 (thickness) only");
    }
    if (p->kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL || p->kind == SANS_FLEXIBLE_CYLINDER) {
        if (!(p->extra[0] > 0.0 && finite(p->extra[0])))
            return fail(SANS_E_INVALID_ARG, "flexible cylinder: Kuhn length extra[0] must be > 0");
        if (p->kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL && !(p->extra[1] > 0.0 && finite(p->extra[1])))
            return fail(SANS_E_INVALID_ARG, "flexible elliptical cylinder: axis ratio extra[1] must be > 0");
        if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
        if (p->mode != SANS_MODE_MC) return fail(SANS_E_UNSUPPORTED, "flexible cylinder: Monte Carlo mode only");
        if (p->poly > 0.0 && (p->poly_mask & 4))
            return fail(SANS_E_UNSUPPORTED, "flexible cylinder: poly_mask bits 0 (radius) and 1 (length) only");
    }
    if (p->kind == SANS_ADSORBED_LAYER) {
        if (!(p->shell > 0.0 && finite(p->shell) && p->extra[0] >= 0.0 && finite(p->extra[0])))
            return fail(SANS_E_INVALID_ARG, "adsorbed layer: need a thickness shell > 0 and a smearing extra[0] >= 0");
        if (p->poly > 0.0) return fail(SANS_E_UNSUPPORTED, "adsorbed layer: monodisperse only");
        if (p->sq_phi > 0.0) return fail(SANS_E_UNSUPPORTED, "adsorbed layer: no structure factor");
    }
    if (p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH
        && !(p->shell >= 0.0 && finite(p->shell) && p->extra[0] >= 0.0 && finite(p->extra[0]) && finite(p->extra[1])
             && p->extra[2] > 0.0 && finite(p->extra[2]) && p->extra[3] >= 0.0 && finite(p->extra[3])))
        return fail(SANS_E_INVALID_ARG, "belt bicelle: need belt shell >= 0, face thickness extra[0] >= 0, a finite "
                                        "face SLD extra[1], ratio extra[2] > 0 and roughness extra[3] >= 0");
    if (p->kind >= SANS_LAMELLAR_HG && p->kind <= SANS_LAMELLAR_STACK_PARACRYSTAL) {
        if (p->kind != SANS_LAMELLAR_HG
            && !(p->extra[0] >= 1.0 && p->extra[0] <= 1000.0 && p->extra[0] == std::floor(p->extra[0])))
            return fail(SANS_E_INVALID_ARG, "lamellar stack: integer sheet count extra[0] in 1..1000");
        if ((p->kind == SANS_LAMELLAR_STACK_CAILLE || p->kind == SANS_LAMELLAR_HG_STACK_CAILLE)
            && !(p->extra[1] >= 0.0 && p->extra[1] <= 1.0))
            return fail(SANS_E_INVALID_ARG, "Caille stack: Caille parameter extra[1] must be in [0, 1]");
        if (p->kind == SANS_LAMELLAR_STACK_PARACRYSTAL && !(p->extra[1] >= 0.0 && finite(p->extra[1])))
            return fail(SANS_E_INVALID_ARG, "paracrystalline stack: spacing spread extra[1] must be >= 0");
        if (p->poly > 0.0) return fail(SANS_E_UNSUPPORTED, "lamellae: monodisperse only");
        if (p->sq_phi > 0.0) return fail(SANS_E_UNSUPPORTED, "lamellae: no structure factor");
    }
    if (p->kind == SANS_SUPERBALL) {
        if (!(p->extra[0] >= 0.25 && p->extra[0] <= 10000.0))
            return fail(SANS_E_INVALID_ARG, "superball: exponent parameter extra[0] must be in [0.25, 10000]");
        if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
        if (p->mode == SANS_MODE_QUAD)
            return fail(SANS_E_UNSUPPORTED, "superball: no quadrature mode (quad_n^2 nodes per orientation node)");
        if (p->poly > 0.0 && p->poly_mask != 1)
            return fail(SANS_E_UNSUPPORTED, "superball: poly_mask must be 1 (one size)");
    }
    if (p->kind == 1 && !(p->shell >= 0.0 && finite(p->shell)))
        return fail(SANS_E_INVALID_ARG, "shell must be >= 0");
    if (p->kind == SANS_HOLLOW_PRISM && !(p->shell > 0.0 && finite(p->shell)))
        return fail(SANS_E_INVALID_ARG, "hollow prism: wall thickness (shell) must be > 0");
    if ((p->kind == SANS_CORE_SHELL_CYLINDER || p->kind == SANS_CORE_SHELL_ELLIPSOID
         || p->kind == SANS_CORE_SHELL_BICELLE || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL
         || p->kind == SANS_STACKED_DISKS)
        && !(p->shell >= 0.0 && finite(p->shell)))
        return fail(SANS_E_INVALID_ARG, "shell must be >= 0");
    if ((p->kind == SANS_CORE_SHELL_BICELLE || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL)
        && !(p->extra[0] >= 0.0 && finite(p->extra[0]) && finite(p->extra[1])))
        return fail(SANS_E_INVALID_ARG, "bicelle: face thickness extra[0] >= 0 and a finite face SLD extra[1]");
    if (p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL && !(p->extra[2] > 0.0 && finite(p->extra[2])))
        return fail(SANS_E_INVALID_ARG, "elliptical bicelle: cross-section ratio extra[2] must be > 0");
    if (p->kind == SANS_STACKED_DISKS
        && !(p->extra[0] >= 1.0 && p->extra[0] <= 1000.0 && p->extra[0] == std::floor(p->extra[0])
             && p->extra[1] >= 0.0 && finite(p->extra[1])))
        return fail(SANS_E_INVALID_ARG, "stacked disks: integer count extra[0] in 1..1000, spread extra[1] >= 0");
    if ((p->kind == SANS_SC_PARACRYSTAL || p->kind == SANS_BCC_PARACRYSTAL || p->kind == SANS_FCC_PARACRYSTAL)
        && !(p->extra[0] > 0.0 && p->extra[0] < 1.0))
        return fail(SANS_E_INVALID_ARG, "paracrystal: distortion factor extra[0] must be in (0, 1)");
    if (p->kind == SANS_CORE_SHELL_PARALLELEPIPED
        && !(p->extra[0] >= 0.0 && p->extra[1] >= 0.0 && p->extra[2] >= 0.0 && finite(p->extra[0])
             && finite(p->extra[1]) && finite(p->extra[2])))
        return fail(SANS_E_INVALID_ARG, "core-shell parallelepiped: slab thicknesses extra[0..2] must be >= 0");
    if (p->kind == SANS_CORE_SHELL_CYLINDER && !(p->extra[0] >= 0.0 && finite(p->extra[0])))
        return fail(SANS_E_INVALID_ARG, "core-shell cylinder: face shell extra[0] must be >= 0");
    if (p->kind == SANS_HOLLOW_CYLINDER && !(p->shell > 0.0 && finite(p->shell)))
        return fail(SANS_E_INVALID_ARG, "hollow cylinder: wall thickness (shell) must be > 0");
    if (p->kind == SANS_HOLLOW_PRISM_THICK) {
        if (!(p->shell > 0.0 && 2.0 * p->shell < std::min(p->size[0], std::min(p->size[1], p->size[2]))))
            return fail(SANS_E_INVALID_ARG, "thick hollow prism: need 0 < 2 shell < every edge");
        if (p->poly > 0.0 && p->poly_mask != 0)
            return fail(SANS_E_UNSUPPORTED, "thick hollow prism: monodisperse edges only");
    }
    if (is_shape_independent(p->kind)) {
        if (!(p->extra[0] >= 0.0 && finite(p->extra[0])))
            return fail(SANS_E_INVALID_ARG, "shape-independent model: scale extra[0] must be >= 0");
        if (p->kind == SANS_POLY_GAUSS_COIL && !(p->extra[1] >= 0.0 && p->extra[1] <= 100.0))
            return fail(SANS_E_INVALID_ARG, "polydisperse coil: U = Mw/Mn - 1 (extra[1]) must be in [0, 100]");
        if (p->kind == SANS_POWER_LAW && !(p->extra[1] >= 0.0 && p->extra[1] <= 10.0))
            return fail(SANS_E_INVALID_ARG, "power law: exponent extra[1] must be in [0, 10]");
        if ((p->kind == SANS_GAUSSIAN_PEAK || p->kind == SANS_LORENTZ_PEAK)
            && !(p->extra[1] >= 0.0 && finite(p->extra[1]) && p->extra[2] > 0.0 && finite(p->extra[2])))
            return fail(SANS_E_INVALID_ARG, "peak: need position extra[1] >= 0 and width extra[2] > 0");
        if (p->kind == SANS_MASS_FRACTAL && !(p->extra[1] > 1.0 && p->extra[1] <= 3.0))
            return fail(SANS_E_INVALID_ARG, "mass fractal: dimension extra[1] must be in (1, 3]");
        if (p->kind == SANS_STAR_POLYMER && !(p->extra[1] >= 1.0 && finite(p->extra[1])))
            return fail(SANS_E_INVALID_ARG, "star polymer: arm number extra[1] must be >= 1");
        if (p->kind == SANS_GAUSS_LORENTZ_GEL && !(p->extra[1] >= 0.0 && finite(p->extra[1])))
            return fail(SANS_E_INVALID_ARG, "gel: Lorentzian scale extra[1] must be >= 0");
        if (p->kind == SANS_SURFACE_FRACTAL && !(p->extra[1] > 2.0 && p->extra[1] <= 3.0))
            return fail(SANS_E_INVALID_ARG, "surface fractal: dimension extra[1] must be in (2, 3]");
        if (p->kind == SANS_TWO_POWER_LAW
            && !(p->extra[1] >= 0.0 && p->extra[1] <= 10.0 && p->extra[3] >= 0.0 && p->extra[3] <= 10.0
                 && p->extra[2] > 0.0 && finite(p->extra[2])))
            return fail(SANS_E_INVALID_ARG, "two power law: exponents in [0, 10], crossover extra[2] > 0");
        if (p->kind == SANS_GUINIER_POROD
            && !(p->extra[1] >= 0.0 && p->extra[1] < 3.0 && p->extra[2] > p->extra[1] && p->extra[2] <= 10.0))
            return fail(SANS_E_INVALID_ARG, "Guinier-Porod: need 0 <= s = extra[1] < 3 and s < m = extra[2] <= 10");
        if (p->kind == SANS_LINE && !(p->extra[1] >= 0.0 && finite(p->extra[1])))
            return fail(SANS_E_INVALID_ARG, "line: slope extra[1] must be >= 0");
        if ((p->kind == SANS_TWO_LORENTZIAN || p->kind == SANS_CORRELATION_LENGTH || p->kind == SANS_BROAD_PEAK)
            && !(p->extra[1] >= 0.0 && p->extra[1] <= 10.0 && p->extra[2] >= 0.0 && finite(p->extra[2])
                 && p->extra[3] > 0.0 && p->extra[3] <= 10.0))
            return fail(SANS_E_INVALID_ARG, "need exponents extra[1] in [0, 10] (> 0 for two Lorentzians), "
                                            "extra[3] in (0, 10] and a scale extra[2] >= 0");
        if ((p->kind == SANS_TWO_LORENTZIAN) && !(p->extra[1] > 0.0))
            return fail(SANS_E_INVALID_ARG, "two Lorentzians: exponent extra[1] must be > 0");
        if (p->kind == SANS_BROAD_PEAK && !(p->size[1] >= 0.0 && finite(p->size[1])))
            return fail(SANS_E_INVALID_ARG, "broad peak: position size[1] must be >= 0");
        if (p->kind == SANS_POLYMER_EXCL_VOLUME && !(p->extra[1] >= 1.0 / 3.0 && p->extra[1] <= 1.0))
            return fail(SANS_E_INVALID_ARG, "excluded-volume polymer: Flory exponent extra[1] must be in [1/3, 1]");
        if (p->kind == SANS_SPINODAL
            && !(p->extra[1] > 0.0 && finite(p->extra[1]) && p->extra[2] > 0.0 && p->extra[2] <= 10.0))
            return fail(SANS_E_INVALID_ARG, "spinodal: need q_max = extra[1] > 0 and 0 < gamma = extra[2] <= 10");
        if (p->kind == SANS_MASS_SURFACE_FRACTAL
            && !(p->extra[1] > 0.0 && p->extra[2] > 0.0 && p->extra[1] + p->extra[2] < 6.0
                 && p->size[1] >= 0.0 && finite(p->size[1])))
            return fail(SANS_E_INVALID_ARG, "mass-surface fractal: need Dm = extra[1] > 0, Ds = extra[2] > 0, "
                                            "Dm + Ds < 6 and a primary radius size[1] >= 0");
        if (p->kind == SANS_GEL_FIT
            && !(p->extra[2] > 0.0 && p->extra[2] <= 6.0 && p->extra[1] >= 0.0 && finite(p->extra[1])
                 && p->size[1] >= 0.0 && finite(p->size[1])))
            return fail(SANS_E_INVALID_ARG, "gel: need dimension extra[2] in (0, 6], a Guinier scale "
                                            "extra[1] >= 0 and a radius size[1] >= 0");
        if (p->poly > 0.0) return fail(SANS_E_UNSUPPORTED, "shape-independent model: no size distribution");
        if (p->sq_phi > 0.0) return fail(SANS_E_UNSUPPORTED, "shape-independent model: no structure factor");
    }
    if (is_sphere_family(p->kind)) {
        if ((p->kind == SANS_FUZZY_SPHERE || p->kind == SANS_FRACTAL_CORE_SHELL) && !(p->shell >= 0.0 && finite(p->shell)))
            return fail(SANS_E_INVALID_ARG, "fuzzy sphere: the fuzz width (shell) must be >= 0");
        if ((p->kind == SANS_VESICLE || p->kind == SANS_MULTILAYER_VESICLE) && !(p->shell > 0.0 && finite(p->shell)))
            return fail(SANS_E_INVALID_ARG, "vesicle: the shell thickness must be > 0");
        if ((p->kind == SANS_MULTILAYER_VESICLE || p->kind == SANS_LINEAR_PEARLS)
            && !(p->size[1] >= 0.0 && finite(p->size[1]) && p->extra[0] >= 1.0 && p->extra[0] <= 1000.0
                 && p->extra[0] == std::floor(p->extra[0])))
            return fail(SANS_E_INVALID_ARG, "need a gap size[1] >= 0 and an integer count extra[0] in 1..1000");
        if (p->kind == SANS_MULTILAYER_VESICLE && p->poly > 0.0 && p->poly_mask != 0)
            return fail(SANS_E_UNSUPPORTED, "multilayer vesicle: monodisperse only");
        if (p->kind == SANS_BINARY_HARD_SPHERE) {
            if (!(p->phi > 0.0 && p->phi < 0.6 && p->extra[0] >= 0.0 && p->extra[0] <= p->phi))
                return fail(SANS_E_INVALID_ARG, "binary hard spheres: need 0 < phi < 0.6 and 0 <= extra[0] <= phi");
            if (p->poly > 0.0) return fail(SANS_E_UNSUPPORTED, "binary hard spheres: monodisperse only");
            if (p->sq_phi > 0.0)
                return fail(SANS_E_UNSUPPORTED, "binary hard spheres: the partial structure factors are built in");
        }
        if (p->kind == SANS_PEARL_NECKLACE) {
            if (!(p->extra[0] >= 1.0 && p->extra[0] <= 1000.0 && p->extra[0] == std::floor(p->extra[0])
                  && p->size[2] >= 0.0 && finite(p->size[2])))
                return fail(SANS_E_INVALID_ARG, "pearl necklace: integer pearl count extra[0] in 1..1000 and a rod "
                                                "diameter size[2] >= 0");
            if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
            if (p->poly > 0.0 && p->poly_mask != 1)
                return fail(SANS_E_UNSUPPORTED, "pearl necklace: poly_mask must be 1 (the pearls)");
        }
        if (p->kind == SANS_RASPBERRY) {
            if (!(p->extra[0] >= 0.0 && p->extra[0] <= 1e4 && p->extra[1] >= 0.0 && p->extra[1] <= 1.0))
                return fail(SANS_E_INVALID_ARG, "raspberry: need a count extra[0] in [0, 1e4] and a penetration "
                                                "extra[1] in [0, 1]");
            if (p->poly > 0.0 && p->poly_mask != 1)
                return fail(SANS_E_UNSUPPORTED, "raspberry: poly_mask must be 1 (the large sphere)");
        }
        if ((p->kind == SANS_FRACTAL || p->kind == SANS_FRACTAL_CORE_SHELL)
            && !(p->extra[1] > 1.0 && p->extra[1] <= 3.0))
            return fail(SANS_E_INVALID_ARG, "fractal aggregate: dimension extra[1] must be in (1, 3]");
    }
    if (p->kind == SANS_POLYMER_MICELLE) {
        if (!(p->extra[0] >= 1.0 && finite(p->extra[0])))
            return fail(SANS_E_INVALID_ARG, "micelle: aggregation number extra[0] must be >= 1");
        for (int k = 1; k < 4; ++k)
            if (!(p->extra[k] >= 0.0 && finite(p->extra[k])))
                return fail(SANS_E_INVALID_ARG, "micelle: volumes and penetration extra[1..3] must be >= 0");
        if (!(p->extra[1] + p->extra[2] > 0.0))
            return fail(SANS_E_INVALID_ARG, "micelle: the chain volume extra[1] + extra[2] must be > 0");
    }
    for (int k = 0; k < 3; ++k)
        if (!finite(p->sld[k])) return fail(SANS_E_INVALID_ARG, "sld must be finite");
    if (!(p->phi >= 0.0 && p->phi < 1.0)) return fail(SANS_E_INVALID_ARG, "phi must be in [0, 1)");
    if (!(p->sq_phi >= 0.0 && p->sq_phi < 0.6)) return fail(SANS_E_INVALID_ARG, "sq_phi must be in [0, 0.6)");
    if (!(p->mu_att >= 0.0 && finite(p->mu_att))) return fail(SANS_E_INVALID_ARG, "mu_att must be >= 0");
    if (!(p->guide[0] >= 0.0 && finite(p->guide[0]))) return fail(SANS_E_INVALID_ARG, "guide length must be >= 0");
    if (p->guide[0] > 0.0) {
        const double* g = p->guide;
        if (!(g[1] > 0.0 && finite(g[1]) && g[2] > 0.0 && finite(g[2]) && g[3] >= 0.0 && finite(g[3])))
            return fail(SANS_E_INVALID_ARG, "guide: width and height must be > 0 and the gap >= 0");
        if (!(g[4] > 0.0 && finite(g[4]) && g[5] > 0.0 && g[5] <= 1.0 && g[6] > 0.0 && finite(g[6])
              && g[7] >= 0.0 && finite(g[7]) && g[8] > 0.0 && finite(g[8])))
            return fail(SANS_E_INVALID_ARG, "guide: need m > 0, R0 in (0, 1], Qc > 0, alpha >= 0 and W > 0");
        if (p->mode == SANS_MODE_SURROGATE) return fail(SANS_E_UNSUPPORTED, "surrogate mode: no guide");
    }
    if (p->mu_att > 0.0 && p->mode == SANS_MODE_SURROGATE)
        return fail(SANS_E_UNSUPPORTED, "surrogate mode: no attenuation");
    if (p->sq_phi > 0.0 && !(p->sq_radius > 0.0)) return fail(SANS_E_INVALID_ARG, "sq_radius must be > 0");
    if (p->sq_kind < SANS_SQ_HARD_SPHERE || p->sq_kind > SANS_SQ_HAYTER_MSA)
        return fail(SANS_E_UNSUPPORTED, "unknown sq_kind");
    if (p->sq_phi > 0.0 && p->sq_kind == SANS_SQ_HAYTER_MSA) {
        if (!(p->sq_extra[0] >= 0.0 && p->sq_extra[0] <= 50.0))
            return fail(SANS_E_INVALID_ARG, "Hayter-Penfold: contact potential sq_extra[0] must be in [0, 50]");
        if (!(p->sq_extra[1] > 0.0 && p->sq_extra[1] <= 50.0))
            return fail(SANS_E_INVALID_ARG, "Hayter-Penfold: screening sq_extra[1] must be in (0, 50]");
        if (!(p->lambda0 > 0.0 && p->dlambda_rel >= 0.0 && p->dlambda_rel < 1.0 && p->cone_alpha > 0.0
              && std::isfinite(msa_kmax(*p))))
            return fail(SANS_E_INVALID_ARG, "Hayter-Penfold: the instrument's q range is not finite");
        std::vector<double> cin(host::kMsaCin);
        if (!host::msa_solve(p->sq_phi, p->sq_extra[0], p->sq_extra[1], cin.data()))
            return fail(SANS_E_DOMAIN, "Hayter-Penfold: no physical solution at these parameters");
    }
    if (p->sq_phi > 0.0 && p->sq_kind == SANS_SQ_STICKY_HARD_SPHERE) {
        if (!(p->sq_extra[0] > 0.0 && finite(p->sq_extra[0])))
            return fail(SANS_E_INVALID_ARG, "adhesive spheres: stickiness sq_extra[0] must be > 0");
        double ca[kPySeriesTerms], cb[kPySeriesTerms], hbc[3];
        if (!host::sticky_constants(p->sq_phi, p->sq_extra[0], kPySeriesTerms, ca, cb, hbc))
            return fail(SANS_E_DOMAIN, "adhesive spheres: no solution at this stickiness and volume fraction");
    }
    if (p->sq_phi > 0.0 && p->sq_kind == SANS_SQ_SQUARE_WELL) {
        if (!(finite(p->sq_extra[0]) && p->sq_extra[1] >= 1.0 && p->sq_extra[1] <= 4.0))
            return fail(SANS_E_INVALID_ARG, "square well: need a finite depth sq_extra[0] and a width sq_extra[1] in [1, 4]");
        // 1/S must stay positive on the instrument's q range (FP64 scan of
        // x = 2 q R from 0 to past the largest q of the cone)
        const double lmin = p->lambda0 * (1.0 - p->dlambda_rel);
        const double qmax = 4.0 * kPi / lmin * std::sin(0.5 * p->cone_alpha);
        const double xmax = 2.0 * p->sq_radius * qmax * 1.01;
        double c[kPySeriesTerms], abg[3];
        host::py_series(p->sq_phi, kPySeriesTerms, c, abg);
        const double w = p->sq_extra[1], d8 = 8.0 * p->sq_phi * p->sq_extra[0];
        auto phi3 = [](double y) {
            if (y < 1e-3) return 1.0 - y * y / 10.0;
            return 3.0 * (std::sin(y) - y * std::cos(y)) / (y * y * y);
        };
        for (int i = 0; i <= 4096; ++i) {
            const double x = xmax * i / 4096.0;
            double gx;
            if (x < 1.0) {
                gx = 0.0;
                for (int m = kPySeriesTerms - 1; m >= 0; --m) gx = gx * x * x + c[m];
            } else {
                const double sx = std::sin(x), cx = std::cos(x), x2 = x * x;
                gx = (abg[0] * (sx - x * cx) / x2 + abg[1] * (2.0 * x * sx + (2.0 - x2) * cx - 2.0) / (x2 * x)
                      + abg[2] * (-x2 * x2 * cx + 4.0 * ((3.0 * x2 - 6.0) * cx + (x2 * x - 6.0 * x) * sx + 6.0))
                            / (x2 * x2 * x)) / x;
            }
            const double inv = 1.0 + 24.0 * p->sq_phi * gx - d8 * (w * w * w * phi3(w * x) - phi3(x));
            if (!(inv > 1e-6))
                return fail(SANS_E_DOMAIN, "square well: 1/S(q) <= 0 inside the instrument's q range");
        }
    }
    if (!(p->poly >= 0.0 && p->poly <= 1.0)) return fail(SANS_E_INVALID_ARG, "poly must be in [0, 1]");
    if (p->poly > 0.0 && p->poly < 1e-4) return fail(SANS_E_INVALID_ARG, "poly must be 0 or >= 1e-4");
    if (p->poly_mask < 0 || p->poly_mask > 7) return fail(SANS_E_INVALID_ARG, "poly_mask must be in 0..7");
    if (p->poly_kind != SANS_POLY_SCHULZ && p->poly_kind != SANS_POLY_GAUSSIAN)
        return fail(SANS_E_UNSUPPORTED, "unknown poly_kind");
    bool sep = false;
    for (int k = 0; k < 3; ++k) {
        if (!(p->poly_sep[k] >= 0.0 && p->poly_sep[k] <= 1.0))
            return fail(SANS_E_INVALID_ARG, "poly_sep must be in [0, 1]");
        if (p->poly_sep[k] > 0.0 && p->poly_sep[k] < 1e-4)
            return fail(SANS_E_INVALID_ARG, "poly_sep must be 0 or >= 1e-4");
        sep |= p->poly_sep[k] > 0.0;
    }
    if (sep) {
        // sizes each model takes independent widths for
        const int nsep = p->kind == SANS_SPHERE ? 1
                       : p->kind == SANS_CYLINDER ? 2
                       : (p->kind == SANS_ELLIPSOID || p->kind == SANS_PARALLELEPIPED
                          || p->kind == SANS_ELLIPTICAL_CYLINDER) ? 3 : 0;
        if (nsep == 0)
            return fail(SANS_E_UNSUPPORTED, "poly_sep: sphere, cylinder, ellipsoid, parallelepiped or "
                                            "elliptical cylinder only");
        for (int k = nsep; k < 3; ++k)
            if (p->poly_sep[k] > 0.0) return fail(SANS_E_INVALID_ARG, "poly_sep: this model has no such size");
        if (p->mode != SANS_MODE_MC) return fail(SANS_E_UNSUPPORTED, "poly_sep: Monte Carlo mode only");
        if (p->poly > 0.0) return fail(SANS_E_INVALID_ARG, "poly_sep: poly must be 0");
        if (p->poly_kind != SANS_POLY_GAUSSIAN)
            return fail(SANS_E_UNSUPPORTED, "poly_sep: the positive Gaussian (SANS_POLY_GAUSSIAN) only");
    }
    if (p->table_size < 64 || p->table_size > 8192 || (p->table_size & 1))
        return fail(SANS_E_INVALID_ARG, "table_size must be even and in 64..8192");
    for (int k = 0; k < 3; ++k) {
        if (!finite(p->orient_mean[k])) return fail(SANS_E_INVALID_ARG, "orient_mean must be finite");
        if (!(p->orient_sigma[k] >= 0.0) || !finite(p->orient_sigma[k]))
            return fail(SANS_E_INVALID_ARG, "orient_sigma must be >= 0");
    }
    const double pos[] = {p->src_w, p->src_h, p->slit_w, p->slit_h, p->lambda0, p->cone_alpha,
                          p->sample_w, p->sample_h, p->sample_d, p->det_w, p->det_h};
    for (double v : pos)
        if (!(v >= 0.0) || !finite(v)) return fail(SANS_E_INVALID_ARG, "instrument sizes must be >= 0");
    if (!(p->lambda0 > 0.0) || !(p->det_w > 0.0) || !(p->det_h > 0.0))
        return fail(SANS_E_INVALID_ARG, "lambda0, det_w, det_h must be > 0");
    if (!(p->cone_alpha > 0.0 && p->cone_alpha < 1.5))
        return fail(SANS_E_INVALID_ARG, "cone_alpha must be in (0, 1.5)");
    if (!(p->dlambda_rel >= 0.0 && p->dlambda_rel < 1.0))
        return fail(SANS_E_INVALID_ARG, "dlambda_rel must be in [0, 1)");
    if (!finite(p->src_z) || !finite(p->slit_z) || !finite(p->det_z) || !(p->slit_z > p->src_z))
        return fail(SANS_E_INVALID_ARG, "need src_z < slit_z (finite)");
    if (p->nx < 1 || p->ny < 1 || (int64_t)p->nx * p->ny > (1 << 26))
        return fail(SANS_E_INVALID_ARG, "nx*ny must be in 1..2^26");
    if (p->mode == SANS_MODE_QUAD) {
        if (p->quad_n < 1 || p->quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
        if (is_aniso(p->kind) && p->orient_kind != SANS_ORIENT_FIXED && p->orient_kind != SANS_ORIENT_ISOTROPIC)
            return fail(SANS_E_UNSUPPORTED, "quadrature mode averages fixed or isotropic orientations only");
    }
    return SANS_OK;
}

// Fills the model's constants and (re)builds tables when needed.
SchulzJob schulz_job(double p, unsigned long long out)
{
    SchulzJob j;
    j.a = 1.0 / (p * p);
    j.lnorm = j.a * std::log(j.a) - std::lgamma(j.a);
    j.ymax = 1.0 + 60.0 * p + 10.0 * p * p;
    j.out = out;
    return j;
}

const GL16& gl16_nodes()
{
    static GL16 g;
    static std::once_flag once;
    std::call_once(once, [] {
        host::gauss_legendre(16, g.x, g.w);
        host::gauss_legendre(4, g.x4, g.w4);
    });
    return g;
}

// Builds njobs Schulz tables of M knots on the device (jobs on the host).
int build_schulz_tables(const SchulzJob* jobs, int njobs, int M, double* d_tables, hipStream_t s)
{
    if (njobs <= 0) return SANS_OK;
    SchulzJob* d_jobs = nullptr;
    HIP_TRY(hipMalloc(&d_jobs, sizeof(SchulzJob) * njobs));
    hipError_t e = hipMemcpyAsync(d_jobs, jobs, sizeof(SchulzJob) * njobs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_schulz_tables, dim3(njobs), dim3(kSchulzBlock), 0, s, d_jobs, M, d_tables,
                           gl16_nodes());
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_jobs);
    if (e != hipSuccess) return fail(SANS_E_HIP, std::string("Schulz tables: ") + hipGetErrorString(e));
    return SANS_OK;
}

// Constants of one experiment (everything but the tables and quadrature
// nodes): geometry in FP64, physics constants, Percus-Yevick series.
void fill_constants(const sans_params* p, TraceArgs& a, double* mean_v, double* wscale, double* omc)
{
    std::memset(&a, 0, sizeof(a));
    a.kind = p->kind;
    a.src_w = p->src_w;
    a.src_h = p->src_h;
    a.src_z = p->src_z;
    a.slit_w = p->slit_w;
    a.slit_h = p->slit_h;
    a.slit_z = p->slit_z;
    a.lambda0 = p->lambda0;
    a.lambda_span = p->lambda0 * p->dlambda_rel;
    a.half_x = 0.5 * p->sample_w;
    a.half_y = 0.5 * p->sample_h;
    a.half_z = 0.5 * p->sample_d;
    a.clear_x = a.half_x * (1.0 - 1e-9);
    a.clear_y = a.half_y * (1.0 - 1e-9);
    const double sh = std::sin(0.5 * p->cone_alpha);
    *omc = 2.0 * sh * sh;
    a.omc = *omc;
    a.mu_att = p->mu_att;
    a.att_on = p->mu_att > 0.0;
    a.guide_on = p->guide[0] > 0.0;
    a.guide_len = p->guide[0];
    a.guide_hw = 0.5 * p->guide[1];
    a.guide_hh = 0.5 * p->guide[2];
    a.guide_gap = p->guide[3];
    a.guide_m = p->guide[4];
    a.guide_r0 = p->guide[5];
    a.guide_qc = p->guide[6];
    a.guide_alpha = p->guide[7];
    a.guide_wc = p->guide[8];
    a.det_z = p->det_z;
    a.det_hw = 0.5 * p->det_w;
    a.det_hh = 0.5 * p->det_h;
    a.inv_px = p->nx / p->det_w;
    a.inv_py = p->ny / p->det_h;
    a.nx = p->nx;
    a.ny = p->ny;
    // FP32 geometry of isotropic models: the source upstream of the slab, the
    // detector downstream
    a.fast_geom = p->src_z < -a.half_z && p->det_z > a.half_z;
    a.f_src_w = (float)p->src_w;
    a.f_src_h = (float)p->src_h;
    a.f_slit_w = (float)p->slit_w;
    a.f_slit_h = (float)p->slit_h;
    a.f_inv_dz = (float)(1.0 / (p->slit_z - p->src_z));
    a.f_lz_in = (float)(-a.half_z - p->src_z);
    a.f_lz_out = (float)(a.half_z - p->src_z);
    a.f_depth = (float)p->sample_d;
    a.f_half_z = (float)a.half_z;
    a.f_clear_x = (float)(a.half_x * (1.0 - 1e-5));
    a.f_clear_y = (float)(a.half_y * (1.0 - 1e-5));
    a.f_omc = (float)*omc;
    a.f_det_z = (float)p->det_z;
    a.f_det_hw = (float)a.det_hw;
    a.f_det_hh = (float)a.det_hh;
    a.f_inv_px = (float)a.inv_px;
    a.f_inv_py = (float)a.inv_py;
    // pixel edges within 6e-7 m (three times the FP32 path's error bound) are
    // decided in FP64
    a.f_eps_x = (float)(6e-7 * a.inv_px);
    a.f_eps_y = (float)(6e-7 * a.inv_py);
    a.f_fz_min = 0.5f;
    *mean_v = host::mean_volume(p->kind, p->size, p->shell, p->poly, p->poly_mask, p->poly_kind, p->extra);
    if (p->poly_sep[0] > 0.0 || p->poly_sep[1] > 0.0 || p->poly_sep[2] > 0.0) {
        // independent draws: V is a product of powers e_k of the sizes, so
        // <V> = V prod_k <y_k^e_k>
        const double* s = p->size;
        double v = 0.0;
        int e[3] = {1, 1, 1};
        switch (p->kind) {
        case SANS_SPHERE: v = 4.0 / 3.0 * kPi * s[0] * s[0] * s[0]; e[0] = 3; e[1] = e[2] = 0; break;
        case SANS_CYLINDER: v = kPi * s[0] * s[0] * s[1]; e[0] = 2; e[2] = 0; break;
        case SANS_ELLIPSOID: v = 4.0 / 3.0 * kPi * s[0] * s[1] * s[2]; break;
        case SANS_PARALLELEPIPED: v = s[0] * s[1] * s[2]; break;
        default: v = kPi * s[0] * s[1] * s[2]; break;   // elliptical cylinder
        }
        for (int k = 0; k < 3; ++k) v *= host::positive_normal_moment(p->poly_sep[k], e[k]);
        *mean_v = v;
    }
    if (p->kind == SANS_BINARY_HARD_SPHERE) {
        // the total volume fraction over the total number density
        const double v1 = 4.0 / 3.0 * kPi * p->size[0] * p->size[0] * p->size[0];
        const double v2 = 4.0 / 3.0 * kPi * p->size[1] * p->size[1] * p->size[1];
        const double n1 = (p->phi - p->extra[0]) / v1, n2 = p->extra[0] / v2;
        *mean_v = p->phi / (n1 + n2);
        a.bhs_sn[0] = (float)std::sqrt(n1);
        a.bhs_sn[1] = (float)std::sqrt(n2);
        a.bhs_int = (float)(1.0 / (n1 + n2));
    }
    const double dOmega = 2.0 * 3.141592653589793 * *omc;
    // n F^2 in 1/Angstrom; a shape-independent model's cross-section is in 1/cm
    *wscale = 1e10 * dOmega * (is_shape_independent(p->kind) ? 1e-8 : p->phi / *mean_v);
    a.wscale = *wscale;
    a.f_wscale = (float)*wscale;
    for (int k = 0; k < 3; ++k) {
        a.size[k] = p->size[k];
        a.fsize[k] = (float)p->size[k];
        a.ang_sin[k] = std::sin(p->orient_mean[k]);
        a.ang_cos[k] = std::cos(p->orient_mean[k]);
        a.ang_sigma[k] = p->orient_sigma[k];
    }
    a.shell = p->shell;
    a.fshell = (float)p->shell;
    if (is_sphere_family(p->kind)) {
        a.sf_n = (int32_t)p->extra[0];
        a.sf_gap = p->size[1];
        if (p->kind == SANS_PEARL_NECKLACE) {
            a.cap_n = p->quad_n;
            a.rb_n = (float)((p->sld[1] - p->sld[2]) * kPi * 0.25 * p->size[2] * p->size[2] * p->size[1]);
        }
        if (p->kind == SANS_RASPBERRY) {
            a.rb_n = (float)p->extra[0];
            a.sf_gap = p->size[1] * (1.0 - 2.0 * p->extra[1]);
        }
        if (p->kind == SANS_FRACTAL || p->kind == SANS_FRACTAL_CORE_SHELL) {
            const double d = p->extra[1];
            a.si_a = d * std::tgamma(d - 1.0);
            a.si_c = d;
            a.si_d = p->size[1];
            a.si_e = std::tgamma(d + 1.0);
        }
    }
    if (p->kind == SANS_CORE_SHELL_CYLINDER || p->kind == SANS_CORE_SHELL_BICELLE
        || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH) {
        a.cs_face = p->extra[0];
        a.fcs_face = (float)p->extra[0];
    }
    if (p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH)
        a.bi_x = p->extra[2];
    if (p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH) {
        // contrasts of the core, face and belt regions (core - face - belt +
        // solvent, face - solvent, belt - solvent) and -sigma^2 / 2
        a.bi_c[0] = (float)(p->sld[0] - p->extra[1] - p->sld[1] + p->sld[2]);
        a.bi_c[1] = (float)(p->extra[1] - p->sld[2]);
        a.bi_c[2] = (float)(p->sld[1] - p->sld[2]);
        a.bi_rough = -0.5 * p->extra[3] * p->extra[3];
    }
    if (p->kind == SANS_STACKED_DISKS) {
        a.sf_n = (int32_t)p->extra[0];
        a.sd_d = p->size[1] + 2.0 * p->shell;
        a.sd_sig = p->extra[1];
    }
    if (p->kind == SANS_SC_PARACRYSTAL || p->kind == SANS_BCC_PARACRYSTAL || p->kind == SANS_FCC_PARACRYSTAL) {
        // primitive vectors in units of the nearest-neighbour distance D
        static const double sc[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        static const double bcc[3][3] = {{-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
        static const double fcc[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
        const double(*v)[3] = p->kind == SANS_SC_PARACRYSTAL ? sc : (p->kind == SANS_BCC_PARACRYSTAL ? bcc : fcc);
        const double scale = p->size[1] / (p->kind == SANS_SC_PARACRYSTAL ? 1.0
                                           : (p->kind == SANS_BCC_PARACRYSTAL ? std::sqrt(3.0) : std::sqrt(2.0)));
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) a.pc_v[k][j] = v[k][j] * scale;
        const double gd = p->extra[0] * p->size[1];
        a.pc_b = 0.5 * gd * gd;
    }
    if (p->kind == SANS_CORE_SHELL_BICELLE || p->kind == SANS_CORE_SHELL_BICELLE_ELLIPTICAL) {
        a.bi_c[0] = (float)(p->sld[0] - p->extra[1]);
        a.bi_c[1] = (float)(p->extra[1] - p->sld[1]);
        a.bi_c[2] = (float)(p->sld[1] - p->sld[2]);
    }
    if (p->kind == SANS_CORE_SHELL_PARALLELEPIPED) {
        for (int k = 0; k < 3; ++k) {
            a.csp_t[k] = p->extra[k];
            a.fcsp_t[k] = (float)p->extra[k];
        }
    }
    if (is_shape_independent(p->kind)) {
        a.si_scale = (float)p->extra[0];
        a.si_u = p->extra[1];
        a.si_z = 1.0 / (1.0 + 2.0 * p->extra[1]);
        const double e1 = p->extra[1], e2 = p->extra[2];
        switch (p->kind) {
        case SANS_POWER_LAW: a.si_a = e1; break;
        case SANS_GAUSSIAN_PEAK:
        case SANS_LORENTZ_PEAK: a.si_a = e1; a.si_b = 1.0 / e2; break;
        case SANS_MASS_FRACTAL: a.si_a = e1 - 1.0; a.si_b = e1 * (e1 + 1.0) / 6.0; break;
        case SANS_STAR_POLYMER: a.si_a = e1 / (3.0 * e1 - 2.0); a.si_b = e1 - 1.0; a.si_c = 1.0 / e1; break;
        case SANS_GAUSS_LORENTZ_GEL: a.si_a = e1; a.si_b = p->size[1]; break;
        case SANS_SURFACE_FRACTAL:
            a.si_a = 5.0 - e1;
            a.si_b = (6.0 - e1) * (7.0 - e1) / 6.0;
            break;
        case SANS_TWO_POWER_LAW:
            a.si_a = e1;
            a.si_b = e2;
            a.si_c = p->extra[3];
            a.si_d = std::pow(e2, p->extra[3] - e1);
            break;
        case SANS_GUINIER_POROD: {
            const double q1 = std::sqrt((e2 - e1) * (3.0 - e1) / 2.0) / p->size[0];
            a.si_a = e1;
            a.si_b = e2;
            a.si_c = q1;
            a.si_d = std::exp(-(e2 - e1) / 2.0) * std::pow(q1, e2 - e1);
            a.si_e = 1.0 / (3.0 - e1);
            break;
        }
        case SANS_SPINODAL: a.si_a = 1.0 / e1; a.si_b = e2; a.si_c = 1.0 + 0.5 * e2; break;
        case SANS_LINE: a.si_a = e1; break;
        case SANS_TWO_LORENTZIAN:
            a.si_a = e1;
            a.si_b = e2;
            a.si_c = p->extra[3];
            a.si_d = p->size[0];
            a.si_e = p->size[1];
            break;
        case SANS_CORRELATION_LENGTH:
        case SANS_BROAD_PEAK:
            a.si_a = e1;
            a.si_b = e2;
            a.si_c = p->extra[3];
            a.si_d = p->size[0];
            a.si_e = p->size[1];
            break;
        case SANS_MASS_SURFACE_FRACTAL: {
            const double pm = 0.5 * e1, ps = 0.5 * (6.0 - e2 - e1);
            a.si_a = 1.0 / (3.0 * pm);
            a.si_b = pm;
            a.si_c = p->size[1] * p->size[1] / (3.0 * ps);
            a.si_d = ps;
            break;
        }
        case SANS_GEL_FIT:
            a.si_a = (e2 + 1.0) / 3.0;
            a.si_b = 0.5 * e2;
            a.si_c = e1;
            a.si_d = p->size[1] * p->size[1] / 3.0;
            break;
        case SANS_POLYMER_EXCL_VOLUME:
            a.si_a = (2.0 * e1 + 1.0) * (2.0 * e1 + 2.0) / 6.0;
            a.si_b = e1;
            a.si_c = 0.5 / e1;
            a.si_d = 1.0 / e1;
            a.si_f = std::tgamma(0.5 / e1);
            a.si_g = std::tgamma(1.0 / e1);
            break;
        default: break;
        }
        if (p->kind == SANS_TEUBNER_STREY) {
            const double k = 2.0 * 3.141592653589793 / p->size[1], ix2 = 1.0 / (p->size[0] * p->size[0]);
            a.ts_c = (float)(ix2 - k * k);
            a.ts_e = (float)(4.0 * k * k * ix2);
            a.ts_n = (float)((k * k + ix2) * (k * k + ix2));
        }
    }
    if (p->kind == SANS_POLYMER_MICELLE) {
        a.mic_n = (float)p->extra[0];
        a.mic_bs = (float)(p->extra[1] * (p->sld[0] - p->sld[2]));
        a.mic_bc = (float)(p->extra[2] * (p->sld[1] - p->sld[2]));
        a.mic_d = p->extra[3];
    }
    if (p->kind == SANS_SUPERBALL) a.cap_n = p->quad_n;
    if (p->kind == SANS_PRINGLE) a.cap_n = p->quad_n;
    if (p->kind == SANS_FLEXIBLE_CYLINDER_ELLIPTICAL || p->kind == SANS_FLEXIBLE_CYLINDER) {
        a.cap_n = p->quad_n;
        a.fc_b = (float)p->extra[0];
        a.fc_eps = p->kind == SANS_FLEXIBLE_CYLINDER ? 1.0f : (float)p->extra[1];
    }
    if (p->kind == SANS_ADSORBED_LAYER) {
        a.lam_c = (float)(6.0 * kPi / p->size[0]);
        a.sd_sig = p->extra[0];
    }
    if (p->kind >= SANS_LAMELLAR_HG && p->kind <= SANS_LAMELLAR_STACK_PARACRYSTAL) {
        const bool hg = p->kind == SANS_LAMELLAR_HG || p->kind == SANS_LAMELLAR_HG_STACK_CAILLE;
        const double delta = hg ? 2.0 * (p->size[0] + p->size[1]) : p->size[0];
        a.lam_c = (float)(2.0 * kPi / delta);
        a.lam_eta = (float)p->extra[1];
        a.sf_n = p->kind == SANS_LAMELLAR_HG ? 1 : (int)p->extra[0];
        a.sd_d = p->kind == SANS_LAMELLAR_HG_STACK_CAILLE ? p->size[2] : p->size[1];
        a.sd_sig = p->kind == SANS_LAMELLAR_STACK_PARACRYSTAL ? p->extra[1] : 0.0;
    }
    if (p->kind == SANS_BARBELL || p->kind == SANS_CAPPED_CYLINDER) {
        double zc, t0, vcaps;
        host::cap_geometry(p->kind == SANS_BARBELL, p->size[0], p->size[1], p->size[2], &zc, &t0, &vcaps);
        a.cap_n = p->quad_n;
        a.cap_zc = zc;
        a.cap_r = p->size[2];
        a.fcap_zc = (float)zc;
        a.fcap_r = (float)p->size[2];
    }
    {
        // fixed-orientation axes for the quadrature path: A = R x, B = R y, C = R z
        const double st = a.ang_sin[0], ct = a.ang_cos[0], sp = a.ang_sin[1], cp = a.ang_cos[1],
                     ss = a.ang_sin[2], cs = a.ang_cos[2];
        const double A[3] = {cp * ct * cs - sp * ss, sp * ct * cs + cp * ss, -st * cs};
        const double B[3] = {-cp * ct * ss - sp * cs, -sp * ct * ss + cp * cs, st * ss};
        const double Cc[3] = {cp * st, sp * st, ct};
        for (int k = 0; k < 3; ++k) {
            a.fA[k] = (float)A[k];
            a.fB[k] = (float)B[k];
            a.fC[k] = (float)Cc[k];
        }
    }
    a.contrast = (float)(p->sld[0] - p->sld[2]);
    a.cs_core = (float)(p->sld[0] - p->sld[1]);
    a.cs_shell = (float)(p->sld[1] - p->sld[2]);
    a.poly_on = p->poly > 0.0;
    a.poly_mask = p->poly_mask;
    a.orient_kind = p->orient_kind;
    const bool aniso = is_aniso(p->kind);
    for (int k = 0; k < 3; ++k) a.sep_on[k] = p->mode == SANS_MODE_MC && p->poly_sep[k] > 0.0;
    a.sep_any = a.sep_on[0] || a.sep_on[1] || a.sep_on[2];
    a.sep_block3 = a.sep_on[1] || a.sep_on[2];
    a.third_block = p->mode == SANS_MODE_MC && (a.poly_on || (aniso && p->orient_kind != 0) || a.sep_any);
    a.sq_on = p->sq_phi > 0.0;
    if (a.sq_on) {
        double c[kPySeriesTerms], abg[3];
        host::py_series(p->sq_phi, kPySeriesTerms, c, abg);
        for (int k = 0; k < kPySeriesTerms; ++k) a.py_c[k] = (float)c[k];
        a.py_alpha = (float)abg[0];
        a.py_beta = (float)abg[1];
        a.py_gamma = (float)abg[2];
        a.sq_2r = (float)(2.0 * p->sq_radius);
        a.sq_24phi = (float)(24.0 * p->sq_phi);
        a.sq_kind = p->sq_kind;
        // the Chebyshev form of G(x)/x up to the instrument's largest x = q sigma
        // (1 % margin), when that stays within 12
        const double lmin = p->lambda0 * (1.0 - p->dlambda_rel);
        const double xmax = 2.0 * p->sq_radius * 4.0 * kPi / lmin * std::sin(0.5 * p->cone_alpha) * 1.01;
        a.py_cheb_xmax = -1.0f;   // none: every x takes the series or the closed form
        if (xmax > 0.0 && xmax <= 12.0) {
            double cc[kPyCheb];
            host::py_chebyshev(p->sq_phi, xmax, kPyCheb, cc);
            for (int k = 0; k < kPyCheb; ++k) a.py_cheb[k] = (float)cc[k];
            a.py_cheb_s = (float)(2.0 / (xmax * xmax));
            a.py_cheb_xmax = (float)xmax;
        }
    }
    a.M = p->table_size;
}

int configure(sans_model_s* m, const sans_params* p)
{
    int rc = validate(p);
    if (rc) return rc;
    const sans_params old = m->p;
    const bool first = (m->d_tab_norm == nullptr && m->d_tab_size == nullptr && m->d_quad == nullptr
                        && m->args.M == 0);
    m->p = *p;
    TraceArgs& a = m->args;
    fill_constants(p, a, &m->mean_v, &m->wscale, &m->omc);
    const bool aniso = is_aniso(p->kind);


    // tables
    const bool need_size = p->mode == SANS_MODE_MC && a.poly_on;
    const bool need_norm = p->mode == SANS_MODE_MC && aniso && p->orient_kind == SANS_ORIENT_GAUSSIAN;
    const bool size_same = !first && old.table_size == p->table_size && old.poly == p->poly
                           && old.poly_kind == p->poly_kind && !m->h_tab_size.empty();
    const bool norm_same = !first && old.table_size == p->table_size && !m->h_tab_norm.empty();
    if (need_size) {
        if (!size_same) {
            if (m->d_tab_size) HIP_TRY(hipFree(m->d_tab_size));
            m->d_tab_size = nullptr;
            HIP_TRY(hipMalloc(&m->d_tab_size, sizeof(double) * p->table_size));
            if (p->poly_kind == SANS_POLY_GAUSSIAN) {
                // closed-form quantile: built on the host
                m->h_tab_size.resize(p->table_size);
                host::positive_normal_table(p->table_size, p->poly, m->h_tab_size.data());
                HIP_TRY(hipMemcpy(m->d_tab_size, m->h_tab_size.data(), sizeof(double) * p->table_size,
                                  hipMemcpyHostToDevice));
            } else {
                const SchulzJob job = schulz_job(p->poly, 0);
                int rc2 = build_schulz_tables(&job, 1, p->table_size, m->d_tab_size, nullptr);
                if (rc2) return rc2;
                HIP_TRY(hipStreamSynchronize(nullptr));
                m->h_tab_size.assign(p->table_size, 0.0);
                HIP_TRY(hipMemcpy(m->h_tab_size.data(), m->d_tab_size, sizeof(double) * p->table_size,
                                  hipMemcpyDeviceToHost));
            }
        }
        a.tab_size = m->d_tab_size;
    }
    if (need_norm) {
        if (!norm_same) {
            m->h_tab_norm.resize(p->table_size);
            host::normal_table(p->table_size, m->h_tab_norm.data());
            if (m->d_tab_norm) HIP_TRY(hipFree(m->d_tab_norm));
            m->d_tab_norm = nullptr;
            HIP_TRY(hipMalloc(&m->d_tab_norm, sizeof(double) * p->table_size));
            HIP_TRY(hipMemcpy(m->d_tab_norm, m->h_tab_norm.data(), sizeof(double) * p->table_size,
                              hipMemcpyHostToDevice));
        }
        a.tab_norm = m->d_tab_norm;
    }
    if (a.sep_any) {
        // one positive-Gaussian table per independent width, [3][M] (rows of
        // sizes without a width are not read)
        const int M = p->table_size;
        m->h_tab_sep.assign((size_t)3 * M, 1.0);
        for (int k = 0; k < 3; ++k)
            if (a.sep_on[k]) host::positive_normal_table(M, p->poly_sep[k], m->h_tab_sep.data() + (size_t)k * M);
        if (m->d_tab_sep) HIP_TRY(hipFree(m->d_tab_sep));
        m->d_tab_sep = nullptr;
        HIP_TRY(hipMalloc(&m->d_tab_sep, sizeof(double) * 3 * M));
        HIP_TRY(hipMemcpy(m->d_tab_sep, m->h_tab_sep.data(), sizeof(double) * 3 * M, hipMemcpyHostToDevice));
        a.tab_sep = m->d_tab_sep;
    }

    // the end caps' rule or the superball's nested rule (every mode), then the
    // constants of an adhesive or square-well structure factor or the
    // Hayter-Penfold knots
    if (node_floats(*p)) {
        std::vector<float> rule(node_floats(*p));
        if (m->d_caps) HIP_TRY(hipFree(m->d_caps));
        m->d_caps = nullptr;
        HIP_TRY(hipMalloc(&m->d_caps, sizeof(float) * rule.size()));
        if (!fill_nodes(*p, rule.data(), m->d_caps, a))
            return fail(SANS_E_DOMAIN, "Hayter-Penfold: no physical solution at these parameters");
        HIP_TRY(hipMemcpy(m->d_caps, rule.data(), sizeof(float) * rule.size(), hipMemcpyHostToDevice));
    }

    // quadrature nodes: mu in [0, 1], beta in [0, pi/2], size y in
    // [max(0, 1 - 6p), 1 + 8p] with Schulz weights normalised to sum 1
    // (also the exact fallback and normalisation of the surrogate mode)
    if (p->mode == SANS_MODE_QUAD || p->mode == SANS_MODE_SURROGATE) {
        const int n = p->quad_n;
        std::vector<double> gx(n), gw(n);
        host::gauss_legendre(n, gx.data(), gw.data());
        int ny = 1;
        std::vector<double> ys(1, 1.0), wy(1, 1.0);
        if (a.poly_on) {
            ny = n;
            ys.assign(n, 0.0);
            wy.assign(n, 0.0);
            const bool gauss = p->poly_kind == SANS_POLY_GAUSSIAN;
            const double lo = std::max(0.0, 1.0 - 6.0 * p->poly), hi = 1.0 + (gauss ? 6.0 : 8.0) * p->poly;
            const double aa = 1.0 / (p->poly * p->poly);
            const double lnorm = aa * std::log(aa) - std::lgamma(aa);
            double tot = 0.0;
            for (int j = 0; j < n; ++j) {
                ys[j] = lo + 0.5 * (hi - lo) * (gx[j] + 1.0);
                const double y = ys[j];
                const double d = (y - 1.0) / p->poly;
                const double pdf = y <= 0.0 ? 0.0
                                 : gauss  ? std::exp(-0.5 * d * d)
                                          : std::exp(lnorm + (aa - 1.0) * std::log(y) - aa * y);
                wy[j] = gw[j] * pdf;
                tot += wy[j];
            }
            for (int j = 0; j < n; ++j) wy[j] /= tot;
        }
        int dims = 0;
        if (aniso && p->orient_kind == SANS_ORIENT_ISOTROPIC) {
            const bool spheroid = (p->kind == SANS_ELLIPSOID || p->kind == SANS_CORE_SHELL_ELLIPSOID)
                                  && p->size[0] == p->size[1]
                                  && ((p->poly_mask & 1) != 0) == ((p->poly_mask & 2) != 0);
            dims = (p->kind == SANS_CYLINDER || p->kind == SANS_BARBELL || p->kind == SANS_CAPPED_CYLINDER
                    || p->kind == SANS_HOLLOW_CYLINDER || p->kind == SANS_CORE_SHELL_CYLINDER
                    || p->kind == SANS_CORE_SHELL_BICELLE || p->kind == SANS_STACKED_DISKS || spheroid)
                       ? 1 : 2;
        }
        a.quad_n = n;
        a.quad_ny = ny;
        a.quad_dims = dims;
        m->h_quad.assign(kQuadArrays * n + 2 * ny, 0.0f);
        for (int i = 0; i < n; ++i) {
            const double mu = 0.5 * (gx[i] + 1.0);
            const double beta = 0.25 * 3.141592653589793 * (gx[i] + 1.0);
            m->h_quad[i] = (float)mu;
            m->h_quad[n + i] = (float)(0.5 * gw[i]);
            m->h_quad[2 * n + i] = (float)std::cos(beta);
            m->h_quad[3 * n + i] = (float)std::sin(beta);
            m->h_quad[4 * n + i] = (float)(0.5 * gw[i]);
            m->h_quad[5 * n + i] = (float)std::sqrt(1.0 - mu * mu);
        }
        for (int j = 0; j < ny; ++j) {
            m->h_quad[kQuadArrays * n + j] = (float)ys[j];
            m->h_quad[kQuadArrays * n + ny + j] = (float)wy[j];
        }
        // <F^2> at q = 0 over the same size nodes: (drho V(y))^2 averaged
        {
            const double drho = p->sld[0] - p->sld[2];
            double f2 = 0.0;
            for (int j = 0; j < ny; ++j) {
                double v = 1.0;
                for (int k = 0; k < 3; ++k) v *= (p->poly_mask >> k & 1) ? p->size[k] * ys[j] : p->size[k];
                if (p->kind == SANS_ELLIPSOID) v *= 4.0 / 3.0 * 3.141592653589793;
                f2 += wy[j] * (drho * v) * (drho * v);
            }
            m->sur_f2_0 = f2;
        }
        if (m->d_quad) HIP_TRY(hipFree(m->d_quad));
        m->d_quad = nullptr;
        HIP_TRY(hipMalloc(&m->d_quad, sizeof(float) * m->h_quad.size()));
        HIP_TRY(hipMemcpy(m->d_quad, m->h_quad.data(), sizeof(float) * m->h_quad.size(),
                          hipMemcpyHostToDevice));
        a.quad_nodes = m->d_quad;
    }
    return SANS_OK;
}

LdsLayout layout(const sans_model_s* m, bool hist)
{
    LdsLayout l{};
    const TraceArgs& a = m->args;
    int off = 0;
    l.hist = off;
    if (hist) off += a.nx * a.ny;
    l.tab_size = off;
    if (a.tab_size) off += a.M;
    l.tab_norm = off;
    if (a.tab_norm) off += a.M;
    l.quad = off;
    l.quad_floats = 0;  // the quadrature nodes are read from global memory (uniform)
    off += (l.quad_floats + 1) / 2;
    l.total = off;
    return l;
}

size_t lds_bytes(const LdsLayout& l) { return sizeof(double) * l.total; }

// LDS budget of the histogram kernels' workgroups
constexpr size_t kTileBytes = 128 * 1024;

// Binned tally: neutrons per chunk times the number of row-band tiles (the
// event buffer holds 8 B per neutron per tile: 1 GiB at 2^27)
#ifndef SANS_BIN_CHUNK_SHIFT
#define SANS_BIN_CHUNK_SHIFT 27
#endif
constexpr int kBinChunkShift = SANS_BIN_CHUNK_SHIFT;

// The emit kernel's launch: 512-lane workgroups, four times as many as fit
// on the chip at once (the grid-stride loop then balances the neutrons whose
// geometry takes the FP64 path; measured on the core-shell and oriented
// cylinder workloads against 256 and 1024 lanes and 1 to 8 times resident)
constexpr int kEmitBlock = 512;
constexpr int kEmitGridPerResident = 4;

// LDS of the emit kernel after its tables: one counter per tile per wave
size_t emit_count_bytes(int ntiles)
{
    return sizeof(unsigned) * (size_t)(kEmitBlock / 64) * (size_t)ntiles;
}

bool hist_fits(const sans_model_s* m)
{
    return lds_bytes(layout(m, true)) <= kLdsMax;
}

int choose_tally(const sans_model_s* m, bool extras)
{
    int t = m->p.tally;
    // the optional sum-of-squares and count outputs use the atomic path, and
    // so do exact-average runs with attenuation or a guide (their histogram
    // and binned kernels are compiled without them)
    if (extras || (needs_instrument(m->p) && m->p.mode != SANS_MODE_MC))
        return t == SANS_TALLY_XCD ? SANS_TALLY_XCD : SANS_TALLY_GLOBAL;
    // the exact average spends thousands of operations per tallied neutron:
    // plain atomics cost nothing there, and the workgroup histogram's LDS
    // would halve the waves per SIMD
    if (t == SANS_TALLY_AUTO && m->p.mode == SANS_MODE_QUAD) t = SANS_TALLY_GLOBAL;
    if (t == SANS_TALLY_AUTO) t = hist_fits(m) ? SANS_TALLY_LDS : SANS_TALLY_BINNED;
    if (t == SANS_TALLY_LDS && !hist_fits(m)) t = SANS_TALLY_BINNED;
    if (t == SANS_TALLY_BINNED) {
        const size_t row_bytes = sizeof(double) * (size_t)m->p.nx;
        const size_t rows = kTileBytes / row_bytes;
        const size_t ntiles = rows ? ((size_t)m->p.ny + rows - 1) / rows : 0;
        const size_t emit_lds = lds_bytes(layout(m, false)) + emit_count_bytes((int)ntiles);
        if (rows == 0 || ntiles > (size_t)kMaxTiles || emit_lds > kLdsMax) t = SANS_TALLY_GLOBAL;
    }
    return t;
}

// Grows a device workspace to at least `count` elements.
template <typename T>
int ensure(T*& ptr, size_t& cap, size_t count)
{
    if (cap >= count && ptr) return SANS_OK;
    if (ptr) HIP_TRY(hipFree(ptr));
    ptr = nullptr;
    cap = 0;
    if (hipMalloc(&ptr, sizeof(T) * count) != hipSuccess) {
        ptr = nullptr;
        return fail(SANS_E_NOMEM, "workspace allocation failed");
    }
    cap = count;
    return SANS_OK;
}

int set_lds_limit(const void* fn, size_t shmem)
{
    if (shmem > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) {
            (void)hipGetLastError();  // do not leave the error for the next call
            return fail(SANS_E_HIP, std::string("LDS limit: ") + hipGetErrorString(e));
        }
    }
    return SANS_OK;
}

int launch_fill(double* p, size_t n, hipStream_t s)
{
    if (n == 0) return SANS_OK;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

}  // namespace

// Constant inputs of the surrogate for this model; false when they lie
// outside the network's domain box.
bool surrogate_inputs(const sans_model_s* m, SurConst& sc)
{
    const sans_params& p = m->p;
    // the networks are trained on Schulz size distributions that scale all
    // three sizes together: any other size distribution takes the exact
    // average throughout
    if (p.poly > 0.0 && (p.poly_kind != SANS_POLY_SCHULZ || (p.poly_mask & 7) != 7)) return false;
    const double x[4] = {0.0, std::log(p.size[1] / p.size[0]), std::log(p.size[2] / p.size[0]), p.poly};
    float u[4];
    for (int k = 1; k < 4; ++k) {
        const double lo = m->sur_lo[k], hi = m->sur_hi[k];
        if (x[k] < lo - 1e-6 || x[k] > hi + 1e-6) return false;
        u[k] = hi > lo ? (float)((2.0 * x[k] - lo - hi) / (hi - lo)) : 0.0f;
    }
    sc.ls0 = (float)std::log(p.size[0]);
    sc.x1 = u[1];
    sc.x2 = u[2];
    sc.x3 = u[3];
    sc.lo0 = m->sur_lo[0];
    sc.hi0 = m->sur_hi[0];
    sc.mid0 = 0.5f * (sc.lo0 + sc.hi0);
    sc.scale0 = sc.hi0 > sc.lo0 ? 2.0f / (sc.hi0 - sc.lo0) : 0.0f;
    sc.f2_0 = (float)m->sur_f2_0;
    const int kind = p.kind == SANS_PARALLELEPIPED ? kParallelepiped : kEllipsoid;
    sc.kref = (float)((p.size[0] * p.size[0] + p.size[1] * p.size[1] + p.size[2] * p.size[2])
                      * sur_rg2_scale(kind) / 6.0);
    sc.ls0d = std::log(p.size[0]);
    sc.jlo = (double)m->sur_lo[0];
    sc.jinv = m->sur_hi[0] > m->sur_lo[0] ? m->sur_nbins / ((double)m->sur_hi[0] - (double)m->sur_lo[0]) : 0.0;
    sc.jnb = m->sur_hi[0] > m->sur_lo[0] ? m->sur_nbins : 0;
    sc.flags = m->d_sur_flags;
    return true;
}

int run_surrogate(sans_model_s* m, const TraceArgs& a, const SurConst& sc, double* det, hipStream_t s)
{
    const uint64_t chunk = std::min<uint64_t>(a.n, 1ull << 22);
    int rc;
    if ((rc = ensure(m->d_queue, m->queue_cap, (size_t)chunk))) return rc;
    if (!m->d_qcount && hipMalloc(&m->d_qcount, sizeof(unsigned)) != hipSuccess) {
        m->d_qcount = nullptr;
        return fail(SANS_E_NOMEM, "surrogate: counter allocation failed");
    }
    const LdsLayout lay = layout(m, false);
    const size_t shmem = lds_bytes(lay);
    if ((rc = set_lds_limit((const void*)sur_kernel(m->p.kind), sur::kSurLdsBytes))) return rc;
    for (uint64_t c0 = 0; c0 < a.n; c0 += chunk) {
        TraceArgs ac = a;
        ac.first = a.first + c0;
        ac.n = std::min<uint64_t>(chunk, a.n - c0);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, m->d_qcount, 1);
        // one workgroup per CU: its LDS holds a hidden layer's 128 KiB of fragments
        const uint64_t blocks = (ac.n + sur::kSurBlock - 1) / sur::kSurBlock;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (uint64_t)m->num_cu));
        hipLaunchKernelGGL(sur_kernel(m->p.kind), dim3(grid), dim3(sur::kSurBlock), sur::kSurLdsBytes, s, ac,
                           m->d_sur_pack, m->d_sur_w, sc, det, m->d_queue, m->d_qcount);
        hipLaunchKernelGGL(sur_queue_kernel(m->p.kind), dim3((unsigned)m->num_cu * 2), dim3(kBlock), shmem, s,
                           ac, lay, m->d_queue, m->d_qcount, det);
        HIP_TRY(hipGetLastError());
    }
    return SANS_OK;
}

// The in-domain judge of the attached network on this model's line of inputs
// (its size ratios and width fixed, x0 = ln(q s0) over the box): the
// network's output against the exact average's target at the edges and
// midpoints of nbins bins; a bin whose error exceeds tol at any of its three
// points is flagged.  err (host, [2 nbins + 1]) and flags (host, [nbins]) are
// optional copies of the result.
int judge_surrogate(sans_model_s* m, double tol, int nbins, float* err, unsigned char* flags)
{
    const sans_params& p = m->p;
    SurConst sc;
    std::memset(&sc, 0, sizeof(sc));
    m->sur_nbins = 0;
    if (!surrogate_inputs(m, sc)) return SANS_OK;   // the whole model takes the exact path
    const int npt = 2 * nbins + 1;
    const double lo = m->sur_lo[0], hi = m->sur_hi[0];
    std::vector<float> x((size_t)npt * mlp::kIn, 0.0f), u((size_t)npt * mlp::kIn, 0.0f);
    for (int j = 0; j < npt; ++j) {
        const double x0 = lo + (hi - lo) * j / (2.0 * nbins);
        float* xr = &x[(size_t)j * mlp::kIn];
        float* ur = &u[(size_t)j * mlp::kIn];
        xr[0] = (float)x0;
        xr[1] = (float)std::log(p.size[1] / p.size[0]);
        xr[2] = (float)std::log(p.size[2] / p.size[0]);
        xr[3] = (float)p.poly;
        ur[0] = hi > lo ? (float)((2.0 * x0 - lo - hi) / (hi - lo)) : 0.0f;
        ur[1] = sc.x1;
        ur[2] = sc.x2;
        ur[3] = sc.x3;
    }
    float *d_x = nullptr, *d_u = nullptr, *d_t = nullptr, *d_y = nullptr, *d_ws = nullptr;
    const size_t wsb = sans_mlp_workspace_bytes(npt);
    hipError_t e = hipMalloc(&d_x, sizeof(float) * x.size());
    if (e == hipSuccess) e = hipMalloc(&d_u, sizeof(float) * u.size());
    if (e == hipSuccess) e = hipMalloc(&d_t, sizeof(float) * npt);
    if (e == hipSuccess) e = hipMalloc(&d_y, sizeof(float) * npt);
    if (e == hipSuccess) e = hipMalloc(&d_ws, wsb);
    if (e == hipSuccess) e = hipMemcpy(d_x, x.data(), sizeof(float) * x.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_u, u.data(), sizeof(float) * u.size(), hipMemcpyHostToDevice);
    int rc = SANS_OK;
    std::vector<float> t(npt), y(npt);
    if (e == hipSuccess) {
        rc = sans_pq_dataset(p.kind, d_x, npt, d_t, p.quad_n, nullptr);
        if (rc == SANS_OK && sans_mlp_forward(m->d_sur_w, d_u, npt, d_y, d_ws, nullptr) != 0)
            rc = fail(SANS_E_HIP, "judge: network forward failed");
        if (rc == SANS_OK) e = hipStreamSynchronize(nullptr);
        if (rc == SANS_OK && e == hipSuccess) e = hipMemcpy(t.data(), d_t, sizeof(float) * npt, hipMemcpyDeviceToHost);
        if (rc == SANS_OK && e == hipSuccess) e = hipMemcpy(y.data(), d_y, sizeof(float) * npt, hipMemcpyDeviceToHost);
    }
    for (float* ptr : {d_x, d_u, d_t, d_y, d_ws})
        if (ptr) (void)hipFree(ptr);
    if (e != hipSuccess) return fail(SANS_E_HIP, std::string("judge: ") + hipGetErrorString(e));
    if (rc) return rc;
    std::vector<unsigned char> fl(nbins);
    for (int b = 0; b < nbins; ++b) {
        const double e0 = std::fabs((double)y[2 * b] - t[2 * b]), e1 = std::fabs((double)y[2 * b + 1] - t[2 * b + 1]),
                     e2 = std::fabs((double)y[2 * b + 2] - t[2 * b + 2]);
        fl[b] = e0 > tol || e1 > tol || e2 > tol;
    }
    if (err)
        for (int j = 0; j < npt; ++j) err[j] = std::fabs(y[j] - t[j]);
    if (flags) std::memcpy(flags, fl.data(), nbins);
    if (m->d_sur_flags) HIP_TRY(hipFree(m->d_sur_flags));
    m->d_sur_flags = nullptr;
    HIP_TRY(hipMalloc(&m->d_sur_flags, nbins));
    HIP_TRY(hipMemcpy(m->d_sur_flags, fl.data(), nbins, hipMemcpyHostToDevice));
    m->sur_nbins = nbins;
    m->sur_tol = tol;
    return SANS_OK;
}

// Scratch of sans_trace_noalloc: the eight per-XCD replicas of the detector,
// in a device array of fixed size that the code object brings with it (every
// GPU the library runs on holds its own copy until the process ends), so the
// entry point needs no allocation.  Host code never passes the array's name to
// a kernel: that is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocMaxPixels = (size_t)1 << 18;            // 512 x 512
static __device__ __align__(256) double scratch[kNoAllocMaxPixels * kXcds];   // 16 MiB

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on
// that device).
int noalloc_scratch(double** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SANS_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SANS_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SANS_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* sans_status_string(int status)
{
    switch (status) {
    case SANS_OK: return "ok";
    case SANS_E_INVALID_ARG: return "invalid argument";
    case SANS_E_UNSUPPORTED: return "unsupported";
    case SANS_E_NOMEM: return "out of memory";
    case SANS_E_HIP: return "HIP runtime error";
    case SANS_E_DOMAIN: return "outside the model domain";
    }
    return "unknown status";
}

const char* sans_last_error(void) { return g_last_error.c_str(); }

uint32_t sans_abi_params_size(void) { return (uint32_t)sizeof(sans_params); }

int sans_model_create(const sans_params* p, sans_model_t* out)
{
    if (!out) return fail(SANS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    sans_model_s* m = new (std::nothrow) sans_model_s();
    if (!m) return fail(SANS_E_NOMEM, "host allocation failed");
    std::memset(&m->args, 0, sizeof(m->args));
    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, m->device) == hipSuccess) m->num_cu = prop.multiProcessorCount;
    } else {
        delete m;
        return fail(SANS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    rc = configure(m, p);
    if (rc) {
        sans_model_destroy(m);
        return rc;
    }
    *out = m;
    return SANS_OK;
}

int sans_model_destroy(sans_model_t m)
{
    if (!m) return SANS_OK;
    if (m->d_tab_size) (void)hipFree(m->d_tab_size);
    if (m->d_tab_norm) (void)hipFree(m->d_tab_norm);
    if (m->d_tab_sep) (void)hipFree(m->d_tab_sep);
    if (m->d_quad) (void)hipFree(m->d_quad);
    if (m->d_caps) (void)hipFree(m->d_caps);
    if (m->d_replicas) (void)hipFree(m->d_replicas);
    if (m->d_partial) (void)hipFree(m->d_partial);
    if (m->d_buckets) (void)hipFree(m->d_buckets);
    if (m->d_bucket_count) (void)hipFree(m->d_bucket_count);
    if (m->d_sur_w) (void)hipFree(m->d_sur_w);
    if (m->d_sur_pack) (void)hipFree(m->d_sur_pack);
    if (m->d_queue) (void)hipFree(m->d_queue);
    if (m->d_qcount) (void)hipFree(m->d_qcount);
    if (m->d_sur_flags) (void)hipFree(m->d_sur_flags);
    delete m;
    return SANS_OK;
}

int sans_model_constants(sans_model_t m, double* out3)
{
    if (!m || !out3) return fail(SANS_E_INVALID_ARG, "NULL argument");
    out3[0] = m->mean_v;
    out3[1] = m->wscale;
    out3[2] = m->omc;
    return SANS_OK;
}

namespace {

// The scattered neutrons' tally of sans_trace_ex (arguments checked there).
int trace_scattered(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                    uint32_t flags, double* det, double* det_w2, uint64_t* det_count, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const size_t npix = (size_t)m->p.nx * m->p.ny;
    const bool acc = flags & SANS_ACCUMULATE;
    if (!acc) {
        int rc = launch_fill(det, npix, s);
        if (rc) return rc;
        if (det_w2 && (rc = launch_fill(det_w2, npix, s))) return rc;
        if (det_count) {
            hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s,
                               (unsigned long long*)det_count, npix);
            HIP_TRY(hipGetLastError());
        }
    }
    if (n == 0) return SANS_OK;
    TraceArgs a = m->args;
    a.first = first;
    a.n = n;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.exp_id = exp_id;
    const unsigned fill_grid = (unsigned)((npix + 255) / 256);
    const unsigned red_grid = (unsigned)((npix + 63) / 64);   // the reductions: 64 pixels per workgroup

    if (m->p.mode == SANS_MODE_SURROGATE) {
        if (det_w2 || det_count) return fail(SANS_E_UNSUPPORTED, "surrogate mode: no det_w2/det_count");
        if (!m->sur_attached) return fail(SANS_E_UNSUPPORTED, "surrogate mode: no network attached");
        SurConst sc;
        if (surrogate_inputs(m, sc)) return run_surrogate(m, a, sc, det, s);
        // the model's own shape lies outside the network's domain: exact path
    }
    const int tally = choose_tally(m, det_w2 != nullptr || det_count != nullptr);

    if (tally == SANS_TALLY_LDS) {
        const LdsLayout lay = layout(m, true);
        const size_t shmem = lds_bytes(lay);
        HistFn fn = pick_hist(m->p.kind, m->p.mode, needs_instrument(m->p));
        int rc = set_lds_limit((const void*)fn, shmem);
        if (rc) return rc;
        const uint64_t blocks_needed = (n + kHistBlock - 1) / kHistBlock;
        const int per_cu = std::max(1, std::min(2, (int)(kLdsMax / shmem)));
        const unsigned grid =
            (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks_needed, (uint64_t)m->num_cu * per_cu));
        if ((rc = ensure(m->d_partial, m->partial_cap, (size_t)grid * npix))) return rc;
        hipLaunchKernelGGL(fn, dim3(grid), dim3(kHistBlock), shmem, s, a, lay, m->d_partial);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_reduce_partials, dim3(red_grid), dim3(64 * kRedWaves), 0, s, det, m->d_partial,
                           (int)grid, (int)npix, 1);
        HIP_TRY(hipGetLastError());
        return SANS_OK;
    }

    if (tally == SANS_TALLY_BINNED) {
        const int rows = (int)(kTileBytes / (sizeof(double) * m->p.nx));
        const int ntiles = (m->p.ny + rows - 1) / rows;
        const int tile_pixels = rows * m->p.nx;
        const int slices = std::max(1, m->num_cu / ntiles);
        // one chunk writes at most 2^(shift + 3) / ntiles bytes of events (8 B
        // each): about the 256 MB last-level cache (2^26 to 2^29 ran within
        // 3 % of each other)
        const uint64_t chunk =
            std::min<uint64_t>(n, std::max<uint64_t>(1u << 20, (1ull << kBinChunkShift) / ntiles));
        // the emit grid (the workgroups that fit on the chip at once: the
        // kernel strides over the chunk) and each wave's segment capacity
        // (its neutrons per chunk)
        const LdsLayout lay = layout(m, false);
        const size_t shmem = lds_bytes(lay) + emit_count_bytes(ntiles);
        EmitFn efn = pick_emit(m->p.kind, m->p.mode, needs_instrument(m->p));
        int rc;
        if ((rc = set_lds_limit((const void*)efn, shmem))) return rc;
        const int eblock = kEmitBlock;
        int occ = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)efn, eblock, shmem));
        const uint64_t eblocks = std::max<uint64_t>(
            1, std::min<uint64_t>((chunk + eblock - 1) / eblock,
                                  (uint64_t)m->num_cu * std::max(1, occ) * kEmitGridPerResident));
        const unsigned nwaves = (unsigned)eblocks * (eblock / 64);
        const uint64_t iters = (chunk + eblocks * eblock - 1) / (eblocks * eblock);
        const unsigned capw = (unsigned)(iters * 64);
        if ((rc = ensure(m->d_partial, m->partial_cap, (size_t)ntiles * slices * tile_pixels))) return rc;
        if ((rc = ensure(m->d_buckets, m->bucket_cap, (size_t)ntiles * nwaves * capw))) return rc;
        if ((rc = ensure(m->d_bucket_count, m->bucket_count_cap, (size_t)ntiles * nwaves))) return rc;
        if ((rc = set_lds_limit((const void*)k_bin_accumulate, sizeof(double) * tile_pixels))) return rc;
        for (uint64_t c0 = 0; c0 < n; c0 += chunk) {
            TraceArgs ac = a;
            ac.first = first + c0;
            ac.n = std::min<uint64_t>(chunk, n - c0);
            hipLaunchKernelGGL(efn, dim3((unsigned)eblocks), dim3(eblock), shmem, s, ac, lay, m->d_buckets,
                               m->d_bucket_count, capw, tile_pixels, ntiles);
            HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(k_bin_accumulate, dim3((unsigned)(ntiles * slices)), dim3(kHistBlock),
                               sizeof(double) * tile_pixels, s, m->d_buckets, m->d_bucket_count, capw, nwaves,
                               tile_pixels, slices, m->d_partial, c0 == 0 ? 1 : 0);
            HIP_TRY(hipGetLastError());
        }
        hipLaunchKernelGGL(k_reduce_binned, dim3(red_grid), dim3(64 * kRedWaves), 0, s, det, m->d_partial,
                           tile_pixels, slices, (int)npix, 1);
        HIP_TRY(hipGetLastError());
        return SANS_OK;
    }

    if (tally == SANS_TALLY_XCD && m->replica_pix != npix) {
        if (m->d_replicas) HIP_TRY(hipFree(m->d_replicas));
        m->d_replicas = nullptr;
        m->replica_pix = 0;
        hipError_t e = hipMalloc(&m->d_replicas, sizeof(double) * npix * kXcds);
        if (e != hipSuccess) return fail(SANS_E_NOMEM, "replica allocation failed");
        m->replica_pix = npix;
        int rc = launch_fill(m->d_replicas, npix * kXcds, s);
        if (rc) return rc;
    }
    const LdsLayout lay = layout(m, false);
    const size_t shmem = lds_bytes(lay);
    TraceFn fn = pick_trace(m->p.kind, m->p.mode, tally);
    if (!fn) return fail(SANS_E_UNSUPPORTED, "no kernel for this model");
    int rc = set_lds_limit((const void*)fn, shmem);
    if (rc) return rc;
    // grid: enough waves to fill every CU; the kernel strides over the range
    const uint64_t blocks_needed = (n + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>(blocks_needed, (uint64_t)m->num_cu * 8));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), shmem, s, a, lay, det, det_w2,
                       (unsigned long long*)det_count, m->d_replicas);
    HIP_TRY(hipGetLastError());
    if (tally == SANS_TALLY_XCD) {
        hipLaunchKernelGGL(k_sum_replicas, dim3(fill_grid), dim3(256), 0, s, det, m->d_replicas,
                           (int)npix, 1);
        HIP_TRY(hipGetLastError());
    }
    return SANS_OK;
}

}  // namespace

int sans_trace_ex(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                  uint32_t flags, double* det, double* det_w2, uint64_t* det_count, void* stream)
{
    (void)hipGetLastError();  // a stale error of an earlier call is not ours
    if (!m || !det) return fail(SANS_E_INVALID_ARG, "model or detector is NULL");
    if (flags & ~(SANS_ACCUMULATE | SANS_TRANSMITTED)) return fail(SANS_E_INVALID_ARG, "unknown flags");
    if (n > 0 && first + n < first) return fail(SANS_E_INVALID_ARG, "neutron range overflows");
    int rc = trace_scattered(m, first, n, seed, exp_id, flags, det, det_w2, det_count, stream);
    if (rc || !(flags & SANS_TRANSMITTED) || n == 0) return rc;
    TraceArgs a = m->args;
    a.first = first;
    a.n = n;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.exp_id = exp_id;
    const unsigned grid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>((n + 255) / 256, (uint64_t)m->num_cu * 8));
    hipLaunchKernelGGL(k_transmit, dim3(grid), dim3(256), 0, (hipStream_t)stream, a, det, det_w2,
                       (unsigned long long*)det_count);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

int sans_debug_transmitted(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                           int32_t* pixel, double* w, void* stream)
{
    (void)hipGetLastError();
    if (!m || !pixel || !w) return fail(SANS_E_INVALID_ARG, "NULL argument");
    if (n > ((uint64_t)1 << 31)) return fail(SANS_E_INVALID_ARG, "n must be at most 2^31");
    if (n > 0 && first + n < first) return fail(SANS_E_INVALID_ARG, "neutron range overflows");
    if (n == 0) return SANS_OK;
    TraceArgs a = m->args;
    a.first = first;
    a.n = n;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.exp_id = exp_id;
    hipLaunchKernelGGL(k_debug_transmit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a,
                       pixel, w);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

int sans_trace_noalloc(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                       uint32_t flags, double* det, void* stream)
{
    (void)hipGetLastError();  // a stale error of an earlier call is not ours
    if (!m || !det) return fail(SANS_E_INVALID_ARG, "model or detector is NULL");
    if (flags & ~SANS_ACCUMULATE) return fail(SANS_E_INVALID_ARG, "unknown flags");
    if (n > 0 && first + n < first) return fail(SANS_E_INVALID_ARG, "neutron range overflows");
    if (m->p.mode == SANS_MODE_SURROGATE)
        return fail(SANS_E_UNSUPPORTED, "sans_trace_noalloc: surrogate mode keeps a queue it allocates");
    const size_t npix = (size_t)m->p.nx * m->p.ny;
    if (npix > kNoAllocMaxPixels)
        return fail(SANS_E_INVALID_ARG, "sans_trace_noalloc: detector of " + std::to_string(npix) +
                                            " pixels exceeds the limit of " + std::to_string(kNoAllocMaxPixels));
    double* rep = nullptr;
    int rc = noalloc_scratch(&rep);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool acc = flags & SANS_ACCUMULATE;
    if (!acc && (rc = launch_fill(det, npix, s))) return rc;
    if (n == 0) return SANS_OK;
    // the previous call on this device may have left anything here
    if ((rc = launch_fill(rep, npix * kXcds, s))) return rc;
    TraceArgs a = m->args;
    a.first = first;
    a.n = n;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.exp_id = exp_id;
    const LdsLayout lay = layout(m, false);
    const size_t shmem = lds_bytes(lay);
    TraceFn fn = pick_trace(m->p.kind, m->p.mode, SANS_TALLY_XCD);
    if (!fn) return fail(SANS_E_UNSUPPORTED, "no kernel for this model");
    if ((rc = set_lds_limit((const void*)fn, shmem))) return rc;
    const uint64_t blocks_needed = (n + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks_needed, (uint64_t)m->num_cu * 8));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), shmem, s, a, lay, det, (double*)nullptr,
                       (unsigned long long*)nullptr, rep);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_replicas, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, det, rep, (int)npix, 1);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

int sans_trace(sans_model_t m, uint64_t n_neutrons, uint64_t seed, const sans_params* params,
               double* detector_out, void* stream)
{
    if (!m) return fail(SANS_E_INVALID_ARG, "model is NULL");
    if (params) {
        int rc = configure(m, params);
        if (rc) return rc;
    }
    return sans_trace_ex(m, 0, n_neutrons, seed, 0, 0, detector_out, nullptr, nullptr, stream);
}

int sans_debug_trace(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                     int32_t* pixel, float* w, float* q, void* stream)
{
    (void)hipGetLastError();  // a stale error of an earlier call is not ours
    if (!m) return fail(SANS_E_INVALID_ARG, "model is NULL");
    if (n == 0) return SANS_OK;
    if (n > (1ull << 31)) return fail(SANS_E_INVALID_ARG, "debug range limited to 2^31 neutrons");
    TraceArgs a = m->args;
    a.first = first;
    a.n = n;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.exp_id = exp_id;
    const LdsLayout lay = layout(m, false);
    DebugFn fn = pick_debug(m->p.kind, m->p.mode, m->p.mu_att > 0.0 || m->p.guide[0] > 0.0);
    if (!fn) return fail(SANS_E_UNSUPPORTED, "no kernel for this model");
    hipLaunchKernelGGL(fn, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), lds_bytes(lay),
                       (hipStream_t)stream, a, lay, pixel, w, q);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

int sans_debug_philox(uint64_t seed, uint64_t first, uint64_t n, uint32_t n_blocks, uint32_t exp_id,
                      uint32_t* out, void* stream)
{
    (void)hipGetLastError();  // a stale error of an earlier call is not ours
    if (!out) return fail(SANS_E_INVALID_ARG, "out is NULL");
    if (n_blocks < 1 || n_blocks > 16) return fail(SANS_E_INVALID_ARG, "n_blocks must be in 1..16");
    if (n == 0) return SANS_OK;
    if (n > (1ull << 30)) return fail(SANS_E_INVALID_ARG, "n too large");
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t)seed, (uint32_t)(seed >> 32), first, n, n_blocks, exp_id, out);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

int sans_debug_weight_scale(const sans_params* p, double* mean_volume, double* wscale)
{
    int rc = validate(p);
    if (rc) return rc;
    TraceArgs a;
    double mv = 0.0, ws = 0.0, omc = 0.0;
    fill_constants(p, a, &mv, &ws, &omc);
    if (mean_volume) *mean_volume = mv;
    if (wscale) *wscale = ws;
    return SANS_OK;
}

int sans_debug_table(sans_model_t m, int32_t which, double* out, int32_t n)
{
    if (!m || !out) return fail(SANS_E_INVALID_ARG, "NULL argument");
    const std::vector<double>& t = which == 0 ? m->h_tab_norm : m->h_tab_size;
    if (which < 0 || which > 1 || t.empty()) return fail(SANS_E_UNSUPPORTED, "no such table");
    if (n != (int32_t)t.size()) return fail(SANS_E_INVALID_ARG, "n must equal table_size");
    std::memcpy(out, t.data(), sizeof(double) * n);
    return SANS_OK;
}

int sans_pq_avg(sans_model_t m, const float* q, const float* qvec, int64_t n, float* out, void* stream)
{
    (void)hipGetLastError();  // a stale error of an earlier call is not ours
    if (!m || !q || !out) return fail(SANS_E_INVALID_ARG, "NULL argument");
    if (m->p.mode != SANS_MODE_QUAD) return fail(SANS_E_UNSUPPORTED, "model is not in quadrature mode");
    if (n < 0) return fail(SANS_E_INVALID_ARG, "n < 0");
    if (m->args.quad_dims == 0 && is_aniso(m->p.kind) && !qvec)
        return fail(SANS_E_INVALID_ARG, "fixed orientation needs qvec");
    if (n == 0) return SANS_OK;
    const LdsLayout lay = layout(m, false);
    hipLaunchKernelGGL(pick_pq(m->p.kind), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       lds_bytes(lay), (hipStream_t)stream, m->args, lay, q, qvec, n, out);
    HIP_TRY(hipGetLastError());
    return SANS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ surrogate C ABI
extern "C" {

int sans_model_attach_surrogate(sans_model_t m, const void* w_bf16, const float* domain_lo,
                                const float* domain_hi)
{
    if (!m || !w_bf16 || !domain_lo || !domain_hi) return fail(SANS_E_INVALID_ARG, "NULL argument");
    for (int k = 0; k < 4; ++k)
        if (!(domain_hi[k] >= domain_lo[k])) return fail(SANS_E_INVALID_ARG, "domain_hi < domain_lo");
    if (!m->d_sur_w) {
        HIP_TRY(hipMalloc(&m->d_sur_w, sizeof(__bf16) * sur::kWeightsPadded));
        HIP_TRY(hipMemset(m->d_sur_w, 0, sizeof(__bf16) * sur::kWeightsPadded));
    }
    if (!m->d_sur_pack) HIP_TRY(hipMalloc(&m->d_sur_pack, sizeof(mlp::bf16x8) * sur::kPackTotal));
    HIP_TRY(hipMemcpy(m->d_sur_w, w_bf16, sizeof(__bf16) * mlp::kParams, hipMemcpyDeviceToDevice));
    hipLaunchKernelGGL(sur::k_pack_surrogate, dim3((unsigned)((sur::kPackTotal + 255) / 256)), dim3(256), 0,
                       nullptr, m->d_sur_w, m->d_sur_pack);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(nullptr));
    for (int k = 0; k < 4; ++k) {
        m->sur_lo[k] = domain_lo[k];
        m->sur_hi[k] = domain_hi[k];
    }
    m->sur_attached = true;
    // the default in-domain judge: 1e-3 on ln <F^2> over 2048 bins
    return judge_surrogate(m, kSurJudgeTol, kSurJudgeBins, nullptr, nullptr);
}

int sans_model_judge_surrogate(sans_model_t m, double tol, int32_t nbins, float* err, uint8_t* flags)
{
    if (!m) return fail(SANS_E_INVALID_ARG, "model is NULL");
    if (!m->sur_attached) return fail(SANS_E_UNSUPPORTED, "judge: no network attached");
    if (nbins < 1 || nbins > 65536) return fail(SANS_E_INVALID_ARG, "judge: nbins must be in 1..65536");
    if (!(tol >= 0.0)) return fail(SANS_E_INVALID_ARG, "judge: tol must be >= 0");
    return judge_surrogate(m, tol, nbins, err, flags);
}

int sans_pq_dataset(int32_t kind, const float* x, int64_t n, float* out, int32_t quad_n, void* stream)
{
    if (!x || !out || n < 0) return fail(SANS_E_INVALID_ARG, "dataset: bad argument");
    if (kind != SANS_ELLIPSOID && kind != SANS_PARALLELEPIPED)
        return fail(SANS_E_UNSUPPORTED, "dataset: ellipsoid (of revolution) or parallelepiped");
    if (quad_n < 1 || quad_n > kMaxQuad) return fail(SANS_E_INVALID_ARG, "quad_n must be in 1..256");
    if (n == 0) return SANS_OK;
    const int nq = quad_n;
    std::vector<double> gx(nq), gw(nq);
    host::gauss_legendre(nq, gx.data(), gw.data());
    std::vector<float> nodes(5 * nq);
    for (int i = 0; i < nq; ++i) {
        const double beta = 0.25 * 3.141592653589793 * (gx[i] + 1.0);
        nodes[i] = (float)(0.5 * (gx[i] + 1.0));
        nodes[nq + i] = (float)(0.5 * gw[i]);
        nodes[2 * nq + i] = (float)std::cos(beta);
        nodes[3 * nq + i] = (float)std::sin(beta);
        nodes[4 * nq + i] = (float)(0.5 * gw[i]);
    }
    hipStream_t s = (hipStream_t)stream;
    float* d_nodes = nullptr;
    double* d_gl = nullptr;
    HIP_TRY(hipMalloc(&d_nodes, sizeof(float) * nodes.size()));
    hipError_t e = hipMalloc(&d_gl, sizeof(double) * 2 * nq);
    if (e == hipSuccess) e = hipMemcpy(d_nodes, nodes.data(), sizeof(float) * nodes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_gl, gx.data(), sizeof(double) * nq, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_gl + nq, gw.data(), sizeof(double) * nq, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        TraceArgs a;
        std::memset(&a, 0, sizeof(a));
        a.contrast = 1.0f;
        a.poly_mask = 7;
        const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(dataset_kernel(kind), dim3(grid), dim3(kBlock), 0, s, a, x, n, out, d_nodes, nq,
                           kind == SANS_PARALLELEPIPED ? 2 : 1, d_gl, d_gl + nq);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_nodes);
    if (d_gl) (void)hipFree(d_gl);
    if (e != hipSuccess) return fail(SANS_E_HIP, std::string("dataset: ") + hipGetErrorString(e));
    return SANS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch host side
namespace {

// A schedule of the batched launch: the tile (neutrons per tile, or cost
// units per tile), how the experiments are split into tiles, and how many
// persistent workgroups share a compute unit.
//   split 0: tiles of `tile` neutrons (an experiment's remainder last), whole
//            tiles in experiment order, then the remainders largest first;
//   split 1: tiles of tile / cost(e) neutrons for the per-neutron cost of
//            experiment e's model, all tiles ordered by their cost, largest
//            first (longest-processing-time order);
//   occ:     persistent workgroups per compute unit (as many as the LDS
//            histogram lets reside together).
struct BatchSchedule {
    long tile = 1l << 18;
    int split = 0;
    int occ = 1;
};

struct BatchCache {
    std::mutex mu;
    TraceArgs* d_exps = nullptr;
    size_t exps_cap = 0;
    BatchTile* d_tiles = nullptr;
    size_t tiles_cap = 0;
    SchulzJob* d_jobs = nullptr;
    size_t jobs_cap = 0;
    double* d_tables = nullptr;
    size_t tables_cap = 0;
    double* d_norm = nullptr;
    int norm_M = 0;
    float* d_caps = nullptr;   // node rules and structure-factor constants, one experiment after another
    size_t caps_cap = 0;
    unsigned* d_counter = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string graph_key;
    std::map<std::string, BatchSchedule> tuned;  // key -> schedule (this process)
    // the Schulz tables in d_tables were built from these jobs (with M knots,
    // in this allocation): a call with the same jobs reuses them, as a model
    // reuses the tables it built when created
    std::vector<SchulzJob> built_jobs;
    double* built_tables = nullptr;
    size_t built_cap = 0;
    int built_M = 0;

    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_key.clear();
        if (d_exps) (void)hipFree(d_exps);
        if (d_tiles) (void)hipFree(d_tiles);
        if (d_jobs) (void)hipFree(d_jobs);
        if (d_tables) (void)hipFree(d_tables);
        built_jobs.clear();
        built_tables = nullptr;
        if (d_norm) (void)hipFree(d_norm);
        if (d_caps) (void)hipFree(d_caps);
        if (d_counter) (void)hipFree(d_counter);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        d_exps = nullptr;
        d_tiles = nullptr;
        d_jobs = nullptr;
        d_tables = nullptr;
        d_norm = nullptr;
        d_caps = nullptr;
        d_counter = nullptr;
        cap_stream = nullptr;
        exps_cap = tiles_cap = jobs_cap = tables_cap = caps_cap = 0;
        norm_M = 0;
    }
};

BatchCache& batch_cache()
{
    static BatchCache c;
    return c;
}

const long kTileCandidates[] = {1l << 16, 1l << 17, 1l << 18, 1l << 19, 1l << 20};

// Relative per-neutron cost of an experiment's model (1 for the closed-form
// amplitudes; models that integrate per event scale with their rule):
// issue-slot counts of the per-neutron steps, about 900 for a plain
// anisotropic particle, 40-60 per node of an inner rule.
double model_cost(const sans_params& p)
{
    const double n = p.quad_n;
    switch (p.kind) {
    case SANS_BARBELL:
    case SANS_CAPPED_CYLINDER: return 1.0 + 43.0 * n / 900.0;
    case SANS_SUPERBALL: return 1.0 + (19.0 * n + 38.0 * n * n) / 900.0;
    case SANS_PRINGLE: return 1.0 + 36.0 * 2.0 * n * n / 900.0;
    case SANS_FLEXIBLE_CYLINDER_ELLIPTICAL: return 0.7 + 40.0 * n / 900.0;
    case SANS_FLEXIBLE_CYLINDER: return 0.7 + 28.0 * n / 900.0;
    case SANS_PEARL_NECKLACE: return 1.0 + (55.0 * n + 8.0 * p.extra[0]) / 900.0;
    case SANS_LAMELLAR_STACK_CAILLE:
    case SANS_LAMELLAR_HG_STACK_CAILLE:
    case SANS_LAMELLAR_STACK_PARACRYSTAL: return 1.0 + 36.0 * p.extra[0] / 900.0;
    case SANS_BINARY_HARD_SPHERE: return 2.1;
    case SANS_POLYMER_EXCL_VOLUME: return 1.6;
    default: return is_shape_independent(p.kind) ? 0.75 : (is_aniso(p.kind) ? 1.1 : 1.0);
    }
}

std::string tune_key(int n_exp, double total_n, int nx, int ny, int num_cu)
{
    std::ostringstream k;
    k << "E" << n_exp << "_S" << (int)std::lround(std::log2(std::max(total_n, 1.0))) << "_D" << nx << "x"
      << ny << "_CU" << num_cu;
    return k.str();
}

// Tuning cache file: one JSON object, one entry per line:
//   "key": {"tile": T, "split": s, "occ": o, "ms": t},
// (an entry without "split" or "occ" takes 0 and 1).
std::map<std::string, BatchSchedule> read_tune_cache(const char* path)
{
    std::map<std::string, BatchSchedule> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
        const size_t t = line.find("\"tile\":");
        if (q0 == std::string::npos || q1 == std::string::npos || t == std::string::npos) continue;
        BatchSchedule sc;
        sc.tile = std::atol(line.c_str() + t + 7);
        const size_t sp = line.find("\"split\":"), oc = line.find("\"occ\":");
        if (sp != std::string::npos) sc.split = std::atoi(line.c_str() + sp + 8);
        if (oc != std::string::npos) sc.occ = std::atoi(line.c_str() + oc + 6);
        if (sc.tile < 1024 || sc.split < 0 || sc.split > 1 || sc.occ < 1 || sc.occ > 8) continue;
        out[line.substr(q0 + 1, q1 - q0 - 1)] = sc;
    }
    return out;
}

void write_tune_cache(const char* path, const std::map<std::string, BatchSchedule>& sched,
                      const std::map<std::string, double>& ms)
{
    std::ofstream f(path, std::ios::trunc);
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : sched) {
        const auto it = ms.find(kv.first);
        f << "\"" << kv.first << "\": {\"tile\": " << kv.second.tile << ", \"split\": " << kv.second.split
          << ", \"occ\": " << kv.second.occ << ", \"ms\": " << (it == ms.end() ? 0.0 : it->second) << "}"
          << (++i < sched.size() ? "," : "") << "\n";
    }
    f << "}\n";
}

// Queues the batch on stream s with schedule sc (graph captured once per
// shape and schedule).  cost: per-neutron cost of each experiment's model.
int run_batch(BatchCache& c, int n_exp, const std::vector<TraceArgs>& exps,
              const std::vector<SchulzJob>& jobs, const uint64_t* n_neutrons, const std::vector<double>& cost,
              const BatchSchedule& sc, int npix, int M, double* dets, size_t lds, int num_cu, hipStream_t s)
{
    std::vector<BatchTile> tiles;
    if (sc.split == 0) {
        // whole tiles first, then the remainders, by decreasing size
        std::vector<BatchTile> rest;
        const uint64_t T = (uint64_t)sc.tile;
        for (int e = 0; e < n_exp; ++e) {
            uint64_t f = 0;
            const uint64_t n = n_neutrons[e];
            for (; f + T <= n; f += T) tiles.push_back(BatchTile{(unsigned)e, (unsigned)T, f});
            if (f < n) rest.push_back(BatchTile{(unsigned)e, (unsigned)(n - f), f});
        }
        std::stable_sort(rest.begin(), rest.end(),
                         [](const BatchTile& x, const BatchTile& y) { return x.count > y.count; });
        tiles.insert(tiles.end(), rest.begin(), rest.end());
    } else {
        // equal-cost tiles, all of them in decreasing order of cost
        std::vector<std::pair<double, BatchTile>> tc;
        for (int e = 0; e < n_exp; ++e) {
            const uint64_t T = (uint64_t)std::max(1024.0, std::min(4.0e9, (double)sc.tile / cost[e]));
            const uint64_t n = n_neutrons[e];
            for (uint64_t f = 0; f < n; f += T) {
                const uint64_t cnt = std::min(T, n - f);
                tc.push_back({cost[e] * (double)cnt, BatchTile{(unsigned)e, (unsigned)cnt, f}});
            }
        }
        std::stable_sort(tc.begin(), tc.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
        tiles.reserve(tc.size());
        for (const auto& t : tc) tiles.push_back(t.second);
    }
    const int ntiles = (int)tiles.size();
    int rc;
    if ((rc = ensure(c.d_tiles, c.tiles_cap, std::max<size_t>(1, tiles.size())))) return rc;
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(c.d_tiles, tiles.data(), sizeof(BatchTile) * tiles.size(),
                               hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.d_exps, exps.data(), sizeof(TraceArgs) * n_exp, hipMemcpyHostToDevice, s));
    if (!jobs.empty())
        HIP_TRY(hipMemcpyAsync(c.d_jobs, jobs.data(), sizeof(SchulzJob) * jobs.size(),
                               hipMemcpyHostToDevice, s));

    std::ostringstream key;
    key << n_exp << "/" << ntiles << "/" << jobs.size() << "/" << npix << "/" << M << "/" << dets << "/"
        << c.d_exps << "/" << c.d_tiles << "/" << c.d_jobs << "/" << c.d_tables << "/" << sc.occ;
    if (c.graph_key != key.str()) {
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
        if (c.graph) (void)hipGraphDestroy(c.graph);
        c.exec = nullptr;
        c.graph = nullptr;
        c.graph_key.clear();
        if (!c.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
        const size_t ndet = (size_t)n_exp * npix;
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((ndet + 255) / 256)), dim3(256), 0, c.cap_stream, dets, ndet);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, c.cap_stream, c.d_counter, 1);
        const unsigned grid = (unsigned)std::max(1, std::min(ntiles, num_cu * sc.occ));
        hipLaunchKernelGGL(batch_kernel(), dim3(grid), dim3(kHistBlock), lds, c.cap_stream, c.d_exps, c.d_tiles,
                           ntiles, c.d_counter, dets, npix, M);
        hipError_t le = hipGetLastError();
        hipError_t ee = hipStreamEndCapture(c.cap_stream, &c.graph);
        if (le != hipSuccess) return fail(SANS_E_HIP, std::string("batch launch: ") + hipGetErrorString(le));
        if (ee != hipSuccess) return fail(SANS_E_HIP, std::string("graph capture: ") + hipGetErrorString(ee));
        HIP_TRY(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
        c.graph_key = key.str();
    }
    // the Schulz tables, unless this allocation already holds them for these
    // very jobs (then they are what the builder would write again)
    const bool tables_ready = c.built_tables == c.d_tables && c.built_cap == c.tables_cap && c.built_M == M
                              && c.built_jobs.size() == jobs.size()
                              && (jobs.empty()
                                  || std::memcmp(c.built_jobs.data(), jobs.data(), sizeof(SchulzJob) * jobs.size()) == 0);
    if (!tables_ready) {
        c.built_tables = nullptr;
        if (!jobs.empty()) {
            hipLaunchKernelGGL(k_schulz_tables, dim3((unsigned)jobs.size()), dim3(kSchulzBlock), 0, s, c.d_jobs, M,
                               c.d_tables, gl16_nodes());
            HIP_TRY(hipGetLastError());
        }
        c.built_jobs = jobs;
        c.built_tables = c.d_tables;
        c.built_cap = c.tables_cap;
        c.built_M = M;
    }
    HIP_TRY(hipGraphLaunch(c.exec, s));
    return SANS_OK;
}

}  // namespace

extern "C" {

int sans_trace_batch(int n_exp, const sans_params* p, const uint64_t* n_neutrons, const uint64_t* seeds,
                     double* detectors_out, const char* tune_cache, void* stream)
{
    (void)hipGetLastError();  // a stale error of an earlier call is not ours
    if (n_exp < 1 || !p || !n_neutrons || !seeds || !detectors_out)
        return fail(SANS_E_INVALID_ARG, "batch: null argument or n_exp < 1");
    const int nx = p[0].nx, ny = p[0].ny, M = p[0].table_size;
    bool any_poly = false, any_norm = false;
    double total_n = 0.0;
    for (int e = 0; e < n_exp; ++e) {
        int rc = validate(&p[e]);
        if (rc == SANS_OK && p[e].mu_att > 0.0)
            rc = fail(SANS_E_UNSUPPORTED, "batched launch: no attenuation (trace attenuated experiments one by one)");
        if (rc == SANS_OK && p[e].guide[0] > 0.0)
            rc = fail(SANS_E_UNSUPPORTED, "batched launch: no guide (trace such experiments one by one)");
        if (rc == SANS_OK && (p[e].poly_sep[0] > 0.0 || p[e].poly_sep[1] > 0.0 || p[e].poly_sep[2] > 0.0))
            rc = fail(SANS_E_UNSUPPORTED, "batched launch: no independent size widths");
        if (rc) return rc;
        if (p[e].mode != SANS_MODE_MC) return fail(SANS_E_UNSUPPORTED, "batch: Monte Carlo mode only");
        if (p[e].nx != nx || p[e].ny != ny) return fail(SANS_E_INVALID_ARG, "batch: detectors must match");
        if (p[e].table_size != M) return fail(SANS_E_INVALID_ARG, "batch: table_size must match");
        if (n_neutrons[e] >= (1ull << 48)) return fail(SANS_E_INVALID_ARG, "batch: neutron count too large");
        any_poly |= p[e].poly > 0.0;
        any_norm |= is_aniso(p[e].kind) && p[e].orient_kind == SANS_ORIENT_GAUSSIAN;
        total_n += (double)n_neutrons[e];
    }
    const int npix = nx * ny;
    const size_t lds = sizeof(double) * (size_t)npix;
    if (lds + 64 > kLdsMax) return fail(SANS_E_UNSUPPORTED, "batch: detector exceeds LDS");
    int device = 0, num_cu = 256;
    HIP_TRY(hipGetDevice(&device));
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) num_cu = prop.multiProcessorCount;
    }
    hipStream_t s = (hipStream_t)stream;
    BatchCache& c = batch_cache();
    std::lock_guard<std::mutex> lock(c.mu);

    // per-experiment constants and table jobs
    std::vector<TraceArgs> exps(n_exp);
    std::vector<SchulzJob> jobs;
    int rc;
    if ((rc = ensure(c.d_exps, c.exps_cap, (size_t)n_exp))) return rc;
    size_t ntab = 0, n_schulz = 0;
    for (int e = 0; e < n_exp; ++e) {
        ntab += p[e].poly > 0.0;
        n_schulz += p[e].poly > 0.0 && p[e].poly_kind == SANS_POLY_SCHULZ;
    }
    std::vector<double> host_tabs;
    std::vector<float> host_caps;
    size_t ncaps = 0;
    for (int e = 0; e < n_exp; ++e) ncaps += node_floats(p[e]);
    if ((rc = ensure(c.d_caps, c.caps_cap, std::max<size_t>(1, ncaps)))) return rc;
    if ((rc = ensure(c.d_tables, c.tables_cap, std::max<size_t>(1, ntab * M)))) return rc;
    if ((rc = ensure(c.d_jobs, c.jobs_cap, std::max<size_t>(1, ntab)))) return rc;
    if (!c.d_counter && hipMalloc(&c.d_counter, sizeof(unsigned)) != hipSuccess) {
        c.d_counter = nullptr;
        return fail(SANS_E_NOMEM, "batch: counter allocation failed");
    }
    if (any_norm && c.norm_M != M) {
        std::vector<double> t(M);
        host::normal_table(M, t.data());
        if (c.d_norm) HIP_TRY(hipFree(c.d_norm));
        c.d_norm = nullptr;
        c.norm_M = 0;
        HIP_TRY(hipMalloc(&c.d_norm, sizeof(double) * M));
        HIP_TRY(hipMemcpy(c.d_norm, t.data(), sizeof(double) * M, hipMemcpyHostToDevice));
        c.norm_M = M;
    }
    for (int e = 0; e < n_exp; ++e) {
        double mv, ws, omc;
        fill_constants(&p[e], exps[e], &mv, &ws, &omc);
        exps[e].seed_lo = (uint32_t)seeds[e];
        exps[e].seed_hi = (uint32_t)(seeds[e] >> 32);
        exps[e].exp_id = (uint32_t)e;
        if (p[e].poly > 0.0 && p[e].poly_kind == SANS_POLY_GAUSSIAN) {
            // closed-form quantiles, built on the host (after the Schulz slots)
            exps[e].tab_size = c.d_tables + (n_schulz + host_tabs.size() / M) * (size_t)M;
            const size_t off = host_tabs.size();
            host_tabs.resize(off + M);
            host::positive_normal_table(M, p[e].poly, host_tabs.data() + off);
        } else if (p[e].poly > 0.0) {
            exps[e].tab_size = c.d_tables + jobs.size() * (size_t)M;
            jobs.push_back(schulz_job(p[e].poly, (unsigned long long)(jobs.size() * (size_t)M)));
        }
        if (is_aniso(p[e].kind) && p[e].orient_kind == SANS_ORIENT_GAUSSIAN) exps[e].tab_norm = c.d_norm;
        if (node_floats(p[e])) {
            const size_t off = host_caps.size();
            host_caps.resize(off + node_floats(p[e]));
            if (!fill_nodes(p[e], host_caps.data() + off, c.d_caps + off, exps[e]))
                return fail(SANS_E_DOMAIN, "Hayter-Penfold: no physical solution at these parameters");
        }
    }
    if (!host_caps.empty())
        HIP_TRY(hipMemcpyAsync(c.d_caps, host_caps.data(), sizeof(float) * host_caps.size(), hipMemcpyHostToDevice, s));
    if (!host_tabs.empty())
        HIP_TRY(hipMemcpyAsync(c.d_tables + n_schulz * (size_t)M, host_tabs.data(), sizeof(double) * host_tabs.size(),
                               hipMemcpyHostToDevice, s));
    if ((rc = set_lds_limit((const void*)batch_kernel(), lds))) return rc;

    // schedule: tuning cache, else autotune (when a cache path is given), else default
    std::vector<double> cost(n_exp);
    for (int e = 0; e < n_exp; ++e) cost[e] = model_cost(p[e]);
    // persistent workgroups that can share a compute unit (LDS histogram)
    const int max_occ = (int)std::max<size_t>(1, std::min<size_t>(4, kLdsMax / (lds + 64)));
    const std::string key = tune_key(n_exp, total_n, nx, ny, num_cu);
    BatchSchedule sched;
    std::map<std::string, BatchSchedule> file_sched;
    if (tune_cache) file_sched = read_tune_cache(tune_cache);
    if (tune_cache && file_sched.count(key)) {
        sched = file_sched[key];
        sched.occ = std::min(sched.occ, max_occ);
    } else if (c.tuned.count(key)) {
        sched = c.tuned[key];
    } else if (tune_cache) {
        // coordinate search: the tile size under the plain split, then the
        // cost-weighted split at the best tile and its neighbours, then the
        // occupancy; each candidate runs the whole batch twice (warm, timed)
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        double best = 1e300;
        auto time_it = [&](const BatchSchedule& cand, double* ms_out) -> int {
            int r;
            if ((r = run_batch(c, n_exp, exps, jobs, n_neutrons, cost, cand, npix, M, detectors_out, lds, num_cu, s)))
                return r;
            HIP_TRY(hipEventRecord(e0, s));
            if ((r = run_batch(c, n_exp, exps, jobs, n_neutrons, cost, cand, npix, M, detectors_out, lds, num_cu, s)))
                return r;
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            *ms_out = ms;
            return SANS_OK;
        };
        auto consider = [&](const BatchSchedule& cand) -> int {
            double ms = 0.0;
            const int r = time_it(cand, &ms);
            if (r == SANS_OK && ms < best) {
                best = ms;
                sched = cand;
            }
            return r;
        };
        for (long t : kTileCandidates) {
            BatchSchedule cand;
            cand.tile = t;
            if ((rc = consider(cand))) return rc;
        }
        const long t0 = sched.tile;
        for (long t : {t0 / 2, t0, t0 * 2}) {
            BatchSchedule cand;
            cand.tile = t;
            cand.split = 1;
            if ((rc = consider(cand))) return rc;
        }
        for (int o = 2; o <= max_occ; o *= 2) {
            BatchSchedule cand = sched;
            cand.occ = o;
            if ((rc = consider(cand))) return rc;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        file_sched[key] = sched;
        std::map<std::string, double> ms;
        ms[key] = best;
        write_tune_cache(tune_cache, file_sched, ms);
    }
    c.tuned[key] = sched;
    return run_batch(c, n_exp, exps, jobs, n_neutrons, cost, sched, npix, M, detectors_out, lds, num_cu, s);
}

int sans_batch_release(void)
{
    BatchCache& c = batch_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    c.release();
    return SANS_OK;
}

}  // extern "C"
