// sans_kernels.hpp -- the per-model kernel templates of libsans (gfx950).
//
//   k_trace_hist<KIND, MODE>    the hot path for detectors that fit in LDS: one
//                               neutron per lane, grid-stride over the range,
//                               FP64 LDS histogram per workgroup
//   k_emit<KIND, MODE>          the hot path for larger detectors: events binned
//                               by detector row band (summed by k_bin_accumulate)
//   k_trace<KIND, MODE, TALLY>  atomic tallies (global / per-XCD replica)
//   k_debug<KIND, MODE, ATT>    the same per-neutron code, writing (pixel, w, q)
//   k_pq_avg<KIND>              the exact average <F^2>(q) alone
//   k_trace_sur<KIND>,          surrogate mode: the network inside the tracer and
//   k_trace_queue<KIND>         the exact pass over the queued neutrons
//   k_pq_dataset<KIND>          training targets by the exact quadrature
// The model switch is a template parameter: a wavefront never diverges on it.
// Each model's instances are compiled in one of several translation units
// (sans_kinds.hip, built once per kind group), which fill a table of kernel
// pointers that the host side of the library launches from.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/sans.h"
#include "sans_device.hpp"
#include "sans_surrogate.hpp"

namespace sans {

constexpr int kBlock = 256;
constexpr int kXcds = 8;
constexpr int kNumKinds = 64;
constexpr int kKindGroups = 8;

// ------------------------------------------------------------------ kernels

// Stage an array into LDS with all threads of the block.
template <typename T>
__device__ __forceinline__ void stage(T* dst, const T* src, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// Dynamic LDS, in doubles: [hist (LDS tally only)] [size table] [normal table]
// [quadrature nodes (floats)]
struct LdsLayout {
    int hist, tab_size, tab_norm, quad, total;  // offsets / total in doubles
    int quad_floats;
};

struct LdsPtrs {
    double* hist;
    double* tsize;
    double* tnorm;
    float* lq;
};

__device__ __forceinline__ LdsPtrs stage_all(const TraceArgs& a, const LdsLayout& lay, double* lds)
{
    LdsPtrs p{lds + lay.hist, lds + lay.tab_size, lds + lay.tab_norm,
              reinterpret_cast<float*>(lds + lay.quad)};
    if (a.tab_size) stage(p.tsize, a.tab_size, a.M);
    if (a.tab_norm) stage(p.tnorm, a.tab_norm, a.M);
    if (lay.quad_floats) stage(p.lq, a.quad_nodes, lay.quad_floats);
    return p;
}

// The trace constants as seen from inside a neutron loop.  They sit in
// memory that no kernel writes (the kernel's argument segment, or the batch's
// parameter array) and are read through a pointer whose value is hidden from
// the compiler at every neutron, so their scalar loads stay inside the loop
// as scalar-cache hits.  Loop-invariant loads hoisted out of the loop would
// overflow the scalar registers (a TraceArgs is a hundred doubles) and come
// back through VALU lane reads, one issue slot each.
using ConstArgs = const __attribute__((address_space(4))) TraceArgs;

__device__ __forceinline__ const TraceArgs& loop_args(ConstArgs* p)
{
    asm volatile("" : "+s"(p));
    return *(const TraceArgs*)p;
}

// The trace kernels take their TraceArgs as the first argument, which the
// argument segment holds at offset 0.
__device__ __forceinline__ ConstArgs* kernel_args()
{
    return (ConstArgs*)__builtin_amdgcn_kernarg_segment_ptr();
}

// Atomic tallies: one FP64 atomic per detected neutron into the detector
// (GLOBAL) or into this XCD's replica of it (XCD).
template <int KIND, int MODE, int TALLY>
__global__ __launch_bounds__(kBlock) void k_trace(const TraceArgs a, LdsLayout lay, double* det,
                                                  double* det_w2, unsigned long long* det_cnt,
                                                  double* replicas)
{
    extern __shared__ double lds_d[];
    const LdsPtrs lp = stage_all(a, lay, lds_d);
    __syncthreads();
    double* target = det;
    if constexpr (TALLY == SANS_TALLY_XCD) {
        const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kXcds - 1);
        target = replicas + (size_t)xcc * a.nx * a.ny;
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n; j += stride) {
        const Event ev = trace_neutron<KIND, MODE, true>(loop_args(kernel_args()), a.first + j, lp.tsize,
                                                         lp.tnorm, lp.lq);
        if (ev.pixel >= 0) {
            const double w = (double)ev.w;
            __hip_atomic_fetch_add(target + ev.pixel, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (det_w2)
                __hip_atomic_fetch_add(det_w2 + ev.pixel, w * w, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            if (det_cnt)
                __hip_atomic_fetch_add(det_cnt + ev.pixel, 1ull, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// LDS tally: the whole detector as an FP64 histogram in LDS, 1024 lanes per
// workgroup; each workgroup writes its histogram to its own partial slot
// (plain stores), summed afterwards by k_reduce_partials.
constexpr int kHistBlock = 1024;

template <int KIND, int MODE, bool ATT = false>
__global__ __launch_bounds__(kHistBlock) void k_trace_hist(const TraceArgs a, LdsLayout lay,
                                                           double* partial)
{
    extern __shared__ double lds_d[];
    const LdsPtrs lp = stage_all(a, lay, lds_d);
    const int npix = a.nx * a.ny;
    for (int i = threadIdx.x; i < npix; i += blockDim.x) lp.hist[i] = 0.0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n; j += stride) {
        const Event ev = trace_neutron<KIND, MODE, ATT>(loop_args(kernel_args()), a.first + j, lp.tsize,
                                                        lp.tnorm, lp.lq);
        if (ev.pixel >= 0)
            __hip_atomic_fetch_add(lp.hist + ev.pixel, (double)ev.w, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    double* out = partial + (size_t)blockIdx.x * npix;
    for (int i = threadIdx.x; i < npix; i += blockDim.x) out[i] = lp.hist[i];
}

// Binned tally, pass 1: the events of one chunk of neutrons go to the
// bucket of their detector tile (rows [t*rows, (t+1)*rows)).  Every wave owns
// one private segment per tile, so no two waves ever write the same
// counter.  A lane takes its rank in the segment from an LDS atomic on the
// wave's counter of its tile: one LDS operation per event whatever the number
// of tiles among the wave's events (the LDS pipe, not the VALU, absorbs the
// lanes that share a tile).  At the end each wave stores its per-tile counts.
// An event is (pixel within the tile, FP32 weight bits); the order of events
// within a segment is immaterial (the second pass sums them).
// compiled for workgroups of up to 1024 lanes (the host picks the size)
constexpr int kEmitBlockMax = 1024;
constexpr int kMaxTiles = 64;

template <int KIND, int MODE, bool ATT = false>
__global__ __launch_bounds__(kEmitBlockMax) void k_emit(const TraceArgs a, LdsLayout lay, uint2* buckets,
                                                     unsigned* seg_count, unsigned capw, int tile_pixels,
                                                     int ntiles)
{
    extern __shared__ double lds_d[];
    const LdsPtrs lp = stage_all(a, lay, lds_d);
    const int lane = threadIdx.x & 63;
    // LDS after the tables: ntiles counters per wave
    unsigned* cnt = reinterpret_cast<unsigned*>(lds_d + lay.total) + (threadIdx.x >> 6) * ntiles;
    if (lane < ntiles) cnt[lane] = 0u;
    __syncthreads();
    const unsigned wpb = blockDim.x >> 6;
    const unsigned nwaves = gridDim.x * wpb;
    const unsigned wv = blockIdx.x * wpb + (threadIdx.x >> 6);
    const float inv_tile = 1.0f / (float)tile_pixels;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n; j += stride) {
        const Event ev = trace_neutron<KIND, MODE, ATT>(loop_args(kernel_args()), a.first + j, lp.tsize,
                                                        lp.tnorm, lp.lq);
        if (ev.pixel >= 0) {
            // tile = pixel / tile_pixels: the FP32 quotient (there are at most
            // 64 tiles, so it is off by at most one) corrected by the remainder
            int t = (int)((float)ev.pixel * inv_tile);
            int local = ev.pixel - __mul24(t, tile_pixels);
            if (local < 0) {
                --t;
                local += tile_pixels;
            } else if (local >= tile_pixels) {
                ++t;
                local -= tile_pixels;
            }
            const unsigned rank = __hip_atomic_fetch_add(cnt + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            buckets[((size_t)t * nwaves + wv) * capw + rank] = make_uint2((unsigned)local, __float_as_uint(ev.w));
        }
    }
    // the counts of this wave's atomics, read back by its own lanes
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (lane < ntiles) seg_count[(size_t)lane * nwaves + wv] = __hip_atomic_load(cnt + lane, __ATOMIC_RELAXED,
                                                                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <int KIND, int MODE, bool ATT>
__global__ __launch_bounds__(kBlock) void k_debug(const TraceArgs a, LdsLayout lay, int32_t* pixel,
                                                  float* w, float* q)
{
    extern __shared__ double lds_d[];
    const LdsPtrs lp = stage_all(a, lay, lds_d);
    __syncthreads();
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const Event ev = trace_neutron<KIND, MODE, ATT>(loop_args(kernel_args()), a.first + j, lp.tsize, lp.tnorm,
                                                    lp.lq);
    if (pixel) pixel[j] = ev.pixel;
    if (w) w[j] = ev.w;
    if (q) q[j] = ev.q;
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_pq_avg(const TraceArgs a, LdsLayout lay, const float* q,
                                                   const float* qvec, int64_t n, float* out)
{
    extern __shared__ double lds_d[];
    (void)stage_all(a, lay, lds_d);
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float qv[3] = {0.0f, 0.0f, 0.0f};
    if (qvec) {
        qv[0] = qvec[3 * j];
        qv[1] = qvec[3 * j + 1];
        qv[2] = qvec[3 * j + 2];
    }
    out[j] = quad_average<KIND>(a, a.quad_nodes, q[j], qv);
}

// ------------------------------------------------------------------ batched experiments
// Persistent kernel over a queue of tiles (experiment e, neutron range).
// Each workgroup pops a tile, traces it into an LDS histogram of the
// experiment's detector (the experiment's size table is read from global
// memory, through the caches: the histogram takes the LDS) and adds the
// histogram to the detector.  The model is uniform per tile, so the
// switch on it is a scalar branch; every workgroup leaves the loop when the
// queue is exhausted.
struct BatchTile {
    unsigned e;
    unsigned count;
    unsigned long long first;
};

template <int KIND>
__device__ __forceinline__ void batch_tile(ConstArgs* ap, unsigned long long first, unsigned count,
                                           double* hist, const double* tab)
{
    for (unsigned j = threadIdx.x; j < count; j += blockDim.x) {
        const TraceArgs& a = loop_args(ap);
        const Event ev = trace_neutron<KIND, 0>(a, first + j, tab, a.tab_norm, nullptr);
        if (ev.pixel >= 0)
            __hip_atomic_fetch_add(hist + ev.pixel, (double)ev.w, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// ------------------------------------------------------------------ surrogate mode
// Rg^2 = (s0^2 + s1^2 + s2^2) / D: D = 12 for the parallelepiped (edges), 5
// for the ellipsoid (semi-axes).
__host__ __device__ constexpr double sur_rg2_scale(int kind) { return kind == kParallelepiped ? 1.0 / 12.0 : 1.0 / 5.0; }

// Inputs of the network for one neutron: ln(q s0), ln(s1/s0), ln(s2/s0), p.
struct SurConst {
    float ls0;            // ln(size[0])
    float x1, x2, x3;     // the constant inputs of this model
    float lo0, hi0;       // domain of ln(q s0)
    float mid0, scale0;   // normalisation of ln(q s0): (x - mid0) * scale0
    float f2_0;           // <F^2>(0)
    float kref;           // Rg^2 / 6 (A^2): P_ref = (1 + q^2 kref)^-2
    // the in-domain judge: bins of ln(q s0) (FP64, from |Q| in FP64) over
    // [jlo, jlo + nbins / jinv); flags[b] sends bin b's neutrons to the exact
    // pass; nbins = 0: no judge
    double ls0d, jlo, jinv;
    int32_t jnb;
    const unsigned char* flags;
};

// Surrogate tracer.  Geometry and S(q) per lane; the network per wave (16
// samples at a time, activations in registers); in-domain neutrons are
// tallied with FP64 global atomics, the others queued for the exact pass.
template <int KIND>
__global__ __launch_bounds__(sur::kSurBlock) void k_trace_sur(const TraceArgs a, const mlp::bf16x8* __restrict__ pk,
                                                              const __bf16* __restrict__ wts, const SurConst sc,
                                                              double* det, unsigned long long* queue,
                                                              unsigned* qcount)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char sur_lds[];
    mlp::bf16x8* wl = (mlp::bf16x8*)sur_lds;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* xs = (float*)(sur_lds + sur::kSurLdsWeights) + wave * 64 * mlp::kIn;
    const __amdgpu_buffer_rsrc_t rw = sur::make_rsrc(wts, (int)(2 * sur::kWeightsPadded));
    const uint64_t stride = (uint64_t)gridDim.x * sur::kSurBlock;
    // the loop bound is the workgroup's, so that every wave reaches the
    // barriers of the staged layers together
    for (uint64_t j0 = (uint64_t)blockIdx.x * sur::kSurBlock; j0 < a.n; j0 += stride) {
        const uint64_t j = j0 + threadIdx.x;
        const bool valid = j < a.n;
        Event ev{-1, 0.0f, 0.0f, 0.0f};
        if (valid) ev = trace_neutron<KIND, 2>(loop_args(kernel_args()), a.first + j, nullptr, nullptr, nullptr);
        const float x0 = __logf(ev.q) + sc.ls0;
        // the domain and the judge's bin from ln(q s0) in FP64
        const double x0d = valid && ev.q > 0.0f ? log((double)ev.q + (double)ev.qlo) + sc.ls0d : -1e300;
        bool in_dom = valid && ev.pixel >= 0 && x0d >= (double)sc.lo0 && x0d <= (double)sc.hi0;
        if (in_dom && sc.jnb > 0) {
            const int b = (int)fmin(fmax(floor((x0d - sc.jlo) * sc.jinv), 0.0), (double)(sc.jnb - 1));
            in_dom = sc.flags[b] == 0;
        }
        float* xr = xs + lane * mlp::kIn;
        xr[0] = (fminf(fmaxf(x0, sc.lo0), sc.hi0) - sc.mid0) * sc.scale0;
        xr[1] = sc.x1;
        xr[2] = sc.x2;
        xr[3] = sc.x3;
        xr[4] = xr[5] = xr[6] = xr[7] = 0.0f;
        float y = 0.0f;
#pragma unroll 1
        for (int c = 0; c < 4; c += 2) {
            asm volatile("" ::: "memory");
            float yc[2];
            sur::forward32_lds(pk, wl, rw, xs, c, yc);
            if ((lane >> 4) == c) y = yc[0];
            if ((lane >> 4) == c + 1) y = yc[1];
        }
        if (in_dom) {
            const float t = __builtin_fmaf(ev.q * ev.q, sc.kref, 1.0f);
            const double w = (double)(ev.w * sc.f2_0 * __expf(y) * rcpf(t * t));
            __hip_atomic_fetch_add(det + ev.pixel, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (valid && ev.pixel >= 0) {
            const unsigned slot = atomicAdd(qcount, 1u);
            queue[slot] = a.first + j;
        }
        __syncthreads();   // the inputs of this round are read before the next round writes them
    }
}

// Exact (quadrature) pass over the queued neutrons: one wave per neutron,
// its 64 lanes share the quadrature nodes and add their partial weights (the
// queue holds few neutrons, each costing thousands of node evaluations).
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_trace_queue(const TraceArgs a, LdsLayout lay,
                                                        const unsigned long long* queue, const unsigned* qcount,
                                                        double* det)
{
    extern __shared__ double lds_d[];
    const LdsPtrs lp = stage_all(a, lay, lds_d);
    __syncthreads();
    const unsigned nq = *qcount;
    const int lane = threadIdx.x & 63;
    const unsigned waves = gridDim.x * (blockDim.x / 64);
    for (unsigned i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); i < nq; i += waves) {
        const Event ev = trace_neutron<KIND, 1>(loop_args(kernel_args()), queue[i], lp.tsize, lp.tnorm, lp.lq,
                                                lane, 64);
        float w = ev.w;
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
        if (lane == 0 && ev.pixel >= 0)
            __hip_atomic_fetch_add(det + ev.pixel, (double)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Training targets: for inputs x = (ln(q s0), ln(s1/s0), ln(s2/s0), p, ...)
// the exact ln(<F^2>(q) / <F^2>(0)) of an isotropically oriented particle
// with sizes s0 (1, e^x1, e^x2), Schulz width p on all sizes.  Orientation
// nodes in LDS as in quad_average; size nodes per sample from gx, gw.
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_pq_dataset(const TraceArgs a, const float* __restrict__ x,
                                                       int64_t n, float* __restrict__ out,
                                                       const float* __restrict__ nodes, int nq, int dims,
                                                       const double* __restrict__ gl_x,
                                                       const double* __restrict__ gl_w)
{
    __shared__ float lq[5 * kMaxQuad];
    for (int i = threadIdx.x; i < 5 * nq; i += blockDim.x) lq[i] = nodes[i];
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float* xi = x + idx * mlp::kIn;
    const float q = __expf(xi[0]);
    const float s1 = __expf(xi[1]), s2 = __expf(xi[2]);
    const double pw = xi[3];
    const float* mu = lq;
    const float* wmu = lq + nq;
    const float* cb = lq + 2 * nq;
    const float* sb = lq + 3 * nq;
    const float* wb = lq + 4 * nq;
    const int ny = pw > 0.0 ? nq : 1;
    double lo = 1.0, hi = 1.0, aa = 0.0, lnorm = 0.0;
    if (pw > 0.0) {
        lo = fmax(0.0, 1.0 - 6.0 * pw);
        hi = 1.0 + 8.0 * pw;
        aa = 1.0 / (pw * pw);
        lnorm = aa * log(aa) - lgamma(aa);
    }
    double num = 0.0, den = 0.0, wsum = 0.0;
    for (int j = 0; j < ny; ++j) {
        double y = 1.0, wy = 1.0;
        if (pw > 0.0) {
            y = lo + 0.5 * (hi - lo) * (gl_x[j] + 1.0);
            wy = y > 0.0 ? gl_w[j] * exp(lnorm + (aa - 1.0) * log(y) - aa * y) : 0.0;
        }
        const float s[3] = {(float)y, (float)(s1 * y), (float)(s2 * y)};
        float avg = 0.0f;
        if (dims == 1) {
            for (int i = 0; i < nq; ++i) {
                const float m = mu[i];
                const float st = sqrtf(fmaxf(1.0f - m * m, 0.0f));
                const float f = amplitude_f<KIND>(a, s, q, q * st, 0.0f, q * m, (float)y);
                avg = __builtin_fmaf(wmu[i], f * f, avg);
            }
        } else {
            for (int i = 0; i < nq; ++i) {
                const float m = mu[i];
                const float qst = q * sqrtf(fmaxf(1.0f - m * m, 0.0f));
                const float qc = q * m;
                float inner = 0.0f;
                for (int l = 0; l < nq; ++l) {
                    const float f = amplitude_f<KIND>(a, s, q, qst * cb[l], qst * sb[l], qc, (float)y);
                    inner = __builtin_fmaf(wb[l], f * f, inner);
                }
                avg = __builtin_fmaf(wmu[i], inner, avg);
            }
        }
        const float f0 = amplitude_f<KIND>(a, s, 0.0f, 0.0f, 0.0f, 0.0f, (float)y);
        num += wy * (double)avg;
        den += wy * (double)f0 * (double)f0;
        wsum += wy;
    }
    (void)wsum;
    // the network's target: ln of the normalised average minus ln P_ref,
    // P_ref = (1 + (q Rg)^2 / 6)^-2 with the body's Rg^2 (Guinier at small q,
    // q^-4 at large q), which takes most of the dynamic range off the network
    const double rg2 = (1.0 + exp(2.0 * (double)xi[1]) + exp(2.0 * (double)xi[2])) * sur_rg2_scale(KIND);
    out[idx] = (float)(log(num / den) + 2.0 * log1p(exp(2.0 * (double)xi[0]) * rg2 / 6.0));
}


// ------------------------------------------------------------------ kernel tables
using TraceFn = void (*)(const TraceArgs, LdsLayout, double*, double*, unsigned long long*, double*);
using HistFn = void (*)(const TraceArgs, LdsLayout, double*);
using EmitFn = void (*)(const TraceArgs, LdsLayout, uint2*, unsigned*, unsigned, int, int);
using DebugFn = void (*)(const TraceArgs, LdsLayout, int32_t*, float*, float*);
using PqFn = void (*)(const TraceArgs, LdsLayout, const float*, const float*, int64_t, float*);

// The kernels of one model: [mode] for MC (0) and QUAD (1); trace[mode][0]
// tallies with global atomics, trace[mode][1] into per-XCD replicas.  The
// atomic kernels carry the attenuation; the histogram and binned kernels
// (unattenuated Monte Carlo runs) do not.
struct KindFns {
    TraceFn trace[2][2];
    HistFn hist[3];        // [0] Monte Carlo, [1] exact average, [2] Monte Carlo with attenuation / guide
    EmitFn emit[3];
    DebugFn debug[2][2];   // [mode][attenuation compiled in]
    PqFn pq;
};

template <int K>
void fill_kind(KindFns* t)
{
    KindFns& f = t[K];
    f.trace[0][0] = k_trace<K, 0, SANS_TALLY_GLOBAL>;
    f.trace[0][1] = k_trace<K, 0, SANS_TALLY_XCD>;
    f.trace[1][0] = k_trace<K, 1, SANS_TALLY_GLOBAL>;
    f.trace[1][1] = k_trace<K, 1, SANS_TALLY_XCD>;
    f.hist[0] = k_trace_hist<K, 0>;
    f.hist[1] = k_trace_hist<K, 1>;
    f.hist[2] = k_trace_hist<K, 0, true>;
    f.emit[0] = k_emit<K, 0>;
    f.emit[1] = k_emit<K, 1>;
    f.emit[2] = k_emit<K, 0, true>;
    // the per-neutron kernel compiles the same instance of the neutron code as
    // the kernels that tally: the attenuation only where those carry it
    f.debug[0][0] = k_debug<K, 0, false>;
    f.debug[0][1] = k_debug<K, 0, true>;
    f.debug[1][0] = k_debug<K, 1, true>;
    f.debug[1][1] = k_debug<K, 1, true>;
    f.pq = k_pq_avg<K>;
}

// Fill t[K] for the kinds K of group g (K % kKindGroups == g); one per
// translation unit of sans_kinds.hip.
void fill_kinds_0(KindFns* t);
void fill_kinds_1(KindFns* t);
void fill_kinds_2(KindFns* t);
void fill_kinds_3(KindFns* t);
void fill_kinds_4(KindFns* t);
void fill_kinds_5(KindFns* t);
void fill_kinds_6(KindFns* t);
void fill_kinds_7(KindFns* t);

// The persistent batched kernel (sans_batch.hip).
using BatchFn = void (*)(const TraceArgs*, const BatchTile*, int, unsigned*, double*, int, int);
BatchFn batch_kernel();

// Surrogate-mode kernels of the networks' models (sans_sur.hip).
using SurFn = void (*)(const TraceArgs, const mlp::bf16x8*, const __bf16*, const SurConst, double*,
                       unsigned long long*, unsigned*);
using QueueFn = void (*)(const TraceArgs, LdsLayout, const unsigned long long*, const unsigned*, double*);
using DatasetFn = void (*)(const TraceArgs, const float*, int64_t, float*, const float*, int, int,
                           const double*, const double*);
SurFn sur_kernel(int kind);
QueueFn sur_queue_kernel(int kind);
DatasetFn dataset_kernel(int kind);

}  // namespace sans
