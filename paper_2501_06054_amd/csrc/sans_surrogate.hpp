// sans_surrogate.hpp -- the surrogate network inside the tracer (gfx950).
//
// Every wave evaluates the network for its own 64 neutrons, 32 at a time
// (two column groups of 16 sharing each weight fragment), with the
// activations held in registers from layer to layer and the fragments staged
// in LDS once per workgroup and layer (forward32_lds):
//   D[16 features][16 samples] += A[16 features][32 inputs] * B[32 inputs][16 samples]
// (v_mfma_f32_16x16x32_bf16).  Lane (g = lane/16, r = lane%16) holds, for
// output tile t, the features 16t + 4g + i (i = 0..3) of sample r.  The
// reduction index of the next layer is ordered so that those values are
// exactly the B operand the lane needs: K-step s, element j maps to input
// 32s + (j < 4 ? 4g + j : 16 + 4g + j - 4) -- the outputs of tiles 2s and
// 2s+1 of the lane itself.  The weights are pre-packed (k_pack_surrogate)
// as A fragments in that order, 16 bytes per lane per (tile, K-step), 390 KiB
// in global memory (L2-resident), one layer of which the LDS holds at a time.
#pragma once

#include "sans_device.hpp"
#include "sans_mlp.hpp"

namespace sans {
namespace sur {

using mlp::bf16x8;
using mlp::f32x4;
using mlp::kHid;
using mlp::kIn;

constexpr int kTiles = kHid / 16;   // 16 output tiles per hidden layer
constexpr int kSteps = kHid / 32;   // 8 K-steps per hidden layer
// packed layout (bf16x8 units): layer 0: [tile][lane]; layers 1..3: [tile][step][lane]
constexpr int64_t kPack0 = (int64_t)kTiles * 64;
constexpr int64_t kPackL = (int64_t)kTiles * kSteps * 64;
constexpr int64_t kPackTotal = kPack0 + 3 * kPackL;
// The flat BF16 parameters as the tracer holds them: padded with zeros to a
// multiple of 8 elements, so that the 8-byte loads of the last parameters
// (b4 is element 199,936) lie wholly inside the buffer resource.
constexpr int64_t kWeightsPadded = (mlp::kParams + 7) / 8 * 8;

__host__ __device__ constexpr int perm_k(int g, int j) { return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4); }

// Packs the flat BF16 parameters into A fragments.  One thread per
// (layer, tile, step, lane).
static __global__ void k_pack_surrogate(const __bf16* __restrict__ w, bf16x8* __restrict__ out)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= kPackTotal) return;
    const int lane = (int)(id % 64);
    const int g = lane >> 4, r = lane & 15;
    bf16x8 v;
    if (id < kPack0) {
        const int t = (int)(id / 64);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = perm_k(g, j);
            // K rows 0..7: W0 for the hi parts of the inputs, 8..15: W0 again for the lo parts
            v[j] = k < 2 * kIn ? w[mlp::offW(0) + (int64_t)(k % kIn) * kHid + 16 * t + r] : (__bf16)0.0f;
        }
    } else {
        const int64_t rem = id - kPack0;
        const int l = 1 + (int)(rem / kPackL);
        const int64_t q = rem % kPackL;
        const int t = (int)(q / (kSteps * 64));
        const int s = (int)((q / 64) % kSteps);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 32 * s + perm_k(g, j);
            v[j] = w[mlp::offW(l) + (int64_t)k * kHid + 16 * t + r];
        }
    }
    out[id] = v;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

// A buffer resource (base, size) for the flat parameters: loads then take
// one lane offset in a VGPR and the element offset in an SGPR, instead of a
// 64-bit address each; reads past the end return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
}

// four consecutive BF16 parameters starting at element e0 + 4g, as floats
__device__ __forceinline__ void load4(__amdgpu_buffer_rsrc_t r, int g, int64_t e0, float v[4])
{
    const i32x2 raw = __builtin_amdgcn_raw_buffer_load_b64(r, 8 * g, (int)(2 * e0), 0);
    const uint32_t lo = (uint32_t)raw[0], hi = (uint32_t)raw[1];
    v[0] = __uint_as_float(lo << 16);
    v[1] = __uint_as_float(lo & 0xFFFF0000u);
    v[2] = __uint_as_float(hi << 16);
    v[3] = __uint_as_float(hi & 0xFFFF0000u);
}

// Orders the evaluation: the value is complete (in registers) at this point of
// the instruction stream, so that the scheduler does not keep dozens of
// independent accumulators live by running ahead.
__device__ __forceinline__ void settle(bf16x8& v) { asm volatile("" : "+v"(v)); }

// The four biases of load4 as an MFMA accumulator: the tracer's layers start
// their sums from the biases (one addition fewer per feature than adding
// them to the finished sum).
__device__ __forceinline__ f32x4 load4v(__amdgpu_buffer_rsrc_t r, int g, int64_t e0)
{
    float v[4];
    load4(r, g, e0, v);
    return f32x4{v[0], v[1], v[2], v[3]};
}

// SiLU of an accumulator tile that already holds the bias, converted to one
// half of the next B operand.
__device__ __forceinline__ void silu_to_bf16(const f32x4& acc, bf16x8& dst, int half)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[4 * half + i] = (__bf16)mlp::silu(acc[i]);
}

// The same network with the weights staged in LDS, one layer at a time, for a
// whole workgroup: kSurBlock lanes (kSurWaves waves) trace their neutrons,
// then every wave evaluates its 64 samples in two passes of 32 (column groups
// c0, c0 + 1) with each layer's fragments read from LDS.  One copy of
// a layer from L2 serves kSurWaves x 32 samples, instead of 32 when every
// wave reads the fragments itself.
constexpr int kSurBlock = 512;
constexpr int kSurWaves = kSurBlock / 64;
// LDS: the largest layer's fragments (a hidden layer, 128 KiB), then the
// waves' inputs [kSurWaves][64][kIn] floats
constexpr size_t kSurLdsWeights = 16 * (size_t)kPackL;
constexpr size_t kSurLdsBytes = kSurLdsWeights + sizeof(float) * kSurBlock * kIn;

// Copies n 16-byte fragments from global memory to LDS with the whole
// workgroup, between two barriers (the previous layer's fragments are no
// longer read; the new ones are all in place).
__device__ __forceinline__ void stage_layer(bf16x8* __restrict__ dst, const bf16x8* __restrict__ src, int n)
{
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kSurBlock) dst[i] = src[i];
    __syncthreads();
}

// Network outputs for the 32 samples of column groups c0 and c0 + 1 of this
// wave (samples 16 c0 + r and 16 (c0 + 1) + r), with the fragments in LDS
// (wl, staged here layer by layer from pk); every wave of the workgroup must
// call it together.  Every fragment read is applied to both groups.  xs:
// this wave's inputs in LDS, [64][8] floats.  Returns, in every lane (g, r),
// y[0] for sample 16 c0 + r and y[1] for sample 16 (c0 + 1) + r.
__device__ __forceinline__ void forward32_lds(const bf16x8* __restrict__ pk, bf16x8* __restrict__ wl,
                                              __amdgpu_buffer_rsrc_t rw, const float* xs, int c0, float y[2])
{
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    // layer 0's fragments; the barriers also publish the inputs xs
    stage_layer(wl, pk, (int)kPack0);
    bf16x8 b0[2];
#pragma unroll
    for (int gi = 0; gi < 2; ++gi)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = perm_k(g, j);
            const float xv = k < 2 * kIn ? xs[(16 * (c0 + gi) + r) * kIn + (k % kIn)] : 0.0f;
            b0[gi][j] = k < kIn ? mlp::bf16_hi(xv) : k < 2 * kIn ? mlp::bf16_lo(xv) : (__bf16)0.0f;
        }
    bf16x8 act[2][kSteps];
#pragma unroll
    for (int t = 0; t < kTiles; t += 2) {
        const bf16x8 fa = wl[t * 64 + lane], fb = wl[(t + 1) * 64 + lane];
        const f32x4 ba = load4v(rw, g, mlp::offB(0) + 16 * t), bb = load4v(rw, g, mlp::offB(0) + 16 * (t + 1));
#pragma unroll
        for (int gi = 0; gi < 2; ++gi) {
            const f32x4 a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, b0[gi], ba, 0, 0, 0);
            const f32x4 a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb, b0[gi], bb, 0, 0, 0);
            silu_to_bf16(a0, act[gi][t / 2], 0);
            silu_to_bf16(a1, act[gi][t / 2], 1);
            settle(act[gi][t / 2]);
        }
    }
    // hidden layers 1..2
#pragma unroll 1
    for (int l = 1; l < 3; ++l) {
        stage_layer(wl, pk + kPack0 + (int64_t)(l - 1) * kPackL, (int)kPackL);
        bf16x8 nxt[2][kSteps];
#pragma unroll
        for (int t = 0; t < kTiles; t += 2) {
            asm volatile("" ::: "memory");
            // the accumulators start from the biases
            const f32x4 ba = load4v(rw, g, mlp::offB(l) + 16 * t), bb = load4v(rw, g, mlp::offB(l) + 16 * (t + 1));
            f32x4 acc[2][2];
#pragma unroll
            for (int gi = 0; gi < 2; ++gi) {
                acc[gi][0] = ba;
                acc[gi][1] = bb;
            }
#pragma unroll
            for (int s = 0; s < kSteps; ++s) {
                const bf16x8 fa = wl[(t * kSteps + s) * 64 + lane];
                const bf16x8 fb = wl[((t + 1) * kSteps + s) * 64 + lane];
#pragma unroll
                for (int gi = 0; gi < 2; ++gi) {
                    acc[gi][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, act[gi][s], acc[gi][0], 0, 0, 0);
                    acc[gi][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb, act[gi][s], acc[gi][1], 0, 0, 0);
                }
            }
#pragma unroll
            for (int gi = 0; gi < 2; ++gi) {
                silu_to_bf16(acc[gi][0], nxt[gi][t / 2], 0);
                silu_to_bf16(acc[gi][1], nxt[gi][t / 2], 1);
                settle(nxt[gi][t / 2]);
            }
        }
#pragma unroll
        for (int gi = 0; gi < 2; ++gi)
#pragma unroll
            for (int s = 0; s < kSteps; ++s) act[gi][s] = nxt[gi][s];
    }
    // hidden layer 3 and the output layer
    stage_layer(wl, pk + kPack0 + 2 * kPackL, (int)kPackL);
    y[0] = y[1] = 0.0f;
#pragma unroll
    for (int t = 0; t < kTiles; ++t) {
        asm volatile("" ::: "memory");
        const f32x4 b = load4v(rw, g, mlp::offB(3) + 16 * t);
        f32x4 acc[2] = {b, b};
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            const bf16x8 f = wl[(t * kSteps + s) * 64 + lane];
#pragma unroll
            for (int gi = 0; gi < 2; ++gi)
                acc[gi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f, act[gi][s], acc[gi], 0, 0, 0);
        }
        float w4[4];
        load4(rw, g, mlp::kOffW4 + 16 * t, w4);
#pragma unroll
        for (int gi = 0; gi < 2; ++gi)
#pragma unroll
            for (int i = 0; i < 4; ++i) y[gi] = __builtin_fmaf(mlp::silu(acc[gi][i]), w4[i], y[gi]);
        asm volatile("" : "+v"(y[0]), "+v"(y[1]));
    }
    float b4[4];
    load4(rw, 0, mlp::kOffB4, b4);
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
        y[gi] += __shfl_xor(y[gi], 16);
        y[gi] += __shfl_xor(y[gi], 32);
        y[gi] += b4[0];
    }
}

}  // namespace sur
}  // namespace sans
