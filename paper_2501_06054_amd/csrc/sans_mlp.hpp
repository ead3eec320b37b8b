// sans_mlp.hpp -- the surrogate network and its BF16 MFMA kernels (gfx950).
//
// Network: 8 inputs -> 4 hidden layers of 256 SiLU units -> 1 output (the
// logarithm of the normalised orientation/size-averaged form factor).
// Parameters, flat FP32 (master) or BF16 (kernel operand), in this order:
//   W0[8][256] b0[256] W1[256][256] b1[256] W2[256][256] b2[256]
//   W3[256][256] b3[256] W4[256] b4[1]                (199,937 values)
// W_l is stored [in][out] row-major.  Matrix products use
// v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation.  The inputs of
// the first layer enter as two BF16 parts, hi = bf16(x) and lo = bf16(x -
// hi), both multiplied by W0 (16 bits of input precision instead of 8); the
// output layer takes the last hidden activations in FP32 (a dot product
// with the BF16 W4, FP32 arithmetic).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sans {
namespace mlp {

constexpr int kIn = 8;
constexpr int kHid = 256;
constexpr int kLayers = 4;  // hidden layers
constexpr int64_t kOffW0 = 0;
constexpr int64_t kOffB0 = kOffW0 + kIn * kHid;
constexpr int64_t kOffW1 = kOffB0 + kHid;
constexpr int64_t kLayerStride = (int64_t)kHid * kHid + kHid;  // W_l + b_l for l >= 1
constexpr int64_t offW(int l) { return l == 0 ? kOffW0 : kOffW1 + (l - 1) * kLayerStride; }
constexpr int64_t offB(int l) { return l == 0 ? kOffB0 : offW(l) + (int64_t)kHid * kHid; }
constexpr int64_t kOffW4 = kOffW1 + 3 * kLayerStride;
constexpr int64_t kOffB4 = kOffW4 + kHid;
constexpr int64_t kParams = kOffB4 + 1;
static_assert(kParams == 199937, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z)
{
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

template <typename T>
__device__ __forceinline__ float to_f(T v) { return (float)v; }

// ---------------------------------------------------------------- tiled GEMM
// C[M][N] = op(A)[M][K] * op(B)[K][N] with BF16 operands (converted on load)
// and FP32 accumulation.  A(m,k) = A_T ? A[k*lda + m] : A[m*lda + k];
// B(k,n) = B_T ? B[n*ldb + k] : B[k*ldb + n].  Tile 64x64x32 per workgroup
// of 4 waves; each wave owns a 32x32 block = 2x2 MFMA 16x16 tiles.
// Epilogues:
enum : int {
    kEpiStore = 0,      // C = acc
    kEpiBiasSilu = 1,   // Z = acc + bias[n] -> C (pre-activation), H = silu(Z) -> aux
    kEpiBias = 2,       // C = acc + bias[n]
    kEpiSiluGrad = 3,   // C = acc * silu'(aux[m][n])  (aux = pre-activation)
    kEpiAtomic = 4,     // C += acc (FP32 atomics; split-K over blockIdx.z)
};

constexpr int kTM = 64, kTN = 64, kTK = 32;

// The two BF16 parts of an FP32 value.
__device__ __forceinline__ __bf16 bf16_hi(float x) { return (__bf16)x; }
__device__ __forceinline__ __bf16 bf16_lo(float x) { return (__bf16)(x - (float)(__bf16)x); }

// SPLIT (first layer, A = X not transposed): K = 2 * lda; A(m, k) is the hi
// part of X[m][k] for k < lda and the lo part of X[m][k - lda] above, and
// B(k, n) = B[k mod lda][n].
template <bool A_T, bool B_T, typename TA, typename TB, int EPI, bool SPLIT = false>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA* __restrict__ A, int lda,
                                              const TB* __restrict__ B, int ldb, float* __restrict__ C,
                                              int ldc, const TB* __restrict__ bias,
                                              float* __restrict__ aux)
{
    // LDS tiles as BF16, both K-contiguous: As[m][k], Bs[n][k] (+8 padding per row)
    __shared__ __bf16 As[kTM][kTK + 8];
    __shared__ __bf16 Bs[kTN][kTK + 8];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int r = lane & 15, g = lane >> 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // split-K (kEpiAtomic): workgroup z takes K range [z*ks, (z+1)*ks)
    int kbeg = 0, kend = K;
    if constexpr (EPI == kEpiAtomic) {
        const int ks = ((K + gridDim.z - 1) / gridDim.z + kTK - 1) / kTK * kTK;
        kbeg = blockIdx.z * ks;
        kend = min(K, kbeg + ks);
    }
    for (int k0 = kbeg; k0 < kend; k0 += kTK) {
        // each thread stages 8 elements of A and 8 of B
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid * 8 + e;         // 0 .. 2047
            int mm, kk;
            if (A_T) { kk = idx / kTM; mm = idx % kTM; } else { mm = idx / kTK; kk = idx % kTK; }
            const int gm = m0 + mm, gk = k0 + kk;
            if constexpr (SPLIT) {
                __bf16 v = (__bf16)0.0f;
                if (gm < M && gk < kend) {
                    const float x = to_f(A[(int64_t)gm * lda + (gk < lda ? gk : gk - lda)]);
                    v = gk < lda ? bf16_hi(x) : bf16_lo(x);
                }
                As[mm][kk] = v;
            } else {
                float v = 0.0f;
                if (gm < M && gk < kend) v = to_f(A_T ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]);
                As[mm][kk] = (__bf16)v;
            }
            int nn, kb;
            if (B_T) { nn = idx / kTK; kb = idx % kTK; } else { kb = idx / kTN; nn = idx % kTN; }
            const int gn = n0 + nn, gkb = k0 + kb;
            float u = 0.0f;
            const int bk = SPLIT && gkb >= K / 2 ? gkb - K / 2 : gkb;
            if (gn < N && gkb < kend) u = to_f(B_T ? B[(int64_t)gn * ldb + bk] : B[(int64_t)bk * ldb + gn]);
            Bs[nn][kb] = (__bf16)u;
        }
        __syncthreads();
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                af[i][j] = As[wm + 16 * i + r][8 * g + j];
                bfr[i][j] = Bs[wn + 16 * i + r][8 * g + j];
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D[4g + q][r] of each 16x16 tile: row m = tile row + 4g + q, column n = tile col + r
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + 4 * g + q;
                const int n = n0 + wn + 16 * j + r;
                if (m >= M || n >= N) continue;
                const float v = acc[i][j][q];
                const int64_t o = (int64_t)m * ldc + n;
                if constexpr (EPI == kEpiStore) {
                    C[o] = v;
                } else if constexpr (EPI == kEpiAtomic) {
                    __hip_atomic_fetch_add(C + o, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else if constexpr (EPI == kEpiBias) {
                    C[o] = v + to_f(bias[n]);
                } else if constexpr (EPI == kEpiBiasSilu) {
                    const float z = v + to_f(bias[n]);
                    C[o] = z;
                    aux[o] = silu(z);
                } else {
                    C[o] = v * silu_grad(aux[o]);
                }
            }
}

// Output layer: y[m] = sum_k H[m][k] W4[k] + b4 with FP32 activations; one
// wave per row, four features per lane.
static __global__ void k_output(const float* __restrict__ H, const __bf16* __restrict__ w4,
                                const __bf16* __restrict__ b4, int M, float* __restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int m = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (m >= M) return;
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kHid / 64; ++i) {
        const int k = i * 64 + lane;
        s = __builtin_fmaf(H[(int64_t)m * kHid + k], (float)w4[k], s);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) y[m] = s + (float)b4[0];
}

// Column sums: out[n] += sum_m X[m][n] (bias gradients); workgroup (x, y)
// sums rows [256 y, 256 y + 256) of columns [256 x, 256 x + 256) and adds
// the result atomically (out cleared beforehand).
static __global__ void k_colsum(const float* __restrict__ X, int M, int N, float* __restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int m0 = blockIdx.y * 256, m1 = min(M, m0 + 256);
    float s = 0.0f;
    for (int m = m0; m < m1; ++m) s += X[(int64_t)m * N + n];
    __hip_atomic_fetch_add(out + n, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static __global__ void k_zero_f32(float* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Adam (Kingma & Ba, 2015) on the FP32 master weights; writes the BF16 copy.
static __global__ void k_adam(float* __restrict__ w, __bf16* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    wb[i] = (__bf16)wi;
}

// Mean-squared-error gradient: dy = 2 (y - t) / n, loss += sum (y - t)^2 / n.
static __global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                      float* __restrict__ dy, float* __restrict__ loss)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.0f;
    if (i < n) {
        const float d = y[i] - t[i];
        dy[i] = 2.0f * d / (float)n;
        e = d * d / (float)n;
    }
    // wave reduction, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, e);
}

static __global__ void k_f32_to_bf16(const float* __restrict__ x, __bf16* __restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (__bf16)x[i];
}

}  // namespace mlp
}  // namespace sans
