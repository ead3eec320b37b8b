// sans_mlp.hip -- C ABI of the surrogate network's training kernels: forward
// (activations kept for the backward pass), backward (all parameter
// gradients), Adam and the mean-squared-error gradient.  Every product is a
// hand-written BF16 MFMA GEMM (k_gemm) with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/sans.h"
#include "sans_mlp.hpp"

using namespace sans::mlp;

namespace {

thread_local std::string g_mlp_error;

int mfail(int status, const std::string& msg)
{
    g_mlp_error = msg;
    return status;
}

template <bool AT, bool BT, typename TA, typename TB, int EPI, bool SPLIT = false>
int gemm(int M, int N, int K, const TA* A, int lda, const TB* B, int ldb, float* C, int ldc,
         const TB* bias, float* aux, hipStream_t s)
{
    // split-K for the atomic epilogue: about 512 workgroups, >= 256 of K each
    unsigned splits = 1;
    if (EPI == kEpiAtomic) {
        const unsigned tiles = (unsigned)(((N + kTN - 1) / kTN) * ((M + kTM - 1) / kTM));
        splits = std::max(1u, std::min((unsigned)(K / 256), 512u / std::max(1u, tiles)));
    }
    const dim3 grid((unsigned)((N + kTN - 1) / kTN), (unsigned)((M + kTM - 1) / kTM), splits);
    hipLaunchKernelGGL((k_gemm<AT, BT, TA, TB, EPI, SPLIT>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, bias, aux);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(SANS_E_HIP, std::string("gemm: ") + hipGetErrorString(e));
    return SANS_OK;
}

int colsum(const float* X, int M, int N, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((N + 255) / 256), (unsigned)((M + 255) / 256)), dim3(256), 0, s,
                       X, M, N, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(SANS_E_HIP, std::string("colsum: ") + hipGetErrorString(e));
    return SANS_OK;
}

// workspace: Z[4][n][256], H[4][n][256], two gradient buffers [n][256]
float* ws_z(float* ws, int64_t n, int l) { return ws + (int64_t)l * n * kHid; }
float* ws_h(float* ws, int64_t n, int l) { return ws + (int64_t)(4 + l) * n * kHid; }
float* ws_g(float* ws, int64_t n, int i) { return ws + (int64_t)(8 + i) * n * kHid; }

}  // namespace

extern "C" {

const char* sans_mlp_last_error(void) { return g_mlp_error.c_str(); }

uint64_t sans_mlp_workspace_bytes(int64_t n) { return (uint64_t)(10 * n * kHid) * sizeof(float); }

int64_t sans_mlp_param_count(void) { return kParams; }

int sans_mlp_forward(const void* w_bf16, const float* x, int64_t n, float* y, void* ws, void* stream)
{
    if (!w_bf16 || !x || !y || !ws) return mfail(SANS_E_INVALID_ARG, "mlp forward: NULL argument");
    if (n < 0 || n > (1 << 24)) return mfail(SANS_E_INVALID_ARG, "mlp forward: n out of range");
    if (n == 0) return SANS_OK;
    hipStream_t s = (hipStream_t)stream;
    const __bf16* w = (const __bf16*)w_bf16;
    float* W = (float*)ws;
    const int N = (int)n;
    int rc;
    // Z0 = (hi(X) + lo(X)) W0 + b0, H0 = silu(Z0)
    if ((rc = gemm<false, false, float, __bf16, kEpiBiasSilu, true>(N, kHid, 2 * kIn, x, kIn, w + offW(0), kHid,
                                                               ws_z(W, n, 0), kHid, w + offB(0),
                                                               ws_h(W, n, 0), s)))
        return rc;
    // Z_l = H_{l-1} W_l + b_l, H_l = silu(Z_l)
    for (int l = 1; l < kLayers; ++l)
        if ((rc = gemm<false, false, float, __bf16, kEpiBiasSilu>(N, kHid, kHid, ws_h(W, n, l - 1), kHid,
                                                                   w + offW(l), kHid, ws_z(W, n, l), kHid,
                                                                   w + offB(l), ws_h(W, n, l), s)))
            return rc;
    // y = H3 W4 + b4 (FP32 activations)
    hipLaunchKernelGGL(k_output, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, ws_h(W, n, 3), w + kOffW4,
                       w + kOffB4, N, y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(SANS_E_HIP, std::string("output layer: ") + hipGetErrorString(e));
    return SANS_OK;
}

int sans_mlp_backward(const void* w_bf16, const float* x, const float* dy, int64_t n, float* dw, void* ws,
                      void* stream)
{
    if (!w_bf16 || !x || !dy || !dw || !ws) return mfail(SANS_E_INVALID_ARG, "mlp backward: NULL argument");
    if (n < 1 || n > (1 << 24)) return mfail(SANS_E_INVALID_ARG, "mlp backward: n out of range");
    hipStream_t s = (hipStream_t)stream;
    const __bf16* w = (const __bf16*)w_bf16;
    float* W = (float*)ws;
    const int N = (int)n;
    int rc;
    // every gradient is accumulated (split-K and column-sum atomics)
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, s, dw, kParams);
    // output layer: dW4 = H3^T dy, db4 = sum dy
    if ((rc = gemm<true, false, float, float, kEpiAtomic>(kHid, 1, N, ws_h(W, n, 3), kHid, dy, 1,
                                                          dw + kOffW4, 1, nullptr, nullptr, s)))
        return rc;
    if ((rc = colsum(dy, N, 1, dw + kOffB4, s))) return rc;
    // dZ3 = (dy W4^T) . silu'(Z3)
    float* g = ws_g(W, n, 0);
    if ((rc = gemm<false, false, float, __bf16, kEpiSiluGrad>(N, kHid, 1, dy, 1, w + kOffW4, kHid, g, kHid,
                                                               nullptr, ws_z(W, n, 3), s)))
        return rc;
    for (int l = kLayers - 1; l >= 0; --l) {
        const float* hin = l == 0 ? x : ws_h(W, n, l - 1);
        const int kin = l == 0 ? kIn : kHid;
        // dW_l = H_{l-1}^T dZ_l, db_l = colsum(dZ_l)
        if ((rc = gemm<true, false, float, float, kEpiAtomic>(kin, kHid, N, hin, kin, g, kHid, dw + offW(l),
                                                              kHid, nullptr, nullptr, s)))
            return rc;
        if ((rc = colsum(g, N, kHid, dw + offB(l), s))) return rc;
        if (l == 0) break;
        // dZ_{l-1} = (dZ_l W_l^T) . silu'(Z_{l-1})
        float* gn = ws_g(W, n, (kLayers - l) & 1);
        if ((rc = gemm<false, true, float, __bf16, kEpiSiluGrad>(N, kHid, kHid, g, kHid, w + offW(l), kHid,
                                                                  gn, kHid, nullptr, ws_z(W, n, l - 1), s)))
            return rc;
        g = gn;
    }
    return SANS_OK;
}

int sans_adam_step(float* w32, void* w_bf16, const float* dw, float* m, float* v, int64_t n, float lr,
                   float beta1, float beta2, float eps, int step, void* stream)
{
    if (!w32 || !w_bf16 || !dw || !m || !v) return mfail(SANS_E_INVALID_ARG, "adam: NULL argument");
    if (n < 0 || step < 1) return mfail(SANS_E_INVALID_ARG, "adam: n < 0 or step < 1");
    if (n == 0) return SANS_OK;
    const float c1 = 1.0f / (1.0f - powf(beta1, (float)step));
    const float c2 = 1.0f / (1.0f - powf(beta2, (float)step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w32,
                       (__bf16*)w_bf16, dw, m, v, n, lr, beta1, beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(SANS_E_HIP, std::string("adam: ") + hipGetErrorString(e));
    return SANS_OK;
}

int sans_mse_grad(const float* y, const float* t, int64_t n, float* dy, float* loss, void* stream)
{
    if (!y || !t || !dy) return mfail(SANS_E_INVALID_ARG, "mse: NULL argument");
    if (n < 1) return mfail(SANS_E_INVALID_ARG, "mse: n < 1");
    hipLaunchKernelGGL(k_mse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, y, t, n,
                       dy, loss);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(SANS_E_HIP, std::string("mse: ") + hipGetErrorString(e));
    return SANS_OK;
}

int sans_f32_to_bf16(const float* x, void* y, int64_t n, void* stream)
{
    if (!x || !y || n < 0) return mfail(SANS_E_INVALID_ARG, "f32_to_bf16: bad argument");
    if (n == 0) return SANS_OK;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, x,
                       (__bf16*)y, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mfail(SANS_E_HIP, std::string("f32_to_bf16: ") + hipGetErrorString(e));
    return SANS_OK;
}

}  // extern "C"
