// gfx950 kernels of the warm-start network: a fully connected tanh MLP whose
// matrix products run on MFMA (bf16 operands with FP32 accumulation, or FP32
// operands for checking), plus its loss, bias gradients and Adam update.
//
// Every product is one wave per 16 x 16 output tile: C = op(A) op(B) with
// A(i, k) = A[i*sai + k*sak] and B(k, j) = B[k*sbk + j*sbj] (strides select
// the transposes), FP32 in memory.  bf16 operands are rounded from FP32 as
// they are loaded (round to nearest even).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tsgls {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
  return (short)(u >> 16);
}

// Epilogues: EPI_NONE C = AB (+ bias), EPI_TANH C = tanh(AB + bias),
// EPI_DTANH C = AB * (1 - H^2) with H the layer output (tanh backward).
enum : int { EPI_NONE = 0, EPI_TANH = 1, EPI_DTANH = 2 };

template <bool BF16, int EPI>
__global__ void __launch_bounds__(64)
k_mlp_gemm(int M, int N, int Kd, const float* __restrict__ A, int64_t sai, int64_t sak,
           const float* __restrict__ B, int64_t sbk, int64_t sbj, const float* __restrict__ bias,
           const float* __restrict__ H, float* __restrict__ C, int64_t ldc) {
  const int lane = threadIdx.x, r = lane & 15, q = lane >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int ia = i0 + r, jb = j0 + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (BF16) {
    // 16x16x16: lane (r, q) holds A(i0 + r, k0 + 4q + e) and B(k0 + 4q + e, j0 + r), e < 4
    for (int k0 = 0; k0 < Kd; k0 += 16) {
      bf16x4 a, b;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + 4 * q + e;
        const float av = (ia < M && k < Kd) ? A[ia * sai + k * sak] : 0.f;
        const float bv = (jb < N && k < Kd) ? B[k * sbk + jb * sbj] : 0.f;
        a[e] = to_bf16(av);
        b[e] = to_bf16(bv);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
  } else {
    // 16x16x4: lane (r, q) holds A(i0 + r, k0 + q) and B(k0 + q, j0 + r)
    for (int k0 = 0; k0 < Kd; k0 += 4) {
      const int k = k0 + q;
      const float a = (ia < M && k < Kd) ? A[ia * sai + k * sak] : 0.f;
      const float b = (jb < N && k < Kd) ? B[k * sbk + jb * sbj] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
  // result: lane (r, q), register t holds C(i0 + 4q + t, j0 + r)
  const int j = j0 + r;
  if (j >= N) return;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = i0 + 4 * q + t;
    if (i >= M) continue;
    float v = acc[t];
    if (EPI != EPI_DTANH && bias) v += bias[j];
    if (EPI == EPI_TANH) v = tanhf(v);
    if (EPI == EPI_DTANH) {
      const float h = H[i * ldc + j];
      v *= 1.f - h * h;
    }
    C[i * ldc + j] = v;
  }
}

hipError_t launch_mlp_gemm(int bf16, int epi, int M, int N, int Kd, const float* A, int64_t sai,
                           int64_t sak, const float* B, int64_t sbk, int64_t sbj,
                           const float* bias, const float* H, float* C, int64_t ldc,
                           hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (Kd <= 0 || epi < 0 || epi > 2 || (epi == EPI_DTANH && !H)) return hipErrorInvalidValue;
  const dim3 grid((N + 15) / 16, (M + 15) / 16);
#define L(BF, E) k_mlp_gemm<BF, E><<<grid, 64, 0, st>>>(M, N, Kd, A, sai, sak, B, sbk, sbj, bias, H, C, ldc)
  if (bf16) {
    if (epi == EPI_NONE) L(true, EPI_NONE);
    else if (epi == EPI_TANH) L(true, EPI_TANH);
    else L(true, EPI_DTANH);
  } else {
    if (epi == EPI_NONE) L(false, EPI_NONE);
    else if (epi == EPI_TANH) L(false, EPI_TANH);
    else L(false, EPI_DTANH);
  }
#undef L
  return hipGetLastError();
}

// Mean-squared error over a [B][n] batch: dO = 2 (O - T) / (B n); the loss
// sum(O - T)^2 / (B n) goes to loss[0] (one block, fixed-order reduction).
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ O, const float* __restrict__ T, float* __restrict__ dO,
      float* __restrict__ loss, int64_t cnt) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const float sc = 2.f / (float)cnt;
  float s = 0.f;
  for (int64_t i = t; i < cnt; i += 256) {
    const float d = O[i] - T[i];
    dO[i] = sc * d;
    s = fmaf(d, d, s);
  }
  red[t] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] += red[t + k];
    __syncthreads();
  }
  if (t == 0) loss[0] = red[0] / (float)cnt;
}

hipError_t launch_mse(const float* O, const float* T, float* dO, float* loss, int64_t cnt,
                      hipStream_t st) {
  if (cnt <= 0) return hipErrorInvalidValue;
  k_mse<<<1, 256, 0, st>>>(O, T, dO, loss, cnt);
  return hipGetLastError();
}

// db[j] = sum_b dZ[b][j] (one thread per column, batch order)
__global__ void k_colsum(const float* __restrict__ dZ, int B, int N, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + j];
  db[j] = s;
}

hipError_t launch_colsum(const float* dZ, int B, int N, float* db, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_colsum<<<(N + 255) / 256, 256, 0, st>>>(dZ, B, N, db);
  return hipGetLastError();
}

// Adam (bias-corrected): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t grid = (n + 255) / 256;
  if (grid > 4096) grid = 4096;
  k_adam<<<(unsigned)grid, 256, 0, st>>>(w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace tsgls
