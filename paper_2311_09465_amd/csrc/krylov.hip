// gfx950 BLAS-1 kernels for the Krylov solver (FP64).  Dot products are
// reduced in two deterministic stages: fixed per-block partial sums, then a
// fixed-order sum over blocks, so results are bitwise reproducible.
#include "internal.h"

namespace tsgls {

static inline unsigned grid_for(int64_t n, int bs) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 65535LL * 32) g = 65535LL * 32;
  return (unsigned)(g < 1 ? 1 : g);
}

__global__ void k_zero(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = 0.0;
}
__global__ void k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = x[i];
}
__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = fma(a, x[i], y[i]);
}
__global__ void k_scal_copy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = a * x[i];
}
__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = a[i] * x[i];
}
__global__ void k_recip(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = 1.0 / x[i];
}
__global__ void k_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = (float)x[i];
}

hipError_t launch_zero(double* x, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_zero<<<grid_for(n, 256), 256, 0, st>>>(x, n);
  return hipGetLastError();
}
hipError_t launch_copy(const double* x, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_copy<<<grid_for(n, 256), 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}
hipError_t launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_axpy<<<grid_for(n, 256), 256, 0, st>>>(a, x, y, n);
  return hipGetLastError();
}
hipError_t launch_scal_copy(double a, const double* x, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_scal_copy<<<grid_for(n, 256), 256, 0, st>>>(a, x, y, n);
  return hipGetLastError();
}
hipError_t launch_mul(const double* a, const double* x, double* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_mul<<<grid_for(n, 256), 256, 0, st>>>(a, x, y, n);
  return hipGetLastError();
}
hipError_t launch_recip(double* x, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_recip<<<grid_for(n, 256), 256, 0, st>>>(x, n);
  return hipGetLastError();
}
hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_to_f32<<<grid_for(n, 256), 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- multi-dot
// Block b owns the contiguous chunk [b*chunk, min(n, (b+1)*chunk)); for a
// tile of up to 8 vectors each thread accumulates strided products, then the
// block reduces in LDS in a fixed tree order.
constexpr int MD_BS = 256;
constexpr int MD_TILE = 8;

__global__ void __launch_bounds__(MD_BS)
k_multidot(const double* __restrict__ V, int64_t ldv, int J, const double* __restrict__ w,
           double* __restrict__ partial, int64_t n, int64_t chunk) {
  __shared__ double red[MD_TILE][MD_BS];
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t lo = (int64_t)b * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  for (int j0 = 0; j0 < J; j0 += MD_TILE) {
    double acc[MD_TILE];
#pragma unroll
    for (int k = 0; k < MD_TILE; ++k) acc[k] = 0.0;
    for (int64_t i = lo + t; i < hi; i += MD_BS) {
      const double wi = w[i];
#pragma unroll
      for (int k = 0; k < MD_TILE; ++k)
        if (j0 + k < J) acc[k] = fma(V[(int64_t)(j0 + k) * ldv + i], wi, acc[k]);
    }
#pragma unroll
    for (int k = 0; k < MD_TILE; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int s = MD_BS / 2; s > 0; s >>= 1) {
      if (t < s) {
#pragma unroll
        for (int k = 0; k < MD_TILE; ++k) red[k][t] += red[k][t + s];
      }
      __syncthreads();
    }
    if (t < MD_TILE && j0 + t < J) partial[(int64_t)b * J + j0 + t] = red[t][0];
    __syncthreads();
  }
}

int multidot_blocks(int64_t n) {
  int64_t b = (n + 4095) / 4096;
  if (b > 1024) b = 1024;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_multidot(const double* V, int64_t ldv, int J, const double* w, double* partial,
                           int nblocks, int64_t n, hipStream_t st) {
  const int64_t chunk = (n + nblocks - 1) / nblocks;
  k_multidot<<<nblocks, MD_BS, 0, st>>>(V, ldv, J, w, partial, n, chunk);
  return hipGetLastError();
}

// One block per output j: strided partial sums over the blocks' partials in
// a fixed assignment, then a fixed-order tree in LDS.
__global__ void __launch_bounds__(256)
k_reduce_partials(const double* __restrict__ partial, int nb, int J, double* __restrict__ out) {
  __shared__ double red[256];
  const int j = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nb; b += 256) s += partial[(int64_t)b * J + j];
  red[t] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) red[t] += red[t + k];
    __syncthreads();
  }
  if (t == 0) out[j] = red[0];
}

hipError_t launch_reduce_partials(const double* partial, int nblocks, int J, double* out, hipStream_t st) {
  k_reduce_partials<<<J, 256, 0, st>>>(partial, nblocks, J, out);
  return hipGetLastError();
}

// Fused Gram-Schmidt update and dots (J <= JT): w += sign * sum_j V[j] h[j]
// (skipped when h is null), then block partials of V[j] . w_new for j < Jd,
// and of w_new . w_new in slot Jd when self != 0.  Same chunking and fixed-order block reduction as
// k_multidot, so the result is reproducible.
template <int JT>
__global__ void __launch_bounds__(MD_BS)
k_axpy_dot(const double* __restrict__ V, int64_t ldv, int J, const double* __restrict__ h,
           double sign, double* __restrict__ w, int Jd, int self, double* __restrict__ partial,
           int64_t n, int64_t chunk) {
  __shared__ double red[MD_TILE][MD_BS];
  __shared__ double sh[JT];
  const int b = blockIdx.x, t = threadIdx.x;
  const int Jo = Jd + (self ? 1 : 0);
  const bool upd = h != nullptr;
  if (t < JT) sh[t] = (upd && t < J) ? sign * h[t] : 0.0;
  __syncthreads();
  const int64_t lo = (int64_t)b * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double d[JT + 1];
#pragma unroll
  for (int j = 0; j <= JT; ++j) d[j] = 0.0;
  for (int64_t i = lo + t; i < hi; i += MD_BS) {
    double vj[JT];
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < JT; ++j) {
      vj[j] = j < J ? V[(int64_t)j * ldv + i] : 0.0;
      acc = fma(vj[j], sh[j], acc);
    }
    const double wn = w[i] + acc;
    if (upd) w[i] = wn;
#pragma unroll
    for (int j = 0; j < JT; ++j) d[j] = fma(vj[j], wn, d[j]);
    d[JT] = fma(wn, wn, d[JT]);
  }
  for (int j0 = 0; j0 < Jo; j0 += MD_TILE) {
#pragma unroll
    for (int k = 0; k < MD_TILE; ++k) {
      const int o = j0 + k;
      double x = 0.0;
      if (self && o == Jd) {
        x = d[JT];
      } else {
#pragma unroll
        for (int j = 0; j < JT; ++j)
          if (j == o) x = d[j];
      }
      red[k][t] = x;
    }
    __syncthreads();
    for (int s = MD_BS / 2; s > 0; s >>= 1) {
      if (t < s) {
#pragma unroll
        for (int k = 0; k < MD_TILE; ++k) red[k][t] += red[k][t + s];
      }
      __syncthreads();
    }
    if (t < MD_TILE && j0 + t < Jo) partial[(int64_t)b * Jo + j0 + t] = red[t][0];
    __syncthreads();
  }
}

hipError_t launch_axpy_dot(const double* V, int64_t ldv, int J, const double* h, double sign,
                           double* w, int Jd, int self, double* partial, int nblocks, int64_t n,
                           hipStream_t st) {
  if (J < 0 || Jd < 0 || Jd > J) return hipErrorInvalidValue;
  const int64_t chunk = (n + nblocks - 1) / nblocks;
#define L(JT) k_axpy_dot<JT><<<nblocks, MD_BS, 0, st>>>(V, ldv, J, h, sign, w, Jd, self, partial, n, chunk)
  if (J <= 8) L(8);
  else if (J <= 16) L(16);
  else if (J <= 32) L(32);
  else return hipErrorInvalidValue;
#undef L
  return hipGetLastError();
}

// Delayed classical Gram-Schmidt (one reduction and one update pass over the
// basis per Arnoldi step).  Reduction: block partials of [Q^T u; Q^T w; u.u;
// u.w; w.w] for the J rows of Q (fixed chunking and block tree, as
// k_multidot).  Update: u <- (u - Q a) / nu, then w <- (w - Q b - u h) / sigma
// with the updated u.
template <int JT>
__global__ void __launch_bounds__(MD_BS)
k_gs_reduce(const double* __restrict__ Q, int64_t ldq, int J, const double* __restrict__ u,
            const double* __restrict__ w, double* __restrict__ partial, int64_t n, int64_t chunk) {
  __shared__ double red[MD_TILE][MD_BS];
  const int b = blockIdx.x, t = threadIdx.x;
  const int Jo = 2 * J + 3;
  const int64_t lo = (int64_t)b * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double da[JT], db[JT], uu = 0.0, uw = 0.0, ww = 0.0;
#pragma unroll
  for (int j = 0; j < JT; ++j) da[j] = db[j] = 0.0;
  for (int64_t i = lo + t; i < hi; i += MD_BS) {
    const double ui = u[i], wi = w[i];
#pragma unroll
    for (int j = 0; j < JT; ++j) {
      const double q = j < J ? Q[(int64_t)j * ldq + i] : 0.0;
      da[j] = fma(q, ui, da[j]);
      db[j] = fma(q, wi, db[j]);
    }
    uu = fma(ui, ui, uu);
    uw = fma(ui, wi, uw);
    ww = fma(wi, wi, ww);
  }
  for (int j0 = 0; j0 < Jo; j0 += MD_TILE) {
#pragma unroll
    for (int k = 0; k < MD_TILE; ++k) {
      const int o = j0 + k;
      double x = 0.0;
#pragma unroll
      for (int j = 0; j < JT; ++j) {
        if (o == j && j < J) x = da[j];
        if (o == J + j && j < J) x = db[j];
      }
      if (o == 2 * J) x = uu;
      if (o == 2 * J + 1) x = uw;
      if (o == 2 * J + 2) x = ww;
      red[k][t] = x;
    }
    __syncthreads();
    for (int s = MD_BS / 2; s > 0; s >>= 1) {
      if (t < s) {
#pragma unroll
        for (int k = 0; k < MD_TILE; ++k) red[k][t] += red[k][t + s];
      }
      __syncthreads();
    }
    if (t < MD_TILE && j0 + t < Jo) partial[(int64_t)b * Jo + j0 + t] = red[t][0];
    __syncthreads();
  }
}

template <int JT>
__global__ void __launch_bounds__(MD_BS)
k_gs_update(const double* __restrict__ Q, int64_t ldq, int J, const double* __restrict__ ab,
            double inv_nu, double h, double inv_sigma, double* __restrict__ u,
            double* __restrict__ w, int64_t n) {
  __shared__ double sa[JT], sb[JT];
  if (threadIdx.x < JT) {
    sa[threadIdx.x] = threadIdx.x < J ? ab[threadIdx.x] : 0.0;
    sb[threadIdx.x] = threadIdx.x < J ? ab[J + threadIdx.x] : 0.0;
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int j = 0; j < JT; ++j) {
      const double q = j < J ? Q[(int64_t)j * ldq + i] : 0.0;
      pa = fma(q, sa[j], pa);
      pb = fma(q, sb[j], pb);
    }
    const double un = (u[i] - pa) * inv_nu;
    u[i] = un;
    w[i] = (w[i] - pb - un * h) * inv_sigma;
  }
}

hipError_t launch_gs_reduce(const double* Q, int64_t ldq, int J, const double* u, const double* w,
                            double* partial, int nblocks, int64_t n, hipStream_t st) {
  if (J < 0 || J > 32) return hipErrorInvalidValue;
  const int64_t chunk = (n + nblocks - 1) / nblocks;
#define L(JT) k_gs_reduce<JT><<<nblocks, MD_BS, 0, st>>>(Q, ldq, J, u, w, partial, n, chunk)
  if (J <= 8) L(8);
  else if (J <= 16) L(16);
  else L(32);
#undef L
  return hipGetLastError();
}

hipError_t launch_gs_update(const double* Q, int64_t ldq, int J, const double* ab, double inv_nu,
                            double h, double inv_sigma, double* u, double* w, int64_t n,
                            hipStream_t st) {
  if (J < 0 || J > 32) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  int64_t g = (n + MD_BS - 1) / MD_BS;
  if (g > 8192) g = 8192;
#define L(JT) k_gs_update<JT><<<(unsigned)g, MD_BS, 0, st>>>(Q, ldq, J, ab, inv_nu, h, inv_sigma, u, w, n)
  if (J <= 8) L(8);
  else if (J <= 16) L(16);
  else L(32);
#undef L
  return hipGetLastError();
}

// w -= sum_j V[j] h[j]   (h on device, J <= 1024)
__global__ void k_multiaxpy(const double* __restrict__ V, int64_t ldv, int J, const double* __restrict__ h,
                            double* __restrict__ w, int64_t n, double sign) {
  __shared__ double sh[1024];
  for (int j = threadIdx.x; j < J; j += blockDim.x) sh[j] = h[j];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < J; ++j) acc = fma(V[(int64_t)j * ldv + i], sh[j], acc);
    w[i] = fma(sign, acc, w[i]);
  }
}

hipError_t launch_multiaxpy(const double* V, int64_t ldv, int J, const double* h, double* w, int64_t n,
                            hipStream_t st) {
  if (n == 0 || J == 0) return hipSuccess;
  k_multiaxpy<<<grid_for(n, 256), 256, 0, st>>>(V, ldv, J, h, w, n, -1.0);
  return hipGetLastError();
}

hipError_t launch_multiaxpy_add(const double* V, int64_t ldv, int J, const double* c, double* y, int64_t n,
                                hipStream_t st) {
  if (n == 0 || J == 0) return hipSuccess;
  k_multiaxpy<<<grid_for(n, 256), 256, 0, st>>>(V, ldv, J, c, y, n, 1.0);
  return hipGetLastError();
}

}  // namespace tsgls
