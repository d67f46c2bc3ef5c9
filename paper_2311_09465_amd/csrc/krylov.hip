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
__global__ void k_fill(double* x, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = a;
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
hipError_t launch_fill(double* x, double a, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_fill<<<grid_for(n, 256), 256, 0, st>>>(x, a, n);
  return hipGetLastError();
}
// bf16 keeps the top 16 bits of the FP32 value; the low half is rounded to
// nearest, ties to even (finite inputs).
__global__ void k_to_bf16(const double* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t u = __float_as_uint((float)x[i]);
  u += 0x7fffu + ((u >> 16) & 1u);
  y[i] = (uint16_t)(u >> 16);
}

hipError_t launch_to_bf16(const double* x, uint16_t* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_to_bf16<<<grid_for(n, 256), 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_to_f32<<<grid_for(n, 256), 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- multi-dot
// Block b owns the contiguous chunk [b*chunk, min(n, (b+1)*chunk)); each
// thread accumulates strided products for a tile of up to 8 vectors, then
// the block sums them in a fixed order (block_sum_tile), so every result is
// reproducible bit for bit.
constexpr int MD_BS = 256;
constexpr int MD_TILE = 8;

// Value of another lane by a DPP move within a 16-lane row (CTRL: the DPP
// control word), for a double.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double read_lane(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Sum over the 64 lanes of a wave (all lanes active), the same on every lane:
// pairs inside each 16-lane row by DPP moves (lane ^ 1, lane ^ 2, the two
// quads of each half row, the two halves of each row; both partners add the
// same two numbers), then the four row sums in row order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x128>(v);   // row_ror:8
  return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

// Block-wide sums of NT per-thread values (MD_BS threads = 4 waves): the sum
// inside each wave (wave_sum), then the four wave sums in wave order.
// Thread k < NT returns sum k; red holds 4 * NT doubles.
template <int NT>
__device__ __forceinline__ double block_sum_tile(double (&x)[NT], double* red, int t) {
  const int lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const double v = wave_sum(x[k]);
    if (lane == 0) red[wv * NT + k] = v;
  }
  __syncthreads();
  double s = 0.0;
  if (t < NT) s = ((red[t] + red[NT + t]) + red[2 * NT + t]) + red[3 * NT + t];
  __syncthreads();   // red may be reused by the caller
  return s;
}

// grid (nblocks, ceil(J / 8), segments): block (b, y, z) handles vectors
// 8y .. 8y+7 of segment z (V and w offset by z sv, partial by z sp).
__global__ void __launch_bounds__(MD_BS)
k_multidot(const double* __restrict__ V, int64_t ldv, int J, const double* __restrict__ w,
           double* __restrict__ partial, int64_t n, int64_t chunk, int64_t sv, int64_t sp,
           const int* __restrict__ skip) {
  __shared__ double red[4 * MD_TILE];
  if (skip && skip[blockIdx.z]) return;   // a segment sitting out
  V += blockIdx.z * sv;
  w += blockIdx.z * sv;
  partial += blockIdx.z * sp;
  const int b = blockIdx.x, t = threadIdx.x, j0 = blockIdx.y * MD_TILE;
  const int64_t lo = (int64_t)b * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double acc[MD_TILE];
#pragma unroll
  for (int k = 0; k < MD_TILE; ++k) acc[k] = 0.0;
  for (int64_t i = lo + t; i < hi; i += MD_BS) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < MD_TILE; ++k)
      if (j0 + k < J) acc[k] = fma(V[(int64_t)(j0 + k) * ldv + i], wi, acc[k]);
  }
  const double sum = block_sum_tile<MD_TILE>(acc, red, t);
  if (t < MD_TILE && j0 + t < J) partial[(int64_t)b * J + j0 + t] = sum;
}

// Chunks of at least 256 entries (one per thread), at most 1024 blocks.
int multidot_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_multidot(const double* V, int64_t ldv, int J, const double* w, double* partial,
                           int nblocks, int64_t n, hipStream_t st, int nseg, int64_t sv, int64_t sp,
                           const int* skip) {
  if (J <= 0 || nseg <= 0) return hipSuccess;
  const int64_t chunk = (n + nblocks - 1) / nblocks;
  k_multidot<<<dim3(nblocks, (J + MD_TILE - 1) / MD_TILE, nseg), MD_BS, 0, st>>>(V, ldv, J, w, partial,
                                                                                 n, chunk, sv, sp, skip);
  return hipGetLastError();
}

// One block per output j (and segment y): strided partial sums over the
// blocks' partials in a fixed assignment, then the fixed-order block sum.
__global__ void __launch_bounds__(256)
k_reduce_partials(const double* __restrict__ partial, int nb, int J, double* __restrict__ out,
                  int64_t sp, int64_t so, const int* __restrict__ skip) {
  __shared__ double red[4];
  if (skip && skip[blockIdx.y]) return;
  partial += blockIdx.y * sp;
  out += blockIdx.y * so;
  const int j = blockIdx.x, t = threadIdx.x;
  double x[1] = {0.0};
  for (int b = t; b < nb; b += 256) x[0] += partial[(int64_t)b * J + j];
  const double sum = block_sum_tile<1>(x, red, t);
  if (t == 0) out[j] = sum;
}

hipError_t launch_reduce_partials(const double* partial, int nblocks, int J, double* out, hipStream_t st,
                                  int nseg, int64_t sp, int64_t so, const int* skip) {
  if (nseg <= 0) return hipSuccess;
  k_reduce_partials<<<dim3(J, nseg), 256, 0, st>>>(partial, nblocks, J, out, sp, so, skip);
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
  __shared__ double red[4 * MD_TILE];
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
    double x[MD_TILE];
#pragma unroll
    for (int k = 0; k < MD_TILE; ++k) {
      const int o = j0 + k;
      x[k] = 0.0;
      if (self && o == Jd) {
        x[k] = d[JT];
      } else {
#pragma unroll
        for (int j = 0; j < JT; ++j)
          if (j == o) x[k] = d[j];
      }
    }
    const double sum = block_sum_tile<MD_TILE>(x, red, t);
    if (t < MD_TILE && j0 + t < Jo) partial[(int64_t)b * Jo + j0 + t] = sum;
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
// k_multidot), on a grid (nblocks, ceil(J / JT)): block (b, y) handles basis
// vectors JT y .. JT y + JT - 1 of chunk b, and tile 0 also the three norms.
// Update: u <- (u - Q a) / nu, then w <- (w - Q b - u h) / sigma with the
// updated u.
template <int JT>
__global__ void __launch_bounds__(MD_BS)
k_gs_reduce(const double* __restrict__ Q, int64_t ldq, int J, const double* __restrict__ u,
            const double* __restrict__ w, double* __restrict__ partial, int64_t n, int64_t chunk,
            int64_t sv, int64_t sp, const int* __restrict__ skip) {
  __shared__ double red[4 * MD_TILE];
  if (skip && skip[blockIdx.z]) return;
  Q += blockIdx.z * sv;
  u += blockIdx.z * sv;
  w += blockIdx.z * sv;
  partial += blockIdx.z * sp;
  const int b = blockIdx.x, t = threadIdx.x;
  const int jb = blockIdx.y * JT;                  // first basis vector of this tile
  const int Jt = J - jb < JT ? J - jb : JT;        // vectors in this tile (0 when J = 0)
  const bool norms = blockIdx.y == 0;
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
      const double q = j < Jt ? Q[(int64_t)(jb + j) * ldq + i] : 0.0;
      da[j] = fma(q, ui, da[j]);
      db[j] = fma(q, wi, db[j]);
    }
    uu = fma(ui, ui, uu);
    uw = fma(ui, wi, uw);
    ww = fma(wi, wi, ww);
  }
  // local outputs k: da (k < JT), db (JT <= k < 2 JT), the norms (2 JT + 0..2)
  constexpr int NO = 2 * JT + 3;
#pragma unroll
  for (int k0 = 0; k0 < NO; k0 += MD_TILE) {
    double x[MD_TILE];
#pragma unroll
    for (int kk = 0; kk < MD_TILE; ++kk) {
      const int k = k0 + kk;
      x[kk] = k < JT ? da[k < JT ? k : 0]
            : k < 2 * JT ? db[k < 2 * JT ? k - JT : 0]
            : k == 2 * JT ? uu : k == 2 * JT + 1 ? uw : ww;
    }
    const double sum = block_sum_tile<MD_TILE>(x, red, t);
    const int k = k0 + t;
    int o = -1;
    if (k < JT) o = k < Jt ? jb + k : -1;
    else if (k < 2 * JT) o = k - JT < Jt ? J + jb + (k - JT) : -1;
    else if (k < NO && norms) o = 2 * J + (k - 2 * JT);
    if (t < MD_TILE && o >= 0) partial[(int64_t)b * Jo + o] = sum;
  }
}

// Gram-Schmidt coefficients [a (J); b (J)] passed by value as a kernel
// argument, so that no copy to the device precedes the update.
template <int JT>
struct GsCoef {
  double v[2 * JT];
};

// Coefficients come from ab (device memory) when it is not null, else from cf.
// Segment blockIdx.y: Q, u, w offset by y sv; ab and sc (device) by y sd.
template <int JT>
__global__ void __launch_bounds__(MD_BS)
k_gs_update(const double* __restrict__ Q, int64_t ldq, int J, const double* __restrict__ ab,
            GsCoef<JT> cf, double inv_nu, double h, double inv_sigma, const double* __restrict__ sc,
            double* __restrict__ u, double* __restrict__ w, int64_t n, int64_t sv, int64_t sd,
            const int* __restrict__ skip) {
  __shared__ double sa[JT], sb[JT];
  if (skip && skip[blockIdx.y]) return;
  Q += blockIdx.y * sv;
  u += blockIdx.y * sv;
  w += blockIdx.y * sv;
  if (ab) ab += blockIdx.y * sd;
  if (sc) sc += blockIdx.y * sd;
  if (sc) {   // scalars from the device-side least-squares update
    inv_nu = sc[0];
    h = sc[1];
    inv_sigma = sc[2];
  }
  if (threadIdx.x < JT) {
    const int t = threadIdx.x;
    sa[t] = t < J ? (ab ? ab[t] : cf.v[t]) : 0.0;
    sb[t] = t < J ? (ab ? ab[J + t] : cf.v[J + t]) : 0.0;
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

// The same update for 32 < J <= GS_DELAYED_MAX: the four waves of a block
// take four contiguous ranges of basis vectors for the same 64 entries, and
// their partial sums are added in wave order (deterministic), so that each
// thread keeps only a quarter of the loads in flight.
__global__ void __launch_bounds__(MD_BS)
k_gs_update_wide(const double* __restrict__ Q, int64_t ldq, int J, const double* __restrict__ ab,
                 GsCoef<GS_DELAYED_MAX> cf, double inv_nu, double h, double inv_sigma,
                 const double* __restrict__ sc, double* __restrict__ u, double* __restrict__ w,
                 int64_t n, int64_t sv, int64_t sd, const int* __restrict__ skip) {
  __shared__ double sa[GS_DELAYED_MAX], sb[GS_DELAYED_MAX];
  __shared__ double spa[4][64], spb[4][64];
  if (skip && skip[blockIdx.y]) return;
  Q += blockIdx.y * sv;
  u += blockIdx.y * sv;
  w += blockIdx.y * sv;
  if (ab) ab += blockIdx.y * sd;
  if (sc) sc += blockIdx.y * sd;
  if (sc) {
    inv_nu = sc[0];
    h = sc[1];
    inv_sigma = sc[2];
  }
  for (int j = threadIdx.x; j < J; j += MD_BS) {
    sa[j] = ab ? ab[j] : cf.v[j];
    sb[j] = ab ? ab[J + j] : cf.v[J + j];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per = (J + 3) / 4, j0 = wv * per, j1 = j0 + per < J ? j0 + per : J;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
    const int64_t i = base + lane;
    double pa = 0.0, pb = 0.0;
    if (i < n) {
      int j = j0;
      for (; j + 8 <= j1; j += 8) {
        double q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = Q[(int64_t)(j + k) * ldq + i];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          pa = fma(q[k], sa[j + k], pa);
          pb = fma(q[k], sb[j + k], pb);
        }
      }
      for (; j < j1; ++j) {
        const double q = Q[(int64_t)j * ldq + i];
        pa = fma(q, sa[j], pa);
        pb = fma(q, sb[j], pb);
      }
    }
    spa[wv][lane] = pa;
    spb[wv][lane] = pb;
    __syncthreads();
    if (wv == 0 && i < n) {
      const double ta = ((spa[0][lane] + spa[1][lane]) + spa[2][lane]) + spa[3][lane];
      const double tb = ((spb[0][lane] + spb[1][lane]) + spb[2][lane]) + spb[3][lane];
      const double un = (u[i] - ta) * inv_nu;
      u[i] = un;
      w[i] = (w[i] - tb - un * h) * inv_sigma;
    }
    __syncthreads();
  }
}

hipError_t launch_gs_reduce(const double* Q, int64_t ldq, int J, const double* u, const double* w,
                            double* partial, int nblocks, int64_t n, hipStream_t st, int nseg,
                            int64_t sv, int64_t sp, const int* skip) {
  if (J < 0 || J > GS_DELAYED_MAX) return hipErrorInvalidValue;
  if (nseg <= 0) return hipSuccess;
  const int64_t chunk = (n + nblocks - 1) / nblocks;
  // Tiles of eight vectors when there are few chunks (short vectors: more
  // blocks, and a shorter block reduction per block); every output sums the
  // same terms in the same order whatever the tile width.
  const int jt = (J <= 8 || nblocks < 512) ? 8 : J <= 16 ? 16 : 32;
  const dim3 grid((unsigned)nblocks, J == 0 ? 1u : (unsigned)((J + jt - 1) / jt), (unsigned)nseg);
#define L(JT) k_gs_reduce<JT><<<grid, MD_BS, 0, st>>>(Q, ldq, J, u, w, partial, n, chunk, sv, sp, skip)
  if (jt == 8) L(8);
  else if (jt == 16) L(16);
  else L(32);
#undef L
  return hipGetLastError();
}

template <int JT>
static GsCoef<JT> gs_coef(const double* ab_host, int J) {
  GsCoef<JT> cf{};
  if (ab_host)
    for (int i = 0; i < 2 * J; ++i) cf.v[i] = ab_host[i];
  return cf;
}

hipError_t launch_gs_update(const double* Q, int64_t ldq, int J, const double* ab,
                            const double* ab_host, double inv_nu, double h, double inv_sigma,
                            const double* sc, double* u, double* w, int64_t n, hipStream_t st,
                            int nseg, int64_t sv, int64_t sd, const int* skip) {
  if (J < 0 || J > GS_DELAYED_MAX) return hipErrorInvalidValue;
  if ((ab == nullptr) == (ab_host == nullptr) && J > 0) return hipErrorInvalidValue;
  if (nseg > 1 && (ab_host || (!sc && J > 0))) return hipErrorInvalidValue;   // segments: device coefficients
  if (n == 0 || nseg <= 0) return hipSuccess;
  int64_t g = (n + MD_BS - 1) / MD_BS;
  if (g > 8192) g = 8192;
#define L(JT)                                                                                     \
  k_gs_update<JT><<<dim3((unsigned)g, nseg), MD_BS, 0, st>>>(Q, ldq, J, ab, gs_coef<JT>(ab_host, J), \
                                                             inv_nu, h, inv_sigma, sc, u, w, n, sv, sd, skip)
  if (J <= 8) L(8);
  else if (J <= 16) L(16);
  else if (J <= 32) L(32);
#undef L
  else {
    int64_t gw = (n + 63) / 64;
    if (gw > 16384) gw = 16384;
    k_gs_update_wide<<<dim3((unsigned)gw, nseg), MD_BS, 0, st>>>(
        Q, ldq, J, ab, gs_coef<GS_DELAYED_MAX>(ab_host, J), inv_nu, h, inv_sigma, sc, u, w, n, sv, sd, skip);
  }
  return hipGetLastError();
}

// w -= sum_j V[j] h[j]   (h on device, J <= 1024); segment blockIdx.y: V and
// w offset by y sv, h by y sh.
__global__ void k_multiaxpy(const double* __restrict__ V, int64_t ldv, int J, const double* __restrict__ h,
                            double* __restrict__ w, int64_t n, double sign, int64_t sv, int64_t shs,
                            const int* __restrict__ skip) {
  __shared__ double sh[1024];
  if (skip && skip[blockIdx.y]) return;
  V += blockIdx.y * sv;
  w += blockIdx.y * sv;
  h += blockIdx.y * shs;
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
  k_multiaxpy<<<grid_for(n, 256), 256, 0, st>>>(V, ldv, J, h, w, n, -1.0, 0, 0, nullptr);
  return hipGetLastError();
}

hipError_t launch_multiaxpy_add(const double* V, int64_t ldv, int J, const double* c, double* y, int64_t n,
                                hipStream_t st, int nseg, int64_t sv, int64_t sc, const int* skip) {
  if (n == 0 || J == 0 || nseg <= 0) return hipSuccess;
  k_multiaxpy<<<dim3(grid_for(n, 256), nseg), 256, 0, st>>>(V, ldv, J, c, y, n, 1.0, sv, sc, skip);
  return hipGetLastError();
}

// ------------------------------------------- device-side GMRES least squares
// The host-side update of the delayed Gram-Schmidt GMRES (host.cpp,
// gmres_delayed) on the device, one wave per GMRES (rows of a Hessenberg
// column in parallel, the Givens rotations on one lane), so that a whole
// cycle runs without the host and can be captured as a graph.  State (GmDev): unrotated Hessenberg H and
// its rotated finalized columns R (column-major, leading dimension m+1),
// rotations, the rotated right-hand side g, the update scalars sc and the
// status st = {k committed columns, cycle over, finalize pending, converged}.
namespace {

__device__ void gm_commit(const GmDev& d, int j) {
  const int ld = d.m + 1;
  double* Rj = d.R + (int64_t)j * ld;
  const double* Hj = d.H + (int64_t)j * ld;
  for (int i = 0; i <= j + 1; ++i) Rj[i] = Hj[i];
  for (int i = 0; i < j; ++i) {
    const double t = d.cs[i] * Rj[i] + d.sn[i] * Rj[i + 1];
    Rj[i + 1] = -d.sn[i] * Rj[i] + d.cs[i] * Rj[i + 1];
    Rj[i] = t;
  }
  const double den = hypot(Rj[j], Rj[j + 1]);
  d.cs[j] = den > 0 ? Rj[j] / den : 1.0;
  d.sn[j] = den > 0 ? Rj[j + 1] / den : 0.0;
  Rj[j] = den;
  Rj[j + 1] = 0.0;
  d.g[j + 1] = -d.sn[j] * d.g[j];
  d.g[j] = d.cs[j] * d.g[j];
}

__device__ void gm_silence(const GmDev& d, int j) {   // updates that leave u, w zero
  for (int i = 0; i < 2 * j; ++i) d.ab[i] = 0.0;
  d.sc[0] = d.sc[1] = d.sc[2] = 0.0;
}

// State of segment s (block s of a segmented launch).
__device__ GmDev gm_seg(GmDev d, int s) {
  const int64_t o = s * d.sd;
  d.H += o;
  d.R += o;
  d.cs += o;
  d.sn += o;
  d.g += o;
  d.y += o;
  d.ab += o;
  d.sc += o;
  d.st += (int64_t)s * d.si;
  return d;
}

}  // namespace

// Cycle start: bb[0] = |r|^2 of the cycle's residual r (already in slot 0).
// first != 0 fixes the absolute tolerance tol |r| for the whole solve.  One
// block (one wave) per segment (bb offset by s sbb); a segment flagged in
// d.skip takes no part in the cycle (it ends at once with zero updates).
__global__ void __launch_bounds__(64)
k_gm_begin(GmDev d0, const double* __restrict__ bb, double tol, int first, int64_t sbb) {
  const int lane = threadIdx.x;
  const GmDev d = gm_seg(d0, blockIdx.x);
  bb += blockIdx.x * sbb;
  const bool skip = d0.skip && d0.skip[blockIdx.x];
  const int ld = d.m + 1;
  for (int i = lane; i < ld * d.m; i += 64) d.H[i] = d.R[i] = 0.0;
  for (int i = lane; i <= d.m; i += 64) d.g[i] = 0.0;
  for (int i = lane; i < d.m; i += 64) d.y[i] = 0.0;
  __syncthreads();
  if (lane != 0) return;
  const double beta = sqrt(fmax(bb[0], 0.0));
  if (first) d.sc[4] = tol * beta;
  d.g[0] = beta;
  d.sc[3] = beta;
  d.sc[5] = (beta > 0 && !skip) ? 1.0 / beta : 0.0;
  const int conv = !(beta > d.sc[4]) || !isfinite(beta) || skip;
  d.st[0] = 0;
  d.st[1] = conv;
  d.st[2] = 0;
  d.st[3] = conv;
  d.st[4] = 0;
  if (conv) gm_silence(d, 0);
}

// Step j after the reduction red = [Q^T u (j); Q^T w (j); u.u; u.w; w.w]
// (one wave per segment, red offset by s sred).  The rows of the new
// Hessenberg column are formed by the lanes in parallel, each with the
// sequential sum of the one-thread form; the Givens rotations stay on lane 0.
__global__ void __launch_bounds__(64)
k_gm_step(GmDev d0, int j, const double* __restrict__ red, int64_t sred) {
  const int lane = threadIdx.x;
  const GmDev d = gm_seg(d0, blockIdx.x);
  red += blockIdx.x * sred;
  __shared__ double sr[2 * 32 + 3];
  auto silence = [&]() {
    for (int i = lane; i < 2 * j; i += 64) d.ab[i] = 0.0;
    if (lane == 0) d.sc[0] = d.sc[1] = d.sc[2] = 0.0;
  };
  if (d.st[1]) {
    silence();
    return;
  }
  for (int i = lane; i < 2 * j + 3; i += 64) sr[i] = red[i];
  __syncthreads();
  const int ld = d.m + 1;
  const double* a = sr;
  const double* bq = sr + j;
  const double uu = sr[2 * j], uw = sr[2 * j + 1], ww = sr[2 * j + 2];
  double aa = 0.0, abq = 0.0, bbq = 0.0;   // the same on every lane
  for (int i = 0; i < j; ++i) {
    aa += a[i] * a[i];
    abq += a[i] * bq[i];
    bbq += bq[i] * bq[i];
  }
  const double nu = sqrt(fmax(uu - aa, 0.0));
  auto H = [&](int i, int c) -> double& { return d.H[(int64_t)c * ld + i]; };
  if (j >= 1) {          // column j-1 for u_j = Q a + nu q_j; now final
    const double sj = H(j, j - 1);
    __syncthreads();     // every lane has read H(j, j-1) before lane 0 rewrites it
    for (int i = lane; i < j; i += 64) H(i, j - 1) += sj * a[i];
    if (lane == 0) H(j, j - 1) = sj * nu;
    __syncthreads();
    if (lane == 0) {
      gm_commit(d, j - 1);
      d.st[0] = j;
    }
    __syncthreads();
  }
  if (d.st[2] || !(nu > 0.0) || !isfinite(uu) || !isfinite(ww)) {
    // converged last step, or u_j in span(Q): the cycle ends here
    __syncthreads();     // every lane has read st[2] before lane 0 changes st
    if (lane == 0) {
      d.st[1] = 1;
      d.st[3] = fabs(d.g[d.st[0]]) <= d.sc[4];
    }
    silence();
    return;
  }
  // provisional column j: A q_j = (w - A Q a) / nu, A Q a = Q (H a); lane i, row i
  const double hj = (uw - abq) / nu;
  for (int i = lane; i <= j; i += 64) {
    double ha = 0.0;
    for (int l = (i > 0 ? i - 1 : 0); l < j; ++l) ha += H(i, l) * a[l];
    H(i, j) = ((i < j ? bq[i] : hj) - ha) / nu;
  }
  const double s2 = ww - bbq - hj * hj;
  const double sigma = sqrt(fmax(s2, 1e-30 * ww));
  if (lane == 0) H(j + 1, j) = sigma / nu;
  for (int i = lane; i < j; i += 64) {
    d.ab[i] = a[i];
    d.ab[j + i] = bq[i];
  }
  if (lane == 0) {
    d.sc[0] = 1.0 / nu;
    d.sc[1] = hj;
    d.sc[2] = 1.0 / sigma;
  }
  __syncthreads();       // column j complete
  if (lane != 0) return;
  // provisional least-squares residual with column j as it stands
  double c0 = 0.0, c1 = 0.0;
  {
    double col[34];
    for (int i = 0; i <= j + 1; ++i) col[i] = H(i, j);
    for (int i = 0; i < j; ++i) {
      const double t = d.cs[i] * col[i] + d.sn[i] * col[i + 1];
      col[i + 1] = -d.sn[i] * col[i] + d.cs[i] * col[i + 1];
      col[i] = t;
    }
    c0 = col[j];
    c1 = col[j + 1];
  }
  const double den = hypot(c0, c1);
  const double res = den > 0 ? fabs(c1 / den * d.g[j]) : fabs(d.g[j]);
  if (res <= d.sc[4]) d.st[2] = 1;   // finalize column j at the next reduction and stop
}

// After the last step: red = [Q^T u_m (m); ...; u_m.u_m at 2m] finalizes
// column m-1 (unless the cycle ended earlier); then R y = g over the k
// committed columns, y zero beyond k (one block per segment).
__global__ void k_gm_final(GmDev d0, const double* __restrict__ red, int64_t sred) {
  if (threadIdx.x != 0) return;
  const GmDev d = gm_seg(d0, blockIdx.x);
  red += blockIdx.x * sred;
  const int ld = d.m + 1, m = d.m;
  if (!d.st[1]) {
    double a2 = 0.0;
    for (int i = 0; i < m; ++i) a2 += red[i] * red[i];
    const double nu2 = sqrt(fmax(red[2 * m] - a2, 0.0));
    double* Hc = d.H + (int64_t)(m - 1) * ld;
    const double sj = Hc[m];
    for (int i = 0; i < m; ++i) Hc[i] += sj * red[i];
    Hc[m] = sj * nu2;
    gm_commit(d, m - 1);
    d.st[0] = m;
    d.st[1] = 1;
    d.st[3] = fabs(d.g[m]) <= d.sc[4];
  }
  const int k = d.st[0];
  for (int i = m - 1; i >= 0; --i) {
    if (i >= k) {
      d.y[i] = 0.0;
      continue;
    }
    double s = d.g[i];
    for (int l = i + 1; l < k; ++l) s -= d.R[(int64_t)l * ld + i] * d.y[l];
    d.y[i] = s / d.R[(int64_t)i * ld + i];
  }
  d.sc[6] = fabs(d.g[k]);   // least-squares residual estimate of the cycle
  d.st[4] = !isfinite(d.sc[6]);
}

// x *= s[0] (device scalar); segment blockIdx.y: x offset by y sx, s by y ss
__global__ void k_scal_dev(double* __restrict__ x, const double* __restrict__ s, int64_t n, int64_t sx,
                           int64_t ss, const int* __restrict__ skip) {
  if (skip && skip[blockIdx.y]) return;
  x += blockIdx.y * sx;
  const double a = s[blockIdx.y * ss];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] *= a;
}

hipError_t launch_gm_begin(const GmDev& d, const double* bb, double tol, int first, hipStream_t st,
                           int nseg, int64_t sbb) {
  if (nseg <= 0) return hipSuccess;
  k_gm_begin<<<nseg, 64, 0, st>>>(d, bb, tol, first, sbb);
  return hipGetLastError();
}
hipError_t launch_gm_step(const GmDev& d, int j, const double* red, hipStream_t st, int nseg, int64_t sred) {
  if (j < 0 || j >= d.m || d.m > 32) return hipErrorInvalidValue;
  if (nseg <= 0) return hipSuccess;
  k_gm_step<<<nseg, 64, 0, st>>>(d, j, red, sred);
  return hipGetLastError();
}
hipError_t launch_gm_final(const GmDev& d, const double* red, hipStream_t st, int nseg, int64_t sred) {
  if (nseg <= 0) return hipSuccess;
  k_gm_final<<<nseg, 64, 0, st>>>(d, red, sred);
  return hipGetLastError();
}
hipError_t launch_scal_dev(double* x, const double* s, int64_t n, hipStream_t st, int nseg, int64_t sx,
                           int64_t ss, const int* skip) {
  if (n == 0 || nseg <= 0) return hipSuccess;
  k_scal_dev<<<dim3(grid_for(n, 256), nseg), 256, 0, st>>>(x, s, n, sx, ss, skip);
  return hipGetLastError();
}

}  // namespace tsgls
