// gfx950 kernels of the Neumann-face terms: backflow stabilization
// -(rho beta / 2)(w, |A_n|_- u)_Gamma_h with |A_n|_- = (A_n - |A_n|)/2
// (section "Stabilizing simulations in the presence of backflow") and the
// traction term -(w, h n)_Gamma_h of eq. Rmc.  3-point degree-2 rule per face.
#include "common.cuh"
#include "face_point.cuh"
#include "internal.h"

namespace tsgls {

template <int K>
struct FaceCfg {
  static constexpr int n = Dim<K>::n, M = Dim<K>::M;
  static constexpr int NP = np_of(n);
  static constexpr int per_group = 2 * n * n + M;
  static constexpr int G0 = 256 / NP;
  static constexpr int Gmem = 32768 / (per_group * 8);
  static constexpr int G = G0 < Gmem ? G0 : (Gmem < 1 ? 1 : Gmem);
  static constexpr int BLOCK = G * NP < 64 ? 64 : G * NP;
  static constexpr int GB = BLOCK / NP;
};

// One group of NP lanes per (face, face point).  A_n = A(u.n) in the
// orthonormal basis; one-sided Jacobi on A_n + sigma I (sigma > ||A_n||, so
// the shifted matrix is SPD) gives eigenpairs; lambda = ||w_c|| - sigma.
template <int K>
__global__ void __launch_bounds__(FaceCfg<K>::BLOCK)
k_face_lin(DevView v, const double* __restrict__ UTs, double* __restrict__ aneg) {
  using C = FaceCfg<K>;
  constexpr int n = C::n, M = C::M, NP = C::NP, P = Dim<K>::P, GB = C::GB;
  __shared__ double sUn[GB][M], sQ[GB][n * n], sL[GB][n];
  const double* __restrict__ F = v.F;
  const int g = threadIdx.x / NP, c = threadIdx.x % NP;
  const int64_t gq = (int64_t)blockIdx.x * GB + g;
  const int64_t f = gq / 3;
  const int q = (int)(gq % 3);
  const bool valid = f < v.n_faces;
  if (valid) {
    const double nx = v.fgeo[f * 4 + 0], ny = v.fgeo[f * 4 + 1], nz = v.fgeo[f * 4 + 2];
    for (int s = c; s < M; s += NP) {
      double un = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double* ut = UTs + (int64_t)v.fconn[f * 3 + b] * 3 * M + s;
        un += flam(q, b) * (nx * ut[0] + ny * ut[M] + nz * ut[2 * M]);
      }
      sUn[g][s] = un;
    }
  }
  __syncthreads();
  double w[n];
#pragma unroll
  for (int a = 0; a < n; ++a) w[a] = 0.0;
  if (valid && c < n) {
    const double invM = 1.0 / M;
#pragma unroll 1
    for (int s = 0; s < M; ++s) {
      const double t = sUn[g][s] * F[c * M + s] * invM;
#pragma unroll
      for (int a = 0; a < n; ++a) w[a] = fma(t, F[a * M + s], w[a]);
    }
  }
  double cn = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a) cn = fma(w[a], w[a], cn);
  const double sigma = 1.01 * sqrt(group_sum<NP>(cn)) + 1e-300;
#pragma unroll
  for (int a = 0; a < n; ++a)
    if (a == c && valid) w[a] += sigma;
  jacobi_columns<n, NP>(w, c);
  double l2 = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a) l2 = fma(w[a], w[a], l2);
  const double nrm = sqrt(l2);
  if (valid && c < n) {
    const double lam = nrm - sigma;
    sL[g][c] = lam < 0.0 ? lam : 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) sQ[g][c * n + a] = nrm > 0.0 ? w[a] / nrm : 0.0;
  }
  __syncthreads();
  if (valid) {
    double* out = aneg + (f * 3 + q) * P;
    for (int p = c; p < P; p += NP) {
      int r, cc;
      packed_rc<n>(p, r, cc);
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc = fma(sL[g][k] * sQ[g][k * n + r], sQ[g][k * n + cc], acc);
      out[p] = acc;
    }
  }
}

// Backflow and traction terms in two steps.  First one block per (face,
// face point): lane (i, m) forms y_i[m] = coef sum_c (|A_n|_-)_mc u_i[c] with
// u the input interpolated at the point (Dirichlet rows of a direction
// masked), coef = -(rho beta / 2) area / 3.  Then the node gather (k_gather)
// sums, per Neumann node, lam_q(node) y over its incident faces and points in
// a fixed order (deterministic), and for the residual subtracts the traction.
template <int K>
__global__ void __launch_bounds__(256)   // 3n lanes rounded up to a wave: 192 at K = 31
k_face_point(DevView v, const double* __restrict__ Y, const double* __restrict__ Ys, int resid,
             const double* __restrict__ an) {
  __shared__ double su[3 * Dim<K>::n];
  face_point_block<K>(v, Y, Ys, resid, an, blockIdx.x, threadIdx.x, su);
}

template <int K>
__global__ void k_face_diag(DevView v, double* __restrict__ d) {
  constexpr int n = Dim<K>::n, S = Dim<K>::S, P = Dim<K>::P;
  const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= v.n_fnodes) return;
  const int64_t node = v.fnode[u];
  double o[n];
#pragma unroll
  for (int m = 0; m < n; ++m) o[m] = 0.0;
  for (int k = v.foff[u]; k < v.foff[u + 1]; ++k) {
    const int64_t f = v.finc[k] / 3;
    const int a = v.finc[k] % 3;
    const double coef = -0.5 * v.rho * v.beta * v.fgeo[f * 4 + 3] / 3.0;
    for (int q = 0; q < 3; ++q) {
      const double* tp = v.aneg + (f * 3 + q) * P;
      const double l = flam(q, a);
      int p = 0;
#pragma unroll
      for (int r = 0; r < n; ++r) {
        o[r] += coef * l * l * tp[p];
        p += n - r;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double* op = d + (node * 4 + i) * S;
    op[0] += o[0];
#pragma unroll
    for (int m = 1; m < n; ++m) op[m + 1] += o[m];
  }
}


hipError_t launch_face_lin(const DevView& v, const double* UTs, double* aneg, hipStream_t st) {
  if (v.n_faces == 0) return hipSuccess;
  switch (v.K) {
#define CASE(k)                                                                        \
  case k: {                                                                            \
    const int64_t groups = v.n_faces * 3;                                              \
    const unsigned grid = (unsigned)((groups + FaceCfg<k>::GB - 1) / FaceCfg<k>::GB);  \
    k_face_lin<k><<<grid, FaceCfg<k>::BLOCK, 0, st>>>(v, UTs, aneg);                   \
    break;                                                                             \
  }
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_face_point(const DevView& v, const double* Y, const double* Ys, int resid,
                             const double* an, hipStream_t st) {
  if (v.n_fnodes == 0 || v.n_faces == 0) return hipSuccess;
  static_assert(3 * Dim<31>::n <= 256, "face point lanes within the launch bound");
  switch (v.K) {
#define CASE(k)                                                                                   \
  case k:                                                                                         \
    k_face_point<k><<<(unsigned)(v.n_faces * 3), (3 * Dim<k>::n + 63) / 64 * 64, 0, st>>>(v, Y, Ys, resid, an); \
    break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_face_diag(const DevView& v, double* d, hipStream_t st) {
  if (v.n_fnodes == 0) return hipSuccess;
  const unsigned grid = (unsigned)((v.n_fnodes + 127) / 128);
  switch (v.K) {
#define CASE(k) case k: k_face_diag<k><<<grid, 128, 0, st>>>(v, d); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tsgls
