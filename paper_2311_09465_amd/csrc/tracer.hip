// gfx950 element operator of the time-spectral GLS convection-diffusion
// equation (eq. 3D-weak, eq. 3D-weak-def): a scalar tracer phi carried by the
// frozen periodic velocity u of a Navier-Stokes state,
//   b(w, phi) = (w, Omega phi + u . grad phi) + (grad w, kappa grad phi)
//             + (L(w), tau L(phi)),   L(phi) = Omega phi + u . grad phi,
// with tau from eq. 3D-tau (kappa in place of nu; computed by k_tau).  With
// the least-squares term dropped (tau = 0) it is the Galerkin method the
// paper compares against.  Linear tetrahedra, 4-point rule (weights V/4).
//
// One element per 64-lane wave (grid-stride over elements); the transforms
// between modes and the M = 3K+1 samples are plain sums over a table of the
// basis in LDS.  Modes sit at positions as in the Navier-Stokes operator
// (mode 2k-1 at 2k-2, mode 2k at 2k-1, mode 0 at 2K).  Output rows use the
// element buffer layout [E][4 nodes][4 fields][n positions] in the slot
// scaling with the tracer in field 0 (fields 1..3 written as zero), so the
// node gather and the Krylov kernels serve it unchanged.
#include "common.cuh"
#include "internal.h"

namespace tsgls {

template <int K>
__global__ void __launch_bounds__(64)
k_cd(DevView v, const double* __restrict__ XP, double kappa, double* __restrict__ out,
     int64_t begin, int64_t end) {
  constexpr int n = 2 * K + 1, M = 3 * K + 1, PW = (n + 15) / 16 * 16, P = n * (n + 1) / 2;
  __shared__ double sF[n * M];        // phi_a(t_s), mode order
  __shared__ double sPhi[4][PW];      // tracer modes of the element's nodes (positions)
  __shared__ double sGp[3][PW];       // grad phi modes
  __shared__ double sU[4][3][M];      // u at the points, samples
  __shared__ double sG[3][M];         // grad phi samples
  __shared__ double sCv[4][M];        // u_q . grad phi, samples
  __shared__ double sL[4][PW];        // L(phi) at the points (positions)
  __shared__ double sZ[4][PW];        // z = tau L(phi)
  __shared__ double sZt[4][M];        // z samples
  __shared__ double sW[4][4][PW];     // modes of (u_q . grad N_a) z_q, [q][a]
  const int lane = threadIdx.x;
  const double omega = v.omega;
  for (int i = lane; i < n * M; i += 64) sF[i] = v.F[i];
  __syncthreads();
  auto om = [&](int p) -> double {   // (Omega x)_p = om(p) x_{p^1}
    return p < 2 * K ? ((p & 1) ? ((p + 1) >> 1) * omega : -((p >> 1) + 1) * omega) : 0.0;
  };
  auto lam = [](int q, int b) -> double { return q == b ? TS_QA : TS_QB; };
  for (int64_t e = begin + blockIdx.x; e < end; e += gridDim.x) {
    int nd[4];
    double dN[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      nd[b] = v.conn[e * 4 + b];
#pragma unroll
      for (int i = 0; i < 3; ++i) dN[b][i] = v.geo[e * 16 + b * 3 + i];
    }
    const double wgt = v.geo[e * 16 + 12];
    for (int i = lane; i < 4 * PW; i += 64) {
      const int b = i / PW, p = i % PW;
      sPhi[b][p] = XP[(int64_t)nd[b] * (4 * PW) + p];   // field 0
    }
    for (int i = lane; i < 12 * M; i += 64) {
      const int q = i / (3 * M), j = (i / M) % 3, s = i % M;
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) acc += lam(q, b) * v.UT[(int64_t)nd[b] * (3 * M) + j * M + s];
      sU[q][j][s] = acc;
    }
    __syncthreads();
    for (int i = lane; i < 3 * PW; i += 64) {
      const int j = i / PW, p = i % PW;
      sGp[j][p] = dN[0][j] * sPhi[0][p] + dN[1][j] * sPhi[1][p] + dN[2][j] * sPhi[2][p] +
                  dN[3][j] * sPhi[3][p];
    }
    __syncthreads();
    for (int i = lane; i < 3 * M; i += 64) {
      const int j = i / M, s = i % M;
      double acc = 0.0;
      for (int a = 0; a < n; ++a) acc = fma(sGp[j][mode_pos(a, K)], sF[a * M + s], acc);
      sG[j][s] = acc;
    }
    __syncthreads();
    for (int i = lane; i < 4 * M; i += 64) {
      const int q = i / M, s = i % M;
      sCv[q][s] = sU[q][0][s] * sG[0][s] + sU[q][1][s] * sG[1][s] + sU[q][2][s] * sG[2][s];
    }
    __syncthreads();
    for (int i = lane; i < 4 * PW; i += 64) {   // L = Omega phi_q + modes of u_q . grad phi
      const int q = i / PW, p = i % PW;
      double Lv = 0.0;
      if (p < n) {
        const int a = pos_mode(p, K), pp = p ^ 1;
        double c = 0.0;
        for (int s = 0; s < M; ++s) c = fma(sF[a * M + s], sCv[q][s], c);
        double phs = 0.0;
        if (p < 2 * K)
#pragma unroll
          for (int b = 0; b < 4; ++b) phs += lam(q, b) * sPhi[b][pp];
        Lv = om(p) * phs + c / M;
      }
      sL[q][p] = Lv;
    }
    __syncthreads();
    for (int i = lane; i < 4 * PW; i += 64) {   // z = tau_q L_q
      const int q = i / PW, p = i % PW;
      double z = 0.0;
      if (p < n) {
        const double* tq = v.tau + (e * 4 + q) * P;
        for (int k = 0; k < n; ++k)
          z = fma(tq[p <= k ? pk_index(p, k, n) : pk_index(k, p, n)], sL[q][k], z);
      }
      sZ[q][p] = z;
    }
    __syncthreads();
    for (int i = lane; i < 4 * M; i += 64) {
      const int q = i / M, s = i % M;
      double acc = 0.0;
      for (int a = 0; a < n; ++a) acc = fma(sZ[q][mode_pos(a, K)], sF[a * M + s], acc);
      sZt[q][s] = acc;
    }
    __syncthreads();
    for (int i = lane; i < 16 * PW; i += 64) {   // modes of (u_q . grad N_a) z_q
      const int q = i / (4 * PW), a = (i / PW) % 4, p = i % PW;
      double acc = 0.0;
      if (p < n) {
        const int m = pos_mode(p, K);
        for (int s = 0; s < M; ++s) {
          const double g = sU[q][0][s] * dN[a][0] + sU[q][1][s] * dN[a][1] + sU[q][2][s] * dN[a][2];
          acc = fma(sF[m * M + s], g * sZt[q][s], acc);
        }
      }
      sW[q][a][p] = acc / M;
    }
    __syncthreads();
    double* oe = out + e * (16 * n);
    for (int i = lane; i < 16 * n; i += 64) {
      const int a = i / (4 * n), f = (i / n) % 4, p = i % n;
      double r = 0.0;
      if (f == 0) {
        const int pp = p ^ 1;
        for (int q = 0; q < 4; ++q) {
          const double lq = lam(q, a);
          const double omz = p < 2 * K ? om(p) * sZ[q][pp] : 0.0;
          r += wgt * (lq * sL[q][p] - lq * omz + sW[q][a][p]);
        }
        // diffusion: kappa V grad N_a . grad phi (sum of the four weights is V)
        r += 4.0 * wgt * kappa * (dN[a][0] * sGp[0][p] + dN[a][1] * sGp[1][p] + dN[a][2] * sGp[2][p]);
        r *= p < 2 * K ? TS_RS2 : 1.0;
      }
      oe[i] = r;
    }
    __syncthreads();   // LDS of this element consumed before the next one
  }
}

hipError_t launch_cd(const DevView& v, const double* XP, double kappa, double* out, int64_t begin,
                     int64_t end, hipStream_t st) {
  if (end <= begin) return hipSuccess;
  int64_t nb = end - begin;
  if (nb > 8192) nb = 8192;
  switch (v.K) {
#define CASE(k) case k: k_cd<k><<<(unsigned)nb, 64, 0, st>>>(v, XP, kappa, out, begin, end); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tsgls
