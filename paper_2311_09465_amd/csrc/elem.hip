// gfx950 kernels of the volume terms: element geometry, time samples of the
// nodal velocity, the stabilization matrix tau per quadrature point, the GLS
// element operator (residual / tangent products) and the Jacobi diagonal.
//
// Basis.  Per field the K harmonics are held as n = 2K+1 real coordinates in
// the orthonormal basis phi_0 = 1, phi_{2k-1} = sqrt2 cos(k w t),
// phi_{2k} = -sqrt2 sin(k w t).  In it the convolution matrix A(u) of the
// paper (eq. phi-def) is the real symmetric matrix of "multiply by u(t),
// project back on K harmonics", Omega is skew-symmetric, and tau is real
// symmetric; the complex Hermitian forms of the paper act identically on
// conjugate-symmetric mode vectors.  Products are formed on M = 3K+1 time
// samples, which reproduces the truncated convolution exactly.
#include "common.cuh"
#include "internal.h"

namespace tsgls {

// ---------------------------------------------------------------- geometry
// grad N_a (node 0 at the parent origin, xi_k = N_k), w = V/4 per point.
__global__ void k_geometry(const double* __restrict__ xyz, const int32_t* __restrict__ conn,
                           double* __restrict__ geo, int64_t E) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  double X[4][3];
  for (int b = 0; b < 4; ++b) {
    const int64_t nd = conn[e * 4 + b];
    for (int i = 0; i < 3; ++i) X[b][i] = xyz[nd * 3 + i];
  }
  double d[3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) d[k][i] = X[k + 1][i] - X[0][i];
  // rows of J^{-1}: cross products of the other two edge vectors / det
  double cr[3][3];
  for (int k = 0; k < 3; ++k) {
    const double* p = d[(k + 1) % 3];
    const double* q = d[(k + 2) % 3];
    cr[k][0] = p[1] * q[2] - p[2] * q[1];
    cr[k][1] = p[2] * q[0] - p[0] * q[2];
    cr[k][2] = p[0] * q[1] - p[1] * q[0];
  }
  const double det = d[0][0] * cr[0][0] + d[0][1] * cr[0][1] + d[0][2] * cr[0][2];
  double* g = geo + e * 16;
  for (int i = 0; i < 3; ++i) {
    const double g1 = cr[0][i] / det, g2 = cr[1][i] / det, g3 = cr[2][i] / det;
    g[3 + i] = g1;
    g[6 + i] = g2;
    g[9 + i] = g3;
    g[i] = -(g1 + g2 + g3);
  }
  g[12] = det / 24.0;
  g[13] = g[14] = g[15] = 0.0;
}

hipError_t launch_geometry(const double* xyz, const int32_t* conn, double* geo, int*,
                           int64_t E, hipStream_t st) {
  if (E == 0) return hipSuccess;
  k_geometry<<<(unsigned)((E + 255) / 256), 256, 0, st>>>(xyz, conn, geo, E);
  return hipGetLastError();
}

// ------------------------------------------------------- nodal time samples
// XT[node][j][s] = u_j(t_s) for the three velocity components.
template <int K>
__global__ void k_prep_time(const double* __restrict__ Y, const uint8_t* __restrict__ nflag,
                            int masked, const double* __restrict__ F, double* __restrict__ XT,
                            int64_t nn) {
  constexpr int n = Dim<K>::n, S = Dim<K>::S, M = Dim<K>::M;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nn * 3) return;
  const int64_t node = idx / 3;
  const int j = (int)(idx % 3);
  const bool zero = masked && (nflag[node] & 1);
  double x[n];
  const double* ys = Y + (node * 4 + j) * S;
#pragma unroll
  for (int a = 0; a < n; ++a) x[a] = zero ? 0.0 : slot_x(ys, a);
  double* o = XT + idx * M;
#pragma unroll
  for (int s = 0; s < M; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) acc = fma(x[a], F[a * M + s], acc);
    o[s] = acc;
  }
}

// ---------------------------------------------------------------------- tau
// One group of NP lanes per (element, quadrature point).  Lane c builds
// column c of S = sum_i A(u_i) A(v_i) + C_I nu^2 (G:G) I, v_i = G_ij u_j
// (eq. 3D-tau), the group runs one-sided Jacobi on the columns, and
// tau = S^(-1/2) = sum_c lambda_c^(-1/2) v_c v_c^T with v_c = w_c / lambda_c.
template <int K>
struct TauCfg {
  static constexpr int n = Dim<K>::n, M = Dim<K>::M;
  static constexpr int NP = np_of(n);
  static constexpr int per_group = 6 * n + 6 * M + n * n;   // doubles of LDS
  static constexpr int G0 = 256 / NP;
  static constexpr int Gmem = 49152 / (per_group * 8);
  static constexpr int G = G0 < Gmem ? G0 : (Gmem < 1 ? 1 : Gmem);
  static constexpr int BLOCK = G * NP < 64 ? 64 : G * NP;
  static constexpr int GB = BLOCK / NP;   // groups per block after rounding up
};

template <int K>
__global__ void __launch_bounds__(TauCfg<K>::BLOCK)
k_tau(DevView v, const double* __restrict__ Y, double* __restrict__ tau) {
  using C = TauCfg<K>;
  constexpr int n = C::n, M = C::M, S = Dim<K>::S, NP = C::NP, P = Dim<K>::P, GB = C::GB;
  __shared__ double sU[GB][3][n], sVv[GB][3][n], sUt[GB][3][M], sVt[GB][3][M], sQ[GB][n * n];
  const double* __restrict__ F = v.F;
  const int g = threadIdx.x / NP;
  const int c = threadIdx.x % NP;
  const int64_t gq = (int64_t)blockIdx.x * GB + g;
  const int64_t e = gq >> 2;
  const int q = (int)(gq & 3);
  const bool valid = e < v.n_tets;
  double dN[4][3];
  double wq = 0.0;
  int nodes[4] = {0, 0, 0, 0};
  if (valid) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      nodes[b] = v.conn[e * 4 + b];
#pragma unroll
      for (int i = 0; i < 3; ++i) dN[b][i] = v.geo[e * 16 + b * 3 + i];
    }
    wq = v.geo[e * 16 + 12];
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 3; ++i) dN[b][i] = 0.0;
  }
  (void)wq;
  double Gm[3][3];
  double GG = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Gm[i][j] = dN[1][i] * dN[1][j] + dN[2][i] * dN[2][j] + dN[3][i] * dN[3][j];
      GG += Gm[i][j] * Gm[i][j];
    }
  const double nu = v.mu / v.rho;
  const double kap = v.C_I * nu * nu * GG;
  if (valid && c < n) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) acc += lamq(q, b) * slot_x(Y + ((int64_t)nodes[b] * 4 + j) * S, c);
      sU[g][j][c] = acc;
    }
  }
  __syncthreads();
  if (valid && c < n) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      sVv[g][i][c] = Gm[i][0] * sU[g][0][c] + Gm[i][1] * sU[g][1][c] + Gm[i][2] * sU[g][2][c];
  }
  __syncthreads();
  if (valid) {
    for (int s = c; s < M; s += NP) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double au = 0.0, av = 0.0;
#pragma unroll
        for (int a = 0; a < n; ++a) {
          au = fma(sU[g][j][a], F[a * M + s], au);
          av = fma(sVv[g][j][a], F[a * M + s], av);
        }
        sUt[g][j][s] = au;
        sVt[g][j][s] = av;
      }
    }
  }
  __syncthreads();
  double w[n];
#pragma unroll
  for (int a = 0; a < n; ++a) w[a] = 0.0;
  if (valid && c < n) {
    const double invM = 1.0 / M;
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      // b = A(v_i) e_c : project v_i(t) phi_c(t) on the K harmonics
      double bb[n];
#pragma unroll
      for (int a = 0; a < n; ++a) bb[a] = 0.0;
#pragma unroll 1
      for (int s = 0; s < M; ++s) {
        const double t = sVt[g][i][s] * F[c * M + s] * invM;
#pragma unroll
        for (int a = 0; a < n; ++a) bb[a] = fma(t, F[a * M + s], bb[a]);
      }
      // w += A(u_i) b
#pragma unroll 1
      for (int s = 0; s < M; ++s) {
        double yb = 0.0;
#pragma unroll
        for (int a = 0; a < n; ++a) yb = fma(bb[a], F[a * M + s], yb);
        const double t = sUt[g][i][s] * yb * invM;
#pragma unroll
        for (int a = 0; a < n; ++a) w[a] = fma(t, F[a * M + s], w[a]);
      }
    }
#pragma unroll
    for (int a = 0; a < n; ++a)
      if (a == c) w[a] += kap;
  }
  jacobi_columns<n, NP>(w, c);
  double l2 = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a) l2 = fma(w[a], w[a], l2);
  const double lam = sqrt(l2);
  if (valid && c < n) {
    const double sc = lam > 0.0 ? pow(lam, -1.25) : 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) sQ[g][c * n + a] = w[a] * sc;
  }
  __syncthreads();
  if (valid) {
    double* out = tau + (e * 4 + q) * P;
    for (int p = c; p < P; p += NP) {
      int r, cc;
      packed_rc<n>(p, r, cc);
      double acc = 0.0;
#pragma unroll 4
      for (int k = 0; k < n; ++k) acc = fma(sQ[g][k * n + r], sQ[g][k * n + cc], acc);
      out[p] = acc;
    }
  }
}

// ------------------------------------------------------- element operator
// One tile of TE elements of the same colour per block; phases over index
// spaces (element, time sample), (element, qp, field), (element, row),
// (element, node, field).  The output is accumulated into `out` with plain
// read-modify-write: elements of one colour share no node.
template <int K, int MODE>
struct ElemCfg {
  static constexpr int n = Dim<K>::n, M = Dim<K>::M;
  static constexpr bool NEWTON = (MODE & MODE_NEWTON) != 0;
  static constexpr bool NOLS = (MODE & MODE_NOLS) != 0;
  static constexpr int per = 13 + 16 * n + 12 * M + (NEWTON ? 12 * M : 0) + 24 * n +
                             (NOLS ? 12 * n : 0) + 9 * M;
  static constexpr int NT = 128;
  static constexpr int TE0 = 40960 / (per * 8);
  static constexpr int TE = TE0 < 1 ? 1 : (TE0 > 16 ? 16 : TE0);
};

template <int K, int MODE>
__global__ void __launch_bounds__(128)
k_elem(DevView v, const double* __restrict__ Y, const double* __restrict__ VT,
       double* __restrict__ Zout, double* __restrict__ out, double shift, int64_t begin,
       int64_t end) {
  using C = ElemCfg<K, MODE>;
  constexpr int n = Dim<K>::n, M = Dim<K>::M, S = Dim<K>::S, P = Dim<K>::P;
  constexpr int TE = C::TE, NT = C::NT;
  constexpr bool RESID = (MODE & MODE_RESID) != 0;
  constexpr bool NEWTON = C::NEWTON, NOLS = C::NOLS;
  constexpr bool STOREZ = (MODE & MODE_STOREZ) != 0;
  __shared__ double sGeo[TE][13];
  __shared__ int sNode[TE][4];
  __shared__ double sV[TE][4][4][n];
  __shared__ double sT[TE][12][M];
  __shared__ double sZT[NEWTON ? TE : 1][12][M];
  __shared__ double sL[TE][12][n];
  __shared__ double sZ[TE][12][n];
  __shared__ double sZc[NOLS ? TE : 1][12][n];
  __shared__ double sW[TE][9][M];
  const double* __restrict__ F = v.F;
  const double* __restrict__ UT = v.UT;
  const int tid = threadIdx.x;
  const int64_t e0 = begin + (int64_t)blockIdx.x * TE;
  const int ne = (int)((end - e0) < TE ? (end - e0) : TE);
  const double rho = v.rho, omega = v.omega;
  const double invM = 1.0 / M;

  for (int i = tid; i < ne * 4; i += NT) sNode[i >> 2][i & 3] = v.conn[(e0 + (i >> 2)) * 4 + (i & 3)];
  for (int i = tid; i < ne * 13; i += NT) sGeo[i / 13][i % 13] = v.geo[(e0 + i / 13) * 16 + i % 13];
  __syncthreads();

  // gather the modal input in the orthonormal basis
  for (int i = tid; i < ne * 16 * n; i += NT) {
    const int e = i / (16 * n);
    const int r = i % (16 * n);
    const int b = r / (4 * n), f = (r / n) & 3, a = r % n;
    const int node = sNode[e][b];
    double val;
    if (!RESID && f < 3 && (v.nflag[node] & 1))
      val = 0.0;
    else
      val = slot_x(Y + ((int64_t)node * 4 + f) * S, a);
    sV[e][b][f][a] = val;
  }

  // convection products on the time samples: conv_i(q,t) = u_j d_j du_i (+ du_j d_j u_i)
  for (int i = tid; i < ne * M; i += NT) {
    const int e = i / M, s = i % M;
    double U[4][3], W[4][3], dN[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t node = sNode[e][b];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        U[b][j] = UT[(node * 3 + j) * M + s];
        W[b][j] = RESID ? U[b][j] : VT[(node * 3 + j) * M + s];
        dN[b][j] = sGeo[e][b * 3 + j];
      }
    }
    double gW[3][3], gU[3][3], sUj[3], sWj[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      sUj[j] = U[0][j] + U[1][j] + U[2][j] + U[3][j];
      sWj[j] = W[0][j] + W[1][j] + W[2][j] + W[3][j];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        gW[j][ii] = dN[0][j] * W[0][ii] + dN[1][j] * W[1][ii] + dN[2][j] * W[2][ii] + dN[3][j] * W[3][ii];
        gU[j][ii] = dN[0][j] * U[0][ii] + dN[1][j] * U[1][ii] + dN[2][j] * U[2][ii] + dN[3][j] * U[3][ii];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double uq[3], wq[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        uq[j] = TS_QB * sUj[j] + (TS_QA - TS_QB) * U[q][j];
        wq[j] = TS_QB * sWj[j] + (TS_QA - TS_QB) * W[q][j];
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        double cv = uq[0] * gW[0][ii] + uq[1] * gW[1][ii] + uq[2] * gW[2][ii];
        if (NEWTON) cv += wq[0] * gU[0][ii] + wq[1] * gU[1][ii] + wq[2] * gU[2][ii];
        sT[e][q * 3 + ii][s] = cv;
      }
    }
  }
  __syncthreads();

  // per (element, qp, field): back to modes, momentum operator L, z = tau L, z(t)
  for (int i = tid; i < ne * 12; i += NT) {
    const int e = i / 12, row = i % 12, q = row / 3, fi = row % 3;
    double cm[n];
#pragma unroll
    for (int a = 0; a < n; ++a) cm[a] = 0.0;
#pragma unroll 2
    for (int s = 0; s < M; ++s) {
      const double t = sT[e][row][s];
#pragma unroll
      for (int a = 0; a < n; ++a) cm[a] = fma(t, F[a * M + s], cm[a]);
    }
    double du[n], gp[n], gal[n];
    const double g0 = sGeo[e][0 * 3 + fi], g1 = sGeo[e][1 * 3 + fi];
    const double g2 = sGeo[e][2 * 3 + fi], g3 = sGeo[e][3 * 3 + fi];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      du[a] = TS_QB * (sV[e][0][fi][a] + sV[e][1][fi][a] + sV[e][2][fi][a] + sV[e][3][fi][a]) +
              (TS_QA - TS_QB) * sV[e][q][fi][a];
      gp[a] = g0 * sV[e][0][3][a] + g1 * sV[e][1][3][a] + g2 * sV[e][2][3][a] + g3 * sV[e][3][3][a];
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      gal[a] = rho * (omx<n>(du, a, omega) + cm[a] * invM);
      sL[e][row][a] = gal[a];
    }
    const double* tp = v.tau + ((e0 + e) * 4 + q) * P;
    double z[n], zc[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      z[a] = 0.0;
      zc[a] = 0.0;
    }
    {
      int p = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
#pragma unroll
        for (int b = a; b < n; ++b) {
          const double t = tp[p++];
          const double La = NOLS ? gal[a] : gal[a] + gp[a];
          const double Lb = NOLS ? gal[b] : gal[b] + gp[b];
          z[a] = fma(t, Lb, z[a]);
          if (b != a) z[b] = fma(t, La, z[b]);
          if (NOLS) {
            zc[a] = fma(t, gp[b], zc[a]);
            if (b != a) zc[b] = fma(t, gp[a], zc[b]);
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      sZ[e][row][a] = z[a];
      if (NOLS) sZc[e][row][a] = zc[a];
    }
    if (STOREZ) {
      double* zo = Zout + (((e0 + e) * 4 + q) * 3 + fi) * n;
#pragma unroll
      for (int a = 0; a < n; ++a) zo[a] = z[a];
    }
#pragma unroll 2
    for (int s = 0; s < M; ++s) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc = fma(z[a], F[a * M + s], acc);
      sT[e][row][s] = acc;
    }
    if (NEWTON) {
      const double* zf = v.Z + (((e0 + e) * 4 + q) * 3 + fi) * n;
      double Zm[n];
#pragma unroll
      for (int a = 0; a < n; ++a) Zm[a] = zf[a];
#pragma unroll 2
      for (int s = 0; s < M; ++s) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < n; ++a) acc = fma(Zm[a], F[a * M + s], acc);
        sZT[NEWTON ? e : 0][row][s] = acc;
      }
    }
  }
  __syncthreads();

  // least-squares test products: W_ji(t) = sum_q w u_j(q,t) z_i(q,t) (+ du_j Z_i)
  for (int i = tid; i < ne * M; i += NT) {
    const int e = i / M, s = i % M;
    double U[4][3], W[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t node = sNode[e][b];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        U[b][j] = UT[(node * 3 + j) * M + s];
        W[b][j] = NEWTON ? VT[(node * 3 + j) * M + s] : 0.0;
      }
    }
    const double wgt = sGeo[e][12];
    double acc[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) acc[r] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double uq[3], wq[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        uq[j] = TS_QB * (U[0][j] + U[1][j] + U[2][j] + U[3][j]) + (TS_QA - TS_QB) * U[q][j];
        wq[j] = TS_QB * (W[0][j] + W[1][j] + W[2][j] + W[3][j]) + (TS_QA - TS_QB) * W[q][j];
      }
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const double zt = sT[e][q * 3 + ii][s];
        const double Zt = NEWTON ? sZT[NEWTON ? e : 0][q * 3 + ii][s] : 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          acc[j * 3 + ii] = fma(uq[j], zt, acc[j * 3 + ii]);
          if (NEWTON) acc[j * 3 + ii] = fma(wq[j], Zt, acc[j * 3 + ii]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) sW[e][r][s] = wgt * acc[r];
  }
  __syncthreads();

  // back to modes; stored over the sT tile (9 n <= 12 M)
  for (int i = tid; i < ne * 9; i += NT) {
    const int e = i / 9, r = i % 9;
    double acc[n];
#pragma unroll
    for (int a = 0; a < n; ++a) acc[a] = 0.0;
#pragma unroll 2
    for (int s = 0; s < M; ++s) {
      const double t = sW[e][r][s];
#pragma unroll
      for (int a = 0; a < n; ++a) acc[a] = fma(t, F[a * M + s], acc[a]);
    }
    double* wm = &sT[e][0][0];
#pragma unroll
    for (int a = 0; a < n; ++a) wm[r * n + a] = acc[a] * invM;
  }
  __syncthreads();

  // assemble per (element, node, field) and add to the global vector
  const double mu = v.mu;
  for (int i = tid; i < ne * 16; i += NT) {
    const int e = i >> 4, b = (i >> 2) & 3, f = i & 3;
    const int64_t node = sNode[e][b];
    if (f < 3 && (v.nflag[node] & 1)) continue;
    const double* dN = &sGeo[e][0];        // dN[c*3 + j]
    const double wgt = sGeo[e][12];
    const double* wm = &sT[e][0][0];
    double o[n];
    if (f < 3) {
      const int fi = f;
      double lw[4], visc[4], mass[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) lw[q] = wgt * lamq(q, b);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        visc[c] = 4.0 * wgt * mu * (dN[b * 3] * dN[c * 3] + dN[b * 3 + 1] * dN[c * 3 + 1] + dN[b * 3 + 2] * dN[c * 3 + 2]);
        const double mbc = (b == c) ? (TS_QA * TS_QA + 3.0 * TS_QB * TS_QB)
                                    : (2.0 * TS_QA * TS_QB + 2.0 * TS_QB * TS_QB);
        mass[c] = shift * wgt * mbc;
      }
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc += lw[q] * (sL[e][q * 3 + fi][a] - omx<n>(&sZ[e][q * 3 + fi][0], a, omega));
        acc += dN[b * 3] * wm[(0 * 3 + fi) * n + a] + dN[b * 3 + 1] * wm[(1 * 3 + fi) * n + a] +
               dN[b * 3 + 2] * wm[(2 * 3 + fi) * n + a];
        const double psum = sV[e][0][3][a] + sV[e][1][3][a] + sV[e][2][3][a] + sV[e][3][3][a];
        acc -= dN[b * 3 + fi] * wgt * psum;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc += (visc[c] + mass[c]) * sV[e][c][fi][a];
        o[a] = acc;
      }
    } else {
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double div = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          div += dN[c * 3] * sV[e][c][0][a] + dN[c * 3 + 1] * sV[e][c][1][a] + dN[c * 3 + 2] * sV[e][c][2][a];
        double ls = 0.0;
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          double zs = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) zs += NOLS ? sZc[NOLS ? e : 0][q * 3 + ii][a] : sZ[e][q * 3 + ii][a];
          ls += dN[b * 3 + ii] * zs;
        }
        o[a] = wgt * div + (wgt / rho) * ls;
      }
    }
    double* op = out + (node * 4 + f) * S;
    op[0] += o[0];
#pragma unroll
    for (int a = 1; a < n; ++a) op[a + 1] += o[a] * TS_RS2;
  }
}

// ------------------------------------------------------- Jacobi diagonal
// Diagonal of the Picard tangent (eq. K_mat): per (element, node)
//  momentum: sum_q w [rho lam A(g)_aa + mu |grad N|^2 + rho b_a^T tau b_a + shift lam^2],
//            g = grad N_b . u(q,t), b_a = lam Omega e_a + A(g) e_a;
//  continuity: sum_q (w/rho) |grad N|^2 tau_aa.
template <int K>
__global__ void __launch_bounds__(128)
k_diag(DevView v, double* __restrict__ d, double shift, int64_t begin, int64_t end) {
  constexpr int n = Dim<K>::n, M = Dim<K>::M, S = Dim<K>::S, P = Dim<K>::P;
  const int64_t idx = begin * 4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= end * 4) return;
  const int64_t e = idx >> 2;
  const int b = (int)(idx & 3);
  const int64_t node = v.conn[e * 4 + b];
  const double dNb[3] = {v.geo[e * 16 + b * 3 + 0], v.geo[e * 16 + b * 3 + 1], v.geo[e * 16 + b * 3 + 2]};
  const double wgt = v.geo[e * 16 + 12];
  const double gn2 = dNb[0] * dNb[0] + dNb[1] * dNb[1] + dNb[2] * dNb[2];
  int nodes[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) nodes[c] = v.conn[e * 4 + c];
  const double* __restrict__ F = v.F;
  const double invM = 1.0 / M;
  double dm[n], dc[n];
#pragma unroll
  for (int a = 0; a < n; ++a) dm[a] = dc[a] = 0.0;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const double lam = lamq(q, b);
    double gs[M];
#pragma unroll 1
    for (int s = 0; s < M; ++s) {
      double gsum = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double* ut = v.UT + (int64_t)nodes[c] * 3 * M + s;
        gsum += lamq(q, c) * (dNb[0] * ut[0] + dNb[1] * ut[M] + dNb[2] * ut[2 * M]);
      }
      gs[s] = gsum;
    }
    const double* tp = v.tau + (e * 4 + q) * P;
#pragma unroll 1
    for (int a = 0; a < n; ++a) {
      double bcol[n];
#pragma unroll
      for (int aa = 0; aa < n; ++aa) bcol[aa] = 0.0;
#pragma unroll 1
      for (int s = 0; s < M; ++s) {
        const double t = gs[s] * F[a * M + s] * invM;
#pragma unroll
        for (int aa = 0; aa < n; ++aa) bcol[aa] = fma(t, F[aa * M + s], bcol[aa]);
      }
      double Aaa = 0.0;
#pragma unroll
      for (int aa = 0; aa < n; ++aa)
        if (aa == a) Aaa = bcol[aa];
      // + lam Omega e_a
      if (a > 0) {
        const int k = (a + 1) >> 1;
        const double om = k * v.omega * lam;
#pragma unroll
        for (int aa = 0; aa < n; ++aa) {
          if ((a & 1) && aa == a + 1) bcol[aa] += om;        // Omega e_{2k-1} = k w e_{2k}
          if (!(a & 1) && aa == a - 1) bcol[aa] -= om;       // Omega e_{2k} = -k w e_{2k-1}
        }
      }
      double quad = 0.0, taa = 0.0;
      int p = 0;
#pragma unroll
      for (int r = 0; r < n; ++r) {
#pragma unroll
        for (int c = r; c < n; ++c) {
          const double t = tp[p++];
          quad += (r == c ? 1.0 : 2.0) * t * bcol[r] * bcol[c];
          if (r == c && r == a) taa = t;
        }
      }
      const double vm = wgt * (v.rho * lam * Aaa + v.mu * gn2 + v.rho * quad + shift * lam * lam);
      const double vc = (wgt / v.rho) * gn2 * taa;
#pragma unroll
      for (int aa = 0; aa < n; ++aa)
        if (aa == a) {
          dm[aa] += vm;
          dc[aa] += vc;
        }
    }
  }
  double* op = d + node * 4 * S;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double* o = op + f * S;
    const double* src = f < 3 ? dm : dc;
    o[0] += src[0];
#pragma unroll
    for (int a = 1; a < n; ++a) o[a + 1] += src[a];
  }
}

template <int K>
__global__ void k_diag_finish(const uint8_t* __restrict__ nflag, double* __restrict__ d, int64_t nn) {
  constexpr int S = Dim<K>::S;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nn * 4 * S) return;
  const int64_t node = idx / (4 * S);
  const int f = (int)((idx / S) % 4), s = (int)(idx % S);
  if (s == 1 || (f < 3 && (nflag[node] & 1)) || d[idx] == 0.0) d[idx] = 1.0;
}

// --------------------------------------------------------------- dispatch
#define TSGLS_FOR_EACH_K(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(11) X(15)

bool supported_K(int K) {
  switch (K) {
#define CASE(k) case k: return true;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return false;
  }
}

int supported_K_list(int* out, int cap) {
  int cnt = 0;
#define ADD(k) if (out && cnt < cap) out[cnt] = k; ++cnt;
  TSGLS_FOR_EACH_K(ADD)
#undef ADD
  return cnt;
}

hipError_t launch_prep_time(int K, const double* Y, const uint8_t* nflag, int masked,
                            const double* F, double* XT, int64_t nn, hipStream_t st) {
  const unsigned grid = (unsigned)((nn * 3 + 255) / 256);
  if (nn == 0) return hipSuccess;
  switch (K) {
#define CASE(k) case k: k_prep_time<k><<<grid, 256, 0, st>>>(Y, nflag, masked, F, XT, nn); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tau(const DevView& v, const double* Y, double* tau, hipStream_t st) {
  if (v.n_tets == 0) return hipSuccess;
  switch (v.K) {
#define CASE(k)                                                                          \
  case k: {                                                                              \
    const int64_t groups = v.n_tets * 4;                                                 \
    const unsigned grid = (unsigned)((groups + TauCfg<k>::GB - 1) / TauCfg<k>::GB);      \
    k_tau<k><<<grid, TauCfg<k>::BLOCK, 0, st>>>(v, Y, tau);                              \
    break;                                                                               \
  }
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K>
static void elem_dispatch(const DevView& v, int mode, const double* Y, const double* VT,
                          double* Zout, double* out, double shift, int64_t begin, int64_t end,
                          hipStream_t st) {
#define LAUNCH(MD)                                                                       \
  {                                                                                      \
    constexpr int TE = ElemCfg<K, MD>::TE;                                               \
    const unsigned grid = (unsigned)((end - begin + TE - 1) / TE);                       \
    k_elem<K, MD><<<grid, 128, 0, st>>>(v, Y, VT, Zout, out, shift, begin, end);         \
  }
  switch (mode) {
    case MODE_RESID: LAUNCH(MODE_RESID) break;
    case MODE_RESID | MODE_STOREZ: LAUNCH(MODE_RESID | MODE_STOREZ) break;
    case 0: LAUNCH(0) break;
    case MODE_NOLS: LAUNCH(MODE_NOLS) break;
    case MODE_NEWTON: LAUNCH(MODE_NEWTON) break;
    default: break;
  }
#undef LAUNCH
}

hipError_t launch_elem(const DevView& v, int mode, const double* Y, const double* VT,
                       double* Zout, double* out, double shift, int64_t begin, int64_t end,
                       hipStream_t st) {
  if (end <= begin) return hipSuccess;
  switch (v.K) {
#define CASE(k) case k: elem_dispatch<k>(v, mode, Y, VT, Zout, out, shift, begin, end, st); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_diag(const DevView& v, double* d, double shift, int64_t begin, int64_t end,
                       hipStream_t st) {
  if (end <= begin) return hipSuccess;
  const unsigned grid = (unsigned)(((end - begin) * 4 + 127) / 128);
  switch (v.K) {
#define CASE(k) case k: k_diag<k><<<grid, 128, 0, st>>>(v, d, shift, begin, end); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_diag_finish(int K, const uint8_t* nflag, double* d, int64_t nn, hipStream_t st) {
  const int64_t tot = nn * 4 * (2 * K + 2);
  if (tot == 0) return hipSuccess;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  switch (K) {
#define CASE(k) case k: k_diag_finish<k><<<grid, 256, 0, st>>>(nflag, d, nn); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tsgls
