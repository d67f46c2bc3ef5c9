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
  constexpr SampleTable<K> TB{};
#pragma unroll
  for (int s = 0; s < M; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) acc = fma(x[a], TB.f[a][s], acc);
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
  constexpr SampleTable<K> TB{};
  const int g = threadIdx.x / NP;
  const int c = threadIdx.x % NP;
  const int64_t gq = xcd_block(blockIdx.x, gridDim.x) * GB + g;
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
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      // b = A(v_i) e_c : project v_i(t) phi_c(t) on the K harmonics
      double bb[n];
#pragma unroll
      for (int a = 0; a < n; ++a) bb[a] = 0.0;
#pragma unroll
      for (int s = 0; s < M; ++s) {
        const double t = sVt[g][i][s] * F[c * M + s];
#pragma unroll
        for (int a = 0; a < n; ++a) bb[a] = fma(t, TB.b[a][s], bb[a]);
      }
      // w += A(u_i) b
#pragma unroll
      for (int s = 0; s < M; ++s) {
        double yb = 0.0;
#pragma unroll
        for (int a = 0; a < n; ++a) yb = fma(bb[a], TB.f[a][s], yb);
        const double t = sUt[g][i][s] * yb;
#pragma unroll
        for (int a = 0; a < n; ++a) w[a] = fma(t, TB.b[a][s], w[a]);
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
    const int64_t slot = v.tslot[e];
    for (int p = c; p < P; p += NP) {
      int r, cc;
      packed_rc<n>(p, r, cc);
      double acc = 0.0;
#pragma unroll 4
      for (int k = 0; k < n; ++k) acc = fma(sQ[g][k * n + r], sQ[g][k * n + cc], acc);
      tau[tau_index(slot, q, p, P, v.TE)] = acc;
    }
  }
}

// ------------------------------------------------------- element operator
// One element per wave (block of 64 lanes).  The lanes are mapped over each
// phase's own index space; the element's intermediates live in wave-private
// LDS, so there is no cross-wave synchronisation and many independent waves
// per CU hide each other's memory latency.
//   gather      (node, field, mode)     modal input, orthonormal basis
//   products    (sample, component)     conv_i(q,t) = u_j d_j du_i (+ du_j d_j u_i)
//   to modes    MFMA                    [16 x M] x [M x n]
//   operator    (row, mode)             gal = rho Omega du + rho conv, L = gal + dp
//   tau apply   (row, mode)             z = tau L (packed tau staged in LDS)
//   to samples  MFMA                    [16 x n] x [n x M]
//   LS products (sample, direction j)   W_ji(t) = sum_q w u_j(q,t) z_i(q,t)
//   to modes    MFMA
//   assembly    (node, field, mode)     then a coalesced read-modify-write
// Rows are (qp q, component i) -> q*3 + i.  Elements of one colour share no
// node, so the read-modify-write needs no atomics.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int K>
struct TileCfg {
  static constexpr int TE = 1;                    // tau / Z storage: one element per tile
};

template <int K, int MODE>
struct ElemCfg {
  static constexpr int n = Dim<K>::n, M = Dim<K>::M, S = Dim<K>::S, P = Dim<K>::P;
  static constexpr bool NEWTON = (MODE & MODE_NEWTON) != 0;
  static constexpr bool NOLS = (MODE & MODE_NOLS) != 0;
  static constexpr int MS = (M + 3) / 4 * 4;      // padded samples (k of back transform)
  static constexpr int NS = (n + 3) / 4 * 4;      // padded modes (k of forward transform)
  static constexpr int NCT = (n + 15) / 16;       // column tiles over modes
  static constexpr int MCT = (M + 15) / 16;       // column tiles over samples
  static constexpr int MX1 = 16 * MS > 4 * P ? 16 * MS : 4 * P;
  static constexpr int XR = MX1 > 16 * S ? MX1 : 16 * S;   // tau -> W(t) -> output slots
};

template <int K, int MODE>
__global__ void __launch_bounds__(64)
k_elem(DevView v, const double* __restrict__ Y, const double* __restrict__ VT,
       double* __restrict__ Zout, double* __restrict__ out, double shift, int64_t begin,
       int64_t end, int64_t tile_off) {
  using C = ElemCfg<K, MODE>;
  constexpr int n = C::n, M = C::M, S = C::S, P = C::P, MS = C::MS, NS = C::NS;
  constexpr int NCT = C::NCT, MCT = C::MCT;
  constexpr bool RESID = (MODE & MODE_RESID) != 0;
  constexpr bool NEWTON = C::NEWTON, NOLS = C::NOLS;
  constexpr bool STOREZ = (MODE & MODE_STOREZ) != 0;
  __shared__ double sV[4][4][n];          // modal input [node][field][mode]
  __shared__ double sT[16][MS];           // conv(t) -> z(t) -> W modes [16][n]
  __shared__ double sC[16][n];            // conv modes
  __shared__ double sX[C::XR];            // packed tau [p][q] -> W(t) [16][MS] -> output
  __shared__ double sZ[16][NS];           // z modes, zero beyond n
  __shared__ double sL[12][n];            // momentum operator L (or gal for NOLS)
  __shared__ double sG[12][n];            // gal, then gal - Omega z
  __shared__ double sLc[NOLS ? 12 : 1][n];   // grad p alone (NOLS)
  __shared__ double sZc[NOLS ? 12 : 1][n];
  __shared__ double sZT[NEWTON ? 16 : 1][MS];
  __shared__ double sZf[NEWTON ? 16 : 1][NS];
  __shared__ double sD[4][3];             // grad N (lane-dependent lookups)
  __shared__ int64_t sN[4];
  // `out` receives this element's contributions [4 nodes][4 fields][S]
  (void)end;
  (void)tile_off;
  const int lane = threadIdx.x;
  const int64_t e = begin + xcd_block(blockIdx.x, gridDim.x);
  const double rho = v.rho, omega = v.omega;

  // element data (uniform across the wave)
  int64_t nd[4];
  double dN[4][3];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    nd[b] = v.conn[e * 4 + b];
#pragma unroll
    for (int j = 0; j < 3; ++j) dN[b][j] = v.geo[e * 16 + b * 3 + j];
  }
  const double wgt = v.geo[e * 16 + 12];

  // per-lane B fragments of the sampling matrices
  double Bb[MS / 4][NCT];   // back: B[k=s][j=a] = phi_a(t_s) / M
  double Bf[NS / 4][MCT];   // forward: B[k=a][j=s] = phi_a(t_s)
  {
    const double invM = 1.0 / M;
#pragma unroll
    for (int ks = 0; ks < MS / 4; ++ks)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int s = ks * 4 + (lane >> 4), a = ct * 16 + (lane & 15);
        Bb[ks][ct] = (s < M && a < n) ? v.F[a * M + s] * invM : 0.0;
      }
#pragma unroll
    for (int ks = 0; ks < NS / 4; ++ks)
#pragma unroll
      for (int ct = 0; ct < MCT; ++ct) {
        const int a = ks * 4 + (lane >> 4), s = ct * 16 + (lane & 15);
        Bf[ks][ct] = (s < M && a < n) ? v.F[a * M + s] : 0.0;
      }
  }

  // tau of the element: contiguous [p][q]; loads issued now, stored later
  constexpr int NTAU = (4 * P + 63) / 64;
  double taubuf[NTAU];
  {
    const double* src = v.tau + e * (int64_t)(4 * P);
#pragma unroll
    for (int k = 0; k < NTAU; ++k) {
      const int i = lane + k * 64;
      taubuf[k] = i < 4 * P ? src[i] : 0.0;
    }
  }
  // gather the modal input (all loads issued before the stores)
  {
    constexpr int NIT = (16 * n + 63) / 64;
    double buf[NIT];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int i = lane + k * 64;
      double val = 0.0;
      if (i < 16 * n) {
        const int b = i / (4 * n), f = (i / n) & 3, a = i % n;
        const int64_t node = v.conn[e * 4 + b];
        const double* ys = Y + (node * 4 + f) * S;
        val = a == 0 ? ys[0] : TS_SQ2 * ys[a + 1];
        if (!RESID && f < 3 && (v.nflag[node] & 1)) val = 0.0;
      }
      buf[k] = val;
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int i = lane + k * 64;
      if (i < 16 * n) (&sV[0][0][0])[i] = buf[k];
    }
  }
  if (lane < 4) sN[lane] = nd[lane];
  if (lane < 12) sD[lane / 3][lane % 3] = v.geo[e * 16 + lane];
  // zero padding entering the MFMA k dimension
  for (int i = lane; i < 16 * MS; i += 64) (&sT[0][0])[i] = 0.0;
  for (int i = lane; i < 16 * NS; i += 64) (&sZ[0][0])[i] = 0.0;
  if (NEWTON)
    for (int i = lane; i < 16 * NS; i += 64) (&sZf[0][0])[i] = 0.0;
  __syncthreads();

  // convection products on the samples: item (sample s, component i)
  const double* __restrict__ UT = v.UT;
  for (int it = lane; it < 3 * M; it += 64) {
    const int s = it % M, ii = it / M;
    double U[4][3], Wi[4], Ui[4], Wj[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        U[b][j] = UT[(nd[b] * 3 + j) * M + s];
        Wj[b][j] = RESID ? U[b][j] : (NEWTON ? VT[(nd[b] * 3 + j) * M + s] : 0.0);
      }
      Ui[b] = UT[(nd[b] * 3 + ii) * M + s];
      Wi[b] = RESID ? Ui[b] : VT[(nd[b] * 3 + ii) * M + s];
    }
    double gW[3], gU[3], sU[3], sW[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gW[j] = dN[0][j] * Wi[0] + dN[1][j] * Wi[1] + dN[2][j] * Wi[2] + dN[3][j] * Wi[3];
      gU[j] = dN[0][j] * Ui[0] + dN[1][j] * Ui[1] + dN[2][j] * Ui[2] + dN[3][j] * Ui[3];
      sU[j] = U[0][j] + U[1][j] + U[2][j] + U[3][j];
      sW[j] = Wj[0][j] + Wj[1][j] + Wj[2][j] + Wj[3][j];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double cv = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double uq = TS_QB * sU[j] + (TS_QA - TS_QB) * U[q][j];
        cv = fma(uq, gW[j], cv);
        if (NEWTON) {
          const double wq = TS_QB * sW[j] + (TS_QA - TS_QB) * Wj[q][j];
          cv = fma(wq, gU[j], cv);
        }
      }
      sT[q * 3 + ii][s] = cv;
    }
  }
#pragma unroll
  for (int k = 0; k < NTAU; ++k) {
    const int i = lane + k * 64;
    if (i < 4 * P) sX[i] = taubuf[k];
  }
  __syncthreads();

  // conv(t) -> modes (MFMA)
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < MS / 4; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[lane & 15][ks * 4 + (lane >> 4)], Bb[ks][ct], acc, 0, 0, 0);
    const int a = ct * 16 + (lane & 15);
    if (a < n) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sC[(lane >> 4) + 4 * r][a] = acc[r];
    }
  }
  __syncthreads();

  // momentum operator per (row, mode)
  for (int it = lane; it < 12 * n; it += 64) {
    const int row = it / n, a = it % n, q = row / 3, fi = row % 3;
    double om = 0.0;   // (Omega du)_a from du at the neighbouring mode
    if (a > 0) {
      const int a2 = (a & 1) ? a + 1 : a - 1;
      const double du2 = TS_QB * (sV[0][fi][a2] + sV[1][fi][a2] + sV[2][fi][a2] + sV[3][fi][a2]) +
                         (TS_QA - TS_QB) * sV[q][fi][a2];
      om = (a & 1) ? -((a + 1) >> 1) * omega * du2 : (a >> 1) * omega * du2;
    }
    const double gal = rho * (om + sC[row][a]);
    const double gp = dN[0][fi] * sV[0][3][a] + dN[1][fi] * sV[1][3][a] + dN[2][fi] * sV[2][3][a] +
                      dN[3][fi] * sV[3][3][a];
    sG[row][a] = gal;
    sL[row][a] = NOLS ? gal : gal + gp;
    if (NOLS) sLc[NOLS ? row : 0][a] = gp;
  }
  __syncthreads();

  // z = tau L per (row, mode); packed tau in sX as [p][q]
  for (int it = lane; it < 12 * n; it += 64) {
    const int row = it / n, a = it % n, q = row / 3, fi = row % 3;
    double z = 0.0, zc = 0.0;
#pragma unroll
    for (int b = 0; b < n; ++b) {
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      const double t = sX[(lo * n - (lo * (lo - 1)) / 2 + (hi - lo)) * 4 + q];
      z = fma(t, sL[row][b], z);
      if (NOLS) zc = fma(t, sLc[NOLS ? row : 0][b], zc);
    }
    sZ[row][a] = z;
    if (NOLS) sZc[NOLS ? row : 0][a] = zc;
    if (STOREZ) Zout[z_index(e, row, a, n, 1)] = z;
    if (NEWTON) sZf[NEWTON ? row : 0][a] = v.Z[z_index(e, row, a, n, 1)];
    (void)fi;
  }
  __syncthreads();

  // gal - Omega z (per (row, mode)) and z modes -> samples (MFMA)
  for (int it = lane; it < 12 * n; it += 64) {
    const int row = it / n, a = it % n;
    if (a > 0) {
      const int a2 = (a & 1) ? a + 1 : a - 1;
      const double z2 = sZ[row][a2];
      sG[row][a] -= (a & 1) ? -((a + 1) >> 1) * omega * z2 : (a >> 1) * omega * z2;
    }
  }
#pragma unroll
  for (int w = 0; w < (NEWTON ? 2 : 1); ++w) {
#pragma unroll
    for (int ct = 0; ct < MCT; ++ct) {
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NS / 4; ++ks) {
        const double av = (w == 0) ? sZ[lane & 15][ks * 4 + (lane >> 4)]
                                   : sZf[NEWTON ? (lane & 15) : 0][ks * 4 + (lane >> 4)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bf[ks][ct], acc, 0, 0, 0);
      }
      const int s = ct * 16 + (lane & 15);
      if (s < M) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (w == 0)
            sT[(lane >> 4) + 4 * r][s] = acc[r];
          else
            sZT[NEWTON ? (lane >> 4) + 4 * r : 0][s] = acc[r];
        }
      }
    }
  }
  __syncthreads();

  // least-squares test products per (sample, direction j); W(t) in sX as [16][MS]
  for (int i = lane; i < 16 * MS; i += 64) sX[i] = 0.0;
  __syncthreads();
  for (int it = lane; it < 3 * M; it += 64) {
    const int s = it % M, j = it / M;
    double Uj[4], Wj[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      Uj[b] = UT[(nd[b] * 3 + j) * M + s];
      Wj[b] = NEWTON ? VT[(nd[b] * 3 + j) * M + s] : 0.0;
    }
    const double su = Uj[0] + Uj[1] + Uj[2] + Uj[3];
    const double sw = Wj[0] + Wj[1] + Wj[2] + Wj[3];
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double uq = TS_QB * su + (TS_QA - TS_QB) * Uj[q];
      const double wq = TS_QB * sw + (TS_QA - TS_QB) * Wj[q];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        acc[ii] = fma(uq, sT[q * 3 + ii][s], acc[ii]);
        if (NEWTON) acc[ii] = fma(wq, sZT[NEWTON ? q * 3 + ii : 0][s], acc[ii]);
      }
    }
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) sX[(j * 3 + ii) * MS + s] = wgt * acc[ii];
  }
  __syncthreads();

  // W(t) -> modes (MFMA), rows j*3 + i, stored over sT as [16][n]
  double* wm = &sT[0][0];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < MS / 4; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[(lane & 15) * MS + ks * 4 + (lane >> 4)], Bb[ks][ct], acc, 0, 0, 0);
    const int a = ct * 16 + (lane & 15);
    __syncthreads();   // all A fragments of sT were read before sT is overwritten
    if (a < n) {
#pragma unroll
      for (int r = 0; r < 4; ++r) wm[((lane >> 4) + 4 * r) * n + a] = acc[r];
    }
  }
  __syncthreads();

  // assembly per (node, field, mode) into output slots (sX as [16][S])
  const double mu = v.mu;
  for (int it = lane; it < 16 * n; it += 64) {
    const int b = it / (4 * n), f = (it / n) & 3, a = it % n;
    double o;
    if (f < 3) {
      const int fi = f;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc += wgt * lamq(q, b) * sG[q * 3 + fi][a];
      acc += sD[b][0] * wm[(0 * 3 + fi) * n + a] + sD[b][1] * wm[(1 * 3 + fi) * n + a] +
             sD[b][2] * wm[(2 * 3 + fi) * n + a];
      const double psum = sV[0][3][a] + sV[1][3][a] + sV[2][3][a] + sV[3][3][a];
      acc -= sD[b][fi] * wgt * psum;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double mbc = (b == c) ? (TS_QA * TS_QA + 3.0 * TS_QB * TS_QB)
                                    : (2.0 * TS_QA * TS_QB + 2.0 * TS_QB * TS_QB);
        const double kbc = 4.0 * wgt * mu * (sD[b][0] * dN[c][0] + sD[b][1] * dN[c][1] + sD[b][2] * dN[c][2]) +
                           shift * wgt * mbc;
        acc += kbc * sV[c][fi][a];
      }
      o = (v.nflag[sN[b]] & 1) ? 0.0 : acc;
    } else {
      double div = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) div += dN[c][0] * sV[c][0][a] + dN[c][1] * sV[c][1][a] + dN[c][2] * sV[c][2][a];
      double ls = 0.0;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        double zs = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) zs += NOLS ? sZc[NOLS ? q * 3 + ii : 0][a] : sZ[q * 3 + ii][a];
        ls += sD[b][ii] * zs;
      }
      o = wgt * div + (wgt / rho) * ls;
    }
    double* so = &sX[(b * 4 + f) * S];
    if (a == 0) {
      so[0] = o;
      so[1] = 0.0;
    } else {
      so[a + 1] = o * TS_RS2;
    }
  }
  __syncthreads();

  // the element's 4 x 4 x S contributions, one contiguous coalesced store
  for (int i = lane; i < 16 * S; i += 64) out[e * (16 * S) + i] = sX[i];
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
  const int64_t idx = begin * 4 + xcd_block(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
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
  constexpr SampleTable<K> TB{};
  double dm[n], dc[n];
#pragma unroll
  for (int a = 0; a < n; ++a) dm[a] = dc[a] = 0.0;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const double lam = lamq(q, b);
    double gs[M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
      double gsum = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double* ut = v.UT + (int64_t)nodes[c] * 3 * M + s;
        gsum += lamq(q, c) * (dNb[0] * ut[0] + dNb[1] * ut[M] + dNb[2] * ut[2 * M]);
      }
      gs[s] = gsum;
    }
    const int64_t slot = v.tslot[e];
#pragma unroll 1
    for (int a = 0; a < n; ++a) {
      double bcol[n];
#pragma unroll
      for (int aa = 0; aa < n; ++aa) bcol[aa] = 0.0;
#pragma unroll
      for (int s = 0; s < M; ++s) {
        const double t = gs[s] * v.F[a * M + s];
#pragma unroll
        for (int aa = 0; aa < n; ++aa) bcol[aa] = fma(t, TB.b[aa][s], bcol[aa]);
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
          const double t = v.tau[tau_index(slot, q, p++, P, v.TE)];
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
  (void)node;
  double* op = d + (e * 4 + b) * 4 * S;      // this element's node-b contributions
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double* o = op + f * S;
    const double* src = f < 3 ? dm : dc;
    o[0] = src[0];
    o[1] = 0.0;
#pragma unroll
    for (int a = 1; a < n; ++a) o[a + 1] = src[a];
  }
}

// Node-wise sum of element contributions (ascending element order): thread
// per (node, slot of the node's 4 S values).
template <int K>
__global__ void k_gather(const int32_t* __restrict__ noff, const int32_t* __restrict__ ninc,
                         const double* __restrict__ ebuf, double* __restrict__ out, int64_t nn) {
  constexpr int S4 = 4 * Dim<K>::S;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nn * S4) return;
  const int64_t node = idx / S4;
  const int j = (int)(idx % S4);
  const int k0 = noff[node], k1 = noff[node + 1];
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) acc += ebuf[(int64_t)ninc[k] * S4 + j];
  out[idx] = acc;
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

int tile_elems(int K) {
  switch (K) {
#define CASE(k) case k: return TileCfg<k>::TE;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return 1;
  }
}

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
                          int64_t tile_off, hipStream_t st) {
#define LAUNCH(MD)                                                                       \
  {                                                                                      \
    const unsigned grid = (unsigned)(end - begin);                                       \
    k_elem<K, MD><<<grid, 64, 0, st>>>(v, Y, VT, Zout, out, shift, begin, end, tile_off); \
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
                       int64_t tile_off, hipStream_t st) {
  if (end <= begin) return hipSuccess;
  switch (v.K) {
#define CASE(k) case k: elem_dispatch<k>(v, mode, Y, VT, Zout, out, shift, begin, end, tile_off, st); break;
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

hipError_t launch_gather(int K, const int32_t* noff, const int32_t* ninc, const double* ebuf,
                         double* out, int64_t nn, hipStream_t st) {
  const int64_t tot = nn * 4 * (2 * K + 2);
  if (tot == 0) return hipSuccess;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  switch (K) {
#define CASE(k) case k: k_gather<k><<<grid, 256, 0, st>>>(noff, ninc, ebuf, out, nn); break;
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
