// gfx950 kernels of the volume terms: element geometry, time samples of the
// nodal velocity, the stabilization matrix tau per quadrature point, the
// Jacobi diagonal and the per-node sum of element contributions.  The GLS
// element operator itself is in elemop.hip.
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
#include "face_point.cuh"
#include "internal.h"

namespace tsgls {

typedef double dbl4 __attribute__((ext_vector_type(4)));

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
// One wave per node (a block of four waves loops over nodes).  Lane
// (field f, position p) writes XP[node][f][p] = mode pos_mode(p) of field f
// in the orthonormal basis; then lane (j, s) forms XT[node][j][s] = u_j(t_s)
// from the modes staged in LDS.  masked != 0 zeroes Dirichlet velocity rows;
// Ys, when given, scales the input entrywise (input = Y * Ys).  Blocks from
// nbp on each form one Neumann face point of the same input (no separate
// launch for the face points of a tangent product).
template <int K, typename TO>
__global__ void __launch_bounds__(256)
k_prep_time(const double* __restrict__ Y, const double* __restrict__ Ys,
            const uint8_t* __restrict__ nflag, int masked, const double* __restrict__ F,
            TO* __restrict__ XT, TO* __restrict__ XP, int64_t nn, int64_t nbp, DevView fv,
            const double* __restrict__ aneg, int fresid, SegMask mk) {
  constexpr int n = Dim<K>::n, S = Dim<K>::S, M = Dim<K>::M, PW = (n + 15) / 16 * 16;
  constexpr int NPT = PW / 16, NR = (3 * M + 63) / 64;
  constexpr bool HOIST = NR == 1;          // the lane's column of F stays in registers
  __shared__ double sx[4][4 * PW];
  if (blockIdx.x >= nbp) {                 // a face point (uniform per block)
    static_assert(3 * n <= 256 && 3 * n <= 16 * PW, "face point lanes and LDS");
    face_point_block<K>(fv, Y, Ys, fresid, aneg, (int64_t)blockIdx.x - nbp, threadIdx.x, &sx[0][0]);
    return;
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int sj[NR], ss[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int it = lane + 64 * r < 3 * M ? lane + 64 * r : 0;
    sj[r] = it / M;
    ss[r] = it % M;
  }
  double Fl[HOIST ? n : 1];
  if (HOIST) {
#pragma unroll
    for (int a = 0; a < n; ++a) Fl[HOIST ? a : 0] = F[a * M + ss[0]];
  }
  const int64_t stride = nbp * 4;
  // the trip count is the same for the four waves of a block (barriers below)
  for (int64_t base = (int64_t)blockIdx.x * 4; base < nn; base += stride) {
    const int64_t node = base + wv;
    const bool act = node < nn && !(mk.skip && mk.skip[(uint32_t)node / (uint32_t)mk.nodes]);
    const bool zero = act && masked && (nflag[node] & 1);
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int fp = pt * 64 + lane, f = fp / PW, pp = fp % PW;
      const int a = pos_mode(pp, K);
      double x = 0.0;
      if (act && a >= 0 && !(zero && f < 3)) {
        const int64_t o = (node * 4 + f) * S + (a == 0 ? 0 : a + 1);
        x = (a == 0 ? 1.0 : TS_SQ2) * (Ys ? Y[o] * Ys[o] : Y[o]);
      }
      if (act) XP[node * (4 * PW) + fp] = TO(x);
      sx[wv][fp] = x;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (act && lane + 64 * r < 3 * M) {
        const double* xr = sx[wv] + sj[r] * PW;
        double acc = 0.0;
        if constexpr (n > 32) {   // large K: bounded unrolling keeps the loads in registers
#pragma unroll 4
          for (int a = 0; a < n; ++a) acc = fma(xr[mode_pos(a, K)], F[a * M + ss[r]], acc);
        } else {
#pragma unroll
          for (int a = 0; a < n; ++a)
            acc = fma(xr[mode_pos(a, K)], HOIST ? Fl[HOIST ? a : 0] : F[a * M + ss[r]], acc);
        }
        XT[(node * 3 + sj[r]) * M + ss[r]] = TO(acc);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------- tau
// One group of NP lanes per (element, quadrature point).  Lane c builds
// column c of S = sum_i A(u_i) A(v_i) + C_I nu^2 (G:G) I, v_i = G_ij u_j
// (eq. 3D-tau), the group runs one-sided Jacobi on the columns, and
// tau = S^(-1/2) = sum_c lambda_c^(-1/2) v_c v_c^T with v_c = w_c / lambda_c.
//
// Column c on the samples: A(v_i) e_c is the band-limited part of
// v_i(t) phi_c(t), i.e. the sampled product minus its K alias harmonics
// (AliasTable); A(u_i) of that is formed the same way, and only the final
// sum over i is projected on the modes.
template <int K>
struct TauCfg {
  static constexpr int n = Dim<K>::n, M = Dim<K>::M;
  static constexpr int NP = np_of(n);              // lanes per point
  static constexpr int PW = (n + 15) / 16 * 16;    // positions, padded to the MFMA tile
  static constexpr int QW = 64 / NP;               // points per wave
  static constexpr int BLOCK = 256;
  static constexpr int GB = BLOCK / NP;            // points per block
  static constexpr bool MFMA_OUT = NP >= 16;       // tau = Q^T Q on MFMA
  static constexpr int QS = PW + 1;                // row stride of Q
  static constexpr int PH1 = 6 * n + 6 * M;        // LDS per point, first phase
  static constexpr int PH2 = MFMA_OUT ? PW * QS : n * n;   // ... output phase
  static constexpr int PG = PH1 > PH2 ? PH1 : PH2;
};

//
// Warm start (Vin not null): Vin holds orthonormal eigenvectors of S from an
// earlier linearization, [point][a][c] with column c the eigenvector of lane
// c.  The Jacobi then runs on the columns of W = S V instead of S: for any
// orthonormal V its rotations J make W J orthogonal, so V J diagonalizes S^2
// and hence S, and the same tau follows; when S changed little since V was
// taken, W is nearly orthogonal already and few sweeps remain.  Vout (not
// null) receives the new eigenvectors w_c / |w_c| in the same layout.
template <int K>
__global__ void __launch_bounds__(TauCfg<K>::BLOCK)
k_tau(DevView v, const double* __restrict__ Y, double* __restrict__ tau,
      const double* Vin, double* Vout) {   // Vin and Vout may be the same array
  using C = TauCfg<K>;
  constexpr int n = C::n, M = C::M, S = Dim<K>::S, NP = C::NP, P = Dim<K>::P, GB = C::GB;
  constexpr int PW = C::PW, QS = C::QS, QW = C::QW;
  __shared__ double lds[GB * C::PG];
  const double* __restrict__ F = v.F;
  constexpr SampleTable<K> TB{};
  constexpr AliasTable<K> AT{};
  const int g = threadIdx.x / NP;
  const int c = threadIdx.x % NP;
  double* sU = lds + g * C::PG;          // [3][n]  u_j modes at the point
  double* sVv = sU + 3 * n;              // [3][n]  v_i = G_ij u_j
  double* sUt = sVv + 3 * n;             // [3][M]  samples
  double* sVt = sUt + 3 * M;             // [3][M]
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t gq = blk * GB + g;
  const int64_t e = gq >> 2;
  const int q = (int)(gq & 3);
  // points of a segment that sits out are left as they are, like those past the end
  const bool valid = e < v.n_tets &&
                     !(v.seg.skip && v.seg.skip[(uint32_t)v.conn[e * 4] / (uint32_t)v.seg.nodes]);
  double dN[4][3];
  int nodes[4] = {0, 0, 0, 0};
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (valid) nodes[b] = v.conn[e * 4 + b];
#pragma unroll
    for (int i = 0; i < 3; ++i) dN[b][i] = valid ? v.geo[e * 16 + b * 3 + i] : 0.0;
  }
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
      sU[j * n + c] = acc;
    }
  }
  __syncthreads();
  if (valid && c < n) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      sVv[i * n + c] = Gm[i][0] * sU[c] + Gm[i][1] * sU[n + c] + Gm[i][2] * sU[2 * n + c];
  }
  __syncthreads();
  if (valid) {
    for (int s = c; s < M; s += NP) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double au = 0.0, av = 0.0;
#pragma unroll
        for (int a = 0; a < n; ++a) {
          au = fma(sU[j * n + a], F[a * M + s], au);
          av = fma(sVv[j * n + a], F[a * M + s], av);
        }
        sUt[j * M + s] = au;
        sVt[j * M + s] = av;
      }
    }
  }
  __syncthreads();
  double w[n];
#pragma unroll
  for (int a = 0; a < n; ++a) w[a] = 0.0;
  if (valid && c < n) {
    double Fc[M], Z[M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
      Fc[s] = F[c * M + s];
      Z[s] = 0.0;
    }
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      double x[M];
#pragma unroll
      for (int s = 0; s < M; ++s) x[s] = sVt[i * M + s] * Fc[s];
#pragma unroll
      for (int r = 0; r < K; ++r) {
        double d = 0.0;
#pragma unroll
        for (int s = 0; s < M; ++s) d = fma(x[s], AT.v[r][s], d);
        d *= AT.coef[r];
#pragma unroll
        for (int s = 0; s < M; ++s) x[s] = fma(-d, AT.v[r][s], x[s]);
      }
#pragma unroll
      for (int s = 0; s < M; ++s) Z[s] = fma(sUt[i * M + s], x[s], Z[s]);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < M; ++s) acc = fma(TB.b[a][s], Z[s], acc);
      w[a] = a == c ? acc + kap : acc;
    }
  }
  if (Vin) {   // w = S v_c (uniform branch)
    double* sS = lds + g * C::PG;          // S [row][col], over the first-phase arrays
    static_assert(n * n <= C::PG, "S fits the point's LDS");
    __syncthreads();
    if (valid && c < n) {
#pragma unroll
      for (int a = 0; a < n; ++a) sS[a * n + c] = w[a];
    }
    __syncthreads();
    if (valid && c < n) {
      const double* vp = Vin + gq * (n * n) + c;
      double vc[n];
#pragma unroll
      for (int b = 0; b < n; ++b) vc[b] = vp[b * n];
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < n; ++b) acc = fma(sS[a * n + b], vc[b], acc);
        w[a] = acc;
      }
    }
  }
  jacobi_columns<n, NP>(w, c);
  double l2 = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a) l2 = fma(w[a], w[a], l2);
  const double sc = l2 > 0.0 ? pow(l2, -0.625) : 0.0;   // lambda^(-5/4), lambda = |w|
  if (Vout && valid && c < n) {
    double* vp = Vout + gq * (n * n) + c;
    const double inv = l2 > 0.0 ? rsq_nr(l2) : 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) vp[a * n] = w[a] * inv;
  }
  __syncthreads();   // the first-phase arrays are reused below
  if constexpr (C::MFMA_OUT) {
    // Q[k][p] = w_k[pos_mode(p)] lambda_k^(-5/4); tau over positions = Q^T Q
    double* sQ = lds + g * C::PG;
    for (int i = c; i < PW * QS; i += NP) sQ[i] = 0.0;
    __syncthreads();
    if (valid && c < n) {
#pragma unroll
      for (int a = 0; a < n; ++a) sQ[c * QS + mode_pos(a, K)] = w[a] * sc;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, gl = lane >> 4, cl = lane & 15;
#pragma unroll 1
    for (int j = 0; j < QW; ++j) {
      const int gg = wv * QW + j;            // point of this wave
      const int64_t gqj = blk * GB + gg;
      const int64_t ej = gqj >> 2;
      if (ej >= v.n_tets) break;             // uniform across the wave
      const double* Qj = lds + gg * C::PG;
      double* tj = tau + gqj * P;
#pragma unroll
      for (int tr = 0; tr < PW / 16; ++tr)
#pragma unroll
        for (int tc = tr; tc < PW / 16; ++tc) {
          dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int ks = 0; ks < PW / 4; ++ks) {
            const double* qr = Qj + (ks * 4 + gl) * QS;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(qr[cl + 16 * tr], qr[cl + 16 * tc], acc, 0, 0, 0);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = gl + 4 * r + 16 * tr, col = cl + 16 * tc;
            if (row <= col && col < n) tj[pk_index(row, col, n)] = acc[r];
          }
        }
    }
  } else {
    double* sQ = lds + g * C::PG;
    if (valid && c < n) {
#pragma unroll
      for (int a = 0; a < n; ++a) sQ[c * n + a] = w[a] * sc;
    }
    __syncthreads();
    if (valid) {
      // packed over positions: entry (pr, pc) is tau between modes
      // pos_mode(pr) and pos_mode(pc)
      for (int p = c; p < P; p += NP) {
        int pr, pc;
        packed_rc<n>(p, pr, pc);
        const int r = pos_mode(pr, K), cc = pos_mode(pc, K);
        double acc = 0.0;
#pragma unroll 4
        for (int k = 0; k < n; ++k) acc = fma(sQ[k * n + r], sQ[k * n + cc], acc);
        tau[(e * 4 + q) * P + p] = acc;
      }
    }
  }
}

// ------------------------------------------------------- Jacobi diagonal
// Triple products of the real orthonormal basis, (1/T) int phi_r phi_m phi_a
// dt, exact from the M = 3K+1 samples (the integrand has degree <= 3K);
// entries that vanish in exact arithmetic are stored as exact zeros, so the
// fully unrolled use below keeps only the (at most two per (r, a)) nonzero
// terms.  A(g) e_a = sum_m g_m T[r][m][a] over output modes r.
template <int K>
struct TripleTable {
  static constexpr int n = 2 * K + 1, M = 3 * K + 1;
  double t[n][n][n];
  constexpr TripleTable() : t() {
    const SampleTable<K> tb{};
    for (int r = 0; r < n; ++r)
      for (int m = 0; m < n; ++m)
        for (int a = 0; a < n; ++a) {
          double acc = 0.0;
          for (int s = 0; s < M; ++s) acc += tb.f[r][s] * tb.f[m][s] * tb.f[a][s];
          acc /= M;
          t[r][m][a] = (acc < 1e-12 && acc > -1e-12) ? 0.0 : acc;
        }
  }
};

// Diagonal of the Picard tangent (eq. K_mat): per (element, node)
//  momentum: sum_q w [rho lam A(g)_aa + mu |grad N|^2 + rho b_a^T tau b_a + shift lam^2],
//            g = grad N_b . u(q,t), b_a = lam Omega e_a + A(g) e_a;
//  continuity: sum_q (w/rho) |grad N|^2 tau_aa.
// For K <= 6 the modes of g are formed once per point and A(g) e_a from the
// triple table (O(n^2) per point instead of O(n^2 M)), with the point's
// packed tau held in registers; larger K keep the sampled form.
template <int K>
__global__ void __launch_bounds__(128)
k_diag(DevView v, double* __restrict__ d, double shift, int64_t begin, int64_t end) {
  constexpr int n = Dim<K>::n, M = Dim<K>::M, S = Dim<K>::S, P = Dim<K>::P;
  constexpr bool MODAL = K <= 6;
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
    const double* tq = v.tau + (e * 4 + q) * P;
    if constexpr (MODAL) {
      constexpr TripleTable<K> T3{};
      double gh[n], tr[P];
#pragma unroll
      for (int m = 0; m < n; ++m) {
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < M; ++s) acc = fma(TB.b[m][s], gs[s], acc);
        gh[m] = acc;
      }
#pragma unroll
      for (int i = 0; i < P; ++i) tr[i] = tq[i];
#pragma unroll
      for (int a = 0; a < n; ++a) {
        double bcol[n];
#pragma unroll
        for (int r = 0; r < n; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < n; ++m)
            if (T3.t[r][m][a] != 0.0) acc = fma(T3.t[r][m][a], gh[m], acc);
          bcol[r] = acc;
        }
        const double Aaa = bcol[a];
        if (a > 0) {   // + lam Omega e_a
          const int k = (a + 1) >> 1;
          const double om = k * v.omega * lam;
          if (a & 1) bcol[a + 1] += om;        // Omega e_{2k-1} = k w e_{2k}
          else bcol[a - 1] -= om;              // Omega e_{2k} = -k w e_{2k-1}
        }
        // b^T tau b = sum_r b_r (tau_rr b_r + 2 sum_{c > r} tau_rc b_c)
        double quad = 0.0;
#pragma unroll
        for (int r = 0; r < n; ++r) {
          double off = 0.0;
#pragma unroll
          for (int c = r + 1; c < n; ++c) {
            const int pr = mode_pos(r, K), pc = mode_pos(c, K);
            off = fma(tr[pr < pc ? pk_index(pr, pc, n) : pk_index(pc, pr, n)], bcol[c], off);
          }
          const int pp = mode_pos(r, K);
          quad = fma(bcol[r], fma(2.0, off, tr[pk_index(pp, pp, n)] * bcol[r]), quad);
        }
        const int pa = mode_pos(a, K);
        const double taa = tr[pk_index(pa, pa, n)];
        dm[a] += wgt * (v.rho * lam * Aaa + v.mu * gn2 + v.rho * quad + shift * lam * lam);
        dc[a] += (wgt / v.rho) * gn2 * taa;
        __builtin_amdgcn_sched_barrier(0);   // one mode at a time: bounds the live registers
      }
      continue;
    }
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
#pragma unroll
      for (int r = 0; r < n; ++r) {
#pragma unroll
        for (int c = r; c < n; ++c) {
          const int pr = mode_pos(r, K), pc = mode_pos(c, K);
          const double t = tq[pr < pc ? pk_index(pr, pc, n) : pk_index(pc, pr, n)];
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
  double* op = d + (e * 4 + b) * 4 * n;      // node b's rows [field][position]
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double* o = op + f * n;
    const double* src = f < 3 ? dm : dc;
#pragma unroll
    for (int a = 0; a < n; ++a) o[mode_pos(a, K)] = src[a];
  }
}

// Node-wise sum of element contributions (ascending element order): one
// wave per node, lane j < 4S producing slot j of the node's output from the
// incident element rows [node][field][position] (slot 1, Im c_0, is zero);
// the incidence list is read with scalar loads.
template <int K, typename TE>
__global__ void __launch_bounds__(256)
k_gather(const int32_t* __restrict__ noff, const int32_t* __restrict__ ninc,
         const uint8_t* __restrict__ nflag, const TE* __restrict__ ebuf,
         double* __restrict__ out, int64_t nn, FaceSum fs, SegMask mk) {
  constexpr int n = Dim<K>::n, S = Dim<K>::S, S4 = 4 * S, R = 4 * n;
  constexpr int NJ = (S4 + 63) / 64;
  const int64_t node = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (node >= nn) return;
  const int lane = threadIdx.x & 63;
  if (mk.skip && mk.skip[(uint32_t)node / (uint32_t)mk.nodes]) {   // segment sitting out
#pragma unroll
    for (int r = 0; r < NJ; ++r)
      if (lane + 64 * r < S4) out[node * S4 + lane + 64 * r] = 0.0;
    return;
  }
  const int k0 = noff[node], k1 = noff[node + 1];
  const bool dir = (nflag[node] & 1) != 0;
  int src[NJ];        // offset of slot j inside an element row, -1 for Im c_0
#pragma unroll
  for (int r = 0; r < NJ; ++r) {
    const int j = lane + 64 * r, f = j / S, sl = j % S;
    src[r] = (j >= S4 || sl == 1) ? -1 : f * n + (sl == 0 ? 2 * K : sl - 2);
  }
  double acc[NJ];
#pragma unroll
  for (int r = 0; r < NJ; ++r) acc[r] = 0.0;
  int k = k0;
  // eight rows in flight, then four, then one: the sum runs over the rows in
  // ascending order whatever the blocking
  for (; k + 8 <= k1; k += 8) {
    int64_t ii[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ii[u] = (int64_t)ninc[k + u] * R;
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
      if (src[r] >= 0) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = ebuf[ii[u] + src[r]];   // FP64 sum
        double t = acc[r];
#pragma unroll
        for (int u = 0; u < 8; ++u) t = t + a[u];
        acc[r] = t;
      }
    }
  }
  for (; k + 4 <= k1; k += 4) {
    const int64_t i0 = (int64_t)ninc[k] * R, i1 = (int64_t)ninc[k + 1] * R;
    const int64_t i2 = (int64_t)ninc[k + 2] * R, i3 = (int64_t)ninc[k + 3] * R;
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
      if (src[r] >= 0) {
        const double a0 = ebuf[i0 + src[r]], a1 = ebuf[i1 + src[r]];
        const double a2 = ebuf[i2 + src[r]], a3 = ebuf[i3 + src[r]];   // FP64 sum
        acc[r] = (((acc[r] + a0) + a1) + a2) + a3;
      }
    }
  }
  for (; k < k1; ++k) {
    const int64_t i0 = (int64_t)ninc[k] * R;
#pragma unroll
    for (int r = 0; r < NJ; ++r)
      if (src[r] >= 0) acc[r] += ebuf[i0 + src[r]];
  }
  // face terms of a Neumann node: per slot of the leading fs.nfield fields
  // (velocity, or the tracer), the sum over its incident faces (ascending) of
  // the three face points weighted by the vertex's P1 value there, minus the
  // traction term for the residual
  const int u = (fs.nfidx && !dir) ? fs.nfidx[node] : -1;
  if (u >= 0) {
    const int f0 = fs.foff[u], f1 = fs.foff[u + 1];
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
      const int j = lane + 64 * r, i = j / S, sl = j % S;
      if (j < fs.nfield * S && sl != 1) {
        const int m = sl == 0 ? 0 : sl - 1;
        double o = 0.0;
        for (int kf = f0; kf < f1; ++kf) {
          const int64_t f = fs.finc[kf] / 3;
          const int a = fs.finc[kf] % 3;
          const double* y = fs.fy + f * 3 * (3 * n) + i * n + m;
          o += flam(0, a) * y[0] + flam(1, a) * y[3 * n] + flam(2, a) * y[6 * n];
          if (fs.resid && fs.fh) o -= fs.fgeo[f * 4 + 3] / 3.0 * fs.fh[f * n + m] * fs.fgeo[f * 4 + i];
        }
        acc[r] += m == 0 ? o : o * TS_RS2;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NJ; ++r) {
    const int j = lane + 64 * r;
    if (j < S4) out[node * S4 + j] = (dir && j < 3 * S) ? 0.0 : acc[r];
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

// ------------------------------------------------------ tau, large K
// tau for n = 2K+1 > 32: one wave per (element, quadrature point).  Lane c
// forms column c of S = sum_i A(u_i) A(v_i) + C_I nu^2 (G:G) I as
// A(u_i) (A(v_i) e_c), each product applied on the M = 3K+1 samples:
// A(x) y = (1/M) sum_s phi(t_s) x(t_s) y(t_s), exact for band-limited x and
// y (the integrand has degree <= 3K).  The sample table is read with
// wave-uniform indices (scalar loads).  Then the one-sided Jacobi on the
// columns and tau = Q^T Q on MFMA, as in k_tau.
template <int K>
__global__ void __launch_bounds__(64)
k_tau_big(DevView v, const double* __restrict__ Y, double* __restrict__ tau) {
  constexpr int n = Dim<K>::n, M = Dim<K>::M, S = Dim<K>::S, P = Dim<K>::P;
  constexpr int PW = (n + 15) / 16 * 16, QS = PW + 1;
  static_assert(n <= 64 && PW <= 64, "one lane per column");
  __shared__ double sX[6 * M];          // u_j(t_s), then v_i(t_s)
  __shared__ double sQ[PW * QS];        // modes of u_j, v_i; then Q
  const double* __restrict__ F = v.F;
  const int c = threadIdx.x;
  const int64_t gq = xcd_block(blockIdx.x, gridDim.x);
  const int64_t e = gq >> 2;
  const int q = (int)(gq & 3);
  if (e >= v.n_tets) return;                      // uniform over the block
  double dN[4][3];
  int nodes[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    nodes[b] = v.conn[e * 4 + b];
#pragma unroll
    for (int i = 0; i < 3; ++i) dN[b][i] = v.geo[e * 16 + b * 3 + i];
  }
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
  double* sUm = sQ;            // [3][n]
  double* sVm = sQ + 3 * n;    // [3][n]
  if (c < n) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) acc += lamq(q, b) * slot_x(Y + ((int64_t)nodes[b] * 4 + j) * S, c);
      sUm[j * n + c] = acc;
    }
  }
  __syncthreads();
  if (c < n) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      sVm[i * n + c] = Gm[i][0] * sUm[c] + Gm[i][1] * sUm[n + c] + Gm[i][2] * sUm[2 * n + c];
  }
  __syncthreads();
  for (int s = c; s < M; s += 64) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double au = 0.0, av = 0.0;
      for (int a = 0; a < n; ++a) {
        au = fma(sUm[j * n + a], F[a * M + s], au);
        av = fma(sVm[j * n + a], F[a * M + s], av);
      }
      sX[j * M + s] = au;
      sX[(3 + j) * M + s] = av;
    }
  }
  __syncthreads();
  const double invM = 1.0 / M;
  double w[n];
#pragma unroll
  for (int a = 0; a < n; ++a) w[a] = 0.0;
  if (c < n) {
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      double y[n];                       // A(v_i) e_c
#pragma unroll
      for (int a = 0; a < n; ++a) y[a] = 0.0;
#pragma unroll 1
      for (int s = 0; s < M; ++s) {
        const double t = sX[(3 + i) * M + s] * F[c * M + s] * invM;
#pragma unroll
        for (int a = 0; a < n; ++a) y[a] = fma(t, F[a * M + s], y[a]);
      }
#pragma unroll 1
      for (int s = 0; s < M; ++s) {      // w += A(u_i) y
        double ys = 0.0;
#pragma unroll
        for (int a = 0; a < n; ++a) ys = fma(y[a], F[a * M + s], ys);
        const double t = sX[i * M + s] * ys * invM;
#pragma unroll
        for (int a = 0; a < n; ++a) w[a] = fma(t, F[a * M + s], w[a]);
      }
    }
#pragma unroll
    for (int a = 0; a < n; ++a)
      if (a == c) w[a] += kap;
  }
  jacobi_columns<n, 64>(w, c);
  double l2 = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a) l2 = fma(w[a], w[a], l2);
  const double sc = l2 > 0.0 ? pow(l2, -0.625) : 0.0;   // lambda^(-5/4), lambda = |w|
  __syncthreads();
  // Q[k][p] = w_k[pos_mode(p)] lambda_k^(-5/4); tau over positions = Q^T Q
  for (int i = c; i < PW * QS; i += 64) sQ[i] = 0.0;
  __syncthreads();
  if (c < n) {
#pragma unroll
    for (int a = 0; a < n; ++a) sQ[c * QS + mode_pos(a, K)] = w[a] * sc;
  }
  __syncthreads();
  const int gl = c >> 4, cl = c & 15;
  double* tj = tau + gq * P;
#pragma unroll 1
  for (int tr = 0; tr < PW / 16; ++tr)
#pragma unroll 1
    for (int tc = tr; tc < PW / 16; ++tc) {
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < PW / 4; ++ks) {
        const double* qr = sQ + (ks * 4 + gl) * QS;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(qr[cl + 16 * tr], qr[cl + 16 * tc], acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = gl + 4 * r + 16 * tr, col = cl + 16 * tc;
        if (row <= col && col < n) tj[pk_index(row, col, n)] = acc[r];
      }
    }
}

// ------------------------------------------- Jacobi diagonal, large K
// One wave per (element, node b); lane a < n forms, per point,
// b_a = A(g) e_a + lam Omega e_a with g = grad N_b . u(q, t) on the samples
// (A(g) e_a = (1/M) sum_s phi(t_s) g(t_s) phi_a(t_s)) and the quadratic form
// b_a^T tau b_a with tau's packed entries read by wave-uniform index.
template <int K>
__global__ void __launch_bounds__(64)
k_diag_big(DevView v, double* __restrict__ d, double shift, int64_t begin, int64_t end) {
  constexpr int n = Dim<K>::n, M = Dim<K>::M, P = Dim<K>::P;
  static_assert(n <= 64, "one lane per mode");
  __shared__ double sg[M];
  const int64_t idx = begin * 4 + xcd_block(blockIdx.x, gridDim.x);
  if (idx >= end * 4) return;                       // uniform over the block
  const int64_t e = idx >> 2;
  const int b = (int)(idx & 3);
  const int a = threadIdx.x;
  const double dNb[3] = {v.geo[e * 16 + b * 3 + 0], v.geo[e * 16 + b * 3 + 1], v.geo[e * 16 + b * 3 + 2]};
  const double wgt = v.geo[e * 16 + 12];
  const double gn2 = dNb[0] * dNb[0] + dNb[1] * dNb[1] + dNb[2] * dNb[2];
  int nodes[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) nodes[c] = v.conn[e * 4 + c];
  const double* __restrict__ F = v.F;
  const double invM = 1.0 / M;
  double dm = 0.0, dc = 0.0;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const double lam = lamq(q, b);
    for (int s = a; s < M; s += 64) {
      double gsum = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double* ut = v.UT + (int64_t)nodes[c] * 3 * M + s;
        gsum += lamq(q, c) * (dNb[0] * ut[0] + dNb[1] * ut[M] + dNb[2] * ut[2 * M]);
      }
      sg[s] = gsum;
    }
    __syncthreads();
    if (a < n) {
      double bc[n];
#pragma unroll
      for (int r = 0; r < n; ++r) bc[r] = 0.0;
#pragma unroll 1
      for (int s = 0; s < M; ++s) {
        const double t = sg[s] * F[a * M + s] * invM;
#pragma unroll
        for (int r = 0; r < n; ++r) bc[r] = fma(t, F[r * M + s], bc[r]);
      }
      double Aaa = 0.0;
#pragma unroll
      for (int r = 0; r < n; ++r)
        if (r == a) Aaa = bc[r];
      if (a > 0) {   // + lam Omega e_a
        const int k = (a + 1) >> 1;
        const double om = k * v.omega * lam;
#pragma unroll
        for (int r = 0; r < n; ++r) {
          if ((a & 1) && r == a + 1) bc[r] += om;        // Omega e_{2k-1} = k w e_{2k}
          if (!(a & 1) && r == a - 1) bc[r] -= om;       // Omega e_{2k} = -k w e_{2k-1}
        }
      }
      const double* tq = v.tau + (e * 4 + q) * P;
      double quad = 0.0;
#pragma unroll
      for (int r = 0; r < n; ++r) {
        double off = 0.0;
#pragma unroll
        for (int c = r + 1; c < n; ++c) {
          const int pr = mode_pos(r, K), pc = mode_pos(c, K);
          off = fma(tq[pr < pc ? pk_index(pr, pc, n) : pk_index(pc, pr, n)], bc[c], off);
        }
        const int pp = mode_pos(r, K);
        quad = fma(bc[r], fma(2.0, off, tq[pk_index(pp, pp, n)] * bc[r]), quad);
      }
      const int pa = mode_pos(a, K);
      const double taa = tq[pk_index(pa, pa, n)];
      dm += wgt * (v.rho * lam * Aaa + v.mu * gn2 + v.rho * quad + shift * lam * lam);
      dc += (wgt / v.rho) * gn2 * taa;
    }
    __syncthreads();
  }
  if (a < n) {
    double* op = d + (e * 4 + b) * 4 * n;      // node b's rows [field][position]
    const int pa = mode_pos(a, K);
#pragma unroll
    for (int f = 0; f < 4; ++f) op[f * n + pa] = f < 3 ? dm : dc;
  }
}

// --------------------------------------------------------------- dispatch

int pos_width(int K) { return (2 * K + 1 + 15) / 16 * 16; }

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

template <typename TO>
static hipError_t prep_launch(int K, const double* Y, const double* Ys, const uint8_t* nflag,
                              int masked, const double* F, TO* XT, TO* XP, int64_t nn,
                              hipStream_t st, const DevView* fv, const double* aneg, int fresid,
                              const SegMask& mk) {
  if (nn == 0) return hipSuccess;
  int64_t nb = (nn + 3) / 4;
  if (nb > 8192) nb = 8192;
  const int64_t nfq = (fv && fv->n_faces > 0 && fv->n_fnodes > 0) ? fv->n_faces * 3 : 0;
  const DevView dv = fv ? *fv : DevView{};
  const unsigned grid = (unsigned)(nb + nfq);
  switch (K) {
#define CASE(k)                                                                                  \
  case k:                                                                                        \
    k_prep_time<k, TO><<<grid, 256, 0, st>>>(Y, Ys, nflag, masked, F, XT, XP, nn, nb, dv, aneg,   \
                                             fresid, mk);                                        \
    break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prep_time(int K, const double* Y, const double* Ys, const uint8_t* nflag,
                            int masked, const double* F, double* XT, double* XP, int64_t nn,
                            hipStream_t st, const DevView* fv, const double* aneg, int fresid,
                            const SegMask& mk) {
  return prep_launch<double>(K, Y, Ys, nflag, masked, F, XT, XP, nn, st, fv, aneg, fresid, mk);
}

hipError_t launch_prep_time_f32(int K, const double* Y, const double* Ys, const uint8_t* nflag,
                                int masked, const double* F, float* XT, float* XP, int64_t nn,
                                hipStream_t st, const DevView* fv, const double* aneg, int fresid,
                                const SegMask& mk) {
  return prep_launch<float>(K, Y, Ys, nflag, masked, F, XT, XP, nn, st, fv, aneg, fresid, mk);
}

hipError_t launch_tau(const DevView& v, const double* Y, double* tau, hipStream_t st,
                      const double* Vin, double* Vout) {
  if (v.n_tets == 0) return hipSuccess;
  switch (v.K) {
#define CASE(k)                                                                          \
  case k: {                                                                              \
    const int64_t groups = v.n_tets * 4;                                                 \
    const unsigned grid = (unsigned)((groups + TauCfg<k>::GB - 1) / TauCfg<k>::GB);      \
    k_tau<k><<<grid, TauCfg<k>::BLOCK, 0, st>>>(v, Y, tau, Vin, Vout);                  \
    break;                                                                               \
  }
    TSGLS_FOR_EACH_K_SMALL(CASE)
#undef CASE
#define CASE(k) case k: k_tau_big<k><<<(unsigned)(v.n_tets * 4), 64, 0, st>>>(v, Y, tau); break;
    TSGLS_FOR_EACH_K_LARGE(CASE)
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
    TSGLS_FOR_EACH_K_SMALL(CASE)
#undef CASE
#define CASE(k) case k: k_diag_big<k><<<(unsigned)((end - begin) * 4), 64, 0, st>>>(v, d, shift, begin, end); break;
    TSGLS_FOR_EACH_K_LARGE(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(int K, const int32_t* noff, const int32_t* ninc, const uint8_t* nflag,
                         const double* ebuf, double* out, int64_t nn, hipStream_t st,
                         const FaceSum& fs, const SegMask& mk) {
  const int64_t tot = nn * 4 * (2 * K + 2);
  if (tot == 0) return hipSuccess;
  const unsigned grid = (unsigned)((nn + 3) / 4);
  switch (K) {
#define CASE(k) case k: k_gather<k, double><<<grid, 256, 0, st>>>(noff, ninc, nflag, ebuf, out, nn, fs, mk); break;
    TSGLS_FOR_EACH_K(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather_f32(int K, const int32_t* noff, const int32_t* ninc, const uint8_t* nflag,
                             const float* ebuf, double* out, int64_t nn, hipStream_t st,
                             const FaceSum& fs, const SegMask& mk) {
  const int64_t tot = nn * 4 * (2 * K + 2);
  if (tot == 0) return hipSuccess;
  const unsigned grid = (unsigned)((nn + 3) / 4);
  switch (K) {
#define CASE(k) case k: k_gather<k, float><<<grid, 256, 0, st>>>(noff, ninc, nflag, ebuf, out, nn, fs, mk); break;
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
