// gfx950 element operator of the GLS method: residual of eq. Rmc and the
// tangent products of eq. tangent / eq. K_mat, element by element on linear
// tetrahedra with the 4-point rule (weights V/4).
//
// One element at a time per 64-lane wave; each wave loops over a contiguous
// Morton range of elements (the ranges are split per XCD so that elements
// sharing nodes share an L2).  Every phase uses a lane layout fixed for the
// whole kernel, so all index arithmetic is done once per wave and LDS
// addresses are a per-lane base plus compile-time offsets.  Lane l has
// g = l / 16 and c = l % 16; "positions" p = c + 16 pt index the modes
// (pos_mode), so the two modes of one harmonic are on lanes c and c ^ 1.
//
//   products   lane (s, i), s < M sample, i < 3 component:
//              conv_{q,i}(t_s) = u_q(t_s) . grad du_i(t_s) for the 4 points
//              (+ du_q . grad u_i for the Newton tangent)
//   to modes   MFMA 16x16x4: rows i*4+q, k = samples  ->  lane (q=g, p), reg i
//   modal      lane (q, p): L_i = rho (Omega du_i + conv_i) + d_i p;
//              z_i = tau_q L_i with tau_q's row p from LDS, L broadcast
//   to samples MFMA: rows q*4+i, k = positions  ->  lane (i=g, s), reg q
//   LS         lane (s, i): W_ji(t_s) = w sum_q u_{q,j} z_{q,i}
//   to modes   MFMA: rows j*4+i  ->  lane (i=g, p), reg j
//   assembly   lane (f=g, p), reg b: Galerkin, viscous, pressure, LS and
//              PSPG terms; element buffer rows [node][field][position] in
//              the slot scaling (the node gather maps positions to slots).
#include <atomic>
#include <type_traits>

#include "common.cuh"
#include "internal.h"

namespace tsgls {

// Arithmetic type of the element operator: FP64 for the residual and the
// tangent, FP32 for the mixed-precision tangent.  Both use the 16x16x4 MFMA
// with the same A/B fragments (lane l: A[l%16][l/16], B[l/16][l%16]); the
// result fragments differ: lane group g, register r hold result row
// g + 4r (FP64) or 4g + r (FP32).
template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int row(int g, int r) { return g + 4 * r; }
};
template <>
struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int row(int g, int r) { return 4 * g + r; }
};

__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int K>
struct OpCfg {
  static constexpr int n = 2 * K + 1, M = 3 * K + 1, S = 2 * K + 2, P = n * (n + 1) / 2;
  static constexpr int PW = (n + 15) / 16 * 16;   // positions per field row
  static constexpr int NPT = PW / 16;             // position tiles
  static constexpr int MS = (M + 3) / 4 * 4;      // samples padded to the MFMA k step
  static constexpr int NKB = MS / 4;              // k steps, samples -> modes
  static constexpr int MT = (M + 15) / 16;        // sample tiles, modes -> samples
  static constexpr int NKF = (n + 3) / 4;         // k steps, modes -> samples
  static constexpr int NPR = (3 * M + 63) / 64;   // passes over (sample, component)
  static constexpr int NTL = (P + 63) / 64;       // loads per packed tau block
  static constexpr bool KEEPU = NPR == 1;         // keep u_q(t_s) in registers
  // LDS row strides, odd so that rows touched by different lane rows fall
  // in different banks
  static constexpr int RP = PW + 1;               // rows over positions
  static constexpr int RS = MS | 1;               // rows over samples (>= M)
  static constexpr int RM = M | 1;                // staged z(t) rows
};

// Value of lane l ^ 1 (quad permutation 1,0,3,2).
__device__ __forceinline__ double swap_pair(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swap_pair(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// Waves per SIMD the register allocation must allow: the Picard tangent
// (the launch repeated inside GMRES) fits three without spilling in FP64,
// four in FP32; so does the Newton tangent in FP32 up to K = 4 (at most 126
// VGPRs; from K = 5 on four would spill).  In FP64 the Newton tangent fits
// three up to K = 3 (at most 164 VGPRs) and two up to K = 7 (at most 254)
// once it re-reads the velocity samples for the least-squares products
// instead of keeping them (see KEEPU in k_op).
template <int K, int MODE, typename T>
constexpr int op_waves() {
  constexpr int m = MODE & ~(MODE_TAU16 | MODE_SEG);
  if (m == 0) return sizeof(T) == 4 ? 4 : 3;
  if (m == MODE_NEWTON && K <= (sizeof(T) == 4 ? 4 : 3)) return sizeof(T) == 4 ? 4 : 3;
  if (m == MODE_NEWTON && sizeof(T) == 8 && K <= 7) return 2;
  return 1;
}

// bf16 bit pattern -> FP32 (bf16 is the top half of an FP32 word)
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Entry idx of the packed tau of the operator's arithmetic (bf16 copy for MODE_TAU16).
template <int MODE, typename T>
__device__ __forceinline__ T tau_entry(const DevView& v, const T* tau, int64_t idx) {
  if constexpr ((MODE & MODE_TAU16) != 0) return T(bf16_to_f32(v.tau16[idx]));
  else return tau[idx];
}

// The packed tau block of the next element is held in registers as loaded
// (bf16 bits for MODE_TAU16) and converted only when it is staged, so the
// load's latency stays hidden behind the current element.
template <int MODE, typename T>
struct TauReg {
  typedef T type;
  static __device__ __forceinline__ T load(const DevView&, const T* tau, int64_t idx) { return tau[idx]; }
  static __device__ __forceinline__ T value(T x) { return x; }
};
template <int MODE>
struct TauReg<MODE, float> {
  static constexpr bool B16 = (MODE & MODE_TAU16) != 0;
  typedef typename std::conditional<B16, uint32_t, float>::type type;
  static __device__ __forceinline__ type load(const DevView& v, const float* tau, int64_t idx) {
    if constexpr (B16) return v.tau16[idx];
    else return tau[idx];
  }
  static __device__ __forceinline__ float value(type x) {
    if constexpr (B16) return __uint_as_float(x << 16);
    else return x;
  }
};

// Frozen fields of the linearization in the kernel's arithmetic type.
template <typename T>
struct Frozen {
  const T* UT;    // [n_nodes][3][M] velocity samples
  const T* tau;   // [E][4][P] packed tau
  const T* Z;     // [E][4][3][n] tau L(u) (Newton tangent)
};
template <typename T>
__device__ __forceinline__ Frozen<T> frozen(const DevView& v) {
  if constexpr (sizeof(T) == 8) return Frozen<T>{v.UT, v.tau, v.Z};
  else return Frozen<T>{v.UT32, v.tau32, v.Z32};
}

// XP: [n_nodes][4][PW] input modes at positions; VT: [n_nodes][3][M]
// direction samples (tangent modes); out: [E][4][4][n] element rows; Zout
// (MODE_STOREZ, FP64 only): tau L(u) [E][4][3][n].
template <int K, int MODE, typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(op_waves<K, MODE, T>())))
k_op(DevView v, const T* __restrict__ XP, const T* __restrict__ VT,
     double* __restrict__ Zout, T* __restrict__ out, T shift, int64_t begin, int64_t end) {
  using C = OpCfg<K>;
  constexpr int n = C::n, M = C::M, S = C::S, P = C::P, PW = C::PW, NPT = C::NPT;
  constexpr int MS = C::MS, NKB = C::NKB, MT = C::MT, NKF = C::NKF, NPR = C::NPR, NTL = C::NTL;
  constexpr int RP = C::RP, RS = C::RS, RM = C::RM;
  constexpr bool RESID = (MODE & MODE_RESID) != 0;
  constexpr bool NEWTON = (MODE & MODE_NEWTON) != 0;
  constexpr bool NOLS = (MODE & MODE_NOLS) != 0;
  constexpr bool STOREZ = (MODE & MODE_STOREZ) != 0;
  // u_q(t_s) of the products phase is kept in registers for the
  // least-squares phase, except in the FP64 Newton tangent, where its 24
  // VGPRs cost a wave per SIMD (two against three at K = 3, one against two
  // at K = 6): there the samples are read again (the same arithmetic on the
  // same values).
  constexpr bool KEEPU = C::KEEPU && !(NEWTON && sizeof(T) == 8 && K <= 7);
  constexpr int NL = NOLS ? 2 : 1;
  using R = Mma<T>;
  typedef typename R::v4 T4;
  const Frozen<T> fz = frozen<T>(v);
  const T* __restrict__ UT = fz.UT;
  const T* TAU = fz.tau;
  const T QB = T(TS_QB), QAB = T(TS_QA - TS_QB);

  constexpr int NC = 16 * (RS > RM ? RS : RM);
  __shared__ T sV[16 * RP];               // modes [node][field][position]
  constexpr int NT = 4 * n * n > NL * 16 * RP ? 4 * n * n : NL * 16 * RP;
  __shared__ T sT[NT];                    // tau_q rows [q][position][position], then z
  __shared__ T sL[NL * 12 * RP];          // L [q][i][position] (+ grad p part), then G
  __shared__ T sC[NC];                    // conv(t) [16][RS] / z(t) [16][RM] / W(t) [16][RS]
  T* const sZ = sT;                       // z [q*4+i][position] (+ tau grad p)
  __shared__ T sZf[NEWTON ? 16 * RP : 1];    // stored tau L(u) [q*4+i][position]
  __shared__ T sZft[NEWTON ? 16 * RM : 1];   // its samples [i*4+q][s]
  __shared__ T sWq[NEWTON ? 12 * RM : 1];    // direction at the points [q][j][s]

  const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
  const T rho = T(v.rho), mu = T(v.mu), omega = T(v.omega), irho = T(1.0 / v.rho);
  const double* __restrict__ F = v.F;

  // ---- per-lane constants (once per wave)
  T Bb[NKB][NPT];   // B[k = s][col = position] = phi(t_s) / M
  T Bf[NKF][MT];    // B[k = position][col = s] = phi(t_s)
#pragma unroll
  for (int ks = 0; ks < NKB; ++ks)
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int s = ks * 4 + g, a = pos_mode(c + 16 * pt, K);
      Bb[ks][pt] = (s < M && a >= 0) ? F[a * M + s] * (1.0 / M) : 0.0;
    }
#pragma unroll
  for (int ks = 0; ks < NKF; ++ks)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int s = c + 16 * mt, a = pos_mode(ks * 4 + g, K);
      Bf[ks][mt] = (s < M && a >= 0) ? F[a * M + s] : 0.0;
    }
  int sP[NPR], iP[NPR];
  bool okP[NPR];
#pragma unroll
  for (int r = 0; r < NPR; ++r) {
    const int it = lane + 64 * r;
    okP[r] = it < 3 * M;
    sP[r] = okP[r] ? it % M : 0;
    iP[r] = okP[r] ? it / M : 0;
  }
  T om[NPT];        // (Omega x)_p = om_p x_{p^1}
  int trow[NPT];         // row of tau_q read by this lane (padding lanes read row 0)
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt) {
    const int p = c + 16 * pt;
    om[pt] = p < 2 * K ? ((p & 1) ? ((p + 1) >> 1) * omega : -((p >> 1) + 1) * omega) : T(0);
    trow[pt] = (g * n + (p < n ? p : 0)) * n;
  }
  int tdst[NTL];         // unpacking of packed tau: (r*n + c) | (c*n + r) << 16
  bool tok[NTL];
#pragma unroll
  for (int j = 0; j < NTL; ++j) {
    const int pi = lane + 64 * j;
    tok[j] = pi < P;
    int r = 0, cc = 0;
    if (tok[j]) packed_rc<n>(pi, r, cc);
    tdst[j] = (r * n + cc) | ((cc * n + r) << 16);
  }
  T oscale[NPT];    // orthonormal -> slot scale of position p
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt) {
    const int p = c + 16 * pt;
    oscale[pt] = p < 2 * K ? T(TS_RS2) : T(1);
  }
  constexpr T MD = TS_QA * TS_QA + 3.0 * TS_QB * TS_QB;      // sum_q lam_qb^2
  constexpr T MO = 2.0 * TS_QA * TS_QB + 2.0 * TS_QB * TS_QB;  // sum_q lam_qb lam_qc

  // LDS words that enter an MFMA as padding (k beyond the data, or rows
  // whose results are discarded) multiply zeros of B, so they must be finite
  // (0 * NaN = NaN).  LDS is undefined at launch: the buffers read as MFMA
  // operands are cleared once, and only finite values are stored afterwards.
  for (int i = lane; i < NC; i += 64) sC[i] = 0.0;
  for (int i = lane; i < NT; i += 64) sT[i] = 0.0;
  if (NEWTON)
    for (int i = lane; i < 16 * RP; i += 64) sZf[i] = 0.0;
  __syncthreads();

  // ---- contiguous element range of this block's XCD.  With a work list
  // (segmented context) the range runs over the positions of the listed
  // segments' elements only: position p is element list[p / elems] * elems
  // + p % elems.
  constexpr bool SEG = (MODE & MODE_SEG) != 0;
  const bool listed = SEG && v.seg.list != nullptr;
  if (listed) {
    begin = 0;
    end = (int64_t)v.seg.count[0] * v.seg.elems;
  }
  auto elem = [&](int64_t p) -> int64_t {
    if (!listed) return p;
    const uint32_t q = (uint32_t)p / (uint32_t)v.seg.elems;
    return (int64_t)v.seg.list[q] * v.seg.elems + (p - (int64_t)q * v.seg.elems);
  };
  const int64_t nbx = gridDim.x >> 3, xcd = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int64_t cnt = end - begin;
  const int64_t lo = begin + cnt * xcd / 8, hi = begin + cnt * (xcd + 1) / 8;

  // packed tau of the next element is loaded one element ahead (it streams
  // from HBM with no reuse, so its latency is hidden behind the current one)
  using TR = TauReg<MODE, T>;
  typename TR::type tv[4][NTL];
  auto load_tau = [&](int64_t en) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < NTL; ++j)
        tv[q][j] = tok[j] ? TR::load(v, TAU, (en * 4 + q) * P + lane + 64 * j) : typename TR::type(0);
  };
  if (lo + jx < hi) load_tau(elem(lo + jx));

  for (int64_t pe = lo + jx; pe < hi; pe += nbx) {
    const int64_t e = elem(pe);
    int nd[4];
    T dN[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      nd[b] = v.conn[e * 4 + b];
#pragma unroll
      for (int j = 0; j < 3; ++j) dN[b][j] = v.geo[e * 16 + b * 3 + j];
    }
    const T wgt = v.geo[e * 16 + 12];

    // modal input first (consumed after the products)
    T xv[4][NPT];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int pt = 0; pt < NPT; ++pt) xv[b][pt] = XP[(int64_t)nd[b] * (4 * PW) + pt * 64 + lane];

    // ---- products at the samples
    T uq[KEEPU ? NPR : 1][4][3];
#pragma unroll
    for (int r = 0; r < NPR; ++r) {
      if (!okP[r]) continue;
      const int s = sP[r], i = iP[r];
      T U[4][3], Wi[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T* ut = UT + (int64_t)nd[b] * (3 * M) + s;
#pragma unroll
        for (int j = 0; j < 3; ++j) U[b][j] = ut[j * M];
        Wi[b] = RESID ? ut[i * M] : VT[(int64_t)nd[b] * (3 * M) + i * M + s];
      }
      T gW[3], su[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        gW[j] = dN[0][j] * Wi[0] + dN[1][j] * Wi[1] + dN[2][j] * Wi[2] + dN[3][j] * Wi[3];
        su[j] = U[0][j] + U[1][j] + U[2][j] + U[3][j];
      }
      T u[4][3];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < 3; ++j) u[q][j] = QB * su[j] + QAB * U[q][j];
      T conv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) conv[q] = u[q][0] * gW[0] + u[q][1] * gW[1] + u[q][2] * gW[2];
      if (NEWTON) {
        T Wd[4][3], Ui[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const T* vt = VT + (int64_t)nd[b] * (3 * M) + s;
#pragma unroll
          for (int j = 0; j < 3; ++j) Wd[b][j] = vt[j * M];
          Ui[b] = UT[(int64_t)nd[b] * (3 * M) + i * M + s];
        }
        T gU[3], sw[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          gU[j] = dN[0][j] * Ui[0] + dN[1][j] * Ui[1] + dN[2][j] * Ui[2] + dN[3][j] * Ui[3];
          sw[j] = Wd[0][j] + Wd[1][j] + Wd[2][j] + Wd[3][j];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T wq[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) wq[j] = QB * sw[j] + QAB * Wd[q][j];
          conv[q] += wq[0] * gU[0] + wq[1] * gU[1] + wq[2] * gU[2];
          // this lane's component i of the direction at point q
          sWq[(q * 3 + i) * RM + s] = i == 0 ? wq[0] : (i == 1 ? wq[1] : wq[2]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) sC[R::row(q, i) * RS + s] = conv[q];
      if (KEEPU)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < 3; ++j) uq[KEEPU ? r : 0][q][j] = u[q][j];
    }
    // stage tau rows and the modal input
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < NTL; ++j)
        if (tok[j]) {
          const T tval = TR::value(tv[q][j]);
          sT[q * n * n + (tdst[j] & 0xffff)] = tval;
          sT[q * n * n + (tdst[j] >> 16)] = tval;
        }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int pt = 0; pt < NPT; ++pt) {
        const int fp = pt * 64 + lane;   // field * PW + position within the node's block
        sV[(b * 4 + fp / PW) * RP + fp % PW] = xv[b][pt];
      }
    if (pe + nbx < hi) load_tau(elem(pe + nbx));
    __syncthreads();

    // ---- conv(t) -> modes: lane (q = g, p), reg i
    T cm[NPT][3];
    {
      T a[NKB];
#pragma unroll
      for (int ks = 0; ks < NKB; ++ks) a[ks] = sC[c * RS + ks * 4 + g];
#pragma unroll
      for (int pt = 0; pt < NPT; ++pt) {
        T4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NKB; ++ks) acc = R::run(a[ks], Bb[ks][pt], acc);
#pragma unroll
        for (int i = 0; i < 3; ++i) cm[pt][i] = acc[i];
      }
    }

    // ---- momentum operator L per (q, position)
    T gal[NPT][3];
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int p = c + 16 * pt;
      T Vb[4][4], Vq[3];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int f = 0; f < 4; ++f) Vb[b][f] = sV[(b * 4 + f) * RP + p];
#pragma unroll
      for (int i = 0; i < 3; ++i) Vq[i] = sV[(g * 4 + i) * RP + p];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T du = QB * (Vb[0][i] + Vb[1][i] + Vb[2][i] + Vb[3][i]) + QAB * Vq[i];
        const T dp = dN[0][i] * Vb[0][3] + dN[1][i] * Vb[1][3] + dN[2][i] * Vb[2][3] + dN[3][i] * Vb[3][3];
        gal[pt][i] = rho * tfma(om[pt], swap_pair(du), cm[pt][i]);
        sL[(g * 3 + i) * RP + p] = NOLS ? gal[pt][i] : gal[pt][i] + dp;
        if (NOLS) sL[12 * RP + (g * 3 + i) * RP + p] = dp;
      }
    }
    __syncthreads();

    // ---- z = tau_q L (and tau_q grad p for the variant without LS coupling)
    T z[NPT][3], zc[NPT][3];
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      T tr[n];
#pragma unroll
      for (int k = 0; k < n; ++k) tr[k] = sT[trow[pt] + k];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T* lr = sL + (g * 3 + i) * RP;
        T acc = 0.0, accc = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
          acc = tfma(tr[k], lr[k], acc);
          if (NOLS) accc = tfma(tr[k], lr[12 * RP + k], accc);
        }
        z[pt][i] = acc;
        zc[pt][i] = accc;
      }
    }
    __syncthreads();
    // G = gal - Omega z (into sL), z rows q*4+i, stored / frozen z
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int p = c + 16 * pt;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        sL[(g * 3 + i) * RP + p] = gal[pt][i] - om[pt] * swap_pair(z[pt][i]);
        sZ[R::row(i, g) * RP + p] = z[pt][i];
        if (NOLS) sZ[16 * RP + R::row(i, g) * RP + p] = zc[pt][i];
        if (p < n) {
          const int64_t zi = ((e * 4 + g) * 3 + i) * n + p;
          if (STOREZ) Zout[zi] = z[pt][i];
          if (NEWTON) sZf[R::row(i, g) * RP + p] = fz.Z[zi];
        }
      }
    }
    __syncthreads();

    // ---- z modes -> samples: lane (i = g, s = c + 16 mt), reg q; staged [i*4+q][s]
    {
      T a[NKF], af[NEWTON ? NKF : 1];
#pragma unroll
      for (int ks = 0; ks < NKF; ++ks) {
        a[ks] = sZ[c * RP + ks * 4 + g];
        if (NEWTON) af[NEWTON ? ks : 0] = sZf[c * RP + ks * 4 + g];
      }
      T4 zt[MT], zft[NEWTON ? MT : 1];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        T4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NKF; ++ks) acc = R::run(a[ks], Bf[ks][mt], acc);
        zt[mt] = acc;
        if (NEWTON) {
          T4 accf = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int ks = 0; ks < NKF; ++ks)
            accf = R::run(af[NEWTON ? ks : 0], Bf[ks][mt], accf);
          zft[NEWTON ? mt : 0] = accf;
        }
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int s = c + 16 * mt;
        if (s < M && g < 3) {   // lane group 3 holds the padding rows
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            sC[(g * 4 + q) * RM + s] = zt[mt][q];
            if (NEWTON) sZft[(g * 4 + q) * RM + s] = zft[NEWTON ? mt : 0][q];
          }
        }
      }
    }
    __syncthreads();

    // ---- least-squares test products W_ji(t_s), lane (s, i)
    {
      T W[NPR][3];
#pragma unroll
      for (int r = 0; r < NPR; ++r) {
        W[r][0] = W[r][1] = W[r][2] = 0.0;
        if (!okP[r]) continue;
        const int s = sP[r], i = iP[r];
        T u[4][3];
        if (KEEPU) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 3; ++j) u[q][j] = uq[KEEPU ? r : 0][q][j];
        } else {
          T U[4][3], su[3];
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int j = 0; j < 3; ++j) U[b][j] = UT[(int64_t)nd[b] * (3 * M) + j * M + s];
#pragma unroll
          for (int j = 0; j < 3; ++j) su[j] = U[0][j] + U[1][j] + U[2][j] + U[3][j];
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 3; ++j) u[q][j] = QB * su[j] + QAB * U[q][j];
        }
        T zq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) zq[q] = sC[(i * 4 + q) * RM + s];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T acc = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) acc = tfma(u[q][j], zq[q], acc);
          W[r][j] = acc;
        }
        if (NEWTON) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T zf = sZft[(i * 4 + q) * RM + s];
#pragma unroll
            for (int j = 0; j < 3; ++j) W[r][j] = tfma(sWq[(q * 3 + j) * RM + s], zf, W[r][j]);
          }
        }
      }
      __syncthreads();   // every lane has read the staged z(t) before W(t) overwrites it
#pragma unroll
      for (int r = 0; r < NPR; ++r) {
        if (!okP[r]) continue;
#pragma unroll
        for (int j = 0; j < 3; ++j) sC[R::row(iP[r], j) * RS + sP[r]] = wgt * W[r][j];
      }
    }
    __syncthreads();

    // ---- W(t) -> modes: lane (i = g, p), reg j
    T wm[NPT][3];
    {
      T a[NKB];
#pragma unroll
      for (int ks = 0; ks < NKB; ++ks) a[ks] = sC[c * RS + ks * 4 + g];
#pragma unroll
      for (int pt = 0; pt < NPT; ++pt) {
        T4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NKB; ++ks) acc = R::run(a[ks], Bb[ks][pt], acc);
#pragma unroll
        for (int j = 0; j < 3; ++j) wm[pt][j] = acc[j];
      }
    }

    // ---- assembly: lane (field f = g, position p), node rows b
    T* oe = out + e * (16 * n);
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int p = c + 16 * pt;
      T o[4];
      if (g < 3) {
        const int i = g;
        T Gq[4], Vf[4], Vp[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) Gq[q] = sL[(q * 3 + i) * RP + p];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          Vf[b] = sV[(b * 4 + i) * RP + p];
          Vp[b] = sV[(b * 4 + 3) * RP + p];
        }
        const T Gs = Gq[0] + Gq[1] + Gq[2] + Gq[3];
        const T ps = Vp[0] + Vp[1] + Vp[2] + Vp[3];
        const T Vs = Vf[0] + Vf[1] + Vf[2] + Vf[3];
        // sum_j dN_bj (W_ji + 4 w mu grad_j du_i): least-squares and viscous terms together
        const T kv = T(4) * wgt * mu, ks = T(shift) * wgt;
        T t[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
          t[j] = tfma(kv, dN[0][j] * Vf[0] + dN[1][j] * Vf[1] + dN[2][j] * Vf[2] + dN[3][j] * Vf[3], wm[pt][j]);
        const T wq = wgt * QAB, km = ks * (MD - MO), wps = -wgt * ps;
        const T base = tfma(wgt * QB, Gs, ks * MO * Vs);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const T dNi = i == 0 ? dN[b][0] : (i == 1 ? dN[b][1] : dN[b][2]);
          T acc = tfma(wq, Gq[b], base);       // sum_q w lam_qb G_qi
          acc = tfma(km, Vf[b], acc);               // mass shift
          acc = tfma(wps, dNi, acc);                // - (d_i N_b, p)
          acc = tfma(dN[b][0], t[0], acc);
          acc = tfma(dN[b][1], t[1], acc);
          o[b] = tfma(dN[b][2], t[2], acc);
        }
      } else {
        T div = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int j = 0; j < 3; ++j) div = tfma(dN[b][j], sV[(b * 4 + j) * RP + p], div);
        T zs[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const T* zr = sZ + (NOLS ? 16 * RP : 0) + p;
          zs[i] = zr[R::row(i, 0) * RP] + zr[R::row(i, 1) * RP] + zr[R::row(i, 2) * RP] + zr[R::row(i, 3) * RP];
        }
        const T wr = wgt * irho, wd = wgt * div;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          o[b] = tfma(wr, dN[b][0] * zs[0] + dN[b][1] * zs[1] + dN[b][2] * zs[2], wd);
      }
      if (p < n) {
#pragma unroll
        for (int b = 0; b < 4; ++b) oe[(b * 4 + g) * n + p] = o[b] * oscale[pt];
      }
    }
    __syncthreads();   // LDS of this element fully consumed before the next one
  }
}

// ------------------------------------------- element operator, large K
// The same operator for K with n = 2K+1 > 32 modes per field (the
// register-blocked kernel above keeps a tile of DFT weights and a packed tau
// block per lane, which does not fit at n = 63).  One block of four waves per
// element (persistent over a contiguous Morton range per XCD); the sample
// table phi_a(t_s) sits in LDS for the whole launch, and every phase uses a
// layout in which one LDS operand is the same for the whole wave:
//   products    thread s < M: conv_{q,i}(t_s) for all (q, i) (+ Newton
//               term), u_q(t_s) and the direction at the points kept in
//               registers for the least-squares products
//   to modes    wave q, lane p: conv modes of point q, then L_i (LDS)
//   z           wave q, lane p: z_i = tau_q L_i, tau_q row p read from the
//               packed block (L1/L2); G = gal - Omega z with the pair
//               partner's z from the neighbouring lane
//   to samples  thread s: z_{q,i}(t_s) in registers
//   LS          thread s: W_ji(t_s) = w sum_q u_{q,j} z_{q,i} -> LDS
//   to modes    wave i, lane p: W modes in registers
//   assembly    wave f, lane p: Galerkin, viscous, pressure, LS and PSPG
//               terms of the four node rows (same element-buffer layout).
template <int K, typename T>
struct BigCfg {
  static constexpr int n = 2 * K + 1, M = 3 * K + 1, P = n * (n + 1) / 2;
  static constexpr int PW = (n + 63) / 64 * 64;   // positions: one per lane of a wave
  static constexpr int RP = PW + 1;               // LDS row stride over positions
  static constexpr int RS = M | 1;                // LDS row stride over samples
  static_assert(PW == 64, "large-K operator: one wave spans the positions");
  static_assert(M <= 256, "large-K operator: one thread per sample");
};

template <int K, int MODE, typename T>
__global__ void __launch_bounds__(256)
k_op_big(DevView v, const T* __restrict__ XP, const T* __restrict__ VT,
         double* __restrict__ Zout, T* __restrict__ out, T shift, int64_t begin, int64_t end) {
  using C = BigCfg<K, T>;
  constexpr int n = C::n, M = C::M, P = C::P, PW = C::PW, RP = C::RP, RS = C::RS;
  constexpr bool RESID = (MODE & MODE_RESID) != 0;
  constexpr bool NEWTON = (MODE & MODE_NEWTON) != 0;
  constexpr bool NOLS = (MODE & MODE_NOLS) != 0;
  constexpr bool STOREZ = (MODE & MODE_STOREZ) != 0;
  const Frozen<T> fz = frozen<T>(v);
  const T* __restrict__ UT = fz.UT;
  const T QB = T(TS_QB), QAB = T(TS_QA - TS_QB);
  constexpr T MD = TS_QA * TS_QA + 3.0 * TS_QB * TS_QB;      // sum_q lam_qb^2
  constexpr T MO = 2.0 * TS_QA * TS_QB + 2.0 * TS_QB * TS_QB;  // sum_q lam_qb lam_qc

  __shared__ T sPhi[M * RP];                 // phi_{mode(p)}(t_s) at [s][p], 0 for p >= n
  __shared__ T sV[16 * RP];                  // input modes [node][field][position]
  __shared__ T sC[12 * RS];                  // conv(t) [q*3+i][s], then W(t) [i*3+j][s]
  __shared__ T sL[(NOLS ? 24 : 12) * RP];    // L [q*3+i][p] (+ grad p part), then G
  __shared__ T sZ[(NOLS ? 32 : 16) * RP];    // z [i*4+q][p] (+ tau grad p)
  __shared__ T sZf[NEWTON ? 16 * RP : 1];    // stored tau L(u) [i*4+q][p]

  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const T rho = T(v.rho), mu = T(v.mu), omega = T(v.omega), irho = T(1.0 / v.rho);
  const T invM = T(1.0 / M);
  for (int i = tid; i < M * RP; i += 256) {
    const int s = i / RP, p = i % RP;
    const int a = p < PW ? pos_mode(p, K) : -1;
    sPhi[i] = a >= 0 ? T(v.F[a * M + s]) : T(0);
  }
  for (int i = tid; i < 16 * RP; i += 256) {
    if (NEWTON) sZf[i] = T(0);
  }
  // per-lane constants of the position layouts
  const int p = lane;
  const T om = p < 2 * K ? ((p & 1) ? T((p + 1) >> 1) * omega : -T((p >> 1) + 1) * omega) : T(0);
  const T oscale = p < 2 * K ? T(TS_RS2) : T(1);
  __syncthreads();

  const int64_t nbx = gridDim.x >> 3, xcd = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int64_t cnt = end - begin;
  const int64_t lo = begin + cnt * xcd / 8, hi = begin + cnt * (xcd + 1) / 8;

  for (int64_t e = lo + jx; e < hi; e += nbx) {
    int nd[4];
    T dN[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      nd[b] = v.conn[e * 4 + b];
#pragma unroll
      for (int j = 0; j < 3; ++j) dN[b][j] = T(v.geo[e * 16 + b * 3 + j]);
    }
    const T wgt = T(v.geo[e * 16 + 12]);

    // ---- modal input
    for (int i = tid; i < 16 * PW; i += 256) {
      const int b = i / (4 * PW), fp = i % (4 * PW);
      sV[(b * 4 + fp / PW) * RP + fp % PW] = XP[(int64_t)nd[b] * (4 * PW) + fp];
    }

    // ---- products at the samples, thread s
    const int s = tid;
    const bool samp = s < M;
    T u[4][3], wq[NEWTON ? 4 : 1][3];
    if (samp) {
      T U[4][3], Wd[4][3];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          U[b][j] = UT[(int64_t)nd[b] * (3 * M) + j * M + s];
          Wd[b][j] = RESID ? U[b][j] : VT[(int64_t)nd[b] * (3 * M) + j * M + s];
        }
      T su[3], sw[3], gW[3][3], gU[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        su[j] = U[0][j] + U[1][j] + U[2][j] + U[3][j];
        sw[j] = Wd[0][j] + Wd[1][j] + Wd[2][j] + Wd[3][j];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          gW[i][j] = dN[0][j] * Wd[0][i] + dN[1][j] * Wd[1][i] + dN[2][j] * Wd[2][i] + dN[3][j] * Wd[3][i];
          gU[i][j] = dN[0][j] * U[0][i] + dN[1][j] * U[1][i] + dN[2][j] * U[2][i] + dN[3][j] * U[3][i];
        }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          u[q][j] = QB * su[j] + QAB * U[q][j];
          if (NEWTON) wq[NEWTON ? q : 0][j] = QB * sw[j] + QAB * Wd[q][j];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          T cv = u[q][0] * gW[i][0] + u[q][1] * gW[i][1] + u[q][2] * gW[i][2];
          if (NEWTON)
            cv += wq[NEWTON ? q : 0][0] * gU[i][0] + wq[NEWTON ? q : 0][1] * gU[i][1] +
                  wq[NEWTON ? q : 0][2] * gU[i][2];
          sC[(q * 3 + i) * RS + s] = cv;
        }
      }
    }
    __syncthreads();

    // ---- conv -> modes and L, wave q, lane p
    const int q = wv;
    T gal[3];
    {
      T cm[3] = {T(0), T(0), T(0)};
      const T* c0 = sC + (q * 3) * RS;
#pragma unroll 2
      for (int t = 0; t < M; ++t) {
        const T ph = sPhi[t * RP + p];
        cm[0] = tfma(c0[t], ph, cm[0]);
        cm[1] = tfma(c0[RS + t], ph, cm[1]);
        cm[2] = tfma(c0[2 * RS + t], ph, cm[2]);
      }
      const int p1 = p ^ 1;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T du1 = QB * (sV[(0 * 4 + i) * RP + p1] + sV[(1 * 4 + i) * RP + p1] + sV[(2 * 4 + i) * RP + p1] +
                            sV[(3 * 4 + i) * RP + p1]) + QAB * sV[(q * 4 + i) * RP + p1];
        const T dp = dN[0][i] * sV[(0 * 4 + 3) * RP + p] + dN[1][i] * sV[(1 * 4 + 3) * RP + p] +
                     dN[2][i] * sV[(2 * 4 + 3) * RP + p] + dN[3][i] * sV[(3 * 4 + 3) * RP + p];
        gal[i] = rho * tfma(om, du1, cm[i] * invM);
        sL[(q * 3 + i) * RP + p] = NOLS ? gal[i] : gal[i] + dp;
        if (NOLS) sL[(12 + q * 3 + i) * RP + p] = dp;
      }
    }
    __syncthreads();

    // ---- z = tau_q L (and tau_q grad p without LS coupling), G = gal - Omega z
    T z[3] = {T(0), T(0), T(0)}, zc[3] = {T(0), T(0), T(0)};
    if (p < n) {
      const int64_t tq = (e * 4 + q) * P;
      const T* l0 = sL + (q * 3) * RP;
#pragma unroll 2
      for (int k = 0; k < n; ++k) {
        const int lo_ = p < k ? p : k, hi_ = p < k ? k : p;
        const T t = tau_entry<MODE, T>(v, fz.tau, tq + pk_index(lo_, hi_, n));
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          z[i] = tfma(t, l0[i * RP + k], z[i]);
          if (NOLS) zc[i] = tfma(t, l0[(12 + i) * RP + k], zc[i]);
        }
      }
    }
    T G[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) G[i] = gal[i] - om * swap_pair(z[i]);
    __syncthreads();   // every lane has read L
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sL[(q * 3 + i) * RP + p] = G[i];
      sZ[(i * 4 + q) * RP + p] = z[i];
      if (NOLS) sZ[(16 + i * 4 + q) * RP + p] = zc[i];
      if (p < n) {
        const int64_t zi = ((e * 4 + q) * 3 + i) * n + p;
        if (STOREZ) Zout[zi] = double(z[i]);
        if (NEWTON) sZf[(i * 4 + q) * RP + p] = fz.Z[zi];
      }
    }
    __syncthreads();

    // ---- z (and the stored tau L(u)) at the samples, then the LS products, thread s
    if (samp) {
      T zt[12], zft[NEWTON ? 12 : 1];
#pragma unroll
      for (int r = 0; r < 12; ++r) {
        zt[r] = T(0);
        if (NEWTON) zft[NEWTON ? r : 0] = T(0);
      }
#pragma unroll 1
      for (int k = 0; k < n; ++k) {
        const T ph = sPhi[s * RP + k];
#pragma unroll
        for (int r = 0; r < 12; ++r) {
          zt[r] = tfma(sZ[r * RP + k], ph, zt[r]);
          if (NEWTON) zft[NEWTON ? r : 0] = tfma(sZf[r * RP + k], ph, zft[NEWTON ? r : 0]);
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T acc = T(0);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            acc = tfma(u[qq][j], zt[i * 4 + qq], acc);
            if (NEWTON) acc = tfma(wq[NEWTON ? qq : 0][j], zft[NEWTON ? i * 4 + qq : 0], acc);
          }
          sC[(i * 3 + j) * RS + s] = wgt * acc;   // conv(t) was consumed before the last barriers
        }
    }
    __syncthreads();

    // ---- W -> modes (wave i) and assembly (wave f = field), lane p
    const int f = wv;
    T o[4];
    if (f < 3) {
      const int i = f;
      T wm[3] = {T(0), T(0), T(0)};
      const T* w0 = sC + (i * 3) * RS;
#pragma unroll 2
      for (int t = 0; t < M; ++t) {
        const T ph = sPhi[t * RP + p];
        wm[0] = tfma(w0[t], ph, wm[0]);
        wm[1] = tfma(w0[RS + t], ph, wm[1]);
        wm[2] = tfma(w0[2 * RS + t], ph, wm[2]);
      }
      T Gq[4], Vf[4], Vp[4];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) Gq[qq] = sL[(qq * 3 + i) * RP + p];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        Vf[b] = sV[(b * 4 + i) * RP + p];
        Vp[b] = sV[(b * 4 + 3) * RP + p];
      }
      const T Gs = Gq[0] + Gq[1] + Gq[2] + Gq[3];
      const T ps = Vp[0] + Vp[1] + Vp[2] + Vp[3];
      const T Vs = Vf[0] + Vf[1] + Vf[2] + Vf[3];
      const T kv = T(4) * wgt * mu, ks = shift * wgt;
      T t3[3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        t3[j] = tfma(kv, dN[0][j] * Vf[0] + dN[1][j] * Vf[1] + dN[2][j] * Vf[2] + dN[3][j] * Vf[3],
                     wm[j] * invM);
      const T wq_ = wgt * QAB, km = ks * (MD - MO), wps = -wgt * ps;
      const T base = tfma(wgt * QB, Gs, ks * MO * Vs);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const T dNi = i == 0 ? dN[b][0] : (i == 1 ? dN[b][1] : dN[b][2]);
        T acc = tfma(wq_, Gq[b], base);
        acc = tfma(km, Vf[b], acc);
        acc = tfma(wps, dNi, acc);
        acc = tfma(dN[b][0], t3[0], acc);
        acc = tfma(dN[b][1], t3[1], acc);
        o[b] = tfma(dN[b][2], t3[2], acc);
      }
    } else {
      T div = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int j = 0; j < 3; ++j) div = tfma(dN[b][j], sV[(b * 4 + j) * RP + p], div);
      T zs[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T* zr = sZ + ((NOLS ? 16 : 0) + i * 4) * RP + p;
        zs[i] = zr[0] + zr[RP] + zr[2 * RP] + zr[3 * RP];
      }
      const T wr = wgt * irho, wd = wgt * div;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        o[b] = tfma(wr, dN[b][0] * zs[0] + dN[b][1] * zs[1] + dN[b][2] * zs[2], wd);
    }
    if (p < n) {
      T* oe = out + e * (16 * n);
#pragma unroll
      for (int b = 0; b < 4; ++b) oe[(b * 4 + f) * n + p] = o[b] * oscale;
    }
    __syncthreads();   // LDS of this element fully consumed before the next one
  }
}

template <int K, int MD, typename T>
static hipError_t op_big_launch(const DevView& v, const T* XP, const T* VT, double* Zout, T* out,
                                double shift, int64_t begin, int64_t end, hipStream_t st) {
  static std::atomic<int> max_blocks_cache{0};
  int max_blocks = max_blocks_cache.load(std::memory_order_relaxed);
  if (max_blocks == 0) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_op_big<K, MD, T>, 256, 0);
    if (e != hipSuccess) return e;
    const int mb = ncu * (per_cu > 0 ? per_cu : 1);
    max_blocks = mb < 8 ? 8 : mb / 8 * 8;
    max_blocks_cache.store(max_blocks, std::memory_order_relaxed);
  }
  int64_t nb = (end - begin + 7) / 8 * 8;
  if (nb > max_blocks) nb = max_blocks;
  k_op_big<K, MD, T><<<(unsigned)nb, 256, 0, st>>>(v, XP, VT, Zout, out, T(shift), begin, end);
  return hipGetLastError();
}

template <int K>
static hipError_t op_big_dispatch(const DevView& v, int mode, const double* XP, const double* VT,
                                  double* Zout, double* out, double shift, int64_t begin, int64_t end,
                                  hipStream_t st) {
  switch (mode) {
    case MODE_RESID: return op_big_launch<K, MODE_RESID>(v, XP, VT, Zout, out, shift, begin, end, st);
    case MODE_RESID | MODE_STOREZ:
      return op_big_launch<K, MODE_RESID | MODE_STOREZ>(v, XP, VT, Zout, out, shift, begin, end, st);
    case 0: return op_big_launch<K, 0>(v, XP, VT, Zout, out, shift, begin, end, st);
    case MODE_NOLS: return op_big_launch<K, MODE_NOLS>(v, XP, VT, Zout, out, shift, begin, end, st);
    case MODE_NEWTON: return op_big_launch<K, MODE_NEWTON>(v, XP, VT, Zout, out, shift, begin, end, st);
    default: return hipErrorInvalidValue;
  }
}

template <int K>
static hipError_t op_big_dispatch(const DevView& v, int mode, const float* XP, const float* VT,
                                  float* out, double shift, int64_t begin, int64_t end, hipStream_t st) {
  switch (mode) {
#define CASE(md) case md: return op_big_launch<K, md>(v, XP, VT, nullptr, out, shift, begin, end, st);
    CASE(0) CASE(MODE_NOLS) CASE(MODE_NEWTON)
    CASE(MODE_TAU16) CASE(MODE_TAU16 | MODE_NOLS) CASE(MODE_TAU16 | MODE_NEWTON)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------- dispatch
template <typename T>
struct OpArgs {
  const T* XP;
  const T* VT;
  T* out;
  double* Zout;
};

template <int K, int MD, typename T>
static hipError_t op_launch(const DevView& v, const OpArgs<T>& a, double shift, int64_t begin,
                            int64_t end, hipStream_t st) {
  // resident blocks on the whole device, multiple of 8 (computed once; the
  // library drives one device model, and concurrent first calls store the
  // same value)
  static std::atomic<int> max_blocks_cache{0};
  int max_blocks = max_blocks_cache.load(std::memory_order_relaxed);
  if (max_blocks == 0) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_op<K, MD, T>, 64, 0);
    if (e != hipSuccess) return e;
    const int mb = ncu * (per_cu > 0 ? per_cu : 1);
    max_blocks = mb < 8 ? 8 : mb / 8 * 8;
    max_blocks_cache.store(max_blocks, std::memory_order_relaxed);
  }
  const int64_t cnt = end - begin;
  int64_t nb = (cnt + 7) / 8 * 8;
  if (nb > max_blocks) nb = max_blocks;
  k_op<K, MD, T><<<(unsigned)nb, 64, 0, st>>>(v, a.XP, a.VT, a.Zout, a.out, T(shift), begin, end);
  return hipGetLastError();
}

// With a work list of segments (v.seg.list set) the MODE_SEG instantiations
// run over the listed segments' elements, so that the plain kernels carry
// none of that logic; otherwise (and for a mode without one) the plain
// kernel computes every element, and the node gather still writes zero rows
// for segments sitting out.
template <int K>
static hipError_t op_dispatch(const DevView& v, int mode, const OpArgs<double>& a, double shift,
                              int64_t begin, int64_t end, hipStream_t st) {
  if (v.seg.list) {
    switch (mode) {
#define CASE(md) case md: return op_launch<K, md | MODE_SEG>(v, a, shift, begin, end, st);
      CASE(MODE_RESID | MODE_STOREZ) CASE(0) CASE(MODE_NOLS) CASE(MODE_NEWTON)
#undef CASE
      default: break;
    }
  }
  switch (mode) {
    case MODE_RESID: return op_launch<K, MODE_RESID>(v, a, shift, begin, end, st);
    case MODE_RESID | MODE_STOREZ: return op_launch<K, MODE_RESID | MODE_STOREZ>(v, a, shift, begin, end, st);
    case 0: return op_launch<K, 0>(v, a, shift, begin, end, st);
    case MODE_NOLS: return op_launch<K, MODE_NOLS>(v, a, shift, begin, end, st);
    case MODE_NEWTON: return op_launch<K, MODE_NEWTON>(v, a, shift, begin, end, st);
    default: return hipErrorInvalidValue;
  }
}

// FP32 instantiations: tangent modes only (the residual stays FP64)
template <int K>
static hipError_t op_dispatch(const DevView& v, int mode, const OpArgs<float>& a, double shift,
                              int64_t begin, int64_t end, hipStream_t st) {
  if (v.seg.list) {
    switch (mode) {
#define CASE(md) case md: return op_launch<K, md | MODE_SEG>(v, a, shift, begin, end, st);
      CASE(0) CASE(MODE_NOLS) CASE(MODE_NEWTON)
#undef CASE
      default: break;
    }
  }
  switch (mode) {
#define CASE(md) case md: return op_launch<K, md>(v, a, shift, begin, end, st);
    CASE(0) CASE(MODE_NOLS) CASE(MODE_NEWTON)
    CASE(MODE_TAU16) CASE(MODE_TAU16 | MODE_NOLS) CASE(MODE_TAU16 | MODE_NEWTON)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_elem(const DevView& v, int mode, const double* XP, const double* VT,
                       double* Zout, double* out, double shift, int64_t begin, int64_t end,
                       hipStream_t st) {
  if (end <= begin) return hipSuccess;
  const OpArgs<double> a{XP, VT, out, Zout};
  switch (v.K) {
#define CASE(k) case k: return op_dispatch<k>(v, mode, a, shift, begin, end, st);
    TSGLS_FOR_EACH_K_SMALL(CASE)
#undef CASE
#define CASE(k) case k: return op_big_dispatch<k>(v, mode, XP, VT, Zout, out, shift, begin, end, st);
    TSGLS_FOR_EACH_K_LARGE(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_elem_f32(const DevView& v, int mode, const float* XP, const float* VT,
                           float* out, double shift, int64_t begin, int64_t end, hipStream_t st) {
  if (end <= begin) return hipSuccess;
  if (mode & (MODE_RESID | MODE_STOREZ)) return hipErrorInvalidValue;
  if (!v.UT32 || !v.tau32 || (!v.Z32 && (mode & MODE_NEWTON))) return hipErrorInvalidValue;
  if ((mode & MODE_TAU16) && !v.tau16) return hipErrorInvalidValue;
  const OpArgs<float> a{XP, VT, out, nullptr};
  switch (v.K) {
#define CASE(k) case k: return op_dispatch<k>(v, mode, a, shift, begin, end, st);
    TSGLS_FOR_EACH_K_SMALL(CASE)
#undef CASE
#define CASE(k) case k: return op_big_dispatch<k>(v, mode, XP, VT, out, shift, begin, end, st);
    TSGLS_FOR_EACH_K_LARGE(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tsgls
