// Device-side helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsgls {

// Sizes for K harmonics: n real modal coordinates per field (orthonormal
// basis 1, sqrt2 cos k wt, -sqrt2 sin k wt), S storage slots, M time samples
// (3K+1: products of two band-limited signals projected back to K harmonics
// are exact), P packed entries of a symmetric n x n matrix.
template <int K>
struct Dim {
  static constexpr int n = 2 * K + 1;
  static constexpr int S = 2 * K + 2;
  static constexpr int M = 3 * K + 1;
  static constexpr int P = n * (n + 1) / 2;
};

// 4-point degree-2 rule on the tet: barycentric alpha at node q, beta elsewhere.
#define TS_QA 0.58541019662496845446
#define TS_QB 0.13819660112501051518
#define TS_SQ2 1.41421356237309504880
#define TS_RS2 0.70710678118654752440

__device__ __forceinline__ double lamq(int q, int b) { return q == b ? TS_QA : TS_QB; }
// 3-point degree-2 rule on a triangle: 2/3 at node q, 1/6 elsewhere.
__device__ __forceinline__ double flam(int q, int b) { return q == b ? (2.0 / 3.0) : (1.0 / 6.0); }

// Storage slot of orthonormal coordinate a (a = 2k-1 -> Re c_k, a = 2k -> Im c_k).
__device__ __forceinline__ double slot_x(const double* ys, int a) {
  return a == 0 ? ys[0] : TS_SQ2 * ys[a + 1];
}

// Compile-time trigonometry for the sampling table (Taylor series after
// reduction to [-pi, pi]; exact integer angle reduction r = k s mod M).
constexpr double cx_pi = 3.14159265358979323846264338327950288;

constexpr double cx_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 30; ++i) {
    term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double cx_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 30; ++i) {
    term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}

// f[a][s] = phi_a(t_s): phi_0 = 1, phi_{2k-1} = sqrt2 cos(2 pi k s / M),
// phi_{2k} = -sqrt2 sin(2 pi k s / M); b[a][s] = f[a][s] / M (projection).
template <int K>
struct SampleTable {
  static constexpr int n = 2 * K + 1, M = 3 * K + 1;
  double f[n][M];
  double b[n][M];
  constexpr SampleTable() : f(), b() {
    for (int s = 0; s < M; ++s) {
      f[0][s] = 1.0;
      for (int k = 1; k <= K; ++k) {
        const int r = (k * s) % M;
        double th = 2.0 * cx_pi * r / M;          // in [0, 2 pi)
        if (th > cx_pi) th -= 2.0 * cx_pi;        // in (-pi, pi]
        double cs = 1.0, sg = 1.0;
        if (th > 0.5 * cx_pi) {                   // sin(pi - x) = sin x, cos(pi - x) = -cos x
          th = cx_pi - th;
          cs = -1.0;
        } else if (th < -0.5 * cx_pi) {
          th = -cx_pi - th;
          cs = -1.0;
        }
        f[2 * k - 1][s] = TS_SQ2 * cs * cx_cos(th);
        f[2 * k][s] = -TS_SQ2 * sg * cx_sin(th);
      }
      for (int a = 0; a < n; ++a) b[a][s] = f[a][s] / M;
    }
  }
};

// The harmonics above K that M = 3K+1 samples still resolve: K real sampled
// vectors v_r (cos and sin of k = K+1 .. M/2; a lone cos at the Nyquist
// frequency when M is even), with v_r . v_r = 1 / coef_r.  The band-limiting
// projection on the samples is x - sum_r coef_r v_r (v_r . x).
template <int K>
struct AliasTable {
  static constexpr int M = 3 * K + 1, R = K > 0 ? K : 1;
  double v[R][M];
  double coef[R];
  constexpr AliasTable() : v(), coef() {
    int r = 0;
    for (int k = K + 1; 2 * k <= M && r < K; ++k) {
      const bool nyq = 2 * k == M;
      for (int s = 0; s < M; ++s) {
        double th = 2.0 * cx_pi * ((k * s) % M) / M;
        if (th > cx_pi) th -= 2.0 * cx_pi;
        double cs = 1.0, ts = th;
        if (th > 0.5 * cx_pi) {
          ts = cx_pi - th;
          cs = -1.0;
        } else if (th < -0.5 * cx_pi) {
          ts = -cx_pi - th;
          cs = -1.0;
        }
        v[r][s] = cs * cx_cos(ts);
        if (!nyq) v[r + 1][s] = cx_sin(ts);
      }
      coef[r] = nyq ? 1.0 / M : 2.0 / M;
      if (!nyq) coef[r + 1] = 2.0 / M;
      r += nyq ? 1 : 2;
    }
  }
};

// (Omega x)_a in the orthonormal basis: time derivative, skew-symmetric.
template <int n>
__device__ __forceinline__ double omx(const double* x, int a, double omega) {
  if (a == 0) return 0.0;
  if (a & 1) return -((a + 1) >> 1) * omega * x[a + 1];
  return (a >> 1) * omega * x[a - 1];
}

template <int n>
__device__ __forceinline__ void packed_rc(int p, int& r, int& c) {
  int a = 0, off = 0;
  while (p >= off + (n - a)) { off += n - a; ++a; }
  r = a;
  c = a + (p - off);
}

// Value held by lane (lane ^ k), 0 < k < 64.  XOR 1..3 within a quad, 7
// within an 8-lane half row, 8 and 15 within a 16-lane row are single DPP
// moves; other distances go through the LDS crossbar (ds_bpermute).
template <int k>
__device__ __forceinline__ int xor_lane(int x) {
  if constexpr (k >= 1 && k <= 3) {
    constexpr int sel = k;   // quad_perm: lane i takes lane i ^ k
    constexpr int ctrl = (0 ^ sel) | ((1 ^ sel) << 2) | ((2 ^ sel) << 4) | ((3 ^ sel) << 6);
    return __builtin_amdgcn_mov_dpp(x, ctrl, 0xF, 0xF, false);
  } else if constexpr (k == 7) {
    return __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);   // row_half_mirror
  } else if constexpr (k == 8) {
    return __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);   // row_ror:8
  } else if constexpr (k == 15) {
    return __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false);   // row_mirror
  } else {
    return __shfl_xor(x, k);
  }
}
template <int k>
__device__ __forceinline__ double xor_lane(double x) {
  return __hiloint2double(xor_lane<k>(__double2hiint(x)), xor_lane<k>(__double2loint(x)));
}

// 1/x and 1/sqrt(x) for x > 0 from the hardware estimates refined by two
// Newton steps (quadratic convergence: full double precision).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// One round of the one-sided Jacobi: the columns of lanes c and c ^ k are
// rotated to be orthogonal.  Both lanes of a pair evaluate the same rotation
// bit for bit (same operands in the same order).  nrm is this lane's |w|^2,
// kept up to date; big is set when (w_c . w_d)^2 > 1e-14 |w_c|^2 |w_d|^2.
// A lane whose group is done (both lanes of a pair belong to one group)
// rotates nothing.
template <int n, int k>
__device__ __forceinline__ void jacobi_round(double (&w)[n], double& nrm, int c, int& big,
                                             int& rot, int done) {
  double o[n];
#pragma unroll
  for (int a = 0; a < n; ++a) o[a] = xor_lane<k>(w[a]);
  const double onrm = xor_lane<k>(nrm);
  const bool low = c < (c ^ k);
  // the same sum on both lanes (fma is commutative in its factors)
  double ga = 0.0;
#pragma unroll
  for (int a = 0; a < n; ++a) ga = fma(w[a], o[a], ga);
  const double al = low ? nrm : onrm, be = low ? onrm : nrm;
  const double ab = al * be;
  const double g2 = ga * ga;
  if (!done && g2 > 1e-14 * ab) big = 1;
  if (!done && g2 > 1e-30 * ab) {
    // tan(theta) = 2 g sgn(d) / (|d| + sqrt(d^2 + 4 g^2)), d = be - al
    const double d = be - al;
    const double r2 = fma(d, d, 4.0 * g2);
    const double r = r2 * rsq_nr(r2);
    const double t = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) * rcp_nr(fabs(d) + r);
    const double cs = rsq_nr(fma(t, t, 1.0));
    const double sn = cs * t;
    // lo' = cs lo - sn hi, hi' = sn lo + cs hi: each lane keeps its own column
    const double so = low ? -sn : sn;
#pragma unroll
    for (int a = 0; a < n; ++a) w[a] = fma(so, o[a], cs * w[a]);
    const double c2 = cs * cs, s2 = sn * sn, cs2 = 2.0 * so * cs * ga;
    nrm = fma(c2, nrm, fma(s2, onrm, cs2));
    rot = 1;
  }
}

template <int n, int k, int NP>
__device__ __forceinline__ void jacobi_rounds(double (&w)[n], double& nrm, int c, int& big,
                                              int& rot, int done) {
  if constexpr (k < NP) {
    jacobi_round<n, k>(w, nrm, c, big, rot, done);
    jacobi_rounds<n, k + 1, NP>(w, nrm, c, big, rot, done);
  }
}

// OR of an int over the NP lanes of this lane's group.
template <int NP>
__device__ __forceinline__ int group_or(int x) {
#pragma unroll
  for (int k = 1; k < NP; k <<= 1) x |= __shfl_xor(x, k);
  return x;
}

// One-sided (Hestenes) cyclic Jacobi on the columns held by a group of NP
// lanes: lane c holds column c (n entries, zero for c >= n).  Pairs per
// round are (c, c xor k), k = 1..NP-1, which covers every pair once per
// sweep.  Sweeps stop after the first one whose largest rotation was below
// 1e-7 in relative terms (convergence is quadratic: the columns are then
// orthogonal to about 1e-14 relative), or that rotated nothing.  Each group
// stops on its own: the wave sweeps until all its groups are done, and a
// group that is done rotates nothing more, so a group's result does not
// depend on which other groups share its wave.
template <int n, int NP>
__device__ __forceinline__ void jacobi_columns(double (&w)[n], int c) {
  int done = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double nrm = 0.0;
#pragma unroll
    for (int a = 0; a < n; ++a) nrm = fma(w[a], w[a], nrm);
    int big = 0, rot = 0;
    jacobi_rounds<n, 1, NP>(w, nrm, c, big, rot, done);
    if (!group_or<NP>(big) || !group_or<NP>(rot)) done = 1;
    if (__all(done)) break;
  }
}

template <int NP>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int k = 1; k < NP; k <<= 1) x += __shfl_xor(x, k);
  return x;
}

// Workgroups are handed to the 8 XCDs of the chip round-robin by block id.
// xcd_block maps block id b of a grid of nb blocks to a logical block so that
// each XCD works on one contiguous range of logical blocks: elements that
// share nodes then share that XCD's L2.  A bijection on [0, nb).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  constexpr int NX = 8;
  const int64_t x = b % NX, j = b / NX;
  const int64_t q = nb / NX, r = nb % NX;
  return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

constexpr int np_of(int n) {
  return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : 64;
}

}  // namespace tsgls
