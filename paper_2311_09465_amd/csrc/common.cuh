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

// One-sided (Hestenes) cyclic Jacobi on the columns held by a group of NP
// lanes: lane c holds column c (n entries, zero for c >= n).  Pairs per
// round are (c, c xor k), k = 1..NP-1, which covers every pair once per
// sweep.  Both lanes of a pair compute the same rotation bit for bit.  On
// return the columns are mutually orthogonal to working precision.
template <int n, int NP>
__device__ __forceinline__ void jacobi_columns(double (&w)[n], int c) {
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rot = 0;
#pragma unroll 1
    for (int k = 1; k < NP; ++k) {
      double o[n];
#pragma unroll
      for (int a = 0; a < n; ++a) o[a] = __shfl_xor(w[a], k);
      const bool low = c < (c ^ k);
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        const double lo = low ? w[a] : o[a];
        const double hi = low ? o[a] : w[a];
        al = fma(lo, lo, al);
        be = fma(hi, hi, be);
        ga = fma(lo, hi, ga);
      }
      if (fabs(ga) > tol * sqrt(al * be)) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
#pragma unroll
        for (int a = 0; a < n; ++a) {
          const double lo = low ? w[a] : o[a];
          const double hi = low ? o[a] : w[a];
          w[a] = low ? (cs * lo - sn * hi) : (sn * lo + cs * hi);
        }
        rot = 1;
      }
    }
    if (!__any(rot)) break;
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
