// One Neumann face point of the backflow term (section "Stabilizing
// simulations in the presence of backflow"): lane (i, m) of the block forms
// y_i[m] = coef sum_c (|A_n|_-)_mc u_i[c] with u the input interpolated at the
// point (Dirichlet rows of a direction masked, input = Y * Ys when Ys is
// given), coef = -(rho beta / 2) area / 3, into v.fy.  Used by the face-point
// kernel and by the extra blocks of the nodal-sample kernel.  Every thread of
// the block must call it (it contains a barrier); su holds 3n doubles of LDS.
#pragma once
#include "common.cuh"
#include "internal.h"

namespace tsgls {

template <int K>
__device__ __forceinline__ void face_point_block(const DevView& v, const double* __restrict__ Y,
                                                 const double* __restrict__ Ys, int resid,
                                                 const double* __restrict__ an, int64_t fq, int t,
                                                 double* su) {
  constexpr int n = Dim<K>::n, S = Dim<K>::S, P = Dim<K>::P;
  const int64_t f = fq / 3;
  const int q = (int)(fq % 3);
  const int i = t / n, m = t % n;
  if (t < 3 * n) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int64_t nb = v.fconn[f * 3 + b];
      const bool z = !resid && (v.nflag[nb] & 1);
      const int64_t o = (nb * 4 + i) * S + (m == 0 ? 0 : m + 1);
      const double x = (m == 0 ? 1.0 : TS_SQ2) * (Ys ? Y[o] * Ys[o] : Y[o]);
      acc += z ? 0.0 : flam(q, b) * x;
    }
    su[i * n + m] = acc;
  }
  __syncthreads();
  if (t < 3 * n) {
    const double* ap = an + fq * P;
    double acc = 0.0;
#pragma unroll
    for (int cc = 0; cc < n; ++cc) {
      const int lo = m < cc ? m : cc, hi = m < cc ? cc : m;
      acc = fma(ap[lo * n - (lo * (lo - 1)) / 2 + (hi - lo)], su[i * n + cc], acc);
    }
    const double coef = -0.5 * v.rho * v.beta * v.fgeo[f * 4 + 3] / 3.0;
    v.fy[fq * (3 * n) + i * n + m] = coef * acc;
  }
}

}  // namespace tsgls
