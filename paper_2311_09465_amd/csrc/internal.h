// Internal interface between the host library (host.cpp) and the gfx950
// kernels (elem.hip, face.hip, krylov.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsgls {

// Harmonic counts K the kernels are instantiated for.  The element operator,
// tau, the Jacobi diagonal and the tracer have register-blocked kernels for
// the small set and LDS-staged kernels for the large set (n = 63 modes per
// field does not fit the register-blocked lane layouts); the other kernels
// are instantiated for both.
#define TSGLS_FOR_EACH_K_SMALL(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(11) X(15)
#define TSGLS_FOR_EACH_K_LARGE(X) X(31)
#define TSGLS_FOR_EACH_K(X) TSGLS_FOR_EACH_K_SMALL(X) TSGLS_FOR_EACH_K_LARGE(X)

// Mode positions.  Inside the element operator the n = 2K+1 real modes of a
// field sit at "positions" p: mode 2k-1 (cos k wt) at p = 2k-2, mode 2k
// (sin k wt) at p = 2k-1, mode 0 at p = 2K; positions 2K+1 .. are padding.
// The two modes of one harmonic then sit at p and p^1, so the time
// derivative Omega pairs neighbouring lanes.
__host__ __device__ constexpr int pos_mode(int p, int K) {
  return p < 2 * K ? p + 1 : (p == 2 * K ? 0 : -1);
}
__host__ __device__ constexpr int mode_pos(int a, int K) { return a == 0 ? 2 * K : a - 1; }
// Packed upper triangle (row-major) of a symmetric n x n matrix, r <= c.
__host__ __device__ constexpr int pk_index(int r, int c, int n) {
  return r * n - (r * (r - 1)) / 2 + (c - r);
}

// tau is stored per element and quadrature point as the packed upper
// triangle over positions: tau[(e*4 + q)*P + pk_index(pr, pc, n)], e in
// processing order.  z = tau L(u) (Newton tangent) is stored as
// Z[((e*4 + q)*3 + i)*n + p].

// Element-operator modes (compile-time flags of the element kernel).
enum : int {
  MODE_RESID = 1,    // input is the state: A built from it, no input mask
  MODE_NEWTON = 2,   // keep the derivative of A (needs frozen tau L(u))
  MODE_NOLS = 4,     // drop least-squares terms of G_i and D_i
  MODE_STOREZ = 8,   // store z = tau L(u) (modal) during a residual pass
  MODE_TAU16 = 16,   // FP32 operator with tau read as bf16 (v.tau16)
  MODE_SEG = 32,     // element operator over the work list of segments in v.seg
};

// Device view of one mesh + linearization.  All pointers are device memory.
// Segments that sit out a pass (segmented contexts): skip[s] != 0 for the
// segment of node blocks [s nodes, (s+1) nodes).  tau (small harmonic
// counts) leaves such a segment's points untouched, the nodal-sample kernel
// its nodes, and the node gather writes zero rows for its nodes.  skip ==
// nullptr: none.  When the segments' elements are contiguous blocks of
// `elems` (segment s owns processing positions [s elems, (s+1) elems)),
// list / count (device) hold the segments taking part, and the element
// operator's launch runs over their elements only (its range is count *
// elems positions); without a list it computes every element.
struct SegMask {
  const int* skip = nullptr;
  int32_t nodes = 1;
  const int* list = nullptr;
  const int* count = nullptr;
  int32_t elems = 0;
};

struct DevView {
  int K;
  int64_t n_nodes, n_tets, n_faces;
  const int32_t* conn;       // [E][4] element nodes, processing (Morton) order
  const double* geo;         // [E][16]: grad N (a-major, 12), w = V/4, pad
  const uint8_t* nflag;      // [n_nodes] bit0: velocity Dirichlet
  const double* F;           // [n][M] phi_a(t_s), real orthonormal basis
  const double* UT;          // [n_nodes][3][M] frozen velocity samples
  const double* tau;         // [E][4][P] packed tau over positions
  const double* Z;           // [E][4][3][n] tau L(u) over positions
  const float* UT32;         // FP32 copies of UT, tau, Z (mixed-precision tangent) or null
  const float* tau32;
  const float* Z32;
  const uint16_t* tau16;     // tau rounded to bf16 (bit patterns), same layout, or null
  const int32_t* noff;       // [n_nodes+1] node -> incident element slots
  const int32_t* ninc;       // element*4 + local node, ascending element
  const int32_t* fconn;      // [nf][3] Neumann faces
  int64_t n_fnodes;          // distinct nodes of the Neumann faces
  const int32_t* fnode;      // [n_fnodes] node ids
  const int32_t* foff;       // [n_fnodes+1] CSR offsets into finc
  const int32_t* finc;       // incident (face*3 + local vertex), ascending
  const double* fgeo;        // [nf][4] unit outward normal, area
  const double* fh;          // [nf][n] traction modes (real basis) or null
  const double* aneg;        // [nf][3][P] |A_n|_- packed per face point
  double* fy;                // [nf][3][3][n] scratch: |A_n|_- u per face point
  double rho, mu, omega, C_I, beta;
  SegMask seg;               // segments skipped by k_op and k_tau (small K)
};

// Launchers (return hipError_t of the launch).  Element ranges [begin, end)
// are in processing (Morton) order; element kernels write per-element
// contributions [E][4 nodes][4 fields][n positions] (slot scaling) that
// launch_gather sums per node into slots.
hipError_t launch_geometry(const double* xyz, const int32_t* conn, double* geo,
                           int* bad, int64_t n_tets, hipStream_t st);
// XT[node][3][M]: time samples of the three velocity components;
// XP[node][4][PW]: the four fields' modes in the orthonormal basis at their
// positions (zero padding).  masked != 0 zeroes Dirichlet velocity rows.  The
// input is Y, or Y * Ys entrywise when Ys is not null.
// When fv is not null, the same launch also forms the Neumann face points of
// the input (as launch_face_point(*fv, Y, Ys, fresid, aneg)) in extra blocks.
// Nodes of segments flagged in mk are left as they are.
hipError_t launch_prep_time(int K, const double* Y, const double* Ys,
                            const uint8_t* nflag, int masked, const double* F,
                            double* XT, double* XP, int64_t n_nodes, hipStream_t st,
                            const DevView* fv = nullptr, const double* aneg = nullptr,
                            int fresid = 0, const SegMask& mk = SegMask());
// The same with FP32 outputs (the sums are formed in FP64).
hipError_t launch_prep_time_f32(int K, const double* Y, const double* Ys,
                                const uint8_t* nflag, int masked, const double* F,
                                float* XT, float* XP, int64_t n_nodes, hipStream_t st,
                                const DevView* fv = nullptr, const double* aneg = nullptr,
                                int fresid = 0, const SegMask& mk = SegMask());
// Positions per field row of XP (16 or 32).
int pos_width(int K);
// tau at every quadrature point.  Vin / Vout (optional, K <= 15 only):
// eigenvectors of S from an earlier linearization as the starting basis of
// the Jacobi iteration / the new eigenvectors, [E][4][n][n] (row a, column
// c).  The result does not depend on Vin beyond rounding (any orthonormal
// basis converges to the same tau).
hipError_t launch_tau(const DevView& v, const double* Y, double* tau,
                      hipStream_t st, const double* Vin = nullptr, double* Vout = nullptr);
// Element operator over elements [begin, end) (processing order); input
// modes from XP, direction samples VT (tangent modes), writes the per-element
// contributions out[E][4][4][n] over positions.  Zout (mode & MODE_STOREZ)
// receives tau L(u).
hipError_t launch_elem(const DevView& v, int mode, const double* XP,
                       const double* VT, double* Zout, double* out,
                       double shift, int64_t begin, int64_t end, hipStream_t st);
// Mixed-precision tangent: the same operator in FP32 (modes 0, MODE_NOLS,
// MODE_NEWTON) on the FP32 copies v.UT32, v.tau32, v.Z32; with MODE_TAU16
// also set, tau comes from the bf16 copy v.tau16 instead of v.tau32.
hipError_t launch_elem_f32(const DevView& v, int mode, const float* XP, const float* VT,
                           float* out, double shift, int64_t begin, int64_t end, hipStream_t st);
hipError_t launch_diag(const DevView& v, double* d, double shift,
                       int64_t begin, int64_t end, hipStream_t st);
// Neumann face terms added by the node gather: nfidx maps a node to its
// index in the Neumann-node list (-1 for other nodes), foff/finc list that
// node's incident (face, vertex) pairs in ascending face order, fy holds
// -(rho beta / 2)(area / 3) |A_n|_- u per face point (launch_face_point) and,
// for the residual (resid != 0), fh the traction modes.  nfidx == nullptr: no
// face terms.
struct FaceSum {
  const int32_t* nfidx = nullptr;
  const int32_t* foff = nullptr;
  const int32_t* finc = nullptr;
  const double* fy = nullptr;
  const double* fgeo = nullptr;
  const double* fh = nullptr;
  int resid = 0;
  int nfield = 3;   // leading fields that receive face terms (3 velocity; 1 for the tracer)
};
// out[node][4][S] = sum over incident (element, local node) of the ebuf rows
// mapped from positions to slots, in ascending element order (deterministic),
// then the node's face terms (fs).  Velocity rows of Dirichlet nodes (nflag
// bit 0) are written as zero.
hipError_t launch_gather(int K, const int32_t* noff, const int32_t* ninc,
                         const uint8_t* nflag, const double* ebuf, double* out,
                         int64_t n_nodes, hipStream_t st, const FaceSum& fs = FaceSum(),
                         const SegMask& mk = SegMask());
// The same from FP32 element rows (accumulated in FP64).
hipError_t launch_gather_f32(int K, const int32_t* noff, const int32_t* ninc,
                             const uint8_t* nflag, const float* ebuf, double* out,
                             int64_t n_nodes, hipStream_t st, const FaceSum& fs = FaceSum(),
                             const SegMask& mk = SegMask());
hipError_t launch_face_lin(const DevView& v, const double* Y, double* aneg,
                           hipStream_t st);
// Per Neumann face point: fy = -(rho beta / 2)(area / 3) |A_n|_- u with u the
// input (Y, times Ys when not null) at the point; Dirichlet velocity rows of
// a direction (resid == 0) are masked.  The node sums are taken by the gather.
hipError_t launch_face_point(const DevView& v, const double* Y, const double* Ys, int resid,
                             const double* aneg, hipStream_t st);
hipError_t launch_face_diag(const DevView& v, double* d, hipStream_t st);
hipError_t launch_diag_finish(int K, const uint8_t* nflag, double* d,
                              int64_t n_nodes, hipStream_t st);
bool supported_K(int K);
int supported_K_list(int* out, int cap);

// BLAS-1 style kernels on float64 vectors of length n.
hipError_t launch_zero(double* x, int64_t n, hipStream_t st);
hipError_t launch_copy(const double* x, double* y, int64_t n, hipStream_t st);
hipError_t launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t st);
hipError_t launch_scal_copy(double a, const double* x, double* y, int64_t n, hipStream_t st);
hipError_t launch_mul(const double* a, const double* x, double* y, int64_t n, hipStream_t st);
hipError_t launch_recip(double* x, int64_t n, hipStream_t st);
// x[i] = a
hipError_t launch_fill(double* x, double a, int64_t n, hipStream_t st);
// Tracer (convection-diffusion) element operator over elements [begin, end):
// input modes from XP field 0, velocity samples v.UT, tau v.tau (with kappa
// in place of nu); element rows [E][4][4][n] with the tracer in field 0.
hipError_t launch_cd(const DevView& v, const double* XP, double kappa, double* out, int64_t begin,
                     int64_t end, hipStream_t st);
// y = x rounded to FP32
hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t st);
// y = bit pattern of x rounded to bf16 (round to nearest even)
hipError_t launch_to_bf16(const double* x, uint16_t* y, int64_t n, hipStream_t st);
// Segmented launches.  A context may hold nseg independent problems whose
// unknowns are nseg contiguous equal segments of every vector.  Launchers
// that take (nseg, strides) run the same computation on each segment in one
// launch (the segment on a grid dimension); segment s reads and writes its
// operands offset by s times the stated stride.  nseg = 1 with zero strides
// is the unsegmented computation.  skip (device, per segment, may be null):
// segments flagged there are left untouched.
// partial[b*J + j] = sum over block b's chunk of V[j]*w; J <= 128.
hipError_t launch_multidot(const double* V, int64_t ldv, int J, const double* w,
                           double* partial, int nblocks, int64_t n, hipStream_t st,
                           int nseg = 1, int64_t sv = 0, int64_t sp = 0, const int* skip = nullptr);
// out[j] = sum_b partial[b*J + j] (fixed order)
hipError_t launch_reduce_partials(const double* partial, int nblocks, int J,
                                  double* out, hipStream_t st, int nseg = 1, int64_t sp = 0,
                                  int64_t so = 0, const int* skip = nullptr);
// w += sign sum_j V[j] h[j] (J <= 32; no update when h is null), then block partials [nblocks][Jo] of
// V[j] . w for j < Jd and, if self, w . w in slot Jd (Jo = Jd + self).
hipError_t launch_axpy_dot(const double* V, int64_t ldv, int J, const double* h, double sign,
                           double* w, int Jd, int self, double* partial, int nblocks, int64_t n,
                           hipStream_t st);
// Delayed Gram-Schmidt passes (J <= GS_DELAYED_MAX, the largest restart of
// the delayed GMRES).  Reduction: partials [nblocks][2J+3]
// of Q^T u, Q^T w, u.u, u.w, w.w.  Update: u <- (u - Q a) inv_nu,
// w <- (w - Q b - u h) inv_sigma with ab = [a (J); b (J)] on the device.
constexpr int GS_DELAYED_MAX = 128;
hipError_t launch_gs_reduce(const double* Q, int64_t ldq, int J, const double* u, const double* w,
                            double* partial, int nblocks, int64_t n, hipStream_t st, int nseg = 1,
                            int64_t sv = 0, int64_t sp = 0, const int* skip = nullptr);
// The coefficients ab = [a (J); b (J)] come either from device memory (ab) or
// from host memory (ab_host, passed by value as a kernel argument); exactly
// one of the two is not null.  (inv_nu, h, inv_sigma) are read from sc[0..2]
// on the device when sc is not null.  Segmented launches read ab and sc from
// the device (offset by s sd).
hipError_t launch_gs_update(const double* Q, int64_t ldq, int J, const double* ab,
                            const double* ab_host, double inv_nu, double h, double inv_sigma,
                            const double* sc, double* u, double* w, int64_t n, hipStream_t st,
                            int nseg = 1, int64_t sv = 0, int64_t sd = 0, const int* skip = nullptr);
// Device-side least-squares state of one GMRES(m) cycle (m <= 32), all device
// pointers: H, R [(m+1) m] column-major; cs, sn, y [m]; g [m+1]; ab [64];
// sc [8] = {1/nu, h, 1/sigma, beta, tol |r0|, 1/beta, |g_k|, -};
// st [5] = {k, cycle over, finalize pending, converged, non-finite estimate}.
// Segmented: segment s's doubles are offset by s sd and its st by s si;
// skip (device, per segment, may be null) marks segments that take no part
// in the cycle.
struct GmDev {
  double *H, *R, *cs, *sn, *g, *y, *ab, *sc;
  int* st;
  int m;
  int64_t sd = 0;
  int si = 0;
  const int* skip = nullptr;
};
hipError_t launch_gm_begin(const GmDev& d, const double* bb, double tol, int first, hipStream_t st,
                           int nseg = 1, int64_t sbb = 0);
hipError_t launch_gm_step(const GmDev& d, int j, const double* red, hipStream_t st, int nseg = 1,
                          int64_t sred = 0);
hipError_t launch_gm_final(const GmDev& d, const double* red, hipStream_t st, int nseg = 1,
                           int64_t sred = 0);
// x *= s[0]
hipError_t launch_scal_dev(double* x, const double* s, int64_t n, hipStream_t st, int nseg = 1,
                           int64_t sx = 0, int64_t ss = 0, const int* skip = nullptr);
// w -= sum_j V[j] h[j]
hipError_t launch_multiaxpy(const double* V, int64_t ldv, int J, const double* h,
                            double* w, int64_t n, hipStream_t st);
// y += sum_j V[j] c[j]  (c on device; segmented: c offset by s sc)
hipError_t launch_multiaxpy_add(const double* V, int64_t ldv, int J, const double* c,
                                double* y, int64_t n, hipStream_t st, int nseg = 1, int64_t sv = 0,
                                int64_t sc = 0, const int* skip = nullptr);
int multidot_blocks(int64_t n);

// Warm-start network (mlp.hip).  C[i][j] (ldc) = epilogue(sum_k A(i,k) B(k,j))
// with A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj]; bf16 != 0 rounds
// the operands to bf16 (FP32 accumulation).  epi 0: + bias (if not null),
// 1: tanh(. + bias), 2: . * (1 - H[i][j]^2).
hipError_t launch_mlp_gemm(int bf16, int epi, int M, int N, int Kd, const float* A, int64_t sai,
                           int64_t sak, const float* B, int64_t sbk, int64_t sbj,
                           const float* bias, const float* H, float* C, int64_t ldc,
                           hipStream_t st);
// dO = 2 (O - T) / cnt, loss[0] = mean (O - T)^2 over cnt entries
hipError_t launch_mse(const float* O, const float* T, float* dO, float* loss, int64_t cnt,
                      hipStream_t st);
// db[j] = sum_b dZ[b][j]
hipError_t launch_colsum(const float* dZ, int B, int N, float* db, hipStream_t st);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st);

}  // namespace tsgls
