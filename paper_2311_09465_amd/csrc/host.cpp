// Host side of the library: context, mesh checks, Morton order and node incidence,
// the public C ABI (include/tsgls.h) and the Newton-GMRES driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tsgls.h"
#include "internal.h"

using namespace tsgls;

struct tsgls_ctx {
  tsgls_params p{};
  hipStream_t st = nullptr;
  int dev = 0;                  // HIP device current at tsgls_create
  int K = 0, n = 1, S = 2, M = 1, P = 1;
  int64_t nn = 0, E = 0, nf = 0;
  std::vector<int32_t> perm;    // processing position -> input element index (Morton order)
  int32_t* noff = nullptr;      // [n_nodes+1] CSR offsets: node -> incident element slots
  int32_t* ninc = nullptr;      // [4E] incident (element*4 + local node), ascending element
  double* ebuf = nullptr;       // [E][4][4][2K+1] per-element contributions over positions
  std::vector<double> hxyz;     // host copy of the coordinates (face geometry)
  int32_t* conn = nullptr;
  double* geo = nullptr;
  uint8_t* nflag = nullptr;
  double* F = nullptr;
  double* UT = nullptr;
  double* VT = nullptr;
  double* XP = nullptr;         // [n_nodes][4][PW] modes at their positions (operator input)
  double* tau = nullptr;
  double* tauV = nullptr;       // [E][4][n][n] eigenvectors of S at the last linearization
                                // (warm start of the next one; K <= 15), or null
  bool tauV_ok = false;         // tauV holds orthonormal eigenvectors
  double* Z = nullptr;
  double* rs = nullptr;         // scratch residual for linearize
  int32_t* fconn = nullptr;
  int64_t n_fnodes = 0;
  int32_t* fnode = nullptr;
  int32_t* foff = nullptr;
  int32_t* finc = nullptr;
  int32_t* nfidx = nullptr;     // [nn] node -> Neumann-node index, -1 elsewhere
  double* fgeo = nullptr;
  double* fh = nullptr;
  double* aneg = nullptr;
  double* fy = nullptr;         // [nf][3][3][n] face-point scratch
  // residual-only scratch (keeps the linearization intact)
  double* UTr = nullptr;
  double* taur = nullptr;
  double* anegr = nullptr;
  // Krylov workspace
  int m_alloc = 0;
  double* V = nullptr;
  double* kx = nullptr;
  double* kt = nullptr;
  double* kt2 = nullptr;
  double* ybak = nullptr;       // previous iterate (rejected pseudo-time steps)
  double* minv = nullptr;
  double* partial = nullptr;
  double* dh = nullptr;
  double* hp = nullptr;         // pinned host staging [4096] for the Krylov scalars:
                                // [0, 2048) device->host, [2560, 3584) least-squares
                                // solution (the Gram-Schmidt coefficients of the delayed
                                // GMRES go as kernel arguments)
  double* hpd = nullptr;        // device address of hp (the delayed GMRES's reductions
                                // are written there by the GPU directly)
  bool linearized = false;
  // tracer mode (convection-diffusion of a scalar in field 0 by the frozen
  // velocity of yvel): residual, tangent and solve use the tracer operator
  bool tracer = false;
  double kappa = 0.0;
  int stabilized = 1;
  double* yvel = nullptr;
  // graph-captured GMRES cycles (device-side least squares)
  hipStream_t gst = nullptr;    // capture / replay stream
  hipEvent_t gev[2] = {nullptr, nullptr};
  hipGraphExec_t gexec = nullptr;
  struct GraphKey {
    int m = -1, jac = -1, prec = -1;
    double dt = 0.0;
    const double* b = nullptr;
    double* x = nullptr;
  } gkey;
  GmDev gm{};
  double* gmbuf = nullptr;
  // independent problems held as nseg equal contiguous segments of the nodes
  // (tsgls_set_segments); 1 = one problem.  The graph cycle keeps per
  // segment: reductions [nseg][128] (red at 0, |r|^2 at 96), block partials
  // [nseg][nb * 67], squared norms [nseg]; pinned staging for the status
  // words and norms.
  int nseg = 1;
  bool seg_checked = false;     // elements and faces verified to stay in their segment
  bool seg_mask_on = false;     // element kernels and gathers skip the segments flagged in gm.skip
  double* segred = nullptr;
  double* segpart = nullptr;
  double* segnrm = nullptr;
  int* hseg = nullptr;          // [nseg][8] status, then the mask: [nseg] skip flags,
                                // [nseg] list of the segments taking part, their count
  int32_t seg_elems = 0;        // elements per segment when all segments have the same
                                // number (then stored segment-major), else 0
  double* hsegd = nullptr;      // [nseg] norms, [nseg] tolerances
  // FP32 copies of the linearization for the mixed-precision tangent
  // (allocated on first use; the FP32 modes, samples and element rows reuse
  // the FP64 buffers XP, VT and ebuf, which they fit in half)
  float* tau32 = nullptr;
  float* UT32 = nullptr;
  float* Z32 = nullptr;
  bool lin32 = false;     // the copies match the last linearize
  uint16_t* tau16 = nullptr;   // tau rounded to bf16 (TSGLS_PREC_BF16), allocated on first use
  bool lin16 = false;          // tau16 matches the last linearize
  // optional per-launch timing with HIP events (benchmark support)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_recs;
  size_t dev_bytes = 0;
  std::vector<void*> allocs;
  std::string err;
};

namespace {

int fail(tsgls_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, TSGLS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

#define CHK(call)                    \
  do {                               \
    int rc_ = (call);                \
    if (rc_ != TSGLS_OK) return rc_; \
  } while (0)

template <class T>
int dalloc(tsgls_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(c, TSGLS_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
  c->allocs.push_back(q);
  c->dev_bytes += count * sizeof(T);
  *p = static_cast<T*>(q);
  return TSGLS_OK;
}

void dfree(tsgls_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  (void)hipFree(p);
}

// Morton (Z-order) key of a point in the unit cube, 21 bits per axis.
uint64_t morton3(double x, double y, double z) {
  auto spread = [](uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
  };
  auto q = [](double t) { return (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0)); };
  return spread(q(x)) | spread(q(y)) << 1 | spread(q(z)) << 2;
}

DevView view(const tsgls_ctx* c) {
  DevView v{};
  v.K = c->K;
  v.n_nodes = c->nn;
  v.n_tets = c->E;
  v.n_faces = c->nf;
  v.conn = c->conn;
  v.geo = c->geo;
  v.nflag = c->nflag;
  v.F = c->F;
  v.UT = c->UT;
  v.tau = c->tau;
  v.Z = c->Z;
  v.UT32 = c->UT32;
  v.tau32 = c->tau32;
  v.Z32 = c->Z32;
  v.tau16 = c->tau16;
  v.noff = c->noff;
  v.ninc = c->ninc;
  v.fconn = c->fconn;
  v.n_fnodes = c->n_fnodes;
  v.fnode = c->fnode;
  v.foff = c->foff;
  v.finc = c->finc;
  v.fgeo = c->fgeo;
  v.fh = c->fh;
  v.aneg = c->aneg;
  v.fy = c->fy;
  v.rho = c->p.rho;
  v.mu = c->p.mu;
  v.omega = c->p.omega;
  v.C_I = c->p.C_I;
  v.beta = c->p.backflow_beta;
  if (c->seg_mask_on && c->nseg > 1 && c->gm.skip) {
    v.seg.skip = c->gm.skip;
    v.seg.nodes = (int32_t)(c->nn / c->nseg);
    if (c->seg_elems > 0) {
      v.seg.list = c->gm.skip + c->nseg;
      v.seg.count = c->gm.skip + 2 * c->nseg;
      v.seg.elems = c->seg_elems;
    }
  }
  return v;
}

int64_t ndof(const tsgls_ctx* c) { return c->nn * 4 * c->S; }

hipEvent_t next_event(tsgls_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// Records an event pair around one launch when profiling is on.
struct ProfScope {
  tsgls_ctx* c;
  int which;
  hipEvent_t b = nullptr;
  ProfScope(tsgls_ctx* ctx, int w) : c(ctx), which(w) {
    if (c->prof) {
      b = next_event(c);
      if (b) (void)hipEventRecord(b, c->st);
    }
  }
  ~ProfScope() {
    if (c->prof && b) {
      hipEvent_t e = next_event(c);
      if (e) {
        (void)hipEventRecord(e, c->st);
        c->prof_recs.push_back({which, {b, e}});
      }
    }
  }
};

// Face terms for the node gather (none without Neumann faces).
FaceSum face_sum(const tsgls_ctx* c, int resid) {
  FaceSum fs;
  if (c->nf == 0) return fs;
  fs.nfidx = c->nfidx;
  fs.foff = c->foff;
  fs.finc = c->finc;
  fs.fy = c->fy;
  fs.fgeo = c->fgeo;
  fs.fh = c->tracer ? nullptr : c->fh;
  fs.resid = resid;
  fs.nfield = c->tracer ? 1 : 3;   // the tracer is field 0 and has no traction
  return fs;
}

// Volume + face terms of the operator into out (overwritten).  The input's
// modes must already be in c->XP (launch_prep_time); Y is the input vector
// itself (face terms).  faces_ready: the face points of Y were formed with
// its nodal samples (launch_prep_time with the face view), so they are not
// launched here.
int apply_operator(tsgls_ctx* c, const DevView& v, int mode, const double* Y, const double* VTp,
                   double* Zout, double* out, double shift, const double* an, int resid,
                   const double* Ys = nullptr, bool faces_ready = false) {
  const int which = (mode & MODE_RESID) ? TSGLS_PROF_ELEM_RESIDUAL : TSGLS_PROF_ELEM_TANGENT;
  if (c->nf && !faces_ready) {   // face points first (they need only the input); the gather adds them
    ProfScope ps(c, TSGLS_PROF_FACE);
    HIPCHK(c, launch_face_point(v, Y, Ys, resid, an, c->st));
  }
  {
    ProfScope ps(c, which);
    HIPCHK(c, launch_elem(v, mode, c->XP, VTp, Zout, c->ebuf, shift, 0, c->E, c->st));
  }
  {
    ProfScope ps(c, TSGLS_PROF_GATHER);
    HIPCHK(c, launch_gather(c->K, c->noff, c->ninc, c->nflag, c->ebuf, out, c->nn, c->st,
                            face_sum(c, resid), v.seg));
  }
  return TSGLS_OK;
}

// Tracer operator applied to the modes in c->XP (element kernel + node sums)
// and, on Neumann faces, its backflow term -(w, (beta/2)|A_n|_- phi) for the
// input Y (times Ys when given; resid: Dirichlet entries of Y not masked).
int apply_tracer(tsgls_ctx* c, double* out, const double* Y, const double* Ys, int resid) {
  DevView v = view(c);
  if (c->nf) {
    DevView vf = v;
    vf.rho = 1.0;   // the tracer's backflow term carries no density
    ProfScope ps(c, TSGLS_PROF_FACE);
    HIPCHK(c, launch_face_point(vf, Y, Ys, resid, c->aneg, c->st));
  }
  {
    ProfScope ps(c, TSGLS_PROF_ELEM_TANGENT);
    HIPCHK(c, launch_cd(v, c->XP, c->kappa, c->ebuf, 0, c->E, c->st));
  }
  ProfScope ps(c, TSGLS_PROF_GATHER);
  HIPCHK(c, launch_gather(c->K, c->noff, c->ninc, c->nflag, c->ebuf, out, c->nn, c->st,
                          face_sum(c, resid)));
  return TSGLS_OK;
}

// Tracer linearization: velocity samples and tau (kappa in place of nu, zero
// for the Galerkin method) from the frozen velocity; the residual of y (the
// operator is linear in the tracer) if r is not null.
int linearize_tracer(tsgls_ctx* c, const double* y, double* r) {
  DevView v = view(c);
  v.mu = c->kappa;
  v.rho = 1.0;
  HIPCHK(c, launch_prep_time(c->K, c->yvel, nullptr, c->nflag, 0, c->F, c->UT, c->XP, c->nn, c->st));
  if (c->stabilized) {
    ProfScope ps(c, TSGLS_PROF_TAU);
    HIPCHK(c, launch_tau(v, c->yvel, c->tau, c->st));
  } else {
    HIPCHK(c, launch_zero(c->tau, c->E * 4 * c->P, c->st));
  }
  if (c->nf) HIPCHK(c, launch_face_lin(v, c->UT, c->aneg, c->st));   // |A_n|_- of the velocity
  c->linearized = true;
  c->lin32 = false;
  c->lin16 = false;
  if (!r) return TSGLS_OK;
  HIPCHK(c, launch_prep_time(c->K, y, nullptr, c->nflag, 0, c->F, c->VT, c->XP, c->nn, c->st));
  return apply_tracer(c, r, y, nullptr, 1);
}

// Eigenvectors of S kept between linearizations (the Jacobi iteration of tau
// starts from them); allocated on the first linearization for K <= 15.  A
// failed allocation only means cold starts.
void ensure_tauV(tsgls_ctx* c) {
  if (c->tauV || c->K > 15) return;
  const size_t cnt = (size_t)c->E * 4 * c->n * c->n;
  void* q = nullptr;
  if (hipMalloc(&q, cnt * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  c->allocs.push_back(q);
  c->dev_bytes += cnt * sizeof(double);
  c->tauV = static_cast<double*>(q);
  c->tauV_ok = false;
}

int linearize_impl(tsgls_ctx* c, const double* y, double* r) {
  if (c->tracer) return linearize_tracer(c, y, r ? r : c->rs);
  DevView v = view(c);
  c->lin32 = false;
  c->lin16 = false;
  ensure_tauV(c);
  HIPCHK(c, launch_prep_time(c->K, y, nullptr, c->nflag, 0, c->F, c->UT, c->XP, c->nn, c->st));
  {
    ProfScope ps(c, TSGLS_PROF_TAU);
    HIPCHK(c, launch_tau(v, y, c->tau, c->st, c->tauV_ok ? c->tauV : nullptr, c->tauV));
    c->tauV_ok = c->tauV != nullptr;
  }
  HIPCHK(c, launch_face_lin(v, c->UT, c->aneg, c->st));
  double* rr = r ? r : c->rs;
  CHK(apply_operator(c, v, MODE_RESID | MODE_STOREZ, y, nullptr, c->Z, rr, 0.0, c->aneg, 1));
  c->linearized = true;
  return TSGLS_OK;
}

// FP32 copies of tau, the velocity samples and tau L(u) of the last
// linearization (made once per linearization, on the first FP32 product).
int ensure_lin32(tsgls_ctx* c) {
  if (c->lin32) return TSGLS_OK;
  if (!c->tau32) {
    CHK(dalloc(c, &c->tau32, (size_t)c->E * 4 * c->P));
    CHK(dalloc(c, &c->UT32, (size_t)c->nn * 3 * c->M));
    CHK(dalloc(c, &c->Z32, (size_t)c->E * 12 * c->n));
  }
  HIPCHK(c, launch_to_f32(c->tau, c->tau32, c->E * 4 * c->P, c->st));
  HIPCHK(c, launch_to_f32(c->UT, c->UT32, c->nn * 3 * c->M, c->st));
  HIPCHK(c, launch_to_f32(c->Z, c->Z32, c->E * 12 * c->n, c->st));
  c->lin32 = true;
  return TSGLS_OK;
}

// bf16 copy of tau for TSGLS_PREC_BF16 (made once per linearization).
int ensure_tau16(tsgls_ctx* c) {
  if (c->lin16) return TSGLS_OK;
  if (!c->tau16) CHK(dalloc(c, &c->tau16, (size_t)c->E * 4 * c->P));
  HIPCHK(c, launch_to_bf16(c->tau, c->tau16, c->E * 4 * c->P, c->st));
  c->lin16 = true;
  return TSGLS_OK;
}

// out = J (x * xs) (xs: optional entrywise scale of the input, e.g. the
// right preconditioner inside GMRES).  prec TSGLS_PREC_F32 (or _BF16, tau in
// bf16) runs the element
// operator in FP32; the node sums and the face terms stay FP64.
int jv_impl(tsgls_ctx* c, const double* x, double* out, int jac, double dt, const double* xs = nullptr,
            int prec = TSGLS_PREC_F64) {
  if (!c->linearized) return fail(c, TSGLS_ESTATE, "jv before linearize");
  if (c->tracer) {   // the tracer operator is linear: its tangent is itself
    if (prec != TSGLS_PREC_F64) return fail(c, TSGLS_EINVAL, "the tracer operator runs in FP64 only");
    HIPCHK(c, launch_prep_time(c->K, x, xs, c->nflag, 1, c->F, c->VT, c->XP, c->nn, c->st));
    return apply_tracer(c, out, x, xs, 0);
  }
  DevView v = view(c);
  const int mode = jac == TSGLS_JAC_PICARD ? 0 : jac == TSGLS_JAC_PICARD_NOLS ? MODE_NOLS : MODE_NEWTON;
  const double shift = dt > 0 ? 1.5 * c->p.rho / dt : 0.0;
  const DevView* fv = c->nf ? &v : nullptr;   // face points in the same launch as the samples
  if (prec == TSGLS_PREC_F64) {
    HIPCHK(c, launch_prep_time(c->K, x, xs, c->nflag, 1, c->F, c->VT, c->XP, c->nn, c->st, fv,
                               c->aneg, 0, v.seg));
    return apply_operator(c, v, mode, x, c->VT, nullptr, out, shift, c->aneg, 0, xs, true);
  }
  CHK(ensure_lin32(c));
  if (prec == TSGLS_PREC_BF16) CHK(ensure_tau16(c));
  v = view(c);
  const int mode32 = prec == TSGLS_PREC_BF16 ? (mode | MODE_TAU16) : mode;
  float* XP32 = reinterpret_cast<float*>(c->XP);
  float* VT32 = reinterpret_cast<float*>(c->VT);
  float* eb32 = reinterpret_cast<float*>(c->ebuf);
  HIPCHK(c, launch_prep_time_f32(c->K, x, xs, c->nflag, 1, c->F, VT32, XP32, c->nn, c->st,
                                 c->nf ? &v : nullptr, c->aneg, 0, v.seg));
  {
    ProfScope ps(c, TSGLS_PROF_ELEM_TANGENT);
    HIPCHK(c, launch_elem_f32(v, mode32, XP32, VT32, eb32, shift, 0, c->E, c->st));
  }
  {
    ProfScope ps(c, TSGLS_PROF_GATHER);
    HIPCHK(c, launch_gather_f32(c->K, c->noff, c->ninc, c->nflag, eb32, out, c->nn, c->st,
                                face_sum(c, 0), v.seg));
  }
  return TSGLS_OK;
}

int diag_impl(tsgls_ctx* c, double* d, double dt) {
  if (!c->linearized) return fail(c, TSGLS_ESTATE, "jacobi_diag before linearize");
  if (c->tracer) {   // no preconditioner for the tracer: unit diagonal
    HIPCHK(c, launch_fill(d, 1.0, ndof(c), c->st));
    return TSGLS_OK;
  }
  DevView v = view(c);
  const double shift = dt > 0 ? 1.5 * c->p.rho / dt : 0.0;
  {
    ProfScope ps(c, TSGLS_PROF_DIAG);
    HIPCHK(c, launch_diag(v, c->ebuf, shift, 0, c->E, c->st));
  }
  HIPCHK(c, launch_gather(c->K, c->noff, c->ninc, c->nflag, c->ebuf, d, c->nn, c->st));
  if (c->nf) HIPCHK(c, launch_face_diag(v, d, c->st));
  HIPCHK(c, launch_diag_finish(c->K, c->nflag, d, c->nn, c->st));
  return TSGLS_OK;
}

// Deterministic dot products of J vectors (rows of V, leading dim ld) with w;
// result to the device array out and, if host != null, to host memory.
int multidot(tsgls_ctx* c, const double* V, int64_t ld, int J, const double* w, double* out,
             double* host) {
  const int64_t n = ndof(c);
  const int nb = multidot_blocks(n);
  HIPCHK(c, launch_multidot(V, ld, J, w, c->partial, nb, n, c->st));
  HIPCHK(c, launch_reduce_partials(c->partial, nb, J, out, c->st));
  if (host) {
    HIPCHK(c, hipMemcpyAsync(c->hp, out, J * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::copy(c->hp, c->hp + J, host);
  }
  return TSGLS_OK;
}

int norm2(tsgls_ctx* c, const double* x, double* nrm) {
  double h = 0.0;
  CHK(multidot(c, x, 0, 1, x, c->dh + 2048, &h));
  *nrm = std::sqrt(h);
  return TSGLS_OK;
}

// A captured GMRES cycle holds the device addresses of the Krylov basis, of
// the face arrays and of the operator it was captured with.  Every call that
// frees or replaces one of them, or switches the operator, drops the graph,
// so that the next graph solve captures a fresh one.
void drop_graph(tsgls_ctx* c) {
  if (c->gexec) {
    if (c->gst) (void)hipStreamSynchronize(c->gst);
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  c->gkey = tsgls_ctx::GraphKey{};
}

int ensure_krylov(tsgls_ctx* c, int m) {
  if (c->m_alloc >= m) return TSGLS_OK;
  drop_graph(c);
  dfree(c, c->V);
  c->V = nullptr;
  const int64_t n = ndof(c);
  CHK(dalloc(c, &c->V, (size_t)(m + 1) * n));
  if (!c->kx) {
    CHK(dalloc(c, &c->kx, n));
    CHK(dalloc(c, &c->kt, n));
    CHK(dalloc(c, &c->kt2, n));
    CHK(dalloc(c, &c->ybak, n));
    CHK(dalloc(c, &c->minv, n));
    CHK(dalloc(c, &c->partial, (size_t)multidot_blocks(n) * 1024));
    CHK(dalloc(c, &c->dh, 4096));
    if (!c->hp) {
      HIPCHK(c, hipHostMalloc((void**)&c->hp, 4096 * sizeof(double), hipHostMallocDefault));
      HIPCHK(c, hipHostGetDevicePointer((void**)&c->hpd, c->hp, 0));
    }
  }
  c->m_alloc = m;
  return TSGLS_OK;
}

// Right-Jacobi-preconditioned restarted GMRES with delayed classical
// Gram-Schmidt (restart <= GS_DELAYED_MAX): the second Gram-Schmidt pass of basis vector
// j is merged into step j+1's single reduction, so each Arnoldi step makes
// one reduction and one update pass over the basis and synchronizes once.
//   step j: w = A u_j (u_j once-orthogonalized, provisional), reduction of
//   [Q^T u; Q^T w; u.u; u.w; w.w] over the final Q = [q_0 .. q_{j-1}];
//   nu = |u - Q a|, q_j = (u - Q a)/nu; column j-1 of H is corrected for
//   u_j = Q a + nu q_j and then passes through the Givens rotations;
//   provisional column j: A q_j = (w - A Q a)/nu with A Q = Q H;
//   update pass: q_j into slot j, u_{j+1} = (w - Q b - q_j h_jj)/sigma.
// The last column is finalized with one extra reduction (no product).
int gmres_delayed(tsgls_ctx* c, const double* b, double* x, double tol, int m, int maxmv, int jac,
                  double dt, int prec, int* mv_out, bool* conv) {
  const int64_t n = ndof(c);
  const int nb = multidot_blocks(n);
  *conv = false;
  HIPCHK(c, launch_zero(x, n, c->st));
  double bnorm;
  CHK(norm2(c, b, &bnorm));
  if (!std::isfinite(bnorm)) return fail(c, TSGLS_ENONFINITE, "non-finite right-hand side");
  int mv = 0;
  if (bnorm == 0.0) {
    *conv = true;
    *mv_out = 0;
    return TSGLS_OK;
  }
  const int ld = m + 1;
  // Hh: Hessenberg of the Arnoldi relation A Q = Q H (unrotated);
  // R: its finalized columns after the Givens rotations (least squares)
  std::vector<double> Hh((size_t)ld * m), R((size_t)ld * m), cs(m), sn(m), g(m + 1), yv(m),
      red(2 * m + 3), ab(2 * m), col(m + 2);
  auto H = [&](int i, int j) -> double& { return Hh[(size_t)j * ld + i]; };
  auto Rr = [&](int i, int j) -> double& { return R[(size_t)j * ld + i]; };
  auto commit = [&](int j) {   // column j of H is final: rotate it into R, new rotation j
    for (int i = 0; i <= j + 1; ++i) Rr(i, j) = H(i, j);
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * Rr(i, j) + sn[i] * Rr(i + 1, j);
      Rr(i + 1, j) = -sn[i] * Rr(i, j) + cs[i] * Rr(i + 1, j);
      Rr(i, j) = t;
    }
    const double den = std::hypot(Rr(j, j), Rr(j + 1, j));
    cs[j] = den > 0 ? Rr(j, j) / den : 1.0;
    sn[j] = den > 0 ? Rr(j + 1, j) / den : 0.0;
    Rr(j, j) = den;
    Rr(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
  };
  auto reduce = [&](int J, const double* u, const double* w) -> int {
    ProfScope ps(c, TSGLS_PROF_ORTHO);
    HIPCHK(c, launch_gs_reduce(c->V, n, J, u, w, c->partial, nb, n, c->st));
    // the second stage writes the sums straight into pinned host memory (no
    // copy launch); they are read after the stream synchronization
    HIPCHK(c, launch_reduce_partials(c->partial, nb, 2 * J + 3, c->hpd, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::copy(c->hp, c->hp + 2 * J + 3, red.begin());
    return TSGLS_OK;
  };
  bool first = true;
  while (mv < maxmv) {
    double* V0 = c->V;
    if (first) {
      HIPCHK(c, launch_copy(b, V0, n, c->st));
    } else {
      CHK(jv_impl(c, x, c->kt, jac, dt, nullptr, prec));
      ++mv;
      HIPCHK(c, launch_copy(b, V0, n, c->st));
      HIPCHK(c, launch_axpy(-1.0, c->kt, V0, n, c->st));
    }
    first = false;
    double beta;
    CHK(norm2(c, V0, &beta));
    if (!std::isfinite(beta)) return fail(c, TSGLS_ENONFINITE, "non-finite GMRES residual");
    if (beta <= tol * bnorm) {
      *conv = true;
      break;
    }
    HIPCHK(c, launch_scal_copy(1.0 / beta, V0, V0, n, c->st));
    std::fill(Hh.begin(), Hh.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool done = false;
    for (int j = 0; j < m && mv < maxmv; ++j) {
      double* u = c->V + (int64_t)j * n;
      double* w = c->V + (int64_t)(j + 1) * n;
      CHK(jv_impl(c, u, w, jac, dt, c->minv, prec));
      ++mv;
      CHK(reduce(j, u, w));
      const double* a = red.data();
      const double* bq = red.data() + j;
      const double uu = red[2 * j], uw = red[2 * j + 1], ww = red[2 * j + 2];
      if (!std::isfinite(uu) || !std::isfinite(ww)) return fail(c, TSGLS_ENONFINITE, "non-finite Krylov vector");
      double aa = 0.0, abq = 0.0, bbq = 0.0;
      for (int i = 0; i < j; ++i) {
        aa += a[i] * a[i];
        abq += a[i] * bq[i];
        bbq += bq[i] * bq[i];
      }
      const double nu = std::sqrt(std::max(uu - aa, 0.0));
      if (!(nu > 0.0)) {   // u_j = Q a lies in span(Q): column j-1 ends the Krylov space
        if (j >= 1) {
          const double sj = H(j, j - 1);
          for (int i = 0; i < j; ++i) H(i, j - 1) += sj * a[i];
          H(j, j - 1) = 0.0;
          commit(j - 1);
        }
        k = j;
        done = true;
        break;
      }
      if (j >= 1) {        // column j-1 for u_j = Q a + nu q_j; now final
        const double sj = H(j, j - 1);
        for (int i = 0; i < j; ++i) H(i, j - 1) += sj * a[i];
        H(j, j - 1) = sj * nu;
        commit(j - 1);
        k = j;
      }
      // provisional column j: A q_j = (w - A Q a) / nu, A Q a = Q (H a)
      const double hj = (uw - abq) / nu;
      for (int i = 0; i <= j; ++i) {
        double ha = 0.0;
        for (int l = (i > 0 ? i - 1 : 0); l < j; ++l) ha += H(i, l) * a[l];
        H(i, j) = ((i < j ? bq[i] : hj) - ha) / nu;
      }
      const double s2 = ww - bbq - hj * hj;
      const double sigma = std::sqrt(std::max(s2, 1e-30 * ww));
      H(j + 1, j) = sigma / nu;
      for (int i = 0; i < j; ++i) {
        ab[i] = a[i];
        ab[j + i] = bq[i];
      }
      {
        ProfScope ps(c, TSGLS_PROF_ORTHO);
        // the coefficients travel as kernel arguments (no copy before the update)
        HIPCHK(c, launch_gs_update(c->V, n, j, nullptr, ab.data(), 1.0 / nu, hj, 1.0 / sigma, nullptr,
                                   u, w, n, c->st));
      }
      // provisional least-squares residual with column j as it stands
      bool last = (j + 1 == m) || (mv >= maxmv);
      if (!last) {
        for (int i = 0; i <= j + 1; ++i) col[i] = H(i, j);
        for (int i = 0; i < j; ++i) {
          const double t = cs[i] * col[i] + sn[i] * col[i + 1];
          col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        const double res = den > 0 ? std::fabs(col[j + 1] / den * g[j]) : std::fabs(g[j]);
        if (res <= tol * bnorm) last = true;
      }
      if (last) {          // finalize column j against the once-orthogonalized u_{j+1}
        CHK(reduce(j + 1, w, w));
        double a2 = 0.0;
        for (int i = 0; i <= j; ++i) a2 += red[i] * red[i];
        const double nu2 = std::sqrt(std::max(red[2 * (j + 1)] - a2, 0.0));
        const double sj = H(j + 1, j);
        for (int i = 0; i <= j; ++i) H(i, j) += sj * red[i];
        H(j + 1, j) = sj * nu2;
        commit(j);
        k = j + 1;
        done = std::fabs(g[k]) <= tol * bnorm;
        break;
      }
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= Rr(i, l) * yv[l];
      yv[i] = s / Rr(i, i);
    }
    std::copy(yv.begin(), yv.begin() + k, c->hp + 2560);
    HIPCHK(c, hipMemcpyAsync(c->dh + 1024, c->hp + 2560, k * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, launch_zero(c->kt, n, c->st));
    HIPCHK(c, launch_multiaxpy_add(c->V, n, k, c->dh + 1024, c->kt, n, c->st));
    HIPCHK(c, launch_mul(c->minv, c->kt, c->kt2, n, c->st));
    HIPCHK(c, launch_axpy(1.0, c->kt2, x, n, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (done) {
      *conv = true;
      break;
    }
  }
  *mv_out = mv;
  return TSGLS_OK;
}

// Device-side least-squares state per segment (doubles), status words per
// segment, reduction slots per segment.
constexpr int64_t GM_SEGD = 2400;
constexpr int GM_ST = 8;
constexpr int64_t GM_RED = 128;
constexpr int64_t GM_BB = 96;    // |r|^2 of the cycle's start within a segment's reduction slots

int ensure_gm(tsgls_ctx* c) {
  if (c->gmbuf) return TSGLS_OK;
  const int S = c->nseg;
  const int64_t L = ndof(c) / S;
  const int nb = multidot_blocks(L);
  CHK(dalloc(c, &c->gmbuf, (size_t)S * GM_SEGD + ((size_t)S * (GM_ST + 2) + 2) / 2 + 16));
  CHK(dalloc(c, &c->segred, (size_t)S * GM_RED));
  CHK(dalloc(c, &c->segpart, (size_t)S * nb * 67));
  CHK(dalloc(c, &c->segnrm, (size_t)S));
  HIPCHK(c, hipHostMalloc((void**)&c->hseg, ((size_t)S * (GM_ST + 2) + 1) * sizeof(int), hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc((void**)&c->hsegd, (size_t)2 * S * sizeof(double), hipHostMallocDefault));
  const int ld = 33;
  double* p = c->gmbuf;
  c->gm.H = p;
  c->gm.R = p + ld * 32;
  c->gm.cs = p + 2 * ld * 32;
  c->gm.sn = c->gm.cs + 32;
  c->gm.g = c->gm.sn + 32;
  c->gm.y = c->gm.g + 33;
  c->gm.ab = c->gm.y + 32;
  c->gm.sc = c->gm.ab + 64;
  c->gm.st = reinterpret_cast<int*>(c->gmbuf + (size_t)S * GM_SEGD);
  c->gm.sd = GM_SEGD;
  c->gm.si = GM_ST;
  c->gm.skip = c->gm.st + (size_t)S * GM_ST;
  std::fill(c->hseg, c->hseg + (size_t)S * (GM_ST + 2) + 1, 0);
  HIPCHK(c, hipMemcpyAsync(c->gm.st, c->hseg, ((size_t)S * (GM_ST + 2) + 1) * sizeof(int), hipMemcpyHostToDevice,
                           c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return TSGLS_OK;
}

// Copy the skip flags staged at hseg + nseg * GM_ST to the device, with the
// list of the segments taking part and its length (one copy).  The caller
// has synchronized since the staging area was last copied.
int write_mask(tsgls_ctx* c) {
  const int S = c->nseg;
  int* skip = c->hseg + (size_t)S * GM_ST;
  int* list = skip + S;
  int n = 0;
  for (int s = 0; s < S; ++s)
    if (!skip[s]) list[n++] = s;
  for (int s = n; s < S; ++s) list[s] = 0;
  list[S] = n;
  HIPCHK(c, hipMemcpyAsync(const_cast<int*>(c->gm.skip), skip, (2 * (size_t)S + 1) * sizeof(int),
                           hipMemcpyHostToDevice, c->st));
  return TSGLS_OK;
}

void free_gm(tsgls_ctx* c) {
  drop_graph(c);
  for (double** q : {&c->gmbuf, &c->segred, &c->segpart, &c->segnrm}) {
    dfree(c, *q);
    *q = nullptr;
  }
  if (c->hseg) (void)hipHostFree(c->hseg);
  if (c->hsegd) (void)hipHostFree(c->hsegd);
  c->hseg = nullptr;
  c->hsegd = nullptr;
  c->gm = GmDev{};
}

// Euclidean norm of each segment of x into out[nseg] (one synchronization);
// with one segment the same kernels and blocking as norm2.
int seg_norms(tsgls_ctx* c, const double* x, double* out) {
  CHK(ensure_gm(c));
  const int S = c->nseg;
  const int64_t L = ndof(c) / S;
  const int nb = multidot_blocks(L);
  const int64_t ps = (int64_t)nb * 67;
  const int* sk = S > 1 ? c->gm.skip : nullptr;
  HIPCHK(c, launch_multidot(x, 0, 1, x, c->segpart, nb, L, c->st, S, L, ps, sk));
  HIPCHK(c, launch_reduce_partials(c->segpart, nb, 1, c->segnrm, c->st, S, ps, 1, sk));
  HIPCHK(c, hipMemcpyAsync(c->hsegd, c->segnrm, S * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int s = 0; s < S; ++s) out[s] = std::sqrt(c->hsegd[s]);
  return TSGLS_OK;
}

// The same delayed Gram-Schmidt GMRES (m <= 32) with the least-squares
// update on the device (k_gm_*), so that one cycle -- the residual norm, m
// Arnoldi steps (tangent product, reduction, update), the final reduction,
// the triangular solve and the update of x -- is one HIP graph, captured
// once per (m, tangent, shift, precision) and replayed for every cycle of
// every Newton step.  The host synchronizes once per cycle to read the
// convergence flags.  Cycles always run m steps: after convergence the
// remaining steps see zero update coefficients and leave zero vectors.
// With segments every launch of the cycle covers all of them (one GMRES per
// segment, each segment's reductions over its own entries with the blocking
// of a lone problem of that size, so each segment follows the iteration its
// problem would follow alone); a segment that has converged, run out of
// products, or is frozen (frozen[s] != 0) sits out the remaining cycles with
// zero updates.  mv_out, conv: per segment.
int gmres_graph(tsgls_ctx* c, const double* b, double* x, double tol, int m, int maxmv, int jac,
                double dt, int prec, int* mv_out, bool* conv, const char* frozen = nullptr) {
  const int S = c->nseg;
  const int64_t n = ndof(c), L = n / S;
  const int nb = multidot_blocks(L);
  const int64_t ps = (int64_t)nb * 67;
  if (m > 32) return fail(c, TSGLS_EINVAL, "graph GMRES needs restart <= 32");
  CHK(ensure_gm(c));
  if (!c->gst) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->gev[0], hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->gev[1], hipEventDisableTiming));
  }
  c->gm.m = m;
  if (prec != TSGLS_PREC_F64) CHK(ensure_lin32(c));
  if (prec == TSGLS_PREC_BF16) CHK(ensure_tau16(c));
  const tsgls_ctx::GraphKey key{m, jac, prec, dt, b, x};
  const bool same = c->gexec && c->gkey.m == key.m && c->gkey.jac == key.jac &&
                    c->gkey.prec == key.prec && c->gkey.dt == key.dt && c->gkey.b == key.b &&
                    c->gkey.x == key.x;
  if (!same) {
    if (c->gexec) {
      HIPCHK(c, hipGraphExecDestroy(c->gexec));
      c->gexec = nullptr;
    }
    // one eager product first: first-call set-up of the kernels is done outside the capture
    CHK(jv_impl(c, b, c->kt, jac, dt, c->minv, prec));
    HIPCHK(c, hipStreamSynchronize(c->st));
    const GmDev d = c->gm;
    double* red = c->segred;
    double* bb = c->segred + GM_BB;
    // segments that sit out the cycle are skipped by the vector kernels too
    // (their least-squares state is silenced by k_gm_begin)
    const int* sk = S > 1 ? d.skip : nullptr;
    auto body = [&]() -> int {
      double* V0 = c->V;
      HIPCHK(c, launch_multidot(V0, 0, 1, V0, c->segpart, nb, L, c->st, S, L, ps, sk));
      HIPCHK(c, launch_reduce_partials(c->segpart, nb, 1, bb, c->st, S, ps, GM_RED, sk));
      HIPCHK(c, launch_gm_begin(d, bb, tol, 0, c->st, S, GM_RED));
      HIPCHK(c, launch_scal_dev(V0, d.sc + 5, L, c->st, S, L, GM_SEGD, sk));
      for (int j = 0; j < m; ++j) {
        double* u = c->V + (int64_t)j * n;
        double* w = c->V + (int64_t)(j + 1) * n;
        CHK(jv_impl(c, u, w, jac, dt, c->minv, prec));
        HIPCHK(c, launch_gs_reduce(c->V, n, j, u, w, c->segpart, nb, L, c->st, S, L, ps, sk));
        HIPCHK(c, launch_reduce_partials(c->segpart, nb, 2 * j + 3, red, c->st, S, ps, GM_RED, sk));
        HIPCHK(c, launch_gm_step(d, j, red, c->st, S, GM_RED));
        HIPCHK(c, launch_gs_update(c->V, n, j, d.ab, nullptr, 0.0, 0.0, 0.0, d.sc, u, w, L, c->st, S, L,
                                   GM_SEGD, sk));
      }
      double* um = c->V + (int64_t)m * n;
      HIPCHK(c, launch_gs_reduce(c->V, n, m, um, um, c->segpart, nb, L, c->st, S, L, ps, sk));
      HIPCHK(c, launch_reduce_partials(c->segpart, nb, 2 * m + 3, red, c->st, S, ps, GM_RED, sk));
      HIPCHK(c, launch_gm_final(d, red, c->st, S, GM_RED));
      HIPCHK(c, launch_zero(c->kt, n, c->st));
      HIPCHK(c, launch_multiaxpy_add(c->V, n, m, d.y, c->kt, L, c->st, S, L, GM_SEGD, sk));
      HIPCHK(c, launch_mul(c->minv, c->kt, c->kt2, n, c->st));
      HIPCHK(c, launch_axpy(1.0, c->kt2, x, n, c->st));
      return TSGLS_OK;
    };
    hipStream_t orig = c->st;
    const bool prof = c->prof;
    c->prof = false;
    c->st = c->gst;
    HIPCHK(c, hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal));
    const int rc = body();
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->gst, &graph);
    c->st = orig;
    c->prof = prof;
    if (rc != TSGLS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HIPCHK(c, ec);
    const hipError_t ei = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(c, ei);
    c->gkey = key;
  }
  HIPCHK(c, launch_zero(x, n, c->st));
  std::vector<double> bn(S);
  CHK(seg_norms(c, b, bn.data()));
  std::vector<char> act(S, 0);
  int* skip = c->hseg + (size_t)S * GM_ST;
  int nact = 0;
  for (int s = 0; s < S; ++s) {
    mv_out[s] = 0;
    conv[s] = false;
    const bool fz = frozen && frozen[s];
    if (!fz && !std::isfinite(bn[s])) return fail(c, TSGLS_ENONFINITE, "non-finite right-hand side");
    if (!fz && bn[s] == 0.0) conv[s] = true;
    act[s] = !fz && bn[s] != 0.0;
    skip[s] = !act[s];
    nact += act[s];
    c->hsegd[S + s] = tol * bn[s];
  }
  if (nact == 0) return TSGLS_OK;
  for (int s = 0; s < S; ++s)
    HIPCHK(c, hipMemcpyAsync(c->gm.sc + (size_t)s * GM_SEGD + 4, c->hsegd + S + s, sizeof(double),
                             hipMemcpyHostToDevice, c->st));
  CHK(write_mask(c));
  bool first = true;
  while (nact > 0) {
    double* V0 = c->V;
    if (first) {
      HIPCHK(c, launch_copy(b, V0, n, c->st));
    } else {
      CHK(jv_impl(c, x, c->kt, jac, dt, nullptr, prec));
      for (int s = 0; s < S; ++s) mv_out[s] += act[s];
      HIPCHK(c, launch_copy(b, V0, n, c->st));
      HIPCHK(c, launch_axpy(-1.0, c->kt, V0, n, c->st));
    }
    first = false;
    HIPCHK(c, hipEventRecord(c->gev[0], c->st));
    HIPCHK(c, hipStreamWaitEvent(c->gst, c->gev[0], 0));
    HIPCHK(c, hipGraphLaunch(c->gexec, c->gst));
    HIPCHK(c, hipEventRecord(c->gev[1], c->gst));
    HIPCHK(c, hipStreamWaitEvent(c->st, c->gev[1], 0));
    HIPCHK(c, hipMemcpyAsync(c->hseg, c->gm.st, (size_t)S * GM_ST * sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    bool changed = false;
    for (int s = 0; s < S; ++s) {
      if (!act[s]) continue;
      mv_out[s] += m;
      const int* stv = c->hseg + (size_t)s * GM_ST;
      if (stv[4]) return fail(c, TSGLS_ENONFINITE, "non-finite Krylov quantity");
      if (stv[3]) conv[s] = true;
      if (stv[3] || mv_out[s] + m > maxmv) {
        act[s] = 0;
        skip[s] = 1;
        --nact;
        changed = true;
      }
    }
    if (changed && nact > 0) CHK(write_mask(c));
  }
  return TSGLS_OK;
}

// Right-Jacobi-preconditioned restarted GMRES with classical Gram-Schmidt and
// one reorthogonalization pass; x = J^{-1} b approximately, x zeroed first.
int gmres(tsgls_ctx* c, const double* b, double* x, double tol, int m, int maxmv, int jac,
          double dt, int prec, int* mv_out, bool* conv) {
  const int64_t n = ndof(c);
  *conv = false;
  HIPCHK(c, launch_zero(x, n, c->st));
  double bnorm;
  CHK(norm2(c, b, &bnorm));
  if (!std::isfinite(bnorm)) return fail(c, TSGLS_ENONFINITE, "non-finite right-hand side");
  int mv = 0;
  if (bnorm == 0.0) {
    *conv = true;
    *mv_out = 0;
    return TSGLS_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 1), h2(2 * m + 3), yv(m);
  bool first = true;
  while (mv < maxmv) {
    double* V0 = c->V;
    if (first) {
      HIPCHK(c, launch_copy(b, V0, n, c->st));
    } else {
      CHK(jv_impl(c, x, c->kt, jac, dt, nullptr, prec));
      ++mv;
      HIPCHK(c, launch_copy(b, V0, n, c->st));
      HIPCHK(c, launch_axpy(-1.0, c->kt, V0, n, c->st));
    }
    first = false;
    double beta;
    CHK(norm2(c, V0, &beta));
    if (!std::isfinite(beta)) return fail(c, TSGLS_ENONFINITE, "non-finite GMRES residual");
    if (beta <= tol * bnorm) {
      *conv = true;
      break;
    }
    HIPCHK(c, launch_scal_copy(1.0 / beta, V0, V0, n, c->st));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool done = false;
    for (int j = 0; j < m && mv < maxmv; ++j) {
      double* Vj = c->V + (int64_t)j * n;
      double* Vn = c->V + (int64_t)(j + 1) * n;
      CHK(jv_impl(c, Vj, Vn, jac, dt, c->minv, prec));   // J (M^-1 V_j), the scale applied on load
      ++mv;
      double hn;
      if (j + 1 <= 32) {
        // CGS2 with the first pass's update fused with the second pass's dots
        // and the second update fused with the norm: three reads of the basis
        // and one host synchronisation per step.
        ProfScope ps(c, TSGLS_PROF_ORTHO);
        const int J = j + 1, nb = multidot_blocks(n);
        double* dh1 = c->dh;            // h  [J]
        double* dh2 = c->dh + J;        // h2 [J]
        double* dnn = c->dh + 2 * J;    // |Vn|^2
        HIPCHK(c, launch_axpy_dot(c->V, n, J, nullptr, 0.0, Vn, J, 0, c->partial, nb, n, c->st));
        HIPCHK(c, launch_reduce_partials(c->partial, nb, J, dh1, c->st));
        HIPCHK(c, launch_axpy_dot(c->V, n, J, dh1, -1.0, Vn, J, 0, c->partial, nb, n, c->st));
        HIPCHK(c, launch_reduce_partials(c->partial, nb, J, dh2, c->st));
        HIPCHK(c, launch_axpy_dot(c->V, n, J, dh2, -1.0, Vn, 0, 1, c->partial, nb, n, c->st));
        HIPCHK(c, launch_reduce_partials(c->partial, nb, 1, dnn, c->st));
        HIPCHK(c, hipMemcpyAsync(c->hp, c->dh, (2 * J + 1) * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        std::copy(c->hp, c->hp + 2 * J + 1, h2.begin());
        for (int i = 0; i < J; ++i) h[i] = h2[i] + h2[J + i];
        hn = std::sqrt(std::max(h2[2 * J], 0.0));
      } else {
        // CGS2: two dot/update passes and the norm, one host synchronisation
        ProfScope ps(c, TSGLS_PROF_ORTHO);
        const int J = j + 1, nb = multidot_blocks(n);
        double* dh1 = c->dh;            // h  [J]
        double* dh2 = c->dh + J;        // h2 [J]
        double* dnn = c->dh + 2 * J;    // |Vn|^2
        HIPCHK(c, launch_multidot(c->V, n, J, Vn, c->partial, nb, n, c->st));
        HIPCHK(c, launch_reduce_partials(c->partial, nb, J, dh1, c->st));
        HIPCHK(c, launch_multiaxpy(c->V, n, J, dh1, Vn, n, c->st));
        HIPCHK(c, launch_multidot(c->V, n, J, Vn, c->partial, nb, n, c->st));
        HIPCHK(c, launch_reduce_partials(c->partial, nb, J, dh2, c->st));
        HIPCHK(c, launch_multiaxpy(c->V, n, J, dh2, Vn, n, c->st));
        HIPCHK(c, launch_multidot(Vn, 0, 1, Vn, c->partial, nb, n, c->st));
        HIPCHK(c, launch_reduce_partials(c->partial, nb, 1, dnn, c->st));
        HIPCHK(c, hipMemcpyAsync(c->hp, c->dh, (2 * J + 1) * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        std::copy(c->hp, c->hp + 2 * J + 1, h2.begin());
        for (int i = 0; i < J; ++i) h[i] = h2[i] + h2[J + i];
        hn = std::sqrt(std::max(h2[2 * J], 0.0));
      }
      if (!std::isfinite(hn)) return fail(c, TSGLS_ENONFINITE, "non-finite Krylov vector");
      if (hn > 0) HIPCHK(c, launch_scal_copy(1.0 / hn, Vn, Vn, n, c->st));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double den = std::hypot(h[j], hn);
      cs[j] = den > 0 ? h[j] / den : 1.0;
      sn[j] = den > 0 ? hn / den : 0.0;
      h[j] = den;
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      if (std::fabs(g[j + 1]) <= tol * bnorm || hn == 0.0) {
        done = true;
        break;
      }
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * yv[l];
      yv[i] = s / H[(size_t)i * m + i];
    }
    std::copy(yv.begin(), yv.begin() + k, c->hp + 2560);
    HIPCHK(c, hipMemcpyAsync(c->dh + 1024, c->hp + 2560, k * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, launch_zero(c->kt, n, c->st));
    HIPCHK(c, launch_multiaxpy_add(c->V, n, k, c->dh + 1024, c->kt, n, c->st));
    HIPCHK(c, launch_mul(c->minv, c->kt, c->kt2, n, c->st));
    HIPCHK(c, launch_axpy(1.0, c->kt2, x, n, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (done) {
      *conv = true;
      break;
    }
  }
  *mv_out = mv;
  return TSGLS_OK;
}

// Processing order: Morton order of the element centroids (locality of the
// node gathers; contributions are summed per node afterwards in a fixed
// order).  Returns processing position -> input element.
std::vector<uint64_t> morton_keys(const double* xyz, int64_t n_nodes, const int32_t* tets, int64_t n_tets) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = 0; i < n_nodes; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[i * 3 + d]);
      hi[d] = std::max(hi[d], xyz[i * 3 + d]);
    }
  std::vector<uint64_t> key(n_tets);
  for (int64_t e = 0; e < n_tets; ++e) {
    double cc[3] = {0, 0, 0};
    for (int b = 0; b < 4; ++b)
      for (int d = 0; d < 3; ++d) cc[d] += 0.25 * xyz[(int64_t)tets[e * 4 + b] * 3 + d];
    for (int d = 0; d < 3; ++d) cc[d] = (cc[d] - lo[d]) / std::max(hi[d] - lo[d], 1e-300);
    key[e] = morton3(cc[0], cc[1], cc[2]);
  }
  return key;
}

std::vector<int32_t> morton_perm(const double* xyz, int64_t n_nodes, const int32_t* tets, int64_t n_tets) {
  const std::vector<uint64_t> key = morton_keys(xyz, n_nodes, tets, n_tets);
  std::vector<int32_t> perm(n_tets);
  for (int64_t e = 0; e < n_tets; ++e) perm[e] = (int32_t)e;
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  return perm;
}

// Install a processing order (position -> input element) for the input-order
// tets: connectivity in that order, node -> incident (element, local node)
// in ascending position, and the element geometry; the linearization is
// invalidated.
int set_order(tsgls_ctx* c, const int32_t* tets, const std::vector<int32_t>& perm) {
  const int64_t n_tets = c->E, n_nodes = c->nn;
  std::vector<int32_t> sconn(n_tets * 4);
  for (int64_t e = 0; e < n_tets; ++e)
    for (int b = 0; b < 4; ++b) sconn[e * 4 + b] = tets[(int64_t)perm[e] * 4 + b];
  std::vector<int32_t> noff(n_nodes + 1, 0), ninc(n_tets * 4);
  for (int64_t k = 0; k < n_tets * 4; ++k) noff[sconn[k] + 1]++;
  for (int64_t i = 0; i < n_nodes; ++i) noff[i + 1] += noff[i];
  {
    std::vector<int32_t> fill(noff.begin(), noff.end() - 1);
    for (int64_t k = 0; k < n_tets * 4; ++k) ninc[fill[sconn[k]]++] = (int32_t)k;
  }
  double* dxyz = nullptr;
  CHK(dalloc(c, &dxyz, n_nodes * 3));
  HIPCHK(c, hipMemcpyAsync(dxyz, c->hxyz.data(), n_nodes * 3 * sizeof(double), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->conn, sconn.data(), n_tets * 4 * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->noff, noff.data(), noff.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->ninc, ninc.data(), ninc.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, launch_geometry(dxyz, c->conn, c->geo, nullptr, n_tets, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  dfree(c, dxyz);
  c->dev_bytes -= n_nodes * 3 * sizeof(double);
  if (&perm != &c->perm) c->perm = perm;
  c->linearized = false;
  c->lin32 = false;
  c->lin16 = false;
  c->tauV_ok = false;
  return TSGLS_OK;
}

// Every element (and Neumann face) must have its nodes in one segment, so
// that the segments are independent problems.
int check_segments(tsgls_ctx* c) {
  if (c->seg_checked || c->nseg == 1) return TSGLS_OK;
  const int64_t Ln = c->nn / c->nseg;
  std::vector<int32_t> h((size_t)c->E * 4);
  HIPCHK(c, hipMemcpy(h.data(), c->conn, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int64_t e = 0; e < c->E; ++e) {
    const int64_t s0 = h[e * 4] / Ln;
    for (int b = 1; b < 4; ++b)
      if (h[e * 4 + b] / Ln != s0)
        return fail(c, TSGLS_EINVAL, "element %lld has nodes in two segments", (long long)c->perm[e]);
  }
  if (c->nf) {
    std::vector<int32_t> f((size_t)c->nf * 3);
    HIPCHK(c, hipMemcpy(f.data(), c->fconn, f.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < c->nf; ++i)
      if (f[i * 3 + 1] / Ln != f[i * 3] / Ln || f[i * 3 + 2] / Ln != f[i * 3] / Ln)
        return fail(c, TSGLS_EINVAL, "Neumann face %lld has nodes in two segments", (long long)i);
  }
  c->seg_checked = true;
  return TSGLS_OK;
}

}  // namespace

extern "C" {

int tsgls_supported_K(int* out, int cap) { return supported_K_list(out, cap); }

int tsgls_create(const double* xyz, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                 const tsgls_params* params, void* hip_stream, tsgls_ctx** out) {
  if (!out) return TSGLS_EINVAL;
  *out = nullptr;
  if (!xyz || !tets || !params || n_nodes <= 0 || n_tets <= 0) return TSGLS_EINVAL;
  tsgls_ctx* c = new (std::nothrow) tsgls_ctx();
  if (!c) return TSGLS_ENOMEM;
  *out = c;
  c->p = *params;
  c->st = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->dev) != hipSuccess) return fail(c, TSGLS_EHIP, "hipGetDevice failed");
  const int K = params->K;
  if (!(params->rho > 0) || !(params->mu > 0) || !(params->C_I >= 0) || !(params->backflow_beta >= 0) ||
      !(params->backflow_beta <= 1) || !std::isfinite(params->omega))
    return fail(c, TSGLS_EINVAL, "invalid physical parameters");
  if (K < 0 || !supported_K(K)) return fail(c, TSGLS_EINVAL, "K=%d is not compiled into this library", K);
  c->K = K;
  c->n = 2 * K + 1;
  c->S = 2 * K + 2;
  c->M = 3 * K + 1;
  c->P = c->n * (c->n + 1) / 2;
  c->nn = n_nodes;
  c->E = n_tets;
  c->hxyz.assign(xyz, xyz + n_nodes * 3);
  // mesh checks
  for (int64_t e = 0; e < n_tets; ++e) {
    const int32_t* t = tets + e * 4;
    for (int b = 0; b < 4; ++b)
      if (t[b] < 0 || t[b] >= n_nodes) return fail(c, TSGLS_EMESH, "tet %lld has node index %d out of range", (long long)e, t[b]);
    double d[3][3];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) d[k][i] = xyz[(int64_t)t[k + 1] * 3 + i] - xyz[(int64_t)t[0] * 3 + i];
    const double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                       d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                       d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    if (!(det > 0)) return fail(c, TSGLS_EMESH, "tet %lld has non-positive volume", (long long)e);
  }
  c->perm = morton_perm(xyz, n_nodes, tets, n_tets);
  // device data
  CHK(dalloc(c, &c->conn, n_tets * 4));
  CHK(dalloc(c, &c->geo, n_tets * 16));
  CHK(dalloc(c, &c->nflag, n_nodes));
  CHK(dalloc(c, &c->F, (size_t)c->n * c->M));
  CHK(dalloc(c, &c->UT, n_nodes * 3 * c->M));
  CHK(dalloc(c, &c->VT, n_nodes * 3 * c->M));
  CHK(dalloc(c, &c->XP, n_nodes * 4 * pos_width(K)));
  CHK(dalloc(c, &c->tau, (size_t)n_tets * 4 * c->P));
  CHK(dalloc(c, &c->Z, (size_t)n_tets * 12 * c->n));
  CHK(dalloc(c, &c->noff, n_nodes + 1));
  CHK(dalloc(c, &c->ninc, n_tets * 4));
  CHK(dalloc(c, &c->ebuf, (size_t)n_tets * 16 * c->n));
  CHK(dalloc(c, &c->rs, n_nodes * 4 * c->S));
  HIPCHK(c, hipMemsetAsync(c->nflag, 0, n_nodes, c->st));
  std::vector<double> F((size_t)c->n * c->M);
  const double pi = 3.14159265358979323846;
  for (int s = 0; s < c->M; ++s) {
    F[s] = 1.0;
    for (int k = 1; k <= K; ++k) {
      const double th = 2.0 * pi * k * s / c->M;
      F[(size_t)(2 * k - 1) * c->M + s] = std::sqrt(2.0) * std::cos(th);
      F[(size_t)(2 * k) * c->M + s] = -std::sqrt(2.0) * std::sin(th);
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->F, F.data(), F.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
  CHK(set_order(c, tets, c->perm));
  return TSGLS_OK;
}

int tsgls_set_dirichlet(tsgls_ctx* c, const int32_t* nodes, int64_t n) {
  if (!c || (n > 0 && !nodes) || n < 0) return fail(c, TSGLS_EINVAL, "bad Dirichlet arguments");
  std::vector<uint8_t> fl(c->nn, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (nodes[i] < 0 || nodes[i] >= c->nn) return fail(c, TSGLS_EINVAL, "Dirichlet node %d out of range", nodes[i]);
    fl[nodes[i]] = 1;
  }
  HIPCHK(c, hipMemcpyAsync(c->nflag, fl.data(), c->nn, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->linearized = false;
  return TSGLS_OK;
}

int tsgls_set_neumann(tsgls_ctx* c, const int32_t* tris, int64_t nf, const double* h) {
  if (!c) return TSGLS_EINVAL;
  if (nf < 0 || (nf > 0 && !tris)) return fail(c, TSGLS_EINVAL, "bad Neumann arguments");
  if (c->tracer && h) return fail(c, TSGLS_EINVAL, "the tracer takes no Neumann traction");
  drop_graph(c);
  c->seg_checked = false;
  dfree(c, c->fconn);
  dfree(c, c->fgeo);
  dfree(c, c->fh);
  dfree(c, c->aneg);
  dfree(c, c->fy);
  dfree(c, c->anegr);
  dfree(c, c->fnode);
  dfree(c, c->foff);
  dfree(c, c->finc);
  dfree(c, c->nfidx);
  c->fconn = c->fnode = c->foff = c->finc = c->nfidx = nullptr;
  c->fgeo = c->fh = c->aneg = c->anegr = c->fy = nullptr;
  c->nf = 0;
  c->n_fnodes = 0;
  c->linearized = false;
  if (nf == 0) return TSGLS_OK;
  std::vector<double> fg(nf * 4);
  for (int64_t f = 0; f < nf; ++f) {
    const int32_t* t = tris + f * 3;
    for (int b = 0; b < 3; ++b)
      if (t[b] < 0 || t[b] >= c->nn) return fail(c, TSGLS_EMESH, "face %lld has node index out of range", (long long)f);
    const double* x0 = &c->hxyz[(size_t)t[0] * 3];
    const double* x1 = &c->hxyz[(size_t)t[1] * 3];
    const double* x2 = &c->hxyz[(size_t)t[2] * 3];
    double a[3], b[3], nv[3];
    for (int i = 0; i < 3; ++i) {
      a[i] = x1[i] - x0[i];
      b[i] = x2[i] - x0[i];
    }
    nv[0] = a[1] * b[2] - a[2] * b[1];
    nv[1] = a[2] * b[0] - a[0] * b[2];
    nv[2] = a[0] * b[1] - a[1] * b[0];
    const double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    if (!(nn > 0)) return fail(c, TSGLS_EMESH, "face %lld is degenerate", (long long)f);
    for (int i = 0; i < 3; ++i) fg[f * 4 + i] = nv[i] / nn;
    fg[f * 4 + 3] = 0.5 * nn;
  }
  // node -> incident (face, local vertex) lists, ascending face order
  std::vector<int32_t> fnode(tris, tris + nf * 3);
  std::sort(fnode.begin(), fnode.end());
  fnode.erase(std::unique(fnode.begin(), fnode.end()), fnode.end());
  std::vector<int32_t> foff(fnode.size() + 1, 0), finc(nf * 3);
  for (int64_t k = 0; k < nf * 3; ++k) {
    const int64_t u = std::lower_bound(fnode.begin(), fnode.end(), tris[k]) - fnode.begin();
    foff[u + 1]++;
  }
  for (size_t u = 0; u < fnode.size(); ++u) foff[u + 1] += foff[u];
  {
    std::vector<int32_t> fill(foff.begin(), foff.end() - 1);
    for (int64_t k = 0; k < nf * 3; ++k) {
      const int64_t u = std::lower_bound(fnode.begin(), fnode.end(), tris[k]) - fnode.begin();
      finc[fill[u]++] = (int32_t)k;
    }
  }
  std::vector<int32_t> sc(tris, tris + nf * 3);
  std::vector<double> sg = fg, sh;
  std::vector<int32_t> perm(nf);
  for (int64_t f = 0; f < nf; ++f) perm[f] = (int32_t)f;
  c->n_fnodes = (int64_t)fnode.size();
  CHK(dalloc(c, &c->fnode, fnode.size()));
  CHK(dalloc(c, &c->foff, foff.size()));
  CHK(dalloc(c, &c->finc, finc.size()));
  HIPCHK(c, hipMemcpyAsync(c->fnode, fnode.data(), fnode.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->foff, foff.data(), foff.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->finc, finc.data(), finc.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  {
    std::vector<int32_t> nfidx(c->nn, -1);
    for (size_t u = 0; u < fnode.size(); ++u) nfidx[fnode[u]] = (int32_t)u;
    CHK(dalloc(c, &c->nfidx, nfidx.size()));
    HIPCHK(c, hipMemcpyAsync(c->nfidx, nfidx.data(), nfidx.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));   // the host arrays are freed at scope end
  }
  CHK(dalloc(c, &c->fconn, nf * 3));
  CHK(dalloc(c, &c->fgeo, nf * 4));
  CHK(dalloc(c, &c->aneg, (size_t)nf * 3 * c->P));
  CHK(dalloc(c, &c->fy, (size_t)nf * 9 * c->n));
  HIPCHK(c, hipMemcpyAsync(c->fconn, sc.data(), sc.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->fgeo, sg.data(), sg.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
  if (h) {
    // slots -> orthonormal coordinates (x_0 = slot 0, x_a = sqrt2 slot a+1)
    sh.assign(nf * c->n, 0.0);
    for (int64_t f = 0; f < nf; ++f) {
      const double* hs = h + (int64_t)perm[f] * c->S;
      sh[f * c->n] = hs[0];
      for (int a = 1; a < c->n; ++a) sh[f * c->n + a] = std::sqrt(2.0) * hs[a + 1];
    }
    CHK(dalloc(c, &c->fh, sh.size()));
    HIPCHK(c, hipMemcpyAsync(c->fh, sh.data(), sh.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->nf = nf;
  return TSGLS_OK;
}

int tsgls_residual(tsgls_ctx* c, const double* y, double* r) {
  if (c && c->tracer) {
    if (!y || !r) return fail(c, TSGLS_EINVAL, "null vector");
    return linearize_tracer(c, y, r);
  }
  if (!c) return TSGLS_EINVAL;
  if (!y || !r) return fail(c, TSGLS_EINVAL, "null vector");
  if (!c->UTr) {
    CHK(dalloc(c, &c->UTr, c->nn * 3 * c->M));
    CHK(dalloc(c, &c->taur, (size_t)c->E * 4 * c->P));
  }
  if (c->nf && !c->anegr) CHK(dalloc(c, &c->anegr, (size_t)c->nf * 3 * c->P));
  DevView v = view(c);
  v.UT = c->UTr;
  v.tau = c->taur;
  v.aneg = c->anegr;
  HIPCHK(c, launch_prep_time(c->K, y, nullptr, c->nflag, 0, c->F, c->UTr, c->XP, c->nn, c->st));
  HIPCHK(c, launch_tau(v, y, c->taur, c->st, c->tauV_ok ? c->tauV : nullptr, nullptr));
  HIPCHK(c, launch_face_lin(v, c->UTr, c->anegr, c->st));
  return apply_operator(c, v, MODE_RESID, y, nullptr, nullptr, r, 0.0, c->anegr, 1);
}

int tsgls_set_tracer(tsgls_ctx* c, const double* y_velocity, double kappa, int stabilized) {
  if (!c) return TSGLS_EINVAL;
  if (!y_velocity || !(kappa > 0) || !std::isfinite(kappa) || (stabilized != 0 && stabilized != 1))
    return fail(c, TSGLS_EINVAL, "bad tracer arguments");
  if (c->fh) return fail(c, TSGLS_EINVAL, "the tracer context must have no Neumann traction");
  if (c->nseg > 1) return fail(c, TSGLS_EINVAL, "a context with segments takes no tracer");
  const int64_t n = ndof(c);
  drop_graph(c);
  if (!c->yvel) CHK(dalloc(c, &c->yvel, n));
  HIPCHK(c, launch_copy(y_velocity, c->yvel, n, c->st));
  c->tracer = true;
  c->kappa = kappa;
  c->stabilized = stabilized;
  c->linearized = false;
  return TSGLS_OK;
}

int tsgls_linearize(tsgls_ctx* c, const double* y, double* r) {
  if (!c) return TSGLS_EINVAL;
  if (!y) return fail(c, TSGLS_EINVAL, "null vector");
  return linearize_impl(c, y, r);
}

int tsgls_jv(tsgls_ctx* c, const double* v, double* Jv, int jacobian, double dt_pseudo) {
  if (!c) return TSGLS_EINVAL;
  if (!v || !Jv || v == Jv) return fail(c, TSGLS_EINVAL, "bad vectors");
  if (jacobian < 0 || jacobian > 2) return fail(c, TSGLS_EINVAL, "bad tangent variant %d", jacobian);
  return jv_impl(c, v, Jv, jacobian, dt_pseudo);
}

int tsgls_jv_prec(tsgls_ctx* c, const double* v, double* Jv, int jacobian, double dt_pseudo,
                  int precision) {
  if (!c) return TSGLS_EINVAL;
  if (!v || !Jv || v == Jv) return fail(c, TSGLS_EINVAL, "bad vectors");
  if (jacobian < 0 || jacobian > 2) return fail(c, TSGLS_EINVAL, "bad tangent variant %d", jacobian);
  if (precision != TSGLS_PREC_F64 && precision != TSGLS_PREC_F32 && precision != TSGLS_PREC_BF16)
    return fail(c, TSGLS_EINVAL, "bad precision %d", precision);
  return jv_impl(c, v, Jv, jacobian, dt_pseudo, nullptr, precision);
}

int tsgls_jacobi_diag(tsgls_ctx* c, double* d, double dt_pseudo) {
  if (!c) return TSGLS_EINVAL;
  if (!d) return fail(c, TSGLS_EINVAL, "null vector");
  return diag_impl(c, d, dt_pseudo);
}

int tsgls_get_tau(tsgls_ctx* c, double* tau_out) {
  if (!c) return TSGLS_EINVAL;
  if (!tau_out) return fail(c, TSGLS_EINVAL, "null pointer");
  if (!c->linearized) return fail(c, TSGLS_ESTATE, "get_tau before linearize");
  std::vector<double> buf((size_t)c->E * 4 * c->P);
  HIPCHK(c, hipMemcpyAsync(buf.data(), c->tau, buf.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  // device storage is packed over positions; the output is packed over modes
  std::vector<int> map(c->P);
  for (int r = 0, p = 0; r < c->n; ++r)
    for (int cc = r; cc < c->n; ++cc, ++p) {
      const int pr = mode_pos(r, c->K), pc = mode_pos(cc, c->K);
      map[p] = pr < pc ? pk_index(pr, pc, c->n) : pk_index(pc, pr, c->n);
    }
  for (int64_t e = 0; e < c->E; ++e)
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < c->P; ++p)
        tau_out[((size_t)c->perm[e] * 4 + q) * c->P + p] = buf[((size_t)e * 4 + q) * c->P + map[p]];
  return TSGLS_OK;
}

int tsgls_solve(tsgls_ctx* c, double* y, const tsgls_solve_opts* o, tsgls_solve_stats* stats) {
  if (!c) return TSGLS_EINVAL;
  if (!y || !o) return fail(c, TSGLS_EINVAL, "null argument");
  if (o->restart < 1 || o->restart > 1000 || o->max_newton < 0 || o->max_matvec < 1 || !(o->rtol > 0) ||
      !(o->lin_rtol > 0) || o->jacobian < 0 || o->jacobian > 2 ||
      (o->tangent_precision != TSGLS_PREC_F64 && o->tangent_precision != TSGLS_PREC_F32 &&
       o->tangent_precision != TSGLS_PREC_BF16) ||
      o->dt_schedule < TSGLS_DT_FIXED || o->dt_schedule > TSGLS_DT_AUTO || !std::isfinite(o->dt_max) ||
      !std::isfinite(o->dt_pseudo))
    return fail(c, TSGLS_EINVAL, "bad solve options");
  if (o->dt_schedule != TSGLS_DT_FIXED && !(o->dt_pseudo > 0))
    return fail(c, TSGLS_EINVAL, "an adaptive pseudo-time schedule needs dt_pseudo > 0");
  if (c->nseg > 1) return fail(c, TSGLS_EINVAL, "a context with segments is solved by tsgls_solve_segments");
  const auto t0 = std::chrono::steady_clock::now();
  tsgls_solve_stats st{};
  st.switched_at = -1;
  CHK(ensure_krylov(c, o->restart));
  const int64_t n = ndof(c);
  double* r = c->rs;
  // the first tau of a solve starts cold, so that the result depends on the
  // arguments only and not on what the context linearized before
  c->tauV_ok = false;
  CHK(linearize_impl(c, y, r));
  double r0;
  CHK(norm2(c, r, &r0));
  if (!std::isfinite(r0)) return fail(c, TSGLS_ENONFINITE, "non-finite initial residual");
  st.r0_norm = r0;
  double rn = r0;
  int it = 0;
  int status = TSGLS_NOT_CONVERGED;
  // pseudo-time state: dt of the next step (0 = no shift), whether the
  // schedule adapts it, and the stall counter of the AUTO schedule
  const bool adaptive = o->dt_schedule != TSGLS_DT_FIXED;
  bool ser = o->dt_schedule == TSGLS_DT_SER;
  double dt = o->dt_schedule == TSGLS_DT_AUTO ? 0.0 : o->dt_pseudo;
  int slow = 0;
  for (;;) {
    const double rel = r0 > 0 ? rn / r0 : 0.0;
    st.rel_residual = rel;
    if (it > 0 && it <= 64) st.history[it - 1] = rel;
    if (rel <= o->rtol || r0 == 0.0) {
      status = TSGLS_OK;
      break;
    }
    if (it >= o->max_newton) break;
    CHK(diag_impl(c, c->minv, dt));
    HIPCHK(c, launch_recip(c->minv, n, c->st));
    // b = -r in place (r is recomputed after the update)
    HIPCHK(c, launch_scal_copy(-1.0, r, r, n, c->st));
    int mv = 0;
    bool lin_ok = false;
    if (o->restart <= 32 && o->gmres_graph)
      CHK(gmres_graph(c, r, c->kx, o->lin_rtol, o->restart, o->max_matvec, o->jacobian, dt,
                      o->tangent_precision, &mv, &lin_ok));
    else if (o->restart <= GS_DELAYED_MAX)
      CHK(gmres_delayed(c, r, c->kx, o->lin_rtol, o->restart, o->max_matvec, o->jacobian, dt,
                        o->tangent_precision, &mv, &lin_ok));
    else
      CHK(gmres(c, r, c->kx, o->lin_rtol, o->restart, o->max_matvec, o->jacobian, dt,
                o->tangent_precision, &mv, &lin_ok));
    st.matvecs += mv;
    if (!lin_ok) ++st.lin_unconverged;
    if (adaptive) HIPCHK(c, launch_copy(y, c->ybak, n, c->st));
    HIPCHK(c, launch_axpy(1.0, c->kx, y, n, c->st));
    CHK(linearize_impl(c, y, r));
    double rnew;
    CHK(norm2(c, r, &rnew));
    ++it;
    st.dt_last = dt;
    if (adaptive && (!std::isfinite(rnew) || rnew > 1e3 * rn)) {
      // rejected: back to the previous iterate, a tenth of the step (a
      // rejected plain Newton step starts the pseudo-time schedule)
      HIPCHK(c, launch_copy(c->ybak, y, n, c->st));
      CHK(linearize_impl(c, y, r));
      ++st.rejected;
      if (!ser) {
        ser = true;
        st.switched_at = it;
        dt = o->dt_pseudo;
      } else {
        dt = (dt > 0 ? dt : o->dt_pseudo) * 0.1;
      }
      if (o->verbose)
        fprintf(stderr, "tsgls step %d rejected (|r|/|r0| %.3e), next dt %.3g\n", it, rnew / r0, dt);
      continue;
    }
    if (!std::isfinite(rnew)) return fail(c, TSGLS_ENONFINITE, "non-finite residual at Newton step %d", it);
    if (o->verbose)
      fprintf(stderr, "tsgls newton %d: |r|/|r0| = %.3e  gmres %d%s  dt %.3g\n", it, rnew / r0, mv,
              lin_ok ? "" : " (short of lin_rtol)", dt);
    if (ser) {
      // switched evolution relaxation: dt grows as the residual falls; a
      // linear solve that ran out of products before reaching lin_rtol
      // halves it instead (the shifted system was too hard for the Krylov
      // budget, and a larger step would only be harder)
      if (dt > 0) {
        if (lin_ok)
          dt *= std::min(10.0, std::max(0.1, rn / rnew));
        else
          dt *= 0.5;
        if (o->dt_max > 0) dt = std::min(dt, o->dt_max);
        else if (dt > 1e12) dt = 0.0;
      }
    } else if (o->dt_schedule == TSGLS_DT_AUTO) {
      slow = rnew > 0.99 * rn ? slow + 1 : 0;
      if (slow >= 3) {   // plain Newton has stalled: continue in pseudo-time
        ser = true;
        st.switched_at = it;
        dt = o->dt_pseudo;
      }
    }
    rn = rnew;
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  st.newton_iters = it;
  st.status = status;
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return status;
}

int tsgls_set_segments(tsgls_ctx* c, int nseg) {
  if (!c) return TSGLS_EINVAL;
  if (nseg < 1 || c->nn % nseg != 0) return fail(c, TSGLS_EINVAL, "nseg must be >= 1 and divide n_nodes");
  if (c->tracer && nseg > 1) return fail(c, TSGLS_EINVAL, "a tracer context takes no segments");
  HIPCHK(c, hipStreamSynchronize(c->st));
  free_gm(c);
  const int old = c->nseg;
  c->nseg = nseg;
  c->seg_checked = false;
  const int rc = check_segments(c);
  if (rc != TSGLS_OK) {
    c->nseg = old;
    c->seg_checked = false;
    return rc;
  }
  // Element order.  Within a segment it is always that of its mesh alone
  // (Morton key, then input order), so sums over a node's elements run in
  // the same order as for the lone problem.  Segments of equal element
  // counts are stored segment-major, and the element operator runs over the
  // elements of the segments taking part only (a list on the device).
  // Otherwise the whole mesh is in Morton order with copies of equal keys
  // ordered by a segment index rotated by a hash of the key: a wave of the
  // element kernel takes every nbx-th element, and with copy s at a fixed
  // offset in every group of nseg it would meet a single segment whenever
  // nbx is a multiple of nseg, leaving whole waves idle while others do
  // their full share when segments sit out.
  std::vector<int32_t> conn((size_t)c->E * 4), tin((size_t)c->E * 4);
  HIPCHK(c, hipMemcpy(conn.data(), c->conn, conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int64_t e = 0; e < c->E; ++e)
    for (int b = 0; b < 4; ++b) tin[(size_t)c->perm[e] * 4 + b] = conn[(size_t)e * 4 + b];
  const std::vector<uint64_t> key = morton_keys(c->hxyz.data(), c->nn, tin.data(), c->E);
  std::vector<int32_t> perm(c->E);
  for (int64_t e = 0; e < c->E; ++e) perm[e] = (int32_t)e;
  c->seg_elems = 0;
  std::vector<int64_t> per(nseg, 0);
  const int64_t Ln = c->nn / nseg;
  for (int64_t e = 0; e < c->E; ++e) ++per[tin[(size_t)e * 4] / Ln];
  const bool equal = nseg > 1 && std::all_of(per.begin(), per.end(), [&](int64_t k) { return k == per[0]; });
  if (equal) {
    // segment-major: segment s owns positions [s E/nseg, (s+1) E/nseg), Morton
    // order inside; the element operator then runs over a list of the
    // segments taking part
    c->seg_elems = (int32_t)per[0];
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
      const int64_t sa = tin[(size_t)a * 4] / Ln, sb = tin[(size_t)b * 4] / Ln;
      return sa != sb ? sa < sb : key[a] < key[b];
    });
  } else if (nseg > 1) {
    auto rot = [&](int32_t e) {
      const uint64_t h = (key[e] * 0x9E3779B97F4A7C15ull) >> 32;
      return (uint64_t)(tin[(size_t)e * 4] / Ln + h) % (uint64_t)nseg;
    };
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
      return key[a] != key[b] ? key[a] < key[b] : rot(a) < rot(b);
    });
  } else {
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  }
  return set_order(c, tin.data(), perm);
}

int tsgls_solve_segments(tsgls_ctx* c, double* y, const tsgls_solve_opts* o, tsgls_solve_stats* stats,
                         double* finish_s) {
  if (!c) return TSGLS_EINVAL;
  if (!y || !o || !stats) return fail(c, TSGLS_EINVAL, "null argument");
  if (o->restart < 1 || o->restart > 32 || o->max_newton < 0 || o->max_matvec < 1 || !(o->rtol > 0) ||
      !(o->lin_rtol > 0) || o->jacobian < 0 || o->jacobian > 2 ||
      (o->tangent_precision != TSGLS_PREC_F64 && o->tangent_precision != TSGLS_PREC_F32 &&
       o->tangent_precision != TSGLS_PREC_BF16) ||
      o->dt_schedule != TSGLS_DT_FIXED || !std::isfinite(o->dt_pseudo))
    return fail(c, TSGLS_EINVAL, "bad options for a segmented solve (restart <= 32, fixed pseudo-time step)");
  if (c->tracer) return fail(c, TSGLS_EINVAL, "segmented solves take the flow operator");
  CHK(check_segments(c));
  const auto t0 = std::chrono::steady_clock::now();
  auto now = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  const int S = c->nseg;
  CHK(ensure_krylov(c, o->restart));
  CHK(ensure_gm(c));
  const int64_t n = ndof(c);
  double* r = c->rs;
  // Segments that have finished sit out the element kernels and gathers:
  // gm.skip flags them (frozen ones during linearization, and during GMRES
  // also those whose linear solve of this step is over).
  struct MaskOn {
    tsgls_ctx* c;
    explicit MaskOn(tsgls_ctx* x) : c(x) { c->seg_mask_on = true; }
    ~MaskOn() { c->seg_mask_on = false; }
  } mask_on(c);
  std::vector<char> frozen(S, 0);
  auto write_skip = [&]() -> int {
    int* skip = c->hseg + (size_t)S * GM_ST;
    for (int s = 0; s < S; ++s) skip[s] = frozen[s];
    return write_mask(c);
  };
  CHK(write_skip());
  c->tauV_ok = false;   // the first tau starts cold, as in tsgls_solve
  CHK(linearize_impl(c, y, r));
  std::vector<double> r0(S), rn(S), rnew(S), fin(S, 0.0);
  CHK(seg_norms(c, r, r0.data()));
  for (int s = 0; s < S; ++s)
    if (!std::isfinite(r0[s])) return fail(c, TSGLS_ENONFINITE, "non-finite initial residual (segment %d)", s);
  std::vector<tsgls_solve_stats> st(S);
  for (int s = 0; s < S; ++s) {
    st[s] = tsgls_solve_stats{};
    st[s].switched_at = -1;
    st[s].status = TSGLS_NOT_CONVERGED;
    st[s].r0_norm = r0[s];
    rn[s] = r0[s];
  }
  std::vector<int> it(S, 0), mv(S, 0);
  std::unique_ptr<bool[]> lin_ok(new bool[S]);
  const double dt = o->dt_pseudo;
  for (;;) {
    int nact = 0;
    for (int s = 0; s < S; ++s) {
      if (frozen[s]) continue;
      const double rel = r0[s] > 0 ? rn[s] / r0[s] : 0.0;
      st[s].rel_residual = rel;
      if (it[s] > 0 && it[s] <= 64) st[s].history[it[s] - 1] = rel;
      if (rel <= o->rtol || r0[s] == 0.0) st[s].status = TSGLS_OK;
      if (st[s].status == TSGLS_OK || it[s] >= o->max_newton) {
        frozen[s] = 1;
        fin[s] = now();
        continue;
      }
      ++nact;
    }
    if (nact == 0) break;
    CHK(diag_impl(c, c->minv, dt));
    HIPCHK(c, launch_recip(c->minv, n, c->st));
    HIPCHK(c, launch_scal_copy(-1.0, r, r, n, c->st));
    CHK(gmres_graph(c, r, c->kx, o->lin_rtol, o->restart, o->max_matvec, o->jacobian, dt,
                    o->tangent_precision, mv.data(), lin_ok.get(), frozen.data()));
    HIPCHK(c, launch_axpy(1.0, c->kx, y, n, c->st));
    CHK(write_skip());
    CHK(linearize_impl(c, y, r));
    CHK(seg_norms(c, r, rnew.data()));
    for (int s = 0; s < S; ++s) {
      if (frozen[s]) continue;
      st[s].matvecs += mv[s];
      if (!lin_ok[s]) ++st[s].lin_unconverged;
      ++it[s];
      st[s].dt_last = dt;
      if (!std::isfinite(rnew[s]))
        return fail(c, TSGLS_ENONFINITE, "non-finite residual at Newton step %d (segment %d)", it[s], s);
      if (o->verbose)
        fprintf(stderr, "tsgls segment %d newton %d: |r|/|r0| = %.3e  gmres %d\n", s, it[s],
                rnew[s] / r0[s], mv[s]);
      rn[s] = rnew[s];
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  int status = TSGLS_OK;
  for (int s = 0; s < S; ++s) {
    st[s].newton_iters = it[s];
    st[s].seconds = fin[s];
    stats[s] = st[s];
    if (finish_s) finish_s[s] = fin[s];
    if (st[s].status != TSGLS_OK) status = TSGLS_NOT_CONVERGED;
  }
  return status;
}

int tsgls_solve_batch(tsgls_ctx* const* ctxs, double* const* ys, int nb, const tsgls_solve_opts* o,
                      tsgls_solve_stats* stats, double* finish_s, int max_concurrent) {
  if (nb < 0) return TSGLS_EINVAL;
  if (nb == 0) return TSGLS_OK;
  if (!ctxs || !ys || !o) return TSGLS_EINVAL;
  {
    std::set<const tsgls_ctx*> seen;
    for (int i = 0; i < nb; ++i) {
      if (!ctxs[i]) return TSGLS_EINVAL;
      if (!ys[i] || !seen.insert(ctxs[i]).second) return fail(ctxs[i], TSGLS_EINVAL, "null state or repeated context in batch");
    }
  }
  const int T = std::max(1, std::min(nb, max_concurrent > 0 ? max_concurrent : 8));
  std::vector<int> rc(nb, TSGLS_OK);
  std::atomic<int> next{0};
  const auto t0 = std::chrono::steady_clock::now();
  auto worker = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= nb) break;
      tsgls_solve_stats st{};
      if (hipSetDevice(ctxs[i]->dev) != hipSuccess) {
        rc[i] = fail(ctxs[i], TSGLS_EHIP, "hipSetDevice failed");
      } else {
        rc[i] = tsgls_solve(ctxs[i], ys[i], o, &st);
      }
      if (stats) stats[i] = st;
      if (finish_s)
        finish_s[i] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < T; ++t) pool.emplace_back(worker);
  } catch (...) {
    // fewer workers (down to this thread alone) if threads cannot be created
  }
  worker();
  for (auto& th : pool) th.join();
  int out = TSGLS_OK;
  for (int i = 0; i < nb; ++i) {
    if (rc[i] < 0) return rc[i];
    if (rc[i] == TSGLS_NOT_CONVERGED) out = TSGLS_NOT_CONVERGED;
  }
  return out;
}

int tsgls_info(const tsgls_ctx* c, int64_t* n_colors, int64_t* n_tets, int64_t* n_nodes,
               int64_t* device_bytes) {
  if (!c) return TSGLS_EINVAL;
  if (n_colors) *n_colors = 1;   // one element launch per operator application
  if (n_tets) *n_tets = c->E;
  if (n_nodes) *n_nodes = c->nn;
  if (device_bytes) *device_bytes = (int64_t)c->dev_bytes;
  return TSGLS_OK;
}

int tsgls_profile(tsgls_ctx* c, int enable) {
  if (!c) return TSGLS_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->prof = enable != 0;
  c->prof_recs.clear();
  c->ev_used = 0;
  return TSGLS_OK;
}

int tsgls_profile_get(tsgls_ctx* c, int which, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return TSGLS_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->st));
  int64_t cnt = 0;
  double tot = 0.0;
  for (auto& r : c->prof_recs) {
    if (r.first != which) continue;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, r.second.first, r.second.second));
    tot += ms;
    ++cnt;
  }
  *launches = cnt;
  *total_ms = tot;
  return TSGLS_OK;
}

const char* tsgls_last_error(const tsgls_ctx* c) { return c ? c->err.c_str() : "null context"; }

void tsgls_destroy(tsgls_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  if (c->gst) (void)hipStreamSynchronize(c->gst);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  for (hipEvent_t e : c->gev)
    if (e) (void)hipEventDestroy(e);
  if (c->gst) (void)hipStreamDestroy(c->gst);
  if (c->hp) (void)hipHostFree(c->hp);
  if (c->hseg) (void)hipHostFree(c->hseg);
  if (c->hsegd) (void)hipHostFree(c->hsegd);
  for (void* p : c->allocs) (void)hipFree(p);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
