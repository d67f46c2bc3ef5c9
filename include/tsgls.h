/*
 * tsgls.h -- C ABI of the MI355X (gfx950) library for the stabilized
 * time-spectral Galerkin/least-squares (GLS) finite element method for
 * time-periodic incompressible Navier-Stokes on linear tetrahedra
 * (Esmaily & Jia, arXiv:2311.09465).
 *
 * What it computes (paper references are to that article):
 *   residual  -- eq. Rmc (momentum rows r^m for non-Dirichlet nodes,
 *                continuity rows r^c for all nodes) plus the backflow
 *                stabilization term of the section "Stabilizing simulations
 *                in the presence of backflow" and the Neumann traction term;
 *   linearize -- freezes the convection matrices A_i and the stabilization
 *                matrix tau = [A_i G_ij A_j + C_I nu^2 G_ij G_ij I]^(-1/2)
 *                (eq. 3D-tau, nu = mu/rho) at every volume quadrature point,
 *                and |A_n|_- at every Neumann-face quadrature point;
 *   jv        -- the tangent-vector product: eq. K_mat ("Picard": A and tau
 *                frozen, remark 5 after eq. K_mat), optionally without the
 *                least-squares part of G_i and D_i (section "Exploiting the
 *                structure of H"), or with the derivative of A_i kept
 *                ("Newton", tau still frozen); optional pseudo-time mass
 *                shift c1 rho / dt (N_A, N_B), c1 = 1.5 (section
 *                "Pseudo-time stepping");
 *   solve     -- Newton-Raphson (eq. NR) with right-Jacobi-preconditioned
 *                restarted GMRES, stopped at ||r|| <= rtol ||r^0|| (remarks
 *                after eq. K_mat); or pseudo-time stepping with one Newton
 *                iteration per pseudo-time step and an adaptive step size
 *                (section "Pseudo-time stepping").
 *
 * Conventions shared by every entry point
 *   Mode count   K = number of harmonics (the paper's N is K+1).
 *   State layout y[n_nodes][4][2K+2] float64, fields (u1, u2, u3, p);
 *                slot 2k = Re c_k, slot 2k+1 = Im c_k, k = 0..K, where a real
 *                periodic field is f(t) = sum_{|k|<=K} c_k exp(i k omega t)
 *                (real-valued unknowns of the section "Using real-valued
 *                unknowns"; slot 1 (Im c_0) is ignored on input and written
 *                as 0 on output).  Residual and tangent outputs use the same
 *                layout: slot 2k = Re r_k, 2k+1 = Im r_k.
 *   Dirichlet    velocity values are part of y (the paper's implementation
 *                builds them into the unknown vector); momentum rows of
 *                Dirichlet nodes are written as 0, and jv treats the
 *                Dirichlet velocity entries of its input as 0.
 *   Memory       mesh and boundary-data arrays passed to create/set_* are
 *                HOST pointers and are copied; y, r, v, Jv, d are DEVICE
 *                pointers (float64, n_nodes*4*(2K+2) entries) owned by the
 *                caller.  The library owns everything it allocates.
 *   Streams      all device work is enqueued on the hip_stream given to
 *                tsgls_create (NULL = default stream).  residual / linearize
 *                / jv / jacobi_diag return without synchronizing; solve
 *                synchronizes before it returns.
 *   Errors       every call returns TSGLS_OK (0) or a negative code; the
 *                message of the last error is in tsgls_last_error(ctx).
 *                solve may return TSGLS_NOT_CONVERGED (+1) with y and the
 *                statistics written.  No exception crosses this boundary.
 */
#ifndef TSGLS_H
#define TSGLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSGLS_OK 0
#define TSGLS_NOT_CONVERGED 1
#define TSGLS_EINVAL (-1)      /* null pointer, bad size, K or nu out of range */
#define TSGLS_EHIP (-2)        /* a HIP runtime call failed */
#define TSGLS_ENOMEM (-3)      /* device or host allocation failed */
#define TSGLS_EMESH (-4)       /* non-positive tet volume, bad index, degenerate face */
#define TSGLS_ENONFINITE (-5)  /* NaN/Inf in the residual or a Krylov quantity */
#define TSGLS_ESTATE (-6)      /* jv / jacobi_diag before linearize */
#define TSGLS_ESCRATCH (-7)    /* request larger than the fixed scratch of an
                                  allocation-free entry point */

/* Tangent variants (jv, jacobi_diag, solve). */
#define TSGLS_JAC_PICARD 0       /* eq. K_mat: A_i and tau frozen (paper's tangent) */
#define TSGLS_JAC_PICARD_NOLS 1  /* eq. K_mat with least-squares terms of G_i, D_i dropped */
#define TSGLS_JAC_NEWTON 2       /* A_i(u) differentiated, tau and |A_n|_- frozen */

/* Arithmetic of the tangent product (jv, solve).  The residual, the
 * linearization (tau from the eigendecomposition of eq. 3D-tau), the Jacobi
 * diagonal, the Newton update and the Krylov orthogonalization are FP64 in
 * both; with TSGLS_PREC_F32 the element operator of the tangent runs in FP32
 * (FP32 MFMA transforms, FP32 copies of tau, of the frozen velocity samples
 * and of tau L(u)) and its element rows are summed per node in FP64, so the
 * FP64 residual of each Newton step corrects the rounding of the linear
 * solves (iterative refinement).  Face terms stay FP64. */
#define TSGLS_PREC_F64 0
#define TSGLS_PREC_F32 1
/* TSGLS_PREC_F32 with tau stored and applied in bf16 (8-bit significand,
 * round to nearest even, made from the FP64 tau once per linearization):
 * the dominant operand stream of the product at half the FP32 bytes; the
 * relative error of the product grows to order 1e-3, still far below the
 * GMRES tolerance, and the FP64 residual of each Newton step corrects it. */
#define TSGLS_PREC_BF16 2

/* Pseudo-time schedule of tsgls_solve (section "Pseudo-time stepping": one
 * Newton iteration per pseudo-time step, the tangent shifted by
 * 1.5 rho / dt (N_A, N_B); the converged solution does not depend on it).
 *   TSGLS_DT_FIXED  every step uses dt_pseudo (<= 0: no shift, plain Newton).
 *   TSGLS_DT_SER    the first step uses dt_pseudo > 0; after each step the
 *                   size is multiplied by ||r_old|| / ||r_new|| clipped to
 *                   [0.1, 10] (switched evolution relaxation), or halved if
 *                   that step's GMRES used max_matvec products without
 *                   reaching lin_rtol, and bounded by dt_max if dt_max > 0
 *                   (else it grows without bound and the shift is dropped
 *                   once dt exceeds 1e12).
 *   TSGLS_DT_AUTO   plain Newton steps while the residual falls; after three
 *                   consecutive steps whose residual ratio exceeds 0.99 (a
 *                   stall) or one rejected step, continues as TSGLS_DT_SER
 *                   from dt_pseudo > 0.
 * Under SER and AUTO a step whose residual is non-finite or grows by more
 * than 1e3 is rejected: y returns to the previous iterate and the next step
 * size is a tenth of the rejected one (a rejected step counts as a Newton
 * iteration). */
#define TSGLS_DT_FIXED 0
#define TSGLS_DT_SER 1
#define TSGLS_DT_AUTO 2

typedef struct tsgls_ctx tsgls_ctx;

typedef struct {
  double rho;            /* density > 0 */
  double mu;             /* dynamic viscosity > 0; nu = mu/rho enters tau */
  double omega;          /* base angular frequency 2 pi / T */
  int K;                 /* harmonics, 0 <= K; compiled set in tsgls_supported_K */
  double C_I;            /* tau diffusive constant, 3 for linear tets */
  double backflow_beta;  /* backflow coefficient beta in [0, 1] */
} tsgls_params;

typedef struct {
  double rtol;       /* Newton stop: ||r|| <= rtol ||r^0||, e.g. 1e-8 */
  double lin_rtol;   /* GMRES relative tolerance, e.g. 0.05 */
  int restart;       /* Krylov dimension, e.g. 100 (1..1000); up to 128 GMRES uses
                        delayed classical Gram-Schmidt (one reduction and one
                        host synchronization per Arnoldi step), above that
                        two-pass classical Gram-Schmidt */
  int max_newton;    /* Newton / pseudo-time iterations */
  int max_matvec;    /* tangent products per linear solve */
  int jacobian;      /* TSGLS_JAC_* */
  double dt_pseudo;  /* pseudo-time step; <= 0 disables the mass shift */
  int verbose;       /* 1: one line per Newton step on stderr */
  int tangent_precision;  /* TSGLS_PREC_F64 (0, default), TSGLS_PREC_F32 or TSGLS_PREC_BF16 */
  int gmres_graph;   /* 1 (restart <= 32): each GMRES cycle is one HIP graph with
                        the least-squares update on the device, captured on the
                        first use of a (restart, tangent, dt_pseudo, precision)
                        and replayed; one host synchronization per cycle, cycles
                        always make restart products (whole cycles count against
                        max_matvec, the first cycle always runs); with
                        restart > 32 the flag is ignored */
  int dt_schedule;   /* TSGLS_DT_FIXED (0, default), TSGLS_DT_SER, TSGLS_DT_AUTO */
  double dt_max;     /* SER / AUTO: upper bound of the pseudo-time step (<= 0: none) */
} tsgls_solve_opts;

typedef struct {
  int newton_iters;
  int matvecs;
  int status;             /* TSGLS_OK or TSGLS_NOT_CONVERGED */
  double rel_residual;    /* ||r|| / ||r^0|| at return */
  double r0_norm;         /* ||r^0|| (Euclidean norm of the masked slot vector) */
  double seconds;         /* wall time of the solve */
  double history[64];     /* ||r||/||r^0|| after each Newton step (first 64) */
  int rejected;           /* pseudo-time steps rejected (SER / AUTO) */
  int switched_at;        /* AUTO: Newton iteration at which pseudo-time began, -1 if never */
  double dt_last;         /* pseudo-time step of the last iteration (0: no shift) */
  int lin_unconverged;    /* Newton steps whose GMRES stopped at max_matvec short of lin_rtol */
} tsgls_solve_stats;

/* Harmonic counts compiled into this library: writes up to cap values into
 * out, returns how many exist. */
int tsgls_supported_K(int* out, int cap);

/* Create a context for one mesh of linear tetrahedra: the P1 shape
 * functions N_A and the metric G_ij of the parent element (section
 * "Convection-diffusion in multiple dimensions", eq. 3D-tau1) are formed
 * here, once per mesh, with the physical parameters of eq. NS-weak (rho, mu;
 * omega the base frequency of the time-periodic solution, K its harmonics).
 * xyz: host [n_nodes][3]; tets: host [n_tets][4] 0-based, positively
 * oriented (TSGLS_EMESH otherwise).  The library orders the elements along a
 * Morton curve, builds the node -> element incidence used to sum element
 * contributions deterministically, and computes the element geometry on the
 * device.  TSGLS_EINVAL for null pointers, non-positive sizes, rho or mu,
 * beta outside [0, 1] or a K that is not compiled; TSGLS_ENOMEM, TSGLS_EHIP.
 * The caller owns xyz and tets (copied); *out must be freed with
 * tsgls_destroy, also after an error (then it may be NULL). */
int tsgls_create(const double* xyz, int64_t n_nodes, const int32_t* tets,
                 int64_t n_tets, const tsgls_params* params, void* hip_stream,
                 tsgls_ctx** out);

/* Nodes whose three velocity components are prescribed (the Dirichlet part
 * Gamma_g of the boundary in eq. NS-weak; the test functions vanish there,
 * so the momentum rows of these nodes are removed from eq. Rmc, as in the
 * remarks after eq. K_mat).  nodes: host, n entries, each in [0, n_nodes)
 * (TSGLS_EINVAL otherwise), copied.  The prescribed values are not passed
 * here: they are the velocity entries of the state y given to the other
 * calls.  Replaces any earlier set and clears the linearization. */
int tsgls_set_dirichlet(tsgls_ctx* ctx, const int32_t* nodes, int64_t n);

/* Neumann (outflow) faces: host tris [nf][3] node ids, ordered so that
 * (x1-x0) x (x2-x0) points out of the domain; h: host [nf][2K+2] traction
 * modes per face (slot layout, constant over the face) or NULL for h = 0
 * (a context in tracer mode takes no traction: TSGLS_EINVAL).
 * Replaces any earlier set. */
int tsgls_set_neumann(tsgls_ctx* ctx, const int32_t* tris, int64_t nf,
                      const double* h);

/* Tracer mode: from this call on, the context solves the time-spectral GLS
 * convection-diffusion equation (eq. 3D-weak; tau of eq. 3D-tau with kappa
 * in place of nu) for a scalar tracer carried by the frozen periodic
 * velocity of y_velocity (device state [n_nodes][4][2K+2]; its velocity
 * fields are copied).  States and residuals keep the [n_nodes][4][2K+2]
 * layout with the tracer in field 0 (fields 1..3 are zero in every
 * residual and product).  tsgls_set_dirichlet gives the tracer's Dirichlet
 * nodes (their values are those of the state passed to tsgls_solve); on
 * the faces given by tsgls_set_neumann (which must carry no traction, h =
 * NULL) the operator includes the backflow term -(w, (beta/2)|A_n|_- phi)
 * of the remark on backflow for the convection-diffusion equation (beta of
 * tsgls_params, A_n from the frozen velocity); elsewhere the diffusive flux
 * is zero.  Returns TSGLS_EINVAL if a traction has been set.
 * stabilized = 0 drops the least-squares term (tau = 0): the Galerkin
 * method.  In tracer mode tsgls_jv ignores the variant and dt_pseudo (the
 * operator is linear), tsgls_jacobi_diag returns ones (GMRES runs without a
 * preconditioner) and only FP64 is available.  kappa > 0. */
int tsgls_set_tracer(tsgls_ctx* ctx, const double* y_velocity, double kappa,
                     int stabilized);

/* r = residual(y) (eq. Rmc + backflow + Neumann traction), masked.
 * Does not change the linearization used by jv. */
int tsgls_residual(tsgls_ctx* ctx, const double* y, double* r);

/* Freeze A_i, tau (and, for the Newton tangent, tau L_i(u)) at y.  If r is
 * not NULL the residual at y is written there as a by-product.  For
 * K <= 15 the eigen-iteration that gives tau starts from the eigenvectors
 * kept from this context's previous linearization (4 E n^2 doubles of device
 * memory, allocated on first use; without them it starts cold), so tau and
 * what follows from it depend on that history at the level of rounding.
 * tsgls_solve starts its first linearization cold. */
int tsgls_linearize(tsgls_ctx* ctx, const double* y, double* r);

/* Jv = J v with the last linearization; variant TSGLS_JAC_*; dt_pseudo > 0
 * adds the pseudo-time mass shift.  v and Jv must not alias. */
int tsgls_jv(tsgls_ctx* ctx, const double* v, double* Jv, int jacobian,
             double dt_pseudo);

/* tsgls_jv with the tangent's arithmetic chosen by precision (TSGLS_PREC_*);
 * TSGLS_PREC_F32 needs device memory for FP32 copies of the linearization
 * (4 P E + 12 n E + 3 M n_nodes floats), allocated on the first such call
 * (TSGLS_ENOMEM if that fails) and refreshed once after each linearize.  The
 * result is within FP32 rounding of the FP64 product (relative error of
 * order 1e-6 of the largest entry).  TSGLS_PREC_BF16 needs the same copies
 * plus a bf16 copy of tau (4 P E 16-bit words); its result carries the bf16
 * rounding of tau (relative error of order 1e-3). */
int tsgls_jv_prec(tsgls_ctx* ctx, const double* v, double* Jv, int jacobian,
                  double dt_pseudo, int precision);

/* d = diagonal of the Picard tangent (with the mass shift if dt_pseudo > 0),
 * 1 on masked slots. */
int tsgls_jacobi_diag(tsgls_ctx* ctx, double* d, double dt_pseudo);

/* Copy the frozen tau of the last linearize to HOST memory tau_out
 * [n_tets][4][n(n+1)/2], input element order, n = 2K+1, upper triangle row
 * by row, in the real orthonormal basis (c_0, sqrt2 Re c_1, sqrt2 Im c_1,
 * ..., sqrt2 Re c_K, sqrt2 Im c_K). */
int tsgls_get_tau(tsgls_ctx* ctx, double* tau_out);

/* Newton-GMRES from y (device, in: initial guess, out: solution).  stats is
 * a host pointer (may be NULL).  TSGLS_EINVAL on a context with segments. */
int tsgls_solve(tsgls_ctx* ctx, double* y, const tsgls_solve_opts* opts,
                tsgls_solve_stats* stats);

/* Segments: one context holding nseg independent problems of the same
 * harmonic count and physical parameters, for solves in lockstep (many
 * inflow waveforms on one mesh; an extension for throughput, the paper
 * solves one problem at a time).  The context's
 * nodes are nseg equal contiguous blocks (n_nodes / nseg each; problem s
 * owns nodes [s n_nodes/nseg, (s+1) n_nodes/nseg) and so the same block of
 * every state vector); no element or Neumann face may join two blocks.
 * Typically the caller repeats one mesh nseg times with the node numbers
 * offset, and gives each copy its own Dirichlet values.  TSGLS_EINVAL if
 * nseg < 1, nseg does not divide n_nodes, an element joins two blocks, or
 * the context is in tracer mode.  nseg = 1 undoes it.  The elements are
 * put in a new processing order (segment by segment when all segments have
 * as many elements, each in its own Morton order), which invalidates the
 * linearization (TSGLS_ESTATE from tsgls_jv until the next linearize).
 * Residual, tangent, linearize and the Jacobi diagonal act on all segments
 * at once as on any context (they are local to elements and nodes). */
int tsgls_set_segments(tsgls_ctx* ctx, int nseg);

/* Newton-GMRES on every segment at once, in lockstep: each Newton step
 * linearizes all of them in one pass, and each GMRES cycle is one captured
 * HIP graph (as with gmres_graph) whose launches cover all segments -- one
 * tangent product of the whole context per Arnoldi step, and reductions,
 * Gram-Schmidt updates and the least-squares (Givens) update per segment in
 * single launches on the device; the host reads one status word per segment
 * per cycle.  Each segment's reductions use the blocking a lone problem of
 * its size would use, so segment s follows, bit for bit, the iteration of
 * tsgls_solve with gmres_graph = 1 on a context holding problem s alone.  A
 * segment that has converged (or reached max_newton / max_matvec) sits out
 * the rest with zero updates; its state is no longer changed, and the
 * kernels skip it (the element operator runs over a device list of the
 * segments taking part when the segments have equal element counts).  Options as
 * tsgls_solve with restart <= 32 and the fixed schedule (TSGLS_EINVAL
 * otherwise); gmres_graph is implied.  stats: host [nseg] (per segment;
 * seconds = time from the call's start until that segment finished);
 * finish_s: host [nseg] or NULL, the same times.  Returns TSGLS_OK if every
 * segment reached rtol, else TSGLS_NOT_CONVERGED, or a negative error
 * (ENONFINITE names the segment in tsgls_last_error). */
int tsgls_solve_segments(tsgls_ctx* ctx, double* y, const tsgls_solve_opts* opts,
                         tsgls_solve_stats* stats, double* finish_s);

/* Batched solves: nb independent problems, ctxs[i] (distinct contexts, each
 * with its own stream for the solves to overlap on the device; any harmonic
 * count K) from the device states ys[i] (in: initial guess, out: solution),
 * all with the options o.  Up to max_concurrent (<= 0: 8) host threads each
 * drive one tsgls_solve at a time; every solve's arithmetic and its result
 * are those of tsgls_solve on the same context (bitwise: no kernel uses
 * atomics).  stats (host [nb], may be NULL) receives each solve's statistics
 * (seconds = the solve's own wall time); finish_s (host [nb], may be NULL)
 * the time from this call's start to the end of solve i, i.e. its latency
 * in the batch.  Returns the first negative code of a failed solve (the
 * other solves still run to the end), else TSGLS_NOT_CONVERGED if any solve
 * did not reach rtol, else TSGLS_OK.  TSGLS_EINVAL for a null or repeated
 * context or a null state. */
int tsgls_solve_batch(tsgls_ctx* const* ctxs, double* const* ys, int nb,
                      const tsgls_solve_opts* o, tsgls_solve_stats* stats,
                      double* finish_s, int max_concurrent);

/* ------------------------------------------------------------------------
 * Learned warm start.  A reduced basis of modal solutions and a fully
 * connected tanh network mapping inflow parameters to reduced-basis
 * coefficients; Newton-GMRES started from its prediction stays the solver
 * and the judge of the result.  Not part of the paper's method: the
 * network's training data are solutions of the method itself.
 *
 * Reduced basis (all arrays device FP64, vectors of length D, row-major):
 * tsgls_rb_greedy picks, r times, the snapshot of Y [N][D] (N <= 65536,
 * r <= min(N, 1024))
 * worst represented by the basis so far (largest |y - mean - P(y - mean)|),
 * orthonormalizes it against the basis (classical Gram-Schmidt, two passes)
 * and stores it in Phi [r][D]; picked (host [r]) receives the snapshot
 * indices.  Returns the number of basis vectors built (< r when the
 * snapshots span fewer directions) or a negative error code.  Allocates its
 * workspace (N*D doubles) on the device.  tsgls_rb_project: coef [N][r] =
 * Phi (Y_i - mean).  tsgls_rb_expand: y = mean + Phi^T coef (coef device
 * [r]).  All run on hip_stream. */
int tsgls_rb_greedy(const double* Y, int64_t N, int64_t D, const double* mean, int r,
                    double* Phi, int32_t* picked, void* hip_stream);
int tsgls_rb_project(const double* Phi, int r, int64_t D, const double* Y, int64_t N,
                     const double* mean, double* coef, void* hip_stream);
int tsgls_rb_expand(const double* Phi, int r, int64_t D, const double* coef,
                    const double* mean, double* y, void* hip_stream);

/* tsgls_rb_project for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and the same result bit for bit,
 * but it calls no allocator.  Its block partial sums and the projected mean
 * live in a fixed device array of 1024 * 1024 + 1024 doubles (8.0 MiB) per
 * GPU, held until the process ends, whose address is looked up on the first
 * call made with that GPU current.  r > 1024 returns TSGLS_ESCRATCH; bad
 * pointers or sizes TSGLS_EINVAL.  Returns without synchronizing (the work
 * is ordered on hip_stream).  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other streams or host threads) race, so a
 * caller serializes them.  Nothing in the array needs to start at zero; each
 * call overwrites what it reads. */
int tsgls_rb_project_noalloc(const double* Phi, int r, int64_t D, const double* Y,
                             int64_t N, const double* mean, double* coef,
                             void* hip_stream);

/* Network: n_in -> n_hidden layers of width (tanh) -> n_out (linear).
 * Weights W_l [d_{l+1}][d_l] and biases b_l, l = 0..n_hidden, stored as one
 * FP32 parameter vector in that order (W_0, b_0, W_1, b_1, ...); initial W
 * uniform in +-1/sqrt(d_l) from splitmix64(seed), b = 0.  precision
 * TSGLS_MLP_BF16: products on bf16 MFMA with FP32 accumulation (operands
 * rounded from the FP32 master weights and activations); TSGLS_MLP_F32:
 * FP32 MFMA (for checking).  x [B][n_in], y and targets [B][n_out] are
 * device FP32 arrays.  tsgls_mlp_gradient evaluates the loss
 * mean_{b,j} (y - t)^2 and its gradient with respect to the parameters
 * (kept on the device; loss to host if not NULL); tsgls_mlp_adam_step
 * applies one bias-corrected Adam step with that gradient.
 * tsgls_mlp_get_params copies parameters and/or the last gradient to host
 * arrays of tsgls_mlp_num_params floats.  Errors: TSGLS_EINVAL for bad
 * sizes or pointers, TSGLS_EHIP, TSGLS_ENOMEM; message in
 * tsgls_mlp_last_error. */
#define TSGLS_MLP_BF16 0
#define TSGLS_MLP_F32 1
typedef struct tsgls_mlp tsgls_mlp;
int tsgls_mlp_create(int n_in, int width, int n_hidden, int n_out, int precision,
                     uint64_t seed, void* hip_stream, tsgls_mlp** out);
int tsgls_mlp_num_params(const tsgls_mlp* m, int64_t* count);
int tsgls_mlp_get_params(tsgls_mlp* m, float* params_out, float* grad_out);
int tsgls_mlp_set_params(tsgls_mlp* m, const float* params_in);
int tsgls_mlp_forward(tsgls_mlp* m, const float* x, int B, float* y);
int tsgls_mlp_gradient(tsgls_mlp* m, const float* x, const float* targets, int B,
                       float* loss);
int tsgls_mlp_adam_step(tsgls_mlp* m, float lr, float beta1, float beta2, float eps);
const char* tsgls_mlp_last_error(const tsgls_mlp* m);
void tsgls_mlp_destroy(tsgls_mlp* m);

/* Introspection: element launches per operator application (1), element and
 * node counts, bytes held on device. */
int tsgls_info(const tsgls_ctx* ctx, int64_t* n_colors, int64_t* n_tets,
               int64_t* n_nodes, int64_t* device_bytes);

/* Per-launch timing with HIP events on the context stream, for benchmarks.
 * tsgls_profile(ctx, 1) clears the records and starts recording an event
 * pair around every launch of the kernels below; tsgls_profile(ctx, 0)
 * stops.  tsgls_profile_get synchronizes the stream and returns, for one
 * kernel class, the number of recorded launches and their summed duration. */
#define TSGLS_PROF_ELEM_TANGENT 0   /* element kernel in jv (one launch per product) */
#define TSGLS_PROF_ELEM_RESIDUAL 1  /* element kernel in residual / linearize */
#define TSGLS_PROF_TAU 2            /* tau kernel (one launch per linearize) */
#define TSGLS_PROF_DIAG 3           /* Jacobi-diagonal element kernel */
#define TSGLS_PROF_FACE 4           /* face-point kernel of the residual (a tangent
                                       product forms its face points in the launch
                                       of its nodal time samples, which is not timed) */
#define TSGLS_PROF_ORTHO 5          /* Gram-Schmidt block of one GMRES iteration */
#define TSGLS_PROF_GATHER 6         /* node-wise sum of element contributions and
                                       of the Neumann face terms */
int tsgls_profile(tsgls_ctx* ctx, int enable);
int tsgls_profile_get(tsgls_ctx* ctx, int which, int64_t* launches, double* total_ms);

const char* tsgls_last_error(const tsgls_ctx* ctx);

void tsgls_destroy(tsgls_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TSGLS_H */
