"""Python binding of libtsgls.so (include/tsgls.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy/torch
arguments to pointers and raises on error codes.  Device vectors are torch
float64 CUDA tensors of shape (n_nodes, 4, 2K+2), contiguous.  The library
is loaded from this package directory; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsgls.so")

TSGLS_OK = 0
TSGLS_NOT_CONVERGED = 1
JAC = {"picard": 0, "picard_nols": 1, "newton": 2}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
DT_SCHEDULE = {"fixed": 0, "ser": 1, "auto": 2}
ERRORS = {-1: "EINVAL", -2: "EHIP", -3: "ENOMEM", -4: "EMESH", -5: "ENONFINITE", -6: "ESTATE",
          -7: "ESCRATCH"}


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("omega", C.c_double), ("K", C.c_int),
                ("C_I", C.c_double), ("backflow_beta", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("lin_rtol", C.c_double), ("restart", C.c_int),
                ("max_newton", C.c_int), ("max_matvec", C.c_int), ("jacobian", C.c_int),
                ("dt_pseudo", C.c_double), ("verbose", C.c_int), ("tangent_precision", C.c_int),
                ("gmres_graph", C.c_int), ("dt_schedule", C.c_int), ("dt_max", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("newton_iters", C.c_int), ("matvecs", C.c_int), ("status", C.c_int),
                ("rel_residual", C.c_double), ("r0_norm", C.c_double), ("seconds", C.c_double),
                ("history", C.c_double * 64), ("rejected", C.c_int), ("switched_at", C.c_int),
                ("dt_last", C.c_double), ("lin_unconverged", C.c_int)]


class TsglsError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libtsgls.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TsglsError(f"{LIB_PATH} not found: build it with "
                             "`python -m paper_2311_09465_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        P, D, I64, I32 = C.c_void_p, C.c_double, C.c_int64, C.c_int
        L.tsgls_supported_K.argtypes = [C.POINTER(C.c_int), I32]
        L.tsgls_create.argtypes = [P, I64, P, I64, C.POINTER(Params), P, C.POINTER(P)]
        L.tsgls_set_dirichlet.argtypes = [P, P, I64]
        L.tsgls_set_neumann.argtypes = [P, P, I64, P]
        L.tsgls_residual.argtypes = [P, P, P]
        L.tsgls_linearize.argtypes = [P, P, P]
        L.tsgls_jv.argtypes = [P, P, P, I32, D]
        L.tsgls_set_tracer.argtypes = [P, P, D, I32]
        L.tsgls_jv_prec.argtypes = [P, P, P, I32, D, I32]
        L.tsgls_jacobi_diag.argtypes = [P, P, D]
        L.tsgls_get_tau.argtypes = [P, P]
        L.tsgls_solve.argtypes = [P, P, C.POINTER(SolveOpts), C.POINTER(SolveStats)]
        L.tsgls_solve_batch.argtypes = [P, P, I32, C.POINTER(SolveOpts), P, P, I32]
        L.tsgls_set_segments.argtypes = [P, I32]
        L.tsgls_solve_segments.argtypes = [P, P, C.POINTER(SolveOpts), P, P]
        L.tsgls_info.argtypes = [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]
        L.tsgls_profile.argtypes = [P, I32]
        L.tsgls_profile_get.argtypes = [P, I32, C.POINTER(I64), C.POINTER(D)]
        L.tsgls_rb_greedy.argtypes = [P, I64, I64, P, I32, P, P, P]
        L.tsgls_rb_project.argtypes = [P, I32, I64, P, I64, P, P, P]
        L.tsgls_rb_expand.argtypes = [P, I32, I64, P, P, P, P]
        L.tsgls_rb_project_noalloc.argtypes = [P, I32, I64, P, I64, P, P, P]
        L.tsgls_mlp_create.argtypes = [I32, I32, I32, I32, I32, C.c_uint64, P, C.POINTER(P)]
        L.tsgls_mlp_num_params.argtypes = [P, C.POINTER(I64)]
        L.tsgls_mlp_get_params.argtypes = [P, P, P]
        L.tsgls_mlp_set_params.argtypes = [P, P]
        L.tsgls_mlp_forward.argtypes = [P, P, I32, P]
        L.tsgls_mlp_gradient.argtypes = [P, P, P, I32, C.POINTER(C.c_float)]
        L.tsgls_mlp_adam_step.argtypes = [P, C.c_float, C.c_float, C.c_float, C.c_float]
        L.tsgls_mlp_last_error.argtypes = [P]
        L.tsgls_mlp_last_error.restype = C.c_char_p
        L.tsgls_mlp_destroy.argtypes = [P]
        L.tsgls_mlp_destroy.restype = None
        L.tsgls_last_error.argtypes = [P]
        L.tsgls_last_error.restype = C.c_char_p
        L.tsgls_destroy.argtypes = [P]
        L.tsgls_destroy.restype = None
        _lib = L
    return _lib


def supported_K():
    buf = (C.c_int * 64)()
    n = lib().tsgls_supported_K(buf, 64)
    return [buf[i] for i in range(min(n, 64))]


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _opts(rtol, lin_rtol, restart, max_newton, max_matvec, jacobian, dt_pseudo, verbose,
          tangent_precision, gmres_graph=False, dt_schedule="fixed", dt_max=0.0):
    return SolveOpts(rtol, lin_rtol, restart, max_newton, max_matvec, JAC[jacobian],
                     float(dt_pseudo or 0.0), int(verbose), PREC[tangent_precision],
                     int(bool(gmres_graph)), DT_SCHEDULE[dt_schedule], float(dt_max or 0.0))


def _stats_dict(rc, st):
    return dict(status=rc, newton_iters=st.newton_iters, matvecs=st.matvecs,
                rel_residual=st.rel_residual, r0_norm=st.r0_norm, seconds=st.seconds,
                history=list(st.history[:min(64, st.newton_iters)]), rejected=st.rejected,
                switched_at=st.switched_at, dt_last=st.dt_last, lin_unconverged=st.lin_unconverged)


def solve_batch(solvers, ys, rtol=1e-8, lin_rtol=0.05, restart=100, max_newton=50,
                max_matvec=10000, jacobian="picard", dt_pseudo=0.0, verbose=False,
                tangent_precision="f64", max_concurrent=8, gmres_graph=False,
                dt_schedule="fixed", dt_max=0.0):
    """tsgls_solve_batch: solve every (solver, y) pair with the same options,
    up to max_concurrent at a time.  Returns (status, per-solve stats dicts,
    per-solve finish times in seconds from the call's start)."""
    nb = len(solvers)
    if nb != len(ys):
        raise TsglsError("solve_batch: one state per solver")
    hs = (C.c_void_p * max(nb, 1))(*[s._h.value for s in solvers])
    yp = (C.c_void_p * max(nb, 1))(*[s._vec(y, "y").value for s, y in zip(solvers, ys)])
    o = _opts(rtol, lin_rtol, restart, max_newton, max_matvec, jacobian, dt_pseudo, verbose,
              tangent_precision, gmres_graph, dt_schedule, dt_max)
    st = (SolveStats * max(nb, 1))()
    fin = (C.c_double * max(nb, 1))()
    rc = lib().tsgls_solve_batch(hs, yp, nb, C.byref(o), C.cast(st, C.c_void_p),
                                 C.cast(fin, C.c_void_p), int(max_concurrent))
    if rc < 0:
        msgs = [lib().tsgls_last_error(s._h).decode() for s in solvers]
        raise TsglsError(f"solve_batch: {ERRORS.get(rc, rc)}: " + "; ".join(m for m in msgs if m))
    return rc, [_stats_dict(0 if st[i].status == 0 else 1, st[i]) for i in range(nb)], \
        [fin[i] for i in range(nb)]


class Solver:
    """One mesh on the current GPU.  Mirrors the C ABI one call to one call."""

    def __init__(self, xyz, tets, K, rho, mu, omega, C_I=3.0, backflow_beta=0.5, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise TsglsError("no GPU visible: the library runs on MI355X only")
        self.K = int(K)
        self.n_nodes = int(xyz.shape[0])
        self.n_tets = int(tets.shape[0])
        self.shape = (self.n_nodes, 4, 2 * self.K + 2)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        p = Params(rho, mu, omega, self.K, C_I, backflow_beta)
        xa, xp = _host(xyz, np.float64)
        ta, tp = _host(tets, np.int32)
        h = C.c_void_p()
        rc = lib().tsgls_create(xp, self.n_nodes, tp, self.n_tets, C.byref(p),
                                C.c_void_p(self._stream.cuda_stream), C.byref(h))
        self._h = h
        if rc != TSGLS_OK:
            msg = lib().tsgls_last_error(h).decode() if h.value else ""
            if h.value:
                lib().tsgls_destroy(h)
            self._h = C.c_void_p()
            raise TsglsError(f"tsgls_create: {ERRORS.get(rc, rc)}: {msg}")

    @classmethod
    def from_problem(cls, prob, **kw):
        s = cls(prob.mesh.xyz, prob.mesh.tets, prob.K, prob.rho, prob.mu, prob.omega,
                prob.C_I, prob.backflow_beta, **kw)
        s.set_dirichlet(prob.dirichlet_nodes)
        s.set_neumann(prob.neumann_tris, prob.neumann_h)
        return s

    def _check(self, rc, what):
        if rc < 0:
            raise TsglsError(f"{what}: {ERRORS.get(rc, rc)}: {lib().tsgls_last_error(self._h).decode()}")
        return rc

    def _vec(self, t, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise TsglsError(f"{name} must be a contiguous float64 CUDA tensor of shape {self.shape}")
        return _ptr(t)

    def set_dirichlet(self, nodes):
        a, p = _host(nodes, np.int32)
        self._check(lib().tsgls_set_dirichlet(self._h, p, a.size), "set_dirichlet")

    def set_neumann(self, tris, h=None):
        a, p = _host(np.asarray(tris).reshape(-1, 3), np.int32)
        hp = None
        if h is not None:
            ha, hp = _host(h, np.float64)
        self._check(lib().tsgls_set_neumann(self._h, p, a.shape[0], hp), "set_neumann")

    def set_tracer(self, y_velocity, kappa, stabilized=True):
        """Switch to the tracer (convection-diffusion) equation carried by the
        velocity of y_velocity (tsgls_set_tracer)."""
        self._check(lib().tsgls_set_tracer(self._h, self._vec(y_velocity, "y_velocity"), float(kappa),
                                           int(bool(stabilized))), "set_tracer")

    def residual(self, y, r):
        self._check(lib().tsgls_residual(self._h, self._vec(y, "y"), self._vec(r, "r")), "residual")

    def linearize(self, y, r=None):
        rp = self._vec(r, "r") if r is not None else None
        self._check(lib().tsgls_linearize(self._h, self._vec(y, "y"), rp), "linearize")

    def jv(self, v, out, jacobian="picard", dt_pseudo=0.0, precision=None):
        if precision is None:
            self._check(lib().tsgls_jv(self._h, self._vec(v, "v"), self._vec(out, "Jv"),
                                       JAC[jacobian], float(dt_pseudo or 0.0)), "jv")
        else:
            self._check(lib().tsgls_jv_prec(self._h, self._vec(v, "v"), self._vec(out, "Jv"),
                                            JAC[jacobian], float(dt_pseudo or 0.0), PREC[precision]),
                        "jv_prec")

    def jacobi_diag(self, d, dt_pseudo=0.0):
        self._check(lib().tsgls_jacobi_diag(self._h, self._vec(d, "d"), float(dt_pseudo or 0.0)),
                    "jacobi_diag")

    def get_tau(self):
        n = 2 * self.K + 1
        out = np.empty((self.n_tets, 4, n * (n + 1) // 2))
        self._check(lib().tsgls_get_tau(self._h, out.ctypes.data_as(C.c_void_p)), "get_tau")
        return out

    def solve(self, y, rtol=1e-8, lin_rtol=0.05, restart=100, max_newton=50, max_matvec=10000,
              jacobian="picard", dt_pseudo=0.0, verbose=False, tangent_precision="f64",
              gmres_graph=False, dt_schedule="fixed", dt_max=0.0):
        o = _opts(rtol, lin_rtol, restart, max_newton, max_matvec, jacobian, dt_pseudo, verbose,
                  tangent_precision, gmres_graph, dt_schedule, dt_max)
        st = SolveStats()
        rc = self._check(lib().tsgls_solve(self._h, self._vec(y, "y"), C.byref(o), C.byref(st)), "solve")
        return _stats_dict(rc, st)

    def set_segments(self, nseg):
        """tsgls_set_segments: the context holds nseg independent problems,
        node blocks of n_nodes / nseg."""
        self._check(lib().tsgls_set_segments(self._h, int(nseg)), "set_segments")
        self.nseg = int(nseg)

    def solve_segments(self, y, rtol=1e-8, lin_rtol=0.05, restart=30, max_newton=50, max_matvec=10000,
                       jacobian="picard", dt_pseudo=0.0, verbose=False, tangent_precision="f64"):
        """tsgls_solve_segments: lockstep Newton-GMRES on every segment.
        Returns (status, per-segment stats dicts, per-segment finish times)."""
        nseg = getattr(self, "nseg", 1)
        o = _opts(rtol, lin_rtol, restart, max_newton, max_matvec, jacobian, dt_pseudo, verbose,
                  tangent_precision, True, "fixed", 0.0)
        st = (SolveStats * nseg)()
        fin = (C.c_double * nseg)()
        rc = self._check(lib().tsgls_solve_segments(self._h, self._vec(y, "y"), C.byref(o),
                                                    C.cast(st, C.c_void_p), C.cast(fin, C.c_void_p)),
                         "solve_segments")
        return rc, [_stats_dict(0 if st[i].status == 0 else 1, st[i]) for i in range(nseg)], \
            [fin[i] for i in range(nseg)]

    PROF = {"elem_tangent": 0, "elem_residual": 1, "tau": 2, "diag": 3, "face": 4, "ortho": 5,
            "gather": 6}

    def profile(self, enable):
        self._check(lib().tsgls_profile(self._h, int(bool(enable))), "profile")

    def profile_get(self, which):
        n, ms = C.c_int64(), C.c_double()
        self._check(lib().tsgls_profile_get(self._h, self.PROF[which], C.byref(n), C.byref(ms)),
                    "profile_get")
        return n.value, ms.value

    def info(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self._check(lib().tsgls_info(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)), "info")
        return dict(n_colors=a.value, n_tets=b.value, n_nodes=c.value, device_bytes=d.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tsgls_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SegmentSolver(Solver):
    """Problems that share a mesh, a harmonic count and the physical
    parameters and differ in their Dirichlet data (e.g. inflow waveforms),
    held as the segments of one context: the mesh repeated once per problem
    with node numbers offset by s n_nodes.  State tensors have shape
    (nseg * n_nodes, 4, 2K+2); problem s is rows [s n_nodes, (s+1) n_nodes)."""

    @classmethod
    def from_problems(cls, probs, stream=None):
        p0 = probs[0]
        nn = p0.mesh.n_nodes
        for p in probs[1:]:
            same = (p.K == p0.K and p.rho == p0.rho and p.mu == p0.mu and p.omega == p0.omega
                    and p.C_I == p0.C_I and p.backflow_beta == p0.backflow_beta
                    and np.array_equal(p.mesh.xyz, p0.mesh.xyz) and np.array_equal(p.mesh.tets, p0.mesh.tets)
                    and np.array_equal(p.dirichlet_nodes, p0.dirichlet_nodes)
                    and np.array_equal(p.neumann_tris, p0.neumann_tris)
                    and p.neumann_h is None and p0.neumann_h is None)
            if not same:
                raise TsglsError("segments need one mesh, K, parameters, Dirichlet node set and "
                                 "Neumann faces (without traction)")
        B = len(probs)
        tets = np.asarray(p0.mesh.tets, dtype=np.int64)
        xyz = np.tile(np.asarray(p0.mesh.xyz, dtype=np.float64), (B, 1))
        utets = np.concatenate([tets + s * nn for s in range(B)])
        s = cls(xyz, utets, p0.K, p0.rho, p0.mu, p0.omega, p0.C_I, p0.backflow_beta, stream=stream)
        dn = np.asarray(p0.dirichlet_nodes, dtype=np.int64)
        s.set_dirichlet(np.concatenate([dn + k * nn for k in range(B)]))
        nt = np.asarray(p0.neumann_tris, dtype=np.int64).reshape(-1, 3)
        s.set_neumann(np.concatenate([nt + k * nn for k in range(B)]))
        s.set_segments(B)
        s.seg_nodes = nn
        return s


# ---------------------------------------------------------------- warm start
def _dev(t, dtype, name, ndim=None):
    import torch
    want = {"f64": torch.float64, "f32": torch.float32}[dtype]
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == want and t.is_contiguous()
            and (ndim is None or t.dim() == ndim)):
        raise TsglsError(f"{name} must be a contiguous {want} CUDA tensor"
                         + (f" with {ndim} dimensions" if ndim else ""))
    return _ptr(t)


def _cur_stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def rb_greedy(Y, mean, r, stream=None):
    """tsgls_rb_greedy on snapshot rows Y [N][D] (float64 CUDA); returns the
    orthonormal basis rows Phi [k][D] (k <= r) and the picked snapshot
    indices."""
    import torch
    N, D = Y.shape
    Phi = torch.zeros((r, D), dtype=torch.float64, device=Y.device)
    picked = (C.c_int32 * r)()
    k = lib().tsgls_rb_greedy(_dev(Y, "f64", "Y", 2), N, D, _dev(mean, "f64", "mean"), int(r),
                              _ptr(Phi), C.cast(picked, C.c_void_p), _cur_stream(stream))
    if k < 0:
        raise TsglsError(f"rb_greedy: {ERRORS.get(k, k)}")
    return Phi[:k].contiguous(), [picked[i] for i in range(k)]


def rb_project(Phi, Y, mean, stream=None):
    """coef [N][r] = Phi (Y_i - mean) (tsgls_rb_project)."""
    import torch
    r, D = Phi.shape
    N = Y.shape[0]
    coef = torch.zeros((N, r), dtype=torch.float64, device=Y.device)
    rc = lib().tsgls_rb_project(_dev(Phi, "f64", "Phi", 2), r, D, _dev(Y, "f64", "Y"), N,
                                _dev(mean, "f64", "mean"), _ptr(coef), _cur_stream(stream))
    if rc < 0:
        raise TsglsError(f"rb_project: {ERRORS.get(rc, rc)}")
    return coef


def rb_project_noalloc(Phi, Y, mean, coef, stream=None):
    """coef [N][r] = Phi (Y_i - mean) into the caller's coef, with no device
    allocation (tsgls_rb_project_noalloc; calls on one GPU must not overlap)."""
    r, D = Phi.shape
    N = Y.shape[0]
    if tuple(coef.shape) != (N, r):
        raise TsglsError("rb_project_noalloc: coef must be [N][r]")
    rc = lib().tsgls_rb_project_noalloc(_dev(Phi, "f64", "Phi", 2), r, D, _dev(Y, "f64", "Y"), N,
                                        _dev(mean, "f64", "mean"), _dev(coef, "f64", "coef"),
                                        _cur_stream(stream))
    if rc < 0:
        raise TsglsError(f"rb_project_noalloc: {ERRORS.get(rc, rc)}")


def rb_expand(Phi, coef, mean, out, stream=None):
    """out = mean + Phi^T coef (tsgls_rb_expand); coef float64 CUDA [r]."""
    r, D = Phi.shape
    rc = lib().tsgls_rb_expand(_dev(Phi, "f64", "Phi", 2), r, D, _dev(coef, "f64", "coef"),
                               _dev(mean, "f64", "mean"), _dev(out, "f64", "out"),
                               _cur_stream(stream))
    if rc < 0:
        raise TsglsError(f"rb_expand: {ERRORS.get(rc, rc)}")


class MLP:
    """tsgls_mlp_*: tanh network n_in -> n_hidden x width -> n_out; bf16 MFMA
    products with FP32 master weights (precision "bf16") or FP32 ("f32")."""

    def __init__(self, n_in, width, n_hidden, n_out, precision="bf16", seed=0, stream=None):
        self.dims = [int(n_in)] + [int(width)] * int(n_hidden) + [int(n_out)]
        self._stream = stream
        h = C.c_void_p()
        rc = lib().tsgls_mlp_create(int(n_in), int(width), int(n_hidden), int(n_out),
                                    {"bf16": 0, "f32": 1}[precision], int(seed),
                                    _cur_stream(stream), C.byref(h))
        self._h = h
        if rc != TSGLS_OK:
            if h.value:
                lib().tsgls_mlp_destroy(h)
            self._h = C.c_void_p()
            raise TsglsError(f"tsgls_mlp_create: {ERRORS.get(rc, rc)}")
        n = C.c_int64()
        lib().tsgls_mlp_num_params(h, C.byref(n))
        self.n_params = n.value

    def _check(self, rc, what):
        if rc < 0:
            raise TsglsError(f"{what}: {ERRORS.get(rc, rc)}: {lib().tsgls_mlp_last_error(self._h).decode()}")

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(lib().tsgls_mlp_get_params(self._h, out.ctypes.data_as(C.c_void_p), None),
                    "get_params")
        return out

    def get_grad(self):
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(lib().tsgls_mlp_get_params(self._h, None, out.ctypes.data_as(C.c_void_p)),
                    "get_grad")
        return out

    def set_params(self, theta):
        a, p = _host(theta, np.float32)
        if a.size != self.n_params:
            raise TsglsError("set_params: wrong parameter count")
        self._check(lib().tsgls_mlp_set_params(self._h, p), "set_params")

    def _shapes(self, x, y, what):
        if x.dim() != 2 or x.shape[1] != self.dims[0] or tuple(y.shape) != (x.shape[0], self.dims[-1]):
            raise TsglsError(f"{what}: x must be [B][{self.dims[0]}] and the output [B][{self.dims[-1]}]")

    def forward(self, x, y):
        self._shapes(x, y, "forward")
        self._check(lib().tsgls_mlp_forward(self._h, _dev(x, "f32", "x", 2), int(x.shape[0]),
                                            _dev(y, "f32", "y", 2)), "forward")

    def gradient(self, x, t):
        self._shapes(x, t, "gradient")
        loss = C.c_float()
        self._check(lib().tsgls_mlp_gradient(self._h, _dev(x, "f32", "x", 2), _dev(t, "f32", "t", 2),
                                             int(x.shape[0]), C.byref(loss)), "gradient")
        return loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(lib().tsgls_mlp_adam_step(self._h, float(lr), float(beta1), float(beta2),
                                              float(eps)), "adam_step")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tsgls_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

