"""GPU parity of the mixed-precision tangent: the element operator in FP32
(FP32 MFMA transforms, FP32 copies of tau, of the frozen velocity samples and
of tau L(u)), its element rows summed per node in FP64, against the FP64
oracle on the same seeded inputs.

Tolerance.  Every entry of an element row is formed from O(10^2) FP32
operations on operands rounded once to FP32 (unit roundoff u = 2^-24 =
6.0e-8).  The errors are largely independent, so an element row carries a
relative error of a few u; the node sum (FP64) adds rows of both signs, so
relative to the largest entry of J v that error is scaled by
max|element row| / max|J v|, of order one on these meshes.  Measured: 0.5 u
to 3.7 u (max-norm) over K = 0 .. 15 and the three variants.  TOL32 = 16 u =
1e-6 (max-norm relative to the largest entry, and L2-relative); the measured
errors are printed per case.

The solve test runs Newton-GMRES with the FP32 tangent and judges the result
with the oracle's FP64 residual: the FP64 residual of each Newton step
corrects the rounding of the inner solves, so the same 1e-8 target as the
FP64 solve is reached.
"""
import numpy as np
import pytest

import oracle as O
from workloads import cube_problem, womersley_problem, junction_problem, tiny_problem
from tests.gpu_helpers import log, to_dev, to_host, rand_state, rand_dir, rel_err

pytestmark = pytest.mark.gpu

TOL32 = 1e-6


def _case(name):
    return {
        "tiny1_K2": lambda: tiny_problem(1, K=2),
        "cube3_K0": lambda: cube_problem(3, K=0),
        "cube3_K1": lambda: cube_problem(3, K=1),
        "cube4_K3": lambda: cube_problem(4, K=3),
        "cube3_K6": lambda: cube_problem(3, K=6),
        "junction_K3": lambda: junction_problem(h=0.35, K=3),
        "cube2_K7": lambda: cube_problem(2, K=7),
        "cube2_K11": lambda: cube_problem(2, K=11),
        "cube2_K15": lambda: cube_problem(2, K=15),
    }[name]()


def _solver(prob):
    import paper_2311_09465_amd as T
    return T.Solver.from_problem(prob)


def _oracle_jv(prob, y, v, variant, dt):
    par = O.Params.from_problem(prob)
    lin = O.linearize(par, prob.mesh.xyz, prob.mesh.tets, y)
    return O.jv(par, prob.mesh.xyz, prob.mesh.tets, lin, v, variant, dt if dt > 0 else None)


def _errs(g, r):
    return np.abs(g - r).max() / np.abs(r).max(), rel_err(g, r)


@pytest.mark.parametrize("name", ["tiny1_K2", "cube3_K0", "cube3_K1", "cube4_K3", "cube3_K6",
                                  "junction_K3", "cube2_K7", "cube2_K11", "cube2_K15"])
@pytest.mark.parametrize("variant", ["picard", "picard_nols", "newton"])
@pytest.mark.parametrize("dt", [0.0, 0.7])
def test_jv_f32_parity(name, variant, dt):
    log(f"[gpu] jv f32 parity {name} {variant} dt={dt}")
    prob = _case(name)
    s = _solver(prob)
    y = rand_state(prob, 3)
    v = rand_dir(prob, 4)
    s.linearize(to_dev(y))
    out = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out, variant, dt, precision="f32")
    jg = to_host(out)
    jr = _oracle_jv(prob, y, v, variant, dt)
    emax, el2 = _errs(jg, jr)
    log(f"[gpu]   K={prob.K} max-rel {emax:.2e} l2-rel {el2:.2e}")
    assert emax <= TOL32
    assert el2 <= TOL32
    # the FP64 product of the same call sequence is unchanged by the FP32 one
    out64 = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out64, variant, dt, precision="f64")
    j64 = to_host(out64)
    assert np.abs(j64 - jr).max() <= 1e-11 * np.abs(jr).max()


def test_jv_f32_follows_relinearization():
    """The FP32 copies are refreshed after every linearize."""
    log("[gpu] jv f32 after relinearization")
    prob = _case("cube4_K3")
    s = _solver(prob)
    y1, y2 = rand_state(prob, 11), rand_state(prob, 12)
    v = rand_dir(prob, 13)
    out = to_dev(np.zeros_like(y1))
    s.linearize(to_dev(y1))
    s.jv(to_dev(v), out, "picard", 0.0, precision="f32")
    s.linearize(to_dev(y2))
    s.jv(to_dev(v), out, "newton", 0.0, precision="f32")
    jr = _oracle_jv(prob, y2, v, "newton", 0.0)
    emax, el2 = _errs(to_host(out), jr)
    assert emax <= TOL32 and el2 <= TOL32


@pytest.mark.parametrize("restart", [150, 100, 20])
def test_solve_f32_tangent_cross_evaluated_by_oracle(restart):
    log(f"[gpu] solve with FP32 tangent restart={restart}")
    from workloads import initial_guess
    prob = womersley_problem(2, 8, K=2)
    s = _solver(prob)
    y0 = initial_guess(prob)
    y = to_dev(y0)
    st = s.solve(y, rtol=1e-9, jacobian="picard", max_newton=60, restart=restart,
                 tangent_precision="f32")
    assert st["status"] == 0, st
    yg = to_host(y)
    par = O.Params.from_problem(prob)
    r0 = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, y0))
    r = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, yg))
    log(f"[gpu]   newton {st['newton_iters']} matvecs {st['matvecs']} oracle rel {r / r0:.2e}")
    assert r <= 1e-8 * r0, (r / r0, st)


def test_jv_prec_rejects_bad_precision():
    import ctypes as C
    import paper_2311_09465_amd as T
    prob = _case("tiny1_K2")
    s = _solver(prob)
    y = to_dev(rand_state(prob, 1))
    s.linearize(y)
    out = to_dev(np.zeros(s.shape))
    rc = T.lib().tsgls_jv_prec(s._h, C.c_void_p(y.data_ptr()), C.c_void_p(out.data_ptr()), 0,
                               C.c_double(0.0), 7)
    assert rc == -1


# --------------------------------------------------------------- bf16 tau
# TSGLS_PREC_BF16: the FP32 operator with tau stored and applied in bf16
# (unit roundoff u_b = 2^-8 = 3.9e-3).  Only the least-squares and PSPG terms
# see tau: z = tau L carries an error of at most u_b sum_k |tau_pk L_k| per
# entry, and relative to the largest entry of J v that is a few u_b at most
# (the Galerkin terms dilute it).  TOLB = 2 u_b = 7.8e-3, max-norm and L2,
# relative to the largest entry; measured errors are printed per case.
TOLB = 2.0 * 2.0 ** -8


@pytest.mark.parametrize("name", ["tiny1_K2", "cube3_K1", "cube4_K3", "cube3_K6", "junction_K3",
                                  "cube2_K7", "cube2_K11", "cube2_K15", "cube2_K31"])
@pytest.mark.parametrize("variant", ["picard", "picard_nols", "newton"])
def test_jv_bf16_tau_parity(name, variant):
    log(f"[gpu] jv bf16-tau parity {name} {variant}")
    prob = cube_problem(2, K=31) if name == "cube2_K31" else _case(name)
    s = _solver(prob)
    y = rand_state(prob, 3, 0.5 if prob.K == 31 else 1.0)
    v = rand_dir(prob, 4)
    s.linearize(to_dev(y))
    out = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out, variant, 0.0, precision="bf16")
    jg = to_host(out)
    jr = _oracle_jv(prob, y, v, variant, 0.0)
    emax, el2 = _errs(jg, jr)
    log(f"[gpu]   K={prob.K} max-rel {emax:.2e} = {emax / 2.0 ** -8:.2f} u_b, l2-rel {el2:.2e}")
    assert emax <= TOLB and el2 <= TOLB
    # the FP32 product afterwards still reads the FP32 tau
    s.jv(to_dev(v), out, variant, 0.0, precision="f32")
    e32, _ = _errs(to_host(out), jr)
    assert e32 <= TOL32


def test_solve_bf16_tau_cross_evaluated_by_oracle():
    """The bf16 tangent inside Newton-GMRES: the FP64 residual of every
    Newton step corrects the 1e-3 error of the products, so the solution
    reaches the same 1e-8 target, judged by the oracle's residual."""
    log("[gpu] solve with bf16-tau tangent")
    from workloads import initial_guess
    prob = womersley_problem(2, 8, K=2)
    s = _solver(prob)
    y0 = initial_guess(prob)
    y = to_dev(y0)
    st = s.solve(y, rtol=1e-9, jacobian="picard", max_newton=60, restart=100,
                 tangent_precision="bf16")
    assert st["status"] == 0, st
    yg = to_host(y)
    par = O.Params.from_problem(prob)
    r0 = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, y0))
    r = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, yg))
    log(f"[gpu]   newton {st['newton_iters']} matvecs {st['matvecs']} oracle rel {r / r0:.2e}")
    assert r <= 1e-8 * r0, (r / r0, st)
