"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Tolerances: tau, residual and tangent products to
1e-11 relative (L2 and max-norm) -- both sides are FP64 with different
summation orders and eigensolvers (LAPACK Hermitian vs one-sided Jacobi);
solve cross-evaluated by the oracle residual to 1e-8 of the initial residual.
"""
import numpy as np
import pytest

import oracle as O
from workloads import cube_problem, womersley_problem, junction_problem, tiny_problem
from tests.gpu_helpers import (log, to_dev, to_host, rand_state, rand_dir, tau_complex_to_real,
                               unpack, rel_err)

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _solver(prob):
    import paper_2311_09465_amd as T
    return T.Solver.from_problem(prob)


def _case(name):
    if name == "cube3_K0":
        return cube_problem(3, K=0)
    if name == "cube3_K1":
        return cube_problem(3, K=1)
    if name == "cube3_K2":
        return cube_problem(3, K=2)
    if name == "cube4_K3":
        return cube_problem(4, K=3)
    if name == "cube3_K6":
        return cube_problem(3, K=6)
    if name == "pipe_K3":
        return womersley_problem(2, 8, K=3)
    if name == "junction_K3":
        return junction_problem(h=0.35, K=3)
    if name == "tiny1_K2":
        return tiny_problem(1, K=2)
    if name == "cube2_K7":
        return cube_problem(2, K=7)
    if name == "cube2_K11":
        return cube_problem(2, K=11)
    raise KeyError(name)


CASES = ["tiny1_K2", "cube3_K0", "cube3_K1", "cube3_K2", "cube4_K3", "cube3_K6", "pipe_K3",
         "junction_K3", "cube2_K7", "cube2_K11"]


@pytest.mark.parametrize("name", CASES)
def test_tau_parity(name):
    log(f"[gpu] tau parity {name}")
    prob = _case(name)
    s = _solver(prob)
    y = rand_state(prob, 1)
    s.linearize(to_dev(y))
    tg = unpack(s.get_tau(), 2 * prob.K + 1)
    lin = O.linearize(O.Params.from_problem(prob), prob.mesh.xyz, prob.mesh.tets, y)
    tr = tau_complex_to_real(lin["tau"], prob.K)
    assert np.abs(tg - tr).max() <= TOL * np.abs(tr).max()
    assert rel_err(tg, tr) <= TOL


@pytest.mark.parametrize("name", CASES)
def test_residual_parity(name):
    log(f"[gpu] residual parity {name}")
    prob = _case(name)
    if name == "cube4_K3":
        rng = np.random.default_rng(5)
        h = rng.standard_normal((len(prob.neumann_tris), 2 * prob.K + 2))
        h[:, 1] = 0
        prob.neumann_h = h
    s = _solver(prob)
    y = rand_state(prob, 2)
    r = to_dev(np.zeros_like(y))
    s.residual(to_dev(y), r)
    rg = to_host(r)
    rr = O.residual(O.Params.from_problem(prob), prob.mesh.xyz, prob.mesh.tets, y)
    assert np.abs(rg - rr).max() <= TOL * np.abs(rr).max()
    assert rel_err(rg, rr) <= TOL
    # linearize gives the same residual as a by-product
    r2 = to_dev(np.zeros_like(y))
    s.linearize(to_dev(y), r2)
    assert np.abs(to_host(r2) - rr).max() <= TOL * np.abs(rr).max()


@pytest.mark.parametrize("name", ["tiny1_K2", "cube3_K1", "cube4_K3", "cube3_K6", "junction_K3", "cube2_K11"])
@pytest.mark.parametrize("variant", ["picard", "picard_nols", "newton"])
@pytest.mark.parametrize("dt", [0.0, 0.7])
def test_jv_parity(name, variant, dt):
    log(f"[gpu] jv parity {name} {variant} dt={dt}")
    prob = _case(name)
    s = _solver(prob)
    y = rand_state(prob, 3)
    v = rand_dir(prob, 4)
    s.linearize(to_dev(y))
    out = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out, variant, dt)
    jg = to_host(out)
    par = O.Params.from_problem(prob)
    lin = O.linearize(par, prob.mesh.xyz, prob.mesh.tets, y)
    jr = O.jv(par, prob.mesh.xyz, prob.mesh.tets, lin, v, variant, dt if dt > 0 else None)
    assert np.abs(jg - jr).max() <= TOL * np.abs(jr).max()
    assert rel_err(jg, jr) <= TOL


@pytest.mark.parametrize("name", ["tiny1_K2", "cube3_K2", "cube4_K3", "junction_K3"])
@pytest.mark.parametrize("dt", [0.0, 0.5])
def test_jacobi_diag_parity(name, dt):
    log(f"[gpu] diag parity {name} dt={dt}")
    prob = _case(name)
    s = _solver(prob)
    y = rand_state(prob, 6)
    s.linearize(to_dev(y))
    d = to_dev(np.zeros_like(y))
    s.jacobi_diag(d, dt)
    dg = to_host(d)
    par = O.Params.from_problem(prob)
    lin = O.linearize(par, prob.mesh.xyz, prob.mesh.tets, y)
    dr = O.jacobian_diagonal(par, prob.mesh.xyz, prob.mesh.tets, lin, dt if dt > 0 else None)
    assert np.abs(dg - dr).max() <= TOL * np.abs(dr).max()


def test_residual_bitwise_deterministic():
    log("[gpu] determinism")
    prob = _case("junction_K3")
    s = _solver(prob)
    y = to_dev(rand_state(prob, 7))
    a = to_dev(np.zeros(s.shape))
    b = to_dev(np.zeros(s.shape))
    s.residual(y, a)
    s.residual(y, b)
    assert np.array_equal(to_host(a), to_host(b))


@pytest.mark.parametrize("restart", [150, 100, 20])
@pytest.mark.parametrize("jac", ["picard", "newton"])
def test_solve_cross_evaluated_by_oracle(jac, restart):
    """Picard: one solve to 1e-9.  Newton: Picard to 1e-3, then the Newton
    tangent (tau frozen) from there; both judged by the oracle residual.
    restart 150 runs GMRES with two-pass classical Gram-Schmidt; restarts
    100 and 20 the delayed variant (one reduction per Arnoldi step; at 100
    its reduction spans four tiles of basis vectors)."""
    log(f"[gpu] solve cross-evaluation {jac} restart={restart}")
    from workloads import initial_guess
    prob = womersley_problem(2, 8, K=2)
    s = _solver(prob)
    y0 = initial_guess(prob)
    y = to_dev(y0)
    if jac == "picard":
        st = s.solve(y, rtol=1e-9, jacobian="picard", max_newton=60, restart=restart)
        assert st["status"] == 0, st
    else:
        st1 = s.solve(y, rtol=1e-3, jacobian="picard", max_newton=60, restart=restart)
        assert st1["status"] == 0, st1
        target = 1e-9 / st1["rel_residual"]
        st = s.solve(y, rtol=target, jacobian="newton", max_newton=30, restart=restart)
        assert st["status"] == 0, st
    yg = to_host(y)
    par = O.Params.from_problem(prob)
    r0 = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, y0))
    r = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, yg))
    assert r <= 1e-8 * r0, (r / r0, st)


def test_error_codes():
    log("[gpu] error codes")
    import torch
    import paper_2311_09465_amd as T
    prob = tiny_problem(2, K=1)
    bad = prob.mesh.tets.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]
    with pytest.raises(T.TsglsError, match="EMESH"):
        T.Solver(prob.mesh.xyz, bad, 1, 1.0, 0.1, 1.0)
    with pytest.raises(T.TsglsError, match="EINVAL"):
        T.Solver(prob.mesh.xyz, prob.mesh.tets, 9, 1.0, 0.1, 1.0)
    with pytest.raises(T.TsglsError, match="EINVAL"):
        T.Solver(prob.mesh.xyz, prob.mesh.tets, 1, 1.0, -0.1, 1.0)
    s = _solver(prob)
    z = torch.zeros(s.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(T.TsglsError, match="ESTATE"):
        s.jv(z, torch.zeros_like(z))
    y = rand_state(prob, 1)
    y[0, 3, 0] = np.nan
    with pytest.raises(T.TsglsError, match="ENONFINITE"):
        s.solve(to_dev(y))
    st = s.solve(to_dev(rand_state(prob, 1)), max_newton=1, rtol=1e-14)
    assert st["status"] == 1 and st["newton_iters"] == 1


@pytest.mark.parametrize("name", ["cube3_K1", "cube4_K3", "cube3_K6", "junction_K3", "cube2_K11"])
def test_tau_warm_start_parity(name):
    """tau's Jacobi iteration starts from the eigenvectors of the previous
    linearization: linearize at y1, then at y2 (warm start from y1's basis),
    then at y2 again (from its own basis); tau and the residual of each match
    the oracle at that state, and a residual evaluation between them (which
    reads the stored basis) does too."""
    log(f"[gpu] tau warm start {name}")
    prob = _case(name)
    s = _solver(prob)
    par = O.Params.from_problem(prob)
    xyz, tets = prob.mesh.xyz, prob.mesh.tets
    y1 = rand_state(prob, 21)
    y2 = y1 + 0.05 * rand_state(prob, 22)
    y2[..., 1] = 0.0
    y2[prob.dirichlet_nodes, :3] = prob.dirichlet_values
    r = to_dev(np.zeros_like(y1))
    for y in (y1, y2, y2):
        s.linearize(to_dev(y), r)
        tg = unpack(s.get_tau(), 2 * prob.K + 1)
        tr = tau_complex_to_real(O.linearize(par, xyz, tets, y)["tau"], prob.K)
        rr = O.residual(par, xyz, tets, y)
        et = np.abs(tg - tr).max() / np.abs(tr).max()
        er = np.abs(to_host(r) - rr).max() / np.abs(rr).max()
        s.residual(to_dev(y1), r)
        er1 = np.abs(to_host(r) - O.residual(par, xyz, tets, y1)).max() / np.abs(rr).max()
        log(f"[gpu]   tau {et:.2e} residual {er:.2e} residual(y1) {er1:.2e}")
        assert et <= TOL and er <= TOL and er1 <= TOL
