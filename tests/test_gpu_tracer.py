"""Tracer (time-spectral GLS convection-diffusion, eq. 3D-weak) on the GPU
against the oracle's assembled operator (oracle/cd.py), with the velocity of
a Navier-Stokes state frozen; stabilized and Galerkin (tau = 0) forms.
Tolerance 1e-11 of the largest entry, as for the Navier-Stokes operator (same
arithmetic, FP64, different summation order and eigensolver for tau)."""
import numpy as np
import pytest

from oracle import cd as OC
from oracle.tsref import QP_BARY, slots_to_modes, modes_to_slots
from workloads import womersley_problem, initial_guess
from tests.gpu_helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _nodes(tris):
    return np.unique(np.asarray(tris).ravel())


def _setup(K, stabilized, kappa=0.01, seed=0, solved_velocity=False):
    """Tracer context on the 2x8 pipe.  Velocity: the Navier-Stokes initial
    guess plus seeded noise (parity), or the converged Navier-Stokes solution
    (solves)."""
    import torch
    import paper_2311_09465_amd as T
    prob = womersley_problem(2, 8, K=K)
    rng = np.random.default_rng(seed)
    yv = initial_guess(prob)
    wall = _nodes(prob.mesh.faces["wall"])
    if solved_velocity:
        ns = T.Solver.from_problem(prob)
        yd = to_dev(yv)
        assert ns.solve(yd, rtol=1e-8, restart=30)["status"] == 0
        yv = to_host(yd)
    else:
        free = np.setdiff1d(np.arange(prob.mesh.n_nodes), prob.dirichlet_nodes)
        yv[free, :3] += 0.2 * rng.standard_normal((free.size, 3, 2 * K + 2))
        yv[..., 1] = 0.0
    dn = np.union1d(_nodes(prob.mesh.faces["inlet"]), _nodes(prob.mesh.faces["outlet"]))
    dn = np.setdiff1d(dn, wall)
    s = T.Solver(prob.mesh.xyz, prob.mesh.tets, K, prob.rho, prob.mu, prob.omega)
    s.set_dirichlet(dn.astype(np.int32))
    s.set_tracer(to_dev(yv), kappa, stabilized)
    torch.cuda.synchronize()
    # oracle operator on complex modes
    C = slots_to_modes(yv[:, :3, :], K)
    uq = np.einsum("qb,ebjn->eqjn", QP_BARY, C[prob.mesh.tets])
    B, _, _, _ = OC.element_matrices(prob.mesh.xyz, prob.mesh.tets, uq, kappa, prob.omega,
                                     stabilized=stabilized)
    A = OC.assemble(prob.mesh.xyz, prob.mesh.tets, B)
    return prob, s, A, dn


def _apply(A, phi, K, dn):
    n = phi.shape[0]
    r = (A @ slots_to_modes(phi, K).ravel()).reshape(n, 2 * K + 1)
    rs = modes_to_slots(r, K)
    rs[dn] = 0.0
    return rs


@pytest.mark.parametrize("stabilized", [True, False])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_tracer_residual_and_product_match_oracle(K, stabilized):
    log(f"[gpu] tracer parity K={K} stabilized={stabilized}")
    prob, s, A, dn = _setup(K, stabilized)
    rng = np.random.default_rng(K)
    y = np.zeros((prob.mesh.n_nodes, 4, 2 * K + 2))
    y[:, 0] = rng.standard_normal((prob.mesh.n_nodes, 2 * K + 2))
    y[:, 0, 1] = 0.0
    r = to_dev(np.zeros_like(y))
    s.linearize(to_dev(y), r)
    rg = to_host(r)
    rr = _apply(A, y[:, 0], K, dn)
    assert np.abs(rg[:, 1:]).max() == 0.0
    assert np.abs(rg[:, 0] - rr).max() <= TOL * np.abs(rr).max()
    v = np.zeros_like(y)
    v[:, 0] = rng.standard_normal((prob.mesh.n_nodes, 2 * K + 2))
    v[:, 0, 1] = 0.0
    out = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out)
    jg = to_host(out)
    vm = v[:, 0].copy()
    vm[dn] = 0.0
    jr = _apply(A, vm, K, dn)
    assert np.abs(jg[:, 0] - jr).max() <= TOL * np.abs(jr).max()


@pytest.mark.parametrize("stabilized", [True, False])
def test_tracer_solve_cross_evaluated_by_oracle(stabilized):
    log(f"[gpu] tracer solve stabilized={stabilized}")
    K = 2
    prob, s, A, dn = _setup(K, stabilized, kappa=0.02, solved_velocity=True)
    y0 = np.zeros((prob.mesh.n_nodes, 4, 2 * K + 2))
    inlet = np.intersect1d(dn, _nodes(prob.mesh.faces["inlet"]))
    y0[inlet, 0, 0] = 1.0
    y = to_dev(y0)
    st = s.solve(y, rtol=1e-9, lin_rtol=1e-6, restart=100, max_newton=10, max_matvec=20000)
    assert st["status"] == 0, st
    yg = to_host(y)
    assert np.abs(yg[:, 1:]).max() == 0.0
    r0 = np.linalg.norm(_apply(A, y0[:, 0], K, dn))
    r = np.linalg.norm(_apply(A, yg[:, 0], K, dn))
    log(f"[gpu]   newton {st['newton_iters']} matvecs {st['matvecs']} oracle rel {r / r0:.2e}")
    assert r <= 1e-8 * r0


def _setup_backflow(K, stabilized, kappa=0.01, seed=0, solved_velocity=False):
    """Tracer with the pipe's inlet as a natural boundary: the flow enters
    through it, so the backflow term -(w, (beta/2)|A_n|_- phi) acts there
    (beta = 0.5); phi prescribed at the outlet (wall nodes excluded)."""
    import torch
    import paper_2311_09465_amd as T
    prob = womersley_problem(2, 8, K=K)
    rng = np.random.default_rng(seed)
    yv = initial_guess(prob)
    wall = _nodes(prob.mesh.faces["wall"])
    if solved_velocity:
        ns = T.Solver.from_problem(prob)
        yd = to_dev(yv)
        assert ns.solve(yd, rtol=1e-8, restart=30)["status"] == 0
        yv = to_host(yd)
    else:
        free = np.setdiff1d(np.arange(prob.mesh.n_nodes), prob.dirichlet_nodes)
        yv[free, :3] += 0.2 * rng.standard_normal((free.size, 3, 2 * K + 2))
        yv[..., 1] = 0.0
    dn = np.setdiff1d(_nodes(prob.mesh.faces["outlet"]), wall)
    inlet = np.asarray(prob.mesh.faces["inlet"], dtype=np.int32)
    s = T.Solver(prob.mesh.xyz, prob.mesh.tets, K, prob.rho, prob.mu, prob.omega, backflow_beta=0.5)
    s.set_dirichlet(dn.astype(np.int32))
    s.set_neumann(inlet)
    s.set_tracer(to_dev(yv), kappa, stabilized)
    torch.cuda.synchronize()
    C = slots_to_modes(yv[:, :3, :], K)
    uq = np.einsum("qb,ebjn->eqjn", QP_BARY, C[prob.mesh.tets])
    B, _, _, _ = OC.element_matrices(prob.mesh.xyz, prob.mesh.tets, uq, kappa, prob.omega,
                                     stabilized=stabilized)
    Bf = OC.face_matrices(prob.mesh.xyz, inlet, C, 0.5)
    A = OC.assemble(prob.mesh.xyz, prob.mesh.tets, B) + OC.assemble(prob.mesh.xyz, inlet, Bf)
    assert abs(Bf).max() > 0          # the flow enters through the natural boundary
    return prob, s, A, dn


@pytest.mark.parametrize("stabilized", [True, False])
@pytest.mark.parametrize("K", [1, 2])
def test_tracer_backflow_residual_and_product_match_oracle(K, stabilized):
    log(f"[gpu] tracer with backflow faces K={K} stabilized={stabilized}")
    prob, s, A, dn = _setup_backflow(K, stabilized)
    rng = np.random.default_rng(10 + K)
    y = np.zeros((prob.mesh.n_nodes, 4, 2 * K + 2))
    y[:, 0] = rng.standard_normal((prob.mesh.n_nodes, 2 * K + 2))
    y[:, 0, 1] = 0.0
    r = to_dev(np.zeros_like(y))
    s.linearize(to_dev(y), r)
    rg = to_host(r)
    rr = _apply(A, y[:, 0], K, dn)
    assert np.abs(rg[:, 1:]).max() == 0.0
    assert np.abs(rg[:, 0] - rr).max() <= TOL * np.abs(rr).max()
    v = np.zeros_like(y)
    v[:, 0] = rng.standard_normal((prob.mesh.n_nodes, 2 * K + 2))
    v[:, 0, 1] = 0.0
    out = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out)
    jg = to_host(out)
    vm = v[:, 0].copy()
    vm[dn] = 0.0
    jr = _apply(A, vm, K, dn)
    assert np.abs(jg[:, 1:]).max() == 0.0
    assert np.abs(jg[:, 0] - jr).max() <= TOL * np.abs(jr).max()


def test_tracer_backflow_solve_cross_evaluated_by_oracle():
    log("[gpu] tracer solve with backflow faces")
    K = 2
    prob, s, A, dn = _setup_backflow(K, True, kappa=0.02, solved_velocity=True)
    y0 = np.zeros((prob.mesh.n_nodes, 4, 2 * K + 2))
    y0[dn, 0, 0] = 1.0
    y = to_dev(y0)
    st = s.solve(y, rtol=1e-9, lin_rtol=1e-6, restart=100, max_newton=10, max_matvec=20000)
    assert st["status"] == 0, st
    yg = to_host(y)
    assert np.abs(yg[:, 1:]).max() == 0.0
    r0 = np.linalg.norm(_apply(A, y0[:, 0], K, dn))
    r = np.linalg.norm(_apply(A, yg[:, 0], K, dn))
    log(f"[gpu]   newton {st['newton_iters']} matvecs {st['matvecs']} oracle rel {r / r0:.2e}")
    assert r <= 1e-8 * r0
