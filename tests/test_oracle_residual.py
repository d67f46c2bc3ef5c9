"""Pins for the oracle residual (eq. Rmc) and tangent (eq. K_mat).

* K = 0: the time-spectral GLS residual must equal a textbook steady
  SUPG/PSPG residual written here independently in real arithmetic, element
  by element, from Appendix B (eq. NSt-weak with d/dt = 0 and omega_hat = 0,
  tau of eq. 3D-taut), including the conventional backflow term.
* Im of the mean-mode residual vanishes and the complex residual is
  conjugate-symmetric (the mode-coupling verification remark in the tracer
  results, and the real-valued-unknowns section).
* Steady data at K > 0: harmonics of the residual vanish and the mean mode
  equals the K = 0 residual.
* Backflow term vanishes without backflow (second remark of the backflow
  section).
* Tangent: Picard tangent = exact derivative of the residual with A and tau
  frozen (affine, so round-off); 'newton' tangent = central finite
  differences of the residual with tau and |A_n|_- frozen; matrix-free
  Picard = assembled eq. K_mat blocks; the Jacobi diagonal = diagonal of the
  dense tangent built column by column.
"""
import numpy as np
import pytest

import oracle as O
from workloads import cube_problem, tiny_problem
from workloads.problems import _complex_to_slots


def _state(prob, seed, steady=False, scale=1.0):
    rng = np.random.default_rng(seed)
    y = scale * rng.standard_normal((prob.mesh.n_nodes, 4, 2 * prob.K + 2))
    y[..., 1] = 0
    if steady:
        y[..., 2:] = 0
    y[prob.dirichlet_nodes, :3] = prob.dirichlet_values
    return y


def _textbook_steady(prob, y):
    """Steady SUPG/PSPG residual, real arithmetic, one element at a time."""
    xyz, tets = prob.mesh.xyz, prob.mesh.tets
    rho, mu, nu, CI = prob.rho, prob.mu, prob.mu / prob.rho, prob.C_I
    u = y[:, :3, 0]
    p = y[:, 3, 0]
    R = np.zeros((xyz.shape[0], 4))
    a5 = (5 + 3 * 5 ** 0.5) / 20
    b5 = (5 - 5 ** 0.5) / 20
    for e in range(tets.shape[0]):
        nd = tets[e]
        X = xyz[nd]
        J = np.column_stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
        Ji = np.linalg.inv(J)
        dN = np.vstack([-Ji.sum(axis=0), Ji])          # dN[a, i]
        V = np.linalg.det(J) / 6
        G = Ji.T @ Ji
        gu = dN.T @ u[nd]                              # gu[j, i] = du_i/dx_j
        gp = dN.T @ p[nd]
        for q in range(4):
            lam = np.full(4, b5)
            lam[q] = a5
            uq = lam @ u[nd]
            pq = lam @ p[nd]
            tau = (uq @ G @ uq + CI * nu * nu * np.sum(G * G)) ** -0.5
            rhat = rho * (uq @ gu) + gp
            w = V / 4
            for a in range(4):
                for i in range(3):
                    R[nd[a], i] += w * (lam[a] * rho * (uq @ gu[:, i]) - dN[a, i] * pq
                                        + mu * dN[a] @ gu[:, i] + (uq @ dN[a]) * tau * rhat[i])
                R[nd[a], 3] += w * (lam[a] * np.trace(gu) + dN[a] @ (tau * rhat) / rho)
    for f in prob.neumann_tris:
        X = xyz[f]
        nv = np.cross(X[1] - X[0], X[2] - X[0])
        area = np.linalg.norm(nv) / 2
        n = nv / np.linalg.norm(nv)
        for q in range(3):
            lam = np.full(3, 1 / 6)
            lam[q] = 2 / 3
            uq = lam @ u[f]
            un = min(uq @ n, 0.0)
            for a in range(3):
                R[f[a], :3] += -0.5 * rho * prob.backflow_beta * (area / 3) * lam[a] * un * uq
    R[prob.dirichlet_nodes, :3] = 0
    return R


@pytest.mark.parametrize("seed", [0, 1])
def test_k0_equals_textbook_supg_pspg(seed):
    prob = cube_problem(3, K=0)
    y = _state(prob, seed)
    par = O.Params.from_problem(prob)
    r = O.residual(par, prob.mesh.xyz, prob.mesh.tets, y)
    ref = _textbook_steady(prob, y)
    assert np.abs(r[..., 1]).max() == 0
    assert np.allclose(r[..., 0], ref, atol=1e-12 * np.abs(ref).max())
    # the random state has backflow somewhere on the outlet
    assert np.abs(r[..., 0] - O.residual(O.Params(**{**par.__dict__, "backflow_beta": 0.0}),
                                         prob.mesh.xyz, prob.mesh.tets, y)[..., 0]).max() > 0


@pytest.mark.parametrize("K", [1, 3])
def test_mean_mode_real_and_conjugate_symmetry(K):
    prob = cube_problem(2, K=K)
    y = _state(prob, 3)
    par = O.Params.from_problem(prob)
    raw = O.residual(par, prob.mesh.xyz, prob.mesh.tets, y, raw=True)
    scale = np.abs(raw).max()
    assert np.abs(raw[..., K].imag).max() < 1e-13 * scale
    assert np.allclose(raw[..., :K][..., ::-1], np.conj(raw[..., K + 1:]), atol=1e-13 * scale)


def test_steady_data_at_k_gt_0_reduces_to_k0():
    p0 = cube_problem(2, K=0)
    p3 = cube_problem(2, K=3)
    y3 = _state(p3, 5, steady=True)
    y3[p3.dirichlet_nodes, :3, 2:] = 0
    y0 = y3[..., :2].copy()
    r3 = O.residual(O.Params.from_problem(p3), p3.mesh.xyz, p3.mesh.tets, y3)
    r0 = O.residual(O.Params.from_problem(p0), p0.mesh.xyz, p0.mesh.tets, y0)
    scale = np.abs(r0).max()
    assert np.abs(r3[..., 2:]).max() < 1e-14 * scale
    assert np.allclose(r3[..., 0], r0[..., 0], atol=1e-13 * scale)


def test_backflow_term_inactive_without_backflow():
    prob = cube_problem(2, K=2)
    y = _state(prob, 4, scale=0.05)
    out = np.unique(prob.neumann_tris)
    y[out, 0, 0] = 1.0            # strong outflow through x = 1 at every harmonic phase
    par = O.Params.from_problem(prob)
    r1 = O.residual(par, prob.mesh.xyz, prob.mesh.tets, y)
    par0 = O.Params(**{**par.__dict__, "backflow_beta": 0.0})
    r0 = O.residual(par0, prob.mesh.xyz, prob.mesh.tets, y)
    assert np.array_equal(r1, r0)


def _tiny(nt, K, seed=1):
    prob = tiny_problem(nt, K=K, seed=seed)
    par = O.Params.from_problem(prob)
    rng = np.random.default_rng(seed + 10)
    y = rng.standard_normal((prob.mesh.n_nodes, 4, 2 * K + 2))
    y[..., 1] = 0
    y[prob.dirichlet_nodes, :3] = prob.dirichlet_values
    v = rng.standard_normal(y.shape)
    v[..., 1] = 0
    v[prob.dirichlet_nodes, :3] = 0
    return prob, par, y, v


@pytest.mark.parametrize("nt,K", [(1, 1), (2, 2), (6, 1), (6, 2)])
def test_jacobian_variants_against_definitions(nt, K):
    prob, par, y, v = _tiny(nt, K)
    xyz, tets = prob.mesh.xyz, prob.mesh.tets
    lin = O.linearize(par, xyz, tets, y)
    jp = O.jv(par, xyz, tets, lin, v, "picard")
    aff = (O.residual(par, xyz, tets, y + v, frozen=("all", lin))
           - O.residual(par, xyz, tets, y, frozen=("all", lin)))
    assert np.linalg.norm(aff - jp) <= 1e-12 * np.linalg.norm(jp)
    eps = 1e-6 * np.linalg.norm(y) / np.linalg.norm(v)
    fd = (O.residual(par, xyz, tets, y + eps * v, frozen=("tau", lin))
          - O.residual(par, xyz, tets, y - eps * v, frozen=("tau", lin))) / (2 * eps)
    jn = O.jv(par, xyz, tets, lin, v, "newton")
    assert np.linalg.norm(fd - jn) <= 1e-7 * np.linalg.norm(jn)
    hb = O.picard_matvec(par, xyz, tets, lin, v)
    assert np.linalg.norm(hb - jp) <= 1e-12 * np.linalg.norm(jp)


def test_picard_nols_drops_only_ls_coupling():
    """Variant without least-squares terms in G_i and D_i: equal to the full
    tangent on pure-velocity and pure-pressure directions' diagonal blocks."""
    prob, par, y, v = _tiny(6, 2)
    xyz, tets = prob.mesh.xyz, prob.mesh.tets
    lin = O.linearize(par, xyz, tets, y)
    vu = v.copy()
    vu[:, 3] = 0
    a = O.jv(par, xyz, tets, lin, vu, "picard")
    b = O.jv(par, xyz, tets, lin, vu, "picard_nols")
    assert np.allclose(a[:, :3], b[:, :3], atol=1e-13)        # K block identical
    assert not np.allclose(a[:, 3], b[:, 3])                   # D block differs
    vp = v.copy()
    vp[:, :3] = 0
    a = O.jv(par, xyz, tets, lin, vp, "picard")
    b = O.jv(par, xyz, tets, lin, vp, "picard_nols")
    assert np.allclose(a[:, 3], b[:, 3], atol=1e-13)          # L block identical
    assert not np.allclose(a[:, :3], b[:, :3])                 # G block differs


@pytest.mark.parametrize("dt", [None, 0.3])
def test_jacobian_diagonal_matches_dense(dt):
    prob, par, y, v = _tiny(6, 2)
    xyz, tets = prob.mesh.xyz, prob.mesh.tets
    lin = O.linearize(par, xyz, tets, y)
    d = O.jacobian_diagonal(par, xyz, tets, lin, dt)
    n = y.size
    diag = np.empty(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        diag[k] = O.jv(par, xyz, tets, lin, e.reshape(y.shape), "picard", dt).ravel()[k]
    diag = diag.reshape(y.shape)
    masked = np.zeros(y.shape, bool)
    masked[..., 1] = True
    masked[prob.dirichlet_nodes, :3] = True
    assert np.allclose(d[~masked], diag[~masked], rtol=1e-12, atol=1e-14)
    assert np.all(d[masked] == 1.0)
