"""Pins of the GLS machinery (tau, convolution matrices, least-squares term)
through the time-spectral convection-diffusion equation, eq. 3D-weak.

* Manufactured smooth solution, diffusive regime (alpha, beta << 1): the L2
  error must fall at rate 2 and the H1 error at rate 1 under refinement (the
  remarks after Theorem 1 on the diffusive regime).
* Lemma 1 with Gamma_h empty: Re(w^H B w) = kappa ||grad w||^2 +
  ||L(w)||_tau^2 and Im(w^H B w) = 0 for discrete w vanishing on Gamma
  (uniform, hence divergence-free, unsteady velocity).
"""
import numpy as np
import pytest

import oracle as O
from oracle import cd
from workloads import cube_kuhn

K = 2
OMEGA = 1.0
UMODES = np.zeros((3, 2 * K + 1), complex)     # u(t) = (1 + 0.5 cos t, 0.3, 0)
UMODES[0, K] = 1.0
UMODES[0, K + 1] = UMODES[0, K - 1] = 0.25
UMODES[1, K] = 0.3


def _phi(x):
    """Exact modes phi_m(x), m = -K..K, with gradients and Laplacians."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    one = np.ones_like(X)
    f0 = np.exp(X) * np.sin(Y) * np.cos(Z)
    g0 = np.stack([f0, np.exp(X) * np.cos(Y) * np.cos(Z), -np.exp(X) * np.sin(Y) * np.sin(Z)], -1)
    l0 = -f0
    f1 = (1 + 1j) * X * X * Y
    g1 = (1 + 1j) * np.stack([2 * X * Y, X * X, 0 * one], -1)
    l1 = (1 + 1j) * 2 * Y
    c = np.cos(np.pi * X)
    s = np.sin(np.pi * X)
    f2 = 0.3j * c * Y * Z
    g2 = 0.3j * np.stack([-np.pi * s * Y * Z, c * Z, c * Y], -1)
    l2 = 0.3j * (-np.pi ** 2) * c * Y * Z
    vals = [np.conj(f2), np.conj(f1), f0.astype(complex), f1, f2]
    grads = [np.conj(g2), np.conj(g1), g0.astype(complex), g1, g2]
    laps = [np.conj(l2), np.conj(l1), l0.astype(complex), l1, l2]
    return np.stack(vals, -1), np.stack(grads, -1), np.stack(laps, -1)


def _source(x, kappa):
    phi, gphi, lap = _phi(x)
    Om = 1j * OMEGA * np.arange(-K, K + 1)
    A = O.toeplitz(UMODES)                                 # (3, N, N)
    conv = np.einsum("imn,...in->...m", A, gphi)
    return Om * phi + conv - kappa * lap


def _solve(n, kappa):
    m = cube_kuhn(n)
    xyz, tets = m.xyz, m.tets
    E = tets.shape[0]
    uq = np.broadcast_to(UMODES, (E, 4, 3, 2 * K + 1)).copy()
    B, tau, P, w = cd.element_matrices(xyz, tets, uq, kappa, OMEGA)
    Amat = cd.assemble(xyz, tets, B)
    xq = np.einsum("qa,eai->eqi", O.QP_BARY, xyz[tets])
    F = cd.source_vector(xyz, tets, P, tau, w, _source(xq, kappa))
    bn = np.unique(np.concatenate(list(m.faces.values())))
    phi_b = _phi(xyz[bn])[0]
    sol = cd.solve_dirichlet(Amat, F, xyz.shape[0], 2 * K + 1, bn, phi_b)
    # errors with the 4-point rule
    grads, vol, _ = O.geometry(xyz, tets)
    ph, gph, _ = _phi(xq)
    eh = np.einsum("qa,eam->eqm", O.QP_BARY, sol[tets]) - ph
    e2 = np.sum(vol[:, None] / 4 * np.sum(np.abs(eh) ** 2, -1))
    gh = np.einsum("eai,eam->eim", grads, sol[tets])[:, None] - gph
    h1 = np.sum(vol[:, None] / 4 * np.sum(np.abs(gh) ** 2, (-1, -2)))
    return np.sqrt(e2), np.sqrt(h1)


@pytest.mark.slow
def test_manufactured_solution_rates_diffusive():
    errs = [_solve(n, kappa=1.0) for n in (4, 8, 16)]
    l2 = [e[0] for e in errs]
    h1 = [e[1] for e in errs]
    r_l2 = np.log2(np.array(l2[:-1]) / np.array(l2[1:]))
    r_h1 = np.log2(np.array(h1[:-1]) / np.array(h1[1:]))
    assert np.all(r_l2 > 1.8), r_l2
    assert np.all(r_h1 > 0.9), r_h1


@pytest.mark.parametrize("kappa", [1.0, 1e-2])
def test_lemma1_identity(kappa):
    m = cube_kuhn(3)
    xyz, tets = m.xyz, m.tets
    E, N = tets.shape[0], 2 * K + 1
    uq = np.broadcast_to(UMODES, (E, 4, 3, N)).copy()
    B, tau, P, w = cd.element_matrices(xyz, tets, uq, kappa, OMEGA)
    Amat = cd.assemble(xyz, tets, B)
    rng = np.random.default_rng(0)
    y = rng.standard_normal((xyz.shape[0], 2 * K + 2))
    y[:, 1] = 0
    c = O.slots_to_modes(y, K)
    bn = np.unique(np.concatenate(list(m.faces.values())))
    c[bn] = 0
    q = np.conj(c.ravel()) @ (Amat @ c.ravel())
    grads, vol, _ = O.geometry(xyz, tets)
    g = np.einsum("eai,eam->eim", grads, c[tets])
    grad2 = np.sum(vol * np.sum(np.abs(g) ** 2, (-1, -2)))
    Om = 1j * OMEGA * np.arange(-K, K + 1)
    cq = np.einsum("qa,eam->eqm", O.QP_BARY, c[tets])
    A = O.toeplitz(UMODES)
    L = Om * cq + np.einsum("imn,ein->em", A, g)[:, None]
    ls = np.sum(vol[:, None] / 4 * np.einsum("eqm,eqmn,eqn->eq", np.conj(L), tau, L).real)
    assert abs(q.imag) < 1e-12 * abs(q)
    assert np.isclose(q.real, kappa * grad2 + ls, rtol=1e-12)


# ---- backflow term on Neumann faces (cd.face_matrices) ----
# One face, the right triangle (0,0,0), (2,0,0), (0,1,0): area 1, outward
# normal +z.  Velocity uniform in space, so |A_n|_- is the same at the three
# face points and the face integrals of N_a N_b are exact: area/12 (1 + d_ab).
_FXYZ = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
_FTRI = np.array([[0, 1, 2]])


def _uniform_velocity(umodes):
    return np.broadcast_to(umodes, (3,) + umodes.shape).copy()


def test_face_backflow_steady_closed_form():
    """K = 0: |A_n|_- = min(u.n, 0), so the block is
    -(beta/2) min(u.n, 0) area/12 (1 + d_ab) (textbook backflow term)."""
    beta = 0.7
    for un in (-1.3, 0.4):
        um = np.zeros((3, 1), complex)
        um[2, 0] = un
        Bf = cd.face_matrices(_FXYZ, _FTRI, _uniform_velocity(um), beta)
        exact = -0.5 * beta * min(un, 0.0) * (1.0 / 12.0) * (np.ones((3, 3)) + np.eye(3))
        assert np.allclose(Bf[0, :, :, 0, 0], exact, rtol=0, atol=1e-15)


def test_face_backflow_vanishes_without_inflow():
    """u.n(t) > 0 at all times: every eigenvalue of A_n is positive and the
    term is exactly zero (it only acts where flow enters)."""
    K2 = 2
    um = np.zeros((3, 2 * K2 + 1), complex)
    um[2, K2] = 1.0                            # u.n = 1 + 0.4 cos t + 0.2 sin 2t > 0
    um[2, K2 + 1] = um[2, K2 - 1] = 0.2
    um[2, K2 + 2], um[2, K2 - 2] = -0.1j, 0.1j
    Bf = cd.face_matrices(_FXYZ, _FTRI, _uniform_velocity(um), 1.0)
    assert np.abs(Bf).max() == 0.0


def test_face_backflow_one_harmonic_trace():
    """K = 1, u.n = a0 + a1 cos t: A_n is tridiagonal Toeplitz (diagonal a0,
    off-diagonals a1/2) with eigenvalues a0 + a1 cos(k pi / 4), k = 1..3, so
    trace(Bf[a, a]) = -(beta/2) (area/6) sum_k min(lambda_k, 0)."""
    a0, a1, beta = -0.3, 1.0, 0.5
    um = np.zeros((3, 3), complex)
    um[2, 1] = a0
    um[2, 0] = um[2, 2] = a1 / 2
    Bf = cd.face_matrices(_FXYZ, _FTRI, _uniform_velocity(um), beta)
    lam = a0 + a1 * np.cos(np.arange(1, 4) * np.pi / 4)
    exact = -0.5 * beta * (1.0 / 6.0) * np.minimum(lam, 0.0).sum()
    for a in range(3):
        assert abs(np.trace(Bf[0, a, a]) - exact) <= 1e-14
    # Hermitian negative part: the block is Hermitian and positive semidefinite
    blk = Bf[0, 0, 0]
    assert np.allclose(blk, blk.conj().T, atol=1e-15)
    assert np.linalg.eigvalsh(blk).min() >= -1e-15
