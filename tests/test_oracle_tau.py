"""Pins for the stabilisation matrix tau (eq. 3D-tau).

* Reduction to the 1D steady formula eq. 1D-Stau: on the right-angled tet
  with legs h, G = I/h^2 and C_I = 3 make the 3D tau equal the 1D tau of an
  element of parent size 2 and physical size 2h.
* Steady velocity: tau is the scalar tau times the identity (first remark
  after eq. 1D-tau).
* Unidirectional one-harmonic velocity: A is tridiagonal Toeplitz, whose
  eigenvalues have the closed form u0 + 2|u1| cos(j pi/(n+1)) (the closed
  form the second remark refers to), so tau's eigenvalues are known.
* Hermitian, positive definite, centrosymmetric (fourth and fifth remarks),
  and tau^2 S = I.
"""
import numpy as np
import pytest

import oracle as O


def _right_tet(h):
    xyz = np.array([[0, 0, 0], [h, 0, 0], [0, h, 0], [0, 0, h]], float)
    return xyz, np.array([[0, 1, 2, 3]])


@pytest.mark.parametrize("h,u,nu", [(0.1, 1.0, 0.01), (0.5, 0.3, 0.2), (0.02, 5.0, 1e-4)])
def test_tau_reduces_to_1d_steady_formula(h, u, nu):
    xyz, tets = _right_tet(h)
    _, _, G = O.geometry(xyz, tets)
    uq = np.zeros((3, 1), complex)
    uq[0, 0] = u
    tau = O.tau_from_velocity(uq, G[0], nu, 3.0)
    H = 2 * h
    tau1d = ((2 * u / H) ** 2 + (12 * nu / H ** 2) ** 2) ** -0.5
    assert np.isclose(tau[0, 0].real, tau1d, rtol=1e-13)


@pytest.mark.parametrize("K", [1, 3, 6])
def test_tau_steady_velocity_is_scalar_identity(K):
    rng = np.random.default_rng(K)
    xyz = rng.standard_normal((4, 3))
    tets = np.array([[0, 1, 2, 3]])
    from workloads.meshgen import orient_positive
    tets = orient_positive(xyz, tets)
    _, _, G = O.geometry(xyz, tets)
    u0 = rng.standard_normal(3)
    uq = np.zeros((3, 2 * K + 1), complex)
    uq[:, K] = u0
    nu = 0.05
    tau = O.tau_from_velocity(uq, G[0], nu, 3.0)
    s = (u0 @ G[0] @ u0 + 3.0 * nu ** 2 * np.sum(G[0] ** 2)) ** -0.5
    assert np.allclose(tau, s * np.eye(2 * K + 1), atol=1e-13 * s)


@pytest.mark.parametrize("K", [1, 2, 5, 10])
def test_tau_unidirectional_one_harmonic_closed_form(K):
    rng = np.random.default_rng(7 + K)
    xyz = rng.standard_normal((4, 3))
    from workloads.meshgen import orient_positive
    tets = orient_positive(xyz, np.array([[0, 1, 2, 3]]))
    _, _, G = O.geometry(xyz, tets)
    n = 2 * K + 1
    u0, u1 = 0.7, 0.4 * np.exp(1.1j)
    uq = np.zeros((3, n), complex)
    uq[0, K] = u0
    uq[0, K + 1] = u1
    uq[0, K - 1] = np.conj(u1)
    nu = 0.03
    tau = O.tau_from_velocity(uq, G[0], nu, 3.0)
    lamA = u0 + 2 * abs(u1) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    expect = np.sort((G[0][0, 0] * lamA ** 2 + 3.0 * nu ** 2 * np.sum(G[0] ** 2)) ** -0.5)
    got = np.sort(np.linalg.eigvalsh(tau))
    assert np.allclose(got, expect, rtol=1e-12)


@pytest.mark.parametrize("K", [1, 3, 6])
def test_tau_invariants(K):
    rng = np.random.default_rng(K + 20)
    xyz = rng.standard_normal((4, 3))
    from workloads.meshgen import orient_positive
    tets = orient_positive(xyz, np.array([[0, 1, 2, 3]]))
    _, _, G = O.geometry(xyz, tets)
    y = rng.standard_normal((3, 2 * K + 2))
    uq = O.slots_to_modes(y, K)
    tau, S = O.tau_from_velocity(uq, G[0], 0.01, 3.0, return_S=True)
    assert np.allclose(tau, tau.conj().T, atol=1e-14 * np.abs(tau).max())
    assert np.linalg.eigvalsh(tau).min() > 0
    assert np.allclose(tau[::-1, ::-1], tau.conj(), atol=1e-13 * np.abs(tau).max())
    assert np.allclose(tau @ tau @ S, np.eye(2 * K + 1), atol=1e-10)
