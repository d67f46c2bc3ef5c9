"""GPU results against closed forms, independent of the oracle.

tau (eq. 3D-tau):

* Zero velocity: S = C_I nu^2 (G:G) I, so tau = (C_I nu^2 G:G)^(-1/2) I at
  every quadrature point.
* A uniform steady velocity U (only c_0 of each velocity field non-zero): the
  convection matrices are A_i = U_i I, so S = (U^T G U + C_I nu^2 G:G) I.

G_ij = sum_k dxi_k/dx_i dxi_k/dx_j comes from the inverse of each tet's
Jacobian.  The pressure field is random: tau must not depend on it.  S is a
multiple of I, so the one-sided Jacobi has nothing to rotate and tau is exact
up to the rounding of S and of the inverse square root: 1e-13 relative.
Cases span one element, several K (including the sampled form, K = 7) and a
ragged element count.

Residual (eq. Rmc): a uniform steady outflow has none.
"""
import numpy as np
import pytest

from workloads import cube_problem, junction_problem, tiny_problem
from tests.gpu_helpers import log, to_dev, unpack

pytestmark = pytest.mark.gpu

CASES = {
    "tiny1_K2": lambda: tiny_problem(1, K=2),
    "cube3_K6": lambda: cube_problem(3, K=6),
    "cube2_K7": lambda: cube_problem(2, K=7),
    "junction_K3": lambda: junction_problem(h=0.35, K=3),
}


def _metric(prob):
    X = prob.mesh.xyz[prob.mesh.tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    Ji = np.linalg.inv(J)                                   # Ji[e, k, i] = dxi_k / dx_i
    return np.einsum("eki,ekj->eij", Ji, Ji)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("steady", [False, True])
def test_tau_closed_form(name, steady):
    import paper_2311_09465_amd as T
    log(f"[gpu] tau closed form {name} steady={steady}")
    prob = CASES[name]()
    n = 2 * prob.K + 1
    rng = np.random.default_rng(3)
    y = np.zeros((prob.mesh.n_nodes, 4, 2 * prob.K + 2))
    y[:, 3] = rng.standard_normal((prob.mesh.n_nodes, 2 * prob.K + 2))
    y[:, 3, 1] = 0.0
    U = np.array([0.7, -1.3, 0.4]) if steady else np.zeros(3)
    y[:, :3, 0] = U
    s = T.Solver.from_problem(prob)
    s.linearize(to_dev(y))
    tg = unpack(s.get_tau(), n)                              # (E, 4, n, n)
    G = _metric(prob)
    nu = prob.mu / prob.rho
    sval = np.einsum("i,eij,j->e", U, G, U) + prob.C_I * nu * nu * np.einsum("eij,eij->e", G, G)
    expect = sval ** -0.5
    diag = np.diagonal(tg, axis1=-2, axis2=-1)               # (E, 4, n)
    off = tg - diag[..., None] * np.eye(n)
    assert np.abs(diag - expect[:, None, None]).max() <= 1e-13 * expect.max()
    assert np.abs(off).max() <= 1e-13 * expect.max()


@pytest.mark.parametrize("name", ["cube3_K6", "cube2_K7"])
def test_uniform_outflow_has_zero_residual(name):
    """A uniform steady velocity with zero pressure solves every volume term
    of eq. Rmc (no time derivative, no convection or viscous flux, zero
    divergence, zero L_i).  Pointed out through the Neumann face, it has no
    backflow term either, so the residual vanishes up to rounding."""
    import torch
    import paper_2311_09465_amd as T
    log(f"[gpu] uniform outflow residual {name}")
    prob = CASES[name]()
    assert prob.neumann_h is None
    xyz, tris = prob.mesh.xyz, prob.neumann_tris
    nrm = np.cross(xyz[tris[:, 1]] - xyz[tris[:, 0]], xyz[tris[:, 2]] - xyz[tris[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    assert np.abs(nrm - nrm[0]).max() < 1e-12            # a planar outlet
    U = 0.9 * nrm[0] + 0.3 * np.cross(nrm[0], [0.6, 0.8, 0.0])
    assert (nrm @ U).min() > 0.5
    y = np.zeros((prob.mesh.n_nodes, 4, 2 * prob.K + 2))
    y[:, :3, 0] = U
    s = T.Solver.from_problem(prob)
    r = torch.zeros(s.shape, dtype=torch.float64, device="cuda")
    s.residual(to_dev(y), r)
    r = r.cpu().numpy()
    X = xyz[prob.mesh.tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    vol = np.abs(np.linalg.det(J)) / 6.0
    grad = np.abs(np.linalg.inv(J)).sum(axis=1).max()
    scale = prob.rho * (U @ U) * grad * vol.max() * 32   # one term of one node's sum
    assert np.abs(r).max() <= 1e-12 * scale
