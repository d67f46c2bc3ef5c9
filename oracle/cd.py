"""FP64 reference for the time-spectral GLS convection-diffusion equation
(section "Convection-diffusion in multiple dimensions", eq. 3D-weak and
eq. 3D-weak-def), assembled as a sparse complex matrix.

TEST INFRASTRUCTURE ONLY (pins the GLS machinery: convergence rates of the
error estimate's remarks and the identity of Lemma 1).

A source term f is allowed so that manufactured solutions can be used; it
enters as (w, f) + (L(w), tau f), which keeps the method consistent.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .tsref import (FACE_QP_BARY, QP_BARY, _face_geometry, _negpart, geometry, omega_diag,
                    tau_from_velocity, toeplitz)


def element_matrices(xyz, tets, uq, kappa, omega, C_I=3.0, stabilized=True):
    """B[e, a, b] (N x N complex) of b(N_a e, N_b e') and tau per qp.

    uq: (E, 4, 3, N) complex velocity modes at the quadrature points.
    stabilized=False drops the least-squares term (tau = 0): the Galerkin
    method of the paper's comparison (section "Importance of stabilization").
    """
    grads, vol, G = geometry(xyz, tets)
    N = uq.shape[-1]
    K = (N - 1) // 2
    Om = np.diag(omega_diag(K, omega))
    w = vol / 4.0
    A = toeplitz(uq)                                               # (E,4,3,N,N)
    tau = tau_from_velocity(uq, G[:, None], kappa, C_I)            # (E,4,N,N)
    if not stabilized:
        tau = np.zeros_like(tau)
    AdN = np.einsum("eqimn,ebi->eqbmn", A, grads, optimize=True)  # A_i dN_b/dx_i
    T = np.einsum("qb,mn->qbmn", QP_BARY, Om)[None] + AdN          # Omega N_b + A.grad N_b
    P = -np.einsum("qa,mn->qamn", QP_BARY, Om)[None] + AdN         # adjoint test operator
    I = np.eye(N)
    B = (np.einsum("e,qa,eqbmn->eabmn", w, QP_BARY, T, optimize=True)
         + kappa * np.einsum("e,eak,ebk,mn->eabmn", vol, grads, grads, I, optimize=True)
         + np.einsum("e,eqamk,eqkl,eqbln->eabmn", w, P, tau, T, optimize=True))
    return B, tau, P, w


def face_matrices(xyz, tris, C, beta):
    """Backflow term of the convection-diffusion equation on Neumann faces
    (remarks after the backflow stabilization of the Navier-Stokes equations):
    -(w, (beta / 2) |A_n|_- phi)_Gamma is added to b(w, phi), with
    |A_n|_- = (A_n - |A_n|) / 2 and A_n the mode-coupling matrix of the
    normal velocity u.n, on the 3-point degree-2 face rule (weights area/3).

    tris: (F, 3) face nodes; C: (n_nodes, 3, N) complex velocity modes.
    Returns Bf[f, a, b] (N x N complex), assembled like element blocks.
    """
    nhat, area = _face_geometry(xyz, tris)
    uf = np.einsum("qa,fain->fqin", FACE_QP_BARY, C[tris][:, :, :3])
    un = np.einsum("fi,fqin->fqn", nhat, uf)
    Aneg = _negpart(toeplitz(un))                                  # (F, 3, N, N)
    return -0.5 * beta * np.einsum("f,qa,qb,fqmn->fabmn", area / 3.0, FACE_QP_BARY,
                                   FACE_QP_BARY, Aneg, optimize=True)


def assemble(xyz, tets, B):
    E, _, _, N, _ = B.shape
    n = xyz.shape[0]
    rows = (tets[:, :, None, None, None] * N + np.arange(N)[None, None, None, :, None])
    cols = (tets[:, None, :, None, None] * N + np.arange(N)[None, None, None, None, :])
    rows = np.broadcast_to(rows, B.shape).ravel()
    cols = np.broadcast_to(cols, B.shape).ravel()
    return sps.csr_matrix((B.ravel(), (rows, cols)), shape=(n * N, n * N))


def source_vector(xyz, tets, P, tau, w, fq):
    """(w, f) + (L(w), tau f): fq (E, 4, N) source modes at the qp."""
    N = fq.shape[-1]
    tf = np.einsum("eqmn,eqn->eqm", tau, fq)
    Fe = (np.einsum("e,qa,eqm->eam", w, QP_BARY, fq)
          + np.einsum("e,eqamn,eqn->eam", w, P, tf, optimize=True))
    F = np.zeros((xyz.shape[0], N), dtype=complex)
    np.add.at(F, tets, Fe)
    return F.ravel()


def solve_dirichlet(Amat, F, n_nodes, N, bnodes, gvals):
    """Solve with phi = g on bnodes (rows replaced, columns moved to the rhs)."""
    phi = np.zeros((n_nodes, N), dtype=complex)
    phi[bnodes] = gvals
    fixed = np.zeros(n_nodes * N, dtype=bool)
    fixed.reshape(n_nodes, N)[bnodes] = True
    free = ~fixed
    rhs = F - Amat @ phi.ravel()
    sol = spla.spsolve(Amat[free][:, free].tocsc(), rhs[free])
    out = phi.ravel().copy()
    out[free] = sol
    return out.reshape(n_nodes, N)
