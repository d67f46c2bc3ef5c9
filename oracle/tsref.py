"""FP64 reference for the time-spectral GLS Navier-Stokes residual, tangent and
Newton-GMRES solve on linear tetrahedra.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
``cpu_baseline`` leg of the benchmark; never by the product path.

Everything here follows the paper's complex-modal formulation literally:

* modes m = -K..K (K harmonics; the paper's N = K+1), c_{-m} = conj(c_m)
  (section "A model problem: 1D convection-diffusion", eq. phiDef);
* Omega = diag(i m omega) and the Toeplitz convolution matrix
  A_mn = u_{m-n}, |m-n| <= K (eq. phi-def);
* tau = [A_i G_ij A_j + C_I kappa^2 G_ij G_ij I]^(-1/2) from an
  eigendecomposition, kappa = mu/rho (eq. 3D-tau and the procedure after it);
* residual r^m, r^c of eq. Rmc with linear shape functions (second derivatives
  dropped), Dirichlet momentum rows removed;
* tangent blocks K, G_i, D_i, L of eq. K_mat (the "Picard" tangent, where the
  dependence of A_i and tau on u is neglected);
* pseudo-time mass shift (N_A, c1 rho / dt N_B I) with c1 = 1.5 (section
  "Pseudo-time stepping");
* backflow term -(rho beta / 2)(w, |A_n|_- u) on Neumann faces with
  |A_n|_- = (A_n - |A_n|)/2 from an eigendecomposition (section "Stabilizing
  simulations in the presence of backflow");
* real-valued unknowns: Re/Im of modes 0..K per field, Im c_0 kept as a zero
  slot (section "Using real-valued unknowns").

Quadrature (the paper does not name one): 4-point degree-2 rule on tets,
3-point degree-2 rule on triangles.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

_A = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
_B = (5.0 - math.sqrt(5.0)) / 20.0
#: QP_BARY[q, a] = N_a at volume quadrature point q (weights V/4)
QP_BARY = np.full((4, 4), _B)
np.fill_diagonal(QP_BARY, _A)
#: FACE_QP_BARY[q, a] = N_a at face quadrature point q (weights area/3)
FACE_QP_BARY = np.full((3, 3), 1.0 / 6.0)
np.fill_diagonal(FACE_QP_BARY, 2.0 / 3.0)

CHUNK = 2048


def _ein(*args):
    return np.einsum(*args, optimize=True)


@dataclasses.dataclass
class Params:
    K: int
    rho: float
    mu: float
    omega: float
    C_I: float = 3.0
    backflow_beta: float = 0.5
    dirichlet_nodes: np.ndarray = None
    neumann_tris: np.ndarray = None
    neumann_h: Optional[np.ndarray] = None   # (nf, 2K+2) slot layout, constant per face

    @property
    def N(self):              # number of complex modes stored, 2K+1
        return 2 * self.K + 1

    @property
    def nu(self):
        return self.mu / self.rho

    @classmethod
    def from_problem(cls, prob):
        return cls(K=prob.K, rho=prob.rho, mu=prob.mu, omega=prob.omega,
                   C_I=prob.C_I, backflow_beta=prob.backflow_beta,
                   dirichlet_nodes=np.asarray(prob.dirichlet_nodes),
                   neumann_tris=np.asarray(prob.neumann_tris),
                   neumann_h=prob.neumann_h)


# ------------------------------------------------------------------ basics
def geometry(xyz, tets):
    """Gradients of the P1 shape functions, volume and the metric tensor.

    Parent coordinates xi_k = N_k (k = 1..3, node 0 at the origin), so
    G_ij = sum_k dxi_k/dx_i dxi_k/dx_j (eq. metric).
    """
    X = xyz[tets]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)                       # Jinv[e, k, i] = dxi_k / dx_i
    grads = np.empty((tets.shape[0], 4, 3))
    grads[:, 1:, :] = Jinv
    grads[:, 0, :] = -Jinv.sum(axis=1)
    vol = np.linalg.det(J) / 6.0
    G = _ein("eki,ekj->eij", Jinv, Jinv)
    return grads, vol, G


def slots_to_modes(y, K):
    """Slot layout (..., 2K+2) -> complex modes (..., 2K+1), index m+K.
    The Im c_0 slot is ignored (a real field has a real mean)."""
    cp = y[..., 0::2] + 1j * y[..., 1::2]
    cp[..., 0] = y[..., 0]
    return np.concatenate([np.conj(cp[..., :0:-1]), cp], axis=-1)


def modes_to_slots(c, K, zero_im0=True):
    cp = c[..., K:]
    s = np.empty(c.shape[:-1] + (2 * K + 2,))
    s[..., 0::2] = cp.real
    s[..., 1::2] = cp.imag
    if zero_im0:
        s[..., 1] = 0.0
    return s


def toeplitz(u):
    """A[..., m, n] = u[..., m-n] for |m-n| <= K, else 0 (eq. phi-def)."""
    N = u.shape[-1]
    K = (N - 1) // 2
    pad = np.zeros(u.shape[:-1] + (K,), dtype=complex)
    up = np.concatenate([pad, u, pad], axis=-1)        # up[j] = u[j - K]
    win = np.lib.stride_tricks.sliding_window_view(up, N, axis=-1)
    # win[..., m, t] = up[m + t]; A[m, n] = up[m - n + 2K] = win[m, 2K - n]
    return np.ascontiguousarray(win[..., :N, ::-1])


def omega_diag(K, omega):
    return 1j * omega * np.arange(-K, K + 1)


def tau_from_velocity(uq, G, nu, C_I, return_S=False):
    """tau = [A_i G_ij A_j + C_I nu^2 (G:G) I]^(-1/2) per point.

    uq: (..., 3, 2K+1) complex velocity modes at the point; G: (..., 3, 3).
    The inverse square root is taken through a Hermitian eigendecomposition
    (eq. 3D-tau and the procedure described after it).
    """
    A = toeplitz(uq)                                         # (..., 3, N, N)
    B = _ein("...ij,...jkn->...ikn", G, A)                   # B_i = G_ij A_j
    S = np.matmul(A, B).sum(axis=-3)                         # sum_i A_i B_i
    GG = _ein("...ij,...ij->...", G, G)
    N = uq.shape[-1]
    S = S + (C_I * nu * nu * GG)[..., None, None] * np.eye(N)
    S = 0.5 * (S + np.conj(np.swapaxes(S, -1, -2)))
    lam, V = np.linalg.eigh(S)
    tau = _ein("...mk,...k,...nk->...mn", V, lam ** -0.5, np.conj(V))
    if return_S:
        return tau, S
    return tau


def _negpart(An):
    """|A_n|_- = (A_n - |A_n|)/2 = V min(Lambda, 0) V^H."""
    An = 0.5 * (An + np.conj(np.swapaxes(An, -1, -2)))
    lam, V = np.linalg.eigh(An)
    return _ein("...mk,...k,...nk->...mn", V, np.minimum(lam, 0.0), np.conj(V))


def _mask_rows(par, R):
    if par.dirichlet_nodes is not None and len(par.dirichlet_nodes):
        R[par.dirichlet_nodes, :3, :] = 0.0


def _chunks(E):
    for s in range(0, E, CHUNK):
        yield slice(s, min(E, s + CHUNK))


# ------------------------------------------------------- element operators
def _conv(A, g):
    """sum_j A[e,q,j] @ g[e,j,i]: (E,4,3,N,N) x (E,3,3,N) -> (E,4,3,N)."""
    T = np.matmul(A, np.swapaxes(g, -1, -2)[:, None])      # (E,4,3j,N,3i)
    return np.swapaxes(T.sum(axis=2), -1, -2)


def _element_apply(par, grads, vol, A, tau, D, variant="picard", newton=None,
                   shift=0.0):
    """Element contributions of the GLS operator with frozen A and tau,
    applied to nodal modes D (Ec, 4 nodes, 4 fields, N).

    With D = the state itself this is eq. Rmc without boundary terms; with
    D = a direction it is the tangent of eq. K_mat (variant 'picard'), the
    tangent with least-squares terms removed from G_i and D_i ('picard_nols',
    section "Exploiting the structure of H"), or the tangent that also keeps
    the derivative of the convection matrices ('newton', tau still frozen).
    """
    K, rho, mu = par.K, par.rho, par.mu
    E, N = D.shape[0], D.shape[-1]
    Om = omega_diag(K, par.omega)
    w = vol / 4.0
    dq = _ein("qa,eafm->eqfm", QP_BARY, D)                        # values at qp
    g = np.matmul(np.swapaxes(grads, 1, 2), D.reshape(E, 4, -1)).reshape(E, 3, 4, N)
    conv = _conv(A, g[:, :, :3])                                   # A_j d_j u_i
    if variant == "newton":
        Ad = toeplitz(dq[:, :, :3])                                # A_j(delta u)
        conv = conv + _conv(Ad, newton["gu"])
    gp = g[:, :, 3][:, None, :, :]                                 # (e,1,3,N) d_i p
    Lm = rho * Om * dq[:, :, :3] + rho * conv

    def tmul(X):                                                   # tau @ X_i
        return np.swapaxes(np.matmul(tau, np.swapaxes(X, -1, -2)), -1, -2)

    if variant == "picard_nols":
        z_mom = tmul(Lm)
        z_con = tmul(np.broadcast_to(gp, Lm.shape))
    else:
        z_mom = tmul(Lm + gp)
        z_con = z_mom
    out = np.zeros(D.shape, dtype=complex)
    wq = w[:, None, None, None]
    # Galerkin terms
    out[:, :, :3] += wq * _ein("qa,eqim->eaim", QP_BARY, rho * Om * dq[:, :, :3] + rho * conv)
    out[:, :, :3] -= _ein("eai,em->eaim", grads * w[:, None, None], dq[:, :, 3].sum(axis=1))
    out[:, :, :3] += mu * np.matmul(grads * vol[:, None, None],
                                    g[:, :, :3].reshape(E, 3, -1)).reshape(E, 4, 3, N)
    out[:, :, 3] += w[:, None, None] * QP_BARY.sum(axis=0)[None, :, None] * \
        (g[:, 0, 0] + g[:, 1, 1] + g[:, 2, 2])[:, None, :]
    # least-squares terms: (-Omega N_A + A_j dN_A/dx_j) tau L_i and (1/rho) dN_A/dx_i tau L_i
    Az = np.matmul(A, np.swapaxes(z_mom, -1, -2)[:, :, None])     # (e,q,j,N,3i)
    if variant == "newton":
        Az = Az + np.matmul(Ad, np.swapaxes(newton["Z"], -1, -2)[:, :, None])
    X = (wq[..., None] * Az).sum(axis=1)                          # (e,j,N,3i)
    out[:, :, :3] += np.swapaxes(np.matmul(grads, X.reshape(E, 3, -1)).reshape(E, 4, N, 3), -1, -2)
    out[:, :, :3] -= wq * _ein("qa,eqim->eaim", QP_BARY, Om * z_mom)
    out[:, :, 3] += _ein("eai,eim->eam", grads * (w / rho)[:, None, None], z_con.sum(axis=1))
    if shift:
        out[:, :, :3] += shift * wq * _ein("qa,eqim->eaim", QP_BARY, dq[:, :, :3])
    return out


def _face_geometry(xyz, tris):
    X = xyz[tris]
    nv = np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0])
    nn = np.linalg.norm(nv, axis=1)
    return nv / nn[:, None], 0.5 * nn


def _face_negpart(par, xyz, C):
    tris = par.neumann_tris
    nhat, _ = _face_geometry(xyz, tris)
    uf = _ein("qa,fain->fqin", FACE_QP_BARY, C[tris][:, :, :3])
    un = _ein("fi,fqin->fqn", nhat, uf)
    return _negpart(toeplitz(un))


def _face_apply(par, xyz, Aneg, D, include_h):
    """Backflow (and Neumann traction) terms of the momentum rows."""
    tris = par.neumann_tris
    nhat, area = _face_geometry(xyz, tris)
    uf = _ein("qa,fain->fqin", FACE_QP_BARY, D[tris][:, :, :3])
    bu = _ein("fqmn,fqin->fqim", Aneg, uf)
    out = np.zeros((tris.shape[0], 3, 4, par.N), dtype=complex)
    out[:, :, :3] = -0.5 * par.rho * par.backflow_beta * _ein(
        "f,qa,fqim->faim", area / 3.0, FACE_QP_BARY, bu)
    if include_h and par.neumann_h is not None:
        h = slots_to_modes(np.asarray(par.neumann_h), par.K)
        out[:, :, :3] -= _ein("f,fi,fm->fim", area / 3.0, nhat, h)[:, None]
    return out


# ------------------------------------------------------------ public calls
def residual(par: Params, xyz, tets, y, frozen=None, raw=False):
    """Masked residual of eq. Rmc (plus backflow) in slot layout.

    frozen: optional linearization whose tau / A / |A_n|_- are used instead of
    the ones at y ('tau' -> tau and |A_n|_- frozen; 'all' -> also A frozen).
    raw=True returns the unmasked complex residual (for symmetry checks).
    """
    K = par.K
    C = slots_to_modes(np.asarray(y, dtype=float), K)
    grads, vol, G = geometry(xyz, tets)
    R = np.zeros(C.shape, dtype=complex)
    mode = None if frozen is None else frozen[0]
    lin = None if frozen is None else frozen[1]
    for sl in _chunks(tets.shape[0]):
        U = C[tets[sl]]
        uq = _ein("qa,eaim->eqim", QP_BARY, U[:, :, :3])
        if mode == "all":
            A = toeplitz(lin["uq"][sl])
        else:
            A = toeplitz(uq)
        if mode in ("tau", "all"):
            tau = lin["tau"][sl]
        else:
            tau = tau_from_velocity(uq, G[sl][:, None], par.nu, par.C_I)
        contrib = _element_apply(par, grads[sl], vol[sl], A, tau, U)
        np.add.at(R, tets[sl], contrib)
    if par.neumann_tris is not None and len(par.neumann_tris):
        Aneg = lin["Aneg"] if mode in ("tau", "all") else _face_negpart(par, xyz, C)
        np.add.at(R, par.neumann_tris, _face_apply(par, xyz, Aneg, C, True))
    if raw:
        return R
    _mask_rows(par, R)
    return modes_to_slots(R, K)


def linearize(par: Params, xyz, tets, y):
    """Quantities frozen for the tangent: velocity modes at the quadrature
    points (for A_i), tau, grad u, Z = tau L_i(u), and |A_n|_- on faces."""
    K = par.K
    C = slots_to_modes(np.asarray(y, dtype=float), K)
    grads, vol, G = geometry(xyz, tets)
    E, N = tets.shape[0], par.N
    lin = dict(uq=np.empty((E, 4, 3, N), complex), tau=np.empty((E, 4, N, N), complex),
               gu=np.empty((E, 3, 3, N), complex), Z=np.empty((E, 4, 3, N), complex))
    Om = omega_diag(K, par.omega)
    for sl in _chunks(E):
        U = C[tets[sl]]
        uq = _ein("qa,eaim->eqim", QP_BARY, U[:, :, :3])
        g = _ein("eaj,eafm->ejfm", grads[sl], U)
        A = toeplitz(uq)
        tau = tau_from_velocity(uq, G[sl][:, None], par.nu, par.C_I)
        conv = _conv(A, g[:, :, :3])
        L = par.rho * Om * uq + par.rho * conv + g[:, :, 3][:, None, :, :]
        lin["uq"][sl] = uq
        lin["tau"][sl] = tau
        lin["gu"][sl] = g[:, :, :3]
        lin["Z"][sl] = np.swapaxes(np.matmul(tau, np.swapaxes(L, -1, -2)), -1, -2)
    if par.neumann_tris is not None and len(par.neumann_tris):
        lin["Aneg"] = _face_negpart(par, xyz, C)
    return lin


def _shift(par, dt_pseudo, c1=1.5):
    return c1 * par.rho / dt_pseudo if (dt_pseudo is not None and dt_pseudo > 0) else 0.0


def jv(par: Params, xyz, tets, lin, v, variant="newton", dt_pseudo=None):
    """Masked tangent-vector product in slot layout (input masked too)."""
    K = par.K
    v = np.array(v, dtype=float)
    v[par.dirichlet_nodes, :3, :] = 0.0
    D = slots_to_modes(v, K)
    grads, vol, _ = geometry(xyz, tets)
    R = np.zeros(D.shape, dtype=complex)
    sh = _shift(par, dt_pseudo)
    for sl in _chunks(tets.shape[0]):
        A = toeplitz(lin["uq"][sl])
        nw = dict(gu=lin["gu"][sl], Z=lin["Z"][sl]) if variant == "newton" else None
        contrib = _element_apply(par, grads[sl], vol[sl], A, lin["tau"][sl], D[tets[sl]],
                                 variant=variant, newton=nw, shift=sh)
        np.add.at(R, tets[sl], contrib)
    if par.neumann_tris is not None and len(par.neumann_tris):
        np.add.at(R, par.neumann_tris, _face_apply(par, xyz, lin["Aneg"], D, False))
    _mask_rows(par, R)
    return modes_to_slots(R, K)


# ------------------------------------------- assembled tangent blocks (K_mat)
def picard_blocks(par: Params, xyz, tets, lin, sl=slice(None)):
    """Element blocks of eq. K_mat, complex (Ec, 4, 4, [3,] N, N)."""
    K, rho, mu = par.K, par.rho, par.mu
    N = par.N
    grads, vol, _ = geometry(xyz, tets[sl])
    w = vol / 4.0
    Om = np.diag(omega_diag(K, par.omega))
    A = toeplitz(lin["uq"][sl])                                    # (e,q,j,N,N)
    tau = lin["tau"][sl]
    I = np.eye(N)
    lam = QP_BARY
    # trial operator T_B = Omega N_B + A_k dN_B/dx_k, test operator P_A = -Omega N_A + A_k dN_A/dx_k
    AdN = _ein("eqkmn,ebk->eqbmn", A, grads)
    T = _ein("qb,mn->qbmn", lam, Om)[None] + AdN
    P = -_ein("qa,mn->qamn", lam, Om)[None] + AdN
    Kb = (_ein("e,qa,qb,mn->eabmn", w, lam, lam, rho * Om)
          + rho * _ein("e,qa,eqbmn->eabmn", w, lam, AdN)
          + mu * _ein("e,eak,ebk,mn->eabmn", vol, grads, grads, I)
          + rho * _ein("e,eqamk,eqkl,eqbln->eabmn", w, P, tau, T))
    Gb = (-_ein("e,eai,qb,mn->eabimn", w, grads, lam, I)
          + _ein("e,eqamk,eqkn,ebi->eabimn", w, P, tau, grads))
    Db = (_ein("e,qa,ebj,mn->eabjmn", w, lam, grads, I)
          + _ein("e,eaj,eqmk,eqbkn->eabjmn", w, grads, tau, T))
    Lb = _ein("e,eak,eqmn,ebk->eabmn", w / rho, grads, tau, grads)
    return Kb, Gb, Db, Lb


def picard_matvec(par: Params, xyz, tets, lin, v):
    """H v assembled block by block from eq. K_mat (plus the frozen backflow
    face term), masked like ``jv``."""
    K = par.K
    v = np.array(v, dtype=float)
    v[par.dirichlet_nodes, :3, :] = 0.0
    D = slots_to_modes(v, K)
    R = np.zeros(D.shape, dtype=complex)
    for sl in _chunks(tets.shape[0]):
        Kb, Gb, Db, Lb = picard_blocks(par, xyz, tets, lin, sl)
        Dn = D[tets[sl]]
        out = np.zeros(Dn.shape, dtype=complex)
        out[:, :, :3] += _ein("eabmn,ebin->eaim", Kb, Dn[:, :, :3])
        out[:, :, :3] += _ein("eabimn,ebn->eaim", Gb, Dn[:, :, 3])
        out[:, :, 3] += _ein("eabjmn,ebjn->eam", Db, Dn[:, :, :3])
        out[:, :, 3] += _ein("eabmn,ebn->eam", Lb, Dn[:, :, 3])
        np.add.at(R, tets[sl], out)
    if par.neumann_tris is not None and len(par.neumann_tris):
        np.add.at(R, par.neumann_tris, _face_apply(par, xyz, lin["Aneg"], D, False))
    _mask_rows(par, R)
    return modes_to_slots(R, K)


def jacobian_diagonal(par: Params, xyz, tets, lin, dt_pseudo=None):
    """Diagonal of the Picard tangent in slot layout (1 on masked slots).

    For an R-linear complex map with block H, d Re r_k / d Re y_k =
    Re(H_kk + H_k,-k) and d Im r_k / d Im y_k = Re(H_kk - H_k,-k)."""
    K, N = par.K, par.N
    n_nodes = xyz.shape[0]
    Hd = np.zeros((n_nodes, 4, N, N), dtype=complex)
    grads, vol, _ = geometry(xyz, tets)
    sh = _shift(par, dt_pseudo)
    for sl in _chunks(tets.shape[0]):
        Kb, _, _, Lb = picard_blocks(par, xyz, tets, lin, sl)
        ar = np.arange(4)
        KA = Kb[:, ar, ar]                                  # (e, a, N, N)
        LA = Lb[:, ar, ar]
        if sh:
            KA = KA + sh * _ein("e,qa,mn->eamn", vol[sl] / 4.0, QP_BARY ** 2, np.eye(N))
        blk = np.zeros((KA.shape[0], 4, 4, N, N), dtype=complex)
        blk[:, :, 0] = blk[:, :, 1] = blk[:, :, 2] = KA
        blk[:, :, 3] = LA
        np.add.at(Hd, tets[sl], blk)
    if par.neumann_tris is not None and len(par.neumann_tris):
        tris = par.neumann_tris
        _, area = _face_geometry(xyz, tris)
        fb = -0.5 * par.rho * par.backflow_beta * _ein(
            "f,qa,fqmn->famn", area / 3.0, FACE_QP_BARY ** 2, lin["Aneg"])
        blk = np.zeros((tris.shape[0], 3, 4, N, N), dtype=complex)
        blk[:, :, :3] = fb[:, :, None]
        np.add.at(Hd, tris, blk)
    k = np.arange(1, K + 1)
    d = np.empty((n_nodes, 4, 2 * K + 2))
    d[..., 0] = Hd[..., K, K].real
    d[..., 1] = 1.0
    d[..., 2::2] = (Hd[..., K + k, K + k] + Hd[..., K + k, K - k]).real
    d[..., 3::2] = (Hd[..., K + k, K + k] - Hd[..., K + k, K - k]).real
    d[par.dirichlet_nodes, :3, :] = 1.0
    return d


# ------------------------------------------------------------------ solver
def gmres(matvec, b, tol, restart=100, maxiter=10000, precond=None, x0=None):
    """Right-preconditioned restarted GMRES (modified Gram-Schmidt, Givens)."""
    shape = b.shape
    b = b.ravel()
    x = np.zeros_like(b) if x0 is None else x0.ravel().copy()
    Minv = (lambda r: r) if precond is None else (lambda r: precond.ravel() * r)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x.reshape(shape), 0
    its = 0
    while its < maxiter:
        r = b - matvec(x.reshape(shape)).ravel()
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            break
        m = restart
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(m):
            w = matvec(Minv(V[j]).reshape(shape)).ravel()
            its += 1
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_used = j + 1
            if abs(g[j + 1]) <= tol * bnorm or its >= maxiter:
                break
        yk = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + Minv(V[:j_used].T @ yk)
        if abs(g[j_used]) <= tol * bnorm:
            break
    return x.reshape(shape), its


def solve(par: Params, xyz, tets, y0, rtol=1e-8, lin_rtol=0.05, restart=100,
          max_newton=50, variant="newton", dt_pseudo=None, verbose=False):
    """Newton-Raphson (or one Newton step per pseudo-time step) with GMRES,
    stopped at ||r|| < rtol ||r^0|| (remarks after eq. K_mat)."""
    y = np.array(y0, dtype=float)
    y[..., 1] = 0.0
    r = residual(par, xyz, tets, y)
    r0 = np.linalg.norm(r)
    hist = [r0]
    n_mv = 0
    for it in range(max_newton):
        if np.linalg.norm(r) <= rtol * r0:
            break
        lin = linearize(par, xyz, tets, y)
        d = jacobian_diagonal(par, xyz, tets, lin, dt_pseudo)
        dy, its = gmres(lambda v: jv(par, xyz, tets, lin, v, variant, dt_pseudo), -r,
                        lin_rtol, restart, precond=1.0 / d)
        n_mv += its
        dy[par.dirichlet_nodes, :3, :] = 0.0
        dy[..., 1] = 0.0
        y = y + dy
        r = residual(par, xyz, tets, y)
        hist.append(np.linalg.norm(r))
        if verbose:
            print(f"newton {it}: |r|/|r0| = {hist[-1] / r0:.3e}  gmres {its}")
    return y, dict(history=np.array(hist), matvecs=n_mv, newton_iters=len(hist) - 1,
                   rel_residual=hist[-1] / r0)
