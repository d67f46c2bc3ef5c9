"""Boundary data and physical parameters for the synthetic workloads.

State layout used everywhere (oracle and library alike): ``y[node][field][slot]``
with fields (u1, u2, u3, p) and 2K+2 slots per field, slot 2k = Re c_k and
slot 2k+1 = Im c_k for k = 0..K, where a real periodic field is
f(t) = sum_{|k|<=K} c_k exp(i k omega t) and c_{-k} = conj(c_k)
(the real-valued unknowns of the paper's section on real-valued unknowns;
the identically-zero Im c_0 slot is kept).

Parameter conventions (paper, section "The case study"): Re = rho U D / mu and
Wo = D sqrt(rho omega / mu) with D the inlet diameter and U the mean inlet
velocity.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.special as sp

from .meshgen import Mesh, pipe, junction, cube_kuhn, _finish


@dataclasses.dataclass
class Problem:
    mesh: Mesh
    K: int
    rho: float
    mu: float
    omega: float
    C_I: float = 3.0
    backflow_beta: float = 0.5
    dirichlet_nodes: np.ndarray = None      # (nd,) int32, velocity prescribed
    dirichlet_values: np.ndarray = None     # (nd, 3, 2K+2) float64, slot layout
    neumann_tris: np.ndarray = None         # (nf, 3) int32, outward oriented
    neumann_h: Optional[np.ndarray] = None  # (nf, 2K+2) traction modes or None
    name: str = ""

    @property
    def n_slots(self) -> int:
        return 2 * self.K + 2

    @property
    def nu(self) -> float:
        return self.mu / self.rho


def initial_guess(prob: Problem) -> np.ndarray:
    """u = 0 inside, u = g on Dirichlet nodes, p = 0 (Newton-Raphson remarks)."""
    y = np.zeros((prob.mesh.n_nodes, 4, prob.n_slots))
    y[prob.dirichlet_nodes, :3, :] = prob.dirichlet_values
    return y


def _nodes_of(tris):
    return np.unique(np.asarray(tris).ravel())


def _complex_to_slots(c):
    """(..., K+1) complex modes k=0..K -> (..., 2K+2) slots."""
    s = np.empty(c.shape[:-1] + (2 * c.shape[-1],))
    s[..., 0::2] = c.real
    s[..., 1::2] = c.imag
    s[..., 1] = 0.0
    return s


# ---------------------------------------------------------------- Womersley
def womersley_exact_modes(xyz, K, R, L, rho, mu, omega, Qmodes):
    """Closed-form periodic pipe flow for prescribed flow-rate modes.

    Qmodes[k], k = 0..K: complex flow-rate Fourier coefficients.  Returns the
    state (n_nodes, 4, 2K+2) in slot layout: axial velocity u3 = U_k(r),
    p_k(z) = Gk (L - z) so that the traction vanishes at z = L.
    """
    nu = mu / rho
    r = np.sqrt(xyz[:, 0] ** 2 + xyz[:, 1] ** 2)
    U = np.zeros((xyz.shape[0], K + 1), dtype=complex)
    G = np.zeros(K + 1, dtype=complex)
    # mean mode: Poiseuille, -dp/dz = 8 mu Qbar / (pi R^4)
    ubar = Qmodes[0] / (np.pi * R * R)
    U[:, 0] = 2 * ubar * (1 - (r / R) ** 2)
    G[0] = 8 * mu * ubar / R ** 2
    for k in range(1, K + 1):
        if Qmodes[k] == 0:
            continue
        lam = (1j ** 1.5) * R * np.sqrt(k * omega / nu)
        j0 = sp.jv(0, lam)
        j1 = sp.jv(1, lam)
        fac = np.pi * R * R / (1j * rho * k * omega) * (1 - 2 * j1 / (lam * j0))
        G[k] = Qmodes[k] / fac
        U[:, k] = G[k] / (1j * rho * k * omega) * (1 - sp.jv(0, lam * r / R) / j0)
    y = np.zeros((xyz.shape[0], 4, 2 * K + 2))
    y[:, 2, :] = _complex_to_slots(U)
    P = G[None, :] * (L - xyz[:, 2])[:, None]
    y[:, 3, :] = _complex_to_slots(P)
    return y


def womersley_problem(n_rings=4, n_layers=16, K=3, Re=100.0, Wo=5.0, amp=0.5,
                      rho=1.0, R=1.0, L=4.0, waveform=None, mesh: Mesh = None) -> Problem:
    """Pipe, inlet flow Q(t) = Qbar (1 + amp sin(omega t)), mean velocity 1.

    waveform, if given, replaces the sinusoid: complex modes k = 0..K of
    Q(t)/Qbar (waveform[0] = 1), e.g. one row of inlet_waveforms."""
    if mesh is None:
        mesh = pipe(n_rings, n_layers, R, L)
    D, U = 2 * R, 1.0
    mu = rho * U * D / Re
    omega = (Wo / D) ** 2 * mu / rho
    Q = np.zeros(K + 1, dtype=complex)
    Q[0] = np.pi * R * R * U
    if waveform is not None:
        Q[1:] = Q[0] * np.asarray(waveform, dtype=complex)[1:K + 1]
    elif K >= 1:
        Q[1] = -1j * amp * Q[0] / 2
    exact = womersley_exact_modes(mesh.xyz, K, R, L, rho, mu, omega, Q)
    inlet = _nodes_of(mesh.faces["inlet"])
    wall = _nodes_of(mesh.faces["wall"])
    dn = np.union1d(inlet, wall).astype(np.int32)
    vals = np.zeros((dn.size, 3, 2 * K + 2))
    is_in = np.isin(dn, inlet) & ~np.isin(dn, wall)
    vals[is_in] = exact[dn[is_in], :3, :]
    prob = Problem(mesh=mesh, K=K, rho=rho, mu=mu, omega=omega,
                   dirichlet_nodes=dn, dirichlet_values=vals,
                   neumann_tris=mesh.faces["outlet"].astype(np.int32),
                   name=f"womersley_r{n_rings}_l{n_layers}_K{K}")
    prob.exact = exact
    prob.Qmodes = Q
    prob.R, prob.L = R, L
    return prob


# ----------------------------------------------------------------- junction
def inlet_waveforms(K, seed, amp=0.5, n_inlets=2):
    """Q(t)/Qbar = 1 + sum_k amp k^-2 cos(k omega t + phi_k), phi_k ~ U[0, 2pi).

    Returns complex modes (n_inlets, K+1) for k = 0..K, drawn from
    numpy.random.default_rng(seed) (PCG64): K phases for inlet 1, then inlet 2.
    """
    rng = np.random.default_rng(seed)
    out = np.zeros((n_inlets, K + 1), dtype=complex)
    for j in range(n_inlets):
        phi = rng.uniform(0.0, 2 * np.pi, size=K)
        a = amp if np.isscalar(amp) else amp[j]
        out[j, 0] = 1.0
        for k in range(1, K + 1):
            out[j, k] = 0.5 * a * k ** -2.0 * np.exp(1j * phi[k - 1])
    return out


def junction_problem(h=0.081, K=6, Re=500.0, Wo=10.0, seed=0, amp=0.5,
                     rho=1.0, mesh: Mesh = None, geom=None) -> Problem:
    """Cross junction; parabolic inflow per mode, mean velocity 1 in each inlet.

    Re and Wo use the larger inlet's diameter.  Outlets carry zero traction
    with backflow stabilisation; walls are no-slip.
    """
    from .meshgen import JUNCTION_DEFAULT
    g = dict(JUNCTION_DEFAULT)
    if geom:
        g.update(geom)
    if mesh is None:
        mesh = junction(h, **g)
    D = 2 * max(g["r_in1"], g["r_in2"])
    mu = rho * 1.0 * D / Re
    omega = (Wo / D) ** 2 * mu / rho
    wf = inlet_waveforms(K, seed, amp)
    wall = _nodes_of(mesh.faces["wall"])
    dn_list, val_list = [wall], [np.zeros((wall.size, 3, 2 * K + 2))]
    for j, (lab, rad, sgn) in enumerate((("in1", g["r_in1"], +1.0), ("in2", g["r_in2"], -1.0))):
        nodes = np.setdiff1d(_nodes_of(mesh.faces[lab]), wall)
        x = mesh.xyz[nodes]
        r2 = (x[:, 0] ** 2 + x[:, 1] ** 2) / rad ** 2
        prof = np.clip(2.0 * (1.0 - r2), 0.0, None)   # mean velocity 1
        v = np.zeros((nodes.size, 3, 2 * K + 2))
        v[:, 2, :] = sgn * prof[:, None] * _complex_to_slots(wf[j])[None, :]
        dn_list.append(nodes)
        val_list.append(v)
    dn = np.concatenate(dn_list).astype(np.int32)
    vals = np.concatenate(val_list)
    order = np.argsort(dn, kind="stable")
    nt = np.concatenate([mesh.faces["out1"], mesh.faces["out2"]]).astype(np.int32)
    prob = Problem(mesh=mesh, K=K, rho=rho, mu=mu, omega=omega,
                   dirichlet_nodes=dn[order], dirichlet_values=vals[order],
                   neumann_tris=nt, name=f"junction_h{h:g}_K{K}_s{seed}")
    prob.waveforms = wf
    return prob


# ----------------------------------------------------- pipe problem family
def pipe_family(n, K=3, seed=0, n_rings=4, n_layers=16, Re_range=(60.0, 140.0),
                Wo_range=(3.0, 7.0), mesh: Mesh = None):
    """n pipe problems on one mesh with seeded inflow waveforms
    1 + sum_k a k^-2 cos(k omega t + phi_k), a ~ U[0.1, 1], and Re, Wo drawn
    uniformly from the ranges.  Returns (problems, features [n][2K+2]) with
    features = (Re w_1..w_K, Im w_1..w_K, Re, Wo), w_k the waveform modes."""
    rng = np.random.default_rng(seed)
    if mesh is None:
        mesh = pipe(n_rings, n_layers)
    probs, feats = [], []
    for _ in range(n):
        a = rng.uniform(0.1, 1.0)
        Re = rng.uniform(*Re_range)
        Wo = rng.uniform(*Wo_range)
        wf = inlet_waveforms(K, int(rng.integers(1 << 31)), a, n_inlets=1)[0]
        probs.append(womersley_problem(K=K, Re=Re, Wo=Wo, waveform=wf, mesh=mesh))
        feats.append(np.concatenate([wf[1:].real, wf[1:].imag, [Re, Wo]]))
    return probs, np.asarray(feats)


# --------------------------------------------------------------- test cubes
def cube_problem(n=3, K=2, Re=50.0, Wo=3.0, rho=1.0, seed=0, amp=0.5) -> Problem:
    """Unit cube; inflow at x=0 (parabola-like bump per mode), outflow at x=1
    (zero traction + backflow), no-slip elsewhere.  For small parity cases."""
    mesh = cube_kuhn(n)
    xyz = mesh.xyz
    allf = np.concatenate(list(mesh.faces.values()))
    cen = xyz[allf].mean(axis=1)
    lab = np.where(cen[:, 0] < 1e-12, "inlet", np.where(cen[:, 0] > 1 - 1e-12, "outlet", "wall"))
    mesh.faces = {k: allf[lab == k] for k in ("inlet", "outlet", "wall")}
    mu = rho * 1.0 / Re
    omega = Wo ** 2 * mu / rho
    wall = _nodes_of(mesh.faces["wall"])
    inl = np.setdiff1d(_nodes_of(mesh.faces["inlet"]), wall)
    x = xyz[inl]
    bump = 16 * x[:, 1] * (1 - x[:, 1]) * x[:, 2] * (1 - x[:, 2])
    wf = inlet_waveforms(K, seed, amp, n_inlets=1)[0]
    v = np.zeros((inl.size, 3, 2 * K + 2))
    v[:, 0, :] = bump[:, None] * _complex_to_slots(wf)[None, :]
    dn = np.concatenate([wall, inl]).astype(np.int32)
    vals = np.concatenate([np.zeros((wall.size, 3, 2 * K + 2)), v])
    order = np.argsort(dn)
    return Problem(mesh=mesh, K=K, rho=rho, mu=mu, omega=omega,
                   dirichlet_nodes=dn[order], dirichlet_values=vals[order],
                   neumann_tris=mesh.faces["outlet"].astype(np.int32),
                   name=f"cube{n}_K{K}")


def tiny_problem(n_tets=1, K=1, seed=0, rho=1.3, mu=0.05, omega=0.7) -> Problem:
    """1, 2 or 6 tets with a few Dirichlet nodes and one Neumann face; for
    finite-difference Jacobian checks."""
    from .meshgen import Mesh as _M, boundary_faces
    rng = np.random.default_rng(seed)
    if n_tets == 1:
        xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
        tets = np.array([[0, 1, 2, 3]])
    elif n_tets == 2:
        xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
        tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]])
    else:
        m = cube_kuhn(1)
        xyz, tets = m.xyz, m.tets
    xyz = xyz + 0.05 * rng.standard_normal(xyz.shape)
    from .meshgen import orient_positive
    tets = orient_positive(xyz, tets.astype(np.int64)).astype(np.int32)
    bf = boundary_faces(xyz, tets)
    mesh = _M(xyz=xyz, tets=tets, faces={"all": bf})
    dn = np.array([0], dtype=np.int32)
    vals = 0.3 * rng.standard_normal((1, 3, 2 * K + 2))
    vals[:, :, 1] = 0
    return Problem(mesh=mesh, K=K, rho=rho, mu=mu, omega=omega,
                   dirichlet_nodes=dn, dirichlet_values=vals,
                   neumann_tris=bf[:1].astype(np.int32), name=f"tiny{n_tets}_K{K}")
