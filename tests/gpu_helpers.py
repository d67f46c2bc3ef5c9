"""Shared helpers of the GPU parity tests (not a test module)."""
import sys

import numpy as np

import oracle as O


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rand_state(prob, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    y = scale * rng.standard_normal((prob.mesh.n_nodes, 4, 2 * prob.K + 2))
    y[..., 1] = 0.0
    y[prob.dirichlet_nodes, :3] = prob.dirichlet_values
    return y


def rand_dir(prob, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((prob.mesh.n_nodes, 4, 2 * prob.K + 2))
    v[..., 1] = 0.0
    return v


def tau_complex_to_real(tau_c, K):
    """Matrix of the oracle's complex tau in the real orthonormal basis
    (c_0, sqrt2 Re c_1, sqrt2 Im c_1, ...): Re(Phi^H tau Phi)."""
    n = 2 * K + 1
    Phi = np.zeros((n, n), complex)      # columns: x basis vectors as complex modes
    Phi[K, 0] = 1.0
    for k in range(1, K + 1):
        Phi[K + k, 2 * k - 1] = Phi[K - k, 2 * k - 1] = 1 / np.sqrt(2)
        Phi[K + k, 2 * k] = 1j / np.sqrt(2)
        Phi[K - k, 2 * k] = -1j / np.sqrt(2)
    return np.einsum("ma,...mn,nb->...ab", np.conj(Phi), tau_c, Phi).real


def unpack(packed, n):
    out = np.zeros(packed.shape[:-1] + (n, n))
    iu = np.triu_indices(n)
    out[..., iu[0], iu[1]] = packed
    out[..., iu[1], iu[0]] = packed
    return out


def rel_err(a, b):
    d = np.linalg.norm((a - b).ravel())
    s = max(np.linalg.norm(b.ravel()), 1e-300)
    return d / s


def subset_for_nodes(prob, nodes):
    """Elements and Neumann faces incident to `nodes`: the oracle evaluated on
    them gives complete rows for those nodes."""
    tets = prob.mesh.tets
    sel = np.isin(tets, nodes).any(axis=1)
    tris = prob.neumann_tris
    fsel = np.isin(tris, nodes).any(axis=1) if tris is not None and len(tris) else None
    return sel, fsel


def oracle_params(prob, tris=None):
    par = O.Params.from_problem(prob)
    if tris is not None:
        par.neumann_tris = tris
        if prob.neumann_h is not None:
            par.neumann_h = prob.neumann_h
    return par
