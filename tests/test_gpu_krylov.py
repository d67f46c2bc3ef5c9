"""GMRES with delayed classical Gram-Schmidt past one tile of basis vectors.

The reduction of the delayed variant runs on a grid of (chunk, tile of 32
basis vectors); restarts up to 128 use it, larger ones the two-pass
classical Gram-Schmidt.  Both orthogonalize to working accuracy, so with the
same products (one Newton step of 70 preconditioned tangent products, no
restart) they produce the same iterate up to rounding: 1e-8 of its largest
entry (observed differences are orders of magnitude smaller).  The Newton
updates are then judged once more by the oracle's residual.
"""
import numpy as np
import pytest

import oracle as O
from workloads import cube_problem, initial_guess
from tests.gpu_helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_delayed_gmres_over_three_tiles_matches_two_pass():
    import torch
    import paper_2311_09465_amd as T
    prob = cube_problem(4, K=3)
    log("[gpu] delayed GMRES (restart 100, 70 products) vs two-pass (restart 150)")
    kw = dict(rtol=1e-300, lin_rtol=1e-300, max_newton=1, max_matvec=70)
    s = T.Solver.from_problem(prob)
    y0 = initial_guess(prob)
    ya, yb = to_dev(y0), to_dev(y0)
    torch.cuda.synchronize()
    sa = s.solve(ya, restart=100, **kw)
    sb = s.solve(yb, restart=150, **kw)
    a, b = to_host(ya), to_host(yb)
    err = np.abs(a - b).max() / np.abs(a).max()
    log(f"[gpu]   rel diff {err:.2e}, matvecs {sa['matvecs']} / {sb['matvecs']}")
    assert sa["matvecs"] == 70 and sb["matvecs"] == 70
    assert err <= 1e-8
    par = O.Params.from_problem(prob)
    r0 = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, y0))
    ra = np.linalg.norm(O.residual(par, prob.mesh.xyz, prob.mesh.tets, a))
    assert ra < r0


def _dense_newton_step(prob, y0):
    """y0 + dx with J dx = -r(y0) solved densely from the oracle's Picard
    tangent (columns of its product), masked slots left unchanged."""
    par = O.Params.from_problem(prob)
    xyz, tets = prob.mesh.xyz, prob.mesh.tets
    r = O.residual(par, xyz, tets, y0).ravel()
    lin = O.linearize(par, xyz, tets, y0)
    free = np.ones(y0.shape, bool)
    free[..., 1] = False
    free[prob.dirichlet_nodes, :3] = False
    idx = np.flatnonzero(free.ravel())
    J = np.empty((idx.size, idx.size))
    for c, j in enumerate(idx):
        e = np.zeros(y0.size)
        e[j] = 1.0
        J[:, c] = O.jv(par, xyz, tets, lin, e.reshape(y0.shape), "picard").ravel()[idx]
    y1 = y0.copy().ravel()
    y1[idx] += np.linalg.solve(J, -r[idx])
    return y1.reshape(y0.shape), idx.size


@pytest.mark.parametrize("n_tets,K,paths", [(1, 0, ((16, False), (32, True), (200, False))),
                                           (6, 1, ((100, False), (200, False)))])
def test_exhausted_krylov_space_all_paths_agree(n_tets, K, paths):
    """Restart at least the number of unknowns: the Krylov space is exhausted
    within one cycle (the delayed variant may meet u_j in span(Q) exactly).
    Delayed, two-pass and graph GMRES then give the exact Newton step, which
    is the oracle's dense solve (1e-8 of the largest entry)."""
    import torch
    import paper_2311_09465_amd as T
    from workloads import tiny_problem
    from tests.gpu_helpers import rand_state
    prob = tiny_problem(n_tets, K=K, seed=3)
    y0 = rand_state(prob, 5, 0.3)
    ref, nfree = _dense_newton_step(prob, y0)
    for m, graph in paths:
        assert m >= nfree
        log(f"[gpu] exhausted Krylov space: {n_tets} tets K={K} ({nfree} unknowns), restart {m}"
            f"{' graph' if graph else ''}")
        s = T.Solver.from_problem(prob)
        y = to_dev(y0)
        torch.cuda.synchronize()
        st = s.solve(y, rtol=1e-300, lin_rtol=1e-12, restart=m, max_newton=1, max_matvec=m,
                     gmres_graph=graph)
        got = to_host(y)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        log(f"[gpu]   matvecs {st['matvecs']}, rel diff to the dense step {err:.2e}")
        assert err <= 1e-8
        s.close()
