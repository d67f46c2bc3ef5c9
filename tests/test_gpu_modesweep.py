"""Mode sweep on the 200k-tet junction (h = 0.081): for K = 3, 7, 15, 31 the
library's residual and tangent product (FP64 and the FP32 element operator)
are compared with the oracle on sampled nodes, whose rows the oracle gives
exactly from the elements and Neumann faces around them.  The errors against
the oracle are printed per K; tolerances as in the small-mesh parity tests
(FP64 1e-11, FP32 tangent 16 units of FP32 roundoff = 1e-6, relative to the
largest sampled entry).  K = 31 runs the LDS-staged large-K kernels.
"""
import numpy as np
import pytest

import oracle as O
from workloads import junction_problem, initial_guess
from tests.gpu_helpers import log, to_dev, to_host, subset_for_nodes

pytestmark = pytest.mark.gpu

TOL = 1e-11
TOL32 = 1e-6


@pytest.mark.parametrize("K", [3, 7, 15, 31])
def test_mode_sweep_junction_200k(K):
    import paper_2311_09465_amd as T
    log(f"[gpu] mode sweep junction h=0.081 K={K}: building mesh")
    prob = junction_problem(h=0.081, K=K, Re=500.0, Wo=10.0, seed=1)
    rng = np.random.default_rng(100 + K)
    y = initial_guess(prob)
    noise = 0.05 * rng.standard_normal(y.shape)
    noise[..., 1] = 0.0
    noise[prob.dirichlet_nodes, :3] = 0.0
    y = y + noise
    v = rng.standard_normal(y.shape)
    v[..., 1] = 0.0
    nn = prob.mesh.n_nodes
    outlet = np.unique(prob.neumann_tris)
    dnodes = np.asarray(prob.dirichlet_nodes)
    free = np.setdiff1d(np.arange(nn), np.union1d(outlet, dnodes))
    nodes = np.unique(np.concatenate([rng.choice(free, 16, replace=False),
                                      rng.choice(outlet, 4, replace=False)]))
    sel, fsel = subset_for_nodes(prob, nodes)
    par = O.Params.from_problem(prob)
    par.neumann_tris = prob.neumann_tris[fsel]
    tets = prob.mesh.tets[sel]
    xyz = prob.mesh.xyz
    log(f"[gpu]   {prob.mesh.n_tets} tets, {nn} nodes; {nodes.size} sampled nodes")
    s = T.Solver.from_problem(prob)
    r = to_dev(np.zeros_like(y))
    s.linearize(to_dev(y), r)
    rg = to_host(r)
    out = to_dev(np.zeros_like(y))
    s.jv(to_dev(v), out, "picard")
    j64 = to_host(out)
    s.jv(to_dev(v), out, "picard", precision="f32")
    j32 = to_host(out)
    lin = O.linearize(par, xyz, tets, y)
    rr = O.residual(par, xyz, tets, y)
    jr = O.jv(par, xyz, tets, lin, v, "picard")

    def err(g, ref):
        a, b = g[nodes], ref[nodes]
        return np.abs(a - b).max() / np.abs(b).max()

    er, e64, e32 = err(rg, rr), err(j64, jr), err(j32, jr)
    log(f"[gpu]   K={K} residual {er:.2e}  jv f64 {e64:.2e}  jv f32 {e32:.2e}")
    assert er <= TOL and e64 <= TOL and e32 <= TOL32
