"""Segments: several problems of one mesh (one harmonic count, one set of
physical parameters, different inflow waveforms) in one context, solved in
lockstep (tsgls_set_segments / tsgls_solve_segments).  Each GMRES cycle is
one captured graph whose launches cover every segment, with per-segment
reductions and device-side least-squares updates.

* Each segment follows the graph-captured solve of its problem alone bit for
  bit: same status, Newton steps, products, residual history and the same
  final state, for the Picard and Newton tangents and the FP32 tangent, and
  when the Newton budget stops the solves before convergence.
* The lockstep solution of two segments is confirmed by the oracle's FP64
  residual (the other segments follow from the bitwise equality).
* Argument errors: a segment count that does not divide the nodes, elements
  that join two segments, options outside the graph-captured GMRES, and the
  unsegmented solver on a segmented context.
"""
import numpy as np
import pytest

import oracle as O
from workloads import womersley_problem, initial_guess
from workloads.problems import inlet_waveforms
from workloads.meshgen import pipe
from tests.gpu_helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu


def _family(K, n, seed=0):
    mesh = pipe(2, 8)
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.1, 1.0, size=n)
    return [womersley_problem(K=K, mesh=mesh,
                              waveform=inlet_waveforms(K, 100 + i, amps[i], n_inlets=1)[0])
            for i in range(n)]


def _lone(probs, opts):
    import torch
    import paper_2311_09465_amd as T
    out = []
    for p in probs:
        s = T.Solver.from_problem(p)
        y = to_dev(initial_guess(p))
        torch.cuda.synchronize()
        st = s.solve(y, gmres_graph=True, **opts)
        out.append((to_host(y), st))
        s.close()
    return out


def _segmented(probs, opts):
    import torch
    import paper_2311_09465_amd as T
    seg = T.SegmentSolver.from_problems(probs)
    y = to_dev(np.concatenate([initial_guess(p) for p in probs]))
    torch.cuda.synchronize()
    rc, stats, fin = seg.solve_segments(y, **opts)
    yh = to_host(y)
    seg.close()
    return rc, stats, fin, yh


@pytest.mark.parametrize("K,jac,prec,max_newton", [(3, "picard", "f64", 30), (2, "newton", "f64", 30),
                                                   (3, "picard", "f32", 30), (3, "picard", "f64", 2)])
def test_segments_follow_lone_solves_bit_for_bit(K, jac, prec, max_newton):
    log(f"[gpu] segments: 5 pipe waveforms K={K} {jac} {prec} max_newton={max_newton}")
    probs = _family(K, 5, seed=K)
    opts = dict(rtol=1e-9, lin_rtol=0.05, restart=16, max_newton=max_newton, jacobian=jac,
                tangent_precision=prec)
    lone = _lone(probs, opts)
    rc, stats, fin, yh = _segmented(probs, opts)
    nn = probs[0].mesh.n_nodes
    log(f"[gpu]   lone: steps {[s['newton_iters'] for _, s in lone]} products "
        f"{[s['matvecs'] for _, s in lone]}; segments finish at {np.round(fin, 3).tolist()} s")
    for i, (yl, sl) in enumerate(lone):
        sg = stats[i]
        for k in ("status", "newton_iters", "matvecs", "lin_unconverged", "history", "rel_residual"):
            assert sg[k] == sl[k], (i, k, sg[k], sl[k])
        assert np.array_equal(yh[i * nn:(i + 1) * nn], yl), i
    assert rc == (0 if all(s["status"] == 0 for _, s in lone) else 1)


def test_segmented_solutions_confirmed_by_oracle():
    log("[gpu] segments: 4 waveforms K=3, two solutions judged by the oracle")
    probs = _family(3, 4, seed=11)
    rc, stats, fin, yh = _segmented(probs, dict(rtol=1e-9, lin_rtol=0.05, restart=16, max_newton=30))
    assert rc == 0
    nn = probs[0].mesh.n_nodes
    for i in (0, 3):
        p = probs[i]
        par = O.Params.from_problem(p)
        r0 = np.linalg.norm(O.residual(par, p.mesh.xyz, p.mesh.tets, initial_guess(p)))
        r = np.linalg.norm(O.residual(par, p.mesh.xyz, p.mesh.tets, yh[i * nn:(i + 1) * nn]))
        log(f"[gpu]   segment {i}: oracle relative residual {r / r0:.2e}")
        assert r <= 1e-8 * r0


def test_segment_argument_errors():
    import torch
    import paper_2311_09465_amd as T
    log("[gpu] segments: argument errors")
    probs = _family(2, 2)
    s = T.Solver.from_problem(probs[0])
    with pytest.raises(T.TsglsError, match="divide"):
        s.set_segments(7 if s.n_nodes % 7 else 11)
    with pytest.raises(T.TsglsError, match="two segments"):
        s.set_segments(3)                 # one pipe split in three node blocks
    s.close()
    seg = T.SegmentSolver.from_problems(probs)
    y = to_dev(np.concatenate([initial_guess(p) for p in probs]))
    with pytest.raises(T.TsglsError, match="restart"):
        seg.solve_segments(y, restart=40)
    with pytest.raises(T.TsglsError, match="segments"):
        seg.solve(y)
    # one segment again: the ordinary solve works on the whole context
    seg.set_segments(1)
    torch.cuda.synchronize()
    st = seg.solve(y, rtol=1e-8, restart=16, max_newton=30)
    assert st["status"] == 0
    seg.close()
    other = _family(3, 1)[0]
    with pytest.raises(T.TsglsError, match="one mesh"):
        T.SegmentSolver.from_problems([probs[0], other])
