"""Learned warm start on the GPU, through the C ABI.

* Network gradients (forward and backward kernels) against the FP64
  reference of oracle/mlp.py on the same parameters and data, with ragged
  tiles (width 40, batch 20, 10 outputs).  FP32 MFMA: the products sum at
  most 48 terms rounded to FP32 (u = 6.0e-8) -> TOL_F32 = 1e-4 of the largest
  gradient entry.  bf16 MFMA: every operand is rounded to bf16
  (u = 2^-8 = 3.9e-3) before FP32 accumulation; entries carry a few u of
  relative error, so the bound is 5e-2 of the largest entry (max-norm) and
  2e-2 relative in L2.
* Adam steps against the reference from the GPU's own gradient (1e-6).
* Greedy reduced basis and projection against the reference (1e-10).
* End to end on a family of pipe problems: solved members train the
  network; for held-out members Newton-GMRES from the prediction needs fewer
  Newton steps than from the plain initial guess, reaches the same absolute
  residual, and the oracle's residual confirms one solution.
"""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
from tests.gpu_helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu


def _f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _grad_case(precision):
    import torch
    import paper_2311_09465_amd as T
    rng = np.random.default_rng(8)
    net = T.MLP(8, 40, 3, 10, precision=precision, seed=5)
    x = rng.standard_normal((20, 8)).astype(np.float32)
    t = rng.standard_normal((20, 10)).astype(np.float32)
    loss = net.gradient(_f32(x), _f32(t))
    torch.cuda.synchronize()
    g = net.get_grad().astype(np.float64)
    theta = net.get_params().astype(np.float64)
    lr, gr = OM.loss_and_gradient(theta, net.dims, x.astype(np.float64), t.astype(np.float64))
    return loss, g, lr, gr


def test_mlp_gradient_f32_matches_oracle():
    log("[gpu] mlp gradient f32")
    loss, g, lr, gr = _grad_case("f32")
    assert abs(loss - lr) <= 1e-5 * abs(lr)
    assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()


def test_mlp_gradient_bf16_matches_oracle():
    log("[gpu] mlp gradient bf16")
    loss, g, lr, gr = _grad_case("bf16")
    emax = np.abs(g - gr).max() / np.abs(gr).max()
    el2 = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    log(f"[gpu]   bf16 gradient error max {emax:.2e} l2 {el2:.2e}; loss {abs(loss - lr) / lr:.2e}")
    assert abs(loss - lr) <= 1e-2 * abs(lr)
    assert emax <= 5e-2 and el2 <= 2e-2


def test_mlp_adam_matches_oracle():
    log("[gpu] mlp adam")
    import torch
    import paper_2311_09465_amd as T
    rng = np.random.default_rng(9)
    net = T.MLP(5, 24, 2, 7, precision="f32", seed=3)
    x, t = _f32(rng.standard_normal((9, 5))), _f32(rng.standard_normal((9, 7)))
    th = net.get_params().astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in (1, 2):
        net.gradient(x, t)
        g = net.get_grad().astype(np.float64)
        net.adam_step(1e-2)
        torch.cuda.synchronize()
        th, m, v = OM.adam_step(th, g, m, v, step, 1e-2)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - th).max() <= 1e-6 * np.abs(th).max()


def test_reduced_basis_matches_oracle():
    log("[gpu] reduced basis")
    import torch
    import paper_2311_09465_amd as T
    rng = np.random.default_rng(10)
    D, N = 3000, 14
    Q, _ = np.linalg.qr(rng.standard_normal((D, 6)))
    mean = rng.standard_normal(D)
    C = rng.standard_normal((N, 6)) * np.array([9.0, 5.0, 3.0, 2.0, 1.0, 0.5])
    Y = mean + C @ Q.T + 1e-3 * rng.standard_normal((N, D))
    Yd, md = to_dev(Y), to_dev(mean)
    Phi, picked = T.rb_greedy(Yd, md, 5)
    Po, pk = OM.greedy_basis(Y, mean, 5)
    assert picked == pk
    assert np.abs(to_host(Phi) - Po).max() <= 1e-10
    coef = to_host(T.rb_project(Phi, Yd, md))
    assert np.abs(coef - (Y - mean) @ Po.T).max() <= 1e-10 * np.abs(coef).max()
    y = torch.empty(D, dtype=torch.float64, device="cuda")
    T.rb_expand(Phi, to_dev(coef[3]), md, y)
    assert np.abs(to_host(y) - (mean + coef[3] @ Po)).max() <= 1e-10 * np.abs(mean).max()


def test_reduced_basis_more_snapshots_than_one_pass():
    """N = 1,100 snapshots: the coefficients of the snapshots on each new basis
    vector are formed 1,024 rows at a time; same result as the reference."""
    log("[gpu] reduced basis, 1,100 snapshots")
    import paper_2311_09465_amd as T
    rng = np.random.default_rng(12)
    D, N = 400, 1100
    Q, _ = np.linalg.qr(rng.standard_normal((D, 5)))
    mean = rng.standard_normal(D)
    C = rng.standard_normal((N, 5)) * np.array([7.0, 4.0, 2.5, 1.5, 1.0])
    Y = mean + C @ Q.T + 1e-3 * rng.standard_normal((N, D))
    Phi, picked = T.rb_greedy(to_dev(Y), to_dev(mean), 4)
    Po, pk = OM.greedy_basis(Y, mean, 4)
    assert picked == pk
    assert np.abs(to_host(Phi) - Po).max() <= 1e-10


def test_learned_warm_start_on_pipe_family():
    import torch
    import paper_2311_09465_amd as T
    from paper_2311_09465_amd.warmstart import WarmStart, fix_dirichlet
    from workloads import pipe_family, initial_guess
    probs, feats = pipe_family(104, K=3, seed=7, n_rings=2, n_layers=8)
    train, test = list(range(96)), list(range(96, 104))
    log(f"[gpu] learned warm start: {len(train)} training solves on {probs[0].mesh.n_tets} tets")
    opts = dict(lin_rtol=0.05, restart=30, max_newton=60)
    solvers = [T.Solver.from_problem(probs[i], stream=torch.cuda.Stream()) for i in train]
    ys = [to_dev(initial_guess(probs[i])) for i in train]
    torch.cuda.synchronize()
    rc, st, _ = T.solve_batch(solvers, ys, rtol=1e-9, max_concurrent=8, **opts)
    assert rc == 0
    Y = torch.stack([y.view(-1) for y in ys]).contiguous()
    del solvers
    ws = WarmStart.fit(feats[train], Y, r=24, steps=1500, lr=1e-3, seed=1)
    log(f"[gpu]   train loss {ws.train_loss:.3e}")
    cold_it, warm_it = [], []
    for i in test:
        p = probs[i]
        s = T.Solver.from_problem(p)
        y0 = to_dev(initial_guess(p))
        r_cold = s.solve(y0.clone(), rtol=1.0, max_newton=0)["r0_norm"]
        yp = fix_dirichlet(ws.predict(feats[i:i + 1], [y0])[0], y0, p.dirichlet_nodes)
        r_warm = s.solve(yp.clone(), rtol=1.0, max_newton=0)["r0_norm"]
        assert r_warm < r_cold
        yc = y0.clone()
        sc = s.solve(yc, rtol=1e-8, **opts)
        sw = s.solve(yp, rtol=1e-8 * r_cold / r_warm, **opts)
        assert sc["status"] == 0 and sw["status"] == 0
        cold_it.append(sc["newton_iters"])
        warm_it.append(sw["newton_iters"])
        log(f"[gpu]   member {i}: |r| prediction / initial guess {r_warm / r_cold:.2e}, "
            f"newton {sc['newton_iters']} -> {sw['newton_iters']}")
        if i == test[0]:
            par = O.Params.from_problem(p)
            r0 = np.linalg.norm(O.residual(par, p.mesh.xyz, p.mesh.tets, to_host(y0)))
            r = np.linalg.norm(O.residual(par, p.mesh.xyz, p.mesh.tets, to_host(yp)))
            assert r <= 1e-8 * r0 * 1.01
    assert np.mean(warm_it) < np.mean(cold_it)
