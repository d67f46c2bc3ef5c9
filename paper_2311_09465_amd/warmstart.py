"""Learned warm start for Newton-GMRES (library calls only).

A family of problems on one mesh is described by a short feature vector per
member (inflow Fourier coefficients, Re, Wo).  From solved members the
library builds a greedy reduced basis of the solutions (tsgls_rb_greedy)
and trains a tanh network (tsgls_mlp_*) from the features to the
solutions' reduced-basis coefficients.  For a new member the prediction is
mean + Phi^T coef, with the Dirichlet rows copied from the member's own
initial guess (so the boundary data are exact); Newton-GMRES then solves
from it and remains the judge: a prediction whose residual exceeds the
initial guess's is discarded.

Host-side arithmetic is limited to standardizing the few features and
coefficients per member (mean and spread over the training set).
"""
from __future__ import annotations

import numpy as np

from . import MLP, rb_expand, rb_greedy, rb_project, solve_batch   # noqa: F401


class WarmStart:
    def __init__(self, Phi, mean, net, xs, ts):
        self.Phi, self.mean, self.net = Phi, mean, net
        self.x_mu, self.x_sd = xs
        self.t_mu, self.t_sd = ts

    @classmethod
    def fit(cls, features, Y, r=48, width=512, n_hidden=3, steps=3000, lr=1e-3,
            precision="bf16", seed=0, log=None):
        """features: host [N][F]; Y: solutions, float64 CUDA [N][D]."""
        import torch
        N, D = Y.shape
        w = torch.full((min(N, 1024),), 1.0 / N, dtype=torch.float64, device=Y.device)
        acc = torch.zeros(D, dtype=torch.float64, device=Y.device)
        mean = torch.empty(D, dtype=torch.float64, device=Y.device)
        for i0 in range(0, N, 1024):                        # mean = sum_i Y_i / N, 1,024 rows a pass
            i1 = min(N, i0 + 1024)
            rb_expand(Y[i0:i1], w[:i1 - i0], acc, mean)
            acc.copy_(mean)
        Phi, _ = rb_greedy(Y, mean, r)
        coef = rb_project(Phi, Y, mean).cpu().numpy()
        F = np.asarray(features, dtype=np.float64)
        x_mu, x_sd = F.mean(axis=0), F.std(axis=0) + 1e-12
        t_mu, t_sd = coef.mean(axis=0), coef.std(axis=0) + 1e-30
        x = torch.from_numpy(((F - x_mu) / x_sd).astype(np.float32)).cuda()
        t = torch.from_numpy(((coef - t_mu) / t_sd).astype(np.float32)).cuda()
        net = MLP(F.shape[1], width, n_hidden, Phi.shape[0], precision=precision, seed=seed)
        hist = []
        for it in range(steps):
            loss = net.gradient(x, t)
            net.adam_step(lr)
            if it % 100 == 0 or it == steps - 1:
                hist.append((it, loss))
                if log:
                    log(f"train step {it}: loss {loss:.4e}")
        ws = cls(Phi, mean, net, (x_mu, x_sd), (t_mu, t_sd))
        ws.history = hist
        ws.train_loss = hist[-1][1]
        return ws

    def predict(self, features, y_init):
        """Predicted states for host features [B][F]; y_init: list of the
        members' initial guesses (float64 CUDA, Dirichlet rows exact).
        Returns a list of new state tensors."""
        import torch
        F = np.atleast_2d(np.asarray(features, dtype=np.float64))
        x = torch.from_numpy(((F - self.x_mu) / self.x_sd).astype(np.float32)).cuda()
        y = torch.empty((F.shape[0], self.Phi.shape[0]), dtype=torch.float32, device=x.device)
        self.net.forward(x, y)
        c = y.cpu().numpy().astype(np.float64) * self.t_sd + self.t_mu
        out = []
        for b in range(F.shape[0]):
            cb = torch.from_numpy(np.ascontiguousarray(c[b])).cuda()
            yp = torch.empty_like(y_init[b])
            rb_expand(self.Phi, cb, self.mean, yp.view(-1))
            out.append(yp)
        return out


def fix_dirichlet(y_pred, y_init, dirichlet_nodes):
    """Copy the velocity rows of the Dirichlet nodes from y_init."""
    import torch
    idx = torch.as_tensor(np.asarray(dirichlet_nodes, dtype=np.int64), device=y_pred.device)
    y_pred[idx, :3] = y_init[idx, :3]
    return y_pred
