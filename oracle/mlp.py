"""FP64 reference of the warm-start network and reduced basis.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
definitions, independent of the HIP kernels:

* network: layers l = 0..L-1, z_l = a_{l-1} W_l^T + b_l with a_{-1} = x,
  a_l = tanh(z_l) for the hidden layers and y = z_{L-1}; loss
  mean over batch and outputs of (y - t)^2; gradients by the chain rule
  (backpropagation), in FP64.
* Adam with bias correction (Kingma & Ba 2015, Algorithm 1).
* greedy reduced basis: repeatedly take the snapshot with the largest
  residual after projection on the current basis, orthonormalize it.

Parameters travel as one flat vector in the order W_0, b_0, W_1, b_1, ...
with W_l stored [d_{l+1}][d_l] row-major.
"""
import numpy as np


def unflatten(theta, dims):
    """Split the flat parameter vector into [(W_l, b_l)]."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for l in range(len(dims) - 1):
        nw = dims[l + 1] * dims[l]
        W = theta[o:o + nw].reshape(dims[l + 1], dims[l])
        o += nw
        b = theta[o:o + dims[l + 1]]
        o += dims[l + 1]
        out.append((W, b))
    assert o == theta.size
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def forward(theta, dims, x):
    """Returns (y, activations a_{-1} .. a_{L-2})."""
    layers = unflatten(theta, dims)
    a = np.asarray(x, dtype=np.float64)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        if l < len(layers) - 1:
            a = np.tanh(z)
            acts.append(a)
        else:
            a = z
    return a, acts


def loss_and_gradient(theta, dims, x, t):
    """Mean squared error over all batch entries and outputs, and its gradient
    with respect to the flat parameter vector."""
    layers = unflatten(theta, dims)
    y, acts = forward(theta, dims, x)
    t = np.asarray(t, dtype=np.float64)
    cnt = y.size
    loss = float(np.sum((y - t) ** 2) / cnt)
    g = 2.0 * (y - t) / cnt          # dL/dz for the output layer
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_in = acts[l]
        grads[l] = (g.T @ a_in, g.sum(axis=0))
        if l > 0:
            g = (g @ W) * (1.0 - acts[l] ** 2)   # through tanh of the layer below
    return loss, flatten(grads)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def greedy_basis(Y, mean, r, tol=1e-12):
    """Greedy reduced basis of the snapshot rows of Y around mean: returns
    (Phi [k][D] orthonormal rows, picked indices), k <= r."""
    Yc = np.asarray(Y, dtype=np.float64) - np.asarray(mean, dtype=np.float64)
    top = max(float(np.max(np.sum(Yc * Yc, axis=1))), 1e-300)
    Phi, picked = [], []
    for _ in range(r):
        if Phi:
            P = np.array(Phi)
            R = Yc - (Yc @ P.T) @ P
        else:
            R = Yc
        res = np.sum(R * R, axis=1)
        res[picked] = -1.0
        i = int(np.argmax(res))
        if res[i] <= 1e-24 * top:
            break
        q = Yc[i].copy()
        for _ in range(2):
            if Phi:
                P = np.array(Phi)
                q -= P.T @ (P @ q)
        nq = np.linalg.norm(q)
        if nq * nq <= 1e-24 * top:
            break
        Phi.append(q / nq)
        picked.append(i)
    return np.array(Phi), picked
