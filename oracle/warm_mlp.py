"""Plain CPU FP64 reference of the warm-start network of the local eigensolver.

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing else); it shares no
code with the GPU library.

The paper solves the local generalized eigenproblems of Sec. 2.3 (the GEVP
abar w = lambda b w, b = b^1 of Sec. 3.4) from scratch in every subdomain.
This module is the reference of an extension: a multilayer perceptron that maps
a subdomain's coefficient features to a start block for that eigensolver.  The
network and its training objective are not in the paper; they are defined here
and the GPU kernels are checked against this definition.

Network (parameters theta = (W1, b1, W2, b2, W3, b3), row-vector convention):
    h1 = relu(x W1 + b1)        W1: n_in x H
    h2 = relu(h1 W2 + b2)       W2: H x H
    y  = h2 W3 + b3             W3: H x (V * n_pos)
y is read as V vectors of length n_pos (vector v = y[v*n_pos:(v+1)*n_pos]),
i.e. a block Y (n_pos x V) on the subdomain's node frame.

Loss of one sample (block Y, node mask s in {0,1}^n_pos, target vectors
t_1..t_m of unit 2-norm on the frame, T = [t_1..t_m]):
    Ys = diag(s) Y,   G = Ys^T Ys + eps I,   C = Ys^T T
    loss = 1 - tr(C^T G^{-1} C) / m
the share of the targets that lies outside span(Ys) (least-squares projection;
eps = 1e-6 keeps G invertible).  It depends on span(Ys) only (up to eps), so any
basis of the wanted eigenspace, in any order and scaling, is a minimiser.
The batch loss is the mean over the samples; a sample with m = 0 contributes 0.

Gradient (derived in closed form, checked by central differences in the tests):
    dloss/dYs = -(2/m) (T C^T G^{-1} - Ys G^{-1} C C^T G^{-1}),
    dloss/dY  = diag(s) dloss/dYs, then back through the layers (relu' = [z > 0]).

Optimiser: Adam (Kingma and Ba, 2015) with bias correction,
    m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
    theta <- theta - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps_a),
b1 = 0.9, b2 = 0.999, eps_a = 1e-8.
"""
from __future__ import annotations

import numpy as np

RIDGE = 1e-6
ADAM_B1 = 0.9
ADAM_B2 = 0.999
ADAM_EPS = 1e-8

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def param_shapes(n_in: int, hidden: int, n_vec: int, n_pos: int):
    out = n_vec * n_pos
    return [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, out), (out,)]


def unflatten(flat: np.ndarray, n_in: int, hidden: int, n_vec: int, n_pos: int):
    """Split the flat parameter vector (W1, b1, W2, b2, W3, b3; row-major) into arrays."""
    flat = np.asarray(flat, dtype=np.float64)
    out, off = [], 0
    for shp in param_shapes(n_in, hidden, n_vec, n_pos):
        cnt = int(np.prod(shp))
        out.append(flat[off:off + cnt].reshape(shp))
        off += cnt
    assert off == flat.size, (off, flat.size)
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in params])


def forward(params, x: np.ndarray):
    """Returns (y, cache) for a batch x (B x n_in)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def sample_loss(Y: np.ndarray, T: np.ndarray, s: np.ndarray):
    """Loss and dloss/dY of one sample.  Y: n_pos x V, T: n_pos x m (unit columns),
    s: n_pos mask."""
    m = T.shape[1]
    if m == 0:
        return 0.0, np.zeros_like(Y)
    Ys = s[:, None] * Y
    V = Y.shape[1]
    G = Ys.T @ Ys + RIDGE * np.eye(V)
    C = Ys.T @ T
    GiC = np.linalg.solve(G, C)                 # G^{-1} C   (V x m)
    loss = 1.0 - np.trace(C.T @ GiC) / m
    # -(2/m) (T C^T G^{-1} - Ys G^{-1} C C^T G^{-1}); G symmetric: C^T G^{-1} = (G^{-1} C)^T
    dYs = -(2.0 / m) * (T @ GiC.T - Ys @ (GiC @ GiC.T))
    return loss, s[:, None] * dYs


def batch_loss(y: np.ndarray, targets: np.ndarray, masks: np.ndarray, counts: np.ndarray,
               n_vec: int, n_pos: int):
    """Mean loss over the batch and dloss/dy (B x V*n_pos).
    targets: B x m_cap x n_pos (unit vectors, first counts[b] used); masks: B x n_pos."""
    B = y.shape[0]
    total = 0.0
    dy = np.zeros_like(y)
    for b in range(B):
        Y = y[b].reshape(n_vec, n_pos).T
        T = targets[b, :counts[b]].T
        lb, dYb = sample_loss(Y, T, masks[b])
        total += lb
        dy[b] = dYb.T.reshape(-1) / B
    return total / B, dy


def backward(params, cache, dy: np.ndarray):
    """Gradients (same order as params) of the loss whose dloss/dy is given."""
    W1, b1, W2, b2, W3, b3 = params
    x, z1, h1, z2, h2 = cache
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def loss_and_grad(params, x, targets, masks, counts, n_vec, n_pos):
    y, cache = forward(params, x)
    loss, dy = batch_loss(y, targets, masks, counts, n_vec, n_pos)
    return loss, backward(params, cache, dy)


def adam_step(params, grads, m_state, v_state, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    newp, newm, newv = [], [], []
    for p, g, m, v in zip(params, grads, m_state, v_state):
        m = ADAM_B1 * m + (1.0 - ADAM_B1) * g
        v = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
        mh = m / (1.0 - ADAM_B1 ** step)
        vh = v / (1.0 - ADAM_B2 ** step)
        newp.append(p - lr * mh / (np.sqrt(vh) + ADAM_EPS))
        newm.append(m)
        newv.append(v)
    return newp, newm, newv
