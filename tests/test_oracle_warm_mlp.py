"""Pins of the warm-start network reference (oracle/warm_mlp.py), CPU only.

Each pin checks the reference against something other than itself: a forward pass
worked out by hand, closed forms of the projection loss, central finite differences
of the loss for every parameter (pins the analytic backward pass), and the closed
form of Adam's first step.
"""
import numpy as np
import pytest

from oracle import warm_mlp as W


def test_forward_by_hand():
    # n_in = 2, H = 2, V = 1, n_pos = 2
    W1 = np.array([[1.0, -1.0], [2.0, 0.5]])
    b1 = np.array([0.5, -3.0])
    W2 = np.array([[1.0, 2.0], [-1.0, 1.0]])
    b2 = np.array([0.0, -10.0])
    W3 = np.array([[1.0, -2.0], [3.0, 4.0]])
    b3 = np.array([0.25, 0.5])
    x = np.array([[1.0, 2.0]])
    # z1 = [1 + 4 + 0.5, -1 + 1 - 3] = [5.5, -3] -> h1 = [5.5, 0]
    # z2 = [5.5, 11 - 10] = [5.5, 1] -> h2 = [5.5, 1]
    # y = [5.5 + 3 + 0.25, -11 + 4 + 0.5] = [8.75, -6.5]
    y, _ = W.forward([W1, b1, W2, b2, W3, b3], x)
    assert np.array_equal(y, np.array([[8.75, -6.5]]))


def test_loss_closed_forms():
    rng = np.random.default_rng(0)
    n, V = 12, 3
    s = np.ones(n)
    Y = rng.standard_normal((n, V))
    # targets inside span(Y): loss = O(ridge)
    Q, _ = np.linalg.qr(Y @ rng.standard_normal((V, 2)))
    l_in, _ = W.sample_loss(Y, Q, s)
    assert 0.0 <= l_in < 1e-6
    # targets orthogonal to span(Y): loss = 1 exactly (C = 0)
    P = np.eye(n) - Y @ np.linalg.pinv(Y)
    T = P @ rng.standard_normal((n, 2))
    T /= np.linalg.norm(T, axis=0)
    l_out, _ = W.sample_loss(Y, T, s)
    assert abs(l_out - 1.0) < 1e-12
    # one vector, one target: loss = 1 - (y.t)^2 / (y.y + ridge)
    y = rng.standard_normal((n, 1))
    t = rng.standard_normal((n, 1))
    t /= np.linalg.norm(t)
    l1, _ = W.sample_loss(y, t, s)
    ref = 1.0 - (y[:, 0] @ t[:, 0]) ** 2 / (y[:, 0] @ y[:, 0] + W.RIDGE)
    assert abs(l1 - ref) < 1e-14
    # invariance under a change of basis of span(Y) (exact for ridge -> 0)
    R = rng.standard_normal((V, V)) + 3 * np.eye(V)
    T = rng.standard_normal((n, 2))
    T /= np.linalg.norm(T, axis=0)
    la, _ = W.sample_loss(Y, T, s)
    lb, _ = W.sample_loss(Y @ R, T, s)
    assert abs(la - lb) < 1e-6
    # masked rows do not count: values there change nothing
    s2 = np.ones(n)
    s2[:4] = 0
    T2 = T.copy()
    T2[:4] = 0
    T2 /= np.linalg.norm(T2, axis=0)
    Yb = Y.copy()
    Yb[:4] = 1e3 * rng.standard_normal((4, V))
    lc, gc = W.sample_loss(Y, T2, s2)
    ld, _ = W.sample_loss(Yb, T2, s2)
    assert abs(lc - ld) < 1e-15 and np.all(gc[:4] == 0)


def _tiny():
    n_in, H, V, n_pos, B = 5, 4, 2, 6, 3
    rng = np.random.default_rng(11)
    params = [rng.standard_normal(s) * 0.7 for s in W.param_shapes(n_in, H, V, n_pos)]
    x = rng.standard_normal((B, n_in))
    counts = np.array([2, 1, 0])
    T = rng.standard_normal((B, 2, n_pos))
    masks = np.ones((B, n_pos))
    masks[1, 4:] = 0
    T[1, :, 4:] = 0
    T /= np.linalg.norm(T, axis=2, keepdims=True)
    return params, x, T, masks, counts, V, n_pos


def test_gradient_matches_central_differences():
    params, x, T, masks, counts, V, n_pos = _tiny()
    _, cache = W.forward(params, x)
    # stay away from the relu kinks so that the finite differences are smooth
    assert np.abs(cache[1]).min() > 1e-3 and np.abs(cache[3]).min() > 1e-3
    loss, grads = W.loss_and_grad(params, x, T, masks, counts, V, n_pos)
    h = 1e-6
    for k, p in enumerate(params):
        num = np.zeros_like(p)
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            pp = [q.copy() for q in params]
            pp[k][idx] += h
            lp, _ = W.loss_and_grad(pp, x, T, masks, counts, V, n_pos)
            pp[k][idx] -= 2 * h
            lm, _ = W.loss_and_grad(pp, x, T, masks, counts, V, n_pos)
            num[idx] = (lp - lm) / (2 * h)
        err = np.abs(num - grads[k]).max()
        assert err <= 1e-7 * max(1.0, np.abs(num).max()), (W.PARAM_NAMES[k], err)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = [rng.standard_normal(7)]
    g = [rng.standard_normal(7)]
    z = [np.zeros(7)]
    lr = 1e-2
    newp, m, v = W.adam_step(p, g, z, z, 1, lr)
    # bias-corrected first moments equal g and g^2: the step is lr * g / (|g| + eps)
    ref = p[0] - lr * g[0] / (np.abs(g[0]) + W.ADAM_EPS)
    assert np.allclose(newp[0], ref, rtol=0, atol=1e-15)
    assert np.allclose(m[0], 0.1 * g[0]) and np.allclose(v[0], 0.001 * g[0] ** 2)


def test_flatten_roundtrip():
    shapes = W.param_shapes(3, 4, 2, 5)
    flat = np.arange(sum(int(np.prod(s)) for s in shapes), dtype=np.float64)
    parts = W.unflatten(flat, 3, 4, 2, 5)
    assert [p.shape for p in parts] == shapes
    assert np.array_equal(W.flatten(parts), flat)
