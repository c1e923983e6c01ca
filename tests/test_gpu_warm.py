"""Learned warm start of the local eigensolver on the GPU, through the C ABI.

The network's kernels are compared with the FP64 reference oracle/warm_mlp.py on the
same seeded weights and inputs; the warm-started setup is compared with the CPU oracle
of the method (its results must not depend on the network), and a trained network
must reduce the eigensolver's work on a problem it was not trained on.

Tolerances (derived, not fitted):
  * forward passes: a first-order elementwise bound of the rounding model, computed
    from the reference's absolute values (see _forward_bound): FP32 path u = 2^-24 per
    accumulation term; BF16 path inputs, weights and hidden activations rounded to
    BF16 (u = 2^-8) with FP32 accumulation;
  * gradients: FP32 sums of at most K terms have relative error <= K u (u = 2^-24), and
    the V x V solves of the loss amplify the errors of G and C by at most cond(G), so
    each parameter block must agree to 4 (n_pos + n_vec n_pos + n_in) u cond(G) in the
    Frobenius norm;
  * warm-started eigenvalues: the same bound as the cold start against the oracle.
"""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle import warm_mlp as O
from oracle.msdd_oracle import Oracle
from test_gpu_parity import _apply_rel, _check_fine_level, _solve

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
UBF = 2.0 ** -8


def _torch():
    import torch
    return torch


def _net(n_in, H, V, n_pos, seed=0):
    from paper_2106_06404_amd import binding as B
    return B.MsddNet(n_in, H, V, n_pos, seed=seed)


def _params(rng, n_in, H, V, n_pos):
    """Seeded FP32 weights of Glorot scale and small biases."""
    out = []
    for shp in O.param_shapes(n_in, H, V, n_pos):
        if len(shp) == 2:
            a = np.sqrt(6.0 / (shp[0] + shp[1]))
            out.append(rng.uniform(-a, a, shp).astype(np.float32))
        else:
            out.append((0.05 * rng.standard_normal(shp)).astype(np.float32))
    return out


def _forward_bound(params, x, u_in, u_w, u_act, u_acc):
    """Elementwise first-order bound on |y_computed - y| when inputs are rounded with unit
    roundoff u_in, weights with u_w, hidden activations with u_act, and every dot
    product of K terms is accumulated with error <= K u_acc / (1 - K u_acc) sum |w||a|."""
    W = [p.astype(np.float64) for p in params]
    a = x.astype(np.float64)
    E = u_in * np.abs(a)
    for layer in range(3):
        Wl, bl = W[2 * layer], W[2 * layer + 1]
        K = Wl.shape[0]
        gam = K * u_acc / (1.0 - K * u_acc)
        aW = np.abs(Wl)
        s = (np.abs(a) + E) @ aW
        z = a @ Wl + bl
        Ez = E @ aW + (u_w + gam * (1.0 + u_w)) * s + U32 * (np.abs(z) + np.abs(bl))
        if layer < 2:
            h = np.maximum(z, 0.0)
            a, E = h, Ez + u_act * (h + Ez)
        else:
            return z, Ez + U32 * (np.abs(z) + Ez)


@pytest.mark.parametrize("sizes,batch", [((40, 32, 4, 50), 7), ((2596, 256, 16, 1369), 37)])
def test_forward_fp32_and_bf16_against_reference(sizes, batch):
    n_in, H, V, n_pos = sizes
    rng = np.random.default_rng(21)
    params = _params(rng, n_in, H, V, n_pos)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    net = _net(n_in, H, V, n_pos)
    net.set_params(O.flatten(params).astype(np.float32))
    y_ref, _ = O.forward([p.astype(np.float64) for p in params], x.astype(np.float64))
    for mode, (u_in, u_w, u_act) in ((0, (0.0, 0.0, U32)), (1, (UBF, UBF, UBF))):
        y = np.zeros((batch, V * n_pos), np.float32)
        net.forward(x, y, mode=mode)
        _, bound = _forward_bound(params, x, u_in, u_w, u_act, U32)
        err = np.abs(y.astype(np.float64) - y_ref)
        assert np.all(err <= 1.001 * bound + 1e-30), (mode, float((err / bound).max()))
        # and the bound is not vacuous: the typical error is far below the values
        assert np.linalg.norm(err) <= (0.05 if mode else 1e-5) * np.linalg.norm(y_ref)
    net.close()


def _training_set(rng, N, V, n_pos, n_in, m_cap=4):
    x = rng.standard_normal((N, n_in)).astype(np.float32)
    cnt = rng.integers(0, m_cap + 1, N).astype(np.int32)
    cnt[0] = m_cap
    mask = (rng.random((N, n_pos)) < 0.85).astype(np.float32)
    tgt = rng.standard_normal((N, m_cap, n_pos)).astype(np.float32) * mask[:, None, :]
    tgt /= np.linalg.norm(tgt, axis=2, keepdims=True)
    return x, tgt.astype(np.float32), mask, cnt


@pytest.mark.parametrize("sizes,idx", [((40, 32, 4, 50), [3, 0, 8, 5, 1, 1]),
                                       ((2596, 256, 16, 1369), [2, 7, 0, 4, 4, 9, 1, 3])])
def test_gradient_against_reference(sizes, idx):
    n_in, H, V, n_pos = sizes
    rng = np.random.default_rng(33)
    params = _params(rng, n_in, H, V, n_pos)
    x, tgt, mask, cnt = _training_set(rng, 10, V, n_pos, n_in)
    idx = np.array(idx, np.int32)
    net = _net(n_in, H, V, n_pos)
    net.set_params(O.flatten(params).astype(np.float32))
    g = np.zeros(net.n_params, np.float32)
    loss = net.grad(idx, x, tgt, mask, cnt, g)
    p64 = [p.astype(np.float64) for p in params]
    lo, go = O.loss_and_grad(p64, x[idx].astype(np.float64), tgt[idx].astype(np.float64),
                             mask[idx].astype(np.float64), cnt[idx], V, n_pos)
    # condition of the Gram matrices of the batch (reference values)
    y, _ = O.forward(p64, x[idx].astype(np.float64))
    conds = []
    for b in range(len(idx)):
        Ys = mask[idx[b]][:, None] * y[b].reshape(V, n_pos).T
        conds.append(np.linalg.cond(Ys.T @ Ys + O.RIDGE * np.eye(V)))
    tol = 4 * (n_pos + V * n_pos + n_in) * U32 * max(1.0, max(conds))
    assert abs(loss - lo) <= tol * max(1.0, abs(lo))
    gg = O.unflatten(g.astype(np.float64), n_in, H, V, n_pos)
    for k, name in enumerate(O.PARAM_NAMES):
        nrm = np.linalg.norm(go[k])
        assert np.linalg.norm(gg[k] - go[k]) <= tol * nrm + 1e-30, (name, tol)
    net.close()


def test_adam_first_step_closed_form():
    """From fresh moments Adam moves every parameter by lr * g / (|g| + eps) against the
    gradient: +-lr wherever the gradient is well above its rounding error."""
    n_in, H, V, n_pos = 40, 32, 4, 50
    rng = np.random.default_rng(44)
    params = _params(rng, n_in, H, V, n_pos)
    x, tgt, mask, cnt = _training_set(rng, 10, V, n_pos, n_in)
    idx = np.array([1, 4, 0, 9], np.int32)
    flat = O.flatten(params).astype(np.float32)
    net = _net(n_in, H, V, n_pos)
    net.set_params(flat)
    lr = 1e-3
    net.train_step(idx, x, tgt, mask, cnt, lr)
    new = net.get_params()
    _, go = O.loss_and_grad([p.astype(np.float64) for p in params], x[idx].astype(np.float64),
                            tgt[idx].astype(np.float64), mask[idx].astype(np.float64), cnt[idx],
                            V, n_pos)
    g = O.flatten(go)
    step = new.astype(np.float64) - flat.astype(np.float64)
    expect = -lr * g / (np.abs(g) + O.ADAM_EPS)
    big = np.abs(g) >= 1e-4 * np.abs(g).max()
    rnd = 2 * U32 * (np.abs(flat) + lr)  # FP32 rounding of theta - step
    assert np.all(np.abs(step[big] - expect[big]) <= 1e-3 * lr + rnd[big])
    assert np.all(np.abs(step) <= lr * (1 + 1e-6) + rnd)
    net.close()


def _frame(prob, delta):
    feat, sub_pos, n_pos = P.warm_frame(prob, delta)
    return feat, sub_pos, n_pos


def _setup_warm(prob, net, feat, sub_pos, n_pos, collect=0, **opts):
    torch = _torch()
    from paper_2106_06404_amd import binding as B
    arrs = B.problem_arrays(prob, device="cuda:0")
    m = B.Msdd(**opts)
    if net is not None or collect:  # otherwise: the plain random start
        m.warm_start(net, prob.n_sub, sub_pos, n_pos,
                     feat=torch.from_numpy(feat).cuda() if net is not None else None,
                     collect=collect)
    m.setup(**arrs)
    return m


def test_warm_started_setup_matches_oracle():
    """An untrained network changes the start block only: eigenpairs, coarse space,
    apply and PCG agree with the oracle as for the random start."""
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e6, seed=5)
    o = Oracle(prob, fine_vectors=8)
    feat, sub_pos, n_pos = _frame(prob, 1)
    net = _net(feat.shape[1], 64, 8, n_pos, seed=3)
    m = _setup_warm(prob, net, feat, sub_pos, n_pos)
    st = m.stats()
    assert st["warm_started"] == prob.n_sub
    _check_fine_level(m, o, prob, prob.eta)
    assert _apply_rel(m, o, prob) < 1e-8
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
    m.close()
    net.close()


def test_cold_start_fallback():
    """With one iteration allowed no warm-started subdomain converges: every one of
    them is solved again from the random start, which cannot converge in one iteration
    either, so the setup fails with MSDD_EEIG (an uncertified count is never accepted)
    and the statistics record the fallbacks."""
    from paper_2106_06404_amd import binding as B
    # subdomains of 12 x 12 elements: rank(b) far above the block, so one iteration
    # cannot reach the backward-error tolerance
    prob = P.small_problem(N=32, P=4, delta=2, contrast=1e4, seed=3)
    feat, sub_pos, n_pos = _frame(prob, 2)
    net = _net(feat.shape[1], 32, 8, n_pos, seed=4)
    with pytest.raises(B.MsddError) as e:
        _setup_warm(prob, net, feat, sub_pos, n_pos, eig_maxit=1)
    assert e.value.code == B.MSDD_EEIG
    st = e.value.stats
    assert st["warm_started"] == prob.n_sub and st["warm_fallbacks"] == prob.n_sub
    assert st["eig_unconverged"] == prob.n_sub
    # one warm and one cold iteration each (a pass with a larger block adds more for
    # subdomains that asked to grow)
    assert st["eig_iters_sum"] >= 2 * prob.n_sub
    net.close()


def test_collected_targets():
    """Targets: the first min(m_i + 1, m_cap) eigenvectors, unit norm on the mask, zero
    off it; the mask marks exactly the frame positions of the subdomain's dofs."""
    torch = _torch()
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e6, seed=5)
    feat, sub_pos, n_pos = _frame(prob, 1)
    m_cap = 6
    m = _setup_warm(prob, None, feat, sub_pos, n_pos, collect=m_cap)
    Pn = prob.n_sub
    tgt = torch.zeros((Pn, m_cap, n_pos), dtype=torch.float32, device="cuda:0")
    mask = torch.zeros((Pn, n_pos), dtype=torch.float32, device="cuda:0")
    cnt = torch.zeros(Pn, dtype=torch.int32, device="cuda:0")
    m.warm_targets(tgt, mask, cnt)
    tgt, mask, cnt = tgt.cpu().numpy(), mask.cpu().numpy(), cnt.cpu().numpy()
    L = prob.n_levels - 1
    mm = m.level_counts(L, Pn)
    assert np.array_equal(cnt, np.minimum(mm + 1, m_cap))
    for i in range(Pn):
        pos = sub_pos[prob.sub_dof_ptr[i]:prob.sub_dof_ptr[i + 1]]
        ref = np.zeros(n_pos, np.float32)
        ref[pos] = 1
        assert np.array_equal(mask[i], ref)
        for j in range(m_cap):
            v = tgt[i, j]
            if j < cnt[i]:
                assert abs(np.linalg.norm(v) - 1) < 1e-5 and np.all(v[ref == 0] == 0)
            else:
                assert np.all(v == 0)
        # the first m_i targets, weighted by the partition of unity, span the coarse basis
        # functions D_i w of the subdomain
        Bi = m.basis(L, i)
        if mm[i]:
            w = prob.sub_weights(i)
            Tm = w[:, None] * tgt[i, :mm[i]][:, pos].T.astype(np.float64)
            Q, _ = np.linalg.qr(Tm)
            assert np.linalg.norm(Bi - Q @ (Q.T @ Bi)) <= 1e-5 * np.linalg.norm(Bi)
    m.close()


def test_trained_network_reduces_eigensolver_work():
    """Train on the method's own eigenvectors of seeded inclusion problems, then set up a
    problem outside the training set: fewer eigensolver iterations than the random start,
    the same eigenvalues, coarse-space sizes and PCG iterations."""
    torch = _torch()
    from paper_2106_06404_amd import binding as B, warm as W

    def inc(seed):
        k = P.inclusions_2d(256, seed)
        return P.build_problem("inc256", 2, 256, k, P=8, delta=2, n_levels=2, eta=0.1)

    parts = []
    n_pos = None
    for sd in range(100, 108):
        p = inc(sd)
        f, sp, n_pos = _frame(p, 2)
        parts.append(W.collect_targets(p, f, sp, n_pos, m_cap=16)[:4])
    feat, tgt, mask, cnt = (torch.cat([q[k] for q in parts]) for k in range(4))
    net = B.MsddNet(feat.shape[1], 256, 16, n_pos, seed=7)
    l0 = W.mean_loss(net, feat, tgt, mask, cnt)
    losses = W.train(net, feat, tgt, mask, cnt, epochs=30, batch=64, lr=1e-3, lr_final=1e-4, seed=3)
    assert losses[-1] < 0.1 * l0
    prob = inc(999)
    f, sp, _ = _frame(prob, 2)
    cold = _setup_warm(prob, None, f, sp, n_pos)
    warm = _setup_warm(prob, net, f, sp, n_pos)
    sc, sw = cold.stats(), warm.stats()
    assert sw["warm_started"] == prob.n_sub and sw["warm_fallbacks"] == 0
    assert sw["eig_iters_sum"] <= 0.95 * sc["eig_iters_sum"], (sw["eig_iters_sum"], sc["eig_iters_sum"])
    L = prob.n_levels - 1
    assert np.array_equal(cold.level_counts(L, prob.n_sub), warm.level_counts(L, prob.n_sub))
    for i in range(prob.n_sub):
        # the m_i selected pairs (the next one only certifies the count: it is checked for
        # its side of eta)
        lc, lw = cold.eigs(L, i, 1), warm.eigs(L, i, 1)
        mi = len(cold.eigs(L, i, 0))
        assert np.all(np.abs(lc[:mi] - lw[:mi]) <= 2.5e-8 * np.maximum(np.abs(lc[:mi]), prob.eta)), (i, lc, lw)
        assert np.all(lc[mi:] >= prob.eta) and np.all(lw[mi:] >= prob.eta)
    ic, _, xc = _solve(cold, prob)
    iw, _, xw = _solve(warm, prob)
    assert abs(ic - iw) <= 1
    assert np.linalg.norm(xc - xw) / np.linalg.norm(xc) < 1e-6
    cold.close()
    warm.close()
    net.close()
