"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances (derived in the design doc):
  * finest-level eigenvalues: |d lambda| <= 1e-10 * max(lambda, eta) (below eta the
    eigenvalues of a high-contrast pencil are fixed in double precision only to an
    absolute ~1e-11: see the 40-digit pin of the oracle);
  * finest-level coarse-space blocks: largest principal angle <= 1e-7;
  * counts m: exact (subdomains with an eigenvalue within 1e-8 eta of eta excepted);
  * coarse levels (generating systems): counts exact, the preconditioner apply
    within 1e-3 relative (the generating system is numerically rank deficient, and
    two valid reductions of it differ at that level);
  * PCG: iteration count within +-1 and solution within 1e-8 relative (2 levels)
    or within the CG attainable-accuracy bound (3 levels).
"""
import json
import os

import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle, neumann_matrix

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _setup(prob, **opts):
    from gpu_common import gpu_setup
    return gpu_setup(prob, **opts)


def _sin_angle(U, V):
    """sin of the largest principal angle between span(U) and span(V)."""
    if U.shape[1] != V.shape[1]:
        return 1.0
    if U.shape[1] == 0:
        return 0.0
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    return float(np.linalg.norm(Qv - Qu @ (Qu.T @ Qv), 2))


def _check_fine_level(m, o, prob, eta, rel=1e-10, angle=1e-7):
    L = prob.n_levels - 1
    lev = o.levels[L]
    mg = m.level_counts(L, prob.n_sub)
    assert list(mg) == list(lev.m)
    for i in range(prob.n_sub):
        lg = m.eigs(L, i, 0)
        lo = lev.lam[i][:len(lg)]
        scale = np.maximum(np.abs(lo), eta)
        assert np.all(np.abs(lg - lo) <= rel * scale), (i, lg, lo)
        assert _sin_angle(m.basis(L, i), lev.basis[i]) <= angle, i


def _apply_rel(m, o, prob, seed=0):
    torch = _torch()
    r = np.random.default_rng(seed).standard_normal(prob.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    m.apply(rt, zt)
    torch.cuda.synchronize()
    zo = o.apply(r)
    return float(np.linalg.norm(zt.cpu().numpy() - zo) / np.linalg.norm(zo))


def _solve(m, prob, rtol=1e-8, maxit=2000):
    torch = _torch()
    b = torch.from_numpy(prob.b).cuda()
    x = torch.zeros_like(b)
    it, rel, rc = m.solve(b, x, rtol, maxit)
    torch.cuda.synchronize()
    return it, rel, x.cpu().numpy()


@pytest.mark.parametrize("contrast,seed", [(1.0, 0), (1e4, 3), (1e6, 5)])
def test_two_level_small(contrast, seed):
    prob = P.small_problem(N=16, P=4, delta=1, contrast=contrast, seed=seed)
    o = Oracle(prob)
    m, _ = _setup(prob)
    _check_fine_level(m, o, prob, prob.eta)
    assert _apply_rel(m, o, prob) < 1e-9
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
    m.close()


@pytest.mark.parametrize("N,Pn,delta,seed", [(16, 4, 1, 11), (20, 4, 2, 12)])
def test_three_level_small(N, Pn, delta, seed):
    """Finest level to full tolerance; the coarse level on its generating system: the
    counts m exactly (they are stable under the truncation of the numerically
    dependent ghost functions), the preconditioner and the PCG (iterations +-1)."""
    prob = P.small_problem(N=N, P=Pn, delta=delta, contrast=1e4, n_levels=3, groups=(2,), seed=seed)
    o = Oracle(prob)
    m, _ = _setup(prob)
    _check_fine_level(m, o, prob, prob.eta)
    lev = o.levels[1]
    assert list(m.level_counts(1, lev.n_sub)) == list(lev.m)
    for i in range(lev.n_sub):
        lg = m.eigs(1, i, 0)
        assert np.all((lg >= -1e-12) & (lg < prob.eta)) and len(lg) == lev.m[i]
    assert _apply_rel(m, o, prob) < 1e-3
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-7
    m.close()


def test_c1_full_against_golden():
    """64x64 channels workload, 2 levels: every subdomain and the PCG against the oracle."""
    with open(os.path.join(HERE, "golden", "c1_oracle.json")) as f:
        g = json.load(f)
    prob = P.config1()
    m, _ = _setup(prob)
    L = prob.n_levels - 1
    lev = g["levels"][str(L)]
    assert list(m.level_counts(L, prob.n_sub)) == lev["m"]
    for i in range(prob.n_sub):
        lg = m.eigs(L, i, 1)   # the m selected pairs and the next one, which certifies m
        lo = np.array(lev["lam"][i][:len(lg)])
        scale = np.maximum(np.abs(lo), prob.eta)
        assert np.all(np.abs(lg - lo) <= 1e-10 * scale), (i, lg, lo)
    st = m.stats()
    assert st["n"] == g["level_sizes"]
    it, rel, x = _solve(m, prob)
    assert abs(it - g["pcg"]["iters"]) <= 1
    xo = np.array(g["pcg"]["x"])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8
    m.close()


def _first_below(h, tau):
    k = np.nonzero(np.asarray(h) < tau)[0]
    return int(k[0]) if len(k) else None


def test_c2_full_against_golden():
    """512x512 inclusions workload, 3 levels (the benchmark workload), against the oracle's
    full run (tests/golden/c2_oracle.json).

    Tolerances, from the arithmetic of this workload:
      * finest-level eigenvalues: 2.5e-8 * max(lambda, eta).  The oracle itself differs
        from LAPACK (scipy.linalg.eigh on the same pencils, all 256 subdomains) by up to
        1.26e-8 * max(lambda, eta) here (contrast 1e6, 1369 dofs per subdomain), so the
        bar is twice the reference's own uncertainty;
      * level-1 eigenvalues (generating systems, numerically rank deficient): 1e-6 *
        max(lambda, eta);
      * PCG: the 2-norm residual of this high-contrast system is erratic (it first grows
        to 3e3, later has isolated spikes), and the attainable accuracy of the residual is
        ~eps ||A|| ||x|| / ||b|| = 3e-6.  GPU and oracle histories agree to 4 digits for
        the first 60 iterations and stay within a factor 1.85 afterwards, but a spike
        (iteration 95: 4.9e-6 against 8.3e-6) moves the crossing of 1e-5 by two
        iterations.  Below the attainable accuracy the recurrence residual is dominated
        by rounding: it contracts by about 0.77 per iteration near 1e-8 (oracle history,
        iterations 115-120), so the history bound below (a factor 10^0.5) allows the
        crossing of 1e-8 to move by log(10^0.5)/log(1/0.77) = 4.4 iterations; the oracle's
        last step lands at 0.98e-8.  So crossings of 1e-2 ... 1e-7 are compared within +-2
        (the +-1 bar holds on the other workloads), the final count within +-4, the whole
        history within a factor 10^0.5, the solution at sampled dofs within 1e-7 and the
        true residual below 1e-5."""
    with open(os.path.join(HERE, "golden", "c2_oracle.json")) as f:
        g = json.load(f)
    prob = P.config2()
    m, _ = _setup(prob)
    assert m.stats()["n"] == g["level_sizes"]
    for L, tol in ((2, 2.5e-8), (1, 1e-6)):
        lev = g["levels"][str(L)]
        assert list(m.level_counts(L, len(lev["m"]))) == lev["m"], L
        for i in range(len(lev["m"])):
            lg = m.eigs(L, i, 1 if L == 2 else 0)
            lo = np.array(lev["lam"][i][:len(lg)])
            assert len(lo) == len(lg)
            scale = np.maximum(np.abs(lo), prob.eta)
            assert np.all(np.abs(lg - lo) <= tol * scale), (L, i, lg, lo)
    it, rel, x = _solve(m, prob)
    h = m.history()
    ho = np.array(g["pcg"]["resnorms"])
    ho = ho / ho[0]
    for tau in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        assert abs(_first_below(h, tau) - _first_below(ho, tau)) <= 2, tau
    assert abs(it - g["pcg"]["iters"]) <= 4
    k = min(len(h), len(ho))
    assert np.max(np.abs(np.log10(h[:k] / ho[:k]))) <= 0.5
    idx = np.array(g["pcg"]["x_sample_idx"])
    xs = np.array(g["pcg"]["x_sample"])
    assert np.linalg.norm(x[idx] - xs) / np.linalg.norm(xs) < 1e-7
    assert np.linalg.norm(prob.b - prob.A @ x) / np.linalg.norm(prob.b) < 1e-5
    m.close()


def test_c1_local_eigenpairs_residual():
    """Eigenpairs returned by the GPU satisfy the local GEVP of the oracle's Neumann matrix."""
    prob = P.config1()
    m, _ = _setup(prob)
    L = prob.n_levels - 1
    for i in [0, 5, 10, 15]:
        d = prob.sub_weights(i)
        Ab = neumann_matrix(prob.elem_dofs, prob.elem_mat, prob.sub_elems(i), prob.sub_dofs(i))
        Bm = d[:, None] * Ab * d[None, :]
        lam = m.eigs(L, i, 0)
        Phi = m.basis(L, i)   # = D W
        # W from Phi: rows with d = 0 are in ker b; compare b-products through Phi
        assert Phi.shape[1] == len(lam)
        if len(lam):
            G = Phi.T @ Ab @ Phi   # = W^T b W = I
            assert np.allclose(G, np.eye(len(lam)), atol=1e-8)
    m.close()


@pytest.mark.parametrize("case", ["c1", "three_level"])
def test_mixed_precision_apply(case):
    """Single-precision Dirichlet factors and fine-level solves (MSDD_MIXED): the coarse
    spaces are those of double precision (bitwise), PCG reaches the same recurrence
    tolerance in at most 3 more iterations, and the true residual stays within 10x of
    the double-precision run's (its error against the oracle is stated, not bounded)."""
    from paper_2106_06404_amd import binding as B
    prob = (P.config1() if case == "c1" else
            P.small_problem(N=20, P=4, delta=2, contrast=1e4, n_levels=3, groups=(2,), seed=12))
    out = {}
    for prec in (B.MSDD_FP64, B.MSDD_MIXED):
        m, _ = _setup(prob, precision=prec)
        L = prob.n_levels - 1
        counts = m.level_counts(L, prob.n_sub)
        eigs = [m.eigs(L, i, 0) for i in range(prob.n_sub)]
        it, rel, x = _solve(m, prob)
        tr = np.linalg.norm(prob.b - prob.A @ x) / np.linalg.norm(prob.b)
        out[prec] = (counts, eigs, it, rel, x, tr)
        m.close()
    c64, e64, it64, _, x64, tr64 = out[B.MSDD_FP64]
    c32, e32, it32, rel32, x32, tr32 = out[B.MSDD_MIXED]
    assert np.array_equal(c64, c32)
    assert all(np.array_equal(a, b) for a, b in zip(e64, e32))
    assert rel32 < 1e-8 and it32 <= it64 + 3
    assert tr32 <= 10 * tr64 + 1e-12


def test_single_subdomain_empty_coarse_space():
    prob = P.small_problem(N=10, P=1, delta=0, contrast=1e3, seed=3)
    m, _ = _setup(prob)
    st = m.stats()
    assert st["n"][0] == 0
    it, rel, x = _solve(m, prob)
    assert it == 1
    m.close()


def test_ragged_boxes_and_block_growth():
    """Boxes of uneven size (N not divisible by P) and a threshold that selects many
    eigenvectors (forces the eigensolver to grow its block)."""
    prob = P.small_problem(N=23, P=3, delta=2, contrast=1e4, seed=21, eta=1.1)
    o = Oracle(prob)
    m, _ = _setup(prob, block=16)
    _check_fine_level(m, o, prob, prob.eta)
    st = m.stats()
    assert max(o.levels[1].m) > 13 and st["eig_restarts"] > 0
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    m.close()


def test_nev_max_cap():
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e4, seed=3)
    m, _ = _setup(prob, nev_max=1)
    assert m.level_counts(1, prob.n_sub).max() <= 1
    it, rel, x = _solve(m, prob)
    assert rel < 1e-8
    m.close()


def test_host_and_device_pointers_agree_bitwise():
    from paper_2106_06404_amd import binding as B
    torch = _torch()
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e4, n_levels=3, groups=(2,), seed=11)
    out = []
    for dev in (None, "cuda:0"):
        arrs = B.problem_arrays(prob, device=dev)
        m = B.Msdd()
        m.setup(**arrs)
        x = np.zeros(prob.n)
        it, rel, _ = m.solve(prob.b.copy(), x, 1e-8, 500)
        out.append((it, x.copy()))
        m.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])
    torch.cuda.synchronize()


def test_repeatable_bitwise():
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e6, n_levels=3, groups=(2,), seed=2)
    xs = []
    for _ in range(2):
        m, _ = _setup(prob)
        it, rel, x = _solve(m, prob)
        xs.append(x)
        m.close()
    assert np.array_equal(xs[0], xs[1])


def test_error_paths():
    from paper_2106_06404_amd import binding as B
    torch = _torch()
    prob = P.small_problem(N=12, P=3, delta=1, contrast=1e3, seed=4)
    # solve before setup
    m = B.Msdd()
    with pytest.raises(B.MsddError) as e:
        m.solve(prob.b.copy(), np.zeros(prob.n))
    assert e.value.code == B.MSDD_ESTATE
    # partition of unity that does not sum to one
    arrs = B.problem_arrays(prob)
    bad = dict(arrs)
    bad["sub_pou"] = arrs["sub_pou"].copy()
    bad["sub_pou"][np.nonzero(bad["sub_pou"])[0][0]] *= 0.9
    with pytest.raises(B.MsddError) as e:
        m.setup(**bad)
    assert e.value.code == B.MSDD_EINVAL
    # an element matrix with the wrong sign: local matrices are not SPD
    bad = dict(arrs)
    bad["elem_mat"] = arrs["elem_mat"].copy()
    bad["elem_mat"][prob.sub_elems(4)[5]] *= -50.0
    with pytest.raises(B.MsddError) as e:
        m.setup(**bad)
    assert e.value.code in (B.MSDD_ENOTSPD, B.MSDD_EINVAL)
    # a good setup, then maxit reached, then NaN in b
    m.setup(**arrs)
    x = np.zeros(prob.n)
    it, rel, rc = m.solve(prob.b.copy(), x, 1e-12, 2, allow_noconv=True)
    assert rc == B.MSDD_ENOCONV and it == 2
    bn = prob.b.copy()
    bn[3] = np.nan
    with pytest.raises(B.MsddError) as e:
        m.solve(bn, np.zeros(prob.n))
    assert e.value.code == B.MSDD_EINVAL
    m.close()
    torch.cuda.synchronize()
