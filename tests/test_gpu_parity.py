"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances (derived in tests/gpu_common.py and the design notes):
  * finest-level eigenvalues of the selected pairs: within 128 u cond (the first-order
    effect of the FP64 evaluation of the pencil) or 1e-10 max(lambda, 1e-3 eta), whichever
    is larger, of the oracle's pair refined in binary128 on the exactly summed element data;
    the pair that certifies the count must lie at or above eta on both sides;
  * finest-level coarse-space blocks: sin of the largest principal angle to the refined
    subspace D X within 1e-8;
  * counts m: exact;
  * coarse levels (generating systems): counts exact, eigenvalues in [0, eta); the
    preconditioner apply within 1e-8 relative (a sum of A-orthogonal projections moves by
    O(theta) when its subspaces turn by theta; 1e-8 is the subspace bar);
  * PCG: iteration count within +-1, solution and the iterates at fixed counts within 1e-8
    relative.
"""
import json
import os

import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle, neumann_matrix

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ANGLE_BAR = 1e-8
APPLY_BAR = 1e-8


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _setup(prob, **opts):
    from gpu_common import gpu_setup
    return gpu_setup(prob, **opts)


def _check_fine_level(m, o, prob, eta, angle_bar=None):
    """Counts, selected eigenvalues, certifying pairs and coarse-space blocks of the finest
    level against the binary128 references (o built with fine_vectors > 0)."""
    angle_bar = ANGLE_BAR if angle_bar is None else angle_bar
    from gpu_common import check_selected_and_certifying, refined_fine_level, sin_angle
    L = prob.n_levels - 1
    lev = o.levels[L]
    mg = m.level_counts(L, prob.n_sub)
    assert list(mg) == list(lev.m)
    st = m.stats()
    assert st["eig_unconverged"] == 0
    refs = refined_fine_level(o, prob)
    worst = 0.0
    fixed = getattr(o, "nev_fixed", 0) > 0
    for i, r in enumerate(refs):
        mi = int(lev.m[i])
        lg = m.eigs(L, i, 1)
        worst = max(worst, check_selected_and_certifying(lg, mi, r.lam, r.fp64_uncertainty,
                                                         r.bound, eta, where=i, fixed=fixed))
        if mi:
            Dx = prob.sub_weights(i)[:, None] * r.X[:, :mi]
            assert sin_angle(m.basis(L, i), Dx) <= angle_bar, i
    return worst


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


def _iterate(m, prob, k):
    """The PCG iterate after exactly k iterations (x0 = 0)."""
    torch = _torch()
    b = torch.from_numpy(prob.b).cuda()
    x = torch.zeros_like(b)
    m.solve(b, x, 1e-30, k, allow_noconv=True)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("contrast,seed", [(1.0, 0), (1e4, 3), (1e6, 5)])
def test_two_level_small(contrast, seed):
    prob = P.small_problem(N=16, P=4, delta=1, contrast=contrast, seed=seed)
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob)
    _check_fine_level(m, o, prob, prob.eta)
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve(record=True)
    assert abs(it - ro.iters) <= 1
    assert _rel(x, ro.x) < 1e-8
    for k in (3, 8):
        assert _rel(_iterate(m, prob, k), ro.iterates[k]) < 1e-8, k
    m.close()


@pytest.mark.parametrize("N,Pn,delta,seed", [(16, 4, 1, 11), (20, 4, 2, 12)])
def test_three_level_small(N, Pn, delta, seed):
    """Finest level to full tolerance; the coarse level on its generating system: the
    counts m exactly (they are stable under the truncation of the numerically
    dependent ghost functions), the preconditioner and the PCG (iterations +-1)."""
    prob = P.small_problem(N=N, P=Pn, delta=delta, contrast=1e4, n_levels=3, groups=(2,), seed=seed)
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob)
    _check_fine_level(m, o, prob, prob.eta)
    lev = o.levels[1]
    assert list(m.level_counts(1, lev.n_sub)) == list(lev.m)
    for i in range(lev.n_sub):
        lg = m.eigs(1, i, 0)
        assert np.all((lg >= -1e-12) & (lg < prob.eta)) and len(lg) == lev.m[i]
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve(record=True)
    assert abs(it - ro.iters) <= 1
    assert _rel(x, ro.x) < 1e-8
    for k in (3, 8):
        assert _rel(_iterate(m, prob, k), ro.iterates[k]) < 1e-8, k
    m.close()


def _golden(name):
    with open(os.path.join(HERE, "golden", f"{name}_oracle.json")) as f:
        g = json.load(f)
    arr = np.load(os.path.join(HERE, "golden", f"{name}_oracle.npz"), allow_pickle=False)
    return g, arr


def _check_golden_fine_level(m, prob, g, arr):
    from gpu_common import check_selected_and_certifying, sin_angle
    L = prob.n_levels - 1
    lev = g["levels"][str(L)]
    ref = lev["lam_ref"]
    assert list(m.level_counts(L, prob.n_sub)) == lev["m"]
    worst = 0.0
    for i in range(prob.n_sub):
        lg = m.eigs(L, i, 1)   # the m selected pairs and the next one, which certifies m
        worst = max(worst, check_selected_and_certifying(
            lg, lev["m"][i], np.array(ref["lam"][i]), np.array(ref["unc"][i]),
            np.array(ref["bound"][i]), prob.eta, where=i))
    for i in g["basis_subdomains"]:
        Bo = arr[f"basis_{L}_{i}"]
        assert sin_angle(m.basis(L, i), Bo) <= ANGLE_BAR, i
    return worst


def test_c1_full_against_golden():
    """64x64 channels workload, 2 levels: every subdomain and the PCG against the oracle."""
    g, arr = _golden("c1")
    prob = P.config1()
    m, _ = _setup(prob)
    assert m.stats()["n"] == g["level_sizes"]
    _check_golden_fine_level(m, prob, g, arr)
    it, rel, x = _solve(m, prob)
    assert abs(it - g["pcg"]["iters"]) <= 1
    assert _rel(x, arr["x"]) < 1e-8
    for k in g["iterates"]:
        assert _rel(_iterate(m, prob, k), arr[f"x_it{k}"]) < 1e-8, k
    m.close()


def _first_below(h, tau):
    k = np.nonzero(np.asarray(h) < tau)[0]
    return int(k[0]) if len(k) else None


def test_c2_full_against_golden():
    """512x512 inclusions workload, 3 levels (the benchmark workload), against the oracle's
    full run (tests/golden/c2_oracle.json, .npz).

      * finest level: every count; every selected eigenvalue to the per-pair bar against the
        binary128 references; coarse-space blocks of 16 sampled subdomains within 1e-8;
      * level 1 (generating systems): counts exact, eigenvalues within 1e-6 max(lambda, eta).
        These pencils are numerically rank deficient (the singular values of abar + b run
        continuously down to the compression threshold); two independent reductions of the
        same pencil (compression and the Schur complement with a pseudo-inverse) agree only
        to 2e-6 at contrast 1e4 (the oracle's coarse-pencil pin), so that is the accuracy to
        which these eigenvalues are defined in FP64;
      * PCG: the iterate after 20 iterations and the final solution within 1e-8, the one
        after 5 within 5e-8.  The first iterations mostly resolve the coarse components, and
        the level-1 coarse spaces are defined only to the accuracy stated above (rank
        deficient generating systems), so the two preconditioners' coarse corrections
        differ at the 1e-8 level, which the early iterate carries with a factor of a few
        (measured: 1.8e-8 after 5 iterations, 3.3e-9 after 20, 9.4e-10 after 60 and at the
        end).  The attainable accuracy of the residual of this contrast-1e6 system is
        eps ||A|| ||x|| / ||b|| = 3e-6 (the true residual of both runs at exit); crossings
        of thresholds at least 100 times above it (1e-2, 1e-3, 1e-4) agree within +-1.  Below
        the floor the recurrence residual is driven by rounding and contracts by about 0.77
        per iteration near 1e-8 (oracle history), so a factor 10^0.3 between the histories
        (the history bound below; measured 10^0.23) moves the crossing of 1e-8 by up to
        log(10^0.3) / log(1/0.77) = 2.6 iterations: the final count is compared within +-3
        (measured: equal, 120)."""
    if not os.path.exists(os.path.join(HERE, "golden", "c2_oracle.npz")):
        pytest.skip("c2 golden (refined references, solution) not generated yet")
    g, arr = _golden("c2")
    prob = P.config2()
    m, _ = _setup(prob)
    assert m.stats()["n"] == g["level_sizes"]
    _check_golden_fine_level(m, prob, g, arr)
    lev1 = g["levels"]["1"]
    assert list(m.level_counts(1, len(lev1["m"]))) == lev1["m"]
    for i in range(len(lev1["m"])):
        lg = m.eigs(1, i, 0)
        lo = np.array(lev1["lam"][i][:len(lg)])
        assert len(lo) == len(lg)
        assert np.all(np.abs(lg - lo) <= 1e-6 * np.maximum(np.abs(lo), prob.eta)), (i, lg, lo)
    for k in g["iterates"]:
        if k <= 20:
            assert _rel(_iterate(m, prob, k), arr[f"x_it{k}"]) < (5e-8 if k < 20 else 1e-8), k
    it, rel, x = _solve(m, prob)
    h = m.history()
    ho = np.array(g["pcg"]["resnorms"])
    ho = ho / ho[0]
    for tau in (1e-2, 1e-3, 1e-4):
        assert abs(_first_below(h, tau) - _first_below(ho, tau)) <= 1, tau
    assert abs(it - g["pcg"]["iters"]) <= 3
    k = min(len(h), len(ho))
    assert np.max(np.abs(np.log10(h[:k] / ho[:k]))) <= 0.3
    assert _rel(x, arr["x"]) < 1e-8
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
def test_mixed_precision_against_oracle(case):
    """Single-precision Dirichlet factors and fine-level solves (MSDD_MIXED) against the
    oracle: the coarse spaces come from the FP64 eigensolver, so counts and eigenvalues meet
    the FP64 bars (and equal the FP64 GPU run bitwise); PCG reaches the recurrence tolerance
    within 3 iterations of the oracle's count, and its solution error against the oracle is
    stated (printed), with the true residual within 10x of the oracle's."""
    from paper_2106_06404_amd import binding as B
    prob = (P.config1() if case == "c1" else
            P.small_problem(N=20, P=4, delta=2, contrast=1e4, n_levels=3, groups=(2,), seed=12))
    o = Oracle(prob, fine_vectors=8)
    ro = o.solve()
    tr_o = np.linalg.norm(prob.b - prob.A @ ro.x) / np.linalg.norm(prob.b)
    out = {}
    for prec in (B.MSDD_FP64, B.MSDD_MIXED):
        m, _ = _setup(prob, precision=prec)
        L = prob.n_levels - 1
        if prec == B.MSDD_MIXED:
            _check_fine_level(m, o, prob, prob.eta)
        eigs = [m.eigs(L, i, 0) for i in range(prob.n_sub)]
        it, rel, x = _solve(m, prob)
        tr = np.linalg.norm(prob.b - prob.A @ x) / np.linalg.norm(prob.b)
        out[prec] = (eigs, it, rel, x, tr)
        m.close()
    e64 = out[B.MSDD_FP64][0]
    e32, it32, rel32, x32, tr32 = out[B.MSDD_MIXED]
    assert all(np.array_equal(a, b) for a, b in zip(e64, e32))
    assert rel32 < 1e-8 and abs(it32 - ro.iters) <= 3
    assert tr32 <= 10 * tr_o + 1e-12
    print(f"mixed {case}: iterations {it32} (oracle {ro.iters}), solution error against the "
          f"oracle {_rel(x32, ro.x):.2e}, true residual {tr32:.2e} (oracle {tr_o:.2e})")


@pytest.mark.parametrize("N,Pn", [(64, 16), (96, 24)])
def test_large_coarsest_tiled(N, Pn):
    """Two levels with 256 and 576 subdomains: the coarsest spaces (781 and 1883 functions,
    neither a multiple of the 64-row tile) are factorised and inverted by the tiled
    whole-device kernels.  The apply, PCG and solution against the oracle."""
    prob = P.small_problem(N=N, P=Pn, delta=1, contrast=1e4, seed=5)
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob)
    assert m.stats()["n"] == o.level_sizes()
    assert o.level_sizes()[0] > 384 and o.level_sizes()[0] % 64
    _check_fine_level(m, o, prob, prob.eta)
    for seed in (0, 1):
        assert _apply_rel(m, o, prob, seed) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert _rel(x, ro.x) < 1e-8
    m.close()


def test_large_subdomain_is_exact():
    """One subdomain of 25281 dofs, half-bandwidth 159 (more than the LDS holds as a vector:
    the restriction reads back from global memory and the local solve keeps a ring of the
    band in LDS): the preconditioner is A^{-1} (b = abar, every lambda = 1, no coarse space),
    so the apply equals a sparse direct solve and CG takes one iteration."""
    import scipy.sparse.linalg as spla
    torch = _torch()
    prob = P.small_problem(N=160, P=1, delta=0, contrast=1.0, seed=1)
    m, _ = _setup(prob)
    assert m.stats()["n"][0] == 0
    r = np.random.default_rng(3).standard_normal(prob.n)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    m.apply(rt, zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    x = spla.spsolve(prob.A.tocsc(), r)
    assert np.linalg.norm(z - x) <= 1e-9 * np.linalg.norm(x)
    it, _, _ = _solve(m, prob)
    assert it == 1
    m.close()


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
    o = Oracle(prob, fine_vectors=8)
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
