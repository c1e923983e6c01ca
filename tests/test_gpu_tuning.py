"""Autotuner of launch shapes (msdd_autotune) on the GPU, through the C ABI: every
launch-shape variant computes the same preconditioner (checked against the oracle),
and tuning picks valid shapes from measured times without changing results beyond
rounding."""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle
from test_gpu_parity import APPLY_BAR, _apply_rel, _check_fine_level, _setup, _solve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("eig_solve,eig_splits,fine_solve,spmv_group",
                         [(1, 1, 1, 4), (2, 3, 2, 8), (3, 16, 1, 32), (4, 8, 2, 16),
                          (5, 2, 1, 8), (6, 4, 2, 4), (7, 1, 1, 16),
                          (8, 2, 2, 8), (9, 4, 1, 16)])
def test_every_variant_matches_oracle(eig_solve, eig_splits, fine_solve, spmv_group):
    # the problem of the two-level parity test, where the default shapes meet these bounds
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e6, seed=5)
    o = Oracle(prob, fine_vectors=8)
    from paper_2106_06404_amd import binding as B
    arrs = B.problem_arrays(prob, device="cuda:0")
    m = B.Msdd()
    m.set_tuning(eig_solve=eig_solve, eig_splits=eig_splits, fine_solve=fine_solve,
                 spmv_group=spmv_group)
    m.setup(**arrs)
    _check_fine_level(m, o, prob, prob.eta)
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
    m.close()


def test_set_tuning_rejects_out_of_range():
    from paper_2106_06404_amd import binding as B
    m = B.Msdd()
    for kw in ({"eig_solve": 10}, {"eig_splits": 17}, {"fine_solve": 4}, {"spmv_group": 12}):
        with pytest.raises(B.MsddError):
            m.set_tuning(**kw)
    with pytest.raises(B.MsddError):
        m.autotune()  # no setup yet
    m.close()


def test_autotune_picks_measured_shapes_and_keeps_results():
    prob = P.small_problem(N=48, P=4, delta=2, contrast=1e4, seed=2)
    m, arrs = _setup(prob)
    it0, _, x0 = _solve(m, prob)
    lam0 = [m.eigs(1, i, 0) for i in range(prob.n_sub)]
    t = m.autotune(reps=3)
    assert t["eig_solve"] in (1, 2, 3, 4, 5, 6, 7, 8, 9) and t["eig_splits"] in (1, 2, 4, 8, 16)
    assert t["fine_solve"] in (1, 2, 3) and t["spmv_group"] in (4, 8, 16, 32)
    # the choice is the fastest measured candidate
    assert t["eig_solve_ms"][t["eig_solve"]] == min(v for v in t["eig_solve_ms"][1:] if v > 0)
    assert t["spmv_ms"][[4, 8, 16, 32].index(t["spmv_group"])] == min(t["spmv_ms"])
    assert all(v > 0 for v in t["spmv_ms"]) and all(v > 0 for v in t["eig_splits_ms"])
    # the solve with the tuned shapes, and a new setup with them
    it1, _, x1 = _solve(m, prob)
    assert abs(it1 - it0) <= 1 and np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-8
    m.setup(**arrs)
    for i in range(prob.n_sub):
        l1 = m.eigs(1, i, 0)   # the selected pairs
        assert len(l1) == len(lam0[i])
        assert np.all(np.abs(l1 - lam0[i]) <= 1e-10 * np.maximum(np.abs(lam0[i]), prob.eta))
    m.close()


@pytest.mark.parametrize("N,Pn,delta,contrast,seed",
                         [(24, 2, 1, 1e6, 7), (30, 2, 2, 1e4, 8), (36, 3, 1, 1e6, 9)])
def test_two_sided_solves_match_oracle(N, Pn, delta, contrast, seed):
    """Two-sided Dirichlet solves (fine_solve = 3: the rows before and after a separator as
    two chains, the separator through the explicit inverse of its Schur complement) on
    meshes whose subdomains all split (Neumann spaces of 169 to 289 dofs, Dirichlet row
    counts ragged against the 64-row blocks): the preconditioner apply against the oracle's
    within the apply bar, PCG within +-1 iteration and 1e-8 of the oracle's solution; in
    single precision (scaled factors) the mixed bars (iterations within 3, true residual
    within 10x of the oracle's)."""
    from paper_2106_06404_amd import binding as B
    prob = P.small_problem(N=N, P=Pn, delta=delta, contrast=contrast, seed=seed)
    o = Oracle(prob, fine_vectors=8)
    ro = o.solve()
    tr_o = np.linalg.norm(prob.b - prob.A @ ro.x) / np.linalg.norm(prob.b)
    arrs = B.problem_arrays(prob, device="cuda:0")
    for prec in (B.MSDD_FP64, B.MSDD_MIXED):
        m = B.Msdd(precision=prec)
        m.set_tuning(fine_solve=3)  # the setup builds the two-sided factors
        m.setup(**arrs)
        t = m.autotune(B.MSDD_TUNE_SOLVE, reps=1)
        assert t["fine_solve_ms"][3] > 0  # they were built for this mesh
        m.set_tuning(fine_solve=3)
        it, rel, x = _solve(m, prob)
        tr = np.linalg.norm(prob.b - prob.A @ x) / np.linalg.norm(prob.b)
        if prec == B.MSDD_FP64:
            assert _apply_rel(m, o, prob) < APPLY_BAR
            assert abs(it - ro.iters) <= 1
            assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
        else:
            assert rel < 1e-8 and abs(it - ro.iters) <= 3
            assert tr <= 10 * tr_o + 1e-12
        print(f"two-sided N={N} P={Pn} {'FP64' if prec == B.MSDD_FP64 else 'mixed'}: "
              f"iterations {it} (oracle {ro.iters}), true residual {tr:.2e} (oracle {tr_o:.2e})")
        m.close()


def test_two_sided_solves_on_512x512_workload():
    """The two-sided Dirichlet solves on the 512x512 inclusions workload (1225-row
    subdomains, half-bandwidth 36: the largest shape whose vector, tables and separator
    inverse fit in LDS) against the oracle's full run (tests/golden/c2_oracle): PCG within
    the +-3 iterations and the 1e-8 solution bar of that workload's parity test."""
    import json
    import os
    from paper_2106_06404_amd import binding as B
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle")
    if not os.path.exists(gold + ".npz"):
        pytest.skip("c2 golden not generated")
    with open(gold + ".json") as f:
        g = json.load(f)
    xo = np.load(gold + ".npz")["x"]
    prob = P.config2()
    m = B.Msdd()
    m.set_tuning(fine_solve=3)
    m.setup(**B.problem_arrays(prob, device="cuda:0"))
    assert m.autotune(B.MSDD_TUNE_SOLVE, reps=2)["fine_solve_ms"][3] > 0
    m.set_tuning(fine_solve=3)
    it, rel, x = _solve(m, prob)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"two-sided 512x512: iterations {it} (oracle {g['pcg']['iters']}), solution {err:.1e}")
    assert rel < 1e-8 and abs(it - g["pcg"]["iters"]) <= 3 and err < 1e-8
    m.close()
