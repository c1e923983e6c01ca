"""The 32-problem log-normal batch (msdd_setup_batch + msdd_solve_batch, every problem in
one set of launches) with its three smallest members checked against the oracle's full runs
of those problems (tests/golden/c4s_oracle.json, .npz, written by make_golden.py from
oracle/ alone), to the bars of the single-problem parity tests: counts on both levels,
every selected finest-level eigenvalue against its binary128 reference (per-pair bar),
level-1 counts exact and eigenvalues within 1e-6 max(lambda, eta), sampled coarse-space
blocks within 1e-8, PCG iterations within +-3 (measured 0, 1 and 2) and the solution within
1e-8.  Run in FP64
(the plain method); the FP32-preconditioner form of the benchmark is checked for the same
members against the same results with the mixed-precision bars (iterations within 3,
solution error stated, true residual within 10x)."""
import json
import multiprocessing as mp
import os

import numpy as np
import pytest

from msdd_inputs import problems as P
from gpu_common import check_selected_and_certifying, sin_angle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "c4s_oracle")


def _golden():
    with open(GOLD + ".json") as f:
        g = json.load(f)
    return g["members"], np.load(GOLD + ".npz")


def _member(mem):
    return P.config4_problem(*mem)


@pytest.fixture(scope="module")
def batch():
    if not os.path.exists(GOLD + ".npz"):
        pytest.skip("c4s oracle results not generated yet")
    members = P.config4_members()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        probs = pool.map(_member, members)
    return members, probs


def _run(probs, precision):
    import torch
    from paper_2106_06404_amd import binding as B
    arrs = B.batch_arrays(probs, device="cuda:0")
    m = B.Msdd(precision=precision)
    m.setup_batch(**arrs)
    b = torch.from_numpy(np.concatenate([p.b for p in probs])).cuda()
    x = torch.zeros_like(b)
    its, rels, _ = m.solve_batch(b, x, 1e-8, 2000)
    torch.cuda.synchronize()
    return m, its, rels, x.cpu().numpy()


@pytest.mark.parametrize("mixed", [False, True])
def test_c4_smallest_members_against_oracle(batch, mixed):
    from paper_2106_06404_amd import binding as B
    members, probs = batch
    golds, arr = _golden()
    m, its, rels, x = _run(probs, B.MSDD_MIXED if mixed else B.MSDD_FP64)
    st = m.stats()
    assert st["eig_unconverged"] == 0
    sub_off = np.cumsum([0] + [p.n_sub for p in probs])
    n1 = [int(np.max(p.parents[0])) + 1 for p in probs]
    l1_off = np.cumsum([0] + n1)
    dof_off = np.cumsum([0] + [p.n for p in probs])
    Lf = probs[0].n_levels - 1
    counts_f = m.level_counts(Lf, int(sub_off[-1]))
    counts_1 = m.level_counts(1, int(l1_off[-1]))
    for g in golds:
        t = g["batch_position"]
        prob = probs[t]
        assert list(g["member"]) == list(members[t])
        L = prob.n_levels - 1
        fine = g["levels"][str(L)]
        ref = fine["lam_ref"]
        assert list(counts_f[sub_off[t]:sub_off[t + 1]]) == fine["m"], t
        assert list(counts_1[l1_off[t]:l1_off[t + 1]]) == g["levels"]["1"]["m"], t
        # level 1: eigenvalues to the 1e-6 max(lambda, eta) to which these rank-deficient
        # pencils are defined in FP64 (as for the single-problem workloads)
        for i, lo in enumerate(g["levels"]["1"]["lam"]):
            lg = m.eigs(1, int(l1_off[t]) + i, 0)
            lo = np.array(lo[:len(lg)])
            assert len(lo) == len(lg), (t, i)
            assert np.all(np.abs(lg - lo) <= 1e-6 * np.maximum(np.abs(lo), prob.eta)), (t, i)
        for i in range(prob.n_sub):
            lg = m.eigs(L, int(sub_off[t]) + i, 1)
            check_selected_and_certifying(lg, fine["m"][i], np.array(ref["lam"][i]),
                                          np.array(ref["unc"][i]), np.array(ref["bound"][i]),
                                          prob.eta, where=(t, i))
        for i in g["basis_subdomains"]:
            Bo = arr[f"m{t}_basis_{L}_{i}"]
            assert sin_angle(m.basis(L, int(sub_off[t]) + i), Bo) <= 1e-8, (t, i)
        xt = x[dof_off[t]:dof_off[t + 1]]
        xo = arr[f"m{t}_x"]
        err = np.linalg.norm(xt - xo) / np.linalg.norm(xo)
        tr = np.linalg.norm(prob.b - prob.A @ xt) / np.linalg.norm(prob.b)
        tro = g["pcg"]["true_relres"]
        print(f"c4 member {t} (N={prob.N}): iterations {its[t]} (oracle {g['pcg']['iters']}), "
              f"solution error {err:.2e}, true residual {tr:.2e} (oracle {tro:.2e})"
              + (" [FP32 preconditioner]" if mixed else ""))
        assert rels[t] < 1e-8
        if mixed:
            assert abs(its[t] - g["pcg"]["iters"]) <= 3
            assert tr <= 10 * tro + 1e-12
        else:
            # the level-1 coarse spaces are defined only to the 1e-6 of their rank-deficient
            # generating systems, so the two preconditioners' CG histories differ by a factor
            # up to 10^0.3 (measured 10^0.23 on the 512x512 workload); the oracle's last
            # steps contract by 0.68 on average and by as little as 0.85 (member 26 crosses
            # 1e-8 on such a step), which moves the crossing by up to 2 to 4 iterations;
            # the solution itself agrees to 1e-8 (measured 5e-13 to 9e-12)
            assert abs(its[t] - g["pcg"]["iters"]) <= 3
            assert err < 1e-8
    m.close()
