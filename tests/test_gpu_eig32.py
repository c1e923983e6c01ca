"""The finest-level eigensolver with a single-precision factor of S (eig_fp32 = 1: the
scaled FP32 factor as the preconditioner of the block iteration, S Y formed in FP64 for
the Rayleigh-Ritz step) against the oracle, to the bars of the FP64 eigensolver: every
count, every selected eigenvalue to the per-pair bar against the binary128 references,
the pair that certifies the count, coarse-space blocks, the preconditioner apply and PCG
(iterations +-1, solution 1e-8) on 2- and 3-level meshes up to contrast 1e6, and the
512x512 workload against its stored oracle run (tests/golden/c2_oracle.*) with the bars
of that workload's parity test.  Alone and with the FP32 preconditioner (MSDD_MIXED).
Subdomains whose FP32-factor iteration does not certify its count in 64 iterations are
solved again with the FP64 factor (none on the 512x512 workload since abar Y is formed in
difference form); the bars hold for either."""
import os

import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle
from test_gpu_parity import (APPLY_BAR, HERE, _apply_rel, _check_fine_level,
                             _check_golden_fine_level, _golden, _rel, _setup, _solve)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("contrast,seed", [(1.0, 0), (1e4, 3), (1e6, 5)])
def test_eig32_two_level_against_oracle(contrast, seed):
    prob = P.small_problem(N=16, P=4, delta=1, contrast=contrast, seed=seed)
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob, eig_fp32=1)
    _check_fine_level(m, o, prob, prob.eta)
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert _rel(x, ro.x) < 1e-8
    m.close()


def test_eig32_three_level_against_oracle():
    prob = P.small_problem(N=20, P=4, delta=2, contrast=1e4, n_levels=3, groups=(2,), seed=12)
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob, eig_fp32=1)
    _check_fine_level(m, o, prob, prob.eta)
    lev = o.levels[1]
    assert list(m.level_counts(1, lev.n_sub)) == list(lev.m)
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert _rel(x, ro.x) < 1e-8
    m.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_eig32_512x512_against_golden(mixed):
    from paper_2106_06404_amd import binding as B
    if not os.path.exists(os.path.join(HERE, "golden", "c2_oracle.npz")):
        pytest.skip("c2 golden not generated")
    g, arr = _golden("c2")
    prob = P.config2()
    m, _ = _setup(prob, eig_fp32=1, precision=B.MSDD_MIXED if mixed else B.MSDD_FP64)
    st = m.stats()
    assert st["eig_unconverged"] == 0
    _check_golden_fine_level(m, prob, g, arr)
    lev1 = g["levels"]["1"]
    assert list(m.level_counts(1, len(lev1["m"]))) == lev1["m"]
    for i in range(len(lev1["m"])):
        lg = m.eigs(1, i, 0)
        lo = np.array(lev1["lam"][i][:len(lg)])
        assert np.all(np.abs(lg - lo) <= 1e-6 * np.maximum(np.abs(lo), prob.eta)), i
    it, rel, x = _solve(m, prob)
    print(f"eig32 512x512 {'mixed' if mixed else 'FP64'}: eigensolver iterations max "
          f"{st['eig_iters_max']}, FP64 fallbacks {st['eig_fp64_fallbacks']}, PCG {it} (oracle {g['pcg']['iters']}), solution "
          f"{_rel(x, arr['x']):.1e}")
    if mixed:
        assert rel < 1e-8 and abs(it - g["pcg"]["iters"]) <= 5
    else:
        assert abs(it - g["pcg"]["iters"]) <= 3
        assert _rel(x, arr["x"]) < 1e-8
    m.close()


def test_eig32_option_rules():
    from paper_2106_06404_amd import binding as B
    with pytest.raises(B.MsddError):
        B.Msdd(eig_fp32=1, geneo_rhs=2)
    with pytest.raises(B.MsddError):
        B.Msdd(eig_fp32=2)
