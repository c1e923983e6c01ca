"""Cell-centred finite volumes and WSIP-DG (Sec. 3.5; the CCFV and DG-Q1 columns of the
SPE10 runs) on the GPU against the oracle: the inputs are cell and face terms, the finest
Dirichlet spaces hold every dof of a subdomain (dirichlet_rule = 1), and everything else is
the same path as for conforming elements.  Bars as for the conforming parity tests: counts
on every level, finest-level eigenvalues against the binary128 references, subspaces, the
apply, PCG within +-1 iteration and the solution within 1e-8."""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle
from test_gpu_parity import APPLY_BAR, _apply_rel, _check_fine_level, _setup, _solve

pytestmark = pytest.mark.gpu

CASES = {
    "fv_2lev": dict(kind="fv", N=32, P=4, delta=1, contrast=1e4, n_levels=2, groups=()),
    "fv_3lev": dict(kind="fv", N=48, P=8, delta=2, contrast=1e6, n_levels=3, groups=(2,)),
    "dg_2lev": dict(kind="dg", N=16, P=4, delta=1, contrast=1e4, n_levels=2, groups=()),
    "dg_3lev": dict(kind="dg", N=24, P=6, delta=1, contrast=1e6, n_levels=3, groups=(2,)),
}


def _problem(c):
    gen = P.fv_problem if c["kind"] == "fv" else P.dg_problem
    field = P.skeleton_field(c["N"], 8, c["contrast"])
    return gen(c["N"], field, c["P"], c["delta"], n_levels=c["n_levels"], groups=c["groups"])


@pytest.mark.parametrize("case", sorted(CASES))
def test_skeleton_against_oracle(case):
    prob = _problem(CASES[case])
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob)
    assert m.stats()["n"] == o.level_sizes()
    _check_fine_level(m, o, prob, prob.eta)
    L = prob.n_levels - 1
    for l in range(1, L):
        lev = o.levels[l]
        assert list(m.level_counts(l, lev.n_sub)) == list(lev.m), l
    rel = _apply_rel(m, o, prob)
    print(f"{case}: n {prob.n}, levels {o.level_sizes()}, apply rel diff {rel:.2e}")
    assert rel < APPLY_BAR
    it, _, x = _solve(m, prob)
    ro = o.solve()
    print(f"{case}: PCG {it} iterations (oracle {ro.iters})")
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
    m.close()


def test_dirichlet_rule_option_is_checked():
    from paper_2106_06404_amd import binding as B
    with pytest.raises(B.MsddError):
        B.Msdd(dirichlet_rule=2)
