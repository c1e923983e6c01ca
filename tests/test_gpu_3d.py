"""3D workloads on the GPU against the oracle: Q1 diffusion and trilinear elasticity
(3 dofs per node, clamped on x = 0, layered fibre/matrix material).  The elasticity
subdomains have half-bandwidths above 64, so these cases run the library's wide-band
paths (global-memory band Cholesky, one-wavefront blocked band sweeps).  Floating
elasticity subdomains have the six rigid body modes in the kernel of abar, so their
GEVPs have a cluster at lambda = 0; eigenvalues and subspaces are compared, as in
the 2D tests."""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle
from test_gpu_parity import APPLY_BAR, _apply_rel, _check_fine_level, _setup, _solve

pytestmark = pytest.mark.gpu

CASES = {
    "q1_2lev": lambda: P.small_problem(N=8, P=2, delta=1, dim=3, contrast=1e4, seed=7),
    "q1_3lev": lambda: P.small_problem(N=8, P=4, delta=1, dim=3, n_levels=3, groups=(2,),
                                       contrast=1e4, seed=8),
    "elasticity_2lev": lambda: P.small_elasticity(N=6, P=2, delta=1),
    "elasticity_3lev": lambda: P.small_elasticity(N=8, P=4, delta=1, n_levels=3, groups=(2,)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_3d_against_oracle(case):
    prob = CASES[case]()
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob)
    _check_fine_level(m, o, prob, prob.eta)
    L = prob.n_levels - 1
    for l in range(1, L):
        lev = o.levels[l]
        assert list(m.level_counts(l, lev.n_sub)) == list(lev.m)
        for i in range(lev.n_sub):
            lg = m.eigs(l, i, 0)
            assert np.all((lg >= -1e-12) & (lg < prob.eta)) and len(lg) == lev.m[i]
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
    if case.startswith("elasticity"):
        assert m.stats()["max_band"] >= 64   # the wide-band kernels ran
    m.close()
