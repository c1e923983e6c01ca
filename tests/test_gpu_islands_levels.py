"""The weak-scaling workload of the Islands problem's shape (Table 3 of the paper: Q1,
overlap 3 element layers, eta = 0.3, Dirichlet on x = 0 and x = 1, Neumann elsewhere) with
up to four levels, at a reduced size the oracle can solve (8 x 8 elements per subdomain
instead of 80 x 80, each coarse level grouping 2 x 2 subdomains of the next finer one), on
the GPU against the oracle to the bars of the plain method: counts on every level (a
coarse subdomain may select nothing), finest-level eigenvalues and coarse spaces, the
apply and PCG."""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle
from test_gpu_parity import APPLY_BAR, _apply_rel, _check_fine_level, _setup, _solve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Ps,levels", [(8, 4), (4, 3), (4, 2)])
def test_islands_shape_against_oracle(Ps, levels):
    prob = P.table3_islands(Ps, levels, elems_per_sub=8, factor=2)
    o = Oracle(prob, fine_vectors=8)
    m, _ = _setup(prob)
    assert m.stats()["n"] == o.level_sizes()
    _check_fine_level(m, o, prob, prob.eta)
    L = prob.n_levels - 1
    for l in range(1, L):
        lev = o.levels[l]
        assert list(m.level_counts(l, lev.n_sub)) == list(lev.m), l
        for i in range(lev.n_sub):
            lg = m.eigs(l, i, 0)
            assert np.all((lg >= -1e-12) & (lg < prob.eta)) and len(lg) == lev.m[i]
    assert _apply_rel(m, o, prob) < APPLY_BAR
    it, rel, x = _solve(m, prob)
    ro = o.solve()
    assert abs(it - ro.iters) <= 1
    assert np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x) < 1e-8
    m.close()


def test_islands_four_levels_hybrid_gmres():
    """The hybrid form with GMRES on the four-level islands shape: the solve meets the
    tolerance up to the FP64 rounding floor of b - A x (contrast 1e6 lifts it to the order
    of the tolerance), as the oracle's GMRES does."""
    import torch
    prob = P.table3_islands(8, 4, elems_per_sub=8, factor=2)
    o = Oracle(prob)
    m, _ = _setup(prob)
    b = torch.from_numpy(prob.b).cuda()
    x = torch.zeros_like(b)
    it, rel, _ = m.solve_gmres(b, x, 1e-8, 300, 600)
    ro = o.solve_gmres(rtol=1e-8, restart=300, maxit=600)
    xg = x.cpu().numpy()
    bn = np.linalg.norm(prob.b)
    floor = 2.0 ** -53 * np.linalg.norm(abs(prob.A) @ np.abs(xg) + np.abs(prob.b)) / bn
    print(f"islands 8x8 L4 hybrid GMRES: {it} iterations (oracle {ro.iters}), relres {rel:.2e}, "
          f"floor {floor:.2e}")
    assert ro.converged
    assert np.linalg.norm(prob.b - prob.A @ xg) / bn < 1e-8 + 64 * floor
    assert rel < 1e-8 + 64 * floor
    assert it <= 2 * ro.iters
    m.close()
