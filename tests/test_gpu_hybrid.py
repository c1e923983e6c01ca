"""The hybrid form of the preconditioner (restricted additive Schwarz within levels,
multiplicative over levels) and GMRES on the GPU, through the C ABI, against the oracle's
hybrid form and GMRES (Sec. 2.1; Sec. 5).

Tolerances.  The hybrid apply subtracts A z from r before every coarser correction; at high
contrast A z has entries far larger than the residual it leaves (the restricted weighting
leaves jumps of z inside high-coefficient regions), so rounding in that difference is
amplified by |A||z| / |r - A z|, and so is any difference between two valid FP64 coarse
spaces (the level-1 generating systems are numerically rank deficient and two reductions
differ by up to ~1e-7 in their eigenvalues): the operator's norm ||A M|| reaches ~2e5 at
contrast 1e6.  The apply is therefore compared elementwise where the coarse spaces agree to
rounding -- two levels (level 0 is the Galerkin matrix of the finest spaces), and three and
four levels at contrast 1 -- within
    64 u (|| |A| |z| || / || r ||) + 1e-12
relative (z the oracle's result: the first-order effect of relative rounding of a few tens of
u in the products A z of every level's correction).  Every case is compared through GMRES,
which stops on its least-squares residual: the recomputed residual below the tolerance plus
64 times its FP64 rounding floor u || |A| |x| + |b| ||, the solution within the accuracy that
fixes, ||x - x*||_A / ||x*||_A <= sqrt(kappa) 1e-8 against a dense direct solve, and, where the
applies agree elementwise, the iteration at which the least-squares residual first meets
the tolerance within +-1 of the oracle's (the refinement cycle that may follow is decided by
the recomputed residual against the tolerance, a comparison at the rounding level, so it
can be taken on one side only); where the two operators differ by up to ~1e-6 the Krylov
iterations are not comparable step by step and only the converged solutions are."""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle.msdd_oracle import Oracle
from test_gpu_parity import _setup

pytestmark = pytest.mark.gpu

CASES = {
    "2lev_1": dict(N=16, P=4, delta=1, contrast=1.0, seed=0),
    "3lev_1": dict(N=20, P=4, delta=2, contrast=1.0, n_levels=3, groups=(2,), seed=12),
    "4lev_1": dict(N=32, P=8, delta=1, contrast=1.0, n_levels=4, groups=(2, 2), seed=14),
    "2lev_1e4": dict(N=16, P=4, delta=2, contrast=1e4, seed=3),
    "2lev_1e6": dict(N=23, P=3, delta=2, contrast=1e6, seed=21),
    "3lev_1e4": dict(N=20, P=4, delta=2, contrast=1e4, n_levels=3, groups=(2,), seed=12),
    "3lev_1e6": dict(N=16, P=4, delta=2, contrast=1e6, n_levels=3, groups=(2,), seed=12),
    "4lev_1e4": dict(N=32, P=8, delta=1, contrast=1e4, n_levels=4, groups=(2, 2), seed=14),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_hybrid_apply_and_gmres_against_oracle(case):
    import torch
    prob = P.small_problem(**CASES[case])
    o = Oracle(prob)
    m, _ = _setup(prob)
    u = 2.0 ** -53
    A = prob.A
    rng = np.random.default_rng(1)
    elementwise = prob.n_levels == 2 or CASES[case]["contrast"] == 1.0
    for _ in range(2):
        r = rng.standard_normal(prob.n)
        zo = o.apply_hybrid(r)
        rt = torch.from_numpy(r).cuda()
        zt = torch.zeros_like(rt)
        m.apply_hybrid(rt, zt)
        torch.cuda.synchronize()
        zg = zt.cpu().numpy()
        absA = abs(A)
        bar = 64 * u * np.linalg.norm(absA @ np.abs(zo)) / np.linalg.norm(r) + 1e-12
        rel = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
        print(f"{case}: hybrid apply rel diff {rel:.2e} (bar {bar:.2e})")
        if elementwise:
            assert rel <= bar
    b = torch.from_numpy(prob.b).cuda()
    x = torch.zeros_like(b)
    it, rel, _ = m.solve_gmres(b, x, 1e-8, 200, 1000)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    ro = o.solve_gmres(rtol=1e-8)
    print(f"{case}: GMRES iterations {it} (oracle {ro.iters}), true relres {rel:.2e}")
    assert ro.converged
    h = m.history()
    assert len(h) == it + 1
    first_g = int(np.argmax(h < 1e-8))
    first_o = int(np.argmax(np.array(ro.resnorms) < 1e-8 * ro.resnorms[0]))
    print(f"{case}: least-squares residual below the tolerance at {first_g} (oracle {first_o})")
    assert first_g > 0 and first_o > 0
    if elementwise:
        assert abs(first_g - first_o) <= 1
    Ad = A.toarray()
    bn = np.linalg.norm(prob.b)
    floor = u * np.linalg.norm(abs(A) @ np.abs(xg) + np.abs(prob.b)) / bn
    assert np.linalg.norm(prob.b - Ad @ xg) / bn < 1e-8 + 64 * floor
    assert rel < 1e-8 + 64 * floor
    xs = np.linalg.solve(Ad, prob.b)
    kap = np.linalg.cond(Ad)
    e = xg - xs
    assert np.sqrt(e @ Ad @ e) <= np.sqrt(kap) * 1e-8 * np.sqrt(xs @ Ad @ xs)
    assert h[-1] < 1e-8
    m.close()


def test_hybrid_one_subdomain_one_iteration():
    import torch
    prob = P.small_problem(N=10, P=1, delta=0, contrast=1e3, seed=3)
    m, _ = _setup(prob)
    b = torch.from_numpy(prob.b).cuda()
    x = torch.zeros_like(b)
    it, rel, _ = m.solve_gmres(b, x, 1e-8, 50, 100)
    assert it == 1 and rel < 1e-8
    m.close()


def test_hybrid_rejected_for_batches():
    from paper_2106_06404_amd import binding as B
    probs = [P.small_problem(N=12, P=2, delta=1, contrast=1e3, seed=5),
             P.small_problem(N=16, P=4, delta=1, contrast=1e3, seed=6)]
    m = B.Msdd()
    m.setup_batch(**B.batch_arrays(probs, device="cuda:0"))
    import torch
    b = torch.from_numpy(np.concatenate([p.b for p in probs])).cuda()
    with pytest.raises(B.MsddError) as e:
        m.solve_gmres(b, torch.zeros_like(b))
    assert e.value.code == B.MSDD_EINVAL
    m.close()
