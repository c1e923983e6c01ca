"""Several problems in one setup (msdd_setup_batch) and one CG per problem
(msdd_solve_batch), against the same problems set up one by one.

Every per-subdomain computation of the batch is the computation of the single
problem (the problems share no subdomain, patch or coarse block, and the PCG
reductions chunk each problem's rows from its own first row), so the batch must
reproduce the individual runs bitwise: counts, eigenvalues, iteration counts and
solutions."""
import numpy as np
import pytest

from msdd_inputs import problems as P

pytestmark = pytest.mark.gpu


def _members(levels):
    if levels == 2:
        return [P.small_problem(N=16, P=4, delta=1, contrast=1e4, seed=3),
                P.small_problem(N=23, P=3, delta=2, contrast=1e6, seed=21),
                P.small_problem(N=12, P=2, delta=1, contrast=1.0, seed=5)]
    return [P.small_problem(N=16, P=4, delta=1, contrast=1e4, n_levels=3, groups=(2,), seed=11),
            P.small_problem(N=20, P=4, delta=2, contrast=1e4, n_levels=3, groups=(2,), seed=12),
            P.small_problem(N=24, P=6, delta=1, contrast=1e6, n_levels=3, groups=(3,), seed=13)]


@pytest.mark.parametrize("levels", [2, 3])
def test_batch_equals_individual_runs(levels):
    import torch
    from paper_2106_06404_amd import binding as B
    probs = _members(levels)
    single = []
    for prob in probs:
        m = B.Msdd()
        m.setup(**B.problem_arrays(prob, device="cuda:0"))
        L = prob.n_levels - 1
        lv = {l: [m.eigs(l, i, 0) for i in range(len(m.level_counts(l, n_l)))]
              for l, n_l in [(L, prob.n_sub)] + [(l, m.stats()["n_sub"][l]) for l in range(1, L)]}
        b = torch.from_numpy(prob.b).cuda()
        x = torch.zeros_like(b)
        it, rel, _ = m.solve(b, x, 1e-8, 1000)
        torch.cuda.synchronize()
        single.append((lv, it, x.cpu().numpy()))
        m.close()
    arrs = B.batch_arrays(probs, device="cuda:0")
    m = B.Msdd()
    m.setup_batch(**arrs)
    st = m.stats()
    assert st["n_sub"][0] == len(probs)
    L = levels - 1
    for l in range(1, L + 1):
        off = 0
        for t, prob in enumerate(probs):
            for i, lam in enumerate(single[t][0][l]):
                assert np.array_equal(m.eigs(l, off + i, 0), lam), (l, t, i)
            off += len(single[t][0][l])
    b = torch.from_numpy(np.concatenate([p.b for p in probs])).cuda()
    x = torch.zeros_like(b)
    its, rels, _ = m.solve_batch(b, x, 1e-8, 1000)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    base = 0
    for t, prob in enumerate(probs):
        assert its[t] == single[t][1], (t, its[t], single[t][1])
        assert rels[t] < 1e-8
        assert np.array_equal(xh[base:base + prob.n], single[t][2]), t
        base += prob.n
    m.close()


def test_batch_rules_are_checked():
    from paper_2106_06404_amd import binding as B
    probs = _members(2)
    arrs = B.batch_arrays(probs)
    m = B.Msdd()
    bad = dict(arrs)
    ptr = arrs["prob_dof_ptr"].copy()
    ptr[1] -= 5   # problem 0's last dofs now belong to problem 1: its subdomains straddle
    bad["prob_dof_ptr"] = ptr
    with pytest.raises(B.MsddError) as e:
        m.setup_batch(**bad)
    assert e.value.code == B.MSDD_EINVAL
    # a matrix entry of problem 0 pointing into problem 1 (subdomains unchanged): the
    # device-side check of the matrix's problem blocks rejects it
    bad = dict(arrs)
    col = arrs["col"].copy()
    col[arrs["rowptr"][0]] = arrs["prob_dof_ptr"][1]
    bad["col"] = col
    with pytest.raises(B.MsddError) as e:
        m.setup_batch(**bad)
    assert e.value.code == B.MSDD_EINVAL and "couples two problems" in str(e.value)
    m.setup_batch(**arrs)   # the context is still usable
    m.close()


def test_context_reused_from_single_to_batch():
    """One context: a single-problem setup and solve, then a batch of three on the same
    context with the same and then a smaller iteration limit.  The residual history is
    kept per problem, so the batch needs a larger history buffer than the single run;
    results must equal a fresh batch context's bitwise."""
    import torch
    from paper_2106_06404_amd import binding as B
    probs = _members(2)
    arrs = B.batch_arrays(probs, device="cuda:0")
    b = torch.from_numpy(np.concatenate([p.b for p in probs])).cuda()

    fresh = B.Msdd()
    fresh.setup_batch(**arrs)
    x_ref = torch.zeros_like(b)
    its_ref, _, _ = fresh.solve_batch(b, x_ref, 1e-8, 200)
    h_ref = fresh.history()
    torch.cuda.synchronize()
    fresh.close()

    m = B.Msdd()
    m.setup(**B.problem_arrays(probs[0], device="cuda:0"))
    b0 = torch.from_numpy(probs[0].b).cuda()
    x0 = torch.zeros_like(b0)
    it0, _, _ = m.solve(b0, x0, 1e-8, 200)
    h0 = m.history()
    assert len(h0) == it0 + 1
    for maxit in (200, 100):
        m.setup_batch(**arrs)
        x = torch.zeros_like(b)
        its, rels, _ = m.solve_batch(b, x, 1e-8, maxit)
        torch.cuda.synchronize()
        assert list(its) == list(its_ref)
        assert np.array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
        h = m.history()
        assert np.array_equal(h, h_ref)
        assert np.array_equal(h, h0)   # problem 0 of the batch is the single problem
    m.close()
