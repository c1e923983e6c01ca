"""msdd_solve_noalloc, the solve for callers that cannot allocate device memory, against
msdd_solve through the C ABI: two calls in a row on one device, the second on a smaller
problem (the shared scratch array still holds the first call's data), each to the parity
bar of the solve (same iteration count, solution within 1e-8, residual history), and its
error paths (host pointers, a request beyond the scratch size)."""
import numpy as np
import pytest

from msdd_inputs import problems as P

pytestmark = pytest.mark.gpu


def _run(prob):
    import torch
    from paper_2106_06404_amd import binding as B
    m = B.Msdd()
    m.setup(**B.problem_arrays(prob, device="cuda:0"))
    b = torch.from_numpy(prob.b).cuda()
    x_ref = torch.zeros_like(b)
    it_ref, rel_ref, _ = m.solve(b, x_ref, 1e-8, 1000)
    h_ref = m.history()
    x = torch.zeros_like(b)
    it, rel, _ = m.solve_noalloc(b, x, 1e-8, 1000)
    torch.cuda.synchronize()
    h = m.history()
    return m, (it_ref, rel_ref, x_ref.cpu().numpy(), h_ref), (it, rel, x.cpu().numpy(), h)


def test_noalloc_solve_matches_solve_on_two_calls():
    probs = [P.small_problem(N=48, P=6, delta=2, contrast=1e6, n_levels=3, groups=(3,), seed=31),
             P.small_problem(N=20, P=4, delta=1, contrast=1e4, seed=32)]
    assert probs[1].n < probs[0].n
    for prob in probs:
        m, ref, got = _run(prob)
        it_ref, rel_ref, x_ref, h_ref = ref
        it, rel, x, h = got
        assert it == it_ref and rel < 1e-8
        assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) <= 1e-8
        assert len(h) == len(h_ref) and np.allclose(h, h_ref, rtol=1e-6, atol=0.0)
        m.close()


def test_noalloc_solve_error_paths():
    import torch
    from paper_2106_06404_amd import binding as B
    prob = P.small_problem(N=16, P=4, delta=1, contrast=1e4, seed=3)
    m = B.Msdd()
    b = torch.from_numpy(prob.b).cuda()
    with pytest.raises(B.MsddError) as e:
        m.solve_noalloc(b, torch.zeros_like(b))
    assert e.value.code == B.MSDD_ESTATE
    m.setup(**B.problem_arrays(prob, device="cuda:0"))
    with pytest.raises(B.MsddError) as e:      # host pointers
        m.solve_noalloc(prob.b.copy(), np.zeros(prob.n))
    assert e.value.code == B.MSDD_EINVAL
    with pytest.raises(B.MsddError) as e:      # history beyond the scratch size
        m.solve_noalloc(b, torch.zeros_like(b), 1e-8, 10_000_000)
    assert e.value.code == B.MSDD_EINVAL and "scratch" in str(e.value)
    it, rel, _ = m.solve_noalloc(b, torch.zeros_like(b), 1e-8, 1000)   # still usable
    assert rel < 1e-8
    m.close()
