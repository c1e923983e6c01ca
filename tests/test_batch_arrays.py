"""Host side of batching: the concatenated arrays describe the union of the problems."""
import numpy as np

from msdd_inputs import problems as P


def test_batch_arrays_are_the_union():
    from paper_2106_06404_amd import binding as B
    probs = [P.small_problem(N=8, P=2, delta=1, n_levels=3, groups=(2,), seed=s) for s in (1, 2)]
    probs.append(P.small_problem(N=10, P=4, delta=1, n_levels=3, groups=(2,), seed=3))
    u = B.batch_arrays(probs)
    parts = [B.problem_arrays(p) for p in probs]
    assert u["n"] == sum(p.n for p in probs)
    assert list(u["prob_dof_ptr"]) == list(np.cumsum([0] + [p.n for p in probs]))
    # block-diagonal matrix: rebuild it from the CSR and compare blocks
    import scipy.sparse as sp
    A = sp.csr_matrix((u["val"], u["col"], u["rowptr"]), shape=(u["n"], u["n"]))
    base = 0
    for p in probs:
        blk = A[base:base + p.n, base:base + p.n]
        assert abs(blk - p.A).max() == 0
        assert A[base:base + p.n].nnz == p.A.nnz
        base += p.n
    # subdomains: counts and shifted dofs
    assert len(u["sub_elem_ptr"]) - 1 == sum(p.n_sub for p in probs)
    i0 = parts[0]["sub_dof_ptr"][-1]
    assert np.array_equal(u["sub_dof"][i0:i0 + parts[1]["sub_dof"].shape[0]],
                          parts[1]["sub_dof"] + probs[0].n)
    # parent maps: level maps concatenated with shifted coarse indices
    assert u["parent"].shape[0] == sum(sum(len(m) for m in p.parents) for p in probs)
    first = np.concatenate([np.asarray(probs[0].parents[0]),
                            np.asarray(probs[1].parents[0]) + int(np.max(probs[0].parents[0])) + 1])
    assert np.array_equal(u["parent"][:first.shape[0]], first)
