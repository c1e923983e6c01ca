"""The host planner on the GPU path: a setup does not depend on how the caller numbers the
elements.  On a 288x288 three-level mesh (331776 element-dof entries: six element ranges on
a host with six threads or more) the planner counts the elements of every dof over element
ranges in parallel, each range in a window of the dofs it touches; with the elements
renumbered by a seeded random permutation every window spans the whole mesh, their sum
exceeds 4 n, and the count takes its serial path instead.  Both numberings
must give the same preconditioner: equal coarse-space counts on every level, the same
selected eigenvalues up to rounding (the numbering changes only the summation order of the
assembly; bar 1e-10 relative to max(lambda, eta), as for repeated setups), PCG within one
iteration and 1e-8 of the same solution."""
import numpy as np
import pytest
import scipy.sparse as sp

from msdd_inputs import problems as P
from test_gpu_parity import _rel, _solve

pytestmark = pytest.mark.gpu


def _renumbered(arrs, seed):
    """The same problem with element q of the new numbering = element perm[q] of the old."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ne = arrs["elem_dofs"].shape[0]
    perm = rng.permutation(ne)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(ne)
    out = dict(arrs)
    out["elem_dofs"] = np.ascontiguousarray(arrs["elem_dofs"][perm])
    out["elem_mat"] = np.ascontiguousarray(arrs["elem_mat"][perm])
    out["sub_elem"] = np.ascontiguousarray(inv[arrs["sub_elem"]].astype(np.int32))
    return out


def _assembled(arrs, n):
    """sum over elements of the element matrices on the free dofs (CPU)."""
    ed = arrs["elem_dofs"]
    k = ed.shape[1]
    em = arrs["elem_mat"].reshape(-1, k, k)
    r = np.repeat(ed, k, axis=1).ravel()
    c = np.tile(ed, (1, k)).ravel()
    v = em.reshape(len(ed), -1).ravel()
    keep = (r >= 0) & (c >= 0)
    return sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(n, n))


def test_setup_does_not_depend_on_element_numbering():
    import torch
    from paper_2106_06404_amd import binding as B
    prob = P.small_problem(N=288, P=9, delta=2, contrast=1e4, n_levels=3, groups=(3,), seed=31)
    a0 = B.problem_arrays(prob)
    a1 = _renumbered(a0, 7)
    assert a0["elem_dofs"].size > 5 * 65536
    # the renumbered input describes the same matrix and the same subdomains
    diff = _assembled(a1, prob.n) - prob.A
    assert abs(diff).max() <= 1e-12 * abs(prob.A).max()
    for i in range(prob.n_sub):
        lo, hi = a0["sub_elem_ptr"][i], a0["sub_elem_ptr"][i + 1]
        assert np.array_equal(np.sort(a1["elem_dofs"][a1["sub_elem"][lo:hi]], axis=None),
                              np.sort(a0["elem_dofs"][a0["sub_elem"][lo:hi]], axis=None))
    runs = []
    for arrs in (a0, a1):
        dev = {key: torch.from_numpy(v).to("cuda:0") if isinstance(v, np.ndarray) else v
               for key, v in arrs.items()}
        m = B.Msdd()
        m.setup(**dev)
        st = m.stats()
        counts = [list(m.level_counts(l, st["n_sub"][l])) for l in range(1, prob.n_levels)]
        L = prob.n_levels - 1
        lam = [m.eigs(L, i, 0) for i in range(prob.n_sub)]
        it, rel, x = _solve(m, prob)
        m.close()
        runs.append((counts, lam, it, x))
    (c0, l0, it0, x0), (c1, l1, it1, x1) = runs
    assert c0 == c1
    for i in range(prob.n_sub):
        assert len(l0[i]) == len(l1[i])
        assert np.all(np.abs(l1[i] - l0[i]) <= 1e-10 * np.maximum(np.abs(l0[i]), prob.eta)), i
    assert abs(it1 - it0) <= 1
    assert _rel(x1, x0) < 1e-8
    print(f"element renumbering: counts {[int(v) for v in c0[-1][:4]]}..., PCG {it0} / {it1}, "
          f"solution {_rel(x1, x0):.1e}")
