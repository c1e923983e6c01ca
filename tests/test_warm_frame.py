"""Host logic of the warm-start frame layout (msdd_inputs.problems.warm_frame), CPU only."""
import numpy as np

from msdd_inputs import problems as P


def test_frame_layout_small():
    prob = P.small_problem(N=12, P=3, delta=1, contrast=1e3, seed=2)
    feat, sub_pos, n_pos = P.warm_frame(prob, 1)
    E = 4 + 2  # core 4 elements + overlap on both sides
    assert n_pos == (E + 1) ** 2 and feat.shape == (9, 2 * E * E + 4)
    coords = P.free_dof_coords(prob)[0] * prob.N
    for i in range(prob.n_sub):
        el = prob.sub_elems(i)
        pres = feat[i, E * E:2 * E * E]
        assert pres.sum() == len(el) and set(np.unique(pres)) <= {0.0, 1.0}
        # the coefficient channel carries log10(k)/4 on present elements only
        vals = feat[i, :E * E]
        assert np.allclose(np.sort(vals[pres == 1]), np.sort(np.log10(prob.coeff[el]) / 4.0))
        assert np.all(vals[pres == 0] == 0)
        lo, hi = prob.sub_dof_ptr[i], prob.sub_dof_ptr[i + 1]
        pos = sub_pos[lo:hi]
        assert len(np.unique(pos)) == len(pos) and pos.min() >= 0 and pos.max() < n_pos
        # frame position = node coordinates relative to the box origin (cut - delta)
        bx, by = i % 3, i // 3
        origin = np.array([4 * bx - 1, 4 * by - 1])
        xy = np.rint(coords[prob.sub_dof[lo:hi]]).astype(int) - origin
        assert np.array_equal(pos, xy[:, 0] + (E + 1) * xy[:, 1])
        flags = feat[i, 2 * E * E:]
        assert np.array_equal(flags, [bx == 0, bx == 2, by == 0, by == 2])
