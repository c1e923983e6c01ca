"""Pins of the cell-centred finite-volume and WSIP-DG paths (Sec. 3.5, Sec. 4.1): the inputs
written as cell and face terms, the local Neumann matrices built from the faces interior to
a subdomain, the Dirichlet spaces of all the subdomain's cells, and the oracle's multilevel
method on them.

  * generators: both discretisations of -div grad u = 1 on the unit square converge to the
    known maximum of the solution at second order;
  * a floating subdomain's Neumann matrix has exactly the constants as kernel (a face to a
    neighbour outside, wrongly kept, removes it: planted);
  * finite volumes: that matrix equals the global matrix on the subdomain's cells minus the
    transmissibilities of the faces that leave the subdomain, computed here from the field;
  * one subdomain covering the domain: every eigenvalue is 1 (b = abar) and the
    preconditioner is exact (one CG iteration);
  * three levels: the oracle's apply equals the sum of the A-orthogonal projections onto the
    subspaces of the splitting, the finest ones spanned by all the subdomain's dofs;
  * the condition estimate stays bounded as the contrast grows from 1 to 1e6; a partition
    of unity that does not vanish on the subdomains' boundary layers breaks that (planted).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from msdd_inputs import problems as P
from oracle import msdd_oracle as O

U_MAX = 0.07367135  # max of u for -div grad u = 1, u = 0 on the boundary of the unit square


def _gen(kind):
    return P.fv_problem if kind == "fv" else P.dg_problem


@pytest.mark.parametrize("kind", ["fv", "dg"])
def test_generators_converge_at_second_order(kind):
    err = []
    for N in (16, 32):
        p = _gen(kind)(N, np.ones(N * N), 2, 1)
        u = spla.spsolve(p.A.tocsc(), p.b)
        err.append(abs(u.max() - U_MAX))
        if p.n <= 4096:
            assert np.linalg.eigvalsh(p.A.toarray()).min() > 0
    assert err[1] < 0.35 * err[0] and err[1] < 3e-4, err


def _floating(p):
    """A subdomain that touches no Dirichlet boundary (an interior box)."""
    side = p.box_shape[0]
    return side + 1


@pytest.mark.parametrize("kind", ["fv", "dg"])
def test_floating_neumann_kernel_is_constants(kind):
    N = 16
    p = _gen(kind)(N, P.skeleton_field(N, 3), 4, 1)
    i = _floating(p)
    dofs = p.sub_dofs(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, p.sub_elems(i), dofs)
    w, V = np.linalg.eigh(Ab)
    scale = w[-1]
    assert np.sum(w < 1e-10 * scale) == 1
    one = np.ones(len(dofs)) / np.sqrt(len(dofs))
    assert abs(abs(V[:, 0] @ one) - 1.0) < 1e-8
    assert O.dirichlet_set(p, i, dofs).all()


def test_planted_crossing_face_removes_the_kernel():
    """Keeping the faces that leave the subdomain (a Robin-like local matrix) is caught."""
    N = 16
    p = P.fv_problem(N, P.skeleton_field(N, 3), 4, 1)
    i = _floating(p)
    dofs = p.sub_dofs(i)
    inside = np.zeros(p.n, bool)
    inside[dofs] = True
    ed = p.elem_dofs
    touching = np.nonzero(np.any((ed >= 0) & inside[np.maximum(ed, 0)], axis=1))[0]
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, touching, dofs)
    w = np.linalg.eigvalsh(Ab)
    assert np.sum(w < 1e-10 * w[-1]) == 0


def test_fv_neumann_matrix_from_transmissibilities():
    N = 16
    k = P.skeleton_field(N, 5)
    p = P.fv_problem(N, k, 4, 2)
    for i in range(p.n_sub):
        cells = p.sub_dofs(i)
        inside = np.zeros(N * N, bool)
        inside[cells] = True
        leave = np.zeros(len(cells))
        for q, c in enumerate(cells):
            x, y = c % N, c // N
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                xx, yy = x + dx, y + dy
                if 0 <= xx < N and 0 <= yy < N and not inside[xx + N * yy]:
                    o = xx + N * yy
                    leave[q] += 2.0 * k[c] * k[o] / (k[c] + k[o])
        ref = p.A[cells][:, cells].toarray() - np.diag(leave)
        Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, p.sub_elems(i), cells)
        assert np.abs(Ab - ref).max() <= 1e-12 * np.abs(ref).max(), i


@pytest.mark.parametrize("kind", ["fv", "dg"])
def test_one_subdomain_all_lambda_one_and_exact(kind):
    N = 8
    p = _gen(kind)(N, P.skeleton_field(N, 2), 1, 0)
    o = O.Oracle(p)
    lam = o.levels[p.n_levels - 1].lam[0]
    assert len(lam) == p.n and np.max(np.abs(lam - 1.0)) < 1e-10
    r = np.random.default_rng(0).standard_normal(p.n)
    z = o.apply(r)
    x = np.linalg.solve(p.A.toarray(), r)
    assert np.linalg.norm(z - x) <= 1e-10 * np.linalg.norm(x)
    assert o.solve().iters == 1


def _bases(o, p):
    bases = []
    for i in range(p.n_sub):
        dofs = p.sub_dofs(i)        # every dof of the subdomain's cells
        E = np.zeros((p.n, len(dofs)))
        E[dofs, np.arange(len(dofs))] = 1.0
        bases.append(E)
    L = o.L
    for l in range(L - 1, 0, -1):
        par = p.parents[L - 1 - l]
        owner = np.repeat(par, o.levels[l + 1].m)
        Pl = o.P[l].toarray()
        for i in range(int(par.max()) + 1):
            bases.append(Pl[:, owner == i])
    bases.append(o.P[0].toarray())
    return bases


@pytest.mark.parametrize("kind", ["fv", "dg"])
def test_three_level_apply_equals_sum_of_projections(kind):
    N = 16 if kind == "dg" else 24
    p = _gen(kind)(N, P.skeleton_field(N, 4), 4, 1, n_levels=3, groups=(2,))
    o = O.Oracle(p)
    A = p.A.toarray()
    G = np.linalg.cholesky(A)
    bases = _bases(o, p)
    rng = np.random.default_rng(7)
    for _ in range(2):
        v = rng.standard_normal(p.n)
        ref = np.zeros_like(v)
        for E in bases:
            if E.shape[1]:
                c, *_ = np.linalg.lstsq(G.T @ E, G.T @ v, rcond=None)
                ref += E @ c
        got = o.apply(A @ v)
        assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["fv", "dg"])
def test_condition_bounded_in_contrast(kind):
    N = 16 if kind == "dg" else 32
    kap = []
    for contrast in (1.0, 1e3, 1e6):
        p = _gen(kind)(N, P.skeleton_field(N, 6, contrast), 4, 1, eta=0.3)
        kap.append(O.Oracle(p).solve().kappa())
    assert max(kap) < 60.0, kap


def test_planted_pou_on_boundary_layer_is_caught():
    """A partition of unity that does not vanish on the subdomains' boundary layers (weights
    1 / multiplicity on every cell) makes b^1 differ from a(chi u, chi v): at contrast 1e6 the
    condition estimate leaves the bound above."""
    N = 32
    p = P.fv_problem(N, P.skeleton_field(N, 6, 1e6), 4, 1, eta=0.3)
    mult = np.bincount(p.sub_dof, minlength=p.n).astype(float)
    p.sub_pou = 1.0 / mult[p.sub_dof]
    assert O.Oracle(p).solve().kappa() > 60.0
