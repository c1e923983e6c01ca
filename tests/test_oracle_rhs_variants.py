"""Pins of the oracle's GEVP right-hand sides b^2 (original GenEO: the overlap elements'
sum) and b^3 ((1 - chi) on both sides), and of the fixed-n_ev selection (Sec. 3.4, Sec. 5).

  * the overlap element sets against the box geometry of the partition;
  * eigenvalues against LAPACK's generalized symmetric eigensolver, counts against
    Sylvester inertia, for each right-hand side;
  * the single subdomain covering Omega (chi = 1): b^2 and b^3 vanish, every eigenvalue is
    infinite and no eigenvector is selected;
  * the local stability constants of the lemma for the three choices,
    ||chi (I - Pi) v||_a^2 <= C_1 ||v||_abar^2 with C_1 = 1/eta, 1 + 1/eta, 2 (1 + 1/eta),
    as the supremum over v (a planted b^2 on the wrong element set violates its constant);
  * fixed n_ev: the n_ev smallest eigenvalues of the LAPACK spectrum.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from msdd_inputs import problems as P
from oracle import msdd_oracle as O
from oracle._dense import jacobi_eigh


def _local(p, i, alpha):
    dofs = p.sub_dofs(i)
    d = p.sub_weights(i)
    el = p.sub_elems(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, el, dofs)
    Ao = None
    if alpha == 2:
        subs = [p.sub_elems(j) for j in range(p.n_sub)]
        Ao = O.neumann_matrix(p.elem_dofs, p.elem_mat, O.overlap_elements(subs, i), dofs)
    return Ab, O.gevp_rhs(alpha, Ab, d, Ao), d


def _boxes_containing(p, delta):
    """Number of overlapping boxes (box partition with `delta` element layers) that contain
    each element, from the element's grid position."""
    N = p.N
    Px, Py = p.box_shape
    ec = P.element_coords(2, N)          # element (x, y) grid indices
    cnt = np.zeros(len(ec), np.int64)
    for bx in range(Px):
        x0, x1 = bx * N // Px - delta, (bx + 1) * N // Px + delta
        for by in range(Py):
            y0, y1 = by * N // Py - delta, (by + 1) * N // Py + delta
            cnt += ((ec[:, 0] >= x0) & (ec[:, 0] < x1) & (ec[:, 1] >= y0) & (ec[:, 1] < y1))
    return cnt


@pytest.mark.parametrize("N,Pn,delta", [(12, 3, 1), (16, 4, 2), (23, 3, 2)])
def test_overlap_elements_from_geometry(N, Pn, delta):
    p = P.small_problem(N=N, P=Pn, delta=delta, contrast=1e3, seed=4)
    cnt = _boxes_containing(p, delta)
    subs = [p.sub_elems(j) for j in range(p.n_sub)]
    for i in range(p.n_sub):
        el = p.sub_elems(i)
        ref = np.sort(el[cnt[el] >= 2])
        assert np.array_equal(np.sort(O.overlap_elements(subs, i)), ref), i


@pytest.mark.parametrize("alpha", [1, 2, 3])
@pytest.mark.parametrize("contrast,seed", [(1.0, 0), (1e3, 2)])
def test_rhs_variants_against_lapack_and_inertia(alpha, contrast, seed):
    p = P.small_problem(N=10, P=2, delta=2, contrast=contrast, seed=seed)
    for i in range(p.n_sub):
        Ab, Bm, d = _local(p, i, alpha)
        g = O.gevp_definite(Ab, Bm, 0.3)
        mu_ref = sla.eigh(Bm, Ab + Bm, eigvals_only=True)[::-1]
        mu_ref = np.where(mu_ref > O.MU_ZERO, mu_ref, 0.0)
        assert np.max(np.abs(mu_ref - g.mu)) < 1e-11 * max(1.0, contrast / 1e2)
        assert np.all(g.lam >= 0.0)
        w, _ = jacobi_eigh(Ab - 0.3 * Bm)
        assert g.m == int(np.sum(w < 0)), (alpha, i)


@pytest.mark.parametrize("alpha,m_expected", [(1, None), (2, 0), (3, 0)])
def test_one_subdomain_rhs_variants(alpha, m_expected):
    """chi = 1 on one subdomain covering Omega: b^1 = abar (every lambda = 1); b^2 = 0 (no
    other subdomain, so no overlap element) and b^3 = 0: no finite eigenvalue, m = 0."""
    p = P.small_problem(N=9, P=1, delta=0, contrast=1e3, seed=2)
    Ab, Bm, d = _local(p, 0, alpha)
    assert np.all(d == 1.0)
    g = O.gevp_definite(Ab, Bm, 2.0)
    if alpha == 1:
        assert np.max(np.abs(g.lam - 1.0)) < 1e-12 and g.m == len(d)
    else:
        assert len(g.lam) == 0 and g.m == m_expected


def _stability_ratio(Ab, Bm, d, eta):
    """sup over v of ||chi (I - Pi) v||_a^2 / ||v||_abar^2, Pi the b-orthogonal projection
    onto the eigenvectors with lambda < eta (a(chi w, chi w) = w^T D abar D w for functions
    vanishing on the interior subdomain boundary).  The kernel of abar (constants of a
    floating subdomain) lies in the selected span, so (I - Pi) annihilates it; the sup is
    the largest eigenvalue of the numerator's matrix on range(abar), scaled by abar^{-1/2}."""
    g = O.gevp_definite(Ab, Bm, eta)
    X = g.X
    n = len(d)
    Pm = np.eye(n) - (X @ (X.T @ Bm) if g.m else 0.0)
    M = Pm.T @ (d[:, None] * Ab * d[None, :]) @ Pm
    w, Q = np.linalg.eigh(0.5 * (Ab + Ab.T))
    keep = w > 1e-12 * w.max()
    Z = Q[:, keep] / np.sqrt(w[keep])[None, :]
    return float(np.linalg.eigvalsh(Z.T @ M @ Z).max())


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_local_stability_constants(alpha):
    eta = 0.2
    C1 = {1: 1.0 / eta, 2: 1.0 + 1.0 / eta, 3: 2.0 * (1.0 + 1.0 / eta)}[alpha]
    p = P.small_problem(N=16, P=4, delta=2, contrast=1e4, seed=9)
    for i in range(p.n_sub):
        Ab, Bm, d = _local(p, i, alpha)
        assert _stability_ratio(Ab, Bm, d, eta) <= C1 * (1 + 1e-9), (alpha, i)


def test_planted_b2_on_interior_elements_is_caught():
    """b^2 assembled on the elements that belong to no other subdomain (the complement of
    the overlap) breaks the alpha = 2 constant, or the overlap geometry pin above."""
    eta = 0.2
    p = P.small_problem(N=16, P=4, delta=2, contrast=1e4, seed=9)
    subs = [p.sub_elems(j) for j in range(p.n_sub)]
    worst = 0.0
    for i in range(p.n_sub):
        dofs, d, el = p.sub_dofs(i), p.sub_weights(i), p.sub_elems(i)
        Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, el, dofs)
        inner = np.setdiff1d(el, O.overlap_elements(subs, i))
        Ai = O.neumann_matrix(p.elem_dofs, p.elem_mat, inner, dofs)
        Bm = d[:, None] * Ai * d[None, :]
        try:
            worst = max(worst, _stability_ratio(Ab, Bm, d, eta))
        except ArithmeticError:
            worst = np.inf   # the pencil is not even definite
    assert worst > 1.0 + 1.0 / eta


@pytest.mark.parametrize("alpha", [1, 3])
def test_fixed_nev_selects_the_smallest(alpha):
    p = P.small_problem(N=12, P=3, delta=1, contrast=1e3, seed=5)
    for i in range(p.n_sub):
        Ab, Bm, d = _local(p, i, alpha)
        g = O.gevp_definite(Ab, Bm, 0.1, nev=4)
        mu = sla.eigh(Bm, Ab + Bm, eigvals_only=True)[::-1]
        mu = mu[mu > O.MU_ZERO]
        lam = np.sort(1.0 / mu - 1.0)
        assert g.m == min(4, len(lam))
        X = g.X
        lx = np.diag(X.T @ Ab @ X) / np.diag(X.T @ Bm @ X)
        assert np.allclose(np.sort(lx), lam[:g.m], rtol=1e-8, atol=1e-12)
