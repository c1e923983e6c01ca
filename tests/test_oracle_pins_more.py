"""More pins of the CPU oracle: the Lanczos condition estimate, the coarse generating
systems, the multilevel additive preconditioner on three and four levels, and the
binary128 refinement of local eigenpairs with its uncertainty measure.

Each test checks the oracle against something computed another way (a spectrum
fixed in advance, eigenvalues of the explicitly formed preconditioned operator,
supports read off the coarse basis functions, A-orthogonal projections by least
squares, a 40-digit reference); the planted mistakes show that the check catches
the plausible errors.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from msdd_inputs import problems as P
from oracle import msdd_oracle as O


# ---------------------------------------------------------------- Lanczos condition estimate
def _kappa_wrong_offdiag(alphas, betas):
    """Planted mistake: the Lanczos off-diagonal without its square root."""
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k and j < len(betas):
            T[j, j + 1] = T[j + 1, j] = betas[j] / alphas[j]
    w = np.linalg.eigvalsh(T)
    return float(w[-1] / w[0])


def _cg_on_known_spectrum():
    n = 60
    lam = np.linspace(1.0, 100.0, n)
    A = np.diag(lam)
    b = np.random.default_rng(0).standard_normal(n)
    return O.pcg(A, b, lambda r: r.copy(), rtol=1e-14, maxit=n)


def test_lanczos_kappa_known_spectrum():
    """CG (no preconditioner) on diag(linspace(1, 100)): the Lanczos matrix built from the
    CG coefficients has the operator's extreme eigenvalues as its extreme Ritz values, so
    the estimate is 100 (Golub-Van Loan, the CG-Lanczos relation)."""
    res = _cg_on_known_spectrum()
    assert abs(res.kappa() - 100.0) < 1e-8 * 100.0
    assert abs(_kappa_wrong_offdiag(res.alphas, res.betas) - 100.0) > 1e-3 * 100.0


def _explicit_kappa(o, p):
    n = p.n
    M = np.stack([o.apply(e) for e in np.eye(n)], 1)
    M = 0.5 * (M + M.T)
    G = np.linalg.cholesky(M)
    w = np.linalg.eigvalsh(G.T @ p.A.toarray() @ G)   # spectrum of M^{1/2} A M^{1/2}
    return w[-1] / w[0]


@pytest.mark.parametrize("levels", [2, 3])
def test_lanczos_kappa_matches_explicit_preconditioned_operator(levels):
    groups = (2,) if levels == 3 else ()
    p = P.small_problem(N=16, P=4, delta=1, contrast=1e4, n_levels=levels, groups=groups, seed=8)
    o = O.Oracle(p)
    kap = _explicit_kappa(o, p)
    res = o.solve(rtol=1e-14, maxit=500)
    assert abs(res.kappa() - kap) <= 1e-6 * kap
    assert abs(_kappa_wrong_offdiag(res.alphas, res.betas) - kap) > 1e-2 * kap


# ---------------------------------------------------------------- generating systems
def _support_generating_sets(o, p):
    """Generating system of each coarse subdomain from the basis functions themselves: the
    columns of P_l (level-l functions on the fine grid) that are nonzero on some element of
    the coarse subdomain (the union of its fine descendants' elements)."""
    out = {}
    for lc in range(o.L - 1, 0, -1):     # coarse levels with GEVPs
        Pl = o.P[lc].tocsc()
        lev = o.levels[lc]
        sets = []
        for i in range(lev.n_sub):
            elems = np.unique(np.concatenate([p.sub_elems(f) for f in o.desc[lc][i]]))
            dofs = np.unique(p.elem_dofs[elems])
            dofs = dofs[dofs >= 0]
            rows = np.zeros(p.n, bool)
            rows[dofs] = True
            cols = [c for c in range(Pl.shape[1])
                    if np.any(rows[Pl.indices[Pl.indptr[c]:Pl.indptr[c + 1]]]
                              & (Pl.data[Pl.indptr[c]:Pl.indptr[c + 1]] != 0))]
            sets.append(np.array(cols))
        out[lc] = sets
    return out


_GEN_CASES = [dict(N=16, P=4, delta=1, contrast=1e4, n_levels=3, groups=(2,), seed=11),
              dict(N=24, P=6, delta=2, contrast=1e3, n_levels=3, groups=(3,), seed=13),
              dict(N=32, P=8, delta=1, contrast=1e4, n_levels=4, groups=(2, 2), seed=14)]


@pytest.mark.parametrize("case", range(len(_GEN_CASES)))
def test_generating_sets_equal_supports(case):
    p = P.small_problem(**_GEN_CASES[case])
    o = O.Oracle(p)
    ref = _support_generating_sets(o, p)
    for lc, sets in ref.items():
        lev = o.levels[lc]
        for i in range(lev.n_sub):
            assert np.array_equal(np.sort(lev.gen_cols[i]), sets[i]), (lc, i)


def test_planted_owned_only_generating_set_is_caught(monkeypatch):
    p = P.small_problem(**_GEN_CASES[0])

    def owned_only(emask_l, emask, par, i):
        return [j for j in range(len(emask_l)) if par[j] == i]

    monkeypatch.setattr(O.Oracle, "_generating_subdomains", staticmethod(owned_only))
    o = O.Oracle(p)
    ref = _support_generating_sets(o, p)
    lev = o.levels[1]
    assert any(not np.array_equal(np.sort(lev.gen_cols[i]), ref[1][i]) for i in range(lev.n_sub))


# ---------------------------------------------------------------- multilevel additive apply
def _subspace_bases(o, p):
    """Fine-level bases of every subspace of the splitting (Sec. 2.1): the finest level's
    Dirichlet spaces, on each coarse level l the functions owned by subdomain i (children j
    with parent i; ownership derived here from the parent maps and the counts), level 0."""
    bases = []
    L = o.L
    for i in range(p.n_sub):
        dofs = p.sub_dofs(i)
        dm = O.dirichlet_mask(p.elem_dofs, p.sub_elems(i), dofs)
        E = np.zeros((p.n, int(dm.sum())))
        E[dofs[dm], np.arange(int(dm.sum()))] = 1.0
        bases.append(E)
    for l in range(L - 1, 0, -1):
        m_child = o.levels[l + 1].m                   # functions per level-(l+1) subdomain
        par = p.parents[L - 1 - l]                    # level-(l+1) subdomain -> level l
        owner = np.repeat(par, m_child)               # coarse owner of each level-l function
        Pl = o.P[l].toarray()
        for i in range(int(par.max()) + 1):
            bases.append(Pl[:, owner == i])
    bases.append(o.P[0].toarray())
    return bases


def _additive_operator_times(bases, A, v):
    """sum over subspaces of the A-orthogonal projection of v, each by least squares in
    the A inner product (A = G G^T): min_c ||G^T (v - E c)||_2."""
    G = np.linalg.cholesky(A)
    out = np.zeros_like(v)
    for E in bases:
        if E.shape[1] == 0:
            continue
        c, *_ = np.linalg.lstsq(G.T @ E, G.T @ v, rcond=None)
        out += E @ c
    return out


@pytest.mark.parametrize("case", range(len(_GEN_CASES)))
def test_multilevel_apply_equals_sum_of_projections(case):
    """B A = sum of the A-orthogonal projections onto the subspaces of the splitting
    (additive subspace correction, Sec. 2.1), for 3 and 4 levels."""
    p = P.small_problem(**_GEN_CASES[case])
    o = O.Oracle(p)
    A = p.A.toarray()
    bases = _subspace_bases(o, p)
    rng = np.random.default_rng(case)
    for _ in range(3):
        v = rng.standard_normal(p.n)
        ref = _additive_operator_times(bases, A, v)
        got = o.apply(A @ v)
        assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_planted_dropped_coarsest_level_is_caught():
    p = P.small_problem(**_GEN_CASES[0])
    o = O.Oracle(p)
    A = p.A.toarray()
    bases = _subspace_bases(o, p)
    o.P[0] = o.P[0] * 0.0          # the level-0 correction vanishes
    v = np.random.default_rng(1).standard_normal(p.n)
    ref = _additive_operator_times(bases, A, v)
    got = o.apply(A @ v)
    assert np.linalg.norm(got - ref) > 1e-3 * np.linalg.norm(ref)


# ---------------------------------------------------------------- binary128 refinement
def _exact_pencil_mp(p, i, dps=40):
    """abar as the exact sum of the element matrices and b = D abar D, in 40-digit
    arithmetic; mu of b x = mu (abar + b) x by Cholesky, inverse and symmetric eigenvalues."""
    import mpmath as mp
    mp.mp.dps = dps
    dofs = p.sub_dofs(i)
    d = p.sub_weights(i)
    eloc, emat = O.local_elements(p.elem_dofs, p.elem_mat, p.sub_elems(i), dofs)
    n = len(dofs)
    A = mp.zeros(n, n)
    for e in range(eloc.shape[0]):
        for a in range(eloc.shape[1]):
            for c in range(eloc.shape[1]):
                if eloc[e, a] >= 0 and eloc[e, c] >= 0:
                    A[int(eloc[e, a]), int(eloc[e, c])] += mp.mpf(float(emat[e, a, c]))
    B = mp.zeros(n, n)
    for a in range(n):
        for c in range(n):
            B[a, c] = mp.mpf(float(d[a])) * A[a, c] * mp.mpf(float(d[c]))
    Li = mp.inverse(mp.cholesky(A + B))
    mus = sorted(mp.eigsy(Li * B * Li.T, eigvals_only=True), reverse=True)
    return [1 / mu - 1 for mu in mus if mu > mp.mpf(10) ** -30]


def test_refine_against_40_digit_exact_assembly():
    """Contrast 1e6: the FP64 oracle's eigenvalues carry errors of up to ~1e-10 there; the
    binary128 refinement from its vectors agrees with a 40-digit computation on the exactly
    assembled pencil to within its own residual bound."""
    import mpmath as mp
    p = P.small_problem(N=10, P=2, delta=2, contrast=1e6, seed=1)
    i = 1
    dofs, d, el = p.sub_dofs(i), p.sub_weights(i), p.sub_elems(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, el, dofs)
    g = O.gevp_definite(Ab, d[:, None] * Ab * d[None, :], 0.3, extra_vec=10)
    r = O.refine_pairs(p.elem_dofs, p.elem_mat, el, dofs, d, g.V, iters=8)
    lam_mp = _exact_pencil_mp(p, i)
    k = g.m + 7
    for j in range(k):
        err = abs(mp.mpf(float(r.lam[j])) + mp.mpf(float(r.lam_lo[j])) - lam_mp[j])
        assert err <= r.bound[j] * (1 + 1e-6) + 1e-30, (j, float(err), r.bound[j])
        assert float(err) <= 1e-25 * max(1.0, float(lam_mp[j])), j
    # the bound itself is far below the parity tolerance 1e-10 max(lambda, 1e-3 eta) for the
    # selected pairs and the one that certifies the count
    assert np.all(r.bound[:g.m + 1] <= 1e-14 * np.maximum(r.lam[:g.m + 1], 1e-3 * 0.3))
    # and the unrefined FP64 oracle is off by far more than the refined values
    e64 = max(abs(float(mp.mpf(float(g.lam[j])) - lam_mp[j])) for j in range(k))
    e128 = max(abs(float(mp.mpf(float(r.lam[j])) + mp.mpf(float(r.lam_lo[j])) - lam_mp[j]))
               for j in range(k))
    assert e64 > 1e6 * e128


def test_refine_one_subdomain_all_lambda_one():
    """chi = 1 on one subdomain covering Omega: b = abar, every lambda is exactly 1."""
    p = P.small_problem(N=9, P=1, delta=0, contrast=1e3, seed=2)
    dofs, d, el = p.sub_dofs(0), p.sub_weights(0), p.sub_elems(0)
    V0 = np.linalg.qr(np.random.default_rng(0).standard_normal((len(dofs), 6)))[0]
    r = O.refine_pairs(p.elem_dofs, p.elem_mat, el, dofs, d, V0, iters=1)
    assert np.all(np.abs(r.lam + r.lam_lo - 1.0) <= 1e-30)


def test_refine_condition_is_first_order_sensitivity():
    """Perturb every element entry by eps |a| with the sign that moves a chosen eigenvalue
    up: the eigenvalue moves by eps * sum |a_pq| |x_p x_q| (1 - lambda d_p d_q), which lies
    between eps (c1 - lambda c2) and eps (c1 + lambda c2) = eps * cond (c1, c2: the two terms
    of cond)."""
    p = P.small_problem(N=12, P=3, delta=2, contrast=1e4, seed=6)
    i = 4
    dofs, d, el = p.sub_dofs(i), p.sub_weights(i), p.sub_elems(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, el, dofs)
    g = O.gevp_definite(Ab, d[:, None] * Ab * d[None, :], 0.3, extra_vec=8)
    r = O.refine_pairs(p.elem_dofs, p.elem_mat, el, dofs, d, g.V, iters=3)
    eloc, emat = O.local_elements(p.elem_dofs, p.elem_mat, el, dofs)
    eps = 1e-9
    for j in (0, g.m):
        x = r.X[:, j]
        lam = r.lam[j]
        xe = np.where(eloc >= 0, x[np.maximum(eloc, 0)], 0.0)
        de = np.where(eloc >= 0, d[np.maximum(eloc, 0)], 0.0)
        w = xe[:, :, None] * xe[:, None, :] * (1.0 - lam * de[:, :, None] * de[:, None, :])
        pert = p.elem_mat.copy()
        pert[el] = emat * (1.0 + eps * np.sign(w) * np.sign(emat))
        r2 = O.refine_pairs(p.elem_dofs, pert, el, dofs, d, r.X, iters=2)
        dl = (r2.lam[j] - r.lam[j]) + (r2.lam_lo[j] - r.lam_lo[j])
        xa = np.abs(xe)
        c2 = float(np.sum(np.abs(emat) * (de * xa)[:, :, None] * (de * xa)[:, None, :]))
        c1 = r.cond[j] - lam * c2
        assert (c1 - lam * c2) * (1 - 1e-5) <= dl / eps <= r.cond[j] * (1 + 1e-5), (j, dl / eps, r.cond[j])
