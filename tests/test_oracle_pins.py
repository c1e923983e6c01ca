"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks one part of the oracle (or of the shared input data) against
something other than the oracle itself: closed-form spectra, kernels of
floating Neumann matrices, LAPACK on tiny meshes, Sylvester inertia, the
Schur form of the coarse pencil, dense direct solves and the condition-number
bound of the multilevel theorem.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from msdd_inputs import problems as P
from oracle import msdd_oracle as O
from oracle._dense import cholesky, jacobi_eigh, NotSPD


# ---------------------------------------------------------------- PIN-1
@pytest.mark.parametrize("dim,N", [(2, 8), (2, 11), (3, 5)])
def test_pin1_q1_closed_form_spectrum(dim, N):
    """Unit-coefficient Q1 stiffness with zero Dirichlet data is the tensor sum of 1D
    stiffness K1 and mass M1 (2-point Gauss is exact); K1, M1 share sine eigenvectors,
    kappa_j = (4/h) sin^2(j pi h/2), mu_j = (h/3)(2 + cos j pi h)."""
    p = P.small_problem(N=N, P=1, delta=0, dim=dim)
    h = 1.0 / N
    j = np.arange(1, N)
    kap = 4.0 / h * np.sin(j * np.pi * h / 2) ** 2
    mu = h / 3.0 * (2.0 + np.cos(j * np.pi * h))
    if dim == 2:
        ref = (kap[:, None] * mu[None, :] + mu[:, None] * kap[None, :]).ravel()
    else:
        ref = (kap[:, None, None] * mu[None, :, None] * mu[None, None, :]
               + mu[:, None, None] * kap[None, :, None] * mu[None, None, :]
               + mu[:, None, None] * mu[None, :, None] * kap[None, None, :]).ravel()
    ref = np.sort(ref)
    w, _ = jacobi_eigh(p.A.toarray())
    assert np.max(np.abs(w - ref) / ref) < 1e-12


# ---------------------------------------------------------------- PIN-2
def test_pin2_floating_neumann_kernel_scalar():
    p = P.small_problem(N=12, P=3, delta=1, contrast=1e3, seed=3)
    i = 4  # centre box: does not touch the Dirichlet boundary
    dofs = p.sub_dofs(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, p.sub_elems(i), dofs)
    assert np.max(np.abs(Ab @ np.ones(len(dofs)))) < 1e-9 * np.abs(Ab).max()
    w, _ = jacobi_eigh(Ab)
    assert np.sum(w < 1e-10 * w.max()) == 1
    # a boundary box is nonsingular
    Ab0 = O.neumann_matrix(p.elem_dofs, p.elem_mat, p.sub_elems(0), p.sub_dofs(0))
    w0, _ = jacobi_eigh(Ab0)
    assert w0.min() > 1e-8 * w0.max()


def test_pin2_floating_neumann_kernel_elasticity():
    p = P.small_elasticity(N=6, P=3, delta=1)
    coords, comp = P.free_dof_coords(p)
    # a box not touching x = 0 floats: six rigid-body modes
    i = 1 + 3 * 1 + 9 * 1
    dofs = p.sub_dofs(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, p.sub_elems(i), dofs)
    x = coords[dofs]
    c = comp[dofs]
    rbm = []
    for t in range(3):
        rbm.append((c == t).astype(float))
    for (a, b) in [(0, 1), (1, 2), (0, 2)]:
        v = np.zeros(len(dofs))
        v[c == a] = -x[c == a, b]
        v[c == b] = x[c == b, a]
        rbm.append(v)
    R = np.stack(rbm, 1)
    assert np.max(np.abs(Ab @ R)) < 1e-10 * np.abs(Ab).max()
    w, _ = jacobi_eigh(Ab)
    assert np.sum(w < 1e-10 * w.max()) == 6


def test_pin2_elements_sum_to_global_matrix():
    p = P.small_problem(N=9, P=3, delta=1, contrast=1e6, seed=1)
    Asum = O.elements_matrix(p.n, p.elem_dofs, p.elem_mat, np.arange(p.n_elem))
    assert abs(Asum - p.A).max() <= 1e-12 * abs(p.A).max()


# ---------------------------------------------------------------- PIN-3
@pytest.mark.parametrize("dim,N,Pn,delta", [(2, 12, 3, 1), (2, 16, 4, 2), (3, 6, 2, 1)])
def test_pin3_partition_of_unity(dim, N, Pn, delta):
    p = P.small_problem(N=N, P=Pn, delta=delta, dim=dim)
    s = np.zeros(p.n)
    for i in range(p.n_sub):
        dofs = p.sub_dofs(i)
        w = p.sub_weights(i)
        dm = O.dirichlet_mask(p.elem_dofs, p.sub_elems(i), dofs)
        assert np.all(w[~dm] == 0.0)  # chi v vanishes on the interior subdomain boundary
        assert np.all(w[dm] > 0.0)
        s[dofs] += w
    assert np.max(np.abs(s - 1.0)) < 1e-15


# ---------------------------------------------------------------- PIN-4
@pytest.mark.parametrize("n", [1, 7, 60, 200])
def test_pin4_cholesky_and_solves(n):
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    L = cholesky(A)
    assert np.allclose(np.triu(L, 1), 0.0)
    u = 2.0 ** -53
    assert np.linalg.norm(L @ L.T - A) <= 10 * n * u * np.linalg.norm(A)
    b = rng.standard_normal(n)
    x = sla.solve_triangular(L.T, sla.solve_triangular(L, b, lower=True), lower=False)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    with pytest.raises(NotSPD):
        cholesky(-A)


# ---------------------------------------------------------------- PIN-5 / PIN-7 / PIN-8
def _local(p, i):
    dofs = p.sub_dofs(i)
    d = p.sub_weights(i)
    Ab = O.neumann_matrix(p.elem_dofs, p.elem_mat, p.sub_elems(i), dofs)
    return Ab, d[:, None] * Ab * d[None, :], d


@pytest.mark.parametrize("contrast", [1.0, 1e4])
def test_pin5_spectrum_structure(contrast):
    p = P.small_problem(N=12, P=3, delta=1, contrast=contrast, seed=5)
    for i in range(p.n_sub):
        Ab, Bm, d = _local(p, i)
        g = O.gevp_definite(Ab, Bm, 0.1)
        w, _ = jacobi_eigh(Ab)
        kerA = int(np.sum(w < 1e-10 * w.max()))
        assert g.m >= kerA
        assert len(g.lam) == len(d) - int(np.sum(d == 0))   # ker b = span{e_p : d_p = 0}
        assert np.all(g.lam >= 0.0)


def _mu_reference_mp(Ab, Bm, dps=40):
    """mu of b x = mu (abar + b) x in 40-digit arithmetic (mpmath): Cholesky, explicit
    inverse, symmetric eigenvalues.  Used where double precision itself is limited by the
    coefficient contrast."""
    import mpmath as mp
    mp.mp.dps = dps
    S = mp.matrix((Ab + Bm).tolist())
    B = mp.matrix(Bm.tolist())
    Li = mp.inverse(mp.cholesky(S))
    E = mp.eigsy(Li * B * Li.T, eigvals_only=True)
    return np.array(sorted([float(x) for x in E], reverse=True))


@pytest.mark.parametrize("contrast,seed,tol", [(1.0, 0, 1e-12), (1e6, 1, 1e-10), (1e3, 2, 1e-11)])
def test_pin7_brute_force_lapack(contrast, seed, tol):
    """mu against LAPACK's generalized symmetric eigensolver (contrast 1) and against a
    40-digit reference (high contrast, where double precision is only good to ~1e-11)."""
    p = P.small_problem(N=10, P=2, delta=2, contrast=contrast, seed=seed)
    rng = np.random.default_rng(seed)
    for i in range(p.n_sub):
        Ab, Bm, d = _local(p, i)
        eta = 0.3
        g = O.gevp_definite(Ab, Bm, eta)
        if contrast == 1.0:
            mu_ref = sla.eigh(Bm, Ab + Bm, eigvals_only=True)[::-1]
        elif i == 1:
            mu_ref = _mu_reference_mp(Ab, Bm)
        else:
            mu_ref = None
        if mu_ref is not None:
            mu_ref = np.where(mu_ref > O.MU_ZERO, mu_ref, 0.0)
            assert np.max(np.abs(mu_ref - g.mu)) < tol
        X = g.X
        if g.m:
            assert np.allclose(X.T @ Bm @ X, np.eye(g.m), atol=1e-10)
            G = X.T @ Ab @ X
            assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-9 * max(1, abs(G).max()))
        # Pi_m stability (Sec. 3.3 lemma): |Pi v|_a <= |v|_a, |v - Pi v|_a <= |v|_a,
        # |v - Pi v|_b^2 <= |v - Pi v|_a^2 / lambda_{m+1}  for m >= dim ker a
        lam_next = g.lam[g.m] if g.m < len(g.lam) else np.inf
        for _ in range(5):
            v = rng.standard_normal(len(d))
            Pv = X @ (X.T @ (Bm @ v)) if g.m else np.zeros_like(v)
            na = v @ Ab @ v
            assert Pv @ Ab @ Pv <= na * (1 + 1e-9) + 1e-12
            e = v - Pv
            assert e @ Ab @ e <= na * (1 + 1e-9) + 1e-12
            if np.isfinite(lam_next):
                assert e @ Bm @ e <= (e @ Ab @ e) / lam_next * (1 + 1e-8) + 1e-12


@pytest.mark.parametrize("eta", [0.05, 0.2, 0.5])
def test_pin8_inertia_count(eta):
    """Sylvester: #{lambda < eta} = #negative eigenvalues of abar - eta b."""
    p = P.small_problem(N=12, P=3, delta=1, contrast=1e4, seed=7, kind="channels")
    for i in range(p.n_sub):
        Ab, Bm, d = _local(p, i)
        g = O.gevp_definite(Ab, Bm, eta)
        w, _ = jacobi_eigh(Ab - eta * Bm)
        scale = np.abs(w).max()
        assert np.all(np.abs(w) > 1e-10 * scale)   # eta not (numerically) an eigenvalue
        assert g.m == int(np.sum(w < 0))


# ---------------------------------------------------------------- PIN-6
def test_pin6_single_subdomain_all_lambda_one():
    """One subdomain covering Omega with chi = 1: b^1 = abar, so every lambda equals 1."""
    p = P.small_problem(N=9, P=1, delta=0, contrast=1e3, seed=2)
    Ab, Bm, d = _local(p, 0)
    assert np.all(d == 1.0)
    g = O.gevp_definite(Ab, Bm, 2.0)
    assert np.max(np.abs(g.lam - 1.0)) < 1e-12
    assert g.m == len(d)


# ---------------------------------------------------------------- PIN-9
@pytest.mark.parametrize("contrast,tol", [(1.0, 1e-9), (1e4, 2e-6)])
def test_pin9_coarse_pencil_schur_form(contrast, tol):
    """With a 0/1 owned mask the generating-system pencil reduces to the Schur pencil
    (A_oo - A_og A_gg^+ A_go) y = lambda A_oo y on the owned block; all lambda in [0,1].

    The restricted ghost functions are nearly dependent (the spectrum of abar + b runs
    continuously down to round-off), so in double precision the coarse eigenvalues are
    determined only to ~1e-7 at high contrast; the two independent reductions
    (compression of abar + b, pseudo-inverse of the ghost block) agree to that level."""
    p = P.small_problem(N=16, P=4, delta=1, contrast=contrast, n_levels=3, groups=(2,), seed=11)
    o = O.Oracle(p, eta=0.4)
    lev = o.levels[1]
    for i in range(lev.n_sub):
        Ab = lev.neumann[i]
        own = lev.owned[i]
        Aoo = Ab[np.ix_(own, own)]
        Aog = Ab[np.ix_(own, ~own)]
        Agg = Ab[np.ix_(~own, ~own)]
        Sc = Aoo - Aog @ sla.pinvh(Agg, rtol=1e-12) @ Aog.T
        lam = sla.eigh(0.5 * (Sc + Sc.T), Aoo, eigvals_only=True)
        assert lam.min() > -1e-8 and lam.max() < 1 + 1e-8
        assert np.max(np.abs(np.sort(lam) - lev.lam[i])) < tol
        assert lev.m[i] == int(np.sum(lam < 0.4))
        # owned block of the generating-system Neumann matrix = owned block of A_l
        A1 = o.Al[1]
        rows = lev.rows[i]
        assert np.allclose(Aoo, A1[np.ix_(rows, rows)], rtol=1e-12, atol=1e-12 * abs(A1).max())


# ---------------------------------------------------------------- PIN-10 / 11 / 12
def _kappa_bound(dim, L, eta):
    k0 = 4 if dim == 2 else 8
    a0 = b0 = k0
    C1 = 1.0 / eta
    C = 2 * (1 + a0 * b0 * C1)
    return C ** L * (1 + b0 * C1 / (C - 1)) * (1 + k0 * L)


@pytest.mark.parametrize("levels", [2, 3])
def test_pin10_kappa_within_theorem_bound(levels):
    groups = (2,) if levels == 3 else ()
    p = P.small_problem(N=16, P=4, delta=1, contrast=1e5, n_levels=levels, groups=groups, seed=4)
    o = O.Oracle(p)
    res = o.solve(rtol=1e-12)
    kap = res.kappa()
    assert 1.0 <= kap <= _kappa_bound(2, levels - 1, p.eta)


def test_pin11_contrast_robustness_and_negative_control():
    """Spectral coarse space: the condition number stays under the contrast-independent
    bound of the multilevel theorem for contrasts 1..1e6.  Negative control: a
    kernel-only coarse space (eta -> 0+) degrades by orders of magnitude."""
    kap, kap0 = [], []
    for c in [1.0, 1e2, 1e4, 1e6]:
        p = P.small_problem(N=24, P=4, delta=1, contrast=c, seed=9, kind="random")
        kap.append(O.Oracle(p, eta=0.1).solve(rtol=1e-12).kappa())
        kap0.append(O.Oracle(p, eta=1e-9).solve(rtol=1e-12, maxit=2000).kappa())
    assert max(kap) <= _kappa_bound(2, 1, 0.1)
    assert max(kap) / min(kap) < 10.0
    assert kap0[-1] > 1e3 * kap0[0]
    assert kap[-1] < 1e-3 * kap0[-1]


@pytest.mark.parametrize("levels,contrast", [(2, 1.0), (2, 1e6), (3, 1e4)])
def test_pin12_solution_vs_dense_direct(levels, contrast):
    groups = (2,) if levels == 3 else ()
    p = P.small_problem(N=16, P=4, delta=2, contrast=contrast, n_levels=levels, groups=groups,
                        seed=12)
    o = O.Oracle(p)
    res = o.solve(rtol=1e-8)
    assert res.converged
    A = p.A.toarray()
    xs = np.linalg.solve(A, p.b)
    e = res.x - xs
    errA = np.sqrt(e @ A @ e) / np.sqrt(xs @ A @ xs)
    assert errA <= np.sqrt(res.kappa()) * 1e-8 * 1.5
    assert np.linalg.norm(p.b - A @ res.x) < 1e-8 * np.linalg.norm(p.b) * 1.01 + 1e-14


def test_pin12_one_subdomain_one_iteration():
    p = P.small_problem(N=10, P=1, delta=0, contrast=1e3, seed=3)
    o = O.Oracle(p)
    assert o.level_sizes()[0] == 0   # all lambda = 1 >= eta: empty coarse space
    res = o.solve()
    assert res.iters == 1


def test_preconditioner_symmetric_positive():
    """The additive preconditioner is symmetric positive definite (so CG applies)."""
    p = P.small_problem(N=12, P=3, delta=1, contrast=1e4, n_levels=3, groups=(2,), seed=8)
    o = O.Oracle(p)
    n = p.n
    M = np.stack([o.apply(e) for e in np.eye(n)], 1)
    assert np.allclose(M, M.T, atol=1e-12 * abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


# ---------------------------------------------------------------- planted mistakes
def test_planted_mistake_dropping_pou_is_caught():
    """A GEVP that forgets chi (b = abar instead of D abar D) gives lambda = 1 everywhere
    for every subdomain; PIN-5's count of finite eigenvalues catches it."""
    p = P.small_problem(N=12, P=3, delta=1, contrast=1e3, seed=5)
    Ab, Bm, d = _local(p, 0)   # boundary box: abar nonsingular, so the wrong pencil is definite
    wrong = O.gevp_definite(Ab, Ab, 0.1)
    assert len(wrong.lam) != len(d) - int(np.sum(d == 0))


def test_planted_mistake_transposed_solve_is_caught():
    """x = L^{-1} y instead of L^{-T} y breaks b-orthonormality / a-orthogonality (PIN-7)."""
    p = P.small_problem(N=10, P=2, delta=2, contrast=1e3, seed=2)
    Ab, Bm, d = _local(p, 1)
    S = Ab + Bm
    L = cholesky(S)
    C = sla.solve_triangular(L, sla.solve_triangular(L, Bm, lower=True).T, lower=True).T
    mu, Y = jacobi_eigh(0.5 * (C + C.T))
    Y = Y[:, ::-1][:, :4]
    Xw = sla.solve_triangular(L, Y, lower=True)
    G = Xw.T @ Ab @ Xw
    assert np.abs(G - np.diag(np.diag(G))).max() > 1e-6 * np.abs(G).max()
