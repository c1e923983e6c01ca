"""Pins of the oracle's hybrid preconditioner (restricted additive Schwarz within a level,
multiplicative over the levels; Sec. 2.1, the form used with GMRES in Sec. 5) and of its
GMRES.

  * GMRES iterates against the definition: x_k minimises ||b - A x|| over the Krylov space,
    computed here by least squares on an explicit Krylov basis; finite termination; one
    iteration with an exact preconditioner;
  * the hybrid apply ends with the exact level-0 correction, so the level-0 restriction of
    the new residual vanishes: P_0^T (r - A z) = 0 (a planted additive-over-levels variant
    fails it);
  * one subdomain covering Omega: the hybrid apply is A^{-1} (one GMRES iteration);
  * GMRES with the hybrid form stops on its least-squares residual; the recomputed residual
    lies within the FP64 rounding floor u || |A| |x| + |b| || of the tolerance and the
    solution agrees with a dense direct solve.
"""
import numpy as np
import pytest

from msdd_inputs import problems as P
from oracle import msdd_oracle as O


def test_gmres_iterates_minimise_the_residual():
    rng = np.random.default_rng(0)
    n = 14
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    for k in range(1, 7):
        res = O.gmres(A, b, lambda v: v.copy(), rtol=1e-30, restart=50, maxit=k)
        K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(k)], 1)
        c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
        xk = K @ c
        assert np.linalg.norm(res.x - xk) <= 1e-9 * np.linalg.norm(xk), k
        assert abs(res.resnorms[-1] - np.linalg.norm(b - A @ xk)) <= 1e-9 * np.linalg.norm(b)


def test_gmres_finite_termination_and_exact_preconditioner():
    rng = np.random.default_rng(1)
    n = 20
    A = np.eye(n) * 3 + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    res = O.gmres(A, b, lambda v: v.copy(), rtol=1e-10, restart=100, maxit=100)
    assert res.converged and res.iters <= n
    Ainv = np.linalg.inv(A)
    res = O.gmres(A, b, lambda v: Ainv @ v, rtol=1e-10, restart=10, maxit=10)
    assert res.converged and res.iters == 1


@pytest.mark.parametrize("levels", [2, 3, 4])
def test_hybrid_ends_with_exact_coarsest_correction(levels):
    groups = {2: (), 3: (2,), 4: (2, 2)}[levels]
    N = 32 if levels == 4 else 16
    Pn = 8 if levels == 4 else 4
    p = P.small_problem(N=N, P=Pn, delta=1, contrast=1e4, n_levels=levels, groups=groups, seed=5)
    o = O.Oracle(p)
    r = np.random.default_rng(levels).standard_normal(p.n)
    z = o.apply_hybrid(r)
    t = o.P[0].T @ (r - p.A @ z)
    assert np.linalg.norm(t) <= 1e-10 * np.linalg.norm(o.P[0].T @ r)


def test_planted_additive_over_levels_is_caught():
    p = P.small_problem(N=16, P=4, delta=1, contrast=1e4, n_levels=3, groups=(2,), seed=5)
    o = O.Oracle(p)
    r = np.random.default_rng(3).standard_normal(p.n)
    # additive over levels: every level corrects the original residual r
    A = p.A
    orig = o.A
    o.A = A * 0.0                  # r - A z = r at every level: no multiplicative update
    z_add = o.apply_hybrid(r)
    o.A = orig
    t = o.P[0].T @ (r - A @ z_add)
    assert np.linalg.norm(t) > 1e-3 * np.linalg.norm(o.P[0].T @ r)


def test_hybrid_one_subdomain_is_exact():
    p = P.small_problem(N=10, P=1, delta=0, contrast=1e3, seed=3)
    o = O.Oracle(p)
    r = np.random.default_rng(0).standard_normal(p.n)
    z = o.apply_hybrid(r)
    x = np.linalg.solve(p.A.toarray(), r)
    assert np.linalg.norm(z - x) <= 1e-10 * np.linalg.norm(x)
    res = o.solve_gmres()
    assert res.converged and res.iters == 1


@pytest.mark.parametrize("levels", [2, 3])
def test_hybrid_gmres_solution_vs_direct(levels):
    groups = (2,) if levels == 3 else ()
    p = P.small_problem(N=16, P=4, delta=2, contrast=1e6, n_levels=levels, groups=groups, seed=12)
    o = O.Oracle(p)
    res = o.solve_gmres(rtol=1e-8)
    assert res.converged
    A = p.A.toarray()
    xs = np.linalg.solve(A, p.b)
    # the stopping rule is on the least-squares residual; the recomputed one exceeds it by
    # at most a modest multiple of the rounding floor of b - A x
    floor = 2.0 ** -53 * np.linalg.norm(abs(p.A) @ np.abs(res.x) + np.abs(p.b))
    assert res.resnorms[-1] < 1e-8 * np.linalg.norm(p.b)
    assert np.linalg.norm(p.b - A @ res.x) < 1e-8 * np.linalg.norm(p.b) + 64 * floor
    e = res.x - xs
    assert np.sqrt(e @ A @ e) <= 1e-6 * np.sqrt(xs @ A @ xs)
