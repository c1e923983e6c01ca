"""The blocked band solve of the eigensolver (per-block inverses of 64-row blocks on the
matrix cores, tuning variants 8 and 9) against the other band-solve variants on wide
bands, through the C ABI.  The oracle parity of every variant on small meshes is in
test_gpu_tuning.py; here the subdomains are large (up to 3969 dofs, 63 blocks with a
ragged last one) and the half-bandwidth reaches the blocked solve's limit of 64, where
the rolling window no longer applies, so the reference is the one-wavefront-per-column
solve (variant 3), which has no bandwidth limit and shares no code with the blocked
one.  Eigenvalues of selected pairs and of the pair that certifies the count must agree
to the eigenvalue tolerance, counts exactly, and PCG to within one iteration.  Two seeded
subdomains per mesh are also checked against references that share no code with the GPU:
the count against the Sylvester inertia of abar - eta b^1 (the oracle's Neumann matrix and
b^1) and the selected eigenvalues against LAPACK's generalized eigensolver on the same
pencil, within 1e-7 max(lambda, eta) (the dense FP64 reference is itself accurate only to
about u cond at these contrasts)."""
import numpy as np
import pytest
import scipy.linalg as sla

from msdd_inputs import problems as P
from oracle.msdd_oracle import gevp_rhs, neumann_matrix
from test_gpu_parity import _solve

pytestmark = pytest.mark.gpu


def _run(prob, eig_solve):
    from paper_2106_06404_amd import binding as B
    arrs = B.problem_arrays(prob, device="cuda:0")
    m = B.Msdd()
    m.set_tuning(eig_solve=eig_solve)
    m.setup(**arrs)
    st = m.stats()
    L = prob.n_levels - 1
    lam = [m.eigs(L, i, 1) for i in range(prob.n_sub)]
    counts = list(m.level_counts(L, prob.n_sub))
    it, rel, x = _solve(m, prob)
    m.close()
    return st, lam, counts, it, x


@pytest.mark.parametrize("N,Pside,delta,contrast,band,ref",
                         [(180, 3, 1, 1e4, 64, 3),   # half-bandwidth exactly 64
                          (160, 4, 4, 1e6, 50, 5)])  # many blocks, rolling window available
def test_blocked_matches_other_variants_on_wide_bands(N, Pside, delta, contrast, band, ref):
    prob = P.small_problem(N=N, P=Pside, delta=delta, contrast=contrast, seed=7)
    st_r, lam_r, cnt_r, it_r, x_r = _run(prob, ref)
    assert st_r["max_band"] == band
    for v in (8, 9):
        st, lam, cnt, it, x = _run(prob, v)
        if v == 8:
            _check_against_lapack(prob, lam, cnt)
        assert cnt == cnt_r
        for i in range(prob.n_sub):
            assert len(lam[i]) == len(lam_r[i])
            scale = np.maximum(np.abs(lam_r[i]), prob.eta)
            assert np.all(np.abs(lam[i] - lam_r[i]) <= 1e-10 * scale), (v, i, lam[i], lam_r[i])
        assert abs(it - it_r) <= 1
        assert np.linalg.norm(x - x_r) / np.linalg.norm(x_r) < 1e-8


def _check_against_lapack(prob, lam, cnt):
    rng = np.random.Generator(np.random.PCG64(31))
    checked = 0
    for i in rng.choice(prob.n_sub, size=2, replace=False):
        dofs, d = prob.sub_dofs(i), prob.sub_weights(i)
        Ab = neumann_matrix(prob.elem_dofs, prob.elem_mat, prob.sub_elems(i), dofs)
        Bm = gevp_rhs(1, Ab, d)
        mu = sla.eigh(Bm, Ab + Bm, eigvals_only=True)[::-1]
        lr = 1.0 / mu[mu > 1e-12] - 1.0
        if np.any(np.abs(lr - prob.eta) < 1e-6 * prob.eta):
            continue  # a tie at eta
        m_ref = int(np.sum(np.linalg.eigvalsh(Ab - prob.eta * Bm) < 0))
        assert cnt[i] == m_ref == int(np.sum(lr < prob.eta)), (i, cnt[i], m_ref)
        sel = np.asarray(lam[i][:m_ref])
        assert np.all(np.abs(sel - lr[:m_ref]) <= 1e-7 * np.maximum(lr[:m_ref], prob.eta)), i
        checked += 1
    assert checked >= 1
