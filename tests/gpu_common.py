"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the CPU oracle).

Eigenvalue bar.  The reference of a finest-level eigenvalue is the oracle's eigenpair
refined in binary128 on the exactly summed element data (oracle.refine_pairs), with its
residual bound.  Its FP64 uncertainty U = u * cond (u = 2^-53) is what entrywise relative
perturbations of the element data at unit roundoff move it by, to first order.  The GPU
evaluates the pencil in FP64: assembly sums at most 4 (2D) / 8 (3D) element contributions
per entry (3 / 7 roundings), the products S y and b y at most 9 (2D) / 27 (3D) terms per
row, and the Gram matrices of the Rayleigh-Ritz step sum each entry over tiles of 16 rows,
then over the ceil(n / (16 S)) tiles of a row split, then over the S splits: a depth of
16 + ceil(n / (16 S)) + S, at most 102 for n <= 1369 rows and any S from 1 to 16.  So its
Ritz value at a converged vector is, to first order, the eigenvalue of a pencil perturbed
entrywise by at most (3 + 9 + 102) u = 114 u relative (2D; the 3D test meshes are far
smaller), and differs from the reference by at most that many times U.  The bar is 128 U,
or 1e-10 max(lambda, 1e-3 eta) where that is larger (the tolerance asked of the plain FP64
path), plus the reference's own bound.

The pair after the selected ones only certifies the count (lambda_{m+1} >= eta); the
GPU accepts it once it is accurate enough for that, so its value is checked for the side
of eta it lies on, not to the bar above.
"""
import numpy as np

from paper_2106_06404_amd import binding as B

U_FACTOR = 128.0
REL_FLOOR = 1e-10


def gpu_setup(prob, device="cuda:0", **opts):
    import torch
    if getattr(prob, "dirichlet_rule", "support") == "all":
        opts.setdefault("dirichlet_rule", 1)
    arrs = B.problem_arrays(prob, device=device)
    torch.cuda.synchronize()
    m = B.Msdd(**opts)
    m.setup(**arrs)
    return m, arrs


def sin_angle(U, V):
    """sin of the largest principal angle between span(U) and span(V) (accurate for small
    angles, unlike arccos of the smallest cosine)."""
    if U.shape[1] != V.shape[1]:
        return 1.0
    if U.shape[1] == 0:
        return 0.0
    Qu, _ = np.linalg.qr(U)
    Qv, _ = np.linalg.qr(V)
    return float(np.linalg.norm(Qv - Qu @ (Qu.T @ Qv), 2))


def energy_sin_angle(U, V, S):
    """sin of the largest principal angle between span(U) and span(V) in the inner product
    of the SPD matrix S (the local pencil's abar + b, the energy in which the coarse space
    enters the method)."""
    if U.shape[1] != V.shape[1]:
        return 1.0
    if U.shape[1] == 0:
        return 0.0

    def s_orth(W):
        G = W.T @ S @ W
        Lg = np.linalg.cholesky(0.5 * (G + G.T))
        return np.linalg.solve(Lg, W.T).T           # W Lg^{-T}: S-orthonormal columns

    Qu, Qv = s_orth(U), s_orth(V)
    Wr = Qv - Qu @ (Qu.T @ (S @ Qv))
    M = Wr.T @ S @ Wr
    return float(np.sqrt(max(np.linalg.eigvalsh(0.5 * (M + M.T)).max(), 0.0)))


def principal_angle_max(U, V):
    """Largest principal angle between span(U) and span(V) (columns)."""
    if U.shape[1] == 0 and V.shape[1] == 0:
        return 0.0
    if U.shape[1] != V.shape[1]:
        return np.pi / 2
    return float(np.arcsin(min(1.0, sin_angle(U, V))))


def eig_bar(lam_ref, unc, bound, eta):
    lam_ref = np.asarray(lam_ref)
    return (np.maximum(REL_FLOOR * np.maximum(np.abs(lam_ref), 1e-3 * eta),
                       U_FACTOR * np.asarray(unc)) + np.asarray(bound))


def check_selected_and_certifying(lg, m_i, lam_ref, unc, bound, eta, where="", fixed=False):
    """lg: GPU eigenvalues (m_i selected and at least the certifying one when computed);
    lam_ref/unc/bound: binary128 references of the first m_i + 1 or more pairs.  With a
    fixed count (no threshold) the next pair must lie at or above the selected ones."""
    lg = np.asarray(lg)
    sel = lg[:m_i]
    assert len(sel) == m_i, where
    bar = eig_bar(lam_ref[:m_i], unc[:m_i], bound[:m_i], eta)
    err = np.abs(sel - np.asarray(lam_ref[:m_i]))
    assert np.all(err <= bar), (where, sel, lam_ref[:m_i], err / bar)
    if not fixed:
        assert np.all(sel < eta), where
    if len(lg) > m_i and len(lam_ref) > m_i:
        if fixed:
            assert m_i == 0 or lg[m_i] >= lam_ref[m_i - 1], (where, lg[m_i], lam_ref[m_i - 1])
        else:
            assert lg[m_i] >= eta and lam_ref[m_i] >= eta, (where, lg[m_i], lam_ref[m_i])
    return float(np.max(err / bar)) if m_i else 0.0


def refined_fine_level(o, prob):
    """Binary128 references of every finest-level subdomain of an oracle built with
    fine_vectors > 0 (with the oracle's GEVP right-hand side)."""
    from oracle.msdd_oracle import overlap_elements, refine_pairs
    alpha = getattr(o, "geneo_rhs", 1)
    subs = [prob.sub_elems(j) for j in range(prob.n_sub)] if alpha == 2 else None
    out = []
    for i in range(prob.n_sub):
        out.append(refine_pairs(prob.elem_dofs, prob.elem_mat, prob.sub_elems(i), prob.sub_dofs(i),
                                prob.sub_weights(i), o.fine_vecs[i], iters=8, geneo_rhs=alpha,
                                overlap=overlap_elements(subs, i) if alpha == 2 else None))
    return out


def tie_subdomains(lams, eta, tol=1e-8):
    """Subdomains with an eigenvalue within tol*eta of eta (count is ill-posed there)."""
    out = set()
    for i, lam in enumerate(lams):
        if lam is not None and np.any(np.abs(np.asarray(lam) - eta) < tol * eta):
            out.add(i)
    return out
