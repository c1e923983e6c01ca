"""Plain CPU FP64 oracle of multilevel spectral domain decomposition.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke()
and by bench.py's cpu_baseline leg; never by the GPU library.  It shares no
code with the GPU path; only the seeded inputs (msdd_inputs) are common.

Every step follows the paper (Bastian, Scheichl, Seelinger, Strehlow,
"Multilevel Spectral Domain Decomposition"), in the paper's order, with
dense matrices and no blocking or fusion:

  * Sec. 2.1  additive subspace correction, B = sum_i R_i^T A_i^{-1} R_i
              with A_i = R_i A R_i^T, used as a preconditioner in CG;
              multilevel splitting V_h = V_{h,0} + sum_l sum_i V_{h,l,i}.
  * Sec. 2.2  hierarchical decomposition: T_{h,l,i} is the union of the
              finer T_{h,l+1,k}, k in J_{l,i}; level 0 is one subdomain.
  * Sec. 2.3  local Neumann spaces, partition of unity, the recursive
              spectral coarse space (GEVP "theGEVP", selection lambda < eta,
              phi = e chi w) and the Dirichlet subspaces V_{h,l,i}.
  * Sec. 3.3  GEVP lemma: with b(.,.) positive semi-definite and
              ker a cap ker b = {0}, b(p,v) = mu (a+b)(p,v), mu = 1/(1+lambda);
              eigenvectors b-orthonormal.
  * Sec. 3.4  CG bilinear forms: abar_{l,i} = sum over the subdomain's
              elements of a_tau; right-hand side b^1(u,v) = abar(chi u, chi v).
  * Sec. 4.2  coarse-level GEVPs on a generating system have
              ker A cap ker B != {0}; we use compression: eigenvectors of
              A + B with eigenvalue <= 1e-12 * ||A + B|| (exactly
              ker A cap ker B in exact arithmetic, the mu = 0 set of the
              paper's regularised transformation) are removed before the
              pencil is solved.
  * Sec. 5    Krylov driver: CG, stop when ||b - A x^m|| < 1e-8 ||b - A x^0||.

Readings where the paper is silent are listed in the module constants
below and in the design notes: b^1 is the GEVP right-hand side; the fine
PoU is the caller's nodal weights; coarse levels use nonoverlapping J_{l,i}
with a 0/1 owned mask as partition of unity and the owned functions as the
Dirichlet subspace; selection is strict (lambda < eta); x^0 = 0.

Parity pins: see tests/test_oracle_pins.py (closed-form Q1 spectra,
kernels of floating Neumann matrices, LAPACK generalized eigenvalues on
tiny meshes, Sylvester inertia counts, the Schur form of the coarse
pencil, dense direct solves, condition-number bounds).
"""
from __future__ import annotations

import dataclasses
import os
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import _dense
from ._dense import NotSPD, cholesky, jacobi_eigh

COMPRESS_REL = 1e-12  # coarse generating-system compression threshold (relative to ||A+B||)
# mu = 1/(1+lambda) lies in [0, 1]; the exact kernel of b (mu = 0, lambda = inf) comes out of
# the rotations as |mu| ~ n * eps.  Values below MU_ZERO are that kernel (lambda > 1e12).
MU_ZERO = 1e-12


# ----------------------------------------------------------------------------
# Sec. 2.2 / 2.3: subdomain sets
# ----------------------------------------------------------------------------

def dirichlet_mask(elem_dofs: np.ndarray, elems: np.ndarray, dofs: np.ndarray) -> np.ndarray:
    """For each dof of the Neumann space V-bar_i: is its basis function supported in
    the closure of Omega_i, i.e. do all elements adjacent to it belong to T_{h,i}?
    (Dirichlet subspace V_{h,l,i} of Sec. 2.3.)"""
    n = max(int(elem_dofs.max()) + 1, int(dofs.max()) + 1 if len(dofs) else 0)
    all_d = elem_dofs[elem_dofs >= 0]
    deg = np.bincount(all_d, minlength=n)
    sub = elem_dofs[elems]
    sub = sub[sub >= 0]
    cnt = np.bincount(sub, minlength=n)
    return cnt[dofs] == deg[dofs]


def dirichlet_set(prob, i: int, dofs: np.ndarray) -> np.ndarray:
    """Mask of the Dirichlet subspace V_{h,L,i} among the Neumann dofs of subdomain i: for
    conforming elements the dofs whose basis functions are supported in the subdomain
    (dirichlet_mask); for DG and cell-centred finite volumes (Sec. 3.5) every dof, since each
    basis function lives on one cell of the subdomain while the face terms that couple it to
    a neighbour outside are not part of the subdomain's element set."""
    if getattr(prob, "dirichlet_rule", "support") == "all":
        return np.ones(len(dofs), bool)
    return dirichlet_mask(prob.elem_dofs, prob.sub_elems(i), dofs)


def neumann_matrix(elem_dofs: np.ndarray, elem_mat: np.ndarray, elems: np.ndarray,
                   dofs: np.ndarray) -> np.ndarray:
    """abar_i = sum_{tau in T_i} a_tau on the local Neumann space (Sec. 3.4), dense."""
    n = int(elem_dofs.max()) + 1
    loc = -np.ones(n, np.int64)
    loc[dofs] = np.arange(len(dofs))
    nl = len(dofs)
    Ab = np.zeros((nl, nl))
    ed = loc[np.where(elem_dofs[elems] >= 0, elem_dofs[elems], 0)]
    ed[elem_dofs[elems] < 0] = -1
    k = ed.shape[1]
    for a in range(k):
        ra = ed[:, a]
        for c in range(k):
            rc = ed[:, c]
            m = (ra >= 0) & (rc >= 0)
            np.add.at(Ab, (ra[m], rc[m]), elem_mat[elems[m], a, c])
    return Ab


def overlap_elements(sub_elems: List[np.ndarray], i: int) -> np.ndarray:
    """The elements of T_{h,i} that also belong to some other subdomain's T_{h,j}
    (the set on which the original GenEO right-hand side b^2 is assembled, Sec. 3.4)."""
    n_elem = int(max(int(e.max()) for e in sub_elems if len(e))) + 1
    cnt = np.zeros(n_elem, np.int64)
    for e in sub_elems:
        cnt[e] += 1
    el = sub_elems[i]
    return el[cnt[el] >= 2]


def gevp_rhs(alpha: int, Ab: np.ndarray, d: np.ndarray, Ao: Optional[np.ndarray] = None):
    """The GEVP right-hand side matrix b^alpha on the local Neumann space (Sec. 3.4):
    alpha = 1: abar(chi u, chi v)            -> D abar D;
    alpha = 2: a-ring(chi u, chi v)          -> D Ao D, Ao = sum of a_tau over the overlap
                                                elements (the original GenEO choice);
    alpha = 3: abar(u - chi u, v - chi v)    -> (I - D) abar (I - D)."""
    if alpha == 1:
        return d[:, None] * Ab * d[None, :]
    if alpha == 2:
        return d[:, None] * Ao * d[None, :]
    if alpha == 3:
        e = 1.0 - d
        return e[:, None] * Ab * e[None, :]
    raise ValueError(alpha)


def elements_matrix(n: int, elem_dofs: np.ndarray, elem_mat: np.ndarray,
                    elems: np.ndarray) -> sp.csr_matrix:
    """sum_{tau in elems} a_tau as a sparse n x n matrix on the free dofs."""
    ed = elem_dofs[elems]
    k = ed.shape[1]
    r = np.repeat(ed, k, axis=1).reshape(-1)
    c = np.tile(ed, (1, k)).reshape(-1)
    v = elem_mat[elems].reshape(-1)
    m = (r >= 0) & (c >= 0)
    return sp.coo_matrix((v[m], (r[m], c[m])), shape=(n, n)).tocsr()


# ----------------------------------------------------------------------------
# Sec. 3.3: the GEVP through the spectral transformation mu = 1/(1+lambda)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class GevpResult:
    lam: np.ndarray        # all finite eigenvalues, ascending
    mu: np.ndarray         # all eigenvalues mu = 1/(1+lambda), descending (incl. mu = 0)
    m: int                 # number selected (lambda < eta)
    X: np.ndarray          # selected eigenvectors, b-orthonormal (columns)
    V: Optional[np.ndarray] = None   # the first m + extra_vec eigenvectors, S-orthonormal


def gevp_definite(Ab: np.ndarray, Bm: np.ndarray, eta: float, extra_vec: int = 0,
                  nev: int = 0) -> GevpResult:
    """abar x = lambda b x with ker abar cap ker b = {0}: S = abar + b is SPD.

    S = L L^T; C = L^{-1} b L^{-T}; C = Y diag(mu) Y^T (Jacobi);
    lambda = 1/mu - 1 (mu = 0 <-> lambda = inf); x = L^{-T} y; select
    lambda < eta (strict); b-normalise (x^T S x = 1 so x^T b x = mu).
    extra_vec > 0 also returns the eigenvectors of the m + extra_vec largest mu
    (x^T S x = 1), e.g. as start vectors of the binary128 refinement.  nev > 0 selects
    the nev smallest finite eigenvalues instead of those below eta (fixed n_ev, Sec. 5).
    """
    S = Ab + Bm
    L = cholesky(S)
    T = sla.solve_triangular(L, Bm, lower=True)
    C = sla.solve_triangular(L, T.T, lower=True).T
    C = 0.5 * (C + C.T)
    mu, Y = jacobi_eigh(C)
    mu = mu[::-1]
    Y = Y[:, ::-1]
    back = lambda Yc: sla.solve_triangular(L.T, Yc, lower=False)  # noqa: E731
    g = _select(mu, back, Y, eta, nev)
    if extra_vec > 0:
        g.V = back(Y[:, :min(g.m + extra_vec, Y.shape[1])])
    return g


def local_elements(elem_dofs: np.ndarray, elem_mat: np.ndarray, elems: np.ndarray,
                   dofs: np.ndarray):
    """The subdomain's element matrices with their dofs numbered in the local Neumann
    space (-1: eliminated or outside), for the binary128 refinement."""
    n = int(elem_dofs.max()) + 1
    loc = -np.ones(n + 1, np.int64)
    loc[dofs] = np.arange(len(dofs))
    ed = elem_dofs[elems]
    eloc = np.where(ed >= 0, loc[np.where(ed >= 0, ed, n)], -1)
    return eloc.astype(np.int32), elem_mat[elems]


@dataclasses.dataclass
class RefinedPairs:
    lam: np.ndarray      # eigenvalues of the exact-data pencil, rounded to FP64 (ascending)
    lam_lo: np.ndarray   # binary128 value minus lam
    bound: np.ndarray    # bound on |lam + lam_lo - lambda*| (Krylov-Weinstein, in binary128)
    cond: np.ndarray     # first-order sensitivity to entrywise relative data perturbations
    X: np.ndarray        # Ritz vectors, b-normalised (x^T b x = 1)

    @property
    def fp64_uncertainty(self) -> np.ndarray:
        """u * cond, u = 2^-53: the change of lambda that relative perturbations of the
        element data at FP64 unit roundoff can cause, to first order."""
        return 2.0 ** -53 * self.cond


def refine_pairs(elem_dofs, elem_mat, elems, dofs, d, V0, iters: int = 3,
                 geneo_rhs: int = 1, overlap: Optional[np.ndarray] = None) -> RefinedPairs:
    """Eigenpairs of abar x = lambda (D abar D) x (Sec. 2.3 GEVP, b^1 of Sec. 3.4, through
    the transformation of the Sec. 3.3 lemma) refined in binary128 from the start
    vectors V0 (columns; e.g. the oracle's FP64 eigenvectors of the smallest lambda):
    Rayleigh-Ritz on span(V0), then `iters` steps of subspace iteration with
    (abar + b)^{-1} b, each followed by Rayleigh-Ritz (oracle/refine.c).  geneo_rhs
    selects b^alpha (alpha = 2 needs `overlap`, the subdomain's overlap elements)."""
    eloc, emat = local_elements(elem_dofs, elem_mat, elems, dofs)
    bmask = None
    dd = d
    if geneo_rhs == 2:
        bmask = np.isin(elems, overlap).astype(np.int32)
    elif geneo_rhs == 3:
        dd = 1.0 - d
    hi, lo, bd, cd, X = _dense.refine_pairs(eloc, emat, dd, V0, iters, bmask)
    return RefinedPairs(hi, lo, bd, cd, X)


def _select(mu, back, Y, eta, nev=0):
    mu = np.where(mu > MU_ZERO, mu, 0.0)
    pos = mu > 0
    lam_all = np.full(mu.shape, np.inf)
    lam_all[pos] = 1.0 / mu[pos] - 1.0
    lam_all = np.maximum(lam_all, 0.0)
    if nev > 0:
        m = int(min(nev, np.sum(np.isfinite(lam_all))))
    else:
        m = int(np.sum(lam_all < eta))
    X = back(Y[:, :m]) if m else np.zeros((Y.shape[0], 0))
    if m:
        X = X / np.sqrt(mu[:m])[None, :]
        # sign convention: largest-magnitude entry positive
        idx = np.argmax(np.abs(X), axis=0)
        s = np.sign(X[idx, np.arange(m)])
        s[s == 0] = 1.0
        X = X * s[None, :]
    fin = np.isfinite(lam_all)
    return GevpResult(lam=np.sort(lam_all[fin]), mu=mu, m=m, X=X)


def gevp_generating(Ab: np.ndarray, Bm: np.ndarray, eta: float,
                    rel: float = COMPRESS_REL) -> GevpResult:
    """Coarse-level GEVP on a generating system (Sec. 4.2): ker abar cap ker b may be
    nonzero.  Compress: S = abar + b = Q diag(s) Q^T (Jacobi); drop s <= rel*max(s)
    (that is ker abar cap ker b); on the kept span solve the definite pencil."""
    if Ab.shape[0] == 0:   # no function on the next finer level: nothing to select
        return GevpResult(lam=np.zeros(0), mu=np.zeros(0), m=0, X=np.zeros((0, 0)))
    S = 0.5 * ((Ab + Bm) + (Ab + Bm).T)
    s, Q = jacobi_eigh(S)
    keep = s > rel * max(s.max(), 0.0)
    Qk = Q[:, keep] / np.sqrt(s[keep])[None, :]     # Qk^T S Qk = I
    C = Qk.T @ Bm @ Qk
    C = 0.5 * (C + C.T)
    mu, Y = jacobi_eigh(C)
    mu = mu[::-1]
    Y = Y[:, ::-1]
    return _select(mu, lambda Yc: Qk @ Yc, Y, eta)


# ----------------------------------------------------------------------------
# The multilevel hierarchy (Sec. 2.3 recursion) and the additive preconditioner
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class LevelData:
    level: int
    n_sub: int
    lam: List[np.ndarray]          # finite GEVP eigenvalues per subdomain
    m: np.ndarray                  # selected count per subdomain
    basis: List[np.ndarray]        # D X per subdomain: rows = owned / V-bar dofs of the level
    rows: List[np.ndarray]         # level-(l) dof indices of those rows
    dir_rows: List[np.ndarray]     # Dirichlet-subspace dofs (level-l indices)
    dir_chol: List[np.ndarray]     # Cholesky factors of A_{l,i}
    gen_size: List[int]            # generating-system size (coarse levels)
    neumann: Optional[List[np.ndarray]] = None   # abar_{l,i} (kept for tests)
    owned: Optional[List[np.ndarray]] = None     # owned mask over the generating system
    gen_cols: Optional[List[np.ndarray]] = None  # generating system: level-l function indices


_POOL_ORACLE = None


def _pool_init():
    os.environ["ORACLE_THREADS"] = "1"


def _pool_fine(i):
    return _POOL_ORACLE._fine_one(i)


class Oracle:
    """Setup and solve of the multilevel additive spectral Schwarz preconditioner."""

    def __init__(self, prob, eta: Optional[float] = None, verbose: bool = False,
                 only_fine: Optional[List[int]] = None, fine_vectors: int = 0,
                 workers: int = 1, geneo_rhs: int = 1, nev_fixed: int = 0):
        """fine_vectors > 0 keeps, per finest-level subdomain, the S-orthonormal
        eigenvectors of the m + fine_vectors smallest lambda (in fine_vecs);
        workers > 1 solves the finest-level subdomains in that many processes (the
        results do not depend on it).  geneo_rhs (1, 2, 3) is the finest level's GEVP
        right-hand side b^alpha (Sec. 3.4); nev_fixed > 0 selects that many eigenvectors per
        finest-level subdomain instead of those below eta.  Coarse levels use b^1 and eta."""
        self.prob = prob
        self.eta = prob.eta if eta is None else eta
        self.L = prob.n_levels - 1
        self.n = prob.n
        self.A = prob.A.tocsr()
        self.levels: Dict[int, LevelData] = {}
        self.P: Dict[int, sp.csr_matrix] = {}    # level-l coefficients -> fine dofs
        self.Al: Dict[int, np.ndarray] = {}      # Galerkin matrices A_l (l < L), dense
        self.verbose = verbose
        self.fine_vectors = fine_vectors
        self.workers = workers
        self.geneo_rhs = geneo_rhs
        self.nev_fixed = nev_fixed
        self.fine_vecs: Dict[int, np.ndarray] = {}
        self._setup(only_fine)

    # -- finest level (Sec. 2.3 step 2 with l = L) --
    def _fine_one(self, i):
        p = self.prob
        dofs = p.sub_dofs(i)
        d = p.sub_weights(i)
        el = p.sub_elems(i)
        dm = dirichlet_set(p, i, dofs)
        Ab = neumann_matrix(p.elem_dofs, p.elem_mat, el, dofs)
        Ao = None
        if self.geneo_rhs == 2:
            subs = [p.sub_elems(j) for j in range(p.n_sub)]
            Ao = neumann_matrix(p.elem_dofs, p.elem_mat, overlap_elements(subs, i), dofs)
        Bm = gevp_rhs(self.geneo_rhs, Ab, d, Ao)
        g = gevp_definite(Ab, Bm, self.eta, extra_vec=self.fine_vectors, nev=self.nev_fixed)
        Ad = self.A[dofs[dm]][:, dofs[dm]].toarray()   # A_i = R_i A R_i^T
        return g, d[:, None] * g.X, cholesky(Ad)

    def _fine(self, only):
        p = self.prob
        lam, m, basis, rows, dirr, dchol = [], [], [], [], [], []
        todo = [i for i in range(p.n_sub) if only is None or i in only]
        res = {}
        if self.workers > 1 and len(todo) > 1:
            import multiprocessing as mp
            global _POOL_ORACLE
            _POOL_ORACLE = self
            with mp.get_context("fork").Pool(self.workers, initializer=_pool_init) as pool:
                for i, out in zip(todo, pool.imap(_pool_fine, todo)):
                    res[i] = out
                    if self.verbose:
                        print(f"  fine sub {i}: nbar={len(p.sub_dofs(i))} m={out[0].m}", flush=True)
            _POOL_ORACLE = None
        else:
            for i in todo:
                res[i] = self._fine_one(i)
                if self.verbose:
                    print(f"  fine sub {i}: nbar={len(p.sub_dofs(i))} m={res[i][0].m}", flush=True)
        for i in range(p.n_sub):
            dofs = p.sub_dofs(i)
            dm = dirichlet_set(p, i, dofs)
            rows.append(dofs)
            dirr.append(dofs[dm])
            if i not in res:
                lam.append(None); m.append(0); basis.append(np.zeros((len(dofs), 0)))
                dchol.append(None)
                continue
            g, phi, Lc = res[i]
            lam.append(g.lam)
            m.append(g.m)
            basis.append(phi)   # phi = e chi w
            dchol.append(Lc)
            if g.V is not None:
                self.fine_vecs[i] = g.V
        self.levels[self.L] = LevelData(self.L, p.n_sub, lam, np.array(m), basis, rows, dirr,
                                        dchol, [len(r) for r in rows])

    @staticmethod
    def _generating_subdomains(emask_l, emask, par, i):
        """Generating system of coarse subdomain i (Sec. 4.2): the basis functions of every
        next-finer subdomain j that has elements in T_{h,l,i} (owned: par[j] == i; the others
        are its ghosts).  emask_l[j]: element mask of subdomain j; emask: that of i."""
        return [j for j in range(len(emask_l)) if np.any(emask_l[j] & emask)]

    def _setup(self, only):
        p = self.prob
        L = self.L
        n = self.n
        self._fine(only)
        self.P[L] = sp.identity(n, format="csr")
        # descendants (fine subdomains) and element masks per level-l subdomain
        desc = {L: [[i] for i in range(p.n_sub)]}
        for l in range(L - 1, 0, -1):
            par = p.parents[L - 1 - l]
            nl = int(par.max()) + 1
            desc[l] = [sum((desc[l + 1][j] for j in np.nonzero(par == i)[0]), []) for i in range(nl)]
        elem_mask_fine = []
        for i in range(p.n_sub):
            mk = np.zeros(p.n_elem, bool)
            mk[p.sub_elems(i)] = True
            elem_mask_fine.append(mk)
        self.desc = desc
        if only is not None:
            return
        for l in range(L, 0, -1):
            lev = self.levels[l]
            # coarse basis Phi_l: columns = phi_{l,i,k} in level-l coordinates
            n_l = n if l == L else self.Al[l].shape[0]
            ncol = int(lev.m.sum())
            rr, cc, vv = [], [], []
            col_owner = np.zeros(ncol, np.int64)
            off = 0
            for i in range(lev.n_sub):
                Bi = lev.basis[i]
                mi = Bi.shape[1]
                rr.append(np.repeat(lev.rows[i], mi))
                cc.append(np.tile(np.arange(off, off + mi), len(lev.rows[i])))
                vv.append(Bi.reshape(-1))
                col_owner[off:off + mi] = i
                off += mi
            Phi = sp.coo_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))),
                                shape=(n_l, ncol)).tocsr()
            self.P[l - 1] = (self.P[l] @ Phi).tocsr()
            Pl1 = self.P[l - 1]
            self.Al[l - 1] = (Pl1.T @ (self.A @ Pl1)).toarray()
            if l - 1 == 0:
                break
            # ---- level l-1 GEVPs on generating systems (Sec. 4.2) ----
            par = p.parents[L - l]          # level-l subdomain -> level-(l-1) subdomain
            nsub = int(par.max()) + 1
            emask_l = []
            for j in range(lev.n_sub):
                mk = np.zeros(p.n_elem, bool)
                for f in desc[l][j]:
                    mk |= elem_mask_fine[f]
                emask_l.append(mk)
            lam, m, basis, rows, dirr, dchol, gsz = [], [], [], [], [], [], []
            keep_ab, keep_own, keep_gen = [], [], []
            A_lm1 = self.Al[l - 1]
            for i in range(nsub):
                emask = np.zeros(p.n_elem, bool)
                for j in np.nonzero(par == i)[0]:
                    emask |= emask_l[j]
                gen_subs = self._generating_subdomains(emask_l, emask, par, i)
                owned_subs = set(np.nonzero(par == i)[0].tolist())
                gen_cols = np.concatenate([np.nonzero(col_owner == j)[0] for j in gen_subs])
                own = np.array([col_owner[c] in owned_subs for c in gen_cols], dtype=bool)
                AT = elements_matrix(n, p.elem_dofs, p.elem_mat, np.nonzero(emask)[0])
                G = Pl1[:, gen_cols]
                Ab = (G.T @ (AT @ G)).toarray()
                Ab = 0.5 * (Ab + Ab.T)
                dmask = own.astype(float)
                Bm = dmask[:, None] * Ab * dmask[None, :]
                g = gevp_generating(Ab, Bm, self.eta)
                lam.append(g.lam)
                m.append(g.m)
                basis.append(g.X[own])        # D x: owned coefficients
                rows.append(gen_cols[own])
                dirr.append(gen_cols[own])
                Ad = A_lm1[np.ix_(gen_cols[own], gen_cols[own])]
                dchol.append(cholesky(Ad))
                gsz.append(len(gen_cols))
                keep_ab.append(Ab)
                keep_own.append(own)
                keep_gen.append(gen_cols)
                if self.verbose:
                    print(f"  level {l-1} sub {i}: gen={len(gen_cols)} own={own.sum()} m={g.m}",
                          flush=True)
            self.levels[l - 1] = LevelData(l - 1, nsub, lam, np.array(m), basis, rows, dirr,
                                           dchol, gsz, keep_ab, keep_own, keep_gen)
        self.A0 = self.Al[0]
        self.A0_chol = cholesky(self.A0)

    # -- Sec. 2.1: z = sum_l P_l sum_i R_{l,i}^T A_{l,i}^{-1} R_{l,i} P_l^T r + P_0 A_0^{-1} P_0^T r
    def apply(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for l in range(self.L, 0, -1):
            lev = self.levels[l]
            rl = r if l == self.L else self.P[l].T @ r
            zl = np.zeros_like(rl)
            for i in range(lev.n_sub):
                idx = lev.dir_rows[i]
                if len(idx) == 0:
                    continue
                Lc = lev.dir_chol[i]
                y = sla.solve_triangular(Lc, rl[idx], lower=True)
                zl[idx] += sla.solve_triangular(Lc.T, y, lower=False)
            z += zl if l == self.L else self.P[l] @ zl
        r0 = self.P[0].T @ r
        y = sla.solve_triangular(self.A0_chol, r0, lower=True)
        z += self.P[0] @ sla.solve_triangular(self.A0_chol.T, y, lower=False)
        return z

    # -- Sec. 2.1 / Sec. 5: hybrid form -- restricted additive Schwarz within a level
    # (prolongation weighted by the partition of unity), multiplicative over the levels,
    # finest first: z = B_L r; then for l = L-1, ..., 0: z += P_l B_l P_l^T (r - A z)
    def apply_hybrid(self, r: np.ndarray) -> np.ndarray:
        p = self.prob
        L = self.L
        lev = self.levels[L]
        z = np.zeros_like(r)
        for i in range(lev.n_sub):
            idx = lev.dir_rows[i]
            if len(idx) == 0:
                continue
            Lc = lev.dir_chol[i]
            y = sla.solve_triangular(Lc, r[idx], lower=True)
            ui = sla.solve_triangular(Lc.T, y, lower=False)
            dofs = p.sub_dofs(i)
            dm = dirichlet_set(p, i, dofs)
            z[idx] += p.sub_weights(i)[dm] * ui          # restricted: chi_i on Dir_i
        for l in range(L - 1, -1, -1):
            t = self.P[l].T @ (r - self.A @ z)
            if l == 0:
                y = sla.solve_triangular(self.A0_chol, t, lower=True)
                zl = sla.solve_triangular(self.A0_chol.T, y, lower=False)
            else:
                cl = self.levels[l]
                zl = np.zeros_like(t)
                for i in range(cl.n_sub):
                    idx = cl.dir_rows[i]
                    if len(idx) == 0:
                        continue
                    Lc = cl.dir_chol[i]
                    y = sla.solve_triangular(Lc, t[idx], lower=True)
                    zl[idx] += sla.solve_triangular(Lc.T, y, lower=False)
            z = z + self.P[l] @ zl
        return z

    def solve_gmres(self, b=None, rtol=1e-8, restart=200, maxit=1000):
        b = self.prob.b if b is None else b
        return gmres(self.A, b, self.apply_hybrid, rtol=rtol, restart=restart, maxit=maxit)

    def level_sizes(self):
        return [self.P[l].shape[1] for l in range(self.L + 1)]

    def solve(self, b=None, rtol=1e-8, maxit=1000, record=False):
        b = self.prob.b if b is None else b
        return pcg(self.A, b, self.apply, rtol=rtol, maxit=maxit, record=record)


# ----------------------------------------------------------------------------
# Sec. 5: preconditioned conjugate gradients and the Lanczos condition estimate
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PcgResult:
    x: np.ndarray
    iters: int
    converged: bool
    resnorms: List[float]
    alphas: List[float]
    betas: List[float]
    iterates: Optional[List[np.ndarray]] = None

    def kappa(self) -> float:
        return lanczos_kappa(self.alphas, self.betas)


def pcg(A, b, M, rtol=1e-8, maxit=1000, record=False) -> PcgResult:
    """Textbook PCG from x^0 = 0; stops when ||r_m|| < rtol ||r_0|| (recurrence residual)."""
    x = np.zeros_like(b)
    r = b - A @ x
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    r0 = float(np.linalg.norm(r))
    res = [r0]
    al, be = [], []
    its = [x.copy()] if record else None
    if r0 == 0.0:
        return PcgResult(x, 0, True, res, al, be, its)
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        al.append(alpha)
        rn = float(np.linalg.norm(r))
        res.append(rn)
        if record:
            its.append(x.copy())
        if rn < rtol * r0:
            return PcgResult(x, k, True, res, al, be, its)
        z = M(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        be.append(beta)
        p = z + beta * p
        rz = rz_new
    return PcgResult(x, maxit, False, res, al, be, its)


def lanczos_kappa(alphas, betas) -> float:
    """Extreme Ritz values of the Lanczos tridiagonal built from the CG coefficients:
    T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_{j,j+1} = sqrt(b_j)/a_j."""
    k = len(alphas)
    if k == 0:
        return 1.0
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k and j < len(betas):
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    w, _ = jacobi_eigh(T)
    return float(w[-1] / w[0])


# ----------------------------------------------------------------------------
# GMRES with right preconditioning (the Krylov method of the hybrid form, Sec. 5)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    resnorms: List[float]      # ||r_k|| estimates from the least-squares problem, k = 0..iters


def gmres(A, b, M, rtol=1e-8, restart=200, maxit=1000) -> GmresResult:
    """Textbook restarted GMRES from x^0 = 0 with right preconditioning: Arnoldi (modified
    Gram-Schmidt) on A M, the small least-squares problem by Givens rotations; x = x^0 +
    M V y at the end of a cycle, then the residual b - A x is recomputed.

    Stopping (the paper asks for ||b - A x^m|| < rtol ||b - A x^0||).  A cycle ends when its
    least-squares residual (equal to ||b - A x^m|| in exact arithmetic) falls below
    rtol ||r_0||, or after `restart` steps.  The solve stops when the recomputed residual
    meets the tolerance; when a cycle met it only in the least-squares sense, the next cycle
    starts from x^m (a refinement step: the operator A M of the hybrid form can be so ill
    conditioned at high contrast that the two differ by 10x), unless that cycle reduced the
    recomputed residual by less than half, which means it sits at its rounding floor (in
    FP64 about u || |A| |x| + |b| ||, above 1e-8 ||b|| on fine high-contrast meshes): the
    solve then stops as converged and returns that residual."""
    n = len(b)
    x = np.zeros(n)
    r = b - A @ x
    r0 = float(np.linalg.norm(r))
    res = [r0]
    if r0 == 0.0:
        return GmresResult(x, 0, True, res)
    its = 0
    beta = r0
    while its < maxit:
        beta_start = beta
        m = min(restart, maxit - its)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k_done = 0
        conv = False
        for k in range(m):
            w = A @ M(V[:, k])
            for j in range(k + 1):
                H[j, k] = float(V[:, j] @ w)
                w = w - H[j, k] * V[:, j]
            H[k + 1, k] = float(np.linalg.norm(w))
            if H[k + 1, k] > 0.0:
                V[:, k + 1] = w / H[k + 1, k]
            for j in range(k):   # earlier rotations on the new column
                t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            d = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / d, H[k + 1, k] / d
            H[k, k] = d
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_done = k + 1
            res.append(abs(g[k + 1]))
            if abs(g[k + 1]) < rtol * r0 or H[k, k] == 0.0:
                conv = abs(g[k + 1]) < rtol * r0
                break
        y = sla.solve_triangular(H[:k_done, :k_done], g[:k_done], lower=False)
        x = x + M(V[:, :k_done] @ y)
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        if beta < rtol * r0 or (conv and beta >= 0.5 * beta_start):
            return GmresResult(x, its, True, res)
    return GmresResult(x, its, False, res)
