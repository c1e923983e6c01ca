"""Seeded synthetic problem generators (inputs only).

This module builds the *inputs* of the multilevel spectral domain
decomposition method: a structured mesh of the unit square/cube, a
coefficient field, conforming Q1 element matrices (scalar diffusion and
trilinear linear elasticity), the assembled stiffness matrix on the free
dofs (Dirichlet dofs eliminated), the load vector, an overlapping box
partition of the elements, the partition-of-unity weights and the
parent maps of the coarse levels.

It holds none of the method's arithmetic (no local matrices, no
eigenproblems, no coarse spaces, no Krylov solver).  Both the CPU oracle
and the GPU library consume exactly these arrays.

Paper sections followed:
  * Sec. 3.4 (continuous Galerkin): a_tau(u,v) = int_tau (K grad u).grad v,
    l(v) = int f v; element-wise stiffness matrices.
  * Sec. 2.2 (hierarchical domain decomposition): finest level = element
    partition plus delta layers of overlap; coarser levels group subdomain
    indices (nonoverlapping index sets J_{l,i}); level 0 is one subdomain.
  * Sec. 2.3 (partition of unity definition): chi_{l,i} vanishes on the
    interior subdomain boundary and the weights sum to one.  The concrete
    construction (nodal multiplicity weights) is not given by the paper;
    we use d_i(p) = [p in Dir_i] / #{j : p in Dir_j}.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional, Sequence

import numpy as np
import scipy.fft
import scipy.sparse as sp

# ----------------------------------------------------------------------------
# Reference Q1 element: 2 Gauss points per direction on [0,1]^d.
# Node a of the reference cell has coordinates bit_d(a) in {0,1}^d
# (x fastest), i.e. lexicographic local numbering.
# ----------------------------------------------------------------------------


def _gauss2():
    g = 1.0 / np.sqrt(3.0)
    return np.array([(1 - g) / 2, (1 + g) / 2]), np.array([0.5, 0.5])


def q1_shape(dim: int, x: np.ndarray):
    """Values [2^dim] and reference gradients [2^dim, dim] of Q1 at x."""
    nn = 2 ** dim
    val = np.ones(nn)
    grad = np.ones((nn, dim))
    for a in range(nn):
        for d in range(dim):
            bit = (a >> d) & 1
            f = x[d] if bit else 1.0 - x[d]
            df = 1.0 if bit else -1.0
            val[a] *= f
            for e in range(dim):
                grad[a, e] *= df if e == d else f
    return val, grad


def _quad_points(dim: int):
    p, w = _gauss2()
    for idx in itertools.product(range(2), repeat=dim):
        yield np.array([p[i] for i in idx]), float(np.prod([w[i] for i in idx]))


def q1_laplace_element(dim: int, h: float) -> np.ndarray:
    """Stiffness of -div(grad u) on an axis-parallel cube of side h (unit coefficient)."""
    nn = 2 ** dim
    K = np.zeros((nn, nn))
    for x, w in _quad_points(dim):
        _, g = q1_shape(dim, x)
        g = g / h
        K += w * h ** dim * (g @ g.T)
    return K


def q1_load_element(dim: int, h: float, ncomp: int = 1, f: Sequence[float] = (1.0,)) -> np.ndarray:
    """Element load vector int f phi_a for a constant body force f (length ncomp)."""
    nn = 2 ** dim
    out = np.zeros(nn * ncomp)
    for x, w in _quad_points(dim):
        v, _ = q1_shape(dim, x)
        for a in range(nn):
            for c in range(ncomp):
                out[a * ncomp + c] += w * h ** dim * v[a] * f[c]
    return out


def isotropic_voigt(E: float, nu: float) -> np.ndarray:
    """6x6 isotropic elasticity matrix, engineering shear strains, order xx,yy,zz,yz,xz,xy."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2 * mu
    C[np.arange(3, 6), np.arange(3, 6)] = mu
    return C


def fibre_voigt(E_f: float, nu: float, axis: Sequence[float]) -> np.ndarray:
    """Isotropic unit-modulus matrix plus (E_f - 1) a(x)a(x)a(x)a along the fibre axis a.

    sigma = C eps with the added term (E_f-1) a (a^T eps a); in Voigt form with
    engineering shears this is (E_f-1) v v^T with v = (a1^2,a2^2,a3^2,a2a3,a1a3,a1a2).
    """
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    v = np.array([a[0] ** 2, a[1] ** 2, a[2] ** 2, a[1] * a[2], a[0] * a[2], a[0] * a[1]])
    return isotropic_voigt(1.0, nu) + (E_f - 1.0) * np.outer(v, v)


def q1_elasticity_element(h: float, C: np.ndarray) -> np.ndarray:
    """24x24 trilinear hexahedral elasticity stiffness on a cube of side h.

    Dof ordering: 3*a + c (node a, component c).
    """
    K = np.zeros((24, 24))
    for x, w in _quad_points(3):
        _, g = q1_shape(3, x)
        g = g / h
        B = np.zeros((6, 24))
        for a in range(8):
            gx, gy, gz = g[a]
            B[0, 3 * a + 0] = gx
            B[1, 3 * a + 1] = gy
            B[2, 3 * a + 2] = gz
            B[3, 3 * a + 1] = gz
            B[3, 3 * a + 2] = gy
            B[4, 3 * a + 0] = gz
            B[4, 3 * a + 2] = gx
            B[5, 3 * a + 0] = gy
            B[5, 3 * a + 1] = gx
        K += w * h ** 3 * (B.T @ C @ B)
    return K


# ----------------------------------------------------------------------------
# Structured mesh of the unit cube [0,1]^dim with N^dim elements.
# ----------------------------------------------------------------------------


def element_nodes(dim: int, N: int) -> np.ndarray:
    """[N^dim, 2^dim] global node ids (lexicographic, x fastest)."""
    M = N + 1
    ev = np.stack(np.meshgrid(*([np.arange(N)] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1]
    # ev[e] = (ex, ey[, ez]) with element id e = ex + N*ey (+ N^2 ez)
    nodes = np.zeros((ev.shape[0], 2 ** dim), dtype=np.int64)
    for a in range(2 ** dim):
        off = np.array([(a >> d) & 1 for d in range(dim)])
        c = ev + off
        gid = np.zeros(ev.shape[0], dtype=np.int64)
        for d in reversed(range(dim)):
            gid = gid * M + c[:, d]
        nodes[:, a] = gid
    return nodes


def element_coords(dim: int, N: int) -> np.ndarray:
    """[N^dim, dim] integer element coordinates (ex, ey[, ez]) for element id e."""
    return np.stack(np.meshgrid(*([np.arange(N)] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1]


def boundary_nodes(dim: int, N: int, which: str = "all") -> np.ndarray:
    M = N + 1
    c = np.stack(np.meshgrid(*([np.arange(M)] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1]
    if which == "all":
        mask = np.any((c == 0) | (c == N), axis=1)
    elif which == "x0":
        mask = c[:, 0] == 0
    elif which == "x01":
        mask = (c[:, 0] == 0) | (c[:, 0] == N)
    else:
        raise ValueError(which)
    return mask


@dataclasses.dataclass
class Problem:
    """All arrays a caller hands to the solver (and to the oracle)."""
    name: str
    dim: int
    ncomp: int
    N: int
    n: int                      # free dofs
    elem_dofs: np.ndarray       # int32 [n_elem, k], -1 = eliminated Dirichlet dof
    elem_mat: np.ndarray        # float64 [n_elem, k, k]
    A: sp.csr_matrix            # free-dof stiffness, float64
    b: np.ndarray               # load vector on free dofs
    sub_elem_ptr: np.ndarray    # int64 [P_L+1]
    sub_elem: np.ndarray        # int32 element ids of T_{h,L,i}
    sub_dof_ptr: np.ndarray     # int64 [P_L+1]
    sub_dof: np.ndarray         # int32 sorted free dofs of T_{h,L,i} (Neumann space)
    sub_pou: np.ndarray         # float64 partition-of-unity weight per (i, dof)
    n_levels: int               # L+1
    parents: List[np.ndarray]   # parents[0]: level L -> L-1, parents[1]: L-1 -> L-2, ...
    eta: float
    coeff: Optional[np.ndarray] = None  # per-element scalar coefficient (diffusion) or material id
    box_shape: Optional[tuple] = None   # subdomains per dimension on the finest level
    # Dirichlet subspace of a finest subdomain: "support" = the dofs all of whose elements lie
    # in the subdomain (conforming elements); "all" = every dof of the subdomain (DG and
    # finite volumes, whose basis functions live on one cell while face terms couple cells)
    dirichlet_rule: str = "support"

    @property
    def n_elem(self):
        return self.elem_dofs.shape[0]

    @property
    def k(self):
        return self.elem_dofs.shape[1]

    @property
    def n_sub(self):
        return len(self.sub_elem_ptr) - 1

    def csr_arrays(self):
        A = self.A
        return (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))

    def sub_dofs(self, i):
        return self.sub_dof[self.sub_dof_ptr[i]:self.sub_dof_ptr[i + 1]]

    def sub_weights(self, i):
        return self.sub_pou[self.sub_dof_ptr[i]:self.sub_dof_ptr[i + 1]]

    def sub_elems(self, i):
        return self.sub_elem[self.sub_elem_ptr[i]:self.sub_elem_ptr[i + 1]]


def _split(n: int, p: int) -> np.ndarray:
    return np.array([(i * n) // p for i in range(p + 1)])


def box_partition(dim: int, N: int, P: int, delta: int):
    """Overlapping box partition: P^dim boxes of elements, each grown by delta layers."""
    cuts = _split(N, P)
    ec = element_coords(dim, N)
    ptr = [0]
    lists = []
    for bidx in itertools.product(range(P), repeat=dim):
        b = bidx[::-1]  # b[0] fastest -> subdomain id = bx + P*by (+P^2 bz)
        mask = np.ones(ec.shape[0], bool)
        for d in range(dim):
            lo = max(cuts[b[d]] - delta, 0)
            hi = min(cuts[b[d] + 1] + delta, N)
            mask &= (ec[:, d] >= lo) & (ec[:, d] < hi)
        el = np.nonzero(mask)[0].astype(np.int32)
        lists.append(el)
        ptr.append(ptr[-1] + len(el))
    return np.array(ptr, np.int64), np.concatenate(lists)


def group_parents(dim: int, P: int, G: int) -> np.ndarray:
    """Nonoverlapping grouping of a P^dim box grid into a G^dim grid of coarse subdomains."""
    par = np.zeros(P ** dim, np.int32)
    for bidx in itertools.product(range(P), repeat=dim):
        b = bidx[::-1]
        i = sum(b[d] * P ** d for d in range(dim))
        g = [(b[d] * G) // P for d in range(dim)]
        par[i] = sum(g[d] * G ** d for d in range(dim))
    return par


def neumann_spaces_and_pou(n: int, elem_dofs: np.ndarray, sub_elem_ptr, sub_elem):
    """V-bar dofs (free dofs of the subdomain's elements) and nodal multiplicity PoU."""
    P = len(sub_elem_ptr) - 1
    valid = elem_dofs >= 0
    deg = np.bincount(elem_dofs[valid], minlength=n)
    vbar, dirs = [], []
    for i in range(P):
        el = sub_elem[sub_elem_ptr[i]:sub_elem_ptr[i + 1]]
        ed = elem_dofs[el]
        ed = ed[ed >= 0]
        cnt = np.bincount(ed, minlength=n)
        dofs = np.nonzero(cnt)[0]
        vbar.append(dofs.astype(np.int32))
        dirs.append(cnt[dofs] == deg[dofs])
    mult = np.zeros(n)
    for i in range(P):
        mult[vbar[i][dirs[i]]] += 1
    if np.any(mult == 0):
        raise ValueError("some free dof lies in no subdomain interior (overlap too small)")
    ptr = [0]
    w = []
    for i in range(P):
        wi = np.where(dirs[i], 1.0 / mult[vbar[i]], 0.0)
        w.append(wi)
        ptr.append(ptr[-1] + len(vbar[i]))
    return np.array(ptr, np.int64), np.concatenate(vbar), np.concatenate(w)


def assemble(n: int, elem_dofs: np.ndarray, elem_mat: np.ndarray) -> sp.csr_matrix:
    ne, k = elem_dofs.shape
    r = np.repeat(elem_dofs, k, axis=1).reshape(-1)
    c = np.tile(elem_dofs, (1, k)).reshape(-1)
    v = elem_mat.reshape(-1)
    m = (r >= 0) & (c >= 0)
    A = sp.coo_matrix((v[m], (r[m], c[m])), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def build_problem(name: str, dim: int, N: int, coeff: np.ndarray, P: int, delta: int,
                  n_levels: int, eta: float, groups: Sequence[int] = (),
                  elasticity_materials: Optional[List[np.ndarray]] = None,
                  bc: str = "all", force: Sequence[float] = (1.0,)) -> Problem:
    """Assemble a structured-box problem.

    coeff: per-element scalar diffusion coefficient, or (elasticity) per-element
    material index into elasticity_materials (list of 6x6 Voigt matrices).
    groups: number of coarse subdomains per dimension for levels L-1, L-2, ...
    """
    h = 1.0 / N
    nodes = element_nodes(dim, N)
    ne = nodes.shape[0]
    bmask = boundary_nodes(dim, N, bc)
    nn = (N + 1) ** dim
    if elasticity_materials is None:
        ncomp = 1
        free = ~bmask
        num = -np.ones(nn, np.int64)
        num[free] = np.arange(free.sum())
        elem_dofs = num[nodes].astype(np.int32)
        Kref = q1_laplace_element(dim, h)
        elem_mat = coeff[:, None, None] * Kref[None]
        fe = q1_load_element(dim, h, 1, force)
    else:
        ncomp = 3
        assert dim == 3
        free_node = ~bmask
        num = -np.ones(nn * 3, np.int64)
        fd = np.repeat(free_node, 3)
        num[fd] = np.arange(fd.sum())
        elem_dofs = np.zeros((ne, 24), np.int32)
        for a in range(8):
            for c in range(3):
                elem_dofs[:, 3 * a + c] = num[3 * nodes[:, a] + c]
        Ks = np.stack([q1_elasticity_element(h, C) for C in elasticity_materials])
        elem_mat = Ks[coeff]
        fe = q1_load_element(3, h, 3, force)
    n = int(elem_dofs.max()) + 1
    A = assemble(n, elem_dofs, elem_mat)
    b = np.zeros(n)
    ed = elem_dofs.reshape(-1)
    fv = np.tile(fe, ne)
    m = ed >= 0
    np.add.at(b, ed[m], fv[m])
    sep, se = box_partition(dim, N, P, delta)
    sdp, sd, sw = neumann_spaces_and_pou(n, elem_dofs, sep, se)
    parents = []
    cur = P
    for G in groups:
        parents.append(group_parents(dim, cur, G))
        cur = G
    assert len(parents) == n_levels - 2, (len(parents), n_levels)
    return Problem(name=name, dim=dim, ncomp=ncomp, N=N, n=n, elem_dofs=elem_dofs,
                   elem_mat=np.ascontiguousarray(elem_mat), A=A, b=b, sub_elem_ptr=sep,
                   sub_elem=se, sub_dof_ptr=sdp, sub_dof=sd, sub_pou=sw, n_levels=n_levels,
                   parents=parents, eta=eta, coeff=coeff, box_shape=(P,) * dim)


# ----------------------------------------------------------------------------
# Cell-centred finite volumes and WSIP discontinuous Galerkin (2D, uniform grid)
# ----------------------------------------------------------------------------
#
# Both are written as sums of "element" matrices in the sense of the solver's input: one per
# cell (DG volume term) and one per face.  An interior face's matrix couples the dofs of its
# two cells, a Dirichlet boundary face's matrix those of its one cell.  A subdomain's element
# set is its cells' volume terms, the interior faces whose two cells both lie in it and the
# Dirichlet faces of its cells: their sum is the local matrix with Neumann conditions on the
# subdomain boundary inside the domain (the DG local form of Sec. 3.5, which for cell-centred
# finite volumes with two-point fluxes is the same construction).


def _cell_faces(N: int, bc: str):
    """Interior faces (cell_minus, cell_plus, axis) and Dirichlet boundary faces
    (cell, axis, side: -1 lower, +1 upper) of an N x N cell grid (cell id x + N y)."""
    inter, bnd = [], []
    for y in range(N):
        for x in range(N):
            c = x + N * y
            if x + 1 < N:
                inter.append((c, c + 1, 0))
            if y + 1 < N:
                inter.append((c, c + N, 1))
    dir_axes = (0, 1) if bc == "all" else (0,) if bc == "x01" else ()
    for ax in dir_axes:
        for t in range(N):
            lo = (0 + N * t) if ax == 0 else (t + 0)
            hi = ((N - 1) + N * t) if ax == 0 else (t + N * (N - 1))
            bnd.append((lo, ax, -1))
            bnd.append((hi, ax, +1))
    return inter, bnd


def _skeleton_subdomains(N: int, P: int, delta: int, inter, bnd, vol: bool):
    """Element sets of the overlapping cell boxes: element ids are [volume terms (cells) if
    vol] + interior faces + boundary faces, in that order."""
    cptr, cells = box_partition(2, N, P, delta)
    nvol = N * N if vol else 0
    fi = np.array([(a, b) for a, b, _ in inter], np.int64).reshape(-1, 2)
    fb = np.array([c for c, _, _ in bnd], np.int64)
    ptr, lists = [0], []
    for i in range(len(cptr) - 1):
        inside = np.zeros(N * N, bool)
        inside[cells[cptr[i]:cptr[i + 1]]] = True
        el = []
        if vol:
            el.append(np.nonzero(inside)[0])
        el.append(nvol + np.nonzero(inside[fi[:, 0]] & inside[fi[:, 1]])[0])
        el.append(nvol + len(fi) + np.nonzero(inside[fb])[0])
        el = np.concatenate(el).astype(np.int32)
        lists.append(el)
        ptr.append(ptr[-1] + len(el))
    return np.array(ptr, np.int64), np.concatenate(lists), cptr, cells


def _cell_pou(N: int, cptr, cells, dofs_per_cell: int):
    """Neumann dofs (all dofs of the box's cells) and the partition of unity: on a cell whose
    neighbours all lie in the box, 1 / #boxes in which it is such an interior cell; 0 on the
    box's boundary layer (cells with a neighbour outside the box inside the domain).  chi u
    then has no jump across the faces that leave the subdomain, so that
    abar(chi u, chi v) = a(chi u, chi v) as the DG right-hand side b^1 requires (Sec. 3.5)."""
    P = len(cptr) - 1
    interior = []
    mult = np.zeros(N * N)
    for i in range(P):
        inside = np.zeros(N * N, bool)
        c = np.sort(cells[cptr[i]:cptr[i + 1]])
        inside[c] = True
        x, y = c % N, c // N
        ok = np.ones(len(c), bool)
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            xx, yy = x + dx, y + dy
            valid = (xx >= 0) & (xx < N) & (yy >= 0) & (yy < N)
            nb = np.where(valid, xx + N * yy, 0)
            ok &= ~valid | inside[nb]
        interior.append(ok)
        mult[c[ok]] += 1
    if np.any(mult == 0):
        raise ValueError("some cell is interior to no subdomain (overlap too small)")
    ptr, dofs, w = [0], [], []
    for i in range(P):
        c = np.sort(cells[cptr[i]:cptr[i + 1]])
        d = (dofs_per_cell * c[:, None] + np.arange(dofs_per_cell)[None, :]).reshape(-1)
        dofs.append(d.astype(np.int32))
        w.append(np.repeat(np.where(interior[i], 1.0 / mult[c], 0.0), dofs_per_cell))
        ptr.append(ptr[-1] + len(d))
    return np.array(ptr, np.int64), np.concatenate(dofs), np.concatenate(w)


def fv_problem(N: int, coeff: np.ndarray, P: int, delta: int, n_levels: int = 2,
               groups: Sequence[int] = (), eta: float = 0.3, bc: str = "all",
               name: str = "fv") -> Problem:
    """Cell-centred finite volumes with two-point fluxes for -div(k grad u) = 1 on the unit
    square, N x N cells (one dof per cell): interior face between cells a, b with
    transmissibility t = 2 k_a k_b / (k_a + k_b) (face length h over centre distance h),
    matrix t [[1, -1], [-1, 1]]; Dirichlet face of cell c (u = 0 on it, centre distance h/2)
    t = 2 k_c on the cell's diagonal; right-hand side h^2 per cell.  Overlapping boxes of cells
    (delta >= 1 cell layers), PoU as in _cell_pou."""
    h = 1.0 / N
    inter, bnd = _cell_faces(N, bc)
    k = np.asarray(coeff, float)
    fi = np.array([(a, b) for a, b, _ in inter], np.int64).reshape(-1, 2)
    fb = np.array([c for c, _, _ in bnd], np.int64)
    ne = len(fi) + len(fb)
    ed = -np.ones((ne, 2), np.int32)
    em = np.zeros((ne, 2, 2))
    ka, kb = k[fi[:, 0]], k[fi[:, 1]]
    t = 2.0 * ka * kb / (ka + kb)
    ed[:len(fi)] = fi
    em[:len(fi)] = t[:, None, None] * np.array([[1.0, -1.0], [-1.0, 1.0]])[None]
    ed[len(fi):, 0] = fb
    em[len(fi):, 0, 0] = 2.0 * k[fb]
    n = N * N
    A = assemble(n, ed, em)
    b = np.full(n, h * h)
    sep, se, cptr, cells = _skeleton_subdomains(N, P, delta, inter, bnd, vol=False)
    sdp, sd, sw = _cell_pou(N, cptr, cells, 1)
    parents, cur = [], P
    for G in groups:
        parents.append(group_parents(2, cur, G))
        cur = G
    assert len(parents) == n_levels - 2
    return Problem(name=f"{name}_{N}", dim=2, ncomp=1, N=N, n=n, elem_dofs=ed, elem_mat=em,
                   A=A, b=b, sub_elem_ptr=sep, sub_elem=se, sub_dof_ptr=sdp, sub_dof=sd,
                   sub_pou=sw, n_levels=n_levels, parents=parents, eta=eta, coeff=k,
                   box_shape=(P, P), dirichlet_rule="all")


def _dg_face_matrix(h: float, km: float, kp: float, axis: int, alpha: float,
                    part: str = "all") -> np.ndarray:
    """WSIP interior-face matrix (8 x 8 over the Q1 dofs of the cell below/left, then the
    cell above/right; normal from the first to the second along `axis`):
      sigma ([u],[v]) - ({k grad u}_w . n, [v]) - ({k grad v}_w . n, [u]),
    [v] = v- - v+, {q}_w = w- q- + w+ q+ with w- = k+ / (k- + k+), w+ = k- / (k- + k+)
    (weights of Ern, Stephansen and Zunino for scalar k), sigma = alpha k_h / h with the
    harmonic mean k_h = 2 k- k+ / (k- + k+); two Gauss points on the face (exact here).
    part: "all", or one of the parts the matrix is linear in: "jump" (the penalty term per
    unit sigma), "minus" / "plus" (the consistency terms per unit w- k- / w+ k+)."""
    pts, wts = _gauss2()
    sig = alpha * (2.0 * km * kp / (km + kp)) / h
    wm, wp = kp / (km + kp), km / (km + kp)
    M = np.zeros((8, 8))
    for s, w in zip(pts, wts):
        xm = np.zeros(2)
        xp = np.zeros(2)
        xm[axis], xp[axis] = 1.0, 0.0          # the face is the upper side of the first cell
        xm[1 - axis] = xp[1 - axis] = s
        vm, gm = q1_shape(2, xm)
        vp, gp = q1_shape(2, xp)
        jump = np.concatenate([vm, -vp])
        zero = np.zeros(4)
        if part == "all":
            flux = np.concatenate([wm * km * gm[:, axis] / h, wp * kp * gp[:, axis] / h])
            M += w * h * (sig * np.outer(jump, jump) - np.outer(jump, flux) - np.outer(flux, jump))
        elif part == "jump":
            M += w * h * np.outer(jump, jump)
        else:
            flux = (np.concatenate([gm[:, axis] / h, zero]) if part == "minus"
                    else np.concatenate([zero, gp[:, axis] / h]))
            M -= w * h * (np.outer(jump, flux) + np.outer(flux, jump))
    return 0.5 * (M + M.T)


def _dg_boundary_matrix(h: float, kc: float, axis: int, side: int, alpha: float) -> np.ndarray:
    """WSIP Dirichlet-face matrix (4 x 4 over the cell's Q1 dofs, outward normal side e_axis):
    sigma (u, v) - (k grad u . n, v) - (k grad v . n, u), sigma = alpha k / h."""
    pts, wts = _gauss2()
    sig = alpha * kc / h
    M = np.zeros((4, 4))
    for s, w in zip(pts, wts):
        x = np.zeros(2)
        x[axis] = 1.0 if side > 0 else 0.0
        x[1 - axis] = s
        v, g = q1_shape(2, x)
        dn = side * kc * g[:, axis] / h
        M += w * h * (sig * np.outer(v, v) - np.outer(v, dn) - np.outer(dn, v))
    return 0.5 * (M + M.T)


def dg_problem(N: int, coeff: np.ndarray, P: int, delta: int, n_levels: int = 2,
               groups: Sequence[int] = (), eta: float = 0.3, bc: str = "all",
               alpha: float = 8.0, name: str = "dg") -> Problem:
    """WSIP discontinuous Galerkin with Q1 on N x N square cells (Sec. 3.5; four dofs per
    cell, the nodal basis at the cell's corners, dof 4 c + a): volume terms k_c times the Q1
    stiffness, interior-face and Dirichlet-face terms as in _dg_face_matrix and
    _dg_boundary_matrix (penalty alpha = 8), load int f v with f = 1.  Elements: cells (4
    dofs), interior faces (8), Dirichlet faces (4), padded to 8 with -1.  Overlapping boxes of
    cells (delta >= 1), PoU as in _cell_pou."""
    h = 1.0 / N
    inter, bnd = _cell_faces(N, bc)
    k = np.asarray(coeff, float)
    nc = N * N
    ne = nc + len(inter) + len(bnd)
    ed = -np.ones((ne, 8), np.int32)
    em = np.zeros((ne, 8, 8))
    Kq = q1_laplace_element(2, h)
    for c in range(nc):
        ed[c, :4] = 4 * c + np.arange(4)
        em[c, :4, :4] = k[c] * Kq
    # the face matrices are linear in (sigma, w- k-, w+ k+) (interior) and (sigma, k)
    # (Dirichlet): build the unit parts once per axis and side, then combine per face
    fa = np.array([(a, b, ax) for a, b, ax in inter], np.int64).reshape(-1, 3)
    for ax in (0, 1):
        sel = np.nonzero(fa[:, 2] == ax)[0]
        if not len(sel):
            continue
        J0 = _dg_face_matrix(h, 1.0, 1.0, ax, 0.0, part="jump")
        Fm = _dg_face_matrix(h, 1.0, 1.0, ax, 0.0, part="minus")
        Fp = _dg_face_matrix(h, 1.0, 1.0, ax, 0.0, part="plus")
        km, kp = k[fa[sel, 0]], k[fa[sel, 1]]
        sig = alpha * (2.0 * km * kp / (km + kp)) / h
        cm, cp = kp / (km + kp) * km, km / (km + kp) * kp
        e = nc + sel
        ed[e, :4] = 4 * fa[sel, 0:1] + np.arange(4)[None]
        ed[e, 4:] = 4 * fa[sel, 1:2] + np.arange(4)[None]
        em[e] = sig[:, None, None] * J0 + cm[:, None, None] * Fm + cp[:, None, None] * Fp
    for q, (c, ax, side) in enumerate(bnd):
        e = nc + len(inter) + q
        ed[e, :4] = 4 * c + np.arange(4)
        em[e, :4, :4] = _dg_boundary_matrix(h, k[c], ax, side, alpha)
    n = 4 * nc
    A = assemble(n, ed, em)
    fe = q1_load_element(2, h)
    b = np.tile(fe, nc)
    sep, se, cptr, cells = _skeleton_subdomains(N, P, delta, inter, bnd, vol=True)
    sdp, sd, sw = _cell_pou(N, cptr, cells, 4)
    parents, cur = [], P
    for G in groups:
        parents.append(group_parents(2, cur, G))
        cur = G
    assert len(parents) == n_levels - 2
    return Problem(name=f"{name}_{N}", dim=2, ncomp=1, N=N, n=n, elem_dofs=ed, elem_mat=em,
                   A=A, b=b, sub_elem_ptr=sep, sub_elem=se, sub_dof_ptr=sdp, sub_dof=sd,
                   sub_pou=sw, n_levels=n_levels, parents=parents, eta=eta, coeff=k,
                   box_shape=(P, P), dirichlet_rule="all")


def skeleton_field(N: int, seed: int, contrast: float = 1e4) -> np.ndarray:
    """Per-cell coefficient for the finite-volume and DG test problems: the seeded inclusion
    field (k = contrast on squares of 1-3 cells covering 10%, 1 elsewhere)."""
    return inclusions_2d(N, seed, smin=1, smax=3, k_hi=contrast)


# ----------------------------------------------------------------------------
# Coefficient fields
# ----------------------------------------------------------------------------


def channels_2d(N: int, rows_sets: Sequence[Sequence[int]], k_hi: float = 1e6) -> np.ndarray:
    ec = element_coords(2, N)
    k = np.ones(ec.shape[0])
    for rows in rows_sets:
        for r in rows:
            k[ec[:, 1] == r] = k_hi
    return k


def inclusions_2d(N: int, seed: int, frac: float = 0.10, smin: int = 2, smax: int = 8,
                  k_hi: float = 1e6) -> np.ndarray:
    """Seeded random square inclusions (side U{smin..smax}) until the union covers >= frac."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((N, N), bool)  # [ey, ex]
    while mask.mean() < frac:
        s = int(rng.integers(smin, smax + 1))
        x0 = int(rng.integers(0, N - s + 1))
        y0 = int(rng.integers(0, N - s + 1))
        mask[y0:y0 + s, x0:x0 + s] = True
    return np.where(mask.reshape(-1), k_hi, 1.0)


def gaussian_field(dim: int, N: int, seed: int, sigma2: float = 4.0, ell: float = 0.05) -> np.ndarray:
    """Stationary Gaussian field with covariance sigma2*exp(-r/ell) on element centres.

    Circulant embedding: the covariance is wrapped on a periodic grid of
    side m >= 2N; m is doubled until the embedding spectrum is nonnegative
    (up to round-off); the sample is the real part of an FFT of complex
    white noise scaled by sqrt(spectrum).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / N
    m = 2 * N
    while True:
        idx = np.arange(m)
        dd = np.minimum(idx, m - idx) * h
        grids = np.meshgrid(*([dd] * dim), indexing="ij")
        r = np.sqrt(sum(g * g for g in grids))
        c = sigma2 * np.exp(-r / ell)
        lam = np.real(scipy.fft.fftn(c))
        if lam.min() >= -1e-8 * lam.max():
            break
        m *= 2
    lam = np.maximum(lam, 0.0)
    xi = rng.standard_normal(lam.shape) + 1j * rng.standard_normal(lam.shape)
    g = scipy.fft.ifftn(np.sqrt(lam) * xi) * np.sqrt(lam.size)
    g = np.real(g)[tuple([slice(0, N)] * dim)]
    # element id e = ex + N ey (+N^2 ez): array axes (ez, ey, ex)
    return np.ascontiguousarray(g).reshape(-1)


def bars_3d(N: int, seed: int, nbars: int = 3, thick: int = 2) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((N, N, N), bool)  # [ez, ey, ex]
    for _ in range(nbars):
        ax = int(rng.integers(0, 3))
        c1 = int(rng.integers(0, N - thick + 1))
        c2 = int(rng.integers(0, N - thick + 1))
        sl = [slice(c1, c1 + thick), slice(c2, c2 + thick)]
        full = [None, None, None]
        # axis index in (x,y,z); array axes are (z,y,x)
        arr_ax = 2 - ax
        others = [a for a in range(3) if a != arr_ax]
        full[arr_ax] = slice(0, N)
        full[others[0]] = sl[0]
        full[others[1]] = sl[1]
        mask[tuple(full)] = True
    return mask.reshape(-1)


# ----------------------------------------------------------------------------
# The workloads (synthetic stand-ins for the paper's test problems)
# ----------------------------------------------------------------------------

C1_ROWS = ((12, 13), (25, 26), (37, 38), (50, 51))


def config1() -> Problem:
    """64x64 Q1, 4 channels of k=1e6, 4x4 boxes, overlap 2, 2 levels, eta=0.1."""
    N = 64
    k = channels_2d(N, C1_ROWS)
    return build_problem("c1_channels_64", 2, N, k, P=4, delta=2, n_levels=2, eta=0.1)


def config2(seed: int = 2) -> Problem:
    """512x512 Q1, binary inclusions (10%, sides 2..8, k=1e6), 16x16 boxes, overlap 2,
    3 levels (256 -> 16 -> 1), eta=0.1."""
    N = 512
    k = inclusions_2d(N, seed)
    return build_problem("c2_inclusions_512", 2, N, k, P=16, delta=2, n_levels=3, eta=0.1,
                         groups=(4,))


def islands_levels(P: int, n_levels: int, factor: int = 4):
    """Coarse groupings for a P x P box partition: each coarser level groups factor x factor
    boxes of the next finer one (fewer where P runs out), level 0 being one subdomain."""
    groups, cur = [], P
    for _ in range(n_levels - 2):
        nxt = max(1, cur // factor)
        if nxt == cur:
            raise ValueError("too many levels for this partition")
        groups.append(nxt)
        cur = nxt
    return tuple(groups)


def table3_islands(P: int, n_levels: int, seed: int = 3, elems_per_sub: int = 80,
                   delta: int = 3, eta: float = 0.3, factor: int = 4) -> Problem:
    """Weak-scaling workload of the Islands problem's shape (Table 3 of the paper): P x P
    subdomains of elems_per_sub^2 Q1 elements each (N = P * elems_per_sub), overlap delta = 3
    element layers, eta = 0.3, Dirichlet on the two planes x = 0 and x = 1 and homogeneous
    Neumann elsewhere.  The paper's island field is given only as a figure; the stand-in is
    the seeded square-inclusion field (k = 1e6 on squares of 2-8 elements covering 10% of the
    domain, 1 elsewhere), whose islands per subdomain stay statistically fixed as P grows."""
    N = P * elems_per_sub
    k = inclusions_2d(N, seed)
    return build_problem(f"t3_islands_{P}x{P}_L{n_levels}", 2, N, k, P=P, delta=delta,
                         n_levels=n_levels, eta=eta, groups=islands_levels(P, n_levels, factor),
                         bc="x01")


def table1_laplace(N: int, delta: int, P: int = 4, eta: float = 0.15) -> Problem:
    """The Laplace column of Table 1 of the paper: Q1 on N x N elements, k = 1, P x P
    subdomains (16), overlap delta element layers, two levels, eta = 0.15, Dirichlet on x = 0
    and x = 1 and homogeneous Neumann elsewhere (the islands problem's boundary conditions)."""
    return build_problem(f"t1_laplace_{N}_d{delta}", 2, N, np.ones(N * N), P=P, delta=delta,
                         n_levels=2, eta=eta, bc="x01")


def config3(E_fibre: float = 1e3, nu: float = 0.3) -> Problem:
    """48^3 trilinear elasticity, 16 plies 3 elements thick (fibre 0/90 deg alternating with
    resin), clamped at x=0, body force -z; 6^3 boxes, overlap 1, 3 levels (216 -> 27 -> 1)."""
    N = 48
    ec = element_coords(3, N)
    ply = ec[:, 2] // 3
    mats = [isotropic_voigt(1.0, nu), fibre_voigt(E_fibre, nu, (1, 0, 0)),
            fibre_voigt(E_fibre, nu, (0, 1, 0))]
    mat = np.where(ply % 2 == 1, 0, np.where(ply % 4 == 0, 1, 2)).astype(np.int64)
    return build_problem("c3_composite_48", 3, N, mat, P=6, delta=1, n_levels=3, eta=0.1,
                         groups=(3,), elasticity_materials=mats, bc="x0", force=(0.0, 0.0, -1.0))


def config5(seed: int = 5, N: int = 96) -> Problem:
    """96^3 Q1 diffusion, seeded bars (k=1e6) over a log-normal field; 8^3 boxes, overlap 1,
    3 levels (512 -> 64 -> 1)."""
    g = gaussian_field(3, N, seed)
    k = np.exp(g)
    k[bars_3d(N, seed)] = 1e6
    return build_problem("c5_mixed_96", 3, N, k, P=8, delta=1, n_levels=3, eta=0.1, groups=(4,))


def config4_members(seed: int = 4, count: int = 32):
    """Sizes of the batch of independent 2D log-normal problems."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = rng.integers(128, 1025, size=count)
    out = []
    for b, N in enumerate(Ns):
        P = int(np.clip(round(N / 32), 4, 32))
        G = max(2, int(np.ceil(P / 4)))
        out.append((int(N), P, G, 4000 + b))
    return out


def config4_problem(N: int, P: int, G: int, seed: int) -> Problem:
    k = np.exp(gaussian_field(2, N, seed))
    return build_problem(f"c4_lognormal_{N}", 2, N, k, P=P, delta=2, n_levels=3, eta=0.1,
                         groups=(G,))


def small_problem(N: int = 8, P: int = 2, delta: int = 1, n_levels: int = 2, groups=(),
                  dim: int = 2, contrast: float = 1.0, seed: int = 0, eta: float = 0.1,
                  kind: str = "random") -> Problem:
    """Tiny test meshes with optional random high-contrast coefficient."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ne = N ** dim
    if contrast == 1.0:
        k = np.ones(ne)
    elif kind == "random":
        k = np.where(rng.random(ne) < 0.2, contrast, 1.0)
    elif kind == "channels":
        ec = element_coords(dim, N)
        k = np.where((ec[:, 1] % 4) == 1, contrast, 1.0)
    else:
        raise ValueError(kind)
    return build_problem(f"small_{dim}d_{N}", dim, N, k, P=P, delta=delta, n_levels=n_levels,
                         eta=eta, groups=groups)


def small_elasticity(N: int = 4, P: int = 2, delta: int = 1, n_levels: int = 2, groups=(),
                     E_fibre: float = 10.0, eta: float = 0.1) -> Problem:
    ec = element_coords(3, N)
    mats = [isotropic_voigt(1.0, 0.3), fibre_voigt(E_fibre, 0.3, (1, 0, 0))]
    mat = (ec[:, 2] % 2).astype(np.int64)
    return build_problem(f"small_elast_{N}", 3, N, mat, P=P, delta=delta, n_levels=n_levels,
                         eta=eta, groups=groups, elasticity_materials=mats, bc="x0",
                         force=(0.0, 0.0, -1.0))


def free_dof_coords(prob: Problem):
    """Coordinates [n, dim] and component index [n] of each free dof (for rigid-body tests)."""
    dim, N = prob.dim, prob.N
    M = N + 1
    nn = M ** dim
    c = np.stack(np.meshgrid(*([np.arange(M)] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1]
    c = c / N
    nodes = element_nodes(dim, N)
    coords = np.zeros((prob.n, dim))
    comp = np.zeros(prob.n, np.int64)
    k = prob.k
    for a in range(2 ** dim):
        for cc in range(prob.ncomp):
            col = a * prob.ncomp + cc
            dd = prob.elem_dofs[:, col]
            m = dd >= 0
            coords[dd[m]] = c[nodes[m, a]]
            comp[dd[m]] = cc
    assert nn > 0 and k > 0
    return coords, comp


# ----------------------------------------------------------------------------
# Frame layout of the learned warm start (inputs only; no solver arithmetic)
# ----------------------------------------------------------------------------

def warm_frame(prob: Problem, delta: int, log_scale: float = 4.0):
    """Features and frame positions of every finest-level box subdomain of a scalar
    problem on the structured mesh.

    The frame of box b is the element block [cut_b - delta, cut_b + core + delta) per
    dimension (core = widest box), so that the box's own elements always sit at the same
    frame place; elements of the frame outside the subdomain (at the domain boundary) are
    absent.  Features per subdomain (float32):
      [log10(k_e) / log_scale on the E^dim frame elements (0 where absent),
       presence flag per frame element,
       2*dim flags: the frame's low / high side reaches the domain boundary].
    sub_pos (int32, aligned with prob.sub_dof): frame node index of each Neumann dof.
    Returns feat [P, 2 E^dim + 2 dim], sub_pos, n_pos = (E+1)^dim.
    """
    if prob.ncomp != 1 or prob.box_shape is None:
        raise ValueError("warm_frame needs a scalar problem on a box partition")
    dim, N = prob.dim, prob.N
    Pd = prob.box_shape[0]
    cuts = _split(N, Pd)
    core = int(np.max(np.diff(cuts)))
    E = core + 2 * delta
    M = E + 1
    n_pos = M ** dim
    ec = element_coords(dim, N)
    logk = np.log10(np.asarray(prob.coeff, np.float64)) / log_scale
    # integer node coordinates of each free dof
    nn = (N + 1) ** dim
    ncoord = np.stack(np.meshgrid(*([np.arange(N + 1)] * dim), indexing="ij"), -1).reshape(-1, dim)[:, ::-1]
    nodes = element_nodes(dim, N)
    dof_node = np.full(prob.n, -1, np.int64)
    ed = prob.elem_dofs
    valid = ed >= 0
    dof_node[ed[valid]] = nodes[valid]
    assert np.all(dof_node >= 0) and nn == ncoord.shape[0]
    dof_xyz = ncoord[dof_node]
    P = prob.n_sub
    feat = np.zeros((P, 2 * E ** dim + 2 * dim), np.float32)
    sub_pos = np.full(prob.sub_dof.shape[0], -1, np.int32)
    strides_e = np.array([E ** d for d in range(dim)])
    strides_n = np.array([M ** d for d in range(dim)])
    for i, bidx in enumerate(itertools.product(range(Pd), repeat=dim)):
        b = bidx[::-1]  # same box numbering as box_partition
        origin = np.array([cuts[b[d]] - delta for d in range(dim)])
        el = prob.sub_elems(i)
        fe = ((ec[el] - origin) * strides_e).sum(1)
        assert fe.min() >= 0 and fe.max() < E ** dim
        feat[i, fe] = logk[el]
        feat[i, E ** dim + fe] = 1.0
        for d in range(dim):
            feat[i, 2 * E ** dim + 2 * d] = float(origin[d] <= 0)
            feat[i, 2 * E ** dim + 2 * d + 1] = float(origin[d] + E >= N)
        lo, hi = prob.sub_dof_ptr[i], prob.sub_dof_ptr[i + 1]
        fp = ((dof_xyz[prob.sub_dof[lo:hi]] - origin) * strides_n).sum(1)
        assert fp.min() >= 0 and fp.max() < n_pos
        sub_pos[lo:hi] = fp
    return feat, sub_pos, n_pos
