// Coarse levels: patch matrices, coarse Neumann matrices on generating systems,
// coarse GEVPs and dense factorisations.
//
// Paper, Sec. 4.1: a volume patch gathers the elements whose set of
// containing subdomains is the same sigma; the patch matrix holds their
// contributions.  Projected onto the coarse basis functions of the patch's
// subdomains, patch matrices give both the Galerkin matrix A_{l-1}
// (the sum of all patches) and the Neumann matrix of a coarse subdomain
// (the sum of the patches that meet it), since a_tau(phi_j, .) vanishes
// unless tau lies in subdomain j.
// Sec. 4.2: on levels l < L the Neumann space is spanned by a generating
// system (owned functions plus restrictions of the neighbours' functions), so
// ker A cap ker B != {0}.  With the 0/1 owned mask as partition of unity,
// B = [[A_oo, 0], [0, 0]] and the finite spectrum of A x = lambda B x is that of
// the generalized Schur pencil (A_oo - A_og A_gg^- A_go) y = lambda A_oo y,
// which is independent of the choice of generalized inverse; we take the one
// of a diagonally pivoted Cholesky factorisation of A_gg (pivots below
// eps_reg * max diag treated as zero), which plays the role of the paper's
// regularised LDL^T.
#include "common.h"
#include "jacobi.h"
#include "kernels.h"

// V[p] (npd x M, column-major): values of the patch's coarse functions at the patch dofs
__global__ void k_patch_gather(const i64* __restrict__ pdof_ptr, const i32* __restrict__ pM,
                               const i64* __restrict__ mem_ptr, const i32* __restrict__ mem_sub,
                               const i32* __restrict__ mem_col, const i64* __restrict__ ploc_off,
                               const i32* __restrict__ ploc, const i32* __restrict__ nb,
                               const i32* __restrict__ msub, const i64* __restrict__ phi_off,
                               const double* __restrict__ Phi, const i64* __restrict__ vpoff,
                               double* __restrict__ Vp) {
  const int p = blockIdx.x;
  const int npd = (int)(pdof_ptr[p + 1] - pdof_ptr[p]);
  const int M = pM[p];
  const int nm = (int)(mem_ptr[p + 1] - mem_ptr[p]);
  double* V = Vp + vpoff[p];
  const i32* pl = ploc + ploc_off[p];
  for (int s = 0; s < nm; ++s) {
    const int j = mem_sub[mem_ptr[p] + s];
    const int c0 = mem_col[mem_ptr[p] + s];
    const int mj = msub[j];
    const double* Pj = Phi + phi_off[j];
    const int nj = nb[j];
    for (int t = threadIdx.x; t < npd * mj; t += blockDim.x) {
      const int r = t % npd, c = t / npd;
      const int loc = pl[(i64)r * nm + s];
      V[r + (i64)(c0 + c) * npd] = loc >= 0 ? Pj[loc + (i64)c * nj] : 0.0;
    }
  }
  (void)M;
}

// U = A_patch V via the patch's dof incidence lists (deterministic gather)
__global__ void k_patch_av(i64 total_rows, const i32* __restrict__ row_patch,
                           const i64* __restrict__ pdof_ptr, const i32* __restrict__ pM,
                           const i64* __restrict__ inc_ptr, const i32* __restrict__ inc_slot,
                           const i32* __restrict__ inc_a, const i32* __restrict__ slot_elem,
                           const i32* __restrict__ slot_loc, int k,
                           const double* __restrict__ elem_mat, const i64* __restrict__ vpoff,
                           const double* __restrict__ Vp, double* __restrict__ Up) {
  i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int p = row_patch[g];
  const int r = (int)(g - pdof_ptr[p]);
  const int npd = (int)(pdof_ptr[p + 1] - pdof_ptr[p]);
  const int M = pM[p];
  const double* V = Vp + vpoff[p];
  double* U = Up + vpoff[p];
  for (int c0 = 0; c0 < M; c0 += 8) {
    double acc[8];
    for (int u = 0; u < 8; ++u) acc[u] = 0;
    for (i64 q = inc_ptr[g]; q < inc_ptr[g + 1]; ++q) {
      const i64 slot = inc_slot[q];
      const int a = inc_a[q];
      const double* Krow = elem_mat + (i64)slot_elem[slot] * k * k + (i64)a * k;
      const i32* loc = slot_loc + slot * k;
      for (int bb = 0; bb < k; ++bb) {
        const int cc = loc[bb];
        if (cc < 0) continue;
        const double kv = Krow[bb];
        for (int u = 0; u < 8; ++u)
          if (c0 + u < M) acc[u] += kv * V[cc + (i64)(c0 + u) * npd];
      }
    }
    for (int u = 0; u < 8; ++u)
      if (c0 + u < M) U[r + (i64)(c0 + u) * npd] = acc[u];
  }
}

// Pm[p] = V^T U  (M x M, column-major), symmetrised
__global__ void k_patch_gram(const i64* __restrict__ pdof_ptr, const i32* __restrict__ pM,
                             const i64* __restrict__ vpoff, const double* __restrict__ Vp,
                             const double* __restrict__ Up, const i64* __restrict__ pmoff,
                             double* __restrict__ Pm) {
  const int p = blockIdx.x;
  const int npd = (int)(pdof_ptr[p + 1] - pdof_ptr[p]);
  const int M = pM[p];
  const double* V = Vp + vpoff[p];
  const double* U = Up + vpoff[p];
  double* Q = Pm + pmoff[p];
  for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
    const int a = t % M, b = t / M;
    if (a > b) continue;
    double s1 = 0, s2 = 0;
    const double* va = V + (i64)a * npd;
    const double* ub = U + (i64)b * npd;
    const double* vb = V + (i64)b * npd;
    const double* ua = U + (i64)a * npd;
    for (int r = 0; r < npd; ++r) {
      s1 += va[r] * ub[r];
      s2 += vb[r] * ua[r];
    }
    const double v = 0.5 * (s1 + s2);
    Q[a + (i64)b * M] = v;
    Q[b + (i64)a * M] = v;
  }
}

// Level-l patch matrix from its child (level l+1) patches: Q = sum_child T^T P_child T,
// T mapping the child patch's functions to the parents' new functions (blocks of Y).
__global__ void k_patch_project(const i64* __restrict__ ch_ptr, const i32* __restrict__ ch_patch,
                                const i32* __restrict__ cM, const i64* __restrict__ cmoff,
                                const double* __restrict__ Pc, const i64* __restrict__ cmem_ptr,
                                const i32* __restrict__ cmem_pslot,
                                const i32* __restrict__ cmem_ownbase,
                                const i32* __restrict__ cmem_m, const i32* __restrict__ cmem_col,
                                const i64* __restrict__ pmem_ptr, const i32* __restrict__ pmem_sub,
                                const i32* __restrict__ pmem_col, const i32* __restrict__ mpar,
                                const i32* __restrict__ nown, const i64* __restrict__ yoff,
                                const double* __restrict__ Y, const i32* __restrict__ pMout,
                                const i64* __restrict__ poutoff, double* __restrict__ Pout,
                                const i64* __restrict__ wsoff, double* __restrict__ Wsc) {
  const int q = blockIdx.x;  // level-l patch
  const int Mo = pMout[q];
  double* Q = Pout + poutoff[q];
  double* W = Wsc + wsoff[q];
  for (int t = threadIdx.x; t < Mo * Mo; t += blockDim.x) Q[t] = 0.0;
  __syncthreads();
  const i64 pm0 = pmem_ptr[q];
  for (i64 cc = ch_ptr[q]; cc < ch_ptr[q + 1]; ++cc) {
    const int cp = ch_patch[cc];
    const int Mc = cM[cp];
    const double* P = Pc + cmoff[cp];
    const i64 c0 = cmem_ptr[cp];
    const int ncm = (int)(cmem_ptr[cp + 1] - c0);
    // W = P T  (Mc x Mo, column-major)
    for (int t = threadIdx.x; t < Mc * Mo; t += blockDim.x) {
      const int row = t % Mc, colo = t / Mc;
      // which parent slot owns output column colo
      int ps = 0;
      const int npm = (int)(pmem_ptr[q + 1] - pm0);
      while (ps + 1 < npm && pmem_col[pm0 + ps + 1] <= colo) ++ps;
      const int ipar = pmem_sub[pm0 + ps];
      const int kcol = colo - pmem_col[pm0 + ps];
      const int no = nown[ipar];
      const double* Yi = Y + yoff[ipar];
      double acc = 0.0;
      for (int s = 0; s < ncm; ++s) {
        if (cmem_pslot[c0 + s] != ps) continue;
        const int mj = cmem_m[c0 + s];
        const int ob = cmem_ownbase[c0 + s];
        const int cb = cmem_col[c0 + s];
        for (int k2 = 0; k2 < mj; ++k2)
          acc += P[row + (i64)(cb + k2) * Mc] * Yi[ob + k2 + (i64)kcol * no];
      }
      W[row + (i64)colo * Mc] = acc;
    }
    __syncthreads();
    // Q += T^T W
    for (int t = threadIdx.x; t < Mo * Mo; t += blockDim.x) {
      const int ro = t % Mo, co = t / Mo;
      int ps = 0;
      const int npm = (int)(pmem_ptr[q + 1] - pm0);
      while (ps + 1 < npm && pmem_col[pm0 + ps + 1] <= ro) ++ps;
      const int ipar = pmem_sub[pm0 + ps];
      const int krow = ro - pmem_col[pm0 + ps];
      const int no = nown[ipar];
      const double* Yi = Y + yoff[ipar];
      double acc = 0.0;
      for (int s = 0; s < ncm; ++s) {
        if (cmem_pslot[c0 + s] != ps) continue;
        const int mj = cmem_m[c0 + s];
        const int ob = cmem_ownbase[c0 + s];
        const int cb = cmem_col[c0 + s];
        for (int k1 = 0; k1 < mj; ++k1)
          acc += Yi[ob + k1 + (i64)krow * no] * W[cb + k1 + (i64)co * Mc];
      }
      Q[t] += acc;
    }
    __syncthreads();
  }
  (void)mpar;
}

// Dense coarse matrix (ng x ng, column-major) of target t = sum of its patches' blocks.
__global__ void k_coarse_assemble(const i64* __restrict__ tp_ptr, const i32* __restrict__ tp_patch,
                                  const i64* __restrict__ tp_map_off, const i32* __restrict__ tp_map,
                                  const i32* __restrict__ pM, const i64* __restrict__ pmoff,
                                  const double* __restrict__ Pm, const i32* __restrict__ ng_arr,
                                  const i64* __restrict__ aoff, double* __restrict__ Aout) {
  const int t = blockIdx.x;
  const int ng = ng_arr[t];
  double* A = Aout + aoff[t];
  for (i64 e = threadIdx.x; e < (i64)ng * ng; e += blockDim.x) A[e] = 0.0;
  __syncthreads();
  for (i64 c = tp_ptr[t]; c < tp_ptr[t + 1]; ++c) {
    const int p = tp_patch[c];
    const int M = pM[p];
    const double* P = Pm + pmoff[p];
    const i32* map = tp_map + tp_map_off[c];  // patch function -> generating index
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
      const int a = e % M, b = e / M;
      const int ga = map[a], gb = map[b];
      if (ga >= 0 && gb >= 0) A[ga + (i64)gb * ng] += P[e];
    }
    __syncthreads();
  }
}

// In-place dense Cholesky of an n x n column-major matrix held in global memory
// (lower triangle); one workgroup.  Returns false on a non-positive pivot.
__device__ bool dense_cholesky_block(int n, double* A, int lda, int* fail_sh) {
  if (threadIdx.x == 0) *fail_sh = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double ajj = A[j + (i64)j * lda];
    if (!(ajj > 0.0)) return false;
    const double l = sqrt(ajj);
    __syncthreads();
    for (int r = j + threadIdx.x; r < n; r += blockDim.x)
      A[r + (i64)j * lda] = (r == j) ? l : A[r + (i64)j * lda] / l;
    __syncthreads();
    const int rem = n - j - 1;
    for (i64 t = threadIdx.x; t < (i64)rem * rem; t += blockDim.x) {
      const int r = j + 1 + (int)(t % rem), c = j + 1 + (int)(t / rem);
      if (c <= r) A[r + (i64)c * lda] -= A[r + (i64)j * lda] * A[c + (i64)j * lda];
    }
    __syncthreads();
  }
  for (i64 t = threadIdx.x; t < (i64)n * n; t += blockDim.x) {
    const int r = (int)(t % n), c = (int)(t / n);
    if (r < c) A[r + (i64)c * lda] = 0.0;
  }
  __syncthreads();
  return true;
}

__global__ void k_dense_cholesky(int n, double* A, int* status) {
  __shared__ int f;
  bool ok = dense_cholesky_block(n, A, n, &f);
  if (threadIdx.x == 0) status[0] = ok ? ST_DONE : ST_NOTSPD;
}

// Coarse GEVP of one level-(l-1) subdomain per workgroup (see file header).
// Abar: ng x ng column-major, owned functions first (no of them).
// Outputs: Lo (no x no, lower Cholesky factor of A_oo, column-major),
// Yout (no x m, column-major: selected eigenvectors, b-normalised),
// lam (no entries, ascending), m, rank of the ghost block.
__global__ void k_coarse_gevp(const i32* __restrict__ ng_arr, const i32* __restrict__ no_arr,
                              const i64* __restrict__ aoff, double* __restrict__ Abar,
                              const i64* __restrict__ loff, double* __restrict__ Lo,
                              const i64* __restrict__ soff, double* __restrict__ scratch,
                              double eta, int nev_max, double eps_reg,
                              double* __restrict__ lam_out, const i64* __restrict__ lamoff,
                              int* __restrict__ m_out, int* __restrict__ status,
                              int* __restrict__ rank_out) {
  const int t = blockIdx.x;
  const int ng = ng_arr[t], no = no_arr[t];
  const int ngh = ng - no;
  double* A = Abar + aoff[t];
  double* L = Lo + loff[t];
  double* G = scratch + soff[t];             // ngh*ngh
  double* Z = G + (i64)ngh * ngh;            // ngh*no  (rows: pivoted ghosts)
  double* Sc = Z + (i64)ngh * no;            // no*no
  double* Mm = Sc + (i64)no * no;            // no*no (row-major for Jacobi)
  double* Qm = Mm + (i64)no * no;            // no*no
  double* Yt = Qm + (i64)no * no;            // no*no (selected eigenvectors)
  int* perm = reinterpret_cast<int*>(Yt + (i64)no * no);  // max(ngh, no)
  __shared__ int sh_rank, sh_piv, sh_fail, cnt;
  __shared__ double sh_dmax, red_v[16];
  __shared__ int red_i[16];
  __shared__ int pp[256], pq[256];
  __shared__ double pc[256], ps[256];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (no == 0) {
    if (tid == 0) { m_out[t] = 0; status[t] = ST_DONE; rank_out[t] = 0; }
    return;
  }
  // (a) pivoted Cholesky of the ghost block
  for (i64 e = tid; e < (i64)ngh * ngh; e += nt) {
    const int r = (int)(e % ngh), c = (int)(e / ngh);
    G[e] = A[(no + r) + (i64)(no + c) * ng];
  }
  for (int r = tid; r < ngh; r += nt) perm[r] = r;
  if (tid == 0) {
    double dm = 0;
    for (int r = 0; r < ngh; ++r) dm = fmax(dm, A[(no + r) + (i64)(no + r) * ng]);
    sh_dmax = dm;
    sh_rank = ngh;
  }
  __syncthreads();
  for (int k = 0; k < ngh; ++k) {
    // argmax of the remaining diagonal
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int r = k + tid; r < ngh; r += nt) {
      const double v = G[r + (i64)r * ngh];
      if (v > bv || (v == bv && r < bi)) { bv = v; bi = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if ((tid & 63) == 0) { red_v[tid >> 6] = bv; red_i[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      double v0 = red_v[0];
      int i0 = red_i[0];
      for (int w = 1; w < nt / 64; ++w)
        if (red_v[w] > v0 || (red_v[w] == v0 && red_i[w] < i0)) { v0 = red_v[w]; i0 = red_i[w]; }
      sh_piv = i0;
      if (!(v0 > eps_reg * sh_dmax)) sh_rank = k;
    }
    __syncthreads();
    if (sh_rank == k) break;
    const int pv = sh_piv;
    if (pv != k) {  // symmetric swap of rows/cols k and pv
      for (int c = tid; c < ngh; c += nt) {
        const double x = G[k + (i64)c * ngh];
        G[k + (i64)c * ngh] = G[pv + (i64)c * ngh];
        G[pv + (i64)c * ngh] = x;
      }
      __syncthreads();
      for (int r = tid; r < ngh; r += nt) {
        const double x = G[r + (i64)k * ngh];
        G[r + (i64)k * ngh] = G[r + (i64)pv * ngh];
        G[r + (i64)pv * ngh] = x;
      }
      if (tid == 0) {
        const int x = perm[k];
        perm[k] = perm[pv];
        perm[pv] = x;
      }
      __syncthreads();
    }
    const double l = sqrt(G[k + (i64)k * ngh]);
    __syncthreads();
    for (int r = k + tid; r < ngh; r += nt)
      G[r + (i64)k * ngh] = (r == k) ? l : G[r + (i64)k * ngh] / l;
    __syncthreads();
    const int rem = ngh - k - 1;
    for (i64 e = tid; e < (i64)rem * rem; e += nt) {
      const int r = k + 1 + (int)(e % rem), c = k + 1 + (int)(e / rem);
      if (c <= r) {
        const double v = G[r + (i64)c * ngh] - G[r + (i64)k * ngh] * G[c + (i64)k * ngh];
        G[r + (i64)c * ngh] = v;
        G[c + (i64)r * ngh] = v;
      }
    }
    __syncthreads();
  }
  const int rk = sh_rank;
  // (b) Z = L11^{-1} A_{g1,o}   (rk x no), thread per owned column
  for (int c = tid; c < no; c += nt) {
    for (int r = 0; r < rk; ++r) {
      double v = A[(no + perm[r]) + (i64)c * ng];
      for (int q = 0; q < r; ++q) v -= G[r + (i64)q * ngh] * Z[q + (i64)c * ngh];
      Z[r + (i64)c * ngh] = v / G[r + (i64)r * ngh];
    }
  }
  __syncthreads();
  // (c) Sc = A_oo - Z^T Z ; copy A_oo into L
  for (i64 e = tid; e < (i64)no * no; e += nt) {
    const int r = (int)(e % no), c = (int)(e / no);
    double v = A[r + (i64)c * ng];
    L[r + (i64)c * no] = 0.5 * (A[r + (i64)c * ng] + A[c + (i64)r * ng]);
    for (int q = 0; q < rk; ++q) v -= Z[q + (i64)r * ngh] * Z[q + (i64)c * ngh];
    Sc[e] = v;
  }
  __syncthreads();
  for (i64 e = tid; e < (i64)no * no; e += nt) {
    const int r = (int)(e % no), c = (int)(e / no);
    if (r < c) {
      const double v = 0.5 * (Sc[r + (i64)c * no] + Sc[c + (i64)r * no]);
      Sc[r + (i64)c * no] = v;
      Sc[c + (i64)r * no] = v;
    }
  }
  __syncthreads();
  // (d) Cholesky of A_oo (the level's Dirichlet matrix)
  if (!dense_cholesky_block(no, L, no, &sh_fail)) {
    if (tid == 0) { status[t] = ST_NOTSPD; m_out[t] = 0; }
    return;
  }
  // (e) M = L^{-1} Sc L^{-T}: first Sc <- L^{-1} Sc (columns), then M = L^{-1} (Sc)^T
  for (int c = tid; c < no; c += nt) {
    for (int r = 0; r < no; ++r) {
      double v = Sc[r + (i64)c * no];
      for (int q = 0; q < r; ++q) v -= L[r + (i64)q * no] * Sc[q + (i64)c * no];
      Sc[r + (i64)c * no] = v / L[r + (i64)r * no];
    }
  }
  __syncthreads();
  // Mm (row-major): column c of M = L^{-1} (row c of Sc)^T
  for (int c = tid; c < no; c += nt) {
    for (int r = 0; r < no; ++r) {
      double v = Sc[c + (i64)r * no];
      for (int q = 0; q < r; ++q) v -= L[r + (i64)q * no] * Mm[(i64)q * no + c];
      Mm[(i64)r * no + c] = v / L[r + (i64)r * no];
    }
  }
  __syncthreads();
  for (i64 e = tid; e < (i64)no * no; e += nt) {
    const int r = (int)(e / no), c = (int)(e % no);
    if (r < c) {
      const double v = 0.5 * (Mm[(i64)r * no + c] + Mm[(i64)c * no + r]);
      Mm[(i64)r * no + c] = v;
      Mm[(i64)c * no + r] = v;
    }
  }
  __syncthreads();
  // (f) eigenvalues lambda of M (they lie in [0,1])
  JacobiScratch<double> js{pp, pq, pc, ps, &cnt};
  jacobi_block<double>(no, Mm, Qm, js, 60, 1e-15, 0.0);
  // (g) sort ascending, select, back-transform y = L^{-T} q into Yt (no x m)
  double* lam = lam_out + lamoff[t];
  if (tid == 0) {
    int* ord = perm;  // reuse
    for (int a = 0; a < no; ++a) ord[a] = a;
    for (int a = 1; a < no; ++a) {
      const int v = ord[a];
      const double lv = Mm[(i64)v * no + v];
      int b = a - 1;
      while (b >= 0 && Mm[(i64)ord[b] * no + ord[b]] > lv) {
        ord[b + 1] = ord[b];
        --b;
      }
      ord[b + 1] = v;
    }
    int m = 0;
    for (int a = 0; a < no; ++a) {
      const double lv = fmax(Mm[(i64)ord[a] * no + ord[a]], 0.0);
      lam[a] = lv;
      if (lv < eta) ++m;
    }
    if (nev_max > 0 && m > nev_max) m = nev_max;
    m_out[t] = m;
    rank_out[t] = rk;
    status[t] = ST_DONE;
  }
  __syncthreads();
  const int m = m_out[t];
  for (int c = tid; c < m; c += nt) {
    const int src = perm[c];
    for (int r = no - 1; r >= 0; --r) {
      double v = Qm[(i64)r * no + src];
      for (int q = r + 1; q < no; ++q) v -= L[q + (i64)r * no] * Yt[q + (i64)c * no];
      Yt[r + (i64)c * no] = v / L[r + (i64)r * no];
    }
  }
}

// Copy the selected eigenvectors (left in the scratch) to the pooled basis, fixing signs.
// Scratch layout per target: G ngh^2 | Z ngh*no | Sc, Mm, Qm, Yt no^2 each | ints.
__global__ void k_coarse_collect(const i32* __restrict__ ng_arr, const i32* __restrict__ no_arr,
                                 const i64* __restrict__ soff, const double* __restrict__ scratch,
                                 const int* __restrict__ m_arr, const i64* __restrict__ yoff,
                                 double* __restrict__ Y) {
  const int t = blockIdx.x;
  const int ng = ng_arr[t], no = no_arr[t];
  const int ngh = ng - no;
  const int m = m_arr[t];
  const double* Z = scratch + soff[t] + (i64)ngh * ngh + (i64)ngh * no + 3 * (i64)no * no;
  double* Yt = Y + yoff[t];
  for (int c = 0; c < m; ++c) {
    __shared__ double sgn;
    if (threadIdx.x == 0) {
      double best = -1, v = 0;
      for (int r = 0; r < no; ++r) {
        const double a = fabs(Z[r + (i64)c * no]);
        if (a > best) { best = a; v = Z[r + (i64)c * no]; }
      }
      sgn = v < 0 ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < no; r += blockDim.x) Yt[r + (i64)c * no] = sgn * Z[r + (i64)c * no];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
void launch_patch_gather(hipStream_t s, int np, const i64* pdof_ptr, const i32* pM,
                         const i64* mem_ptr, const i32* mem_sub, const i32* mem_col,
                         const i64* ploc_off, const i32* ploc, const i32* nb, const i32* msub,
                         const i64* phi_off, const double* Phi, const i64* vpoff, double* Vp) {
  if (!np) return;
  hipLaunchKernelGGL(k_patch_gather, dim3(np), dim3(MSDD_WG), 0, s, pdof_ptr, pM, mem_ptr,
                     mem_sub, mem_col, ploc_off, ploc, nb, msub, phi_off, Phi, vpoff, Vp);
}
void launch_patch_av(hipStream_t s, i64 total_rows, const i32* row_patch, const i64* pdof_ptr,
                     const i32* pM, const i64* inc_ptr, const i32* inc_slot, const i32* inc_a,
                     const i32* slot_elem, const i32* slot_loc, int k, const double* elem_mat,
                     const i64* vpoff, const double* Vp, double* Up) {
  if (!total_rows) return;
  dim3 g((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG));
  hipLaunchKernelGGL(k_patch_av, g, dim3(MSDD_WG), 0, s, total_rows, row_patch, pdof_ptr, pM,
                     inc_ptr, inc_slot, inc_a, slot_elem, slot_loc, k, elem_mat, vpoff, Vp, Up);
}
void launch_patch_gram(hipStream_t s, int np, const i64* pdof_ptr, const i32* pM,
                       const i64* vpoff, const double* Vp, const double* Up, const i64* pmoff,
                       double* Pm) {
  if (!np) return;
  hipLaunchKernelGGL(k_patch_gram, dim3(np), dim3(MSDD_WG), 0, s, pdof_ptr, pM, vpoff, Vp, Up,
                     pmoff, Pm);
}
void launch_patch_project(hipStream_t s, int nq, const i64* ch_ptr, const i32* ch_patch,
                          const i32* cM, const i64* cmoff, const double* Pc,
                          const i64* cmem_ptr, const i32* cmem_pslot, const i32* cmem_ownbase,
                          const i32* cmem_m, const i32* cmem_col, const i64* pmem_ptr,
                          const i32* pmem_sub, const i32* pmem_col, const i32* mpar,
                          const i32* nown, const i64* yoff, const double* Y, const i32* pMout,
                          const i64* poutoff, double* Pout, const i64* wsoff, double* Wsc) {
  if (!nq) return;
  hipLaunchKernelGGL(k_patch_project, dim3(nq), dim3(MSDD_WG), 0, s, ch_ptr, ch_patch, cM, cmoff,
                     Pc, cmem_ptr, cmem_pslot, cmem_ownbase, cmem_m, cmem_col, pmem_ptr,
                     pmem_sub, pmem_col, mpar, nown, yoff, Y, pMout, poutoff, Pout, wsoff, Wsc);
}
void launch_coarse_assemble(hipStream_t s, int nt, const i64* tp_ptr, const i32* tp_patch,
                            const i64* tp_map_off, const i32* tp_map, const i32* pM,
                            const i64* pmoff, const double* Pm, const i32* ng_arr,
                            const i64* aoff, double* Aout) {
  if (!nt) return;
  hipLaunchKernelGGL(k_coarse_assemble, dim3(nt), dim3(MSDD_WG), 0, s, tp_ptr, tp_patch,
                     tp_map_off, tp_map, pM, pmoff, Pm, ng_arr, aoff, Aout);
}
void launch_dense_cholesky(hipStream_t s, int n, double* A, int* status) {
  hipLaunchKernelGGL(k_dense_cholesky, dim3(1), dim3(1024), 0, s, n, A, status);
}
void launch_coarse_gevp(hipStream_t s, int nt, const i32* ng_arr, const i32* no_arr,
                        const i64* aoff, double* Abar, const i64* loff, double* Lo,
                        const i64* soff, double* scratch, double eta, int nev_max,
                        double eps_reg, double* lam_out, const i64* lamoff, int* m_out,
                        int* status, int* rank_out) {
  if (!nt) return;
  hipLaunchKernelGGL(k_coarse_gevp, dim3(nt), dim3(MSDD_WG), 0, s, ng_arr, no_arr, aoff, Abar,
                     loff, Lo, soff, scratch, eta, nev_max, eps_reg, lam_out, lamoff, m_out,
                     status, rank_out);
}
void launch_coarse_collect(hipStream_t s, int nt, const i32* ng_arr, const i32* no_arr,
                           const i64* soff, const double* scratch, const int* m_arr,
                           const i64* yoff, double* Y) {
  if (!nt) return;
  hipLaunchKernelGGL(k_coarse_collect, dim3(nt), dim3(MSDD_WG), 0, s, ng_arr, no_arr, soff,
                     scratch, m_arr, yoff, Y);
}
