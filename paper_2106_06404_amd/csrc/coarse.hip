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
// B = [[A_oo, 0], [0, 0]].  The common kernel is removed by compression: the
// eigenvectors of A + B whose eigenvalue is below eps_reg times the largest are
// dropped (in exact arithmetic exactly ker A cap ker B, the mu = 0 part of the
// paper's regularised transformation), and the definite pencil is solved on
// the rest.
#include "common.h"
#include "symeig.h"
#include "wg_gemm.h"
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
// In-place Cholesky factorisation A = L L^T of one n x n SPD block (column-major,
// leading dimension lda) by the whole workgroup; L is left in the lower triangle, the
// upper triangle is zeroed.  One barrier per column: the trailing update subtracts
// a_rj a_cj / a_jj with the unscaled column, whose scaled copy goes to the upper
// triangle (not touched by the update) and is moved down at the end.  Returns false
// for a non-positive pivot.
__device__ __forceinline__ bool dense_cholesky_block(int n, double* A, int lda, int* fail_sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tr = tid >> 5, tc = tid & 31, ng = nt >> 5;
  if (tid == 0) *fail_sh = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double ajj = A[j + (i64)j * lda];
    if (!(ajj > 0.0)) return false;
    const double il = 1.0 / sqrt(ajj), ia = 1.0 / ajj;
    for (int r = j + 1 + tid; r < n; r += nt) A[j + (i64)r * lda] = A[r + (i64)j * lda] * il;
    for (int r = j + 1 + tr; r < n; r += ng) {
      const double arj = A[r + (i64)j * lda] * ia;
      for (int c = j + 1 + tc; c <= r; c += 32) A[r + (i64)c * lda] -= arj * A[c + (i64)j * lda];
    }
    __syncthreads();
  }
  for (i64 t = tid; t < (i64)n * n; t += nt) {
    const int r = (int)(t % n), c = (int)(t / n);
    if (r > c) A[r + (i64)c * lda] = A[c + (i64)r * lda];
  }
  __syncthreads();
  for (i64 t = tid; t < (i64)n * n; t += nt) {
    const int r = (int)(t % n), c = (int)(t / n);
    if (r < c) A[r + (i64)c * lda] = 0.0;
    if (r == c) A[r + (i64)c * lda] = sqrt(A[r + (i64)c * lda]);
  }
  __syncthreads();
  return true;
}

// One dense SPD block per workgroup (the coarsest level: one block per problem).
__global__ void k_dense_cholesky(const i64* __restrict__ off, const i32* __restrict__ n_arr,
                                 double* __restrict__ A, int* __restrict__ status) {
  __shared__ int f;
  const int t = blockIdx.x;
  const int n = n_arr[t];
  bool ok = n == 0 || dense_cholesky_block(n, A + off[t], n, &f);
  if (threadIdx.x == 0) status[t] = ok ? ST_DONE : ST_NOTSPD;
}

// The same factorisation with the trailing matrix in LDS, packed lower triangle
// (column c at c n - c (c - 1) / 2): the right-looking update a_rc -= a_rj a_cj / a_jj
// reads column j unscaled while its scaled copy goes to the output; one barrier per
// column.  For blocks whose packed triangle fits in LDS (dynamic size n (n + 1) / 2).
__global__ void k_dense_cholesky_lds(const i64* __restrict__ off, const i32* __restrict__ n_arr,
                                     double* __restrict__ A, int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* P = reinterpret_cast<double*>(smem_raw);
  __shared__ int fail;
  const int t = blockIdx.x;
  const int n = n_arr[t];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tr = tid >> 5, tc = tid & 31, ng = nt >> 5;
  double* Ag = A + off[t];
  auto idx = [n](int r, int c) { return c * n - (c * (c - 1)) / 2 + (r - c); };
  if (tid == 0) fail = 0;
  for (int c = 0; c < n; ++c)
    for (int r = c + tid; r < n; r += nt) P[idx(r, c)] = Ag[r + (i64)c * n];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double ajj = P[idx(j, j)];
    if (!(ajj > 0.0)) {
      if (tid == 0) status[t] = ST_NOTSPD;
      return;
    }
    const double il = 1.0 / sqrt(ajj), ia = 1.0 / ajj;
    const double* Pj = P + idx(j, j);  // column j from its diagonal
    for (int r = j + 1 + tid; r < n; r += nt) Ag[r + (i64)j * n] = Pj[r - j] * il;
    for (int c = j + 1 + tc; c < n; c += 32) {
      const double acj = Pj[c - j] * ia;
      double* Pc = P + idx(c, c);
      for (int r = c + tr; r < n; r += ng) Pc[r - c] -= Pj[r - j] * acj;
    }
    __syncthreads();
  }
  for (i64 e = tid; e < (i64)n * n; e += nt) {
    const int r = (int)(e % n), c = (int)(e / n);
    if (r < c) Ag[e] = 0.0;
    if (r == c) Ag[e] = sqrt(P[idx(r, r)]);
  }
  if (tid == 0) status[t] = ST_DONE;
}

// Coarse GEVP of one level-(l-1) subdomain per workgroup, on its generating system
// (owned functions first, no of them; Abar is ng x ng column-major):
//   S = Abar + B with B = D Abar D, D the 0/1 owned mask;
//   S = Q diag(s) Q^T (wg_syev_dc; Q and Y stored transposed); keep s > tau * max(s) (the
//   rest is the numerical kernel of abar and b, their common kernel in exact arithmetic);
//   Qk = Q_keep diag(s_keep)^{-1/2};  C = Qk^T B Qk = Qk_o^T A_oo Qk_o (matrix cores);
//   C = Y diag(mu) Y^T (wg_syev_dc);  lambda = 1/mu - 1;  select lambda < eta;
//   x = Qk y / sqrt(mu) (b-normalised); the coarse basis block is x on the owned rows.
// The owned block A_oo is the level's Dirichlet matrix; its Cholesky factor is kept.
// Scratch layout per target (doubles): S ng^2 | Q ng^2 | Qk ng^2 | C ng^2 | Yc ng^2 | ints ng.
__global__ void k_coarse_gevp(const i32* __restrict__ ng_arr, const i32* __restrict__ no_arr,
                              const i64* __restrict__ aoff, double* __restrict__ Abar,
                              const i64* __restrict__ loff, double* __restrict__ Lo,
                              const i64* __restrict__ soff, double* __restrict__ scratch,
                              double eta, int nev_max, double tau,
                              double* __restrict__ lam_out, const i64* __restrict__ lamoff,
                              int* __restrict__ m_out, int* __restrict__ status,
                              int* __restrict__ rank_out, int* __restrict__ sweeps_out,
                              int ng_max, int in_lds, int vec_in_lds) {
  const int t = blockIdx.x;
  const int ng = ng_arr[t], no = no_arr[t];
  const double* A = Abar + aoff[t];
  double* L = Lo + loff[t];
  const i64 g2 = (i64)ng * ng;
  double* S = scratch + soff[t];
  double* Q = S + g2;
  double* Qk = Q + g2;
  double* C = Qk + g2;
  double* Yc = C + g2;
  int* keep = reinterpret_cast<int*>(Yc + g2);
  __shared__ int sh_fail, sh_r, sh_m, sh_bad;
  __shared__ double sh_smax, red[64];
  // dynamic LDS: eigenvalues d (ng_max), workspace (syev_dc_ws), then (in_lds) the matrix
  // being diagonalised, later the tridiagonal problem's eigenvectors.  Generating systems
  // too large for that (vec_in_lds = 0) keep d and the workspace in the target's scratch,
  // after its matrices (the kernels address them through generic pointers, and their
  // barriers order the global accesses within the workgroup).
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* d = vec_in_lds ? reinterpret_cast<double*>(smem_raw) : S + 5 * g2 + ng + 2;
  double* wsp = d + (vec_in_lds ? ng_max : ng);
  double* Alds = wsp + syev_dc_ws(ng_max);
  const int tid = threadIdx.x, nt = blockDim.x;
  if (no == 0) {
    if (tid == 0) {
      m_out[t] = 0;
      status[t] = ST_DONE;
      rank_out[t] = 0;
      for (int q = 0; q < 4; ++q) sweeps_out[4 * t + q] = 0;
    }
    return;
  }
  double* Sx = in_lds ? Alds : S;  // S, then C, live in LDS when they fit
  double* Cx = in_lds ? Alds : C;
  // S (row-major, symmetric)
  for (i64 e = tid; e < g2; e += nt) {
    const int r = (int)(e / ng), c = (int)(e % ng);
    const double a = 0.5 * (A[r + (i64)c * ng] + A[c + (i64)r * ng]);
    Sx[e] = (r < no && c < no) ? 2.0 * a : a;
  }
  __syncthreads();
  // S = Q diag(d) Q^T (Q transposed in global memory); separate calls so that the LDS
  // case is compiled with LDS accesses
  if (in_lds)
    wg_syev_dc(ng, Alds, Q, C, Yc, d, wsp, red);
  else
    wg_syev_dc(ng, S, Q, C, Yc, d, wsp, red);
  if (tid == 0) {
    double smax = 0.0;
    int bad = 0;
    for (int a = 0; a < ng; ++a) {
      smax = fmax(smax, d[a]);
      bad |= !isfinite(d[a]);
    }
    int r = 0;
    for (int a = 0; a < ng; ++a)
      if (d[a] > tau * smax) keep[r++] = a;
    sh_smax = smax;
    sh_r = r;
    sh_bad = bad;
  }
  __syncthreads();
  const int r = sh_r;
  // Qk (ng x r, row-major): kept eigenvectors scaled by s^{-1/2}
  for (i64 e = tid; e < (i64)ng * r; e += nt) {
    const int row = (int)(e / r), k = (int)(e % r);
    const int a = keep[k];
    Qk[e] = Q[(i64)a * ng + row] / sqrt(d[a]);  // Q stored transposed
  }
  __syncthreads();
  // C = Qk_o^T A_oo Qk_o on the matrix cores: first Q <- A_oo Qk_o (no x r), then C
  // (r x r, row-major), made exactly symmetric
  const int wave = tid >> 6, nwv = nt >> 6;
  {
    const int tnr = (r + 15) / 16, tmo = (no + 15) / 16;
    wave_gemm_tiles(
        no, r, no, tnr, wave, tmo * tnr, nwv,
        [&](int row, int q) { return 0.5 * (A[row + (i64)q * ng] + A[q + (i64)row * ng]); },
        [&](int q, int k) { return Qk[(i64)q * r + k]; },
        [&](int row, int k, double v) { Q[(i64)row * r + k] = v; });
    __syncthreads();
    wave_gemm_tiles(
        r, r, no, tnr, wave, tnr * tnr, nwv, [&](int a, int q) { return Qk[(i64)q * r + a]; },
        [&](int q, int b) { return Q[(i64)q * r + b]; },
        [&](int a, int b, double v) { Cx[(i64)a * r + b] = v; });
    __syncthreads();
    for (i64 e = tid; e < (i64)r * r; e += nt) {
      const int a = (int)(e / r), b = (int)(e % r);
      if (a < b) {
        const double v = 0.5 * (Cx[(i64)a * r + b] + Cx[(i64)b * r + a]);
        Cx[(i64)a * r + b] = v;
        Cx[(i64)b * r + a] = v;
      }
    }
  }
  __syncthreads();
  // C = Y diag(mu) Y^T (Y transposed in Yc); mu in d
  if (in_lds)
    wg_syev_dc(r, Alds, Yc, S, Q, d, wsp, red);
  else
    wg_syev_dc(r, C, Yc, S, Q, d, wsp, red);
  if (tid == 0) {
    sweeps_out[4 * t] = 0;
    sweeps_out[4 * t + 1] = 0;
    sweeps_out[4 * t + 2] = ng;
    sweeps_out[4 * t + 3] = r;
  }
  // mu descending (the eigensolver returns them ascending), lambda = 1/mu - 1 ascending
  double* lam = lam_out + lamoff[t];
  int* ord = keep;  // reused (r entries)
  if (tid == 0) {
    int bad = sh_bad;
    for (int a = 0; a < r; ++a) {
      ord[a] = r - 1 - a;
      bad |= !isfinite(d[a]);
    }
    sh_bad = bad;
    int m = 0, nl = 0;
    for (int a = 0; a < r && nl < no; ++a) {
      const double mu = d[ord[a]];
      if (mu <= 1e-12) break;
      const double lv = fmax(1.0 / mu - 1.0, 0.0);
      lam[nl++] = lv;
      if (lv < eta) ++m;
    }
    for (int a = nl; a < no; ++a) lam[a] = INFINITY;
    if (nev_max > 0 && m > nev_max) m = nev_max;
    sh_m = m;
    m_out[t] = m;
    rank_out[t] = r;
  }
  __syncthreads();
  const int m = sh_m;
  // selected b-normalised eigenvectors, owned rows: Xo[row, c] = (Qk_o y_c)[row] / sqrt(mu_c)
  double* Xo = S;  // reuse S as no x m column-major output
  wave_gemm_tiles(
      no, m, r, (m + 15) / 16, wave, ((no + 15) / 16) * ((m + 15) / 16), nwv,
      [&](int row, int k) { return Qk[(i64)row * r + k]; },
      [&](int k, int c) { return Yc[(i64)ord[c] * r + k]; },  // Yc transposed
      [&](int row, int c, double v) { Xo[row + (i64)c * no] = v / sqrt(d[ord[c]]); });
  // Dirichlet factor of the owned block (in LDS when the generating system was there)
  double* Lw = in_lds ? Alds : L;
  for (i64 e = tid; e < (i64)no * no; e += nt) {
    const int rr = (int)(e % no), cc = (int)(e / no);
    Lw[e] = 0.5 * (A[rr + (i64)cc * ng] + A[cc + (i64)rr * ng]);
  }
  __syncthreads();
  const bool spd = in_lds ? dense_cholesky_block(no, Alds, no, &sh_fail)
                          : dense_cholesky_block(no, L, no, &sh_fail);
  if (!spd) {
    if (tid == 0) status[t] = ST_NOTSPD;
    return;
  }
  if (in_lds) {
    for (i64 e = tid; e < (i64)no * no; e += nt) L[e] = Alds[e];
  }
  if (tid == 0) status[t] = sh_bad ? ST_NOCONV : ST_DONE;
}

// Dense lower factor (column-major, n x n) -> the row and column band layouts with
// b = n-1 used by the blocked wavefront solves: R[j*n+d] = L(j,j-d), C[j*n+d] = L(j+d,j).
__global__ void k_dense_to_layouts(const i64* __restrict__ off, const i32* __restrict__ n_arr,
                                   const double* __restrict__ L, double* __restrict__ R,
                                   double* __restrict__ C) {
  const int t = blockIdx.x;
  const int n = n_arr[t];
  const double* Lt = L + off[t];
  double* Rt = R + off[t];
  double* Ct = C + off[t];
  for (i64 e = threadIdx.x; e < (i64)n * n; e += blockDim.x) {
    const int j = (int)(e / n), d = (int)(e % n);
    Rt[e] = (d <= j) ? Lt[j + (i64)(j - d) * n] : 0.0;
    Ct[e] = (j + d < n) ? Lt[(j + d) + (i64)j * n] : 0.0;
  }
}

// Explicit inverse of SPD blocks from their Cholesky factors (coarse levels and A_0):
// the apply then costs one parallel matrix-vector product instead of two
// sequential triangular sweeps.  Step 1: Linv = L^{-1} (one thread per column,
// forward substitution); step 2: Inv = Linv^T Linv (one thread per entry).
// grid: (ceil(nmax / 256), targets); L, Linv, Inv column-major n x n at off[t].
// Inverse of a lower triangular block (column-major, n x n), one wavefront per column:
// L x = e_c by column-oriented forward substitution, x held in registers (lane l owns
// rows l, l + 64, ...); each step finishes x_q and subtracts L(r, q) x_q from the rows
// below it, the same operations in the same order as a row-oriented substitution.
template <int NR>
__global__ void __launch_bounds__(64) k_tri_inverse(const i64* __restrict__ off,
                                                    const i32* __restrict__ n_arr,
                                                    const double* __restrict__ L,
                                                    double* __restrict__ Linv) {
  const int t = blockIdx.y;
  const int n = n_arr[t];
  const int c = blockIdx.x;
  if (c >= n) return;
  const double* Lt = L + off[t];
  double* X = Linv + off[t];
  const int lane = threadIdx.x;
  double x[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) x[k] = (lane + 64 * k == c) ? 1.0 : 0.0;
  for (int q = c; q < n; ++q) {
    const double* Lq = Lt + (i64)q * n;  // column q
    const int kq = q >> 6;
    double xq = 0.0;
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k == kq) xq = x[k];
    xq = __shfl(xq, q & 63) / Lq[q];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int r = lane + 64 * k;
      if (r == q)
        x[k] = xq;
      else if (r > q && r < n)
        x[k] -= Lq[r] * xq;
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int r = lane + 64 * k;
    if (r < n) X[r + (i64)c * n] = r >= c ? x[k] : 0.0;
  }
}

// Larger blocks (up to 8192): one thread per column, row-oriented substitution.
__global__ void k_tri_inverse_rows(const i64* __restrict__ off, const i32* __restrict__ n_arr,
                                   const double* __restrict__ L, double* __restrict__ Linv) {
  const int t = blockIdx.y;
  const int n = n_arr[t];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double* Lt = L + off[t];
  double* X = Linv + off[t];
  for (int r = 0; r < c; ++r) X[r + (i64)c * n] = 0.0;
  for (int r = c; r < n; ++r) {
    double v = (r == c) ? 1.0 : 0.0;
    for (int q = c; q < r; ++q) v -= Lt[r + (i64)q * n] * X[q + (i64)c * n];
    X[r + (i64)c * n] = v / Lt[r + (i64)r * n];
  }
}

__global__ void k_gram_lower(const i64* __restrict__ off, const i32* __restrict__ n_arr,
                             const double* __restrict__ Linv, double* __restrict__ Inv) {
  const int t = blockIdx.y;
  const int n = n_arr[t];
  const i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (i64)n * n) return;
  const int a = (int)(e % n), b = (int)(e / n);
  const double* X = Linv + off[t];
  const int r0 = a > b ? a : b;
  double acc = 0.0;
  for (int r = r0; r < n; ++r) acc += X[r + (i64)a * n] * X[r + (i64)b * n];
  Inv[off[t] + e] = acc;
}

// Copy the selected eigenvectors (left at the start of the scratch) to the pooled basis,
// fixing signs (largest-magnitude owned entry positive).
__global__ void k_coarse_collect(const i32* __restrict__ ng_arr, const i32* __restrict__ no_arr,
                                 const i64* __restrict__ soff, const double* __restrict__ scratch,
                                 const int* __restrict__ m_arr, const i64* __restrict__ yoff,
                                 double* __restrict__ Y) {
  const int t = blockIdx.x;
  const int no = no_arr[t];
  const int m = m_arr[t];
  const double* Z = scratch + soff[t];
  double* Yt = Y + yoff[t];
  __shared__ double sgn;
  for (int c = 0; c < m; ++c) {
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
  (void)ng_arr;
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
void launch_dense_cholesky(hipStream_t s, int nt, int nmax, const i64* off, const i32* n_arr,
                           double* A, int* status) {
  if (nt == 0) return;
  const size_t lds = (size_t)nmax * (nmax + 1) / 2 * sizeof(double);
  if (lds <= 150 * 1024) {
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)k_dense_cholesky_lds,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_dense_cholesky_lds, dim3(nt), dim3(1024), lds, s, off, n_arr, A, status);
  } else {
    hipLaunchKernelGGL(k_dense_cholesky, dim3(nt), dim3(1024), 0, s, off, n_arr, A, status);
  }
}
int64_t coarse_gevp_vec_doubles(int ng) { return (int64_t)ng + syev_dc_ws(ng); }

void launch_coarse_gevp(hipStream_t s, int nt, const i32* ng_arr, const i32* no_arr,
                        const i64* aoff, double* Abar, const i64* loff, double* Lo,
                        const i64* soff, double* scratch, double eta, int nev_max,
                        double eps_reg, double* lam_out, const i64* lamoff, int* m_out,
                        int* status, int* rank_out, int* sweeps_out, int ng_max) {
  if (!nt) return;
  const size_t vecs = ((size_t)ng_max + syev_dc_ws(ng_max)) * sizeof(double);
  const size_t full = vecs + (size_t)ng_max * ng_max * sizeof(double);
  hipFuncAttributes fa;
  size_t stat = 4096;
  if (hipFuncGetAttributes(&fa, (const void*)k_coarse_gevp) == hipSuccess) stat = fa.sharedSizeBytes;
  const int in_lds = full + stat <= 160 * 1024;  // LDS per workgroup, with the static part
  const int vec_in_lds = vecs + stat <= 160 * 1024;
  const size_t lds = in_lds ? full : vec_in_lds ? vecs : 0;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_coarse_gevp,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_coarse_gevp, dim3(nt), dim3(1024), lds, s, ng_arr, no_arr, aoff, Abar,
                     loff, Lo, soff, scratch, eta, nev_max, eps_reg, lam_out, lamoff, m_out,
                     status, rank_out, sweeps_out, ng_max, in_lds, vec_in_lds);
}
void launch_dense_to_layouts(hipStream_t s, int nt, const i64* off, const i32* n_arr,
                             const double* L, double* R, double* C) {
  if (!nt) return;
  hipLaunchKernelGGL(k_dense_to_layouts, dim3(nt), dim3(MSDD_WG), 0, s, off, n_arr, L, R, C);
}
void launch_spd_inverse(hipStream_t s, int nt, int nmax, const i64* off, const i32* n_arr,
                        const double* L, double* Linv, double* Inv) {
  if (!nt || nmax <= 0) return;
  // one wavefront per column, rows in registers, up to 1024 x 1024 blocks
  if (nmax <= 256)
    hipLaunchKernelGGL(k_tri_inverse<4>, dim3(nmax, nt), dim3(64), 0, s, off, n_arr, L, Linv);
  else if (nmax <= 1024)
    hipLaunchKernelGGL(k_tri_inverse<16>, dim3(nmax, nt), dim3(64), 0, s, off, n_arr, L, Linv);
  else
    hipLaunchKernelGGL(k_tri_inverse_rows, dim3((nmax + 255) / 256, nt), dim3(256), 0, s, off,
                       n_arr, L, Linv);
  const i64 nn = (i64)nmax * nmax;
  hipLaunchKernelGGL(k_gram_lower, dim3((unsigned)((nn + 255) / 256), nt), dim3(256), 0, s, off,
                     n_arr, Linv, Inv);
}
void launch_coarse_collect(hipStream_t s, int nt, const i32* ng_arr, const i32* no_arr,
                           const i64* soff, const double* scratch, const int* m_arr,
                           const i64* yoff, double* Y) {
  if (!nt) return;
  hipLaunchKernelGGL(k_coarse_collect, dim3(nt), dim3(MSDD_WG), 0, s, ng_arr, no_arr, soff,
                     scratch, m_arr, yoff, Y);
}
