// Finest-level local matrices in lower-band storage and their factorisation.
//
// Layout (per subdomain, half-bandwidth b, order n):
//   column-major lower band  Bc[j*(b+1) + d] = A(j+d, j),  0 <= d <= b
//   row layout of a factor   Lr[j*(b+1) + d] = L(j, j-d)
// Padding entries (j+d >= n, or j-d < 0) are zero.
//
// Paper: the local Neumann matrix abar_{l,i} is the sum of the element
// matrices a_tau over the subdomain's elements (Sec. 3.4); the Dirichlet
// matrix is A_i = R_i A R_i^T (Sec. 2.1); the shifted pencil matrix
// abar + sigma*b, b = D abar D (Sec. 3.3 lemma, b^1 of Sec. 3.4) is SPD.
#include "common.h"
#include <algorithm>
#include "kernels.h"
#include "trsv.h"

// ---------------------------------------------------------------------------
// abar_i = sum_{tau in T_i} a_tau, gathered row by row: the thread that owns
// local row r adds every element contribution (r, c), c <= r, in the fixed
// order of r's incidence list, so the result is deterministic without atomics.
// The same pass fills the symmetric ELL copy (full rows) used by b = D abar D, and, when
// elem_ov is given, the band and ELL copies of the overlap elements' sum (the matrix of the
// b^2 right-hand side, Sec. 3.4) in band2 / ell_val2.
// ---------------------------------------------------------------------------
__global__ void k_neumann_assemble(i64 total_rows, const i32* __restrict__ row_sub,
                                   const i64* __restrict__ voff, const i32* __restrict__ bw,
                                   const i64* __restrict__ boff, const i64* __restrict__ inc_ptr,
                                   const i32* __restrict__ inc_slot, const i32* __restrict__ inc_a,
                                   const i32* __restrict__ slot_elem, const i32* __restrict__ slot_loc,
                                   int k, const double* __restrict__ elem_mat,
                                   double* __restrict__ band, int ell_w,
                                   const i32* __restrict__ ell_col, double* __restrict__ ell_val,
                                   int* __restrict__ status, const i32* __restrict__ elem_ov,
                                   double* __restrict__ band2, double* __restrict__ ell_val2) {
  i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int i = row_sub[g];
  const int r = (int)(g - voff[i]);
  const int b = bw[i];
  double* B = band + boff[i];
  double* B2 = band2 ? band2 + boff[i] : nullptr;
  const i32* ec = ell_col + g * ell_w;
  double* ev = ell_val + g * ell_w;
  double* ev2 = ell_val2 ? ell_val2 + g * ell_w : nullptr;
  for (i64 q = inc_ptr[g]; q < inc_ptr[g + 1]; ++q) {
    const i64 slot = inc_slot[q];
    const int a = inc_a[q];
    const int e = slot_elem[slot];
    const bool ov = elem_ov && elem_ov[e];  // an overlap element (also in the b^2 sum)
    const double* Krow = elem_mat + (i64)e * k * k + (i64)a * k;
    const i32* loc = slot_loc + slot * k;
    for (int bb = 0; bb < k; ++bb) {
      const int c = loc[bb];
      if (c < 0) continue;
      const double v = Krow[bb];
      if (!(v == v)) status[i] = ST_BADINPUT;
      if (c <= r) {
        if (r - c > b) {
          status[i] = ST_BADINPUT;
        } else {
          B[(i64)c * (b + 1) + (r - c)] += v;
          if (ov) B2[(i64)c * (b + 1) + (r - c)] += v;
        }
      }
      int t = 0;
      while (t < ell_w && ec[t] != c) ++t;
      if (t < ell_w) {
        ev[t] += v;
        if (ov) ev2[t] += v;
      } else {
        status[i] = ST_BADINPUT;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// A_i = R_i A R_i^T from the global CSR matrix: the thread of Dirichlet row r
// walks CSR row dglob[r] and finds each column among the subdomain's sorted
// Dirichlet dofs by binary search.
// ---------------------------------------------------------------------------
__global__ void k_dirichlet_extract(i64 total_rows, const i32* __restrict__ drow_sub,
                                    const i64* __restrict__ doff, const i32* __restrict__ nd,
                                    const i32* __restrict__ bd, const i64* __restrict__ dboff,
                                    const i32* __restrict__ dglob, const i64* __restrict__ rowptr,
                                    const i32* __restrict__ col, const double* __restrict__ val,
                                    double* __restrict__ band, int* __restrict__ status) {
  i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int i = drow_sub[g];
  const int r = (int)(g - doff[i]);
  const int b = bd[i];
  const i32* list = dglob + doff[i];
  const int len = nd[i];
  double* B = band + dboff[i];
  const int p = dglob[g];
  for (i64 e = rowptr[p]; e < rowptr[p + 1]; ++e) {
    const int q = col[e];
    int lo = 0, hi = len - 1, c = -1;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      int v = list[mid];
      if (v == q) { c = mid; break; }
      if (v < q) lo = mid + 1; else hi = mid - 1;
    }
    if (c < 0 || c > r) continue;
    const double v = val[e];
    if (!(v == v)) status[i] = ST_BADINPUT;
    if (r - c > b) status[i] = ST_BADINPUT;
    else B[(i64)c * (b + 1) + (r - c)] = v;
  }
}

// ---------------------------------------------------------------------------
// Band Cholesky with a sliding (b+1) x (b+1) window in LDS, one workgroup per
// subdomain.  Column c of the active window lives in slot c mod (b+1).  The
// matrix factorised is S = A + sigma * D A D (D = diag(dv)), formed while each
// column enters the window; sigma = 0 / dv = nullptr factorises A itself.
// Writes L in both column (Lc) and row (Lr) band layouts.
// ---------------------------------------------------------------------------
constexpr int CHOL_RB = 32;    // columns per batch of global loads / stores
constexpr int CHOL_MAXI = 8;   // trailing-update items per thread kept in registers

template <typename T>
__global__ void k_band_cholesky(const i32* __restrict__ subs, const i32* __restrict__ n_arr,
                                const i32* __restrict__ b_arr, const i64* __restrict__ src_off,
                                const double* __restrict__ src, const i64* __restrict__ dv_off,
                                const double* __restrict__ dv, double sigma,
                                const i64* __restrict__ dst_off, T* __restrict__ Lc,
                                T* __restrict__ Lr, int* __restrict__ status,
                                const double* __restrict__ src2) {
  // The (b+1) x (b+1) active window lives in LDS (column c in slot c mod (b+1)).  Global
  // traffic is batched: the next CHOL_RB input columns are loaded into an LDS ring once
  // every CHOL_RB steps and the factor columns are staged in a second ring and written
  // out every CHOL_RB steps, so the two barriers of a step wait on LDS work only (a
  // barrier also waits for the wavefront's outstanding global loads and stores).
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  const int n = n_arr[i];
  const int b = b_arr[i];
  const int w = b + 1;
  T* W = reinterpret_cast<T*>(smem_raw);   // w*w
  T* lcol = W + (size_t)w * w;             // w
  T* ain = lcol + w;                       // CHOL_RB*w  upcoming input columns
  T* lout = ain + (size_t)CHOL_RB * w;     // CHOL_RB*w  factor columns not yet written
  const double* A = src + src_off[i];
  const double* A2 = src2 ? src2 + src_off[i] : nullptr;
  const double* d = dv ? dv + dv_off[i] : nullptr;
  T* Lci = Lc + dst_off[i];
  T* Lri = Lr + dst_off[i];
  auto in_val = [&](int c, int t) -> T {
    double a = A[(i64)c * w + t];
    if (d) a = A2 ? a + sigma * d[c + t] * d[c] * A2[(i64)c * w + t] : a * (1.0 + sigma * d[c + t] * d[c]);
    return (T)a;
  };
  for (int c = 0; c < w && c < n; ++c)
    for (int t = threadIdx.x; t < w; t += blockDim.x) W[c * w + t] = (c + t < n) ? in_val(c, t) : (T)0;
  int flushed = 0;  // columns < flushed are written to Lc / Lr
  auto flush = [&](int upto) {  // write staged columns [flushed, upto)
    const int cnt = upto - flushed;
    for (int e = threadIdx.x; e < cnt * w; e += blockDim.x) {
      const int jj = flushed + e / w, t = e % w;
      const T l = lout[(jj % CHOL_RB) * w + t];
      Lci[(i64)jj * w + t] = l;
      if (jj + t < n) Lri[(i64)(jj + t) * w + t] = l;
    }
    flushed = upto;
  };
  // this thread's items (p, q), 1 <= q <= p <= b, of the lower triangle, enumerated once
  // (row-wise index t = p (p - 1) / 2 + q - 1) when they fit in registers
  const int nitems = b * (b + 1) / 2;
  const bool fast = nitems <= CHOL_MAXI * (int)blockDim.x;
  int ip[CHOL_MAXI], iq[CHOL_MAXI], ni = 0;
  if (fast)
    for (int t = threadIdx.x; t < nitems; t += blockDim.x) {
      int p = (int)((1.0 + sqrt(1.0 + 8.0 * t)) * 0.5);
      while (p * (p - 1) / 2 > t) --p;
      while ((p + 1) * p / 2 <= t) ++p;
      ip[ni] = p;
      iq[ni] = t - p * (p - 1) / 2 + 1;
      ++ni;
    }
  bool failed = false;
  int slot = 0;
  for (int j = 0; j < n; ++j, slot = (slot + 1 == w) ? 0 : slot + 1) {
    if (j % CHOL_RB == 0) {
      // factor columns of the previous batch out, input columns j+w .. j+w+RB-1 in (after
      // every thread has consumed the previous batch's last input column)
      if (j > 0) lds_barrier();
      flush(j);
      for (int e = threadIdx.x; e < CHOL_RB * w; e += blockDim.x) {
        const int c = j + w + e / w, t = e % w;
        ain[e] = (c < n && c + t < n) ? in_val(c, t) : (T)0;
      }
    }
    lds_barrier();  // the window, factor column and rings are in LDS
    const T ajj = W[slot * w];
    if (!(ajj > (T)0)) {
      if (threadIdx.x == 0) status[i] = ST_NOTSPD;
      failed = true;
      break;
    }
    const T ljj = sqrt(ajj);
    const T rl = (T)1 / ljj;
    for (int t = threadIdx.x; t < w; t += blockDim.x) {
      T l = 0;
      if (j + t < n) l = (t == 0) ? ljj : W[slot * w + t] * rl;
      lcol[t] = l;
      lout[(j % CHOL_RB) * w + t] = l;
    }
    lds_barrier();
    // trailing update of the window: A(j+p, j+q) -= L(j+p, j) L(j+q, j), 1 <= q <= p <= b
    if (fast) {
#pragma unroll
      for (int u = 0; u < CHOL_MAXI; ++u) {
        if (u >= ni) break;
        const int pp = ip[u], qq = iq[u];
        if (j + pp < n) {
          int sl = slot + qq;
          if (sl >= w) sl -= w;
          W[sl * w + (pp - qq)] -= lcol[pp] * lcol[qq];
        }
      }
    } else {
      for (int t = threadIdx.x; t < b * b; t += blockDim.x) {
        const int p = t / b + 1, q = t % b + 1;
        if (q <= p && j + p < n) W[((j + q) % w) * w + (p - q)] -= lcol[p] * lcol[q];
      }
    }
    if (j + w < n)
      for (int t = threadIdx.x; t < w; t += blockDim.x) W[slot * w + t] = ain[(j % CHOL_RB) * w + t];
  }
  if (!failed) {
    __syncthreads();
    flush(n);
  }
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// ---------------------------------------------------------------------------
// Sylvester inertia of M = A + sigma * D A D (with sigma = -eta: abar - eta b), one
// workgroup per subdomain: the number of negative pivots of its LDL^T factorisation
// without pivoting, which equals the number of eigenvalues of abar x = lambda b x below
// eta (congruence; the eigenvalues of b's kernel are infinite).  Same sliding window as
// k_band_cholesky, with the column scaled by 1/sqrt|pivot| and the trailing update signed.
// A pivot at or below 1e-13 times the column's original diagonal makes the count unreliable
// (rounding could flip its sign): neg[i] = -1 then, else the count.  Nothing is stored.
// ---------------------------------------------------------------------------
__global__ void k_band_inertia(const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
                               const i64* __restrict__ src_off, const double* __restrict__ src,
                               const i64* __restrict__ dv_off, const double* __restrict__ dv,
                               double sigma, int* __restrict__ neg,
                               const double* __restrict__ src2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x;
  const int n = n_arr[i];
  const int b = b_arr[i];
  const int w = b + 1;
  double* W = reinterpret_cast<double*>(smem_raw);  // w*w
  double* lcol = W + (size_t)w * w;                 // w
  double* ain = lcol + w;                           // CHOL_RB*w  upcoming input columns
  double* dgi = ain + (size_t)CHOL_RB * w;          // CHOL_RB    original diagonals
  const double* A = src + src_off[i];
  const double* d = dv + dv_off[i];
  const double* A2 = src2 ? src2 + src_off[i] : nullptr;
  auto in_val = [&](int c, int t) -> double {
    const double a = A[(i64)c * w + t];
    return A2 ? a + sigma * d[c + t] * d[c] * A2[(i64)c * w + t] : a * (1.0 + sigma * d[c + t] * d[c]);
  };
  for (int c = 0; c < w && c < n; ++c)
    for (int t = threadIdx.x; t < w; t += blockDim.x) W[c * w + t] = (c + t < n) ? in_val(c, t) : 0.0;
  // this thread's items (p, q), 1 <= q <= p <= b, of the trailing triangle (as in
  // k_band_cholesky)
  const int nitems = b * (b + 1) / 2;
  const bool fast = nitems <= CHOL_MAXI * (int)blockDim.x;
  int ip[CHOL_MAXI], iq[CHOL_MAXI], ni = 0;
  if (fast)
    for (int t = threadIdx.x; t < nitems; t += blockDim.x) {
      int p = (int)((1.0 + sqrt(1.0 + 8.0 * t)) * 0.5);
      while (p * (p - 1) / 2 > t) --p;
      while ((p + 1) * p / 2 <= t) ++p;
      ip[ni] = p;
      iq[ni] = t - p * (p - 1) / 2 + 1;
      ++ni;
    }
  int count = 0;
  bool unreliable = false;
  int slot = 0;
  for (int j = 0; j < n; ++j, slot = (slot + 1 == w) ? 0 : slot + 1) {
    if (j % CHOL_RB == 0) {
      if (j > 0) lds_barrier();
      for (int e = threadIdx.x; e < CHOL_RB * w; e += blockDim.x) {
        const int c = j + w + e / w, t = e % w;
        ain[e] = (c < n && c + t < n) ? in_val(c, t) : 0.0;
      }
      for (int t = threadIdx.x; t < CHOL_RB; t += blockDim.x) dgi[t] = (j + t < n) ? in_val(j + t, 0) : 0.0;
    }
    lds_barrier();
    const double ajj = W[slot * w];
    if (!(fabs(ajj) > 1e-13 * fabs(dgi[j % CHOL_RB]))) {
      unreliable = true;
      break;
    }
    if (ajj < 0.0) ++count;
    const double sg = ajj < 0.0 ? -1.0 : 1.0;
    const double rl = 1.0 / sqrt(fabs(ajj));
    for (int t = threadIdx.x; t < w; t += blockDim.x) lcol[t] = (j + t < n && t > 0) ? W[slot * w + t] * rl : 0.0;
    lds_barrier();
    if (fast) {
#pragma unroll
      for (int u = 0; u < CHOL_MAXI; ++u) {
        if (u >= ni) break;
        const int pp = ip[u], qq = iq[u];
        if (j + pp < n) {
          int sl = slot + qq;
          if (sl >= w) sl -= w;
          W[sl * w + (pp - qq)] -= sg * lcol[pp] * lcol[qq];
        }
      }
    } else {
      for (int t = threadIdx.x; t < b * b; t += blockDim.x) {
        const int p = t / b + 1, q = t % b + 1;
        if (q <= p && j + p < n) W[((slot + q) % w) * w + (p - q)] -= sg * lcol[p] * lcol[q];
      }
    }
    if (j + w < n)
      for (int t = threadIdx.x; t < w; t += blockDim.x) W[slot * w + t] = ain[(j % CHOL_RB) * w + t];
  }
  if (threadIdx.x == 0) neg[i] = unreliable ? -1 : count;
}

// Inertia counts of every subdomain (k_band_inertia); subdomains whose window does not fit
// in LDS get -1 (no count).
void launch_band_inertia(hipStream_t s, int nsubs, int bmax, const i32* n_arr, const i32* b_arr,
                         const i64* src_off, const double* src, const i64* dv_off,
                         const double* dv, double sigma, int* neg, const double* src2) {
  if (nsubs == 0) return;
  const size_t w = (size_t)bmax + 1;
  const size_t lds = (w * w + w + CHOL_RB * w + CHOL_RB) * sizeof(double);
  if (lds > 160 * 1024) {
    hipLaunchKernelGGL(k_fill_int, dim3((nsubs + 255) / 256), dim3(256), 0, s, neg, nsubs, -1);
    return;
  }
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_band_inertia,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_band_inertia, dim3(nsubs), dim3(MSDD_WG), lds, s, n_arr, b_arr, src_off, src,
                     dv_off, dv, sigma, neg, src2);
}

// ---------------------------------------------------------------------------
// Same factorisation for half-bandwidths whose window does not fit in LDS: S is first
// written to Lc (lower band, column layout) and factorised in place, right-looking, in
// panels of CHB_P columns.  A panel (its columns' band entries, zero-padded) is factorised
// in LDS; the trailing window it touches (columns j0+p .. j0+p+b-1, rows up to j0+p-1+b)
// is then updated once by the rank-p product, each thread owning 4 x 4 tiles of the window
// with the panel rows in registers, so the window is read and written once per panel
// instead of once per column.
// ---------------------------------------------------------------------------
constexpr int CHB_P = 16;  // panel width

template <typename T>
__global__ void __launch_bounds__(MSDD_WG) k_band_cholesky_blocked(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ src_off, const double* __restrict__ src,
    const i64* __restrict__ dv_off, const double* __restrict__ dv, double sigma,
    const i64* __restrict__ dst_off, T* __restrict__ Lc, T* __restrict__ Lr,
    int* __restrict__ status, const double* __restrict__ src2, int pw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Pn = reinterpret_cast<T*>(smem_raw);  // CHB_P x pw: column c of the panel, offsets d
  __shared__ int bad;
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  const int n = n_arr[i];
  const int b = b_arr[i];
  const int w = b + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* A = src + src_off[i];
  const double* d = dv ? dv + dv_off[i] : nullptr;
  T* Li = Lc + dst_off[i];
  T* Ri = Lr + dst_off[i];
  for (i64 t = tid; t < (i64)n * w; t += nt) {
    const int c = (int)(t / w), dd = (int)(t % w);
    double a = 0.0;
    if (c + dd < n) {
      a = A[t];
      if (d) a = src2 ? a + sigma * d[c + dd] * d[c] * src2[src_off[i] + t] : a * (1.0 + sigma * d[c + dd] * d[c]);
    }
    Li[t] = (T)a;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  const int tb = (b + 3) / 4;  // 4 x 4 tiles per window side
  for (int j0 = 0; j0 < n; j0 += CHB_P) {
    const int pc = min(CHB_P, n - j0);
    // panel: Pn[c * pw + dd] = entry (j0 + c + dd, j0 + c), zero outside the band/matrix
    for (int t = tid; t < CHB_P * pw; t += nt) {
      const int c = t / pw, dd = t % pw;
      Pn[t] = (c < pc && dd < w && j0 + c + dd < n) ? Li[(i64)(j0 + c) * w + dd] : (T)0;
    }
    __syncthreads();
    for (int c = 0; c < pc; ++c) {
      const T ajj = Pn[c * pw];
      if (!(ajj > (T)0)) {
        if (tid == 0) bad = 1;
        break;
      }
      const T ljj = sqrt(ajj);
      __syncthreads();
      for (int dd = tid; dd < w; dd += nt) Pn[c * pw + dd] = dd == 0 ? ljj : Pn[c * pw + dd] / ljj;
      __syncthreads();
      // columns c2 > c of the panel: entry (j0+c2+d2, j0+c2) -= L(j0+c2+d2, j0+c) L(j0+c2, j0+c)
      for (int t = tid; t < (pc - 1 - c) * w; t += nt) {
        const int c2 = c + 1 + t / w, d2 = t % w;
        const int o = c2 - c + d2;  // offset of row j0+c2+d2 in column j0+c
        if (o <= b) Pn[c2 * pw + d2] -= Pn[c * pw + o] * Pn[c * pw + (c2 - c)];
      }
      __syncthreads();
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) status[i] = ST_NOTSPD;
      return;
    }
    for (int t = tid; t < pc * w; t += nt) {
      const int c = t / w, dd = t % w;
      if (j0 + c + dd < n) Li[(i64)(j0 + c) * w + dd] = Pn[c * pw + dd];
    }
    // trailing window: column k = kb + kk, row r = kb + rr, 0 <= kk <= rr < b, where
    // kb = j0 + pc; L(x, j0+c) = Pn[c * pw + (x - j0 - c)] (zero beyond the band)
    const int kb = j0 + pc;
    if (kb < n) {
      // row tiles run fastest over the threads, so the rows a wavefront writes in one
      // column are contiguous
      for (int t = tid; t < tb * tb; t += nt) {
        const int tk = t / tb, tr = t % tb;
        if (tk > tr) continue;
        const int rr0 = 4 * tr, kk0 = 4 * tk;
        T acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[a][e] = (T)0;
        for (int c = 0; c < pc; ++c) {
          const T* col = Pn + c * pw + (pc - c);
          T lr[4], lk[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            lr[q] = col[rr0 + q];
            lk[q] = col[kk0 + q];
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[a][e] += lr[a] * lk[e];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int rr = rr0 + a, kk = kk0 + e;
            const int r = kb + rr, k = kb + kk;
            if (kk <= rr && rr < b && r < n) Li[(i64)k * w + (rr - kk)] -= acc[a][e];
          }
      }
    }
    __syncthreads();
  }
  for (i64 t = tid; t < (i64)n * w; t += nt) {
    const int c = (int)(t / w), dd = (int)(t % w);
    if (c + dd < n) Ri[(i64)(c + dd) * w + dd] = Li[t];
  }
}

// ---------------------------------------------------------------------------
// Column-by-column variant for half-bandwidths whose panel does not fit in LDS either
// (b above about 1250): the trailing b x b triangle updated in global memory each column.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_band_cholesky_global(const i32* __restrict__ subs, const i32* __restrict__ n_arr,
                                       const i32* __restrict__ b_arr,
                                       const i64* __restrict__ src_off,
                                       const double* __restrict__ src,
                                       const i64* __restrict__ dv_off,
                                       const double* __restrict__ dv, double sigma,
                                       const i64* __restrict__ dst_off, T* __restrict__ Lc,
                                       T* __restrict__ Lr, int* __restrict__ status,
                                       const double* __restrict__ src2) {
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  const int n = n_arr[i];
  const int b = b_arr[i];
  const int w = b + 1;
  const double* A = src + src_off[i];
  const double* d = dv ? dv + dv_off[i] : nullptr;
  T* Li = Lc + dst_off[i];
  T* Ri = Lr + dst_off[i];
  for (i64 t = threadIdx.x; t < (i64)n * w; t += blockDim.x) {
    const int c = (int)(t / w), dd = (int)(t % w);
    double a = 0.0;
    if (c + dd < n) {
      a = A[t];
      if (d) a = src2 ? a + sigma * d[c + dd] * d[c] * src2[src_off[i] + t] : a * (1.0 + sigma * d[c + dd] * d[c]);
    }
    Li[t] = (T)a;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const T ajj = Li[(i64)j * w];
    if (!(ajj > (T)0)) {
      if (threadIdx.x == 0) status[i] = ST_NOTSPD;
      return;
    }
    const T ljj = sqrt(ajj);
    __syncthreads();
    for (int t = threadIdx.x; t < w; t += blockDim.x)
      if (j + t < n) Li[(i64)j * w + t] = (t == 0) ? ljj : Li[(i64)j * w + t] / ljj;
    __syncthreads();
    const T* lj = Li + (i64)j * w;
    for (int t = threadIdx.x; t < b * b; t += blockDim.x) {
      const int p = t / b + 1, q = t % b + 1;
      if (q <= p && j + p < n) Li[(i64)(j + q) * w + (p - q)] -= lj[p] * lj[q];
    }
    __syncthreads();
  }
  for (i64 t = threadIdx.x; t < (i64)n * w; t += blockDim.x) {
    const int c = (int)(t / w), dd = (int)(t % w);
    if (c + dd < n) Ri[(i64)(c + dd) * w + dd] = Li[t];
  }
}

// ---------------------------------------------------------------------------
// Y = A^{-1} W for K right-hand sides (column-major n x K, ld n) with the LDL^T
// factor of A (Fc column layout, Fr row layout, see trsv.h).  Half-bandwidths below
// 64: NW right-hand sides per workgroup, rolling-window sweeps sharing tables in LDS;
// otherwise one wavefront per right-hand side with the blocked sweeps.
// ---------------------------------------------------------------------------
template <typename T, typename V, int NW>
__global__ void __launch_bounds__(64 * NW) k_band_solve_rot(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ l_off, const T* __restrict__ Fc, const T* __restrict__ Fr,
    const i64* __restrict__ v_off, int K, const V* __restrict__ Win, V* __restrict__ Yout,
    const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i];
  const int c0 = blockIdx.y * NW;
  const int ncol = min(NW, K - c0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V* Y = Yout + v_off[i] + (i64)c0 * n;
  if (wave < ncol) {
    // each lane copies the rows it will own in the forward sweep
    const V* Wc = Win + v_off[i] + (i64)(c0 + wave) * n;
    V* Yc = Y + (i64)wave * n;
    for (int q = lane; q < n; q += 64) Yc[q] = Wc[q];
  }
  wg_ldl_solve_rot_cols<T, V, NW>(n, b_arr[i], Fc + l_off[i], Fr + l_off[i], Y, ncol,
                                  reinterpret_cast<V*>(smem_raw));
}

// NW wavefronts of NC columns each: 16 columns per workgroup with one LDS table read
// shared by NC chains (see rot_block_m)
template <typename T, typename V, int NW, int NC>
__global__ void __launch_bounds__(64 * NW) k_band_solve_rotm(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ l_off, const T* __restrict__ Fc, const T* __restrict__ Fr,
    const i64* __restrict__ v_off, int K, const V* __restrict__ Win, V* __restrict__ Yout,
    const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i];
  const int c0 = blockIdx.y * NW * NC;
  const int ncol = min(NW * NC, K - c0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V* Y = Yout + v_off[i] + (i64)c0 * n;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int col = wave * NC + q;
    if (col < ncol) {
      // each lane copies the rows it will own in the forward sweep
      const V* Wc = Win + v_off[i] + (i64)(c0 + col) * n;
      V* Yc = Y + (i64)col * n;
      for (int r = lane; r < n; r += 64) Yc[r] = Wc[r];
    }
  }
  wg_ldl_solve_rot_mcols<T, V, NW, NC>(n, b_arr[i], Fc + l_off[i], Fr + l_off[i], Y, ncol,
                                       reinterpret_cast<V*>(smem_raw));
}

// NW computing wavefronts of NC columns plus NS staging wavefronts
template <typename T, typename V, int NW, int NC, int NS>
__global__ void __launch_bounds__(64 * (NW + NS)) k_band_solve_rotms(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ l_off, const T* __restrict__ Fc, const T* __restrict__ Fr,
    const i64* __restrict__ v_off, int K, const V* __restrict__ Win, V* __restrict__ Yout,
    const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i];
  const int c0 = blockIdx.y * NW * NC;
  const int ncol = min(NW * NC, K - c0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  V* Y = Yout + v_off[i] + (i64)c0 * n;
  if (wave < NW) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int col = wave * NC + q;
      if (col < ncol) {
        const V* Wc = Win + v_off[i] + (i64)(c0 + col) * n;
        V* Yc = Y + (i64)col * n;
        for (int r = lane; r < n; r += 64) Yc[r] = Wc[r];
      }
    }
  }
  wg_ldl_solve_rot_mcols_st<T, V, NW, NC, NS>(n, b_arr[i], Fc + l_off[i], Fr + l_off[i], Y, ncol,
                                              reinterpret_cast<V*>(smem_raw));
}

template <typename T, typename V>
__global__ void __launch_bounds__(64) k_band_solve_wave(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ l_off, const T* __restrict__ Fr, const i64* __restrict__ v_off,
    const V* __restrict__ Win, V* __restrict__ Yout, const int* __restrict__ active, int K) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // columns run fastest over the grid, so the K waves of one subdomain run side by side
  // and read its factor from L2 rather than each from HBM
  const int c = (int)(blockIdx.x % (unsigned)K);
  const int q = (int)(blockIdx.x / (unsigned)K);
  const int i = subs ? subs[q] : q;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i];
  V* ring = reinterpret_cast<V*>(smem_raw);
  const int b = b_arr[i];
  const V* Wc = Win + v_off[i] + (i64)c * n;
  V* Yc = Yout + v_off[i] + (i64)c * n;
  wave_ldl_solve_ring<T, V, V>(n, b, Fr + l_off[i], Wc, Yc, nullptr, ring,
                               wave_ring_size(b) - 1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_neumann_assemble(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                             const i32* bw, const i64* boff, const i64* inc_ptr,
                             const i32* inc_slot, const i32* inc_a, const i32* slot_elem,
                             const i32* slot_loc, int k, const double* elem_mat, double* band,
                             int ell_w, const i32* ell_col, double* ell_val, int* status,
                             const i32* elem_ov, double* band2, double* ell_val2) {
  if (total_rows == 0) return;
  dim3 g((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG));
  hipLaunchKernelGGL(k_neumann_assemble, g, dim3(MSDD_WG), 0, s, total_rows, row_sub, voff, bw,
                     boff, inc_ptr, inc_slot, inc_a, slot_elem, slot_loc, k, elem_mat, band,
                     ell_w, ell_col, ell_val, status, elem_ov, band2, ell_val2);
}

void launch_dirichlet_extract(hipStream_t s, i64 total_rows, const i32* drow_sub,
                              const i64* doff, const i32* nd, const i32* bd, const i64* dboff,
                              const i32* dglob, const i64* rowptr, const i32* col,
                              const double* val, double* band, int* status) {
  if (total_rows == 0) return;
  dim3 g((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG));
  hipLaunchKernelGGL(k_dirichlet_extract, g, dim3(MSDD_WG), 0, s, total_rows, drow_sub, doff,
                     nd, bd, dboff, dglob, rowptr, col, val, band, status);
}

template <typename T>
void launch_band_cholesky(hipStream_t s, int nsubs, const i32* subs, int bmax, const i32* n_arr,
                          const i32* b_arr, const i64* src_off, const double* src,
                          const i64* dv_off, const double* dv, double sigma, const i64* dst_off,
                          T* Lc, T* Lr, int* status, const double* src2) {
  if (nsubs == 0) return;
  size_t w = (size_t)bmax + 1;
  size_t lds = (w * w + w + 2 * CHOL_RB * w) * sizeof(T);
  if (lds <= 160 * 1024) {
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)k_band_cholesky<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_band_cholesky<T>, dim3(nsubs), dim3(MSDD_WG), lds, s, subs, n_arr,
                       b_arr, src_off, src, dv_off, dv, sigma, dst_off, Lc, Lr, status, src2);
  } else {
    // panel rows padded so that the window's 4 x 4 tiles read zeros past the band
    const int pw = (int)w + CHB_P + 4;
    const size_t plds = (size_t)CHB_P * pw * sizeof(T);
    if (plds > 150 * 1024) {
      hipLaunchKernelGGL(k_band_cholesky_global<T>, dim3(nsubs), dim3(MSDD_WG), 0, s, subs, n_arr,
                         b_arr, src_off, src, dv_off, dv, sigma, dst_off, Lc, Lr, status, src2);
      return;
    }
    if (plds > 65536)
      (void)hipFuncSetAttribute((const void*)k_band_cholesky_blocked<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds);
    hipLaunchKernelGGL(k_band_cholesky_blocked<T>, dim3(nsubs), dim3(MSDD_WG), plds, s, subs,
                       n_arr, b_arr, src_off, src, dv_off, dv, sigma, dst_off, Lc, Lr, status,
                       src2, pw);
  }
}
template void launch_band_cholesky<double>(hipStream_t, int, const i32*, int, const i32*,
                                           const i32*, const i64*, const double*, const i64*,
                                           const double*, double, const i64*, double*, double*,
                                           int*, const double*);
template void launch_band_cholesky<float>(hipStream_t, int, const i32*, int, const i32*,
                                          const i32*, const i64*, const double*, const i64*,
                                          const double*, double, const i64*, float*, float*,
                                          int*, const double*);

// Cholesky factor L (column layout Lc[j*w + d] = L(j+d, j)) -> LDL^T factor A =
// Lt D Lt^T.  Row layout F[j*w + d] = L(j, j-d) / L(j-d, j-d) (d >= 1, 0 before
// the first column), F[j*w] = 1 / L(j, j)^2 (the inverse of D).  grid.y = subdomain.
template <typename T>
__global__ void k_band_to_ldl(const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
                              const i64* __restrict__ off, const T* __restrict__ Lc,
                              T* __restrict__ F) {
  const int i = blockIdx.y;
  const int n = n_arr[i], w = b_arr[i] + 1;
  const T* L = Lc + off[i];
  T* Fi = F + off[i];
  const i64 cnt = (i64)n * w;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (i64)gridDim.x * blockDim.x) {
    const int j = (int)(e / w), d = (int)(e - (i64)j * w);
    T v = 0;
    if (d == 0) {
      const T l = L[(i64)j * w];
      v = (T)1 / (l * l);
    } else if (j - d >= 0) {
      v = L[(i64)(j - d) * w + d] / L[(i64)(j - d) * w];
    }
    Fi[e] = v;
  }
}

// In place on the column layout, after k_band_to_ldl has read it: column c of L
// becomes column c of the unit factor, Lc[c*w + d] = L(c+d, c) / L(c, c) (0 past
// the last row), and Lc[c*w] = 1 / L(c, c)^2.  One thread per column.
template <typename T>
__global__ void k_band_unit_cols(const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
                                 const i64* __restrict__ off, T* __restrict__ Lc) {
  const int i = blockIdx.y;
  const int n = n_arr[i], w = b_arr[i] + 1;
  T* L = Lc + off[i];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    T* col = L + (i64)c * w;
    const T l = col[0];
    const T il = (T)1 / l;
    for (int d = 1; d < w; ++d) col[d] = (c + d < n) ? col[d] * il : (T)0;
    col[0] = il * il;
  }
}

template <typename T>
void launch_band_to_ldl(hipStream_t s, int nsubs, int nmax, int bmax, const i32* n_arr,
                        const i32* b_arr, const i64* off, T* Lc, T* F) {
  if (nsubs == 0 || nmax == 0) return;
  const i64 cnt = (i64)nmax * (bmax + 1);
  const int gx = (int)std::min<i64>((cnt + 255) / 256, 64);
  hipLaunchKernelGGL(k_band_to_ldl<T>, dim3(gx, nsubs), dim3(256), 0, s, n_arr, b_arr, off, Lc, F);
  const int gc = std::min((nmax + 255) / 256, 16);
  hipLaunchKernelGGL(k_band_unit_cols<T>, dim3(gc, nsubs), dim3(256), 0, s, n_arr, b_arr, off, Lc);
}
template void launch_band_to_ldl<double>(hipStream_t, int, int, int, const i32*, const i32*,
                                         const i64*, double*, double*);
template void launch_band_to_ldl<float>(hipStream_t, int, int, int, const i32*, const i32*,
                                        const i64*, float*, float*);

// Diagonal scaling of the Dirichlet band matrices (column layout B[c*w + d] =
// A(c+d, c)): sc[j] = 1/sqrt(A(j,j)), then B <- diag(sc) B diag(sc) in place (unit
// diagonal).  With coefficient jumps the scaled matrix is far better conditioned,
// which lets its factorisation run in single precision.  grid.y = subdomain.
__global__ void k_band_diag_scale(const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
                                  const i64* __restrict__ off, const i64* __restrict__ doff,
                                  const double* __restrict__ B, double* __restrict__ sc,
                                  int* __restrict__ status) {
  const int i = blockIdx.y;
  const int n = n_arr[i], w = b_arr[i] + 1;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double a = B[off[i] + (i64)j * w];
    if (!(a > 0.0)) status[i] = ST_NOTSPD;
    sc[doff[i] + j] = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
  }
}
__global__ void k_band_apply_scale(const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
                                   const i64* __restrict__ off, const i64* __restrict__ doff,
                                   double* __restrict__ B, const double* __restrict__ sc) {
  const int i = blockIdx.y;
  const int n = n_arr[i], w = b_arr[i] + 1;
  const double* si = sc + doff[i];
  double* Bi = B + off[i];
  const i64 cnt = (i64)n * w;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (i64)gridDim.x * blockDim.x) {
    const int c = (int)(e / w), d = (int)(e - (i64)c * w);
    if (c + d < n) Bi[e] *= si[c] * si[c + d];
  }
}
void launch_band_scale(hipStream_t s, int nsubs, int nmax, int bmax, const i32* n_arr,
                       const i32* b_arr, const i64* off, const i64* doff, double* B, double* sc,
                       int* status) {
  if (nsubs == 0 || nmax == 0) return;
  hipLaunchKernelGGL(k_band_diag_scale, dim3(std::min((nmax + 255) / 256, 16), nsubs), dim3(256), 0,
                     s, n_arr, b_arr, off, doff, B, sc, status);
  const i64 cnt = (i64)nmax * (bmax + 1);
  hipLaunchKernelGGL(k_band_apply_scale, dim3((int)std::min<i64>((cnt + 255) / 256, 64), nsubs),
                     dim3(256), 0, s, n_arr, b_arr, off, doff, B, sc);
}

size_t band_cholesky_lds(int bmax, int elem_size) {
  size_t w = (size_t)bmax + 1;
  return (w * w + w) * elem_size;
}

template <typename T, typename V>
void launch_band_solve_multi(hipStream_t s, int nsubs, const i32* subs, int nmax,
                             const i32* n_arr, const i32* b_arr, const i64* l_off, const T* Fc,
                             const T* Fr, const i64* v_off, int K, const V* W, V* Y,
                             const int* active, int bmax, int variant) {
  // variant: 0 = by shape (rolling window with 16 or 8 columns per workgroup when the
  // half-bandwidth is below 64, else one wavefront per column), 1 = rolling window with 8
  // columns, 2 = rolling window with 16 columns, 3 = one wavefront per column, 4 = rolling
  // window, 4 wavefronts of 4 columns, 5 = rolling window, 8 wavefronts of 2 columns,
  // 6 = as 5 with 4 staging wavefronts, 7 = as 4 with 4 staging wavefronts
  if (nsubs == 0 || K == 0) return;
  if (variant == 0) variant = bmax < 64 ? (K >= 16 ? 2 : 1) : 3;
  if (bmax >= 64) variant = 3;  // the rolling window needs a half-bandwidth below 64
  if (variant == 6 || variant == 7) {
    const size_t lds = 2 * (size_t)ROT_TILE * sizeof(V);
    if (variant == 6) {
      (void)hipFuncSetAttribute((const void*)k_band_solve_rotms<T, V, 8, 2, 4>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_band_solve_rotms<T, V, 8, 2, 4>), dim3(nsubs, (K + 15) / 16),
                         dim3(768), lds, s, subs, n_arr, b_arr, l_off, Fc, Fr, v_off, K, W, Y,
                         active);
    } else {
      (void)hipFuncSetAttribute((const void*)k_band_solve_rotms<T, V, 4, 4, 4>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_band_solve_rotms<T, V, 4, 4, 4>), dim3(nsubs, (K + 15) / 16),
                         dim3(512), lds, s, subs, n_arr, b_arr, l_off, Fc, Fr, v_off, K, W, Y,
                         active);
    }
    return;
  }
  if (variant == 4 || variant == 5) {
    const size_t lds = 2 * (size_t)ROT_TILE * sizeof(V);
    if (variant == 4) {
      (void)hipFuncSetAttribute((const void*)k_band_solve_rotm<T, V, 4, 4>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_band_solve_rotm<T, V, 4, 4>), dim3(nsubs, (K + 15) / 16), dim3(256),
                         lds, s, subs, n_arr, b_arr, l_off, Fc, Fr, v_off, K, W, Y, active);
    } else {
      (void)hipFuncSetAttribute((const void*)k_band_solve_rotm<T, V, 8, 2>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_band_solve_rotm<T, V, 8, 2>), dim3(nsubs, (K + 15) / 16), dim3(512),
                         lds, s, subs, n_arr, b_arr, l_off, Fc, Fr, v_off, K, W, Y, active);
    }
    return;
  }
  if (variant != 3) {
    const size_t lds = 2 * (size_t)ROT_TILE * sizeof(V);
    if (variant == 2) {
      (void)hipFuncSetAttribute((const void*)k_band_solve_rot<T, V, 16>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_band_solve_rot<T, V, 16>), dim3(nsubs, (K + 15) / 16), dim3(1024), lds,
                         s, subs, n_arr, b_arr, l_off, Fc, Fr, v_off, K, W, Y, active);
    } else {
      (void)hipFuncSetAttribute((const void*)k_band_solve_rot<T, V, 8>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((k_band_solve_rot<T, V, 8>), dim3(nsubs, (K + 7) / 8), dim3(512), lds, s,
                         subs, n_arr, b_arr, l_off, Fc, Fr, v_off, K, W, Y, active);
    }
    return;
  }
  (void)nmax;
  const size_t lds = (size_t)wave_ring_size(bmax) * sizeof(V);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_band_solve_wave<T, V>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_band_solve_wave<T, V>), dim3((unsigned)((i64)K * nsubs)), dim3(64), lds, s,
                     subs, n_arr, b_arr, l_off, Fr, v_off, W, Y, active, K);
}
template void launch_band_solve_multi<double, double>(hipStream_t, int, const i32*, int,
                                                      const i32*, const i32*, const i64*,
                                                      const double*, const double*, const i64*,
                                                      int, const double*, double*, const int*,
                                                      int, int);
template void launch_band_solve_multi<float, double>(hipStream_t, int, const i32*, int,
                                                     const i32*, const i32*, const i64*,
                                                     const float*, const float*, const i64*, int,
                                                     const double*, double*, const int*, int,
                                                     int);
template void launch_band_solve_multi<float, float>(hipStream_t, int, const i32*, int,
                                                    const i32*, const i32*, const i64*,
                                                    const float*, const float*, const i64*, int,
                                                    const float*, float*, const int*, int, int);
