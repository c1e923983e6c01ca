// Two-sided (twisted) band solve for the finest-level Dirichlet matrices of the
// preconditioner apply (the local solves A_i^{-1} of the additive Schwarz operator,
// Sec. 2.1): the same solution as the two sweeps of the LDL^T factor, with two dependent
// chains of about n/2 rows running side by side instead of one chain of n rows.
//
// Rows of A (n x n, half-bandwidth b < 64) are split into T = [0, k), S = [k, k + b) and
// B = [k + b, n) with k a multiple of 64.  T and B are not coupled (their rows are more
// than b apart), so in the order (T, B, S)
//   A = M diag(D_T, D_B, D_C) M^T,   M = [L_T 0 0; 0 U_B 0; F_T F_B L_C],
// where A_TT = L_T D_T L_T^T is given by the leading rows of A's LDL^T factor (whose S rows
// hold F_T = A_ST L_T^{-T} D_T^{-1} in the T columns), A_BB = U_B D_B U_B^T is the LDL^T
// factor of rows [k, n) in reversed order (whose S rows hold F_B), and
// C = L_C D_C L_C^T = A_SS - F_T D_T F_T^T - F_B D_B F_B^T is the Schur complement on S.
// A x = r becomes
//   forward     w_T = L_T^{-1} r_T  and  w_B = U_B^{-1} r_B         (independent chains)
//   separator   x_S = C^{-1} (r_S - F_T w_T - F_B w_B)             (explicit C^{-1})
//   backward    x_T = L_T^{-T} (D_T^{-1} w_T - F_T^T x_S), x_B likewise (independent).
// The forward chains end with r_S - F_T w_T and r_S - F_B w_B in the accumulators of the
// S rows (the rolling window carries the next block's rows), and each backward chain
// starts with the S block: x_S held fixed (no in-block updates) while F^T x_S enters the
// accumulators of the adjacent rows.
//
// Reversed order of the bottom part: position rho of the bottom factor is row
// n - 1 + p - rho for rho >= p; the first p positions are padding rows (identity, zero
// right-hand side) so that the S rows start a 64-row block: with m = n - k - b bottom rows
// and nbb = ceil(m / 64) blocks before S, p = 64 nbb - m; the bottom factor has
// nB = 64 nbb + b rows, its last b rows (positions 64 nbb + s) being row k + b - 1 - s.
#include "common.h"
#include "trsv.h"

// ---------------------------------------------------------------------------
// Bottom part: band of rows [k, n) in reversed order with p padding rows in front, in the
// column layout of the Dirichlet band (Bt[c*w + d] = A'(c + d, c), 0 past the end).
//   src: column layout of A (B[c*w + d] = A(c + d, c)).  grid.y = subdomain.
// ---------------------------------------------------------------------------
__global__ void k_twist_extract(const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
                                const i32* __restrict__ nbt_arr, const i32* __restrict__ nbb_arr,
                                const i64* __restrict__ off, const double* __restrict__ src,
                                const i64* __restrict__ toff, double* __restrict__ dst) {
  const int i = blockIdx.y;
  const int n = n_arr[i], b = b_arr[i], w = b + 1;
  if (nbt_arr[i] <= 0) return;
  const int k = 64 * nbt_arr[i];
  const int m = n - k - b;
  const int p = 64 * nbb_arr[i] - m;
  const int nB = p + n - k;
  const double* A = src + off[i];
  double* Bt = dst + toff[i];
  const i64 cnt = (i64)nB * w;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (i64)gridDim.x * blockDim.x) {
    const int c = (int)(e / w), d = (int)(e - (i64)c * w);
    double v = 0.0;
    if (c < p) {
      v = d == 0 ? 1.0 : 0.0;
    } else if (c + d < nB) {
      const int r = n - 1 + p - c;  // row of position c; position c + d is row r - d
      v = A[(i64)(r - d) * w + d];  // A(r, r - d) = A(r - d + d, r - d)
    }
    Bt[e] = v;
  }
}

// ---------------------------------------------------------------------------
// C^{-1} per subdomain (b x b, column-major, symmetric up to rounding) from the two LDL^T
// factors (row layouts: Fr[j*w + d] = Lt(j, j - d), Fr[j*w] = 1/D_j) and A_SS (column
// layout of A), in FP64 whatever the factor's precision.  One 256-thread workgroup per
// subdomain; C in LDS, inverted by Gauss-Jordan elimination without pivoting (C is SPD).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_twist_schur(
    const i32* __restrict__ n_arr, const i32* __restrict__ b_arr, const i32* __restrict__ nbt_arr,
    const i32* __restrict__ nbb_arr, const i64* __restrict__ off, const double* __restrict__ A,
    const T* __restrict__ Fr, const i64* __restrict__ toff, const T* __restrict__ Gr,
    const i64* __restrict__ coff, T* __restrict__ Cinv, int* __restrict__ status) {
  __shared__ double C[63 * 63];
  __shared__ double rowp[64], colp[64];
  const int i = blockIdx.x;
  if (nbt_arr[i] <= 0) return;
  const int n = n_arr[i], b = b_arr[i], w = b + 1;
  const int k = 64 * nbt_arr[i];
  const int s0 = 64 * nbb_arr[i];  // first S position of the bottom factor
  const double* Ai = A + off[i];
  const T* F = Fr + off[i];
  const T* G = Gr + toff[i];
  (void)n;
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int r = e % b, c = e / b;  // C(k + r, k + c)
    const int lo = min(r, c), d = abs(r - c);
    double v = Ai[(i64)(k + lo) * w + d];
    // top: sum over T columns j < k with j >= k + max(r, c) - b
    const int rr = k + r, cc = k + c;
    for (int j = max(0, max(rr, cc) - b); j < k; ++j)
      v -= (double)F[(i64)rr * w + (rr - j)] * (double)F[(i64)cc * w + (cc - j)] /
           (double)F[(i64)j * w];
    // bottom: S index r is position s0 + b - 1 - r; its B columns are positions < s0
    const int pr = s0 + b - 1 - r, pc = s0 + b - 1 - c;
    for (int j = max(0, max(pr, pc) - b); j < s0; ++j)
      v -= (double)G[(i64)pr * w + (pr - j)] * (double)G[(i64)pc * w + (pc - j)] /
           (double)G[(i64)j * w];
    C[c * b + r] = v;
  }
  __syncthreads();
  // in-place Gauss-Jordan: after pivot q, C holds the inverse on the pivoted indices
  for (int q = 0; q < b; ++q) {
    const double piv = C[q * b + q];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) status[i] = ST_NOTSPD;
      return;  // uniform: every thread read the same pivot
    }
    if (threadIdx.x < b) {
      rowp[threadIdx.x] = C[threadIdx.x * b + q];  // C(q, j)
      colp[threadIdx.x] = C[q * b + threadIdx.x];  // C(j, q)
    }
    __syncthreads();
    const double ip = 1.0 / piv;
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
      const int r = e % b, c = e / b;
      double v;
      if (r == q && c == q) v = ip;
      else if (r == q) v = rowp[c] * ip;
      else if (c == q) v = -colp[r] * ip;
      else v = C[e] - colp[r] * rowp[c] * ip;
      C[e] = v;
    }
    __syncthreads();
  }
  T* out = Cinv + coff[i];
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) out[e] = (T)C[e];
}

// ---------------------------------------------------------------------------
// The solve.  One workgroup of TW_NT threads per subdomain: wavefront 0 runs the top
// chain, wavefront 1 the bottom chain, wavefronts 2-4 and 5-7 stage their tables.  The
// vector is in LDS.  Each chain is the rolling-window recurrence of wg_ldl_solve_rot
// (two accumulators per lane: the row in the current 64-row block and the row in the next
// one; tables Tc[k][l] and Tn[k][l] of the block's factor entries), with the tables
// staged per half block (32 steps) so that both chains' double buffers fit in LDS.
// Half-step t runs half a block of each chain; the forward sweeps take 2 max(nbt, nbb)
// half-steps, then the separator, then 2 (max(nbt, nbb) + 1) half-steps of backward
// sweeps (the first block of each is the S block).  One barrier per half-step.
// ---------------------------------------------------------------------------
constexpr int TW_NT = 512;
constexpr int TW_TAB = 32 * 64;        // one table of a half block
constexpr int TW_BUF = 2 * TW_TAB + 128;  // Tc, Tn, 1/D of the next block's rows, 64 dummies
constexpr int TW_STG = 192;            // staging threads per chain
constexpr int TW_PER = (32 * 64 + TW_STG - 1) / TW_STG;  // entries per staging thread
constexpr int TW_DEPTH = 6;            // half-steps between a segment's read and its use

// 32 substitution steps (steps 32 h .. 32 h + 31 of the block) in chunks of TW_CH, each
// chunk's table entries read while the previous one runs.
constexpr int TW_CH = 16;
template <typename V>
__device__ __forceinline__ void tw_half(const V* buf, int lane, V& a, V& a2, int h) {
  constexpr int NC = 32 / TW_CH;
  const V* Tc = buf;
  const V* Tn = buf + TW_TAB;
  const int s0 = 32 * h;
  V tc[2][TW_CH], tn[2][TW_CH];
#pragma unroll
  for (int t = 0; t < TW_CH; ++t) {
    tc[0][t] = Tc[t * 64 + lane];
    tn[0][t] = Tn[t * 64 + lane];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c + 1 < NC) {
#pragma unroll
      for (int t = 0; t < TW_CH; ++t) {
        tc[(c + 1) & 1][t] = Tc[(TW_CH * (c + 1) + t) * 64 + lane];
        tn[(c + 1) & 1][t] = Tn[(TW_CH * (c + 1) + t) * 64 + lane];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < TW_CH; ++t) {
      const V y = wave_bcast(a, s0 + TW_CH * c + t);
      a -= tc[c & 1][t] * y;
      a2 -= tn[c & 1][t] * y;
    }
    asm volatile("" : "+v"(a2));
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename T>
__global__ void __launch_bounds__(TW_NT) k_apply_fine_twist(
    const i32* __restrict__ nd, const i32* __restrict__ bd, const i64* __restrict__ doff,
    const i64* __restrict__ dboff, const T* __restrict__ Fc, const T* __restrict__ Fr,
    const i32* __restrict__ nbt_arr, const i32* __restrict__ nbb_arr, const i64* __restrict__ toff,
    const T* __restrict__ Gc, const T* __restrict__ Gr, const i64* __restrict__ coff,
    const T* __restrict__ Cinv, const double* __restrict__ scale, double* __restrict__ u,
    int nd_max, int cinv_lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x;
  const int n = nd[i], b = bd[i], w = b + 1;
  const int nbt = nbt_arr[i], nbb = nbb_arr[i];
  const int k = 64 * nbt;
  const int p = 64 * nbb - (n - k - b);
  T* rl = reinterpret_cast<T*>(smem_raw);
  T* tiles = rl + ((nd_max + 3) & ~3);  // [chain][buffer], TW_BUF each
  T* gS = tiles + 4 * TW_BUF;           // S accumulators of both chains, then g
  T* cl = gS + 192;                     // C^{-1} (when it fits)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* ui = u + doff[i];
  const double* si = scale ? scale + doff[i] : nullptr;
  const T* ci = Cinv + coff[i];
  for (int q = threadIdx.x; q < n; q += TW_NT) rl[q] = (T)(si ? ui[q] * si[q] : ui[q]);
  for (int t = threadIdx.x; t < 4 * TW_BUF; t += TW_NT) tiles[t] = (T)0;
  if (cinv_lds)
    for (int t = threadIdx.x; t < b * b; t += TW_NT) cl[t] = ci[t];
  const T* cm = cinv_lds ? cl : ci;
  const int NF = max(nbt, nbb);
  const int HF = 2 * NF;
  // half-steps, rounded up to whole rounds of the staging ring (the extra ones are idle)
  const int HT = (HF + 2 * (NF + 1) + TW_DEPTH - 1) / TW_DEPTH * TW_DEPTH;
  // this wavefront's chain (stagers: the chain they stage for)
  const int ch = wave < 2 ? wave : (wave - 2) / 3;
  const int nblk = ch ? nbb : nbt;

  if (wave >= 2) {
    // ---- staging wavefronts: the segment of half-step u is read into registers at
    // half-step u - TW_DEPTH + 1 (a ring of TW_DEPTH register sets) and scattered into the
    // chain's buffer (u & 1) during half-step u - 1
    const T* Lc = ch ? Gc + toff[i] : Fc + dboff[i];
    const T* Lr = ch ? Gr + toff[i] : Fr + dboff[i];
    const int tl = threadIdx.x - 128 - TW_STG * ch;
    // thread tl stages entries e = tl + TW_STG u of the segment (32 columns or rows of w
    // entries, contiguous in memory, so that a wavefront's read is contiguous); the
    // segment row of e is e / w, taken as (e * mw) >> 20 (exact for e < 2^14, w <= 64)
    const int mw = ((1 << 20) + w - 1) / w;
    T gv[TW_DEPTH][TW_PER];
    T gd[TW_DEPTH];
    // Every half-step issues the same TW_PER + 1 loads, from clamped in-range addresses
    // when the chain is idle or the entry is not kept (no branch around a load), so that
    // the compiler counts the loads in flight exactly and waits only for the set a store
    // needs; what is kept is decided again at the store.
    const int rmax = 64 * nblk + b - 1;  // last factor row read (the S rows)
    const i64 lim_r = (i64)(rmax + 1) * w - 1;
    auto load = [&](int t, T* v, T& dv) {
      const bool fwd = t < HF;
      const int h = t & 1;
      const int qf = min(t >> 1, nblk - 1);
      const int Q = fwd ? nblk : max(nblk - ((t - HF) >> 1), 0);  // backward row block
      const i64 r0 = fwd ? (i64)(64 * qf + 32 * h) * w : (i64)(64 * Q + 32 - 32 * h) * w;
      const i64 lim = fwd ? r0 + 32 * w - 1 : lim_r;
      const T* src = fwd ? Lc : Lr;
#pragma unroll
      for (int uu = 0; uu < TW_PER; ++uu) v[uu] = src[min(r0 + tl + uu * TW_STG, lim)];
      dv = Lr[(i64)(64 * max(Q - 1, 0) + 63 - (tl & 63)) * w];
    };
    // invalid entries go to the lane's own dummy slot (no branch around a store)
    const int dummy = 2 * TW_TAB + 64 + (tl & 63);
    auto store = [&](int t, const T* v, T dv) {
      T* buf = tiles + (2 * ch + (t & 1)) * TW_BUF;
      const int h = t & 1;
      const int cnt = 32 * w;
      if (t < HF) {
        if ((t >> 1) >= nblk) return;
#pragma unroll
        for (int uu = 0; uu < TW_PER; ++uu) {
          const int e = tl + uu * TW_STG;
          const int kk = (e * mw) >> 20, d = e - kk * w;
          const int kst = 32 * h + kk;  // the step that broadcasts column kk
          const int l = (kst + d) & 63;
          const int pos = ((l > kst) ? 0 : TW_TAB) + kk * 64 + l;
          buf[(e < cnt && d > 0) ? pos : dummy] = v[uu];
        }
      } else {
        const int qq = (t - HF) >> 1;
        if (qq > nblk) return;
#pragma unroll
        for (int uu = 0; uu < TW_PER; ++uu) {
          const int e = tl + uu * TW_STG;
          const int kk = (e * mw) >> 20, d = e - kk * w;
          const int kr = 32 - 32 * h + kk;  // row kr of the row block
          const int st = 63 - kr;           // the step that broadcasts it
          const int l = (st + d) & 63;
          const int pos = ((l > st) ? 0 : TW_TAB) + (31 - kk) * 64 + l;
          // the S block keeps only the couplings of S rows to the rows before S
          const bool keep = qq > 0 || (kr < b && d > kr);
          buf[(e < cnt && d > 0) ? pos : dummy] = keep ? v[uu] : (T)0;
        }
        if (h == 0 && tl < 64) buf[2 * TW_TAB + tl] = nblk - qq >= 1 ? dv : (T)0;
      }
    };
    // the first segments' reads overlap the set-up of the vector and tables
#pragma unroll
    for (int j = 0; j < TW_DEPTH; ++j) load(j, gv[j], gd[j]);
    __syncthreads();
    store(0, gv[0], gd[0]);
    lds_barrier();
    for (int t0 = 0; t0 < HT; t0 += TW_DEPTH) {
#pragma unroll
      for (int j = 0; j < TW_DEPTH; ++j) {
        const int t = t0 + j;
        if (t == HF) {
          lds_barrier();
          lds_barrier();
        }
        constexpr int one = 1;
        store(t + 1, gv[(j + one) % TW_DEPTH], gd[(j + one) % TW_DEPTH]);
        load(t + TW_DEPTH, gv[j], gd[j]);
        lds_barrier();
      }
    }
  } else {
    // ---- chain wavefronts
    auto row_of = [&](int rho) { return ch ? n - 1 + p - rho : rho; };
    auto valid = [&](int rho) { return ch ? rho >= p : true; };
    // S index s (0..b-1, in the chain's order) -> row
    auto srow = [&](int s) { return ch ? k + b - 1 - s : k + s; };
    T a = 0, a2 = 0;
    __syncthreads();
    lds_barrier();
    for (int t = 0; t < HT; ++t) {
      if (t == HF) {
        // separator: g = (r_S - F_T w_T) + (r_S - F_B w_B) - r_S, x_S = C^{-1} g
        if (wave == 0 && lane < b)
          gS[128 + lane] = gS[lane] + gS[64 + b - 1 - lane] - rl[k + lane];
        lds_barrier();
        if (wave == 0 && lane < b) {
          T x = 0;
          for (int j = 0; j < b; ++j) x += cm[(i64)j * b + lane] * gS[128 + j];
          rl[k + lane] = x;
        }
        lds_barrier();
      }
      const T* buf = tiles + (2 * ch + (t & 1)) * TW_BUF;
      // set up the block's accumulators at its first half, run the half block, store
      // the block's rows at its second half
      const int h = t & 1;
      const bool fwd = t < HF;
      const int qb = fwd ? (t >> 1) : ((t - HF) >> 1);  // block (forward) or reversed block
      const bool act = fwd ? qb < nblk : qb <= nblk;
      const int Q = nblk - qb;                           // backward: row block
      const int rho = fwd ? 64 * qb + lane : 64 * Q + 63 - lane;
      if (act && h == 0) {
        if (fwd) {
          if (qb == 0) a = valid(rho) ? rl[row_of(rho)] : (T)0;
          if (qb + 1 < nblk) a2 = valid(rho + 64) ? rl[row_of(rho + 64)] : (T)0;
          else a2 = lane < b ? rl[srow(lane)] : (T)0;
        } else {
          if (qb == 0) {
            const int sidx = 63 - lane;
            a = sidx < b ? rl[srow(sidx)] : (T)0;
          }
          a2 = (Q >= 1 && valid(rho - 64)) ? rl[row_of(rho - 64)] * buf[2 * TW_TAB + lane] : (T)0;
        }
      }
      if (act) tw_half<T>(buf, lane, a, a2, h);
      if (act && h == 1) {
        if ((fwd || qb > 0) && valid(rho)) rl[row_of(rho)] = a;
        a = a2;
        if (fwd && qb + 1 == nblk && lane < b) gS[64 * ch + lane] = a;
      }
      lds_barrier();
    }
  }
  for (int q = threadIdx.x; q < n; q += TW_NT)
    ui[q] = si ? (double)rl[q] * si[q] : (double)rl[q];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
void twist_split(int n, int b, int* nbt, int* nbb) {
  *nbt = 0;
  *nbb = 0;
  if (b >= 64 || n - b - 1 < 64) return;
  const int t = std::min((n - b + 127) / 128, (n - b - 1) / 64);
  *nbt = t;
  *nbb = (n - 64 * t - b + 63) / 64;
}

size_t apply_fine_twist_lds(int nd_max, int bd_max, size_t elem, bool cinv_lds) {
  return ((size_t)((nd_max + 3) & ~3) + 4 * (size_t)TW_BUF + 192 +
          (cinv_lds ? (size_t)bd_max * bd_max : 0)) * elem;
}

void launch_twist_extract(hipStream_t s, int P, int nB_max, int bd_max, const i32* nd,
                          const i32* bd, const i32* nbt, const i32* nbb, const i64* dboff,
                          const double* Dband, const i64* toff, double* Bt) {
  if (P == 0 || nB_max == 0) return;
  const i64 cnt = (i64)nB_max * (bd_max + 1);
  const int gx = (int)std::min<i64>((cnt + 255) / 256, 64);
  hipLaunchKernelGGL(k_twist_extract, dim3(gx, P), dim3(256), 0, s, nd, bd, nbt, nbb, dboff, Dband,
                     toff, Bt);
}

template <typename T>
void launch_twist_schur(hipStream_t s, int P, const i32* nd, const i32* bd, const i32* nbt,
                        const i32* nbb, const i64* dboff, const double* Dband, const T* Fr,
                        const i64* toff, const T* Gr, const i64* coff, T* Cinv, int* status) {
  if (P == 0) return;
  hipLaunchKernelGGL(k_twist_schur<T>, dim3(P), dim3(256), 0, s, nd, bd, nbt, nbb, dboff, Dband,
                     Fr, toff, Gr, coff, Cinv, status);
}
template void launch_twist_schur<double>(hipStream_t, int, const i32*, const i32*, const i32*,
                                         const i32*, const i64*, const double*, const double*,
                                         const i64*, const double*, const i64*, double*, int*);
template void launch_twist_schur<float>(hipStream_t, int, const i32*, const i32*, const i32*,
                                        const i32*, const i64*, const double*, const float*,
                                        const i64*, const float*, const i64*, float*, int*);

// false when the shape does not fit (the caller then takes the one-chain solve)
bool launch_apply_fine_twist(hipStream_t s, int P, int nd_max, int bd_max, const i32* nd,
                             const i32* bd, const i64* doff, const i64* dboff, const void* Fc,
                             const void* Fr, const i32* nbt, const i32* nbb, const i64* toff,
                             const void* Gc, const void* Gr, const i64* coff, const void* Cinv,
                             int fp32, const double* scale, double* u) {
  if (P == 0) return true;
  const size_t elem = fp32 ? sizeof(float) : sizeof(double);
  int cinv_lds = 1;
  size_t lds = apply_fine_twist_lds(nd_max, bd_max, elem, true);
  if (lds > 160 * 1024) {
    cinv_lds = 0;
    lds = apply_fine_twist_lds(nd_max, bd_max, elem, false);
    if (lds > 160 * 1024) return false;
  }
  if (fp32) {
    (void)hipFuncSetAttribute((const void*)k_apply_fine_twist<float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_apply_fine_twist<float>, dim3(P), dim3(TW_NT), lds, s, nd, bd, doff, dboff,
                       (const float*)Fc, (const float*)Fr, nbt, nbb, toff, (const float*)Gc,
                       (const float*)Gr, coff, (const float*)Cinv, scale, u, nd_max, cinv_lds);
  } else {
    (void)hipFuncSetAttribute((const void*)k_apply_fine_twist<double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_apply_fine_twist<double>, dim3(P), dim3(TW_NT), lds, s, nd, bd, doff,
                       dboff, (const double*)Fc, (const double*)Fr, nbt, nbb, toff,
                       (const double*)Gc, (const double*)Gr, coff, (const double*)Cinv, scale, u,
                       nd_max, cinv_lds);
  }
  return true;
}
