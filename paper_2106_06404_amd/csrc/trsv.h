// One-wavefront blocked triangular solves with a banded (or dense) Cholesky factor.
//
// The right-hand side lives in LDS (v[0..n)) and is overwritten by the
// solution.  Rows are processed in blocks of 64 (one row per lane):
//   1. "pull": each lane subtracts the contributions of the already solved
//      rows outside the block that lie within the band; the loop runs over a
//      static index range with predication so every load issues up front;
//   2. the 64 x 64 triangular diagonal block is solved in registers: the lane
//      that owns row k finishes y_k, v_readlane broadcasts it, every other lane
//      applies its (preloaded) factor entry.  Static unrolling keeps the
//      factor block in registers (lane j holds row/column j of the block).
// Band layouts: Lr[j*(b+1)+d] = L(j, j-d) (rows), Lc[j*(b+1)+d] = L(j+d, j)
// (columns).  A dense n x n factor is stored in the same two layouts with
// b = n-1 (ld = n).
// Must be called by every lane of a wavefront; the workgroup synchronises
// between blocks with __syncthreads().
#pragma once
#include "common.h"

__device__ inline double wave_bcast(double v, int lane) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_readlane(lo, lane);
  hi = __builtin_amdgcn_readlane(hi, lane);
  return __hiloint2double(hi, lo);
}
__device__ inline float wave_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// L y = v  (forward), in place on v (LDS).  ld = b+1 for band storage.
template <typename T, typename V>
__device__ __forceinline__ void wave_trsv_lower(int n, int b, const T* __restrict__ Lr, V* v, int ld = -1) {
  const int lane = threadIdx.x & 63;
  const int w = ld > 0 ? ld : b + 1;
  for (int j0 = 0; j0 < n; j0 += 64) {
    const int nb = min(64, n - j0);
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0, dinv = 0;
    V lk[64];
    if (act) {
      const T* Lrow = Lr + (i64)row * w;
      a = v[row];
      // pull: columns row - dd < j0 (dd > lane) within the band
      for (int d0 = lane + 1; d0 <= b && row - d0 >= 0; d0 += 16) {
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int dd = d0 + t;
          if (dd <= b && row - dd >= 0) acc += (V)Lrow[dd] * v[row - dd];
        }
        a -= acc;
      }
      dinv = (V)1 / (V)Lrow[0];
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        const int dd = lane - k;
        lk[k] = (dd > 0 && dd <= b) ? (V)Lrow[dd] : (V)0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 64; ++k) lk[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      if (k < nb) {
        const V yk = wave_bcast(a * dinv, k);
        if (lane == k) a = yk;
        else a -= lk[k] * yk;
      }
    }
    if (act) v[row] = a;
    __syncthreads();
  }
}

// L^T x = v  (backward), in place on v (LDS).  ld = b+1 for band storage.
template <typename T, typename V>
__device__ __forceinline__ void wave_trsv_upper(int n, int b, const T* __restrict__ Lc, V* v, int ld = -1) {
  const int lane = threadIdx.x & 63;
  const int w = ld > 0 ? ld : b + 1;
  for (int j1 = n; j1 > 0; j1 -= 64) {
    const int j0 = max(0, j1 - 64);
    const int nb = j1 - j0;
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0, dinv = 0;
    V lk[64];
    if (act) {
      const T* Lcol = Lc + (i64)row * w;
      a = v[row];
      // pull: rows row + dd >= j1 within the band
      for (int d0 = j1 - row; d0 <= b && row + d0 < n; d0 += 16) {
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int dd = d0 + t;
          if (dd <= b && row + dd < n) acc += (V)Lcol[dd] * v[row + dd];
        }
        a -= acc;
      }
      dinv = (V)1 / (V)Lcol[0];
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        const int dd = k - lane;
        lk[k] = (dd > 0 && dd <= b) ? (V)Lcol[dd] : (V)0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 64; ++k) lk[k] = 0;
    }
#pragma unroll
    for (int k = 63; k >= 0; --k) {
      if (k < nb) {
        const V xk = wave_bcast(a * dinv, k);
        if (lane == k) a = xk;
        else a -= lk[k] * xk;
      }
    }
    if (act) v[row] = a;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Staged variants for half-bandwidths b < 64: the factor rows (or columns) of a
// 64-row block form one contiguous segment of 64*(b+1) entries in band layout.
// All waves of the workgroup load that segment cooperatively into LDS
// (coalesced), and the segment of the next block is fetched into registers
// while the current block is solved, so the solve itself reads only LDS.
// Every wave of the workgroup solves its own right-hand side v (LDS) with the
// shared staged factor; all waves must have the same n and b.
//   stage: LDS buffer of 2 * 64 * (b+1) entries of T.
// ---------------------------------------------------------------------------
template <typename T, typename V, int NWV, int WMAX, bool UPPER>
__device__ __forceinline__ void wg_trsv_staged(int n, int b, const T* __restrict__ L, V* v,
                                               T* stage) {
  constexpr int PRE = (WMAX + NWV - 1) / NWV;  // prefetch registers per thread (64 rows x w <= WMAX)
  const int lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  const int nt = 64 * NWV;
  const int w = b + 1;
  const int seg = 64 * w;
  const int nblk = (n + 63) / 64;
  // block q covers rows [j0, j0+nb); the backward sweep visits blocks in reverse
  auto blk_j0 = [&](int q) { return UPPER ? (nblk - 1 - q) * 64 : q * 64; };
  {
    const int j0 = blk_j0(0);
    const int cnt = min(64, n - j0) * w;
    for (int t = tid; t < cnt; t += nt) stage[t] = L[(i64)j0 * w + t];
  }
  __syncthreads();
  int buf = 0;
  for (int q = 0; q < nblk; ++q) {
    const int j0 = blk_j0(q);
    const int nb = min(64, n - j0);
    // prefetch the next block's segment into registers
    T pre[PRE];
    int ncnt = 0;
    if (q + 1 < nblk) {
      const int j0n = blk_j0(q + 1);
      ncnt = min(64, n - j0n) * w;
      const T* src = L + (i64)j0n * w;
#pragma unroll
      for (int u = 0; u < PRE; ++u) {
        const int t = tid + u * nt;
        pre[u] = (t < ncnt) ? src[t] : (T)0;
      }
    }
    const T* Lb = stage + buf * seg;
    const int row = j0 + lane;
    const bool act = lane < nb;
    const T* Lrow = Lb + lane * w;
    // this lane's row (column) of the diagonal block, from LDS into registers
    V lk[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const int dd = UPPER ? k - lane : lane - k;
      const bool ok = dd > 0 && dd <= b;
      const V lv = (V)Lrow[ok ? dd : 0];
      lk[k] = ok ? lv : (V)0;
    }
    V a = 0, dinv = 1;
    if (act) {
      a = v[row];
      if (!UPPER) {
        // columns row - dd < j0 within the band (dd > lane)
        for (int d0 = lane + 1; d0 <= b && row - d0 >= 0; d0 += 16) {
          V acc = 0;
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            const int dd = d0 + t;
            const bool ok = dd <= b && row - dd >= 0;
            const V lv = (V)Lrow[ok ? dd : 0];
            const V xv = v[ok ? row - dd : row];
            acc += ok ? lv * xv : (V)0;
          }
          a -= acc;
        }
      } else {
        const int j1 = j0 + nb;
        for (int d0 = j1 - row; d0 <= b && row + d0 < n; d0 += 16) {
          V acc = 0;
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            const int dd = d0 + t;
            const bool ok = dd <= b && row + dd < n;
            const V lv = (V)Lrow[ok ? dd : 0];
            const V xv = v[ok ? row + dd : row];
            acc += ok ? lv * xv : (V)0;
          }
          a -= acc;
        }
      }
      dinv = (V)1 / (V)Lrow[0];
    }
    if (!UPPER) {
#pragma unroll
      for (int k = 0; k < 64; ++k) {
        if (k < nb) {
          const V yk = wave_bcast(a * dinv, k);
          a = (lane == k) ? yk : a - lk[k] * yk;
        }
      }
    } else {
#pragma unroll
      for (int k = 63; k >= 0; --k) {
        if (k < nb) {
          const V xk = wave_bcast(a * dinv, k);
          a = (lane == k) ? xk : a - lk[k] * xk;
        }
      }
    }
    if (act) v[row] = a;
    if (q + 1 < nblk) {
      T* dst = stage + (buf ^ 1) * seg;
#pragma unroll
      for (int u = 0; u < PRE; ++u) {
        const int t = tid + u * nt;
        if (t < ncnt) dst[t] = pre[u];
      }
    }
    __syncthreads();
    buf ^= 1;
  }
}

// ---------------------------------------------------------------------------
// Solves with an LDL^T band factor, right-hand side v in LDS (overwritten by the
// solution).
//   F (row layout, ld w = b+1): F[j*w + d] = Lt(j, j-d) for 1 <= d <= b, where
//   Lt is the unit lower triangular factor of A = Lt D Lt^T, and F[j*w] = 1/D_jj.
// Forward sweep Lt y = v (unit diagonal: the diagonal-block chain is one
// broadcast and one FMA per row), then y <- D^{-1} y folded into the first
// touch of each row in the backward sweep Lt^T x = y.
// ---------------------------------------------------------------------------

// Unstaged variant for any b (factor read from global memory).
template <typename T, typename V>
__device__ __forceinline__ void wave_ldl_solve(int n, int b, const T* __restrict__ F, V* v) {
  const int lane = threadIdx.x & 63;
  const int w = b + 1;
  for (int j0 = 0; j0 < n; j0 += 64) {
    const int nb = min(64, n - j0);
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0;
    if (act) {
      const T* Fr = F + (i64)row * w;
      a = v[row];
      for (int d0 = lane + 1; d0 <= b && row - d0 >= 0; d0 += 16) {
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int dd = d0 + t;
          const bool ok = dd <= b && row - dd >= 0;
          const V lv = (V)Fr[ok ? dd : 0];
          const V xv = v[ok ? row - dd : row];
          acc += ok ? lv * xv : (V)0;
        }
        a -= acc;
      }
    }
    for (int k = 0; k < nb; ++k) {
      const int dd = lane - k;
      const bool ok = act && dd > 0 && dd <= b;
      const V lv = ok ? (V)F[(i64)row * w + dd] : (V)0;
      const V yk = wave_bcast(a, k);
      a -= lv * yk;
    }
    if (act) v[row] = a;
    __syncthreads();
  }
  for (int j1 = n; j1 > 0; j1 -= 64) {
    const int j0 = max(0, j1 - 64);
    const int nb = j1 - j0;
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0;
    if (act) {
      a = v[row] * (V)F[(i64)row * w];
      const int imax = min(n - 1, row + b);
      for (int i0 = j1; i0 <= imax; i0 += 16) {
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int i = i0 + t;
          const bool ok = i <= imax;
          const int ic = ok ? i : row;
          const V lv = ok ? (V)F[(i64)ic * w + (ic - row)] : (V)0;
          acc += lv * v[ic];
        }
        a -= acc;
      }
    }
    for (int k = nb - 1; k >= 0; --k) {
      const int dd = k - lane;
      const bool ok = act && dd > 0 && dd <= b;
      const V lv = ok ? (V)F[(i64)(j0 + k) * w + dd] : (V)0;
      const V xk = wave_bcast(a, k);
      a -= lv * xk;
    }
    if (act) v[row] = a;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Rolling-window LDL^T band solve for b < 64 with one workgroup of ROT_NT
// threads: wavefront 0 runs the substitution, the others stage the factor.
//
//   Fc (column layout, ld w = b+1): Fc[c*w + d] = Lt(c+d, c) for 1 <= d <= b;
//   Fr (row layout):                Fr[j*w + d] = Lt(j, j-d) for 1 <= d <= b,
//                                   Fr[j*w] = 1/D_jj,
//   where A = Lt D Lt^T with Lt unit lower triangular (entries outside the
//   matrix are stored as 0).
//
// Forward sweep Lt y = v: lane l owns the rows r = l (mod 64).  At step j (one
// per row) y_j is final in lane j mod 64; it is broadcast (v_readlane) and every
// lane subtracts Lt(r, j) y_j for its row r.  Because b < 64 a row receives
// contributions only from the 63 rows before it, so a lane carries two
// accumulators: a for its row in the current 64-row block and a2 for its row in
// the next block.  Per block (rows j0..j0+63) the tables
//   Tc[k][l] = Lt(j0+l, j0+k)      (l > k: the row in this block),
//   Tn[k][l] = Lt(j0+64+l, j0+k)   (l < k: the row in the next block),
// zero elsewhere, make step k two FMAs without any lane selection:
//   y = bcast(a, k);  a -= Tc[k][l] y;  a2 -= Tn[k][l] y.
// At the end of a block a holds the block's final y, a <- a2, and a2 <- the
// right-hand side of the block after next.  Entry (column k, offset d) of the
// block's column segment goes to position (k, (k+d) mod 64).
// Backward sweep Lt^T x = D^{-1} y: the same recurrence on the reversed row
// order rho = N-1-j (N = 64 * number of blocks), where it is lower triangular
// with entries Lt(j, j-d); reversed block q' is row block nblk-1-q', whose row
// segment entry (local row kk, offset d) goes to position (63-kk, (63-kk+d) mod
// 64).  Both sweeps thus write the same table positions, which are zeroed once.
// The staging wavefronts build the tables of the next step in the other LDS
// buffer from the contiguous band segment (read into registers one step ahead),
// so the substitution reads only LDS.
//   v:     the right-hand side (LDS, n entries), overwritten by the solution;
//   tiles: 2 * ROT_TILE entries of V in LDS.
// All ROT_NT threads must call it.
// ---------------------------------------------------------------------------
constexpr int ROT_NT = 512;
constexpr int ROT_TILE = 2 * 4096 + 64;          // Tc, Tn, 1/D of the next block's rows
constexpr int ROT_PER = (64 * 64 + ROT_NT - 65) / (ROT_NT - 64);  // segment entries per stager

// 64 substitution steps of one block, in 4 chunks of 16; the table entries of
// chunk c+1 are read while chunk c runs (scheduling barriers keep the reads ahead).
template <typename V>
__device__ __forceinline__ void rot_block(const V* buf, int lane, V& a, V& a2) {
  const V* Tc = buf;
  const V* Tn = buf + 4096;
  V tc[2][16], tn[2][16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    tc[0][t] = Tc[t * 64 + lane];
    tn[0][t] = Tn[t * 64 + lane];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c < 3) {
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        tc[(c + 1) & 1][t] = Tc[(16 * (c + 1) + t) * 64 + lane];
        tn[(c + 1) & 1][t] = Tn[(16 * (c + 1) + t) * 64 + lane];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const V y = wave_bcast(a, 16 * c + t);
      a -= tc[c & 1][t] * y;
      a2 -= tn[c & 1][t] * y;
    }
    // keep the a2 updates inside their chunk (otherwise they are sunk to the end
    // of the block, holding 64 broadcast values in scalar registers)
    asm volatile("" : "+v"(a2));
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename T, typename V>
__device__ __forceinline__ void wg_ldl_solve_rot(int n, int b, const T* __restrict__ Fc,
                                                 const T* __restrict__ Fr, V* v, V* tiles) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = b + 1;
  const int nblk = (n + 63) >> 6;
  const int nsteps = 2 * nblk;
  const int N = nblk * 64;
  const int seg = 64 * w;
  const int tl = threadIdx.x - 64;  // staging thread index
  constexpr int NS = ROT_NT - 64;
  // staging registers: one segment of the step after next
  T gv[ROT_PER];
  int gpos[ROT_PER];  // table position (k*64 + l) + 1, 0 = no entry; bit 30 = Tn
  T gd = 0;
  auto stage_load = [&](int s) {
    const bool fwd = s < nblk;
    const int q = fwd ? s : nsteps - 1 - s;  // row block
    const int j0 = q * 64;
    const T* src = (fwd ? Fc : Fr) + (i64)j0 * w;
    const int cnt = min(64, n - j0) * w;
#pragma unroll
    for (int u = 0; u < ROT_PER; ++u) {
      const int e = tl + u * NS;
      const int kk = e / w, d = e - kk * w;
      int pos = 0;
      if (e < cnt && d > 0) {
        const int k = fwd ? kk : 63 - kk;
        const int l = (k + d) & 63;
        pos = (k * 64 + l + 1) | ((l > k) ? 0 : (1 << 30));
      }
      gpos[u] = pos;
      gv[u] = src[min(e, cnt - 1)];
    }
    gd = 0;
    // 1/D of the rows of the next reversed block (row block q-1), lane order of
    // the reversed rows: lane l <-> row j0 - 1 - l
    if (!fwd && tl < 64 && q > 0) gd = Fr[(i64)(j0 - 1 - tl) * w];
  };
  auto stage_store = [&](V* buf) {
#pragma unroll
    for (int u = 0; u < ROT_PER; ++u) {
      const int pos = gpos[u];
      if (pos) {
        const int p = (pos & ((1 << 30) - 1)) - 1;
        buf[(pos >> 30) ? 4096 + p : p] = (V)gv[u];
      }
    }
    if (tl < 64) buf[8192 + tl] = (V)gd;
  };
  // zero both buffers (positions without an entry stay zero), then stage step 0
  for (int t = threadIdx.x; t < 2 * ROT_TILE; t += ROT_NT) tiles[t] = (V)0;
  __syncthreads();
  if (wave > 0) {
    stage_load(0);
    stage_store(tiles);
    if (nsteps > 1) stage_load(1);
  }
  __syncthreads();
  V a = 0, a2 = 0;
  for (int s = 0; s < nsteps; ++s) {
    V* buf = tiles + (s & 1) * ROT_TILE;
    if (wave > 0) {
      if (s + 1 < nsteps) {
        stage_store(tiles + ((s + 1) & 1) * ROT_TILE);
        if (s + 2 < nsteps) stage_load(s + 2);
      }
    } else if (s < nblk) {  // forward, row block s
      const int row = s * 64 + lane;
      if (s == 0) a = row < n ? v[row] : (V)0;
      a2 = row + 64 < n ? v[row + 64] : (V)0;
      rot_block<V>(buf, lane, a, a2);
      if (row < n) v[row] = a;
      a = a2;
    } else {  // backward, reversed block s - nblk: lane l <-> row N-1-(64(s-nblk)+l)
      const int row = N - 1 - (64 * (s - nblk) + lane);
      if (s == nblk) a = row < n ? v[row] * (V)Fr[(i64)row * w] : (V)0;
      a2 = (row - 64 >= 0 && row - 64 < n) ? v[row - 64] * buf[8192 + lane] : (V)0;
      rot_block<V>(buf, lane, a, a2);
      if (row < n) v[row] = a;
      a = a2;
    }
    __syncthreads();
  }
}
