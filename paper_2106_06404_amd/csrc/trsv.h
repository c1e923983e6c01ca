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
