// One-wavefront blocked triangular solves with a banded Cholesky factor.
//
// The right-hand side lives in LDS (v[0..n)) and is overwritten by the
// solution.  Rows are processed in blocks of 64 (one row per lane):
//   1. "pull": each lane subtracts the contributions of the already solved
//      rows outside the block that lie within the band (a dot product of
//      length <= b over a contiguous stretch of the factor);
//   2. the 64 x 64 triangular diagonal block is solved in registers: the lane
//      that owns row k finishes y_k, v_readlane broadcasts it, every other lane
//      applies its (preloaded) factor entry.  Static unrolling keeps the
//      factor block in registers (lane j holds row/column j of the block).
// Band layouts: Lr[j*(b+1)+d] = L(j, j-d) (rows), Lc[j*(b+1)+d] = L(j+d, j) (columns).
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

// L y = v  (forward), in place on v (LDS)
template <typename T, typename V>
__device__ void wave_trsv_lower(int n, int b, const T* __restrict__ Lr, V* v) {
  const int lane = threadIdx.x & 63;
  const int w = b + 1;
  for (int j0 = 0; j0 < n; j0 += 64) {
    const int nb = min(64, n - j0);
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0, dinv = 0;
    V lk[64];
    if (act) {
      const T* Lrow = Lr + (i64)row * w;
      a = v[row];
      // pull: rows col = row - dd < j0 within the band
      for (int dd = lane + 1; dd <= b && row - dd >= 0; ++dd) a -= (V)Lrow[dd] * v[row - dd];
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

// L^T x = v  (backward), in place on v (LDS)
template <typename T, typename V>
__device__ void wave_trsv_upper(int n, int b, const T* __restrict__ Lc, V* v) {
  const int lane = threadIdx.x & 63;
  const int w = b + 1;
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
      for (int dd = j1 - row; dd <= b && row + dd < n; ++dd) a -= (V)Lcol[dd] * v[row + dd];
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
