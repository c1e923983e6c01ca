// Small dense FP64 products inside one workgroup on the matrix cores
// (v_mfma_f64_16x16x4f64): each wavefront takes 16 x 16 output tiles and runs over
// the inner dimension four at a time.  Per lane and step one element of A (row
// lane % 16, inner index lane / 16) and one of B (inner index lane / 16, column
// lane % 16) are loaded; the tile's 256 results come back four per lane (rows
// lane / 16 + 4 q, q = 0..3, column lane % 16).  Against 4 x 4 register tiles on the vector
// units this needs an eighth of the operand loads per multiply-add, which is what
// bounds these products when an operand streams from L2.
#pragma once
#include "common.h"

typedef double dbl4 __attribute__((ext_vector_type(4)));

// C(i, j) = sum_k A(i, k) B(k, j) over the tiles t = first, first + stride, ... of a
// grid of tm x tn tiles; tile t covers rows 16 (t / tn) + 0..15 and columns
// 16 (t % tn) + 0..15, clipped to M x N.  a(i, k), b(k, j) load the operands and are
// called with indices clamped into range (out-of-range operands are then replaced by
// zeros, without branches, so that the loads of four steps are issued together);
// c(i, j, value) stores a result.  Called by whole wavefronts.
template <class FA, class FB, class FC>
__device__ __forceinline__ void wave_gemm_tiles(int M, int N, int K, int tn, int t0, int tcount,
                                                int tstride, FA a, FB b, FC c) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int nsteps = (K + 3) >> 2;
  for (int t = t0; t < tcount; t += tstride) {
    const int i0 = 16 * (t / tn), j0 = 16 * (t % tn);
    const int ia = i0 + r16, jb = j0 + r16;
    const bool ai = ia < M, bj = jb < N;
    const int iac = ai ? ia : M - 1, jbc = bj ? jb : N - 1;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    int st = 0;
    for (; st + 4 <= nsteps; st += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = 4 * (st + u) + k4;
        const bool in = kk < K;
        const int kc = in ? kk : K - 1;
        const double x = a(iac, kc), y = b(kc, jbc);
        av[u] = (ai && in) ? x : 0.0;
        bv[u] = (bj && in) ? y : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    for (; st < nsteps; ++st) {
      const int kk = 4 * st + k4;
      const bool in = kk < K;
      const int kc = in ? kk : K - 1;
      const double x = a(iac, kc), y = b(kc, jbc);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64((ai && in) ? x : 0.0, (bj && in) ? y : 0.0, acc,
                                                 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + k4 + 4 * q;
      if (i < M && bj) c(i, jb, acc[q]);
    }
  }
}
