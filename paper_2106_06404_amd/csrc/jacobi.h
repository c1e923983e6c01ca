// Workgroup-parallel cyclic Jacobi eigensolver for a dense symmetric matrix.
//
// Round-robin (circle) ordering: in each of the m-1 rounds of a sweep the
// m/2 index pairs are disjoint, so the rotations of a round are applied by
// all threads at once: first to rows p,q (J^T A), then to columns p,q
// ((J^T A) J) and to the eigenvector matrix.  A rotation is taken when
// |a_pq| > eps*sqrt(|a_pp a_qq|) and |a_pq| > floor; the sweep loop stops
// after a sweep without rotations.  A and V are row-major n x n (any address
// space); pair scratch lives in LDS.
#pragma once
#include "common.h"

template <typename R>
struct JacobiScratch {
  int* pp;
  int* pq;
  R* pc;
  R* ps;
  int* cnt;  // single int
  int* tot;  // single int: rotations applied (accumulated; may be null)
};

template <typename R>
__device__ inline void jacobi_pair(int r, int k, int m, int& p, int& q) {
  if (k == 0) {
    p = r;
    q = m - 1;
  } else {
    p = (r + k) % (m - 1);
    q = (r - k + (m - 1)) % (m - 1);
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
}

// Returns the number of sweeps used (or -1 if max_sweeps was hit).
// Each round: (1) the rotation of every pair of the round is computed from the
// current A; (2) A <- J^T A J is applied block by block: the 2x2 block of rows
// {p_k, q_k} and columns {p_k', q_k'} depends only on that block and the two
// rotations, so every block is rotated in one pass (row rotation first, then
// the column rotation), V <- V J in the same pass; one barrier per phase.
// Pairs without a rotation act as the identity; blocks of two such pairs are
// skipped.  With n odd, the dummy index m-1 = n drops out of its pair.
// VT: V is stored transposed (V[col*n + row]); the column updates of V then touch
// two contiguous rows, which matters when V lives in global memory.  JU / JV: work
// items per thread whose loads are issued together (A blocks / V entries).
template <typename R, int JU = 4, bool VT = false, int JV = JU>
// skip_below: pairs whose two diagonal entries are both below it are not rotated
// (for a positive semi-definite A the whole 2x2 block is then below it: its
// rotations only mix directions that the caller discards).
__device__ __forceinline__ int jacobi_block(int n, R* A, R* V, JacobiScratch<R> s, int max_sweeps, R eps,
                            R floor_abs, R skip_below = 0) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nwv = (nt + 63) >> 6;
  for (int r0 = wv; r0 < n; r0 += nwv)
    for (int c0 = lane; c0 < n; c0 += 64) V[r0 * n + c0] = (r0 == c0) ? (R)1 : (R)0;
  __syncthreads();
  if (n <= 1) return 0;
  const int m = (n & 1) ? n + 1 : n;
  const int np = m / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *s.cnt = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      for (int k = tid; k < np; k += nt) {
        int p, q;
        jacobi_pair<R>(r, k, m, p, q);
        R c = 1, sn = 0;
        int use = 0;
        if (q < n) {
          const R apq = A[p * n + q];
          const R app = A[p * n + p], aqq = A[q * n + q];
          if (fabs(apq) > eps * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs &&
              (fabs(app) >= skip_below || fabs(aqq) >= skip_below)) {
            const R theta = (aqq - app) / (2 * apq);
            const R t = (theta >= 0 ? (R)1 : (R)-1) / (fabs(theta) + sqrt((R)1 + theta * theta));
            c = (R)1 / sqrt((R)1 + t * t);
            sn = t * c;
            use = 1;
            atomicAdd(s.cnt, 1);
          }
        }
        s.pp[k] = use ? p : -1 - p;  // the index survives in the unused case
        s.pq[k] = q;
        s.pc[k] = c;
        s.ps[k] = sn;
      }
      __syncthreads();
      // A <- J^T A J on 2x2 blocks (pair k = rows, pair k2 = columns), then V <- V J.
      // Each thread first loads JU work items, then rotates and stores them, so the
      // loads of a round are in flight together (the compiler cannot move a load
      // above a store to the same array by itself).
      {
        const int nblk2 = np * np;
        for (int t0 = tid; t0 < nblk2; t0 += nt * JU) {
          R x[JU], y[JU], z[JU], w[JU];
          int ia[JU], ib[JU];  // flat index of A[p][p2]; -1 = nothing to do
          int dq[JU], dq2[JU];  // row / column offsets of q, q2 (0 when absent)
#pragma unroll
          for (int u = 0; u < JU; ++u) {
            const int t = t0 + u * nt;
            ia[u] = -1;
            x[u] = y[u] = z[u] = w[u] = 0;
            dq[u] = dq2[u] = 0;
            ib[u] = 0;
            if (t < nblk2) {
              const int k = t / np, k2 = t - k * np;
              const int pk = s.pp[k], pk2 = s.pp[k2];
              if (pk >= 0 || pk2 >= 0) {
                const int p = pk >= 0 ? pk : -1 - pk, q = s.pq[k];
                const int p2 = pk2 >= 0 ? pk2 : -1 - pk2, q2 = s.pq[k2];
                ia[u] = p * n + p2;
                ib[u] = k * np + k2;
                dq[u] = q < n ? (q - p) * n : 0;
                dq2[u] = q2 < n ? q2 - p2 : 0;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < JU; ++u) {
            if (ia[u] >= 0) {
              const int a0 = ia[u];
              x[u] = A[a0];
              z[u] = A[a0 + dq2[u]];
              y[u] = A[a0 + dq[u]];
              w[u] = A[a0 + dq[u] + dq2[u]];
            }
          }
#pragma unroll
          for (int u = 0; u < JU; ++u) {
            if (ia[u] < 0) continue;
            const int k = ib[u] / np, k2 = ib[u] - k * np;
            const R c = s.pc[k], sn = s.ps[k], c2 = s.pc[k2], s2 = s.ps[k2];
            const R x1 = c * x[u] - sn * y[u], y1 = sn * x[u] + c * y[u];
            const R z1 = c * z[u] - sn * w[u], w1 = sn * z[u] + c * w[u];
            R npp = c2 * x1 - s2 * z1, npq = s2 * x1 + c2 * z1;
            R nqp = c2 * y1 - s2 * w1, nqq = s2 * y1 + c2 * w1;
            if (k == k2 && s.pp[k] >= 0) {
              npq = 0;
              nqp = 0;
            }
            const int a0 = ia[u];
            // absent q / q2 (odd n): the aliased writes below are skipped
            if (dq[u] != 0 && dq2[u] != 0) A[a0 + dq[u] + dq2[u]] = nqq;
            if (dq[u] != 0) A[a0 + dq[u]] = nqp;
            if (dq2[u] != 0) A[a0 + dq2[u]] = npq;
            A[a0] = npp;
          }
        }
        const int nv = n * np;
        for (int t0 = tid; t0 < nv; t0 += nt * JV) {
          R x[JV], y[JV];
          int ia[JV], ib[JV];
#pragma unroll
          for (int u = 0; u < JV; ++u) {
            const int t = t0 + u * nt;
            ia[u] = -1;
            ib[u] = 0;
            x[u] = y[u] = 0;
            if (t < nv) {
              // VT: consecutive threads take consecutive rows of one column pair
              const int row = VT ? t % n : t / np;
              const int k2 = VT ? t / n : t - row * np;
              const int pk2 = s.pp[k2];
              if (pk2 >= 0) {
                ia[u] = VT ? pk2 * n + row : row * n + pk2;
                ib[u] = k2;
              }
            }
          }
#pragma unroll
          for (int u = 0; u < JV; ++u) {
            if (ia[u] >= 0) {
              const int k2 = ib[u];
              const int dq = VT ? (s.pq[k2] - s.pp[k2]) * n : s.pq[k2] - s.pp[k2];
              x[u] = V[ia[u]];
              y[u] = V[ia[u] + dq];
            }
          }
#pragma unroll
          for (int u = 0; u < JV; ++u) {
            if (ia[u] < 0) continue;
            const int k2 = ib[u];
            const int dq = VT ? (s.pq[k2] - s.pp[k2]) * n : s.pq[k2] - s.pp[k2];
            const R c2 = s.pc[k2], s2 = s.ps[k2];
            V[ia[u]] = c2 * x[u] - s2 * y[u];
            V[ia[u] + dq] = s2 * x[u] + c2 * y[u];
          }
        }
      }
      __syncthreads();
    }
    const int c = *s.cnt;
    __syncthreads();
    if (tid == 0 && s.tot) *s.tot += c;
    if (c == 0) break;
  }
  return sweep < max_sweeps ? sweep + 1 : -1;
}
