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
template <typename R>
__device__ int jacobi_block(int n, R* A, R* V, JacobiScratch<R> s, int max_sweeps, R eps,
                            R floor_abs) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int t = tid; t < n * n; t += nt) V[t] = (t / n == t % n) ? (R)1 : (R)0;
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
          if (fabs(apq) > eps * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
            const R theta = (aqq - app) / (2 * apq);
            const R t = (theta >= 0 ? (R)1 : (R)-1) / (fabs(theta) + sqrt((R)1 + theta * theta));
            c = (R)1 / sqrt((R)1 + t * t);
            sn = t * c;
            use = 1;
            atomicAdd(s.cnt, 1);
          }
        }
        s.pp[k] = use ? p : -1;
        s.pq[k] = q;
        s.pc[k] = c;
        s.ps[k] = sn;
      }
      __syncthreads();
      // rows p, q
      for (int t = tid; t < np * n; t += nt) {
        const int k = t / n, j = t % n;
        const int p = s.pp[k];
        if (p < 0) continue;
        const int q = s.pq[k];
        const R c = s.pc[k], sn = s.ps[k];
        const R x = A[p * n + j], y = A[q * n + j];
        A[p * n + j] = c * x - sn * y;
        A[q * n + j] = sn * x + c * y;
      }
      __syncthreads();
      // columns p, q of A and V
      for (int t = tid; t < np * n; t += nt) {
        const int row = t / np, k = t % np;
        const int p = s.pp[k];
        if (p < 0) continue;
        const int q = s.pq[k];
        const R c = s.pc[k], sn = s.ps[k];
        R x = A[row * n + p], y = A[row * n + q];
        A[row * n + p] = c * x - sn * y;
        A[row * n + q] = sn * x + c * y;
        x = V[row * n + p];
        y = V[row * n + q];
        V[row * n + p] = c * x - sn * y;
        V[row * n + q] = sn * x + c * y;
      }
      __syncthreads();
      for (int k = tid; k < np; k += nt) {
        const int p = s.pp[k];
        if (p < 0) continue;
        const int q = s.pq[k];
        A[p * n + q] = 0;
        A[q * n + p] = 0;
      }
      __syncthreads();
    }
    const int c = *s.cnt;
    __syncthreads();
    if (c == 0) break;
  }
  return sweep < max_sweeps ? sweep + 1 : -1;
}
