/*
 * Plain FP64 dense kernels of the CPU oracle.  TEST INFRASTRUCTURE ONLY:
 * nothing in the GPU library links or calls this file.
 *
 *  - oracle_cholesky: textbook Cholesky-Crout, A = L L^T (row-major, in place).
 *    Used for the shifted pencil (a + b) that the spectral transformation of
 *    the GEVP lemma (Sec. 3.3) makes SPD, for the subdomain Dirichlet matrices
 *    A_i = R_i A R_i^T of the additive Schwarz preconditioner (Sec. 2.1), and
 *    for the coarsest-level matrix A_0.
 *  - oracle_jacobi: cyclic two-sided Jacobi rotations for a dense symmetric
 *    matrix (round-robin ordering, so the n/2 rotations of one round touch
 *    disjoint index pairs and may be applied by several threads; the result
 *    does not depend on the thread count).  Used for every symmetric
 *    eigenproblem of the oracle.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* A (n x n, row-major, symmetric) -> L in the lower triangle, zeros above.
 * Returns 0, or -(j+1) if the j-th pivot is not positive. */
int oracle_cholesky(int n, double* a) {
  for (int j = 0; j < n; ++j) {
    double s = a[(size_t)j * n + j];
    const double* rj = a + (size_t)j * n;
    for (int k = 0; k < j; ++k) s -= rj[k] * rj[k];
    if (!(s > 0.0)) return -(j + 1);
    double ljj = sqrt(s);
    a[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double* ri = a + (size_t)i * n;
      double t = ri[j];
      for (int k = 0; k < j; ++k) t -= ri[k] * rj[k];
      ri[j] = t / ljj;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) a[(size_t)i * n + j] = 0.0;
  return 0;
}

/* Eigen-decomposition of a symmetric n x n matrix by cyclic Jacobi rotations.
 *   a: row-major, destroyed; w[n] receives the eigenvalues (unsorted),
 *   v: row-major n x n, receives the eigenvectors as columns.
 * A rotation on (p,q) is taken when |a_pq| > eps*sqrt(|a_pp a_qq|) and
 * |a_pq| > abs_floor * ||A||_F; the iteration stops after a sweep with no
 * rotation.  Returns the number of sweeps, or -1 if max_sweeps was reached. */
int oracle_jacobi(int n, double* a, double* v, double* w, int max_sweeps,
                  double abs_floor, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const double eps = 2.220446049250313e-16;
  double fro = 0.0;
  for (size_t i = 0; i < (size_t)n * n; ++i) fro += a[i] * a[i];
  fro = sqrt(fro);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) v[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  if (n <= 1) {
    if (n == 1) w[0] = a[0];
    return 0;
  }
  const int m = (n % 2) ? n + 1 : n; /* players, one dummy if n is odd */
  const int np = m / 2;
  int* pos = (int*)malloc(sizeof(int) * m);
  int* pp = (int*)malloc(sizeof(int) * np);
  int* pq = (int*)malloc(sizeof(int) * np);
  double* pc = (double*)malloc(sizeof(double) * np);
  double* ps = (double*)malloc(sizeof(double) * np);
  for (int i = 0; i < m; ++i) pos[i] = i;
  int sweep, result = -1;
  const int par = (n >= 96);
  for (sweep = 0; sweep < max_sweeps; ++sweep) {
    long nrot = 0;
    for (int round = 0; round < m - 1; ++round) {
      /* 1. rotation parameters of this round's disjoint pairs */
      int cnt = 0;
      for (int k = 0; k < np; ++k) {
        int p = pos[k], q = pos[m - 1 - k];
        if (p >= n || q >= n) continue;
        if (p > q) { int t = p; p = q; q = t; }
        double apq = a[(size_t)p * n + q];
        double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        if (!(fabs(apq) > eps * sqrt(fabs(app * aqq))) || !(fabs(apq) > abs_floor * fro)) continue;
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
        double c = 1.0 / sqrt(1.0 + t * t);
        pp[cnt] = p; pq[cnt] = q; pc[cnt] = c; ps[cnt] = t * c;
        ++cnt;
      }
      nrot += cnt;
      if (cnt) {
        /* 2. rows p,q <- J^T A  (pairs are disjoint: independent) */
#pragma omp parallel for schedule(static) if (par)
        for (int r = 0; r < cnt; ++r) {
          double* rp = a + (size_t)pp[r] * n;
          double* rq = a + (size_t)pq[r] * n;
          double c = pc[r], s = ps[r];
          for (int k = 0; k < n; ++k) {
            double x = rp[k], y = rq[k];
            rp[k] = c * x - s * y;
            rq[k] = s * x + c * y;
          }
        }
        /* 3. columns p,q <- (J^T A) J, row by row */
#pragma omp parallel for schedule(static) if (par)
        for (int k = 0; k < n; ++k) {
          double* rk = a + (size_t)k * n;
          double* vk = v + (size_t)k * n;
          for (int r = 0; r < cnt; ++r) {
            int p = pp[r], q = pq[r];
            double c = pc[r], s = ps[r];
            double x = rk[p], y = rk[q];
            rk[p] = c * x - s * y;
            rk[q] = s * x + c * y;
            x = vk[p]; y = vk[q];
            vk[p] = c * x - s * y;
            vk[q] = s * x + c * y;
          }
        }
        /* 4. the annihilated couplings are exactly zero */
        for (int r = 0; r < cnt; ++r) {
          int p = pp[r], q = pq[r];
          a[(size_t)p * n + q] = 0.0;
          a[(size_t)q * n + p] = 0.0;
        }
      }
      /* next round-robin arrangement: keep pos[0], rotate the others */
      int last = pos[m - 1];
      for (int i = m - 1; i > 1; --i) pos[i] = pos[i - 1];
      pos[1] = last;
    }
    if (nrot == 0) { result = sweep + 1; break; }
  }
  for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
  free(pos); free(pp); free(pq); free(pc); free(ps);
  return result;
}
