/*
 * Eigenpairs of one local GEVP refined in binary128 arithmetic.  TEST
 * INFRASTRUCTURE ONLY: nothing in the GPU library links or calls this file.
 *
 * The local problem of the spectral coarse space (Sec. 2.3, GEVP of the
 * definition; right-hand side b^1 of Sec. 3.4):
 *     abar x = lambda b x,   abar = sum of the subdomain's element matrices,
 *                            b = D abar D (D = partition-of-unity weights),
 * taken through the spectral transformation of the lemma in Sec. 3.3:
 *     b x = mu S x,  S = abar + b  (SPD),  mu = 1/(1 + lambda).
 *
 * The element matrices and weights are FP64 numbers; abar is their exact sum
 * (at most a few terms per entry, exact in the 113-bit significand), so the
 * pencil refined here is the one the FP64 inputs define, free of the rounding
 * of an FP64 assembly.  Starting from FP64 approximations of the wanted
 * eigenvectors, the refinement runs Rayleigh-Ritz on their span and then a few
 * steps of subspace iteration with S^{-1} b, each followed by Rayleigh-Ritz,
 * all in binary128 with S in band form (band Cholesky, band solves).
 *
 * Per Ritz pair (mu, v), v^T S v = 1, it reports:
 *   - bound: sqrt(r^T S^{-1} r), r = b v - mu S v.  In the S inner product the
 *     operator S^{-1} b is self-adjoint, and this is ||S^{-1} b v - mu v||_S, so
 *     some eigenvalue mu* lies within it (Krylov-Weinstein); for lambda the
 *     bound is bound / (mu (mu - bound)).
 *   - cond: with x = v / sqrt(mu) (x^T b x = 1), |x|^T E |x| + lambda |Dx|^T Eb |Dx|,
 *     E = sum over the elements of |a_tau| entrywise, Eb the same over b's elements.  To first order, entrywise
 *     relative perturbations of the element matrices of size eps move lambda by at
 *     most eps * cond (lambda = x^T abar x / x^T b x at the eigenvector).  With
 *     eps = 2^-53 this is the part of lambda that FP64 input data already leaves
 *     undetermined.
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 q;

static q qabs(q x) { return x < 0 ? -x : x; }

/* Lower band storage: M[j*(b+1) + t] = M(j+t, j), 0 <= t <= b. */
typedef struct {
  int n, b;
  q* v;
} band_t;

/* y = M x for symmetric M in lower band storage */
static void band_symv(const band_t* M, const q* x, q* y) {
  const int n = M->n, b = M->b;
  for (int i = 0; i < n; ++i) y[i] = 0;
  for (int j = 0; j < n; ++j) {
    const q* col = M->v + (size_t)j * (b + 1);
    y[j] += col[0] * x[j];
    for (int t = 1; t <= b && j + t < n; ++t) {
      y[j + t] += col[t] * x[j];
      y[j] += col[t] * x[j + t];
    }
  }
}

/* Cholesky S = L L^T in place (band), returns 0 or -(j+1) for a non-positive pivot. */
static int band_chol(band_t* S) {
  const int n = S->n, b = S->b;
  q* v = S->v;
  for (int j = 0; j < n; ++j) {
    q* cj = v + (size_t)j * (b + 1);
    /* column j: subtract contributions of columns k = j-b .. j-1 */
    for (int k = (j - b > 0 ? j - b : 0); k < j; ++k) {
      const q* ck = v + (size_t)k * (b + 1);
      const q ljk = ck[j - k];
      for (int t = 0; t <= b && j + t < n && (j + t - k) <= b; ++t) cj[t] -= ck[j + t - k] * ljk;
    }
    if (!(cj[0] > 0)) return -(j + 1);
    const q d = sqrtq(cj[0]);
    cj[0] = d;
    for (int t = 1; t <= b && j + t < n; ++t) cj[t] /= d;
  }
  return 0;
}

/* x <- L^{-1} x, then x <- L^{-T} x  (S^{-1} x with S = L L^T) */
static void band_solve(const band_t* L, q* x) {
  const int n = L->n, b = L->b;
  const q* v = L->v;
  for (int j = 0; j < n; ++j) {
    const q* cj = v + (size_t)j * (b + 1);
    x[j] /= cj[0];
    for (int t = 1; t <= b && j + t < n; ++t) x[j + t] -= cj[t] * x[j];
  }
  for (int j = n - 1; j >= 0; --j) {
    const q* cj = v + (size_t)j * (b + 1);
    q s = x[j];
    for (int t = 1; t <= b && j + t < n; ++t) s -= cj[t] * x[j + t];
    x[j] = s / cj[0];
  }
}

/* Eigen-decomposition of a small symmetric k x k matrix (row-major, destroyed) by
 * cyclic Jacobi rotations; w[k] eigenvalues, V (row-major) eigenvectors as columns. */
static int small_jacobi(int k, q* a, q* V, q* w) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) V[i * k + j] = (i == j) ? 1 : 0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    q off = 0, tot = 0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        tot += a[i * k + j] * a[i * k + j];
        if (i != j) off += a[i * k + j] * a[i * k + j];
      }
    if (off <= 1e-70Q * tot) {
      for (int i = 0; i < k; ++i) w[i] = a[i * k + i];
      return sweep;
    }
    for (int p = 0; p < k - 1; ++p)
      for (int r = p + 1; r < k; ++r) {
        const q apr = a[p * k + r];
        if (apr == 0) continue;
        const q theta = (a[r * k + r] - a[p * k + p]) / (2 * apr);
        const q t = (theta >= 0 ? 1 : -1) / (qabs(theta) + sqrtq(1 + theta * theta));
        const q c = 1 / sqrtq(1 + t * t), s = t * c;
        for (int m = 0; m < k; ++m) { /* rows p, r */
          const q x = a[p * k + m], y = a[r * k + m];
          a[p * k + m] = c * x - s * y;
          a[r * k + m] = s * x + c * y;
        }
        for (int m = 0; m < k; ++m) { /* columns p, r */
          const q x = a[m * k + p], y = a[m * k + r];
          a[m * k + p] = c * x - s * y;
          a[m * k + r] = s * x + c * y;
          const q vx = V[m * k + p], vy = V[m * k + r];
          V[m * k + p] = c * vx - s * vy;
          V[m * k + r] = s * vx + c * vy;
        }
        a[p * k + r] = a[r * k + p] = 0;
      }
  }
  return -1;
}

typedef struct {
  band_t A, L; /* abar; Cholesky factor of S = abar + b */
  band_t Bo;   /* the matrix inside b = D Bo D (abar itself, or the overlap elements' sum) */
  const q* d;
  int n;
} pencil_t;

static void apply_b(const pencil_t* P, const q* x, q* y, q* tmp) {
  for (int i = 0; i < P->n; ++i) tmp[i] = P->d[i] * x[i];
  band_symv(&P->Bo, tmp, y);
  for (int i = 0; i < P->n; ++i) y[i] *= P->d[i];
}

static void apply_s(const pencil_t* P, const q* x, q* y, q* tmp, q* tmp2) {
  band_symv(&P->A, x, y);
  apply_b(P, x, tmp2, tmp);
  for (int i = 0; i < P->n; ++i) y[i] += tmp2[i];
}

/* Rayleigh-Ritz of (b, S) on span(V) (n x k, column-major, overwritten by the
 * S-orthonormal Ritz vectors, mu descending).  Returns 0 or < 0. */
static int rayleigh_ritz(const pencil_t* P, int k, q* V, q* mu, q* work) {
  const int n = P->n;
  q* SV = work;
  q* BV = SV + (size_t)n * k;
  q* tmp = BV + (size_t)n * k;
  q* tmp2 = tmp + n;
  q* GS = tmp2 + n;
  q* GB = GS + (size_t)k * k;
  q* R = GB + (size_t)k * k;
  q* C = R + (size_t)k * k;
  q* Y = C + (size_t)k * k;
  q* w = Y + (size_t)k * k;
  q* Vn = w + k;
  for (int j = 0; j < k; ++j) {
    apply_s(P, V + (size_t)j * n, SV + (size_t)j * n, tmp, tmp2);
    apply_b(P, V + (size_t)j * n, BV + (size_t)j * n, tmp);
  }
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < k; ++c) {
      q s1 = 0, s2 = 0;
      for (int i = 0; i < n; ++i) {
        s1 += V[(size_t)a * n + i] * SV[(size_t)c * n + i];
        s2 += V[(size_t)a * n + i] * BV[(size_t)c * n + i];
      }
      GS[a * k + c] = s1;
      GB[a * k + c] = s2;
    }
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < a; ++c) {
      const q s1 = 0.5Q * (GS[a * k + c] + GS[c * k + a]), s2 = 0.5Q * (GB[a * k + c] + GB[c * k + a]);
      GS[a * k + c] = GS[c * k + a] = s1;
      GB[a * k + c] = GB[c * k + a] = s2;
    }
  /* GS = R R^T (lower R) */
  memset(R, 0, sizeof(q) * k * k);
  for (int j = 0; j < k; ++j) {
    q s = GS[j * k + j];
    for (int m = 0; m < j; ++m) s -= R[j * k + m] * R[j * k + m];
    if (!(s > 0)) return -1;
    R[j * k + j] = sqrtq(s);
    for (int i = j + 1; i < k; ++i) {
      q t = GS[i * k + j];
      for (int m = 0; m < j; ++m) t -= R[i * k + m] * R[j * k + m];
      R[i * k + j] = t / R[j * k + j];
    }
  }
  /* C = R^{-1} GB R^{-T}: first T = R^{-1} GB (columns), then C = (R^{-1} T^T)^T */
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < k; ++i) {
      q t = GB[i * k + c];
      for (int m = 0; m < i; ++m) t -= R[i * k + m] * C[m * k + c];
      C[i * k + c] = t / R[i * k + i];
    }
  for (int i = 0; i < k; ++i)
    for (int c = 0; c < k; ++c) Y[i * k + c] = C[c * k + i]; /* Y = T^T */
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < k; ++i) {
      q t = Y[i * k + c];
      for (int m = 0; m < i; ++m) t -= R[i * k + m] * C[m * k + c];
      C[i * k + c] = t / R[i * k + i];
    }
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < a; ++c) {
      const q s = 0.5Q * (C[a * k + c] + C[c * k + a]);
      C[a * k + c] = C[c * k + a] = s;
    }
  if (small_jacobi(k, C, Y, w) < 0) return -2;
  /* order mu descending */
  int* ord = (int*)malloc(sizeof(int) * k);
  for (int i = 0; i < k; ++i) ord[i] = i;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j)
      if (w[ord[j]] > w[ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
  /* W = R^{-T} Y (back substitution per column), V <- V W */
  for (int jj = 0; jj < k; ++jj) {
    const int j = ord[jj];
    q* z = C; /* reuse: one column of W */
    for (int i = k - 1; i >= 0; --i) {
      q t = Y[i * k + j];
      for (int m = i + 1; m < k; ++m) t -= R[m * k + i] * z[m];
      z[i] = t / R[i * k + i];
    }
    for (int i = 0; i < n; ++i) {
      q s = 0;
      for (int m = 0; m < k; ++m) s += V[(size_t)m * n + i] * z[m];
      Vn[(size_t)jj * n + i] = s;
    }
    mu[jj] = w[j];
  }
  memcpy(V, Vn, sizeof(q) * (size_t)n * k);
  free(ord);
  return 0;
}

/*
 * n: local dofs; ne elements with kk local dofs each: eloc[ne*kk] (local index or
 * -1 for an eliminated dof), emat[ne*kk*kk] (row-major per element); d[n] weights.
 * bmask[ne] (may be NULL): the elements whose matrices form the matrix inside
 * b = D (sum a_tau) D (NULL: all, b = D abar D; the b^2 right-hand side passes the
 * overlap elements, b^3 passes d = 1 - chi).
 * X0[n*k] (column-major): FP64 start vectors, k >= 1.  iters: subspace steps after
 * the first Rayleigh-Ritz.
 * Outputs (k each, mu descending = lambda ascending): lam_hi + lam_lo = lambda
 * (binary128 value split into two doubles), lam_bound (bound on |lambda - lambda*|),
 * cond (see above); Xout[n*k] (may be NULL): the Ritz vectors x, x^T b x = 1, in FP64.
 * Returns 0, -1 (S not positive definite), -2 (Rayleigh-Ritz failed), -3 (bad input).
 */
int oracle_refine(int n, int ne, int kk, const int* eloc, const double* emat, const double* d,
                  const int* bmask, int k, const double* X0, int iters, double* lam_hi,
                  double* lam_lo, double* lam_bound, double* cond, double* Xout) {
  if (n <= 0 || k <= 0 || k > n || ne < 0 || kk <= 0) return -3;
  int b = 0;
  for (int e = 0; e < ne; ++e)
    for (int r = 0; r < kk; ++r)
      for (int c = 0; c < kk; ++c) {
        const int p = eloc[e * kk + r], s = eloc[e * kk + c];
        if (p >= n || s >= n) return -3;
        if (p >= 0 && s >= 0 && abs(p - s) > b) b = abs(p - s);
      }
  pencil_t P;
  P.n = n;
  P.A.n = P.L.n = n;
  P.A.b = P.L.b = b;
  const size_t bs = (size_t)n * (b + 1);
  P.A.v = (q*)calloc(bs, sizeof(q));
  P.L.v = (q*)calloc(bs, sizeof(q));
  P.Bo = P.A;
  if (bmask) {
    P.Bo.v = (q*)calloc(bs, sizeof(q));
  }
  q* E = (q*)calloc(bs, sizeof(q));  /* sum of |a_tau| */
  q* Eb = bmask ? (q*)calloc(bs, sizeof(q)) : E;  /* the same over b's elements */
  q* dq = (q*)malloc(sizeof(q) * n);
  for (int i = 0; i < n; ++i) dq[i] = d[i];
  P.d = dq;
  for (int e = 0; e < ne; ++e)
    for (int r = 0; r < kk; ++r)
      for (int c = 0; c < kk; ++c) {
        const int p = eloc[e * kk + r], s = eloc[e * kk + c];
        if (p < 0 || s < 0 || p < s) continue; /* lower triangle */
        const double a = emat[((size_t)e * kk + r) * kk + c];
        const size_t o = (size_t)s * (b + 1) + (p - s);
        P.A.v[o] += (q)a;
        E[o] += (q)fabs(a);
        if (bmask && bmask[e]) {
          P.Bo.v[o] += (q)a;
          Eb[o] += (q)fabs(a);
        }
      }
  /* S = abar + D Bo D */
  for (int j = 0; j < n; ++j)
    for (int t = 0; t <= b && j + t < n; ++t) {
      const size_t o = (size_t)j * (b + 1) + t;
      P.L.v[o] = P.A.v[o] + dq[j + t] * P.Bo.v[o] * dq[j];
    }
  int rc = band_chol(&P.L);
  q* V = NULL;
  q* work = NULL;
  q* mu = NULL;
  if (rc != 0) { rc = -1; goto done; }
  V = (q*)malloc(sizeof(q) * (size_t)n * k);
  for (size_t i = 0; i < (size_t)n * k; ++i) V[i] = X0[i];
  work = (q*)malloc(sizeof(q) * ((size_t)3 * n * k + 2 * n + 5 * (size_t)k * k + k));
  mu = (q*)malloc(sizeof(q) * k);
  if (rayleigh_ritz(&P, k, V, mu, work) != 0) { rc = -2; goto done; }
  for (int it = 0; it < iters; ++it) {
    q* tmp = work;
    for (int j = 0; j < k; ++j) {
      q* v = V + (size_t)j * n;
      apply_b(&P, v, tmp + n, tmp);
      memcpy(v, tmp + n, sizeof(q) * n);
      band_solve(&P.L, v);
    }
    if (rayleigh_ritz(&P, k, V, mu, work) != 0) { rc = -2; goto done; }
  }
  {
    q* r = work;
    q* w = r + n;
    q* t1 = w + n;
    q* t2 = t1 + n;
    q* t3 = t2 + n;
    for (int j = 0; j < k; ++j) {
      const q* v = V + (size_t)j * n;
      apply_b(&P, v, r, t1);
      apply_s(&P, v, w, t1, t2);
      for (int i = 0; i < n; ++i) r[i] -= mu[j] * w[i];
      memcpy(t3, r, sizeof(q) * n);
      band_solve(&P.L, t3);
      q e2 = 0;
      for (int i = 0; i < n; ++i) e2 += r[i] * t3[i];
      const q eps = sqrtq(qabs(e2));
      const q m = mu[j];
      const q lam = 1 / m - 1;
      lam_hi[j] = (double)lam;
      lam_lo[j] = (double)(lam - (q)lam_hi[j]);
      lam_bound[j] = (m - eps > 0) ? (double)(eps / (m * (m - eps))) : INFINITY;
      /* condition with x = v / sqrt(mu) */
      const q sc = 1 / sqrtq(m);
      for (int i = 0; i < n; ++i) t1[i] = qabs(v[i]) * sc;
      q c1 = 0, c2 = 0;
      for (int jj = 0; jj < n; ++jj)
        for (int t = 0; t <= b && jj + t < n; ++t) {
          const q e = E[(size_t)jj * (b + 1) + t], eb = Eb[(size_t)jj * (b + 1) + t];
          const q x1 = t1[jj + t] * t1[jj], x2 = dq[jj + t] * t1[jj + t] * dq[jj] * t1[jj];
          c1 += (t == 0 ? 1 : 2) * e * x1;
          c2 += (t == 0 ? 1 : 2) * eb * x2;
        }
      cond[j] = (double)(c1 + lam * c2);
      if (Xout)
        for (int i = 0; i < n; ++i) Xout[(size_t)j * n + i] = (double)(v[i] * sc);
    }
  }
  rc = 0;
done:
  if (bmask) {
    free(P.Bo.v);
    free(Eb);
  }
  free(P.A.v);
  free(P.L.v);
  free(E);
  free(dq);
  free(V);
  free(work);
  free(mu);
  return rc;
}

/* lambda of the pencil for k given vectors' Rayleigh quotients only (no iteration):
 * used by the tests to evaluate x^T abar x / x^T b x exactly for a given FP64 x. */
int oracle_rayleigh(int n, int ne, int kk, const int* eloc, const double* emat, const double* d,
                    int k, const double* X, double* lam) {
  int b = 0;
  for (int e = 0; e < ne; ++e)
    for (int r = 0; r < kk; ++r)
      for (int c = 0; c < kk; ++c) {
        const int p = eloc[e * kk + r], s = eloc[e * kk + c];
        if (p >= n || s >= n) return -3;
        if (p >= 0 && s >= 0 && abs(p - s) > b) b = abs(p - s);
      }
  band_t A = {n, b, (q*)calloc((size_t)n * (b + 1), sizeof(q))};
  for (int e = 0; e < ne; ++e)
    for (int r = 0; r < kk; ++r)
      for (int c = 0; c < kk; ++c) {
        const int p = eloc[e * kk + r], s = eloc[e * kk + c];
        if (p < 0 || s < 0 || p < s) continue;
        A.v[(size_t)s * (b + 1) + (p - s)] += (q)emat[((size_t)e * kk + r) * kk + c];
      }
  q* x = (q*)malloc(sizeof(q) * n);
  q* y = (q*)malloc(sizeof(q) * n);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < n; ++i) x[i] = X[(size_t)j * n + i];
    band_symv(&A, x, y);
    q num = 0;
    for (int i = 0; i < n; ++i) num += x[i] * y[i];
    for (int i = 0; i < n; ++i) x[i] *= d[i];
    band_symv(&A, x, y);
    q den = 0;
    for (int i = 0; i < n; ++i) den += x[i] * y[i];
    lam[j] = (double)(num / den);
  }
  free(A.v);
  free(x);
  free(y);
  return 0;
}
