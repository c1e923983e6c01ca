// Workgroup-parallel divide-and-conquer eigensolver for a symmetric tridiagonal matrix
// (Cuppen's method with the Gu-Eisenstat eigenvector formula; Golub and Van Loan,
// "Matrix Computations", Sec. 8.4).  The matrix is torn into 1 x 1 leaves by rank-one
// tears at every off-diagonal entry, and the leaves are merged pairwise, level by
// level, all merges of a level side by side:
//
//   T = diag(T1, T2) + rho v v^T,  v = (last row of Q1, +-first row of Q2) / sqrt(2),
//
// where T1 = Q1 D1 Q1^T and T2 = Q2 D2 Q2^T are the halves' eigendecompositions and a
// coupling beta gives rho = 2 |beta| (the tear takes |beta| off both adjacent diagonal
// entries, the sign of beta goes into v).  A merge
//   1. deflates: components with rho |z_i| <= tol, and pairs of nearly equal poles
//      (a plane rotation zeroes one z component when the off-diagonal entry it creates
//      is <= tol), tol = 8 eps max(|D|, rho); the eigenvector columns take the rotations;
//   2. solves the secular equation 1/rho + sum_i z_i^2 / (d_i - lambda) = 0 for each
//      root between consecutive poles (one small group of lanes per root), each root
//      kept as (origin pole, offset) so that every difference lambda - d_i is accurate;
//   3. recomputes z from the roots (the Gu-Eisenstat product formula), so that the
//      vectors z_i / (d_i - lambda_j) are orthogonal to working precision;
//   4. multiplies the block's eigenvector columns by those vectors and sorts.
//
// Secular iteration (per root): the origin is the nearer end pole of the root's
// interval (decided by the sign of f at the midpoint).  Each step models f as the
// origin's own term w_o / (d_o - x) (exact weight) plus the rest of f replaced by one
// pole matching its value, slope and curvature at the current point (a linear function
// if the rest has no curvature, the fallback when the first model has no root in the
// bracket); the model's root is solved for the offset from the origin directly.  A
// bracket on the root is kept from the signs of f and a step leaving it becomes a
// (geometric, across many orders of magnitude) bisection.  The iteration stops at the
// rounding level of f, when the step is below 2 eps of the offset, or when the bracket
// is exhausted.
#pragma once
#include "common.h"
#include "wg_gemm.h"

// LDS doubles used by wg_tridiag_dc for a matrix of order n.
__host__ __device__ constexpr int dc_lds_doubles(int n) { return 13 * n; }

namespace dcimpl {

constexpr double kEps = 2.220446049250313e-16;

// 1 / x from the hardware reciprocal refined by two Newton steps (error below one ulp
// beyond rounding; x finite and nonzero)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double grp_prod(double x, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) x *= __shfl_xor(x, o, G);
  return x;
}

__device__ __forceinline__ double grp_sum(double x, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
  return x;
}

// root of a x^2 + b x + c0 = 0 strictly inside (lo, hi) closest to t; false if none
__device__ __forceinline__ bool quad_pick(double a, double b, double c0, double t, double lo,
                                          double hi, double* x) {
  double x1, x2;
  if (a == 0.0) {
    if (b == 0.0) return false;
    x1 = -c0 / b;
    x2 = x1;
  } else {
    const double disc = fmax(b * b - 4.0 * a * c0, 0.0);
    const double q = -0.5 * (b + copysign(sqrt(disc), b));
    if (q == 0.0) return false;
    x1 = q / a;
    x2 = c0 / q;
  }
  const bool in1 = lo < x1 && x1 < hi, in2 = lo < x2 && x2 < hi;
  if (in1 && in2) {
    *x = fabs(x1 - t) <= fabs(x2 - t) ? x1 : x2;
    return true;
  }
  if (in1) {
    *x = x1;
    return true;
  }
  if (in2) {
    *x = x2;
    return true;
  }
  return false;
}

// Root j (of k) of 1/rho + sum_i zK_i^2 / (dK_i - lambda) = 0, dK strictly increasing,
// computed by the G lanes of a group (lane g); lambda = dK[org] + tau.  All lanes of the
// group take the same path (butterfly sums are bitwise equal on every lane).
__device__ __forceinline__ void secular_root(int j, int k, const double* dK, const double* zK,
                                             double rho, int g, int G, int* org_out,
                                             double* tau_out) {
  const double irho = 1.0 / rho;
  if (k == 1) {
    *org_out = 0;
    *tau_out = rho * zK[0] * zK[0];
    return;
  }
  int org;
  double lo, hi, tau;
  if (j < k - 1) {
    const double dj = dK[j];
    const double mid = 0.5 * (dK[j + 1] - dj);
    double s = 0.0;
    for (int i = g; i < k; i += G) s += zK[i] * zK[i] * rcp_nr((dK[i] - dj) - mid);
    s = grp_sum(s, G);
    if (irho + s >= 0.0) {
      org = j;
      lo = 0.0;
      hi = mid;
    } else {
      org = j + 1;
      lo = (dj - dK[j + 1]) + mid;
      hi = 0.0;
    }
    tau = 0.5 * (lo + hi);
  } else {
    org = k - 1;
    double zz = 0.0;
    for (int i = g; i < k; i += G) zz += zK[i] * zK[i];
    zz = grp_sum(zz, G);
    const double dl = dK[org];
    lo = 0.0;
    hi = rho * zz;
    for (int t = 0; t < 8; ++t) {  // f(hi) >= 0 up to rounding; widen if not
      double s = 0.0;
      for (int i = g; i < k; i += G) s += zK[i] * zK[i] * rcp_nr((dK[i] - dl) - hi);
      s = grp_sum(s, G);
      if (irho + s >= 0.0) break;
      hi *= 2.0;
    }
    tau = 0.5 * hi;
  }
  const double dorg = dK[org];
  const double wo = zK[org] * zK[org];
  for (int it = 0; it < 64; ++it) {
    double f = 0.0, fa = 0.0, r1 = 0.0, r2 = 0.0;
    for (int i = g; i < k; i += G) {
      const double rr = rcp_nr((dK[i] - dorg) - tau);
      const double t = zK[i] * rr;
      const double term = zK[i] * t;
      f += term;
      fa += fabs(term);
      if (i != org) {
        r1 += t * t;
        r2 += t * t * rr;
      }
    }
    f = grp_sum(f, G);
    fa = grp_sum(fa, G);
    r1 = grp_sum(r1, G);
    r2 = 2.0 * grp_sum(r2, G);
    const double F = irho + f;
    if (!(fabs(F) > 8.0 * kEps * (irho + fa))) break;  // rounding level (or NaN)
    if (F < 0.0)
      lo = tau;
    else
      hi = tau;
    const double R = F + wo / tau;  // f without the origin's term -wo / x, at x = tau
    double tn = 0.0;
    bool ok = false;
    if (r2 != 0.0) {
      const double ap = 2.0 * r1 / r2;  // osculating pole, offset from tau
      const double ds = tau + ap;
      const double S = r1 * ap * ap;
      const double c = R - S / ap;
      ok = quad_pick(-c, wo + S + c * ds, -wo * ds, tau, lo, hi, &tn);
    }
    if (!ok) ok = quad_pick(r1, R - r1 * tau, -wo, tau, lo, hi, &tn);
    if (!ok) {
      tn = 0.5 * (lo + hi);
      if (lo > 0.0 && hi > 1e3 * lo)
        tn = sqrt(lo * hi);
      else if (hi < 0.0 && lo < 1e3 * hi)
        tn = -sqrt(lo * hi);
    }
    const bool small_step = fabs(tn - tau) <= 2.0 * kEps * fabs(tn);
    tau = tn;
    if (small_step || hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi))) break;
  }
  *org_out = org;
  *tau_out = tau;
}

}  // namespace dcimpl

// Eigen-decomposition of the symmetric tridiagonal matrix with diagonal d[0..n) and
// off-diagonal e[i] = T(i+1, i), i < n-1 (e[n-1] is not read), by all threads of the
// workgroup.
//   d  : in: diagonal; out: eigenvalues in ascending order (LDS).
//   W  : n x n output, row-major, W[r*n + a] = component r of eigenvector a (LDS or
//        global; may not alias Wn).
//   Wn : n x n global workspace.
//   v  : LDS workspace of dc_lds_doubles(n) doubles.
// All threads must call it.
__device__ __forceinline__ void wg_tridiag_dc(int n, double* d, const double* e, double* W,
                                              double* Wn, double* v) {
  using namespace dcimpl;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* zs = v;           // z in sorted order; later the merged values
  double* Ds = v + n;       // poles in sorted order
  double* dK = v + 2 * n;   // non-deflated poles (compacted)
  double* zK = v + 3 * n;   // their z (later the recomputed z)
  double* tau = v + 4 * n;  // root offsets
  double* Dd = v + 5 * n;   // deflated values
  double* rc = v + 6 * n;   // deflation rotations: cosines, sines
  double* rs = v + 7 * n;
  int* ps = reinterpret_cast<int*>(v + 8 * n);  // sorted order; later new positions
  int* K = ps + n;     // non-deflated columns (local index in the block)
  int* Kd = K + n;     // deflated columns
  int* org = Kd + n;   // root origins (index into the compacted poles)
  int* rp = org + n;   // rotation column pairs
  int* ri = rp + n;
  int* kc = ri + n;    // per block (at the block's first index): non-deflated count,
  int* dcn = kc + n;   // deflated count, rotation count
  int* rcn = dcn + n;
  double* dorg = Ds;  // after the scan: the roots' origin poles
  double* invn = rc;  // after the rotations: 1 / |u_j|
  // leaves: each coupling is torn out of both adjacent diagonal entries
  for (int i = tid; i < n; i += nt) {
    double di = d[i];
    if (i > 0) di -= fabs(e[i - 1]);
    if (i < n - 1) di -= fabs(e[i]);
    d[i] = di;
  }
  for (i64 t = tid; t < (i64)n * n; t += nt) W[t] = (t / n == t % n) ? 1.0 : 0.0;
  __syncthreads();
  const double r2 = 0.70710678118654752440;
  // lanes per secular root: as many as let one pass cover n roots
  int G = 1;
  int lg = 0;
  while (G < 16 && 2 * G * n <= nt) {
    G *= 2;
    ++lg;
  }
  for (int lb = 0; (1 << lb) < n; ++lb) {
    const int bs = 1 << lb, bw = 2 * bs;  // half and merged block width (bw = 2^(lb+1))
    const int bm = bw - 1, lw = lb + 1;
    // ---- z (from the boundary rows of W) and the sorted order of the poles, scattered
    // by rank (ties by index)
    for (int gc = tid; gc < n; gc += nt) {
      const int s0 = gc & ~bm, c = gc - s0;
      const int s = min(bw, n - s0), n1 = min(bs, s);
      if (s == n1) continue;  // no partner: carried
      const double beta = e[s0 + n1 - 1];
      const double z = c < n1 ? W[(i64)(s0 + n1 - 1) * n + gc] * r2
                              : (beta >= 0.0 ? r2 : -r2) * W[(i64)(s0 + n1) * n + gc];
      const double da = d[gc];
      int rank = 0;
      for (int b = 0; b < s; ++b) {
        const double db = d[s0 + b];
        rank += (db < da || (db == da && b < c)) ? 1 : 0;
      }
      zs[s0 + rank] = z;
      Ds[s0 + rank] = da;
      ps[s0 + rank] = c;
    }
    __syncthreads();
    // ---- deflation scan, one thread per merging block
    for (int s0 = tid * bw; s0 < n; s0 += nt * bw) {
      const int s = min(bw, n - s0), n1 = min(bs, s);
      if (s == n1) continue;
      const double rho = 2.0 * fabs(e[s0 + n1 - 1]);
      double dmax = rho;
      for (int p = 0; p < s; ++p) dmax = fmax(dmax, fabs(Ds[s0 + p]));
      const double tol = 8.0 * kEps * dmax;
      int k = 0, nd = 0, nr = 0, prev = -1;
      double dp = 0.0, zp = 0.0;
      // the next element is loaded before this one's stores (the loads are not held
      // back behind them)
      int i_n = ps[s0];
      double z_n = zs[s0], d_n = Ds[s0];
      for (int p = 0; p < s; ++p) {
        const int i = i_n;
        double zi = z_n, di = d_n;
        const int pn = p + 1 < s ? p + 1 : p;
        i_n = ps[s0 + pn];
        z_n = zs[s0 + pn];
        d_n = Ds[s0 + pn];
        if (rho * fabs(zi) <= tol) {
          Kd[s0 + nd] = i;
          Dd[s0 + nd] = di;
          ++nd;
          continue;
        }
        if (prev >= 0) {
          // the rotation's off-diagonal entry is (di - dp) c s with c s = zi zp / t^2
          const double t2 = zp * zp + zi * zi;
          if (fabs((di - dp) * zi * zp) <= tol * t2) {
            const double t = sqrt(t2);
            const double c = zi / t, sn = zp / t;
            // rotate (prev, i) so that prev's z vanishes; prev is deflated
            rp[s0 + nr] = prev;
            ri[s0 + nr] = i;
            rc[s0 + nr] = c;
            rs[s0 + nr] = sn;
            ++nr;
            Kd[s0 + nd] = prev;
            Dd[s0 + nd] = c * c * dp + sn * sn * di;
            ++nd;
            di = sn * sn * dp + c * c * di;
            zi = t;
            --k;  // prev was the last non-deflated entry
          }
        }
        K[s0 + k] = i;
        dK[s0 + k] = di;
        zK[s0 + k] = zi;
        ++k;
        prev = i;
        dp = di;
        zp = zi;
      }
      kc[s0] = k;
      dcn[s0] = nd;
      rcn[s0] = nr;
    }
    __syncthreads();
    // ---- deflation rotations on the block's eigenvector columns (one thread per row,
    // in order), and the secular roots (one group of G lanes per root)
    for (int gr = tid; gr < n; gr += nt) {
      const int s0 = gr & ~bm;
      const int s = min(bw, n - s0), n1 = min(bs, s);
      if (s == n1) continue;
      const int nr = rcn[s0];
      double* Wr = W + (i64)gr * n + s0;
      for (int q = 0; q < nr; ++q) {
        const int a = rp[s0 + q], b = ri[s0 + q];
        const double c = rc[s0 + q], sn = rs[s0 + q];
        const double wa = Wr[a], wb = Wr[b];
        Wr[a] = c * wa - sn * wb;
        Wr[b] = sn * wa + c * wb;
      }
    }
    {
      const int g = tid & (G - 1);
      for (int gj = tid >> lg; gj < n; gj += nt >> lg) {
        const int s0 = gj & ~bm, j = gj - s0;
        const int s = min(bw, n - s0), n1 = min(bs, s);
        if (s == n1 || j >= kc[s0]) continue;
        int o;
        double t;
        secular_root(j, kc[s0], dK + s0, zK + s0, 2.0 * fabs(e[s0 + n1 - 1]), g, G, &o, &t);
        if (g == 0) {
          org[s0 + j] = o;
          tau[s0 + j] = t;
          dorg[s0 + j] = dK[s0 + o];
        }
      }
    }
    __syncthreads();
    // ---- z recomputed from the roots: z_i^2 = prod_j (lambda_j - d_i) /
    // (rho prod_{j != i} (d_j - d_i)), factors paired so that each is at most one in
    // magnitude; the G lanes of a group take every G-th factor
    {
      const int g = tid & (G - 1);
      for (int gi = tid >> lg; gi < n; gi += nt >> lg) {
        const int s0 = gi & ~bm, i = gi - s0;
        const int s = min(bw, n - s0), n1 = min(bs, s);
        if (s == n1) continue;
        const int k = kc[s0];
        if (i >= k) continue;
        const double* dk = dK + s0;
        const double* tk = tau + s0;
        const double* ok = dorg + s0;
        const double di = dk[i];
        const double rho = 2.0 * fabs(e[s0 + n1 - 1]);
        double pr = g == 0 ? ((ok[k - 1] - di) + tk[k - 1]) * rcp_nr(rho) : 1.0;
        for (int jj = g; jj < i; jj += G) pr *= ((ok[jj] - di) + tk[jj]) * rcp_nr(dk[jj] - di);
        for (int jj = i + g; jj < k - 1; jj += G) pr *= ((ok[jj] - di) + tk[jj]) * rcp_nr(dk[jj + 1] - di);
        pr = grp_prod(pr, G);
        // own element only: no other group reads zK in this phase
        if (g == 0) zK[gi] = copysign(sqrt(fmax(pr, 0.0)), zK[gi]);
      }
    }
    __syncthreads();
    // ---- norms of the rank-one problem's eigenvectors u_j = (z_i / (d_i - lambda_j))_i
    // (their entries are formed again inside the product below); merged values into zs
    {
      const int g = tid & (G - 1);
      for (int gj = tid >> lg; gj < n; gj += nt >> lg) {
        const int s0 = gj & ~bm, j = gj - s0;
        const int s = min(bw, n - s0), n1 = min(bs, s);
        if (s == n1) continue;
        const int k = kc[s0];
        if (j >= k) {
          const int q = j - k;  // deflated value q goes after the k roots
          if (g == 0) zs[gj] = Dd[s0 + q];
          continue;
        }
        const double dl = dorg[gj], tj = tau[gj];
        double nrm = 0.0;
        for (int i = g; i < k; i += G) {
          const double u = zK[s0 + i] * rcp_nr((dK[s0 + i] - dl) - tj);
          nrm += u * u;
        }
        nrm = grp_sum(nrm, G);
        if (g == 0) {
          invn[gj] = 1.0 / sqrt(nrm);
          zs[gj] = dl + tj;
        }
      }
    }
    __syncthreads();
    // ---- positions in ascending order (rank, ties by index) and the new values
    for (int ga = tid; ga < n; ga += nt) {
      const int s0 = ga & ~bm, a = ga - s0;
      const int s = min(bw, n - s0), n1 = min(bs, s);
      if (s == n1) continue;
      const double va = zs[ga];
      int rank = 0;
      for (int b = 0; b < s; ++b) {
        const double vb = zs[s0 + b];
        rank += (vb < va || (vb == va && b < a)) ? 1 : 0;
      }
      ps[ga] = rank;
      d[s0 + rank] = va;
    }
    __syncthreads();
    // ---- new eigenvector columns: Wn(block rows, pos_j) = W(block) U(:, j) for the
    // roots (16 x 16 matrix-core tiles, one wavefront each), deflated columns copied
    {
      const int tpb = (bw + 15) / 16;  // tiles per block side
      const int tiles = ((n + bm) >> lw) * tpb * tpb;
      const int wave = tid >> 6, nwv = nt >> 6;
      for (int T = wave; T < tiles; T += nwv) {
        const int b = T / (tpb * tpb), t = T - b * tpb * tpb;
        const int s0 = b * bw;
        const int s = min(bw, n - s0), n1 = min(bs, s);
        if (s == n1) continue;
        const int k = kc[s0];
        if (16 * (t / tpb) >= s || 16 * (t % tpb) >= k) continue;
        const double* Wb = W + (i64)s0 * n + s0;
        double* Wnb = Wn + (i64)s0 * n + s0;
        const int* pb = ps + s0;
        const int* Kb = K + s0;
        const double *zb = zK + s0, *db = dK + s0, *ob = dorg + s0, *tb = tau + s0, *nb = invn + s0;
        // A = the block's non-deflated columns of W, B(i, j) = z_i / (d_i - lambda_j) / |u_j|
        wave_gemm_tiles(
            s, k, k, tpb, t, t + 1, 1, [&](int r, int i) { return Wb[(i64)r * n + Kb[i]]; },
            [&](int i, int j) { return zb[i] * rcp_nr((db[i] - ob[j]) - tb[j]) * nb[j]; },
            [&](int r, int j, double v) { Wnb[(i64)r * n + pb[j]] = v; });
      }
      for (int it = tid; it < n * bw; it += nt) {
        const int gr = it >> lw, q = it & bm;
        const int s0 = gr & ~bm;
        const int s = min(bw, n - s0), n1 = min(bs, s);
        if (s == n1) continue;
        const int k = kc[s0];
        if (q >= s - k) continue;
        Wn[(i64)gr * n + s0 + ps[s0 + k + q]] = W[(i64)gr * n + s0 + Kd[s0 + q]];
      }
    }
    __syncthreads();
    // ---- merged blocks back into W
    for (int it = tid; it < n * bw; it += nt) {
      const int gr = it >> lw, c = it & bm;
      const int s0 = gr & ~bm;
      const int s = min(bw, n - s0), n1 = min(bs, s);
      if (s == n1 || c >= s) continue;
      W[(i64)gr * n + s0 + c] = Wn[(i64)gr * n + s0 + c];
    }
    __syncthreads();
  }
}
