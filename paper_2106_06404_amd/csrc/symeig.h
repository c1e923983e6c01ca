// Workgroup-parallel symmetric eigensolver for one dense n x n matrix:
// Householder reduction to tridiagonal form, then implicit QL iteration with
// Wilkinson-type shifts on the tridiagonal matrix (the textbook symmetric QR/QL
// algorithm, Golub and Van Loan, "Matrix Computations", Sec. 8.3), with the
// orthogonal transformations accumulated into the eigenvector matrix.
//
//   A  : n x n symmetric, row-major (LDS or global); overwritten (the Householder
//        vectors are kept in its strictly lower part).
//   Zt : n x n output, eigenvectors stored transposed: Zt[a*n + k] = component k of
//        eigenvector a (so rotations of eigenvector pairs touch two contiguous rows).
//        If Zl is not null, the QL rotations run on the copy Zl (LDS, n x n) and the
//        result is copied to Zt.
//   d  : n eigenvalues (LDS), unsorted, d[a] belongs to eigenvector a.
//   w  : LDS workspace of 6n entries.
// All threads of the workgroup must call it.  Returns the number of QL steps, or -1
// if some eigenvalue needed more than 60 QL steps.
#pragma once
#include "common.h"

// Householder reduction of the n x n symmetric A (row-major, LDS or global) to
// tridiagonal form: d (diagonal), w[0..n) (subdiagonal, e[i] = T(i+1, i), e[n-1] = 0),
// w[n..2n) the Householder scalars (H_k = I - beta_k v_k v_k^T), w[2n..3n) scratch; the
// Householder vectors are left in the strictly lower part of A (v_k in column k, rows
// k+1..n-1).  n >= 2.  red: LDS, >= 48 entries.  Two barriers per column: the
// reflector's norm comes from per-wavefront partial sums taken during the previous
// column's update, and every thread derives the reflector from them itself.
template <typename R>
__device__ __forceinline__ void wg_tridiagonalize(int n, R* A, R* d, R* w, R* red) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6;
  const int nw = (nt + 63) >> 6;
  R* e = w;
  R* beta = w + n;
  R* p = w + 2 * n;
  // norm partials of column 0 below the subdiagonal
  {
    R part = 0;
    for (int i = 2 + tid; i < n; i += nt) part += A[(i64)i * n] * A[(i64)i * n];
    part = wave_sum(part);
    if (lane == 0) red[wv] = part;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // reflector length (rows k+1..n-1)
    const int pb = (k & 1) * 16, pn = 16 - pb;  // norm partials: this column's, the next's
    R sig = 0;
    for (int q = 0; q < nw; ++q) sig += red[pb + q];
    const R x0 = A[(i64)(k + 1) * n + k];
    R bt = 0, alpha = x0, v0 = x0;
    if (sig != (R)0) {
      const R nx = sqrt(x0 * x0 + sig);
      alpha = x0 >= 0 ? -nx : nx;
      v0 = x0 - alpha;
      bt = (R)2 / (v0 * v0 + sig);
    }
    if (tid == 0) {
      e[k] = alpha;
      beta[k] = bt;
    }
    const R* vc = A + (i64)(k + 1) * n + k;  // v_i = vc[i n] for i >= 1, v_0 = v0
    if (bt == (R)0) {  // already reduced: only the next column's partials
      R part = 0;
      for (int i = k + 3 + tid; i < n; i += nt) part += A[(i64)i * n + k + 1] * A[(i64)i * n + k + 1];
      part = wave_sum(part);
      if (lane == 0) red[pn + wv] = part;
      __syncthreads();
      continue;
    }
    // p = bt A_sub v, tpr threads per row; partials of v . p
    int tpr = 1;
    while (tpr < 16 && 2 * tpr * m <= nt) tpr *= 2;
    R vp = 0;
    for (int i0 = 0; i0 < m; i0 += nt / tpr) {
      const int i = i0 + tid / tpr, l = tid & (tpr - 1);
      R acc = 0;
      if (i < m) {
        const R* Ar = A + (i64)(k + 1 + i) * n + (k + 1);
        for (int j = l; j < m; j += tpr) acc += Ar[j] * (j == 0 ? v0 : vc[(i64)j * n]);
      }
      for (int o = tpr >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, tpr);
      if (i < m && l == 0) {
        const R pi = bt * acc;
        p[i] = pi;
        vp += (i == 0 ? v0 : vc[(i64)i * n]) * pi;
      }
    }
    vp = wave_sum(vp);
    if (lane == 0) red[32 + wv] = vp;
    __syncthreads();
    R kp = 0;
    for (int q = 0; q < nw; ++q) kp += red[32 + q];
    const R Kc = (R)0.5 * bt * kp;
    // A_sub -= v q^T + q v^T with q = p - Kc v; 32 columns per row group; the next
    // column's norm partials from the updated values
    R part = 0;
    const int tr = tid >> 5, tc = tid & 31, ng = nt >> 5;
    for (int i = tr; i < m; i += ng) {
      const R vi = i == 0 ? v0 : vc[(i64)i * n];
      const R qi = p[i] - Kc * vi;
      R* Ar = A + (i64)(k + 1 + i) * n + (k + 1);
      for (int j = tc; j < m; j += 32) {
        const R vj = j == 0 ? v0 : vc[(i64)j * n];
        const R nv = Ar[j] - (vi * (p[j] - Kc * vj) + qi * vj);
        Ar[j] = nv;
        if (j == 0 && i >= 2) part += nv * nv;
      }
    }
    part = wave_sum(part);
    if (lane == 0) red[pn + wv] = part;
    if (tid == 0) A[(i64)(k + 1) * n + k] = v0;  // v stored in column k below the diagonal
    __syncthreads();
  }
  for (int i = tid; i < n; i += nt) d[i] = A[(i64)i * n + i];
  if (tid == 0) {
    e[n - 2] = A[(i64)(n - 1) * n + (n - 2)];
    beta[n - 2] = 0;
    e[n - 1] = 0;
  }
  __syncthreads();
}

// Q = H_0 H_1 ... H_{n-3} from the reflectors left by wg_tridiagonalize, stored
// transposed in Zt (Zt[a*n + k] = Q(k, a)); applied backwards, two barriers per
// reflector.  All threads must call it.
template <typename R>
__device__ __forceinline__ void wg_accumulate_q(int n, const R* A, R* Zt, R* w) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const R* beta = w + n;
  R* sn = w + 2 * n;
  for (i64 t = tid; t < (i64)n * n; t += nt) Zt[t] = (t / n == t % n) ? (R)1 : (R)0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const R bt = beta[k];
    if (bt == (R)0) continue;
    const int m = n - k - 1;
    const R* vc = A + (i64)(k + 1) * n + k;  // v_r = vc[r n]
    // Q[k+1:, k+1:] -= bt v (v^T Q[k+1:, k+1:]):  sn_c = bt v . Zt[c][k+1:]
    int tpr = 1;
    while (tpr < 16 && 2 * tpr * m <= nt) tpr *= 2;
    for (int c0 = 0; c0 < m; c0 += nt / tpr) {
      const int c = c0 + tid / tpr, l = tid & (tpr - 1);
      R acc = 0;
      if (c < m) {
        const R* Zr = Zt + (i64)(k + 1 + c) * n + (k + 1);
        for (int r = l; r < m; r += tpr) acc += Zr[r] * vc[(i64)r * n];
      }
      for (int o = tpr >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, tpr);
      if (c < m && l == 0) sn[c] = bt * acc;
    }
    __syncthreads();
    const int tr = tid >> 5, tc = tid & 31, ng = nt >> 5;
    for (int c = tr; c < m; c += ng) {
      const R sc = sn[c];
      R* Zr = Zt + (i64)(k + 1 + c) * n + (k + 1);
      for (int r = tc; r < m; r += 32) Zr[r] -= sc * vc[(i64)r * n];
    }
    __syncthreads();
  }
}

template <typename R>
__device__ __forceinline__ int wg_syev(int n, R* A, R* Zt, R* Zl, R* d, R* w, R* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  R* e = w;          // subdiagonal: e[i] = T(i+1, i)
  __shared__ int sh_state[5];  // l, m, lo, iterations at l, failed
  if (n == 1) {
    if (tid == 0) {
      d[0] = A[0];
      Zt[0] = (R)1;
    }
    __syncthreads();
    return 0;
  }
  wg_tridiagonalize(n, A, d, w, red);
  wg_accumulate_q(n, A, Zt, w);
  // the QL rotations run on the LDS copy Zl when there is one
  if (Zl) {
    for (i64 t = tid; t < (i64)n * n; t += nt) Zl[t] = Zt[t];
    __syncthreads();
  }
  // ---- 3. implicit QL on (d, e).  Wavefront 0 runs the control: it finds the next
  // unreduced block with a wave-wide scan of e (deflation test relative to the norm of
  // T: absolute accuracy eps ||A|| for every eigenvalue; a test relative to the
  // neighbouring diagonal entries can stall on clusters near zero) and one lane computes
  // the step's rotations, a dependent chain, with its loads issued one rotation ahead.
  // The other wavefronts apply the previous step's rotations to the rows of Z
  // meanwhile (rotation arrays double buffered), so a step costs the longer of the two.
  const R eps = (R)2.220446049250313e-16;
  __shared__ R sh_tnorm;
  __shared__ int q_m[2], q_lo[2], q_has[2];
  // rotation buffer b: cosines at w + (2 + 2b) n, sines at w + (3 + 2b) n (offsets from w,
  // so that the compiler keeps them in the LDS address space)
  if (tid == 0) {
    R tn = 0;
    for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(d[i]) + fabs(e[i]));
    sh_tnorm = tn;
    sh_state[4] = 0;
  }
  __syncthreads();
  const R thr = eps * sh_tnorm;
  const int lane = tid & 63;
  // wavefront-0 state (uniform over its lanes)
  int ql_l = 0, ql_it = 0, ql_failed = 0;
  // one QL step into buffer b (wavefront 0 only); q_has[b] = 0 when all have converged
  auto ql_step = [&](int b) {
    int m = 0;
    while (ql_l < n) {
      // first m >= l with |e[m]| <= thr, or n - 1
      m = -1;
      for (int base = ql_l; base < n - 1 && m < 0; base += 64) {
        const int idx = base + lane;
        const bool hit = idx >= n - 1 || fabs(e[idx]) <= thr;
        const unsigned long long mk = __ballot(hit);
        if (mk) m = base + __ffsll((long long)mk) - 1;
      }
      if (m < 0 || m > n - 1) m = n - 1;
      if (m == ql_l || ql_it >= 60) {  // eigenvalue l converged (or given up)
        if (m != ql_l) ql_failed = 1;
        ++ql_l;
        ql_it = 0;
        continue;
      }
      break;
    }
    if (ql_l >= n) {
      if (lane == 0) q_has[b] = 0;
      return;
    }
    ++ql_it;
    const int l = ql_l;
    if (lane == 0) {
      R* cb = w + (2 + 2 * b) * n;
      R* sb = cb + n;
      R g = (d[l + 1] - d[l]) / ((R)2 * e[l]);
      R r = sqrt(g * g + (R)1);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      R s = 1, c = 1, p = 0;
      int i = m - 1, lo = l;
      R ei = e[i], di = d[i], di1 = d[i + 1];
      for (; i >= l; --i) {
        // values of the next rotation, loaded before this one's stores (they are not
        // written by it)
        const int ip = i > 0 ? i - 1 : 0;  // unconditional (clamped) loads, no branch
        const R en = e[ip];
        const R dn = d[ip];
        const R f = s * ei, bb = c * ei;
        // r = sqrt(f^2 + g^2), s = f / r, c = g / r through one reciprocal square root:
        // the rotation chain is the critical path of the whole solver, and this halves
        // its dependent latency against a square root and two divisions
        const R q = f * f + g * g;
        if (q == (R)0) {  // deflation inside the sweep
          e[i + 1] = 0;
          d[i + 1] = di1 - p;
          e[m] = 0;
          lo = i + 1;
          break;
        }
        const R ri = rsqrt(q);
        r = q * ri;
        e[i + 1] = r;
        s = f * ri;
        c = g * ri;
        g = di1 - p;
        r = (di - g) * s + (R)2 * c * bb;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - bb;
        cb[i] = c;
        sb[i] = s;
        di1 = di;
        ei = en;
        di = dn;
      }
      if (i < l) {
        d[l] -= p;
        e[l] = g;
        e[m] = 0;
      }
      q_m[b] = m;
      q_lo[b] = lo;
      q_has[b] = 1;
    }
  };
  if (tid < 64) ql_step(0);
  __syncthreads();
  int steps = 0, cur = 0;
  while (q_has[cur]) {
    if (tid < 64) {
      ql_step(cur ^ 1);
    } else {
      // rotations i = m-1 down to lo on eigenvector rows (i, i+1) of Z (transposed),
      // eight at a time with their operands loaded first; Z is the LDS copy when there
      // is one (two call sites, so that each keeps its address space)
      const int m = q_m[cur], lo = q_lo[cur];
      const R* cb = w + (2 + 2 * cur) * n;
      const R* sb = cb + n;
      auto apply = [&](R* Z) {
        for (int k = tid - 64; k < n; k += nt - 64) {
          R zi1 = Z[(i64)m * n + k];
          for (int i0 = m - 1; i0 >= lo; i0 -= 8) {
            const int cnt = min(8, i0 - lo + 1);
            R zb[8], cv[8], sv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (u < cnt) {
                zb[u] = Z[(i64)(i0 - u) * n + k];
                cv[u] = cb[i0 - u];
                sv[u] = sb[i0 - u];
              }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (u < cnt) {
                Z[(i64)(i0 - u + 1) * n + k] = sv[u] * zb[u] + cv[u] * zi1;
                zi1 = cv[u] * zb[u] - sv[u] * zi1;
              }
          }
          Z[(i64)lo * n + k] = zi1;
        }
      };
      if (Zl)
        apply(Zl);
      else
        apply(Zt);
    }
    __syncthreads();
    cur ^= 1;
    ++steps;
  }
  if (tid == 0) sh_state[4] = ql_failed;
  __syncthreads();
  if (Zl) {
    for (i64 t = tid; t < (i64)n * n; t += nt) Zt[t] = Zl[t];
    __syncthreads();
  }
  return sh_state[4] ? -1 : steps;
}

// Workgroup-parallel cyclic Jacobi eigensolver for one small symmetric matrix
// (n even, n <= 64): the round-robin ("tournament") ordering gives n/2 disjoint
// rotation planes per round, each annihilating one off-diagonal pair with the
// symmetric Schur rotation (Golub and Van Loan, Sec. 8.5); the n/2 rotations of a
// round are applied together as 2x2 block updates of A, so one round costs one
// parallel rotation step.  A matrix that is nearly diagonal already (the Gram
// matrices of a subspace iteration close to convergence) finishes in one or two
// sweeps.
//   A  : n x n symmetric, row-major (LDS); overwritten, its diagonal holds the
//        eigenvalues on return.
//   Zt : n x n output (LDS), eigenvectors stored transposed (Zt[a*n + k] = component k
//        of eigenvector a), as in wg_syev.
//   d  : n eigenvalues, unsorted.
// A rotation is skipped when |a_pq| <= 1e-16 sqrt(|a_pp a_qq|) (relative test:
// graded eigenvalues keep their relative accuracy).  All threads must call it.
// Returns the number of sweeps, or -1 after 40 sweeps without convergence.
template <typename R>
__device__ __forceinline__ int wg_jacobi(int n, R* A, R* Zt, R* d) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ R rc[64], rs[64];
  __shared__ int pp[32], pq[32];
  __shared__ int sh_flag;
  const R tol = (R)1e-16;
  const int h = n / 2;
  for (int t = tid; t < n * n; t += nt) Zt[t] = (t / n == t % n) ? (R)1 : (R)0;
  int sweeps = 0;
  for (; sweeps < 40; ++sweeps) {
    // convergence test over all off-diagonal pairs
    if (tid == 0) sh_flag = 0;
    __syncthreads();
    int any = 0;
    for (int t = tid; t < n * n; t += nt) {
      const int p = t / n, q = t - p * n;
      if (p < q) {
        const R apq = A[t];
        if (apq != (R)0 && fabs(apq) > tol * sqrt(fabs(A[p * n + p] * A[q * n + q]))) any = 1;
      }
    }
    if (any) sh_flag = 1;
    __syncthreads();
    if (!sh_flag) break;
    for (int r = 0; r < n - 1; ++r) {
      // rotation of each pair of this round
      for (int k = tid; k < h; k += nt) {
        int p, q;
        if (k == 0) {
          p = n - 1;
          q = r;
        } else {
          p = (r + k) % (n - 1);
          q = (r - k + n - 1) % (n - 1);
        }
        const R apq = A[p * n + q], app = A[p * n + p], aqq = A[q * n + q];
        R c = 1, s = 0;
        if (apq != (R)0 && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
          const R th = (aqq - app) / ((R)2 * apq);
          const R at = fabs(th);
          // t = sign(th) / (|th| + sqrt(1 + th^2)), the smaller root
          R t = at > (R)1e150 ? (R)0.5 / at : (R)1 / (at + sqrt((R)1 + th * th));
          if (th < 0) t = -t;
          c = (R)1 / sqrt((R)1 + t * t);
          s = t * c;
        }
        pp[k] = p;
        pq[k] = q;
        rc[k] = c;
        rs[k] = s;
      }
      __syncthreads();
      // A <- G^T A G as 2x2 blocks (row pair k1, column pair k2)
      for (int t = tid; t < h * h; t += nt) {
        const int k1 = t / h, k2 = t - k1 * h;
        const int p1 = pp[k1], q1 = pq[k1], p2 = pp[k2], q2 = pq[k2];
        const R c1 = rc[k1], s1 = rs[k1], c2 = rc[k2], s2 = rs[k2];
        const R a = A[p1 * n + p2], b = A[p1 * n + q2], dd = A[q1 * n + p2], e = A[q1 * n + q2];
        const R a1 = c1 * a - s1 * dd, b1 = c1 * b - s1 * e;
        const R d1 = s1 * a + c1 * dd, e1 = s1 * b + c1 * e;
        R a2 = c2 * a1 - s2 * b1, b2 = s2 * a1 + c2 * b1;
        R d2 = c2 * d1 - s2 * e1, e2 = s2 * d1 + c2 * e1;
        if (k1 == k2 && s1 != (R)0) {
          b2 = 0;
          d2 = 0;
        }
        A[p1 * n + p2] = a2;
        A[p1 * n + q2] = b2;
        A[q1 * n + p2] = d2;
        A[q1 * n + q2] = e2;
      }
      // Zt <- G^T Zt (rows p, q)
      for (int t = tid; t < h * n; t += nt) {
        const int k = t / n, col = t - k * n;
        const R c = rc[k], s = rs[k];
        if (s == (R)0) continue;
        const int p = pp[k], q = pq[k];
        const R zp = Zt[p * n + col], zq = Zt[q * n + col];
        Zt[p * n + col] = c * zp - s * zq;
        Zt[q * n + col] = s * zp + c * zq;
      }
      __syncthreads();
    }
  }
  for (int t = tid; t < n; t += nt) d[t] = A[t * n + t];
  __syncthreads();
  return sweeps < 40 ? sweeps : -1;
}

#include "tridiag_dc.h"

// Dense symmetric eigensolver through the tridiagonal divide-and-conquer method:
// Householder reduction (wg_tridiagonalize), Q accumulated (wg_accumulate_q), the
// tridiagonal problem solved by wg_tridiag_dc with its eigenvector matrix W kept in A's
// storage (free once Q is formed), and Zt = (Q W)^T.
//   A  : n x n symmetric, row-major (LDS or global); destroyed.
//   Zt : n x n output (global), Zt[a*n + k] = component k of eigenvector a.
//   U, Wn : n x n global workspace (distinct from A and Zt).
//   d  : n eigenvalues (LDS), ascending, d[a] belongs to eigenvector a.
//   w  : LDS workspace of 14n doubles; red: LDS, >= 48 entries.
// All threads of the workgroup must call it.
__device__ __forceinline__ void wg_syev_dc(int n, double* A, double* Zt, double* U, double* Wn,
                                           double* d, double* w, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (n <= 0) return;
  if (n == 1) {
    if (tid == 0) {
      d[0] = A[0];
      Zt[0] = 1.0;
    }
    __syncthreads();
    return;
  }
  wg_tridiagonalize(n, A, d, w, red);
  wg_accumulate_q(n, A, Zt, w);
  wg_tridiag_dc(n, d, w, A, U, Wn, w + n);
  // Wn[a*n + k] = sum_b Q(k, b) W(b, a) = sum_b Zt[b*n + k] A[b*n + a], 4 x 4 tiles
  const int tp = (n + 3) / 4;
  for (int it = tid; it < tp * tp; it += nt) {
    const int a0 = 4 * (it / tp), k0 = 4 * (it % tp);
    const int amax = min(4, n - a0), kmax = min(4, n - k0);
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
#pragma unroll 2
    for (int b = 0; b < n; ++b) {
      double wv[4], qv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) wv[x] = x < amax ? A[(i64)b * n + a0 + x] : 0.0;
#pragma unroll
      for (int y = 0; y < 4; ++y) qv[y] = y < kmax ? Zt[(i64)b * n + k0 + y] : 0.0;
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += wv[x] * qv[y];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
      if (x < amax)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          if (y < kmax) Wn[(i64)(a0 + x) * n + k0 + y] = acc[x][y];
  }
  __syncthreads();
  for (i64 t = tid; t < (i64)n * n; t += nt) Zt[t] = Wn[t];
  __syncthreads();
}
