// Workgroup-parallel dense symmetric eigensolvers: Householder reduction to
// tridiagonal form followed by divide and conquer (wg_syev_dc, for the coarse
// generating systems), and a parallel cyclic Jacobi method for small, nearly diagonal
// matrices (wg_jacobi, for the Rayleigh-Ritz problems of the subspace iteration).
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
    constexpr int NQ = 5;
    if (m <= 32 * NQ) {
      // the thread's columns j = tc + 32 q: v_j and q_j in registers, each row's
      // elements loaded together before the stores
      R vj[NQ], qj[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = tc + 32 * q;
        vj[q] = j < m ? (j == 0 ? v0 : vc[(i64)j * n]) : (R)0;
        qj[q] = j < m ? p[j] - Kc * vj[q] : (R)0;
      }
      for (int i = tr; i < m; i += ng) {
        const R vi = i == 0 ? v0 : vc[(i64)i * n];
        const R qi = p[i] - Kc * vi;
        R* Ar = A + (i64)(k + 1 + i) * n + (k + 1);
        R a[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] = tc + 32 * q < m ? Ar[tc + 32 * q] : (R)0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (tc + 32 * q < m) {
            const R nv = a[q] - (vi * qj[q] + qi * vj[q]);
            Ar[tc + 32 * q] = nv;
            if (q == 0 && tc == 0 && i >= 2) part += nv * nv;
          }
      }
    } else {
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
//        of eigenvector a), as in wg_syev_dc.
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

// wg_jacobi for n = 16 on a single wavefront (the Rayleigh-Ritz problems of the
// 16-column subspace iteration): the same rotations, ordering, skip test (compared in
// squares) and output as wg_jacobi, with the round's pairs computed from constants, the
// rotation from refined hardware reciprocals and reciprocal square roots (two Newton
// steps each), the convergence vote taken with a wavefront ballot, and the 64 2x2 block updates and
// 128 eigenvector-row updates of a round spread one and two per lane.  It synchronises
// within its wavefront only (wave_lds_sync), so it is called by exactly one wavefront
// (lanes threadIdx.x & 63) while the workgroup's other wavefronts wait at a barrier.
//   A, Zt: 16 x 16 (LDS), as for wg_jacobi; prm: 16 doubles of LDS.
__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// LDS hand-off inside one wavefront: its LDS operations complete in order, so waiting
// for its own outstanding ones (and keeping the compiler from moving memory operations
// across) makes every lane's earlier writes visible to every lane's later reads; the
// other wavefronts of the workgroup are not involved.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ double rsqrt_refined(double x) {
  double r = __builtin_amdgcn_rsq(x);
  // r <- r (3 - x r^2) / 2, twice
  r = r * fma(-0.5 * x, r * r, 1.5);
  return r * fma(-0.5 * x, r * r, 1.5);
}
__device__ __forceinline__ int wave_jacobi16(double* A, double* Zt, double* d, double* prm) {
  constexpr int n = 16, h = 8;
  const int lane = threadIdx.x & 63;
  const double tol2 = 1e-32;  // the skip test of wg_jacobi, |a_pq| > 1e-16 sqrt(|a_pp a_qq|), squared
  for (int t = lane; t < n * n; t += 64) Zt[t] = ((t >> 4) == (t & 15)) ? 1.0 : 0.0;
  wave_lds_sync();
  // round r pairs k: k = 0 -> (15, r); else ((r + k) mod 15, (r - k) mod 15)
  auto pair = [](int r, int k, int& p, int& q) {
    if (k == 0) {
      p = n - 1;
      q = r;
    } else {
      p = r + k;
      if (p >= n - 1) p -= n - 1;
      q = r - k;
      if (q < 0) q += n - 1;
    }
  };
  int sweeps = 0;
  for (; sweeps < 40; ++sweeps) {
    bool big = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = lane + 64 * u, p = t >> 4, q = t & 15;
      if (p < q) {
        const double apq = A[t];
        if (apq != 0.0 && apq * apq > tol2 * fabs(A[p * (n + 1)] * A[q * (n + 1)])) big = true;
      }
    }
    if (!__any(big)) break;
    for (int r = 0; r < n - 1; ++r) {
      if (lane < h) {
        int p, q;
        pair(r, lane, p, q);
        const double apq = A[p * n + q], app = A[p * (n + 1)], aqq = A[q * (n + 1)];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && apq * apq > tol2 * fabs(app * aqq)) {
          const double th = (aqq - app) * rcp_refined(2.0 * apq);
          const double at = fabs(th);
          const double w = 1.0 + th * th;
          double t = at > 1e150 ? 0.5 * rcp_refined(at) : rcp_refined(at + w * rsqrt_refined(w));
          if (th < 0) t = -t;
          c = rsqrt_refined(1.0 + t * t);
          s = t * c;
        }
        prm[2 * lane] = c;
        prm[2 * lane + 1] = s;
      }
      wave_lds_sync();
      {
        const int k1 = lane >> 3, k2 = lane & 7;
        int p1, q1, p2, q2;
        pair(r, k1, p1, q1);
        pair(r, k2, p2, q2);
        const double c1 = prm[2 * k1], s1 = prm[2 * k1 + 1], c2 = prm[2 * k2], s2 = prm[2 * k2 + 1];
        const double a = A[p1 * n + p2], b = A[p1 * n + q2], dd = A[q1 * n + p2], e = A[q1 * n + q2];
        const double a1 = c1 * a - s1 * dd, b1 = c1 * b - s1 * e;
        const double d1 = s1 * a + c1 * dd, e1 = s1 * b + c1 * e;
        double a2 = c2 * a1 - s2 * b1, b2 = s2 * a1 + c2 * b1;
        double d2 = c2 * d1 - s2 * e1, e2 = s2 * d1 + c2 * e1;
        if (k1 == k2 && s1 != 0.0) {
          b2 = 0.0;
          d2 = 0.0;
        }
        A[p1 * n + p2] = a2;
        A[p1 * n + q2] = b2;
        A[q1 * n + p2] = d2;
        A[q1 * n + q2] = e2;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int t = lane + 64 * u, k = t >> 4, col = t & 15;
          const double c = prm[2 * k], s = prm[2 * k + 1];
          if (s != 0.0) {
            int p, q;
            pair(r, k, p, q);
            const double zp = Zt[p * n + col], zq = Zt[q * n + col];
            Zt[p * n + col] = c * zp - s * zq;
            Zt[q * n + col] = s * zp + c * zq;
          }
        }
      }
      wave_lds_sync();
    }
  }
  for (int t = lane; t < n; t += 64) d[t] = A[t * (n + 1)];
  wave_lds_sync();
  return sweeps < 40 ? sweeps : -1;
}

#include "tridiag_dc.h"

// LDS doubles of wg_syev_dc's workspace for a matrix of order up to n: the
// tridiagonal solver's (e, then 13 n) and the back-transformation's panel data.
__host__ __device__ constexpr int syev_dc_ws(int n) { return 14 * n > n + 528 ? 14 * n : n + 528; }

// Dense symmetric eigensolver through the tridiagonal divide-and-conquer method:
// Householder reduction (wg_tridiagonalize); the reflectors are moved to Zt's storage;
// the tridiagonal problem is solved by wg_tridiag_dc with its eigenvector matrix W in
// A's storage; then Z = H_0 H_1 ... H_{n-3} W is formed in place, sixteen reflectors at
// a time in compact WY form (Golub and Van Loan, Sec. 5.1.7): for a panel V_b of
// reflectors H_k = I - beta_k v_k v_k^T, H_k0 ... H_k1-1 = I - V_b T V_b^T with
// T^{-1} = S = strict_upper(V_b^T V_b) + diag(1 / beta) (T by one wavefront), so
//   Z <- Z - V_b (T (V_b^T Z)),
// the products on the matrix cores.  Zt = Z^T at the end.
//   A  : n x n symmetric, row-major (LDS or global); destroyed.
//   Zt : n x n output (global), Zt[a*n + k] = component k of eigenvector a.
//   U, Wn : n x n global workspace (distinct from A and Zt).
//   d  : n eigenvalues (LDS), ascending, d[a] belongs to eigenvector a.
//   w  : LDS workspace of syev_dc_ws(n) doubles; red: LDS, >= 48 entries.
// All threads of the workgroup must call it.
__device__ __forceinline__ void wg_syev_dc(int n, double* A, double* Zt, double* U, double* Wn,
                                           double* d, double* w, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, nwv = nt >> 6, lane = tid & 63;
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
  // reflectors: V[k*n + r] = v_k(r) for r > k, V[k*n + k] = beta_k (zero reflector when
  // beta_k = 0); rows k >= n-2 and entries r < k are not read
  double* V = Zt;
  {
    const double* beta = w + n;
    for (i64 t = tid; t < (i64)(n - 2) * n; t += nt) {
      const int k = (int)(t / n), r = (int)(t - (i64)k * n);
      const double bk = beta[k];
      V[t] = r > k ? (bk != 0.0 ? A[(i64)r * n + k] : 0.0) : (r == k ? bk : 0.0);
    }
  }
  __syncthreads();
  wg_tridiag_dc(n, d, w, A, Wn, w + n);
  // W (in A) <- H_0 ... H_{n-3} W, panels from the last
  // the panel's S, T = S^{-1} and beta, in the workspace the tridiagonal solver used
  double* Sl = w + n;
  double* Tl = Sl + 256;
  double* bl = Tl + 256;
  for (int k1 = n - 2; k1 > 0; k1 -= 16) {
    const int k0 = k1 > 16 ? k1 - 16 : 0, nb = k1 - k0;
    const int r0 = k0 + 1, m0 = n - r0;  // rows touched: r0..n-1
    auto vb = [&](int i, int kk) {       // V_b(row r0 + i, reflector k0 + kk)
      const int k = k0 + kk, r = r0 + i;
      return r > k ? V[(i64)k * n + r] : 0.0;
    };
    // wavefront 0: S = V_b^T V_b and T = S^{-1}; the others: Y = V_b^T W(r0:, :) into
    // U (nb x n)
    const int tn = (n + 15) / 16;
    if (wave == 0) {
      wave_gemm_tiles(
          nb, nb, m0, 1, 0, 1, 1, [&](int i, int r) { return vb(r, i); },
          [&](int r, int j) { return vb(r, j); }, [&](int i, int j, double v) { Sl[i * 16 + j] = v; });
      if (lane < nb) bl[lane] = V[(i64)(k0 + lane) * n + k0 + lane];
      // upper triangular inverse, column j by lane j: T(j, j) = beta_j,
      // T(i, j) = -beta_i sum_{i < l <= j} S(i, l) T(l, j)
      if (lane < nb) {
        const int j = lane;
        Tl[j * 16 + j] = bl[j];
#pragma unroll 1
        for (int i = j - 1; i >= 0; --i) {
          double acc = 0.0;
          for (int l = i + 1; l <= j; ++l) acc += Sl[i * 16 + l] * Tl[l * 16 + j];
          Tl[i * 16 + j] = -bl[i] * acc;
        }
      }
    }
    if (wave > 0 || nwv == 1) {  // a lone wavefront does both
      const int w0 = nwv > 1 ? wave - 1 : 0, ws = nwv > 1 ? nwv - 1 : 1;
      wave_gemm_tiles(
          nb, n, m0, tn, w0, tn, ws, [&](int i, int r) { return vb(r, i); },
          [&](int r, int a) { return A[(i64)(r0 + r) * n + a]; },
          [&](int i, int a, double v) { U[(i64)i * n + a] = v; });
    }
    __syncthreads();
    // X = T Y in place (each tile reads its columns of Y before writing them)
    wave_gemm_tiles(
        nb, n, nb, tn, wave, tn, nwv, [&](int i, int l) { return l >= i ? Tl[i * 16 + l] : 0.0; },
        [&](int l, int a) { return U[(i64)l * n + a]; },
        [&](int i, int a, double v) { U[(i64)i * n + a] = v; });
    __syncthreads();
    // W(r0:, :) -= V_b X
    {
      const int tm = (m0 + 15) / 16;
      wave_gemm_tiles(
          m0, n, nb, tn, wave, tm * tn, nwv, [&](int i, int kk) { return vb(i, kk); },
          [&](int kk, int a) { return U[(i64)kk * n + a]; },
          [&](int i, int a, double v) { A[(i64)(r0 + i) * n + a] -= v; });
    }
    __syncthreads();
  }
  for (i64 t = tid; t < (i64)n * n; t += nt) {
    const int a = (int)(t / n), k = (int)(t - (i64)a * n);
    Zt[t] = A[(i64)k * n + a];
  }
  __syncthreads();
}
