// Finest-level local generalized eigenproblems (Sec. 2.3 "theGEVP", b^1 of
// Sec. 3.4), batched over subdomains.
//
// abar x = lambda b x,  b = D abar D  (D = partition-of-unity weights).
// The lemma of Sec. 3.3 (ker abar cap ker b = {0}) makes S = abar + sigma*b SPD
// for every sigma > 0, and the wanted smallest lambda are the largest
//   nu = 1/(lambda + sigma)  of  b x = nu S x.
// Block subspace iteration with the exact factor of S (shift-invert) and a
// Rayleigh-Ritz step per iteration:
//   Y = S^{-1} (B X);  Z = B Y;  G_S = Y^T (B X) (= Y^T S Y);  G_B = Y^T Z;
//   G_B c = nu G_S c;  X <- Y C,  BX <- Z C,  SX <- (B X_old) C.
// Convergence of a selected pair: the normwise backward error
// ||BX_j - nu_j SX_j|| / (nu_j ||S|| ||X_j||) is <= tol, and the energy residual of the
// previous Ritz pair (nu, x), x^T S x = 1,
//   eps = ||S^{-1} b x - nu x||_S,  eps^2 = (y - nu x)^T (b x - nu S x),  y = S^{-1} b x,
// is <= tol_e nu (y is the next block before the Rayleigh-Ritz step).  eps bounds the
// S-angle between x and the eigenvector (sin <= eps / gap), which the normwise test does
// not: at high coefficient contrast ||S|| is set by the high-coefficient rows and a vector
// whose error lies in the low-coefficient region passes it while still off by 1e-7.  The
// pair after the selected ones only certifies the count m; as a safety net a pair also
// counts as converged when its residuals have stopped falling and its Ritz value no
// longer moves (relative change <= 1e-14).
#include "common.h"
#include "symeig.h"
#include "kernels.h"

__device__ inline double hash_uniform(unsigned long long x) {
  // splitmix64 finaliser -> uniform in [-1, 1)
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// deterministic start block (rows with zero weight get zero: they lie in ker b)
template <typename V>
__global__ void k_eig_init(i64 total_rows, const i32* __restrict__ row_sub,
                           const i64* __restrict__ voff, const i32* __restrict__ nb,
                           const i64* __restrict__ kvoff, int K, const double* __restrict__ dv,
                           V* __restrict__ X, unsigned long long seed,
                           const i32* __restrict__ seed_id) {
  i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int i = row_sub[g];
  const int r = (int)(g - voff[i]);
  const int n = nb[i];
  V* Xi = X + kvoff[i];
  const bool z = dv[g] == 0.0;
  // the start block depends on the subdomain's index within its problem, so a problem
  // gets the same start whether it is set up alone or in a batch
  const unsigned long long sid = (unsigned long long)seed_id[i];
  for (int c = 0; c < K; ++c) {
    unsigned long long key = seed ^ (sid << 40) ^ ((unsigned long long)r << 12) ^
                             (unsigned long long)c;
    Xi[r + (i64)c * n] = z ? (V)0 : (V)hash_uniform(key);
  }
}

// Z = D abar D Y  with the symmetric ELL copy of abar (full rows)
template <typename V>
__global__ void k_bapply_ell(i64 total_rows, const i32* __restrict__ row_sub,
                             const i64* __restrict__ voff, const i32* __restrict__ nb,
                             const i64* __restrict__ kvoff, int K, const double* __restrict__ dv,
                             int ell_w, const i32* __restrict__ ell_col,
                             const double* __restrict__ ell_val, const V* __restrict__ Y,
                             V* __restrict__ Z, const int* __restrict__ active) {
  i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int i = row_sub[g];
  if (active && active[i] != ST_RUNNING) return;
  const int r = (int)(g - voff[i]);
  const int n = nb[i];
  const V* Yi = Y + kvoff[i];
  V* Zi = Z + kvoff[i];
  const double* d = dv + voff[i];
  const double dr = d[r];
  if (dr == 0.0) {
    for (int c = 0; c < K; ++c) Zi[r + (i64)c * n] = 0;
    return;
  }
  const i32* ec = ell_col + g * ell_w;
  const double* ev = ell_val + g * ell_w;
  // padding entries (column -1) are read as column 0 with coefficient 0, so the loop has
  // no data-dependent exits and the loads of different entries can be issued together
  constexpr int CB = 16;
  for (int c0 = 0; c0 < K; c0 += CB) {
    V acc[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) acc[u] = 0;
    for (int t = 0; t < ell_w; ++t) {
      const int c_raw = ec[t];
      const int cc = c_raw < 0 ? 0 : c_raw;
      const V a = c_raw < 0 ? (V)0 : (V)(ev[t] * d[cc]);
      const V* yc = Yi + cc + (i64)c0 * n;
#pragma unroll
      for (int u = 0; u < CB; ++u)
        if (c0 + u < K) acc[u] += a * yc[(i64)u * n];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u)
      if (c0 + u < K) Zi[r + (i64)(c0 + u) * n] = (V)(dr * acc[u]);
  }
}

// The same product with the columns staged in LDS: workgroup (i, j) computes rows
// 256 j .. 256 j + 255 of subdomain i; the rows it reads (those within the
// half-bandwidth b of its own) are loaded once per group of 16 columns, coalesced, into
// LDS (column-major, tile[u * rows + row - lo]), instead of every row fetching its
// neighbours' values from L2 (each value is read by about nine rows).
__global__ void __launch_bounds__(256) k_bapply_tile(
    const i64* __restrict__ voff, const i32* __restrict__ nb, const i32* __restrict__ bw,
    const i64* __restrict__ kvoff, int K, const double* __restrict__ dv, int ell_w,
    const i32* __restrict__ ell_col, const double* __restrict__ ell_val,
    const double* __restrict__ Y, double* __restrict__ Z, const int* __restrict__ active) {
  extern __shared__ double tile[];
  const int i = blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = nb[i];
  const int r0 = blockIdx.y * 256;
  if (r0 >= n) return;
  const int b = bw[i];
  const int lo = max(0, r0 - b), hi = min(n, r0 + 256 + b);
  const int rows = hi - lo;
  const double* Yi = Y + kvoff[i];
  double* Zi = Z + kvoff[i];
  const double* d = dv + voff[i];
  const int r = r0 + threadIdx.x;
  const bool own = r < n;
  const i64 g = voff[i] + (own ? r : 0);
  const i32* ec = ell_col + g * ell_w;
  const double* ev = ell_val + g * ell_w;
  const double dr = own ? d[r] : 0.0;
  for (int c0 = 0; c0 < K; c0 += 16) {
    const int kc = min(16, K - c0);
    __syncthreads();  // the previous group's reads of the tile are done
    for (int e = threadIdx.x; e < kc * rows; e += 256) {
      const int u = e / rows, rr = e - u * rows;
      tile[u * rows + rr] = Yi[(i64)(c0 + u) * n + lo + rr];
    }
    __syncthreads();
    if (!own) continue;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    if (dr != 0.0) {
      // padding entries (column -1) read this row's own values with coefficient 0
      for (int t = 0; t < ell_w; ++t) {
        const int c_raw = ec[t];
        const int cc = c_raw < 0 ? r : c_raw;
        const double a = c_raw < 0 ? 0.0 : ev[t] * d[cc];
        const double* tc = tile + (cc - lo);
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (u < kc) acc[u] += a * tc[u * rows];
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (u < kc) Zi[r + (i64)(c0 + u) * n] = dr * acc[u];
  }
}

// ||S||_inf estimate per subdomain: max row sum of |abar| (1 + sigma d_r d_c)
__global__ void k_row_norm(const i64* __restrict__ voff, int ell_w, const i32* __restrict__ ell_col,
                           const double* __restrict__ ell_val, const double* __restrict__ dv,
                           double sigma, double* __restrict__ normS,
                           const double* __restrict__ ell_val2) {
  const int i = blockIdx.x;
  const i64 r0 = voff[i], r1 = voff[i + 1];
  double mx = 0.0;
  for (i64 g = r0 + threadIdx.x; g < r1; g += blockDim.x) {
    double s = 0.0;
    const double dr = dv[g];
    for (int t = 0; t < ell_w; ++t) {
      const int c = ell_col[g * ell_w + t];
      if (c < 0) break;
      s += ell_val2 ? fabs(ell_val[g * ell_w + t] + sigma * dr * dv[r0 + c] * ell_val2[g * ell_w + t])
                    : fabs(ell_val[g * ell_w + t]) * (1.0 + sigma * dr * dv[r0 + c]);
    }
    mx = fmax(mx, s);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
    normS[i] = m;
  }
}

// G_S = Y^T W, G_B = Y^T Z (K x K each, double), one workgroup per subdomain
template <typename V, int TR>
__global__ void k_gram(const i32* __restrict__ nb, const i64* __restrict__ kvoff, int K,
                       const V* __restrict__ Y, const V* __restrict__ W, const V* __restrict__ Z,
                       double* __restrict__ GS, double* __restrict__ GB,
                       const int* __restrict__ active, int S) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x, sp = blockIdx.y;  // subdomain, row split
  if (active && active[i] != ST_RUNNING) return;
  const int n = nb[i];
  const int chunk = ((n + S - 1) / S + TR - 1) / TR * TR;
  const int r_lo = sp * chunk, r_hi = min(n, r_lo + chunk);
  V* ty = reinterpret_cast<V*>(smem_raw);
  V* tw = ty + TR * K;
  V* tz = tw + TR * K;
  const V* Yi = Y + kvoff[i];
  const V* Wi = W + kvoff[i];
  const V* Zi = Z + kvoff[i];
  const int KK = K * K;
  constexpr int MAXP = 16;  // K <= 64 -> K*K/256 <= 16 pairs per thread
  double as[MAXP], ab[MAXP];
  for (int u = 0; u < MAXP; ++u) as[u] = ab[u] = 0.0;
  for (int r0 = r_lo; r0 < r_hi; r0 += TR) {
    const int rn = min(TR, r_hi - r0);
    __syncthreads();
    for (int t = threadIdx.x; t < TR * K; t += blockDim.x) {
      const int c = t / TR, rr = t % TR;
      V y = 0, w = 0, z = 0;
      if (rr < rn) {
        const i64 idx = r0 + rr + (i64)c * n;
        y = Yi[idx];
        w = Wi[idx];
        z = Zi[idx];
      }
      ty[rr * K + c] = y;
      tw[rr * K + c] = w;
      tz[rr * K + c] = z;
    }
    __syncthreads();
    int u = 0;
    for (int t = threadIdx.x; t < KK; t += blockDim.x, ++u) {
      const int a = t / K, bcol = t % K;
      double s1 = 0, s2 = 0;
      for (int rr = 0; rr < rn; ++rr) {
        const double y = (double)ty[rr * K + a];
        s1 += y * (double)tw[rr * K + bcol];
        s2 += y * (double)tz[rr * K + bcol];
      }
      as[u] += s1;
      ab[u] += s2;
    }
  }
  // partial Gram matrices of this row split (an empty split writes zeros)
  int u = 0;
  const i64 o = ((i64)i * S + sp) * KK;
  for (int t = threadIdx.x; t < KK; t += blockDim.x, ++u) {
    GS[o + t] = as[u];
    GB[o + t] = ab[u];
  }
}

// Rayleigh-Ritz: G_B c = nu G_S c  ->  C (K x K, row-major), nu (descending).
// Robust to a rank-deficient G_S: a Cholesky factorisation of the diagonally scaled
// G_S drops the columns that depend on earlier ones (they get nu = 0 and a zero
// column); the projected standard problem is solved by cyclic Jacobi.
__global__ void k_rayleigh_ritz(int K, const double* __restrict__ GS,
                                const double* __restrict__ GB, double* __restrict__ Cout,
                                double* __restrict__ nu_out, const int* __restrict__ active,
                                int nsplit, double* __restrict__ gs_diag) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int KK = K * K;
  double* S = reinterpret_cast<double*>(smem_raw);  // K*K
  double* U = S + KK;                                // K*K
  double* M = U + KK;                                // K*K
  double* sc = M + KK;                               // K  (diagonal scaling)
  double* ev = sc + K;                               // K
  double* wsp = ev + K;                              // 4K (eigensolver workspace)
  int* ord = reinterpret_cast<int*>(wsp + 4 * K);    // K
  const int tid = threadIdx.x, nt = blockDim.x;
  // G_S and G_B arrive as nsplit partial sums over row splits
  const double* gs = GS + (i64)i * nsplit * KK;
  const double* gb = GB + (i64)i * nsplit * KK;
  for (int t = tid; t < KK; t += nt) {
    double a = 0.0;
    for (int q = 0; q < nsplit; ++q) a += gs[(i64)q * KK + t];
    S[t] = a;
  }
  __syncthreads();
  for (int t = tid; t < K; t += nt) {
    const double dgs = S[t * K + t];
    // y_t^T S y_t = ||S^{-1} b x_t||_S^2 for the previous Ritz vector x_t (error bound)
    gs_diag[(i64)i * K + t] = dgs;
    sc[t] = dgs > 0 ? 1.0 / sqrt(dgs) : 0.0;
  }
  __syncthreads();
  for (int t = tid; t < KK; t += nt) {  // symmetrise and scale (each pair by one thread)
    const int a = t / K, b = t % K;
    if (a <= b) {
      const double v = 0.5 * (S[a * K + b] + S[b * K + a]) * sc[a] * sc[b];
      S[a * K + b] = v;
      S[b * K + a] = v;
    }
  }
  __syncthreads();
  // scaled G_S = L L^T by a Cholesky factorisation that drops dependent columns: a
  // column whose pivot (its squared G_S-distance from the span of the kept earlier
  // columns, relative to its own G_S-norm, which the scaling makes 1) is <= 1e-13
  // gets a zero column in L.  L overwrites the lower triangle of S; ord[j] = kept.
  for (int j = 0; j < K; ++j) {
    if (tid == 0) {
      const double dj = S[j * K + j];
      ord[j] = dj > 1e-13;
      S[j * K + j] = dj > 1e-13 ? sqrt(dj) : 0.0;
    }
    __syncthreads();
    const double ljj = S[j * K + j];
    for (int r = j + 1 + tid; r < K; r += nt) S[r * K + j] = ljj > 0.0 ? S[r * K + j] / ljj : 0.0;
    __syncthreads();
    const int m = K - j - 1;
    for (int t = tid; t < m * m; t += nt) {
      const int r = j + 1 + t / m, c = j + 1 + t % m;
      if (c <= r) S[r * K + c] -= S[r * K + j] * S[c * K + j];
    }
    __syncthreads();
  }
  // Z = L^{-1} (rows of dropped columns are zero), row by row into M
  for (int a = 0; a < K; ++a) {
    for (int c = tid; c < K; c += nt) {
      double z = 0.0;
      if (ord[a] && c <= a) {
        double acc = c == a ? 1.0 : 0.0;
        for (int k = c; k < a; ++k) acc -= S[a * K + k] * M[k * K + c];
        z = acc / S[a * K + a];
      }
      M[a * K + c] = z;
    }
    __syncthreads();
  }
  // T = diag(sc) L^{-T} in U: T^T G_S T = I on the kept columns, zero columns elsewhere
  for (int t = tid; t < KK; t += nt) {
    const int r = t / K, a = t % K;
    U[t] = sc[r] * M[a * K + r];
  }
  __syncthreads();
  // M = T^T GB T: GB (summed, symmetrised) into M, then S <- GB T, then M = T^T S
  for (int t = tid; t < KK; t += nt) {
    double a = 0.0;
    for (int q = 0; q < nsplit; ++q) a += gb[(i64)q * KK + t];
    M[t] = a;
  }
  __syncthreads();
  for (int t = tid; t < KK; t += nt) {
    const int a = t / K, b = t % K;
    if (a < b) {
      const double v = 0.5 * (M[a * K + b] + M[b * K + a]);
      M[a * K + b] = v;
      M[b * K + a] = v;
    }
  }
  __syncthreads();
  for (int t = tid; t < KK; t += nt) {
    const int r = t / K, a = t % K;
    double acc = 0;
    for (int q = 0; q < K; ++q) acc += M[r * K + q] * U[q * K + a];
    S[t] = acc;
  }
  __syncthreads();
  for (int t = tid; t < KK; t += nt) {
    const int a = t / K, b = t % K;
    double acc = 0;
    for (int q = 0; q < K; ++q) acc += U[q * K + a] * S[q * K + b];
    M[t] = acc;
  }
  __syncthreads();
  for (int t = tid; t < KK; t += nt) {
    const int a = t / K, b = t % K;
    if (a < b) {
      const double v = 0.5 * (M[a * K + b] + M[b * K + a]);
      M[a * K + b] = v;
      M[b * K + a] = v;
    }
  }
  __syncthreads();
  // M = Q diag(ev) Q^T, eigenvectors transposed into S (S[a*K + q] = Q(q, a))
  if (K == 16 && nt >= 64) {
    // the 16 x 16 Jacobi runs in wavefront 0 (it synchronises within the wavefront only)
    if (tid < 64) wave_jacobi16(M, S, ev, wsp);
    __syncthreads();
  } else
    wg_jacobi<double>(K, M, S, ev);
  if (tid == 0) {  // sort descending (insertion sort, K <= 64)
    for (int a = 0; a < K; ++a) ord[a] = a;
    for (int a = 1; a < K; ++a) {
      int v = ord[a];
      int b = a - 1;
      while (b >= 0 && ev[ord[b]] < ev[v]) {
        ord[b + 1] = ord[b];
        --b;
      }
      ord[b + 1] = v;
    }
  }
  __syncthreads();
  // C = T Q (columns reordered)
  double* C = Cout + (i64)i * KK;
  for (int t = tid; t < KK; t += nt) {
    const int r = t / K, a = t % K;
    const int src = ord[a];
    double acc = 0;
    for (int q = 0; q < K; ++q) acc += U[r * K + q] * S[src * K + q];
    C[t] = acc;
  }
  for (int t = tid; t < K; t += nt) nu_out[(i64)i * K + t] = fmax(ev[ord[t]], 0.0);
}

// X = Y C, BX = Z C, SX = BX_old C (in place on BX), residual norms, convergence
// logic.  One workgroup per subdomain; K divides the workgroup size.
// Also the energy residual of the previous pair (X_old, SX_old, BX_old, nu_old = nu_prev):
// per column sum (y - nu_old x_old)(bx_old - nu_old sx_old) and a bound on its rounding.
// SY: S Y when the solves are not exact (the FP32-factor iteration), else null and
// S Y = BX_old.
template <typename V, int TR>
__global__ void k_eig_update(const i32* __restrict__ nb, const i64* __restrict__ kvoff, int K,
                             const double* __restrict__ Cm, const double* __restrict__ nu,
                             const V* __restrict__ Y, const V* __restrict__ Z,
                             V* __restrict__ X, V* __restrict__ BX, V* __restrict__ SX,
                             const int* __restrict__ status, double* __restrict__ part, int S,
                             const double* __restrict__ nu_prev, const V* __restrict__ SY) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x, sp = blockIdx.y;  // subdomain, row split
  if (status[i] != ST_RUNNING) return;
  const int n = nb[i];
  const int chunk = ((n + S - 1) / S + TR - 1) / TR * TR;
  const int r_lo = sp * chunk, r_hi = min(n, r_lo + chunk);
  const int KK = K * K;
  double* C = reinterpret_cast<double*>(smem_raw);  // KK
  V* ty = reinterpret_cast<V*>(C + KK);             // TR*K
  V* tz = ty + TR * K;
  V* tb = tz + TR * K;
  V* tsy = SY ? tb + TR * K : tb;  // the tile that gives S X_new = (S Y) C
  __shared__ double red_r[MSDD_WG], red_s[MSDD_WG], red_e[MSDD_WG], red_f[MSDD_WG];
  const int tid = threadIdx.x;
  for (int t = tid; t < KK; t += blockDim.x) C[t] = Cm[(i64)i * KK + t];
  const int c = tid % K;
  const int lanes = blockDim.x / K;
  const int rl = tid / K;
  const double nuc = nu[(i64)i * K + c];
  // nu_old = 0 on a pass's first iteration: X is the start block and SX is not set yet
  const double nuo = nu_prev[(i64)i * K + c];
  double accr = 0, accs = 0;  // residual^2, ||x||^2
  double acce = 0, accf = 0;  // previous pair's eps^2 and the rounding bound of its sum
  const V* Yi = Y + kvoff[i];
  const V* Zi = Z + kvoff[i];
  V* Xi = X + kvoff[i];
  V* Bi = BX + kvoff[i];
  V* Si = SX + kvoff[i];
  const V* SYi = SY ? SY + kvoff[i] : nullptr;
  for (int r0 = r_lo; r0 < r_hi; r0 += TR) {
    const int rn = min(TR, r_hi - r0);
    __syncthreads();
    for (int t = tid; t < TR * K; t += blockDim.x) {
      const int cc = t / TR, rr = t % TR;
      V y = 0, z = 0, bb = 0;
      if (rr < rn) {
        const i64 idx = r0 + rr + (i64)cc * n;
        y = Yi[idx];
        z = Zi[idx];
        bb = Bi[idx];
      }
      ty[rr * K + cc] = y;
      tz[rr * K + cc] = z;
      tb[rr * K + cc] = bb;
      if (SYi) tsy[rr * K + cc] = rr < rn ? SYi[r0 + rr + (i64)cc * n] : (V)0;
    }
    __syncthreads();
    if (rl < lanes) {
      for (int rr = rl; rr < rn; rr += lanes) {
        double x = 0, bx = 0, sx = 0;
        for (int a = 0; a < K; ++a) {
          const double ca = C[a * K + c];
          x += (double)ty[rr * K + a] * ca;
          bx += (double)tz[rr * K + a] * ca;
          sx += (double)tsy[rr * K + a] * ca;
        }
        const i64 idx = r0 + rr + (i64)c * n;
        if (nuo > 0.0) {  // read the previous pair before this thread overwrites it
          const double yo = (double)ty[rr * K + c], bo = (double)tb[rr * K + c];
          const double xo = (double)Xi[idx], so = (double)Si[idx];
          const double dd = yo - nuo * xo, ro = bo - nuo * so;
          acce += dd * ro;
          accf += (fabs(yo) + 2.0 * nuo * fabs(xo)) * fabs(ro) +
                  fabs(dd) * (fabs(bo) + 2.0 * nuo * fabs(so));
        }
        Xi[idx] = (V)x;
        Bi[idx] = (V)bx;
        Si[idx] = (V)sx;
        const double rres = bx - nuc * sx;
        accr += rres * rres;
        accs += x * x;
      }
    }
  }
  red_r[tid] = accr;
  red_s[tid] = accs;
  red_e[tid] = acce;
  red_f[tid] = accf;
  __syncthreads();
  if (tid < K) {  // partial sums of this row split, per column
    double sr = 0, ss = 0, se = 0, sf = 0;
    for (int l = 0; l < lanes; ++l) {
      sr += red_r[l * K + tid];
      ss += red_s[l * K + tid];
      se += red_e[l * K + tid];
      sf += red_f[l * K + tid];
    }
    const i64 o = ((i64)i * S + sp) * UPD_PARTS * K;
    part[o + tid] = sr;
    part[o + K + tid] = ss;
    part[o + 2 * K + tid] = se;
    part[o + 3 * K + tid] = sf;
  }
}

// backward error at which the pair that certifies the count is accepted (its relative
// eigenvalue error then stays near 1e-11)
constexpr double CERT_TOL = 1e-11;
// A pair whose Ritz value no longer moves (1e-14 relative between iterations) and whose
// residuals no longer fall (by more than half per iteration) is at the rounding floor of
// its pencil; it is accepted if its backward error is within 1e6 times the tolerance (1e-8
// at the default 1e-14) and its energy residual within 1e3 times tol_e.  The host counts
// such pairs.
constexpr double STAG_FACTOR = 1e6;
constexpr double STAG_FACTOR_E = 1e3;
// The Krylov-Weinstein interval shows that an eigenvalue lies near the certifying Ritz
// value, not that none lies above it in nu (Ritz values bound eigenvalues from below), so
// it is used only after KW_MIN_IT iterations: an eigenvalue below eta that the block had
// not yet captured would by then dominate it (its component grows by
// (lambda_{m+1} + sigma) / (lambda* + sigma) per iteration; the rule is needed only for
// certifying pairs in the slow cluster near lambda = 1, where that factor is large).
constexpr int KW_MIN_IT = 30;

// Convergence decision of each running subdomain (one wavefront): sums the row-split
// partials of k_eig_update, then the backward errors, Ritz values, count m and status.
__global__ void k_eig_judge(int K, const double* __restrict__ nu, const double* __restrict__ part,
                            int S, double sigma, double eta, int nev_max, double tol, int maxit,
                            int* __restrict__ status, int* __restrict__ iters,
                            int* __restrict__ mcount, double* __restrict__ lam_out,
                            double* __restrict__ res_out, int Kmax_allowed,
                            const i32* __restrict__ rankb, const double* __restrict__ normS,
                            double* __restrict__ nu_prev, const double* __restrict__ gs_diag,
                            const int* __restrict__ inertia, int nev_fixed, double tol_e,
                            double* __restrict__ res_e_out) {
  const int i = blockIdx.x;
  if (status[i] != ST_RUNNING) return;
  __shared__ double sh_res[64], sh_lam[64], sh_stag[64], sh_kwup[64], sh_rese[64];
  const int tid = threadIdx.x;
  if (tid < K) {
    double sr = 0, ss = 0, se = 0, sf = 0;
    for (int q = 0; q < S; ++q) {
      const i64 o = ((i64)i * S + q) * UPD_PARTS * K;
      sr += part[o + tid];
      ss += part[o + K + tid];
      se += part[o + 2 * K + tid];
      sf += part[o + 3 * K + tid];
    }
    const double nv = nu[(i64)i * K + tid];
    const double rel = (nv > 0 && ss > 0) ? sqrt(sr) / (nv * normS[i] * sqrt(ss)) : 0.0;
    const double lv = nv > 0 ? 1.0 / nv - sigma : INFINITY;
    const double np = nu_prev[(i64)i * K + tid];
    const double rp = res_out[(i64)i * K + tid];  // this column's backward error last time
    const double rpe = res_e_out[(i64)i * K + tid];
    // energy residual of the previous pair (np, x): eps^2 = sum (y - np x)(b x - np S x),
    // raised by a bound on the rounding of that sum (8 u times the sum of the magnitudes
    // of its factors' rounding errors, taken generously); infinite on a pass's first
    // iteration, where np = 0
    const double e2 = fmax(se, 0.0) + 8.0 * 2.220446049250313e-16 * sf;
    const double eps = np > 0.0 ? sqrt(e2) : INFINITY;
    const double rel_e = np > 0.0 ? eps / np : INFINITY;
    res_out[(i64)i * K + tid] = rel;
    res_e_out[(i64)i * K + tid] = rel_e;
    lam_out[(i64)i * K + tid] = lv;
    nu_prev[(i64)i * K + tid] = nv;
    sh_res[tid] = rel;
    sh_rese[tid] = tol_e > 0.0 ? rel_e : 0.0;
    sh_lam[tid] = lv;
    // at the rounding floor: the Ritz value has stopped moving (its error is about the
    // square of the vector's) and so have the residuals (while the vector still converges
    // they fall by the convergence factor every iteration)
    const bool stag_e = tol_e <= 0.0 || rel_e <= tol_e ||
                        (rel_e <= STAG_FACTOR_E * tol_e && rel_e >= 0.5 * rpe);
    sh_stag[tid] = (rel <= fmax(STAG_FACTOR * tol, CERT_TOL) && fabs(nv - np) <= 1e-14 * fabs(nv) &&
                    rel >= 0.5 * rp && stag_e) ? 1.0 : 0.0;
    // Krylov-Weinstein: the previous Ritz pair (np, x) of this column has an eigenvalue of
    // S^{-1} b within eps.  The Gram diagonal gives eps^2 = y^T S y - np^2 as well, with a
    // rounding floor of 16 u y^T S y (accurate only to sqrt(u) np); the smaller bound is
    // used.  sh_kwup = np + eps, the interval's upper end (nu of the pair).
    const double g = gs_diag[(i64)i * K + tid];
    const double e2g = fmax(g - np * np, 0.0) + 16.0 * 2.220446049250313e-16 * fabs(g);
    const double epsk = fmin(eps, g > 0.0 ? sqrt(e2g) : INFINITY);
    sh_kwup[tid] = np > 0.0 ? np + epsk : INFINITY;
  }
  __syncthreads();
  if (tid == 0) {
    const int it = iters[i] + 1;
    iters[i] = it;
    const int kb = min(K, rankb[i]);  // usable columns
    int m = 0;
    if (nev_fixed > 0) {
      // fixed count: the nev_fixed smallest finite eigenvalues
      while (m < kb && m < nev_fixed && sh_lam[m] < INFINITY) ++m;
    } else {
      while (m < kb && sh_lam[m] < eta) ++m;
    }
    // Ritz values bound the eigenvalues from above in lambda, so m never exceeds the true
    // count; when it equals the inertia count of abar - eta b, no eigenvalue below eta is
    // missing and the next pair need not converge
    const bool by_inertia = nev_fixed == 0 && inertia != nullptr && inertia[i] >= 0 &&
                            inertia[i] == m && m < kb;
    if (nev_max > 0 && m > nev_max) m = nev_max;
    const int guard = 2;
    bool grow = (m + 1 + guard > kb) && (kb < rankb[i]) && (K < Kmax_allowed);
    int need = min(m + 1, kb);
    bool ok = true;
    // the pair after the selected ones only certifies the count (its eigenvalue is at
    // least eta); its Ritz value is accurate to about its backward error, so it is
    // accepted at CERT_TOL, below the accuracy asked of reported eigenvalues
    // with a fixed count the next pair shows that the selected ones are the smallest: its
    // Krylov-Weinstein interval must clear the largest selected Ritz value
    const double nu_sep = nev_fixed > 0 ? (m > 0 ? 1.0 / (sh_lam[m - 1] + sigma) : INFINITY)
                                        : 1.0 / (eta + sigma);
    for (int a = 0; a < need; ++a) {
      if (a == m && (nev_fixed > 0 || sh_lam[a] >= eta)) {
        // the certifying pair: not needed when the inertia certifies the count; else
        // accepted at CERT_TOL, or once the Krylov-Weinstein interval of its previous
        // iterate lies entirely on the lambda > eta side (its eigenvalue then certifies
        // the count whatever its remaining error)
        const bool kw = it >= KW_MIN_IT && sh_kwup[a] < nu_sep;
        ok = ok && (by_inertia || sh_res[a] <= fmax(tol, CERT_TOL) || sh_stag[a] > 0.0 || kw);
      } else {
        ok = ok && ((sh_res[a] <= tol && sh_rese[a] <= tol_e) || sh_stag[a] > 0.0);
      }
    }
    mcount[i] = m;
    if (grow) status[i] = ST_GROW;
    else if (ok) status[i] = ST_DONE;
    else if (it >= maxit) status[i] = ST_NOCONV;
  }
}

// Coarse basis block phi = D X / sqrt(nu) for the m selected pairs, b-normalised,
// sign fixed so the largest-magnitude entry is positive; written column-major
// over the Neumann dofs (Phi) and row-major over the Dirichlet dofs (PhiD).
template <typename V>
__global__ void k_eig_finalize(const i32* __restrict__ nb, const i64* __restrict__ voff,
                               const i64* __restrict__ kvoff, int K, const double* __restrict__ dv,
                               const V* __restrict__ X, const double* __restrict__ nu,
                               const int* __restrict__ mcount, const i64* __restrict__ phi_off,
                               double* __restrict__ Phi, const i32* __restrict__ nd,
                               const i64* __restrict__ doff, const i32* __restrict__ dpos,
                               const i64* __restrict__ phid_off, double* __restrict__ PhiD) {
  const int i = blockIdx.x;
  const int n = nb[i];
  const int m = mcount[i];
  const V* Xi = X + kvoff[i];
  const double* d = dv + voff[i];
  double* P = Phi + phi_off[i];
  __shared__ double sh[16];
  __shared__ double sgn;
  for (int c = 0; c < m; ++c) {
    const double s = 1.0 / sqrt(nu[(i64)i * K + c]);
    // sign: entry of largest magnitude (first on ties) made positive
    double best = -1.0;
    int bidx = 0x7fffffff;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      const double v = fabs(d[r] * (double)Xi[r + (i64)c * n]);
      if (v > best) { best = v; bidx = r; }
    }
    // reduce (max, then min index)
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bidx, o, 64);
      if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
    }
    __shared__ double wb[16];
    __shared__ int wi[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { wb[w] = best; wi[w] = bidx; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double b0 = wb[0];
      int i0 = wi[0];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
        if (wb[q] > b0 || (wb[q] == b0 && wi[q] < i0)) { b0 = wb[q]; i0 = wi[q]; }
      const double v = d[i0] * (double)Xi[i0 + (i64)c * n];
      sgn = v < 0 ? -1.0 : 1.0;
    }
    __syncthreads();
    const double f = s * sgn;
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      P[r + (i64)c * n] = d[r] * (double)Xi[r + (i64)c * n] * f;
  }
  (void)sh;
  __syncthreads();
  // Dirichlet rows, row-major
  const int ndi = nd[i];
  const i32* dp = dpos + doff[i];
  double* PD = PhiD + phid_off[i];
  for (int t = threadIdx.x; t < ndi * m; t += blockDim.x) {
    const int q = t / m, c = t % m;
    PD[t] = P[dp[q] + (i64)c * n];
  }
}

// ---------------------------------------------------------------------------
void launch_eig_init(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                     const i32* nb, const i64* kvoff, int K, const double* dv, double* X,
                     unsigned long long seed, const i32* seed_id) {
  if (!total_rows) return;
  dim3 g((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG));
  hipLaunchKernelGGL(k_eig_init<double>, g, dim3(MSDD_WG), 0, s, total_rows, row_sub, voff, nb,
                     kvoff, K, dv, X, seed, seed_id);
}

void launch_bapply_ell(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                       const i32* nb, const i64* kvoff, int K, const double* dv, int ell_w,
                       const i32* ell_col, const double* ell_val, const double* Y, double* Z,
                       const int* active) {
  if (!total_rows) return;
  dim3 g((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG));
  hipLaunchKernelGGL(k_bapply_ell<double>, g, dim3(MSDD_WG), 0, s, total_rows, row_sub, voff, nb,
                     kvoff, K, dv, ell_w, ell_col, ell_val, Y, Z, active);
}

bool launch_bapply_tile(hipStream_t s, int P, int nmax, int bmax, const i64* voff, const i32* nb,
                        const i32* bw, const i64* kvoff, int K, const double* dv, int ell_w,
                        const i32* ell_col, const double* ell_val, const double* Y, double* Z,
                        const int* active) {
  const size_t lds = (size_t)16 * (256 + 2 * (size_t)bmax) * sizeof(double);
  if (lds > 64 * 1024) return false;  // wider bands: the untiled kernel
  if (P == 0 || nmax == 0 || K == 0) return true;
  hipLaunchKernelGGL(k_bapply_tile, dim3(P, (nmax + 255) / 256), dim3(256), lds, s, voff, nb, bw,
                     kvoff, K, dv, ell_w, ell_col, ell_val, Y, Z, active);
  return true;
}

void launch_gram(hipStream_t s, int P, const i32* nb, const i64* kvoff, int K, const double* Y,
                 const double* W, const double* Z, double* GS, double* GB, const int* active,
                 int nsplit) {
  constexpr int TR = 32;
  size_t lds = 3 * TR * K * sizeof(double);
  hipLaunchKernelGGL((k_gram<double, TR>), dim3(P, nsplit), dim3(MSDD_WG), lds, s, nb, kvoff, K,
                     Y, W, Z, GS, GB, active, nsplit);
}

void launch_rayleigh_ritz(hipStream_t s, int P, int K, const double* GS, const double* GB,
                          double* C, double* nu, const int* active, int nsplit, double* gs_diag) {
  size_t lds = (3 * (size_t)K * K + 6 * K) * sizeof(double) + K * sizeof(int) + 16;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_rayleigh_ritz,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  // four wavefronts per subdomain (for K = 16 the Jacobi itself runs in one of them)
  const int nt = 256;
  hipLaunchKernelGGL(k_rayleigh_ritz, dim3(P), dim3(nt), lds, s, K, GS, GB, C, nu, active, nsplit,
                     gs_diag);
}

void launch_row_norm(hipStream_t s, int P, const i64* voff, int ell_w, const i32* ell_col,
                     const double* ell_val, const double* dv, double sigma, double* normS,
                     const double* ell_val2) {
  hipLaunchKernelGGL(k_row_norm, dim3(P), dim3(MSDD_WG), 0, s, voff, ell_w, ell_col, ell_val, dv,
                     sigma, normS, ell_val2);
}

void launch_eig_update(hipStream_t s, int P, const i32* nb, const i64* kvoff, int K,
                       const double* C, const double* nu, const double* Y, const double* Z,
                       double* X, double* BX, double* SX, double sigma, double eta, int nev_max,
                       double tol, int maxit, int* status, int* iters, int* mcount,
                       double* lam_out, double* res_out, int Kmax_allowed, const i32* rankb,
                       const double* normS, double* nu_prev, double* part, int nsplit,
                       const double* gs_diag, const int* inertia, int nev_fixed, double tol_e,
                       double* res_e_out, const double* SY) {
  constexpr int TR = 16;
  size_t lds = (size_t)K * K * sizeof(double) + (SY ? 4 : 3) * TR * K * sizeof(double);
  hipLaunchKernelGGL((k_eig_update<double, TR>), dim3(P, nsplit), dim3(MSDD_WG), lds, s, nb, kvoff,
                     K, C, nu, Y, Z, X, BX, SX, status, part, nsplit, nu_prev, SY);
  hipLaunchKernelGGL(k_eig_judge, dim3(P), dim3(64), 0, s, K, nu, part, nsplit, sigma, eta,
                     nev_max, tol, maxit, status, iters, mcount, lam_out, res_out, Kmax_allowed,
                     rankb, normS, nu_prev, gs_diag, inertia, nev_fixed, tol_e, res_e_out);
}

void launch_eig_finalize(hipStream_t s, int P, const i32* nb, const i64* voff, const i64* kvoff,
                         int K, const double* dv, const double* X, const double* nu,
                         const int* mcount, const i64* phi_off, double* Phi, const i32* nd,
                         const i64* doff, const i32* dpos, const i64* phid_off, double* PhiD) {
  hipLaunchKernelGGL(k_eig_finalize<double>, dim3(P), dim3(MSDD_WG), 0, s, nb, voff, kvoff, K, dv,
                     X, nu, mcount, phi_off, Phi, nd, doff, dpos, phid_off, PhiD);
}

// ---------------------------------------------------------------------------
// Eigensolver with an FP32 factor of S (a10, opt-in): the scaled single-precision factor
// M of diag(sc) S diag(sc), sc = diag(S)^{-1/2}, serves as the preconditioner of the
// block iteration  Y = X N + diag(sc) M^{-1} diag(sc) (B X - S X N)  (N = the current Ritz
// values; exact shift-invert when M = the scaled S), followed by the FP64 Rayleigh-Ritz
// step on (Y^T S Y, Y^T B Y) with S Y formed explicitly, so the converged pairs are those
// of the FP64 pencil.
// ---------------------------------------------------------------------------
// sc = (S_jj)^{-1/2}, S_jj = abar_jj (1 + sigma d_j^2) for b = D abar D; one thread per row
__global__ void k_s_diag_scale(i64 total_rows, const i32* __restrict__ row_grp,
                               const i64* __restrict__ voff, const i64* __restrict__ boff,
                               const i32* __restrict__ bw, const double* __restrict__ band,
                               const double* __restrict__ gw, double sigma,
                               double* __restrict__ sc, int* __restrict__ status) {
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < total_rows;
       g += (i64)gridDim.x * blockDim.x) {
    const int i = row_grp[g];
    const i64 j = g - voff[i];
    const double a = band[boff[i] + j * (bw[i] + 1)];
    const double d = gw[g];
    const double sjj = a * (1.0 + sigma * d * d);
    if (!(sjj > 0.0)) status[i] = ST_NOTSPD;
    sc[g] = sjj > 0.0 ? 1.0 / sqrt(sjj) : 0.0;
  }
}

// out = diag(sc) band diag(sc) in the column layout (out[c*w + d] = A(c+d, c)); one thread
// per column
__global__ void k_band_scale_sym(i64 total_rows, const i32* __restrict__ row_grp,
                                 const i64* __restrict__ voff, const i64* __restrict__ boff,
                                 const i32* __restrict__ bw, const i32* __restrict__ nrows,
                                 const double* __restrict__ band, const double* __restrict__ sc,
                                 double* __restrict__ out) {
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < total_rows;
       g += (i64)gridDim.x * blockDim.x) {
    const int i = row_grp[g];
    const i64 c = g - voff[i];
    const int w = bw[i] + 1, n = nrows[i];
    const i64 o = boff[i] + c * w;
    for (int d = 0; d < w; ++d) out[o + d] = c + d < n ? band[o + d] * sc[g] * sc[g + d] : 0.0;
  }
}

// Per running subdomain, over its n x K block (column c at c*n):
//   mode 0: W = sc (BX - SX nu_c)            (the scaled residual)
//   mode 1: Y = X nu_c + sc W                (the new block)
//   mode 2: SY = T + sigma Z                 (S Y = abar Y + sigma b Y)
__global__ void k_eig32_combine(int mode, const i32* __restrict__ nb, const i64* __restrict__ voff,
                                const i64* __restrict__ kvoff, int K, const double* __restrict__ P1,
                                const double* __restrict__ P2, const double* __restrict__ nu,
                                const double* __restrict__ sc, double sigma,
                                double* __restrict__ out, const int* __restrict__ status) {
  const int i = blockIdx.y;
  if (status[i] != ST_RUNNING) return;
  const int n = nb[i];
  const i64 cnt = (i64)n * K, o = kvoff[i];
  const double* sci = sc + voff[i];
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (i64)gridDim.x * blockDim.x) {
    const int c = (int)(e / n), r = (int)(e - (i64)c * n);
    const double nuc = nu[(i64)i * K + c];
    double v;
    if (mode == 0) v = sci[r] * (P1[o + e] - nuc * P2[o + e]);
    else if (mode == 1) v = nuc * P1[o + e] + sci[r] * P2[o + e];
    else v = P1[o + e] + sigma * P2[o + e];
    out[o + e] = v;
  }
}

void launch_s_diag_scale(hipStream_t s, i64 total_rows, const i32* row_grp, const i64* voff,
                         const i64* boff, const i32* bw, const double* band, const double* gw,
                         double sigma, double* sc, int* status) {
  if (!total_rows) return;
  const int g = (int)std::min<i64>((total_rows + 255) / 256, 65535);
  hipLaunchKernelGGL(k_s_diag_scale, dim3(g), dim3(256), 0, s, total_rows, row_grp, voff, boff,
                     bw, band, gw, sigma, sc, status);
}
void launch_band_scale_sym(hipStream_t s, i64 total_rows, const i32* row_grp, const i64* voff,
                           const i64* boff, const i32* bw, const i32* nrows, const double* band,
                           const double* sc, double* out) {
  if (!total_rows) return;
  const int g = (int)std::min<i64>((total_rows + 255) / 256, 65535);
  hipLaunchKernelGGL(k_band_scale_sym, dim3(g), dim3(256), 0, s, total_rows, row_grp, voff, boff,
                     bw, nrows, band, sc, out);
}
void launch_eig32_combine(hipStream_t s, int mode, int P, int nmax, const i32* nb,
                          const i64* voff, const i64* kvoff, int K, const double* P1,
                          const double* P2, const double* nu, const double* sc, double sigma,
                          double* out, const int* status) {
  if (!P) return;
  const int gx = (int)std::min<i64>(((i64)nmax * K + 255) / 256, 64);
  hipLaunchKernelGGL(k_eig32_combine, dim3(gx, P), dim3(256), 0, s, mode, nb, voff, kvoff, K, P1,
                     P2, nu, sc, sigma, out, status);
}
