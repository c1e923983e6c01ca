// Coarsest level of one large problem (Sec. 2.1, level 0): Cholesky factorisation
// A_0 = L L^T, L^{-1} and the explicit inverse A_0^{-1} = L^{-T} L^{-1} spread over the
// whole device in 64 x 64 tiles.  The one-workgroup kernels of coarse.hip serve the many
// small blocks of batches and coarse levels; a single A_0 of several thousand rows needs
// every compute unit (n_0 = 3606 took 11.9 s on one workgroup).
//
// All matrices are n x n, column-major, leading dimension n.  T = ceil(n / 64) tiles per
// side; tile row/column q covers indices [64 q, min(64 q + 64, n)).  Entries beyond n are
// treated as those of the identity (the last tile is padded), so every kernel runs full
// 64 x 64 tiles with guarded loads and stores.
//
// Factorisation, right-looking, for k = 0 .. T-1:
//   diag:   L_kk = chol(A_kk)                       (one workgroup, LDS)
//   panel:  L_ik = A_ik L_kk^{-T}, i > k             (one thread per row)
//   update: A_ij -= L_ik L_jk^T, i >= j > k          (one workgroup per tile, lower part)
// Inverse of L by block forward substitution on L X = I (X starts as I), for k = 0 .. T-1:
//   X_kj = L_kk^{-1} X_kj, j <= k                    (one thread per column)
//   X_ij -= L_ik X_kj, i > k, j <= k                 (one workgroup per tile)
// Explicit inverse: Inv_IJ = sum_{k >= I} X_kI^T X_kJ for I >= J, mirrored to Inv_JI.
// Flops: n^3 / 3 for each of the three phases.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace {

constexpr int TB = 64;    // tile side
constexpr int TNT = 256;  // threads of a tile-product workgroup: 16 x 16, 4 x 4 outputs each

__device__ __forceinline__ double ld_guard(const double* A, int n, int r, int c) {
  if (r < n && c < n) return A[r + (i64)c * n];
  return r == c ? 1.0 : 0.0;
}

// 64 x 64 tile product C -= As^T Bs over kk (As[kk][r], Bs[kk][c] in LDS, padded by one
// column against bank conflicts); thread (ty, tx) owns rows 4 ty .. 4 ty + 3 and columns
// 4 tx .. 4 tx + 3.
struct TileAcc {
  double c[4][4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
  }
  __device__ __forceinline__ void mac(const double (*As)[TB + 1], const double (*Bs)[TB + 1],
                                      int ty, int tx) {
#pragma unroll 8
    for (int kk = 0; kk < TB; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][4 * ty + q];
        b[q] = Bs[kk][4 * tx + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[p][q] = fma(a[p], b[q], c[p][q]);
    }
  }
};

// tile (I, J) of the lower triangle from its linear index e = I (I + 1) / 2 + J
__device__ __forceinline__ void tri_index(i64 e, int& I, int& J) {
  int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
  while ((i64)(i + 1) * (i + 2) / 2 <= e) ++i;
  while ((i64)i * (i + 1) / 2 > e) --i;
  I = i;
  J = (int)(e - (i64)i * (i + 1) / 2);
}

// L_kk = chol(A_kk) in place (lower; the strictly upper part of the tile set to zero).
__global__ void __launch_bounds__(TNT) k_bchol_diag(double* __restrict__ A, int n, int k,
                                                    int* __restrict__ status) {
  __shared__ double S[TB][TB + 1];  // S[r][c]
  const int tid = threadIdx.x;
  const int k0 = k * TB;
  for (int e = tid; e < TB * TB; e += TNT) {
    const int r = e % TB, c = e / TB;
    S[r][c] = ld_guard(A, n, k0 + r, k0 + c);
  }
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < TB; ++j) {
    const double d = S[j][j];
    bad = bad || !(d > 0.0);
    const double ld = sqrt(fmax(d, 0.0));
    const double il = ld > 0.0 ? 1.0 / ld : 0.0;
    __syncthreads();  // every thread has read S[j][j]
    if (tid == 0) S[j][j] = ld;
    for (int r = j + 1 + tid; r < TB; r += TNT) S[r][j] *= il;
    __syncthreads();
    const int w = TB - 1 - j;  // trailing rows/columns j+1 .. 63
    for (int e = tid; e < w * w; e += TNT) {
      const int r = j + 1 + e % w, c = j + 1 + e / w;
      if (r >= c) S[r][c] -= S[r][j] * S[c][j];
    }
    __syncthreads();
  }
  if (bad && tid == 0) status[0] = ST_NOTSPD;
  for (int e = tid; e < TB * TB; e += TNT) {
    const int r = e % TB, c = e / TB;
    if (k0 + r < n && k0 + c < n) A[(k0 + r) + (i64)(k0 + c) * n] = r >= c ? S[r][c] : 0.0;
  }
}

// L_ik = A_ik L_kk^{-T} for the rows below tile k: thread per row, x L_kk^T = a by forward
// substitution over the 64 columns (row in registers, L_kk in LDS); the 64-row panel tile
// passes through LDS so that the global reads and writes are contiguous.
__global__ void __launch_bounds__(64) k_bchol_panel(double* __restrict__ A, int n, int k) {
  __shared__ double Lk[TB][TB + 1], Pt[TB][TB + 1];
  const int k0 = k * TB;
  const int r0 = k0 + TB + blockIdx.x * 64;
  const int lane = threadIdx.x;
  for (int e = lane; e < TB * TB; e += 64) {
    const int r = e % TB, c = e / TB;
    Lk[r][c] = ld_guard(A, n, k0 + r, k0 + c);
    Pt[r][c] = (r0 + r < n && k0 + c < n) ? A[(r0 + r) + (i64)(k0 + c) * n] : 0.0;
  }
  __syncthreads();
  double x[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) x[j] = Pt[lane][j];
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    double v = x[j];
#pragma unroll
    for (int i = 0; i < j; ++i) v = fma(-Lk[j][i], x[i], v);
    x[j] = v / Lk[j][j];
  }
#pragma unroll
  for (int j = 0; j < TB; ++j) Pt[lane][j] = x[j];
  __syncthreads();
  for (int e = lane; e < TB * TB; e += 64) {
    const int r = e % TB, c = e / TB;
    if (r0 + r < n && k0 + c < n) A[(r0 + r) + (i64)(k0 + c) * n] = Pt[r][c];
  }
}

// A_ij -= L_ik L_jk^T for the lower-triangle tiles (i >= j) of the trailing matrix
// (tiles k+1 .. T-1); diagonal tiles update their lower part only.
__global__ void __launch_bounds__(TNT) k_bchol_update(double* __restrict__ A, int n, int k) {
  __shared__ double As[TB][TB + 1], Bs[TB][TB + 1];
  int I, J;
  tri_index(blockIdx.x, I, J);
  I += k + 1;
  J += k + 1;
  const int k0 = k * TB, i0 = I * TB, j0 = J * TB;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int e = tid; e < TB * TB; e += TNT) {
    const int r = e % TB, kk = e / TB;
    As[kk][r] = (i0 + r < n && k0 + kk < n) ? A[(i0 + r) + (i64)(k0 + kk) * n] : 0.0;
    Bs[kk][r] = (j0 + r < n && k0 + kk < n) ? A[(j0 + r) + (i64)(k0 + kk) * n] : 0.0;
  }
  __syncthreads();
  TileAcc acc;
  acc.zero();
  acc.mac(As, Bs, ty, tx);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = i0 + 4 * ty + p, c = j0 + 4 * tx + q;
      if (r < n && c < n && r >= c) A[r + (i64)c * n] -= acc.c[p][q];
    }
}

// X_kj = L_kk^{-1} X_kj for the tiles j <= k of block row k: thread per column of tile j
// (blockIdx.x), forward substitution over the 64 rows; the tile passes through LDS so that
// the global reads and writes are contiguous.
__global__ void __launch_bounds__(64) k_btri_rowsolve(const double* __restrict__ L,
                                                      double* __restrict__ X, int n, int k) {
  __shared__ double Lk[TB][TB + 1], Bt[TB][TB + 1];
  const int k0 = k * TB, j0 = blockIdx.x * TB;
  const int lane = threadIdx.x;
  for (int e = lane; e < TB * TB; e += 64) {
    const int r = e % TB, c = e / TB;
    Lk[r][c] = ld_guard(L, n, k0 + r, k0 + c);
    Bt[r][c] = (k0 + r < n && j0 + c < n) ? X[(k0 + r) + (i64)(j0 + c) * n] : 0.0;
  }
  __syncthreads();
  double x[TB];
#pragma unroll
  for (int r = 0; r < TB; ++r) x[r] = Bt[r][lane];
#pragma unroll
  for (int r = 0; r < TB; ++r) {
    double v = x[r];
#pragma unroll
    for (int i = 0; i < r; ++i) v = fma(-Lk[r][i], x[i], v);
    x[r] = v / Lk[r][r];
  }
#pragma unroll
  for (int r = 0; r < TB; ++r) Bt[r][lane] = x[r];
  __syncthreads();
  for (int e = lane; e < TB * TB; e += 64) {
    const int r = e % TB, c = e / TB;
    if (k0 + r < n && j0 + c < n) X[(k0 + r) + (i64)(j0 + c) * n] = Bt[r][c];
  }
}

// X_ij -= L_ik X_kj for i > k, j <= k: blockIdx.x = (i - k - 1) * (k + 1) + j.
__global__ void __launch_bounds__(TNT) k_btri_update(const double* __restrict__ L,
                                                     double* __restrict__ X, int n, int k) {
  __shared__ double As[TB][TB + 1], Bs[TB][TB + 1];
  const int I = k + 1 + (int)(blockIdx.x / (k + 1)), J = (int)(blockIdx.x % (k + 1));
  const int k0 = k * TB, i0 = I * TB, j0 = J * TB;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int e = tid; e < TB * TB; e += TNT) {
    const int r = e % TB, kk = e / TB;
    As[kk][r] = (i0 + r < n && k0 + kk < n) ? L[(i0 + r) + (i64)(k0 + kk) * n] : 0.0;
    // Bs[kk][c] = X(k0 + kk, j0 + c): kk runs fastest, so the reads are contiguous
    const int kk2 = e % TB, c2 = e / TB;
    Bs[kk2][c2] = (k0 + kk2 < n && j0 + c2 < n) ? X[(k0 + kk2) + (i64)(j0 + c2) * n] : 0.0;
  }
  __syncthreads();
  TileAcc acc;
  acc.zero();
  acc.mac(As, Bs, ty, tx);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = i0 + 4 * ty + p, c = j0 + 4 * tx + q;
      if (r < n && c < n) X[r + (i64)c * n] -= acc.c[p][q];
    }
}

// Inv_IJ = sum_{k >= I} X_kI^T X_kJ for I >= J (linear lower-triangle tile index), written
// to both Inv_IJ and Inv_JI.
__global__ void __launch_bounds__(TNT) k_bgram(const double* __restrict__ X,
                                               double* __restrict__ Inv, int n, int T) {
  __shared__ double As[TB][TB + 1], Bs[TB][TB + 1];
  int I, J;
  tri_index(blockIdx.x, I, J);
  const int i0 = I * TB, j0 = J * TB;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  TileAcc acc;
  acc.zero();
  for (int k = I; k < T; ++k) {
    const int k0 = k * TB;
    __syncthreads();
    for (int e = tid; e < TB * TB; e += TNT) {
      const int kk = e % TB, c = e / TB;
      As[kk][c] = (k0 + kk < n && i0 + c < n) ? X[(k0 + kk) + (i64)(i0 + c) * n] : 0.0;
      Bs[kk][c] = (k0 + kk < n && j0 + c < n) ? X[(k0 + kk) + (i64)(j0 + c) * n] : 0.0;
    }
    __syncthreads();
    acc.mac(As, Bs, ty, tx);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = i0 + 4 * ty + p, c = j0 + 4 * tx + q;
      if (r < n && c < n) {
        Inv[r + (i64)c * n] = acc.c[p][q];
        Inv[c + (i64)r * n] = acc.c[p][q];
      }
    }
}

__global__ void k_bidentity(double* __restrict__ X, int n) {
  const i64 nn = (i64)n * n;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (i64)gridDim.x * blockDim.x)
    X[e] = (e % n == e / n) ? 1.0 : 0.0;
}

// zero the tiles strictly above the diagonal (they still hold A's upper triangle)
__global__ void k_bzero_upper(double* __restrict__ A, int n) {
  const i64 nn = (i64)n * n;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (i64)gridDim.x * blockDim.x) {
    const int r = (int)(e % n), c = (int)(e / n);
    if (r / TB < c / TB) A[e] = 0.0;
  }
}

}  // namespace

void launch_blocked_spd_inverse(hipStream_t s, int n, double* A, double* Linv, double* Inv,
                                int* status) {
  if (n <= 0) return;
  const int T = (n + TB - 1) / TB;
  for (int k = 0; k < T; ++k) {
    hipLaunchKernelGGL(k_bchol_diag, dim3(1), dim3(TNT), 0, s, A, n, k, status);
    const int rows = n - (k + 1) * TB;
    if (rows > 0) {
      hipLaunchKernelGGL(k_bchol_panel, dim3((rows + 63) / 64), dim3(64), 0, s, A, n, k);
      const i64 t = T - k - 1;
      hipLaunchKernelGGL(k_bchol_update, dim3((unsigned)(t * (t + 1) / 2)), dim3(TNT), 0, s, A,
                         n, k);
    }
  }
  const unsigned fill = (unsigned)std::min<i64>(((i64)n * n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_bzero_upper, dim3(fill), dim3(256), 0, s, A, n);
  hipLaunchKernelGGL(k_bidentity, dim3(fill), dim3(256), 0, s, Linv, n);
  for (int k = 0; k < T; ++k) {
    hipLaunchKernelGGL(k_btri_rowsolve, dim3(k + 1), dim3(64), 0, s, A, Linv, n, k);
    if (k + 1 < T)
      hipLaunchKernelGGL(k_btri_update, dim3((unsigned)((i64)(T - k - 1) * (k + 1))), dim3(TNT),
                         0, s, A, Linv, n, k);
  }
  hipLaunchKernelGGL(k_bgram, dim3((unsigned)((i64)T * (T + 1) / 2)), dim3(TNT), 0, s, Linv, Inv,
                     n, T);
}
