// Dense vector kernels of GMRES with the hybrid preconditioner (Sec. 5: the Krylov method
// used with the hybrid form).  Arnoldi by classical Gram-Schmidt applied twice: the
// projections on all previous basis vectors are one pass over V (multi_dot, then
// multi_axpy), each reduction over fixed blocks in a fixed order (bitwise repeatable).
#include "common.h"
#include "kernels.h"

namespace {
constexpr int MD_THREADS = 256;
constexpr int MD_COLS = 8;  // basis columns per pass of a block
}

int multi_dot_blocks(i64 n) {
  i64 b = (n + 4 * MD_THREADS - 1) / (4 * MD_THREADS);  // about 1024 rows per block
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

// partial[c * nb + blk] = sum over the block's rows of V(r, c) w(r)
__global__ void __launch_bounds__(MD_THREADS) k_multi_dot_part(i64 n, int k, const double* __restrict__ V,
                                                               const double* __restrict__ w,
                                                               double* __restrict__ partial) {
  __shared__ double red[MD_THREADS / 64][MD_COLS];
  const int nb = gridDim.x, blk = blockIdx.x;
  const i64 rows_per = (n + nb - 1) / nb;
  const i64 r0 = (i64)blk * rows_per, r1 = min(n, r0 + rows_per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c0 = 0; c0 < k; c0 += MD_COLS) {
    double acc[MD_COLS];
#pragma unroll
    for (int t = 0; t < MD_COLS; ++t) acc[t] = 0.0;
    for (i64 r = r0 + threadIdx.x; r < r1; r += MD_THREADS) {
      const double x = w[r];
#pragma unroll
      for (int t = 0; t < MD_COLS; ++t)
        if (c0 + t < k) acc[t] += V[(i64)(c0 + t) * n + r] * x;
    }
#pragma unroll
    for (int t = 0; t < MD_COLS; ++t) {
      double v = acc[t];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[wv][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < MD_COLS && c0 + threadIdx.x < k) {
      double v = 0.0;
      for (int q = 0; q < MD_THREADS / 64; ++q) v += red[q][threadIdx.x];
      partial[(i64)(c0 + threadIdx.x) * nb + blk] = v;
    }
    __syncthreads();
  }
}

// h[c] = sum of the column's partials (one wavefront per column, fixed order)
__global__ void k_multi_dot_sum(int k, int nb, const double* __restrict__ partial,
                                double* __restrict__ h) {
  const int c = blockIdx.x;
  if (c >= k) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) v += partial[(i64)c * nb + b];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (threadIdx.x == 0) h[c] = v;
}

void launch_multi_dot(hipStream_t s, i64 n, int k, const double* V, const double* w,
                      double* partial, double* h) {
  if (k <= 0) return;
  const int nb = multi_dot_blocks(n);
  hipLaunchKernelGGL(k_multi_dot_part, dim3(nb), dim3(MD_THREADS), 0, s, n, k, V, w, partial);
  hipLaunchKernelGGL(k_multi_dot_sum, dim3(k), dim3(64), 0, s, k, nb, partial, h);
}

__global__ void k_multi_axpy(i64 n, int k, const double* __restrict__ V, const double* __restrict__ h,
                             double* __restrict__ w) {
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
    double s = w[r];
    for (int c = 0; c < k; ++c) s -= V[(i64)c * n + r] * h[c];
    w[r] = s;
  }
}

__global__ void k_gemv_cols(i64 n, int k, const double* __restrict__ V, const double* __restrict__ cc,
                            double* __restrict__ y, int acc) {
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
    double s = acc ? y[r] : 0.0;
    for (int c = 0; c < k; ++c) s += V[(i64)c * n + r] * cc[c];
    y[r] = s;
  }
}

__global__ void k_scale_dev(i64 n, const double* __restrict__ ap, int inv, const double* __restrict__ x,
                            double* __restrict__ y) {
  // inv: 0 = ap[0], 1 = 1 / ap[0], 2 = 1 / sqrt(ap[0])
  const double a = inv == 2 ? 1.0 / sqrt(ap[0]) : (inv ? 1.0 / ap[0] : ap[0]);
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x)
    y[r] = a * x[r];
}

__global__ void k_fill(i64 n, double v, double* __restrict__ y) {
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x)
    y[r] = v;
}

static unsigned vec_grid(i64 n) {
  i64 g = (n + MSDD_WG - 1) / MSDD_WG;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (unsigned)g;
}

void launch_multi_axpy(hipStream_t s, i64 n, int k, const double* V, const double* h, double* w) {
  if (k <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_multi_axpy, dim3(vec_grid(n)), dim3(MSDD_WG), 0, s, n, k, V, h, w);
}
void launch_gemv_cols(hipStream_t s, i64 n, int k, const double* V, const double* c, double* y,
                      int acc) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gemv_cols, dim3(vec_grid(n)), dim3(MSDD_WG), 0, s, n, k, V, c, y, acc);
}
void launch_scale_dev(hipStream_t s, i64 n, const double* ap, int inv, const double* x, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale_dev, dim3(vec_grid(n)), dim3(MSDD_WG), 0, s, n, ap, inv, x, y);
}
void launch_fill(hipStream_t s, i64 n, double v, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(vec_grid(n)), dim3(MSDD_WG), 0, s, n, v, y);
}

__global__ void k_axpy(i64 n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x)
    y[r] += a * x[r];
}

void launch_axpy(hipStream_t s, i64 n, double a, const double* x, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(vec_grid(n)), dim3(MSDD_WG), 0, s, n, a, x, y);
}
