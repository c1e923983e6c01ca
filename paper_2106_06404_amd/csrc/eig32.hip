// ---------------------------------------------------------------------------
// The product T = abar Y of the eigensolver with the single-precision factor (Sec. 2.3,
// the GEVP operators), in difference form.  Row r of a subdomain's Neumann matrix gives
//     (abar y)_r = sum_j a_rj (y_j - y_r) + s_r y_r,   s_r = sum_j a_rj,
// the same value as sum_j a_rj y_j in exact arithmetic.  For vectors close to the kernel
// of abar (nearly constant where the coefficients are large) the differences are small,
// so the rounding error of the product scales with them instead of with |a| |y|; s_r is
// summed once per setup with compensated (Neumaier) summation, so that the row sums of
// the stored entries, often zero up to their rounding, enter exactly enough.
// ---------------------------------------------------------------------------
#include "common.h"
#include "kernels.h"

// s[g] = sum of the stored entries of Neumann row g (ELL layout, padding column -1)
__global__ void k_abar_rowsum(i64 total_rows, int ell_w, const i32* __restrict__ ell_col,
                              const double* __restrict__ ell_val, double* __restrict__ s) {
  for (i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x; g < total_rows;
       g += (i64)gridDim.x * blockDim.x) {
    double sum = 0.0, comp = 0.0;
    for (int t = 0; t < ell_w; ++t) {
      if (ell_col[g * ell_w + t] < 0) continue;
      const double v = ell_val[g * ell_w + t];
      const double u = sum + v;
      comp += fabs(sum) >= fabs(v) ? (sum - u) + v : (v - u) + sum;
      sum = u;
    }
    s[g] = sum + comp;
  }
}

// T = abar Y for the K columns of every running subdomain (Y, T: n_i x K column-major
// blocks at kvoff[i]); one thread per row
__global__ void k_abar_diff(i64 total_rows, const i32* __restrict__ row_sub,
                            const i64* __restrict__ voff, const i32* __restrict__ nb,
                            const i64* __restrict__ kvoff, int K, int ell_w,
                            const i32* __restrict__ ell_col, const double* __restrict__ ell_val,
                            const double* __restrict__ s, const double* __restrict__ Y,
                            double* __restrict__ T, const int* __restrict__ active) {
  const i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int i = row_sub[g];
  if (active && active[i] != ST_RUNNING) return;
  const int r = (int)(g - voff[i]);
  const int n = nb[i];
  const double* Yi = Y + kvoff[i];
  double* Ti = T + kvoff[i];
  const i32* ec = ell_col + g * ell_w;
  const double* ev = ell_val + g * ell_w;
  const double sr = s[g];
  for (int c = 0; c < K; ++c) {
    const double* y = Yi + (i64)c * n;
    const double yr = y[r];
    double acc = 0.0;
    for (int t = 0; t < ell_w; ++t) {
      const int j = ec[t];
      if (j >= 0) acc += ev[t] * (y[j] - yr);
    }
    Ti[r + (i64)c * n] = acc + sr * yr;
  }
}

void launch_abar_rowsum(hipStream_t s, i64 total_rows, int ell_w, const i32* ell_col,
                        const double* ell_val, double* rs) {
  if (!total_rows) return;
  hipLaunchKernelGGL(k_abar_rowsum, dim3((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG)),
                     dim3(MSDD_WG), 0, s, total_rows, ell_w, ell_col, ell_val, rs);
}

void launch_abar_diff(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                      const i32* nb, const i64* kvoff, int K, int ell_w, const i32* ell_col,
                      const double* ell_val, const double* rs, const double* Y, double* T,
                      const int* active) {
  if (!total_rows) return;
  hipLaunchKernelGGL(k_abar_diff, dim3((unsigned)((total_rows + MSDD_WG - 1) / MSDD_WG)),
                     dim3(MSDD_WG), 0, s, total_rows, row_sub, voff, nb, kvoff, K, ell_w,
                     ell_col, ell_val, rs, Y, T, active);
}
