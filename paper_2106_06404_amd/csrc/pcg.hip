// Preconditioned conjugate gradients (Sec. 5) with the multilevel additive
// Schwarz preconditioner (Sec. 2.1):
//   z = sum_{l=1}^{L} P_l sum_i R_{l,i}^T A_{l,i}^{-1} R_{l,i} P_l^T r + P_0 A_0^{-1} P_0^T r,
//   P_L = I, P_{l-1} = P_l Phi_l.
// Reductions are two-pass (fixed grid of partial sums, then one workgroup in a
// fixed order), so results are bitwise repeatable.
#include "common.h"
#include "kernels.h"
#include "trsv.h"

enum { SC_RZ = 0, SC_PQ = 1, SC_RR = 2, SC_ALPHA = 3, SC_BETA = 4, SC_RR0 = 5, SC_TMP = 6 };

// q = A p (CSR, SG lanes per row) and per-block partial sums of p.q
template <int SG>
__global__ void k_spmv_dot(i64 n, const i64* __restrict__ rowptr, const i32* __restrict__ col,
                           const double* __restrict__ val, const double* __restrict__ p,
                           double* __restrict__ q, double* __restrict__ partial, int want_dot) {
  __shared__ double sh[16];
  const int lane = threadIdx.x % SG;
  const i64 rows_per_grid = (i64)gridDim.x * (blockDim.x / SG);
  double dacc = 0.0;
  for (i64 row = (i64)blockIdx.x * (blockDim.x / SG) + threadIdx.x / SG; row < n;
       row += rows_per_grid) {
    double s = 0.0;
    for (i64 e = rowptr[row] + lane; e < rowptr[row + 1]; e += SG) s += val[e] * p[col[e]];
    for (int o = SG / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, SG);
    if (lane == 0) {
      q[row] = s;
      dacc += s * p[row];
    }
  }
  if (want_dot) {
    const double t = block_sum(dacc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

// sc[slot] = sum(partial); then an update rule on the scalars
enum { RED_SET = 0, RED_ALPHA = 1, RED_BETA = 2 };
__global__ void k_reduce(const double* __restrict__ partial, int np, double* __restrict__ sc,
                         int slot, int rule) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    if (rule == RED_SET) {
      sc[slot] = s;
    } else if (rule == RED_ALPHA) {  // s = p.q
      sc[SC_PQ] = s;
      sc[SC_ALPHA] = sc[SC_RZ] / s;
    } else {  // s = r.z (new)
      sc[SC_BETA] = s / sc[SC_RZ];
      sc[SC_RZ] = s;
    }
  }
}

// x += alpha p; r -= alpha q; partial r.r
__global__ void k_update_xr(i64 n, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            const double* __restrict__ sc, double* __restrict__ partial) {
  __shared__ double sh[16];
  const double a = sc[SC_ALPHA];
  double acc = 0.0;
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ void k_dot(i64 n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ partial) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// p = z + beta p   (beta_from_sc = 0: p = z)
__global__ void k_update_p(i64 n, const double* __restrict__ z, double* __restrict__ p,
                           const double* __restrict__ sc, int use_beta) {
  const double be = use_beta ? sc[SC_BETA] : 0.0;
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    p[i] = use_beta ? z[i] + be * p[i] : z[i];
}

// r = b - q ; partial r.r
__global__ void k_residual(i64 n, const double* __restrict__ b, const double* __restrict__ q,
                           double* __restrict__ r, double* __restrict__ partial) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
    const double v = b[i] - q[i];
    r[i] = v;
    acc += v * v;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// Preconditioner apply, finest level, in two kernels:
//  k_apply_fine_restrict (one 256-thread workgroup per subdomain):
//    r_loc = R_i r (Dirichlet dofs) into u_i, rc[i,:] = PhiD_i^T r_loc
//    (restriction to the next coarser level);
//  k_apply_fine_rot / k_apply_fine_wave: u_i = A_i^{-1} u_i by the two band sweeps
//    of the LDL^T factor (see trsv.h).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_apply_fine_restrict(
    const i32* __restrict__ nd, const i64* __restrict__ doff, const i32* __restrict__ dglob,
    const i32* __restrict__ msub, const i64* __restrict__ moff, const i64* __restrict__ phid_off,
    const double* __restrict__ PhiD, const double* __restrict__ r, double* __restrict__ rc,
    double* __restrict__ u) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16 * 8];
  const int i = blockIdx.x;
  const int n = nd[i];
  const int tid = threadIdx.x;
  double* rl = reinterpret_cast<double*>(smem_raw);  // n
  const i32* dg = dglob + doff[i];
  double* ui = u + doff[i];
  for (int q0 = tid; q0 < n; q0 += 4 * 256) {
    int g[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) g[t] = dg[min(q0 + t * 256, n - 1)];
    double x[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = r[g[t]];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = q0 + t * 256;
      if (q < n) {
        rl[q] = x[t];
        ui[q] = x[t];
      }
    }
  }
  __syncthreads();
  const int m = msub[i];
  const double* PD = PhiD + phid_off[i];
  const int lane = tid & 63, wv = tid >> 6;
  for (int c0 = 0; c0 < m; c0 += 8) {
    double acc[8];
#pragma unroll
    for (int u2 = 0; u2 < 8; ++u2) acc[u2] = 0.0;
    const int cl = m - 1 - c0;  // last valid column offset of this chunk
    for (int q = tid; q < n; q += 256) {
      const double x = rl[q];
      const double* prow = PD + (i64)q * m + c0;
#pragma unroll
      for (int u2 = 0; u2 < 8; ++u2) {
        const double pv = prow[min(u2, cl)];
        acc[u2] += (u2 <= cl ? pv : 0.0) * x;
      }
    }
#pragma unroll
    for (int u2 = 0; u2 < 8; ++u2) {
      const double s2 = wave_sum(acc[u2]);
      if (lane == 0) red[wv * 8 + u2] = s2;
    }
    __syncthreads();
    if (tid < 8 && c0 + tid < m) {
      double s3 = 0.0;
      for (int w2 = 0; w2 < 4; ++w2) s3 += red[w2 * 8 + tid];
      rc[moff[i] + c0 + tid] = s3;
    }
    __syncthreads();
  }
}

// u_i = A_i^{-1} u_i with the LDL^T factor: rolling-window sweeps for half-bandwidths
// below 64 (one ROT_NT-thread workgroup per subdomain), else the one-wavefront
// blocked sweeps from the row layout.
template <typename T>
__global__ void __launch_bounds__(ROT_NT) k_apply_fine_rot(
    const i32* __restrict__ nd, const i32* __restrict__ bd, const i64* __restrict__ doff,
    const i64* __restrict__ dboff, const T* __restrict__ Fc, const T* __restrict__ Fr,
    const double* __restrict__ scale, double* __restrict__ u, int nd_max) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x;
  const int n = nd[i];
  T* rl = reinterpret_cast<T*>(smem_raw);  // nd_max (rounded up to a multiple of 4)
  T* tiles = rl + ((nd_max + 3) & ~3);
  double* ui = u + doff[i];
  const double* si = scale ? scale + doff[i] : nullptr;
  for (int q = threadIdx.x; q < n; q += ROT_NT) rl[q] = (T)(si ? ui[q] * si[q] : ui[q]);
  __syncthreads();
  wg_ldl_solve_rot<T, T>(n, bd[i], Fc + dboff[i], Fr + dboff[i], rl, tiles);
  for (int q = threadIdx.x; q < n; q += ROT_NT) ui[q] = si ? (double)rl[q] * si[q] : (double)rl[q];
}

template <typename T>
__global__ void __launch_bounds__(64) k_apply_fine_wave(
    const i32* __restrict__ nd, const i32* __restrict__ bd, const i64* __restrict__ doff,
    const i64* __restrict__ dboff, const T* __restrict__ Fr, const double* __restrict__ scale,
    double* __restrict__ u) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x;
  const int n = nd[i];
  T* rl = reinterpret_cast<T*>(smem_raw);
  double* ui = u + doff[i];
  const double* si = scale ? scale + doff[i] : nullptr;
  for (int q = threadIdx.x; q < n; q += 64) rl[q] = (T)(si ? ui[q] * si[q] : ui[q]);
  __syncthreads();
  wave_ldl_solve<T, T>(n, bd[i], Fr + dboff[i], rl);
  for (int q = threadIdx.x; q < n; q += 64) ui[q] = si ? (double)rl[q] * si[q] : (double)rl[q];
}

// coarse level l: per subdomain, r_o = r_l[own]; rc = Y^T r_o; z_l[own] = A_oo^{-1} r_o
// with the explicit inverse (column-major, symmetric)
__global__ void k_apply_coarse_down(const i32* __restrict__ nown, const i64* __restrict__ own_ptr,
                                    const i32* __restrict__ own_idx, const i64* __restrict__ loff,
                                    const double* __restrict__ Inv, const i32* __restrict__ msub,
                                    const i64* __restrict__ yoff, const double* __restrict__ Y,
                                    const i64* __restrict__ moff, const double* __restrict__ rl,
                                    double* __restrict__ zl, double* __restrict__ rc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i = blockIdx.x;
  const int no = nown[i];
  double* v = reinterpret_cast<double*>(smem_raw);
  const i32* own = own_idx + own_ptr[i];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int o = tid; o < no; o += nt) v[o] = rl[own[o]];
  __syncthreads();
  const int m = msub[i];
  const double* Yi = Y + yoff[i];
  for (int c = tid; c < m; c += nt) {
    double s = 0.0;
    for (int o = 0; o < no; ++o) s += Yi[o + (i64)c * no] * v[o];
    rc[moff[i] + c] = s;
  }
  const double* A = Inv + loff[i];
  for (int o = tid; o < no; o += nt) {
    double s = 0.0;
    for (int q = 0; q < no; ++q) s += A[o + (i64)q * no] * v[q];
    zl[own[o]] = s;
  }
}

// coarsest level: z0 = A_0^{-1} r0 with the explicit inverse, one thread per row
__global__ void k_apply_coarsest(int n0, const double* __restrict__ Inv,
                                 const double* __restrict__ r0, double* __restrict__ z0) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n0) return;
  double s = 0.0;
  for (int q = 0; q < n0; ++q) s += Inv[o + (i64)q * n0] * r0[q];
  z0[o] = s;
}

// coarse level l, upward: z_l[own] += Y z_{l-1}[i,:]
__global__ void k_apply_coarse_up(const i32* __restrict__ nown, const i64* __restrict__ own_ptr,
                                  const i32* __restrict__ own_idx, const i32* __restrict__ msub,
                                  const i64* __restrict__ yoff, const double* __restrict__ Y,
                                  const i64* __restrict__ moff, const double* __restrict__ zc,
                                  double* __restrict__ zl) {
  const int i = blockIdx.x;
  const int no = nown[i];
  const int m = msub[i];
  const i32* own = own_idx + own_ptr[i];
  const double* Yi = Y + yoff[i];
  const double* z = zc + moff[i];
  for (int o = threadIdx.x; o < no; o += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += Yi[o + (i64)c * no] * z[c];
    zl[own[o]] += s;
  }
}

// finest level, upward and gather: z[p] = sum over subdomains whose Dirichlet space
// contains p of (u_i + PhiD_i zc_i)[local index of p]
__global__ void k_apply_fine_up(i64 n, const i64* __restrict__ dinc_ptr,
                                const i32* __restrict__ dinc_sub, const i32* __restrict__ dinc_q,
                                const i64* __restrict__ doff, const i32* __restrict__ msub,
                                const i64* __restrict__ moff, const i64* __restrict__ phid_off,
                                const double* __restrict__ PhiD, const double* __restrict__ u,
                                const double* __restrict__ zc, double* __restrict__ z) {
  for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (i64)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (i64 e = dinc_ptr[p]; e < dinc_ptr[p + 1]; ++e) {
      const int i = dinc_sub[e];
      const int q = dinc_q[e];
      double v = u[doff[i] + q];
      const int m = msub[i];
      const double* row = PhiD + phid_off[i] + (i64)q * m;
      const double* zz = zc + moff[i];
      for (int c = 0; c < m; ++c) v += row[c] * zz[c];
      s += v;
    }
    z[p] = s;
  }
}

// ---------------------------------------------------------------------------
static inline unsigned grid_for(i64 n) {
  i64 g = (n + MSDD_WG - 1) / MSDD_WG;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (unsigned)g;
}
int pcg_grid(i64 n) { return (int)grid_for(n); }

void launch_spmv_dot(hipStream_t s, i64 n, int sg, const i64* rowptr, const i32* col,
                     const double* val, const double* p, double* q, double* partial, int want_dot) {
  const unsigned g = grid_for(n);
  if (sg <= 4)
    hipLaunchKernelGGL(k_spmv_dot<4>, dim3(g), dim3(MSDD_WG), 0, s, n, rowptr, col, val, p, q, partial, want_dot);
  else if (sg <= 8)
    hipLaunchKernelGGL(k_spmv_dot<8>, dim3(g), dim3(MSDD_WG), 0, s, n, rowptr, col, val, p, q, partial, want_dot);
  else if (sg <= 16)
    hipLaunchKernelGGL(k_spmv_dot<16>, dim3(g), dim3(MSDD_WG), 0, s, n, rowptr, col, val, p, q, partial, want_dot);
  else
    hipLaunchKernelGGL(k_spmv_dot<32>, dim3(g), dim3(MSDD_WG), 0, s, n, rowptr, col, val, p, q, partial, want_dot);
}
void launch_reduce(hipStream_t s, const double* partial, int np, double* sc, int slot, int rule) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(MSDD_WG), 0, s, partial, np, sc, slot, rule);
}
void launch_update_xr(hipStream_t s, i64 n, double* x, double* r, const double* p,
                      const double* q, const double* sc, double* partial) {
  hipLaunchKernelGGL(k_update_xr, dim3(grid_for(n)), dim3(MSDD_WG), 0, s, n, x, r, p, q, sc, partial);
}
void launch_dot(hipStream_t s, i64 n, const double* a, const double* b, double* partial) {
  hipLaunchKernelGGL(k_dot, dim3(grid_for(n)), dim3(MSDD_WG), 0, s, n, a, b, partial);
}
void launch_update_p(hipStream_t s, i64 n, const double* z, double* p, const double* sc,
                     int use_beta) {
  hipLaunchKernelGGL(k_update_p, dim3(grid_for(n)), dim3(MSDD_WG), 0, s, n, z, p, sc, use_beta);
}
void launch_residual(hipStream_t s, i64 n, const double* b, const double* q, double* r,
                     double* partial) {
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n)), dim3(MSDD_WG), 0, s, n, b, q, r, partial);
}
void launch_apply_fine_restrict(hipStream_t s, int P, int nd_max, const i32* nd, const i64* doff,
                                const i32* dglob, const i32* msub, const i64* moff,
                                const i64* phid_off, const double* PhiD, const double* r,
                                double* rc, double* u) {
  if (P == 0) return;
  const size_t lds = (size_t)nd_max * sizeof(double);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_apply_fine_restrict,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_apply_fine_restrict, dim3(P), dim3(256), lds, s, nd, doff, dglob, msub,
                     moff, phid_off, PhiD, r, rc, u);
}
size_t apply_fine_rot_lds(int nd_max, size_t elem) {
  return ((size_t)((nd_max + 3) & ~3) + 2 * (size_t)ROT_TILE) * elem;
}
void launch_apply_fine_solve(hipStream_t s, int P, int nd_max, int bd_max, const i32* nd,
                             const i32* bd, const i64* doff, const i64* dboff, const void* Fc,
                             const void* Fr, int fp32, const double* scale, double* u) {
  if (P == 0) return;
  const size_t lds = apply_fine_rot_lds(nd_max, fp32 ? sizeof(float) : sizeof(double));
  if (bd_max < 64 && lds <= 160 * 1024) {
    if (fp32) {
      (void)hipFuncSetAttribute((const void*)k_apply_fine_rot<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k_apply_fine_rot<float>, dim3(P), dim3(ROT_NT), lds, s, nd, bd, doff,
                         dboff, (const float*)Fc, (const float*)Fr, scale, u, nd_max);
    } else {
      (void)hipFuncSetAttribute((const void*)k_apply_fine_rot<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k_apply_fine_rot<double>, dim3(P), dim3(ROT_NT), lds, s, nd, bd, doff,
                         dboff, (const double*)Fc, (const double*)Fr, scale, u, nd_max);
    }
  } else {
    const size_t l2 = (size_t)nd_max * sizeof(double);
    if (fp32) {
      if (l2 > 65536)
        (void)hipFuncSetAttribute((const void*)k_apply_fine_wave<float>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2);
      hipLaunchKernelGGL(k_apply_fine_wave<float>, dim3(P), dim3(64), l2, s, nd, bd, doff, dboff,
                         (const float*)Fr, scale, u);
    } else {
      if (l2 > 65536)
        (void)hipFuncSetAttribute((const void*)k_apply_fine_wave<double>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2);
      hipLaunchKernelGGL(k_apply_fine_wave<double>, dim3(P), dim3(64), l2, s, nd, bd, doff, dboff,
                         (const double*)Fr, scale, u);
    }
  }
}
void launch_apply_coarse_down(hipStream_t s, int P, int no_max, const i32* nown,
                              const i64* own_ptr, const i32* own_idx, const i64* loff,
                              const double* Inv, const i32* msub, const i64* yoff,
                              const double* Y, const i64* moff, const double* rl, double* zl,
                              double* rc) {
  hipLaunchKernelGGL(k_apply_coarse_down, dim3(P), dim3(MSDD_WG), (size_t)no_max * sizeof(double),
                     s, nown, own_ptr, own_idx, loff, Inv, msub, yoff, Y, moff, rl, zl, rc);
}
void launch_apply_coarsest(hipStream_t s, int n0, const double* Inv, const double* r0, double* z0) {
  if (n0 <= 0) return;
  hipLaunchKernelGGL(k_apply_coarsest, dim3((n0 + 127) / 128), dim3(128), 0, s, n0, Inv, r0, z0);
}
void launch_apply_coarse_up(hipStream_t s, int P, const i32* nown, const i64* own_ptr,
                            const i32* own_idx, const i32* msub, const i64* yoff, const double* Y,
                            const i64* moff, const double* zc, double* zl) {
  hipLaunchKernelGGL(k_apply_coarse_up, dim3(P), dim3(MSDD_WG), 0, s, nown, own_ptr, own_idx,
                     msub, yoff, Y, moff, zc, zl);
}
void launch_apply_fine_up(hipStream_t s, i64 n, const i64* dinc_ptr, const i32* dinc_sub,
                          const i32* dinc_q, const i64* doff, const i32* msub, const i64* moff,
                          const i64* phid_off, const double* PhiD, const double* u,
                          const double* zc, double* z) {
  hipLaunchKernelGGL(k_apply_fine_up, dim3(grid_for(n)), dim3(MSDD_WG), 0, s, n, dinc_ptr,
                     dinc_sub, dinc_q, doff, msub, moff, phid_off, PhiD, u, zc, z);
}
