// Preconditioned conjugate gradients (Sec. 5) with the multilevel additive
// Schwarz preconditioner (Sec. 2.1):
//   z = sum_{l=1}^{L} P_l sum_i R_{l,i}^T A_{l,i}^{-1} R_{l,i} P_l^T r + P_0 A_0^{-1} P_0^T r,
//   P_L = I, P_{l-1} = P_l Phi_l.
// Reductions are two-pass (fixed grid of partial sums, then one workgroup in a
// fixed order), so results are bitwise repeatable.
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "msdd.h"
#include "trsv.h"

// ---------------------------------------------------------------------------
// PCG on several independent systems at once ("segments": contiguous row ranges,
// one per problem; a single problem is one segment).  Vector kernels work on
// "chunks" (row ranges inside one segment), one workgroup per chunk, and write one
// partial sum per chunk; k_seg_reduce sums a segment's chunks in a fixed order and
// applies the CG scalar rule of that segment.  Convergence is decided on the device:
// a segment that converged (or hit maxit) gets alpha = beta = 0 and stays frozen, so
// iterations can run in chunks without reading anything back.
// ---------------------------------------------------------------------------
template <int SG>
__global__ void __launch_bounds__(256) k_spmv_chunk(
    const i64* __restrict__ ch_lo, const i64* __restrict__ ch_hi, const i64* __restrict__ rowptr,
    const i32* __restrict__ col, const double* __restrict__ val, const double* __restrict__ p,
    double* __restrict__ q, double* __restrict__ partial) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  const int lane = threadIdx.x % SG;
  const i64 hi = ch_hi[c];
  double dacc = 0.0;
  for (i64 row = ch_lo[c] + threadIdx.x / SG; row < hi; row += blockDim.x / SG) {
    double s = 0.0;
    for (i64 e = rowptr[row] + lane; e < rowptr[row + 1]; e += SG) s += val[e] * p[col[e]];
    for (int o = SG / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, SG);
    if (lane == 0) {
      q[row] = s;
      dacc += s * p[row];
    }
  }
  const double t = block_sum(dacc, sh);
  if (threadIdx.x == 0) partial[c] = t;
}

// r = b - q; partial r.r
__global__ void k_residual_chunk(const i64* __restrict__ ch_lo, const i64* __restrict__ ch_hi,
                                 const double* __restrict__ b, const double* __restrict__ q,
                                 double* __restrict__ r, double* __restrict__ partial) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (i64 i = ch_lo[c] + threadIdx.x; i < ch_hi[c]; i += blockDim.x) {
    const double v = b[i] - q[i];
    r[i] = v;
    acc += v * v;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[c] = acc;
}

// x += alpha_s p; r -= alpha_s q; partial r.r
__global__ void k_update_xr_chunk(const i64* __restrict__ ch_lo, const i64* __restrict__ ch_hi,
                                  const i32* __restrict__ ch_seg, double* __restrict__ x,
                                  double* __restrict__ r, const double* __restrict__ p,
                                  const double* __restrict__ q, const double* __restrict__ D,
                                  double* __restrict__ partial) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  const double a = D[ch_seg[c] * PCG_SD + PCG_ALPHA];
  double acc = 0.0;
  for (i64 i = ch_lo[c] + threadIdx.x; i < ch_hi[c]; i += blockDim.x) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[c] = acc;
}

__global__ void k_dot_chunk(const i64* __restrict__ ch_lo, const i64* __restrict__ ch_hi,
                            const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ partial) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (i64 i = ch_lo[c] + threadIdx.x; i < ch_hi[c]; i += blockDim.x) acc += a[i] * b[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[c] = acc;
}

// p = z + beta_s p  (first: p = z)
__global__ void k_update_p_chunk(const i64* __restrict__ ch_lo, const i64* __restrict__ ch_hi,
                                 const i32* __restrict__ ch_seg, const double* __restrict__ z,
                                 double* __restrict__ p, const double* __restrict__ D, int first) {
  const int c = blockIdx.x;
  const double be = first ? 0.0 : D[ch_seg[c] * PCG_SD + PCG_BETA];
  for (i64 i = ch_lo[c] + threadIdx.x; i < ch_hi[c]; i += blockDim.x)
    p[i] = first ? z[i] : z[i] + be * p[i];
}

// Per segment: sum its chunks' partial sums (fixed order) and apply the rule.
// Segment state: D[s*PCG_SD + field], I[s*PCG_SI + field].
__global__ void k_seg_reduce(const i64* __restrict__ seg_ch, const double* __restrict__ partial,
                             double* __restrict__ D, int* __restrict__ I, int rule, double rtol,
                             int maxit, double* __restrict__ hist, int nseg) {
  __shared__ double sh[16];
  const int sg = blockIdx.x;
  double acc = 0.0;
  for (i64 c = seg_ch[sg] + threadIdx.x; c < seg_ch[sg + 1]; c += blockDim.x) acc += partial[c];
  acc = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  double* d = D + sg * PCG_SD;
  int* st = I + sg * PCG_SI;
  const bool run = st[PCG_ACTIVE] == PCG_RUNNING;
  switch (rule) {
    case PCG_R_RR0:
      d[PCG_RR0] = acc;
      d[PCG_RR] = acc;
      d[PCG_TOL2] = rtol * rtol * acc;
      st[PCG_IT] = 0;
      st[PCG_ITERS] = 0;
      hist[sg] = acc > 0.0 ? 1.0 : 0.0;
      st[PCG_ACTIVE] = !isfinite(acc) ? PCG_BREAKDOWN : (acc > 0.0 ? PCG_RUNNING : PCG_CONVERGED);
      break;
    case PCG_R_RZ0:
      d[PCG_RZ] = acc;
      break;
    case PCG_R_PQ:
      d[PCG_PQ] = acc;
      d[PCG_ALPHA] = 0.0;
      if (run) {
        const double a = d[PCG_RZ] / acc;
        if (!isfinite(a)) {
          st[PCG_ACTIVE] = PCG_BREAKDOWN;
          st[PCG_ITERS] = st[PCG_IT];
        } else {
          st[PCG_IT] += 1;
          d[PCG_ALPHA] = a;
        }
      }
      break;
    case PCG_R_RR:
      if (run) {
        d[PCG_RR] = acc;
        const int it = st[PCG_IT];
        if (it <= maxit) hist[(i64)it * nseg + sg] = sqrt(acc / d[PCG_RR0]);
        if (!isfinite(acc)) {
          st[PCG_ACTIVE] = PCG_BREAKDOWN;
          st[PCG_ITERS] = it;
        } else if (acc < d[PCG_TOL2]) {
          st[PCG_ACTIVE] = PCG_CONVERGED;
          st[PCG_ITERS] = it;
        } else if (it >= maxit) {
          st[PCG_ACTIVE] = PCG_MAXIT;
          st[PCG_ITERS] = it;
        }
      }
      break;
    case PCG_R_RZ:
      d[PCG_BETA] = 0.0;
      if (run) {
        d[PCG_BETA] = acc / d[PCG_RZ];
        d[PCG_RZ] = acc;
      }
      break;
  }
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
    double* __restrict__ u, int in_lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16 * 8];
  const int i = blockIdx.x;
  const int n = nd[i];
  const int tid = threadIdx.x;
  // the gathered residual in LDS, or (subdomains too large for it) read back from u after
  // the barrier below
  double* rl = in_lds ? reinterpret_cast<double*>(smem_raw) : u + doff[i];
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
        if (in_lds) rl[q] = x[t];
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
  wg_ldl_solve_rot<T, T>(n, bd[i], Fc + dboff[i], Fr + dboff[i], rl, tiles, [&] {
    for (int q = threadIdx.x; q < n; q += ROT_NT) rl[q] = (T)(si ? ui[q] * si[q] : ui[q]);
  });
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
  T* ring = reinterpret_cast<T*>(smem_raw);
  double* ui = u + doff[i];
  const double* si = scale ? scale + doff[i] : nullptr;
  wave_ldl_solve_ring<T, T, double>(n, bd[i], Fr + dboff[i], ui, ui, si, ring,
                                    wave_ring_size(bd[i]) - 1);
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

// coarsest level: z0 = A_0^{-1} r0 with the explicit inverse of each diagonal block
// (one block per problem).  One wavefront per row: row o of the symmetric inverse is
// its column o, read contiguously.  grid = (ceil(n_max / 4), blocks), 256 threads.
__global__ void __launch_bounds__(256) k_apply_coarsest(
    const i64* __restrict__ zoff, const i64* __restrict__ aoff, const i32* __restrict__ n_arr,
    const double* __restrict__ Inv, const double* __restrict__ r0, double* __restrict__ z0) {
  const int t = blockIdx.y;
  const int n = n_arr[t];
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= n) return;
  const double* col = Inv + aoff[t] + (i64)o * n;
  const double* r = r0 + zoff[t];
  double acc = 0.0;
  for (int q = lane; q < n; q += 64) acc += col[q] * r[q];
  acc = wave_sum(acc);
  if (lane == 0) z0[zoff[t] + o] = acc;
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
// contains p of (u_i + PhiD_i zc_i)[local index of p].  Variants for the hybrid form:
// w (per Dirichlet entry, may be null) weights u_i (restricted additive Schwarz: the
// partition of unity), u or zc null drops that term, acc adds to z instead of writing it.
__device__ __forceinline__ double fine_up_row(i64 p, const i64* __restrict__ dinc_ptr,
                                              const i32* __restrict__ dinc_sub,
                                              const i32* __restrict__ dinc_q,
                                              const i64* __restrict__ doff,
                                              const i32* __restrict__ msub,
                                              const i64* __restrict__ moff,
                                              const i64* __restrict__ phid_off,
                                              const double* __restrict__ PhiD,
                                              const double* __restrict__ u,
                                              const double* __restrict__ zc,
                                              const double* __restrict__ w) {
  double s = 0.0;
  for (i64 e = dinc_ptr[p]; e < dinc_ptr[p + 1]; ++e) {
    const int i = dinc_sub[e];
    const int q = dinc_q[e];
    double v = 0.0;
    if (u) v = w ? w[doff[i] + q] * u[doff[i] + q] : u[doff[i] + q];
    if (zc) {
      const int m = msub[i];
      const double* row = PhiD + phid_off[i] + (i64)q * m;
      const double* zz = zc + moff[i];
      for (int c = 0; c < m; ++c) v += row[c] * zz[c];
    }
    s += v;
  }
  return s;
}

__global__ void k_apply_fine_up(i64 n, const i64* __restrict__ dinc_ptr,
                                const i32* __restrict__ dinc_sub, const i32* __restrict__ dinc_q,
                                const i64* __restrict__ doff, const i32* __restrict__ msub,
                                const i64* __restrict__ moff, const i64* __restrict__ phid_off,
                                const double* __restrict__ PhiD, const double* __restrict__ u,
                                const double* __restrict__ zc, double* __restrict__ z,
                                const double* __restrict__ w, int acc) {
  for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (i64)gridDim.x * blockDim.x) {
    const double s = fine_up_row(p, dinc_ptr, dinc_sub, dinc_q, doff, msub, moff, phid_off, PhiD,
                                 u, zc, w);
    z[p] = acc ? z[p] + s : s;
  }
}

// The same gather over the PCG chunks (one workgroup per chunk), each also writing its
// chunk's partial sum of r.z, summed as k_dot_chunk sums it (same rows per thread, same
// workgroup sum), for the CG scalar that follows the preconditioner.
__global__ void __launch_bounds__(256) k_apply_fine_up_dot(
    const i64* __restrict__ ch_lo, const i64* __restrict__ ch_hi, const i64* __restrict__ dinc_ptr,
    const i32* __restrict__ dinc_sub, const i32* __restrict__ dinc_q, const i64* __restrict__ doff,
    const i32* __restrict__ msub, const i64* __restrict__ moff, const i64* __restrict__ phid_off,
    const double* __restrict__ PhiD, const double* __restrict__ u, const double* __restrict__ zc,
    double* __restrict__ z, const double* __restrict__ r, double* __restrict__ partial) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (i64 p = ch_lo[c] + threadIdx.x; p < ch_hi[c]; p += blockDim.x) {
    const double s = fine_up_row(p, dinc_ptr, dinc_sub, dinc_q, doff, msub, moff, phid_off, PhiD,
                                 u, zc, nullptr);
    z[p] = s;
    acc += r[p] * s;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[c] = acc;
}

// ---------------------------------------------------------------------------
static inline unsigned grid_for(i64 n) {
  i64 g = (n + MSDD_WG - 1) / MSDD_WG;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (unsigned)g;
}

void launch_spmv_chunk(hipStream_t s, int nch, int sg, const i64* ch_lo, const i64* ch_hi,
                       const i64* rowptr, const i32* col, const double* val, const double* p,
                       double* q, double* partial) {
  if (sg <= 4)
    hipLaunchKernelGGL(k_spmv_chunk<4>, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, rowptr, col, val, p, q, partial);
  else if (sg <= 8)
    hipLaunchKernelGGL(k_spmv_chunk<8>, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, rowptr, col, val, p, q, partial);
  else if (sg <= 16)
    hipLaunchKernelGGL(k_spmv_chunk<16>, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, rowptr, col, val, p, q, partial);
  else
    hipLaunchKernelGGL(k_spmv_chunk<32>, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, rowptr, col, val, p, q, partial);
}
void launch_residual_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                           const double* b, const double* q, double* r, double* partial) {
  hipLaunchKernelGGL(k_residual_chunk, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, b, q, r, partial);
}
void launch_update_xr_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                            const i32* ch_seg, double* x, double* r, const double* p,
                            const double* q, const double* D, double* partial) {
  hipLaunchKernelGGL(k_update_xr_chunk, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, ch_seg, x, r, p,
                     q, D, partial);
}
void launch_dot_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi, const double* a,
                      const double* b, double* partial) {
  hipLaunchKernelGGL(k_dot_chunk, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, a, b, partial);
}
void launch_update_p_chunk(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                           const i32* ch_seg, const double* z, double* p, const double* D,
                           int first) {
  hipLaunchKernelGGL(k_update_p_chunk, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, ch_seg, z, p, D,
                     first);
}
void launch_seg_reduce(hipStream_t s, int nseg, const i64* seg_ch, const double* partial,
                       double* D, int* I, int rule, double rtol, int maxit, double* hist) {
  hipLaunchKernelGGL(k_seg_reduce, dim3(nseg), dim3(256), 0, s, seg_ch, partial, D, I, rule, rtol,
                     maxit, hist, nseg);
}
void launch_apply_fine_restrict(hipStream_t s, int P, int nd_max, const i32* nd, const i64* doff,
                                const i32* dglob, const i32* msub, const i64* moff,
                                const i64* phid_off, const double* PhiD, const double* r,
                                double* rc, double* u) {
  if (P == 0) return;
  const int in_lds = (size_t)nd_max * sizeof(double) <= 150 * 1024;
  const size_t lds = in_lds ? (size_t)nd_max * sizeof(double) : 0;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)k_apply_fine_restrict,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_apply_fine_restrict, dim3(P), dim3(256), lds, s, nd, doff, dglob, msub,
                     moff, phid_off, PhiD, r, rc, u, in_lds);
}
size_t apply_fine_rot_lds(int nd_max, size_t elem) {
  return ((size_t)((nd_max + 3) & ~3) + 2 * (size_t)ROT_TILE) * elem;
}
void launch_apply_fine_solve(hipStream_t s, int P, int nd_max, int bd_max, const i32* nd,
                             const i32* bd, const i64* doff, const i64* dboff, const void* Fc,
                             const void* Fr, int fp32, const double* scale, double* u,
                             int variant) {
  // variant: 0 = by shape, 1 = rolling window (needs a half-bandwidth below 64 and the
  // window in LDS), 2 = one wavefront per subdomain
  if (P == 0) return;
  const size_t lds = apply_fine_rot_lds(nd_max, fp32 ? sizeof(float) : sizeof(double));
  const bool rot_ok = bd_max < 64 && lds <= 160 * 1024;
  if (rot_ok && variant != 2) {
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
    const size_t l2 = (size_t)wave_ring_size(bd_max) * sizeof(double);
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
void launch_apply_coarsest(hipStream_t s, int nt, int nmax, const i64* zoff, const i64* aoff,
                           const i32* n_arr, const double* Inv, const double* r0, double* z0) {
  if (nt <= 0 || nmax <= 0) return;
  hipLaunchKernelGGL(k_apply_coarsest, dim3((nmax + 3) / 4, nt), dim3(256), 0, s, zoff, aoff,
                     n_arr, Inv, r0, z0);
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
                          const double* zc, double* z, const double* w, int acc) {
  hipLaunchKernelGGL(k_apply_fine_up, dim3(grid_for(n)), dim3(MSDD_WG), 0, s, n, dinc_ptr,
                     dinc_sub, dinc_q, doff, msub, moff, phid_off, PhiD, u, zc, z, w, acc);
}
void launch_apply_fine_up_dot(hipStream_t s, int nch, const i64* ch_lo, const i64* ch_hi,
                              const i64* dinc_ptr, const i32* dinc_sub, const i32* dinc_q,
                              const i64* doff, const i32* msub, const i64* moff,
                              const i64* phid_off, const double* PhiD, const double* u,
                              const double* zc, double* z, const double* r, double* partial) {
  hipLaunchKernelGGL(k_apply_fine_up_dot, dim3(nch), dim3(256), 0, s, ch_lo, ch_hi, dinc_ptr,
                     dinc_sub, dinc_q, doff, msub, moff, phid_off, PhiD, u, zc, z, r, partial);
}

// ---------------------------------------------------------------------------
// Scratch memory of msdd_solve_noalloc: a file-scope device array of fixed size, one copy
// per device (resident while the library is loaded).  Host code never names the array: its
// device address is looked up once per device (with that device current) and kept here.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MSDD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return 0;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return -1;
  }
  g_scratch_ptr[device] = ptr;
  return 0;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Input check of a batched matrix: every row's columns lie in its own problem's dof range
// (pdp[t] <= col < pdp[t+1] for the problem t holding the row).  One thread per row; a
// violation sets *flag (any writer, same value).
__global__ void k_check_problem_coupling(i64 n, const i64* __restrict__ rowptr,
                                         const i32* __restrict__ col, const i64* __restrict__ pdp,
                                         int nprob, int* __restrict__ flag) {
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
    int lo = 0, hi = nprob;  // pdp[lo] <= r < pdp[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pdp[mid] <= r) lo = mid;
      else hi = mid;
    }
    const i64 a = pdp[lo], b = pdp[lo + 1];
    bool bad = false;
    for (i64 e = rowptr[r]; e < rowptr[r + 1]; ++e) bad |= col[e] < a || col[e] >= b;
    if (bad) *flag = 1;
  }
}
void launch_check_problem_coupling(hipStream_t s, i64 n, const i64* rowptr, const i32* col,
                                   const i64* pdp, int nprob, int* flag) {
  if (n == 0) return;
  const int g = (int)std::min<i64>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_check_problem_coupling, dim3(g), dim3(256), 0, s, n, rowptr, col, pdp, nprob,
                     flag);
}
