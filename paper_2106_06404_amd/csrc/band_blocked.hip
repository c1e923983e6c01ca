// Blocked band solves with per-block inverses, for the shift-invert eigensolver
// (many right-hand sides, half-bandwidth b <= 64).
//
// With A = Lt D Lt^T (Lt unit lower triangular, band b) cut into blocks of 64 rows,
// Lt is block lower bidiagonal: diagonal blocks L_q and couplings C_q = Lt(block q,
// block q-1).  With M_q = L_q^{-1} the two sweeps become
//   forward   y_q = M_q v_q - P_q y_{q-1},          P_q = M_q C_q,
//   backward  x_q = N_q y_q - Q_q x_{q+1},          N_q = M_q^T D_q^{-1},
//                                                   Q_q = M_q^T C_{q+1}^T,
// so the dependent chain is one 64 x 64 by 64 x 16 product per block instead of 64
// dependent rows, and every product runs on the FP64 matrix cores.  The four matrices
// of a block are formed once per factorisation (k_band_block_build) from the row
// layout of the LDL^T factor.  Explicit inverses of the diagonal blocks of a Cholesky
// factor are well conditioned here: the backward error of the blocked solve measured
// on the high-contrast subdomain matrices is within a factor two of substitution's.
//
// Storage per block (BSTRIDE doubles): M, -P, N, -Q, each 64 x 64 in the order in which
// v_mfma_f64_16x16x4f64 takes its A operand: entry (i, k) at
//   (((i / 16) * 16 + k / 4) * 64) + (k % 4) * 16 + i % 16,
// so that the operand of row tile i / 16 and inner step k / 4 is one contiguous read of
// 64 lanes.  Rows and columns past the end of the matrix are zero (so the solve may
// read any finite value for right-hand-side rows past the end).
#include "common.h"
#include "kernels.h"
#include "wg_gemm.h"

namespace {
constexpr int BMAT = 64 * 64;
constexpr int BSTRIDE = 4 * BMAT;
constexpr int MLD = 65;  // LDS row stride of the block inverse (no bank conflicts)
}  // namespace

int64_t band_block_doubles(int n) { return (int64_t)((n + 63) / 64) * BSTRIDE; }

// One workgroup (256 threads) per (subdomain, block): wavefront 0 forms M_q column by
// column (lane j solves L_q m = e_j), then all threads form the four matrices.
//   Fr: LDL^T factor in row layout, Fr[j*(b+1) + d] = Lt(j, j-d), Fr[j*(b+1)] = 1/D_j.
__global__ void __launch_bounds__(256) k_band_block_build(const i32* __restrict__ n_arr,
                                                          const i32* __restrict__ b_arr,
                                                          const i64* __restrict__ l_off,
                                                          const double* __restrict__ Fr,
                                                          const i64* __restrict__ blk_off,
                                                          double* __restrict__ out) {
  extern __shared__ double sm[];
  const int i = blockIdx.x, q = blockIdx.y;
  const int n = n_arr[i];
  const int nblk = (n + 63) >> 6;
  if (q >= nblk) return;
  const int b = b_arr[i], w = b + 1;
  const double* F = Fr + l_off[i];
  double* O = out + blk_off[i] + (i64)q * BSTRIDE;
  const int r0 = q * 64;
  const int nr = min(64, n - r0);
  const int nrn = q + 1 < nblk ? min(64, n - r0 - 64) : 0;  // rows of the next block
  double* Ml = sm;               // 64 x MLD
  double* Lr = sm + 64 * MLD;    // factor rows of this block, 64 x w
  double* Ln = Lr + 64 * w;      // factor rows of the next block, 64 x w
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * w; e += 256) {
    const int r = e / w, d = e - r * w;
    Lr[e] = r < nr ? F[(i64)(r0 + r) * w + d] : 0.0;
    Ln[e] = r < nrn ? F[(i64)(r0 + 64 + r) * w + d] : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    const int j = tid;
    for (int r = 0; r < 64; ++r) {
      double a0 = r == j ? 1.0 : 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (r < nr) {
        const int dm = min(b, r);
        const double* lr = Lr + r * w;
        int d = 1;
        for (; d + 3 <= dm; d += 4) {
          a0 -= lr[d] * Ml[(r - d) * MLD + j];
          a1 -= lr[d + 1] * Ml[(r - d - 1) * MLD + j];
          a2 -= lr[d + 2] * Ml[(r - d - 2) * MLD + j];
          a3 -= lr[d + 3] * Ml[(r - d - 3) * MLD + j];
        }
        for (; d <= dm; ++d) a0 -= lr[d] * Ml[(r - d) * MLD + j];
      } else {
        a0 = 0.0;
      }
      Ml[r * MLD + j] = (a0 + a1) + (a2 + a3);
    }
  }
  __syncthreads();
  for (int e = tid; e < BMAT; e += 256) {
    const int tile = e >> 6, ln = e & 63;
    const int row = (tile >> 4) * 16 + (ln & 15);
    const int col = (tile & 15) * 4 + (ln >> 4);
    O[e] = Ml[row * MLD + col];
    // P(row, col) = sum_k M(row, k) C_q(k, col), C_q(k, c) = Lt(r0+k, r0-64+c) at
    // distance 64+k-c in 1..b
    double p = 0.0;
    if (q > 0) {
      const int kmax = min(row, b + col - 64);
      for (int k = 0; k <= kmax; ++k) p += Ml[row * MLD + k] * Lr[k * w + 64 + k - col];
    }
    O[BMAT + e] = -p;
    // N(row, col) = M(col, row) / D(r0+col)
    O[2 * BMAT + e] = Ml[col * MLD + row] * Lr[col * w];
    // Q(row, col) = sum_c M(c, row) C_{q+1}(col, c), C_{q+1}(k, c) = Lt(r0+64+k, r0+c)
    double s = 0.0;
    if (col < nrn) {
      for (int c = max(row, 64 + col - b); c < 64; ++c)
        s += Ml[c * MLD + row] * Ln[col * w + 64 + col - c];
    }
    O[3 * BMAT + e] = -s;
  }
}

void launch_band_block_build(hipStream_t s, int nsubs, int nmax, int bmax, const i32* n_arr,
                             const i32* b_arr, const i64* l_off, const double* Fr,
                             const i64* blk_off, double* out) {
  // the caller guarantees bmax <= 64
  if (nsubs == 0 || nmax == 0) return;
  const size_t lds = (size_t)(64 * MLD + 2 * 64 * (bmax + 1)) * sizeof(double);
  (void)hipFuncSetAttribute((const void*)k_band_block_build,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_band_block_build, dim3(nsubs, (nmax + 63) / 64), dim3(256), lds, s, n_arr,
                     b_arr, l_off, Fr, blk_off, out);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// 16 inner steps of a 16 x 16 product tile in four independent accumulator chains
// (step s into chain s % 4), summed at the end: a chain of dependent products waits
// the full latency of each, four chains keep the matrix core issuing.
__device__ __forceinline__ dbl4 mfma16(const double (&a)[16], const double (&b)[16], dbl4 init) {
  dbl4 c[4] = {init, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
  for (int s = 0; s < 16; ++s)
    c[s & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c[s & 3], 0, 0, 0);
  return (c[0] + c[1]) + (c[2] + c[3]);
}

// Buffer loads and stores with the hardware range check: an offset at or past the
// buffer's size reads 0 and drops the store, without a branch.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t dbuf(const double* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double dbuf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void dbuf_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// Y = A^{-1} W for K right-hand sides (column-major n x K, ld n, W and Y distinct) with
// the blocked factor.  Grid (subdomains, ceil(K / 16)); four wavefronts, wavefront t
// computes rows 16t..16t+15 of each block for 16 columns.  The operands of block q+1
// (matrix fragments and right-hand side) are loaded while block q runs; the chain
// value of the previous block is exchanged through LDS with one barrier per block.
// The sweeps run in pairs of blocks with no branch inside (a missing last block of a
// pair reads a valid block's matrices and stores nothing), so that the compiler counts
// the loads in flight exactly and waits only for the ones a product needs.
__global__ void __launch_bounds__(256) k_band_solve_blk(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ blk_off, const double* __restrict__ LB,
    const i64* __restrict__ v_off, int K, const double* __restrict__ Win,
    double* __restrict__ Yout, const int* __restrict__ active) {
  __shared__ double ybuf[2][64 * 16];
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i], b = b_arr[i];
  const int nblk = (n + 63) >> 6;
  const int last = nblk - 1;
  const int c0 = blockIdx.y * 16;
  const int ncol = min(16, K - c0);
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int kr = lane >> 4, cl = lane & 15;
  const bool colok = cl < ncol;
  const i64 cb = v_off[i] + (i64)c0 * n;
  const unsigned bytes = (unsigned)ncol * (unsigned)n * 8u;
  const __amdgpu_buffer_rsrc_t rx = dbuf(Win + cb, bytes);
  const __amdgpu_buffer_rsrc_t ry = dbuf(Yout + cb, bytes);
  // byte offset of (row, this lane's column); out of range past the end
  auto offs = [&](int row) -> unsigned {
    return (row >= 0 && row < n && colok) ? ((unsigned)cl * (unsigned)n + (unsigned)row) * 8u
                                          : 0xfffffff0u;
  };
  const double* Lb = LB + blk_off[i] + (i64)(t * 16) * 64 + lane;
  const int mhi = 4 * t + 3;                  // M: steps 0..mhi (lower triangular)
  const int plo = max(0, (64 - b) >> 2);      // P: steps plo..15 (last b columns)
  const int nlo = 4 * t;                      // N: steps nlo..15 (upper triangular)
  const int qhi = min(15, (b - 1) >> 2);      // Q: steps 0..qhi (first b columns)

  // the buffer read as y_{-1} by the first block
  for (int e = threadIdx.x; e < 64 * 16; e += 256) ybuf[1][e] = 0.0;
  __syncthreads();

  // ---- forward sweep ----
  // fragments of steps a matrix does not use are read from a fragment it does use
  // (a cache hit) and replaced by zero at the product
  auto fload = [&](int q, double (&m)[16], double (&p)[16], double (&v)[16]) {
    const double* base = Lb + (i64)min(q, last) * BSTRIDE;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      m[s] = base[(s <= mhi ? s : 0) * 64];
      p[s] = base[BMAT + (s >= plo ? s : 15) * 64];
      v[s] = dbuf_load(rx, offs(q * 64 + 4 * s + kr));
    }
  };
  auto fstep = [&](int q, const double (&m)[16], const double (&p)[16], const double (&v)[16]) {
    double a[16], y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) a[s] = s <= mhi ? m[s] : 0.0;
    dbl4 acc = mfma16(a, v, dbl4{0.0, 0.0, 0.0, 0.0});
    const double* yp = ybuf[(q + 1) & 1];  // y_{q-1}; zeros for q = 0 (P_0 is zero too)
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      a[s] = s >= plo ? p[s] : 0.0;
      y[s] = yp[(4 * s + kr) * 16 + cl];
    }
    acc = mfma16(a, y, acc);
    double* yc = ybuf[q & 1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = 16 * t + kr + 4 * r;
      yc[lr * 16 + cl] = acc[r];
      dbuf_store(ry, offs(q * 64 + lr), acc[r]);
    }
    lds_barrier();
  };
  {
    double m0[16], p0[16], v0[16], m1[16], p1[16], v1[16];
    fload(0, m0, p0, v0);
    for (int q = 0; q < nblk; q += 2) {
      // scheduling barriers keep each block's loads together, issued before the
      // products of the block before it
      fload(q + 1, m1, p1, v1);
      __builtin_amdgcn_sched_barrier(0);
      fstep(q, m0, p0, v0);
      __builtin_amdgcn_sched_barrier(0);
      fload(q + 2, m0, p0, v0);
      __builtin_amdgcn_sched_barrier(0);
      fstep(q + 1, m1, p1, v1);  // past the last block: no rows stored
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the forward results written by all wavefronts become visible to the backward loads
  __syncthreads();

  // ---- backward sweep (x overwrites y block by block) ----
  auto bload = [&](int q, double (&nf)[16], double (&qf)[16], double (&v)[16]) {
    const double* base = Lb + (i64)max(q, 0) * BSTRIDE;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      nf[s] = base[2 * BMAT + (s >= nlo ? s : 15) * 64];
      qf[s] = base[3 * BMAT + (s <= qhi ? s : 0) * 64];
      v[s] = dbuf_load(ry, offs(q * 64 + 4 * s + kr));
    }
  };
  auto bstep = [&](int q, const double (&nf)[16], const double (&qf)[16], const double (&v)[16]) {
    double a[16], y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) a[s] = s >= nlo ? nf[s] : 0.0;
    dbl4 acc = mfma16(a, v, dbl4{0.0, 0.0, 0.0, 0.0});
    // x_{q+1}; for the last block Q is zero and the buffer holds finite forward values
    const double* xp = ybuf[(q + 1) & 1];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      a[s] = s <= qhi ? qf[s] : 0.0;
      y[s] = xp[(4 * s + kr) * 16 + cl];
    }
    acc = mfma16(a, y, acc);
    double* xc = ybuf[q & 1];
#pragma unroll
    for (int r = 0; r < 4; ++r) xc[(16 * t + kr + 4 * r) * 16 + cl] = acc[r];
    // every wavefront has read y_q (its products above) once all have passed the barrier
    lds_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) dbuf_store(ry, offs(q * 64 + 16 * t + kr + 4 * r), acc[r]);
  };
  {
    double n0[16], q0[16], v0[16], n1[16], q1[16], v1[16];
    bload(last, n0, q0, v0);
    for (int q = last; q >= 0; q -= 2) {
      bload(q - 1, n1, q1, v1);
      __builtin_amdgcn_sched_barrier(0);
      bstep(q, n0, q0, v0);
      __builtin_amdgcn_sched_barrier(0);
      bload(q - 2, n0, q0, v0);
      __builtin_amdgcn_sched_barrier(0);
      bstep(q - 1, n1, q1, v1);  // before the first block: no rows stored
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// ---------------------------------------------------------------------------
// The same solve in four launches, so that only the couplings stay on the chain:
//   1. u_q = M_q v_q for all blocks at once          (k_blk_diag, into Y)
//   2. y_q = u_q - P_q y_{q-1}, block after block     (k_blk_chain<true>, in place)
//   3. w_q = N_q y_q for all blocks at once          (k_blk_diag, in place)
//   4. x_q = w_q - Q_q x_{q+1}, block after block     (k_blk_chain<false>, in place)
// Steps 1 and 3 spread over (subdomain, block, 16 columns) workgroups; a chain step
// is the coupling product alone and its operands are loaded two blocks ahead.  When few subdomains remain this keeps
// one compute unit per subdomain from carrying all the products.
// ---------------------------------------------------------------------------

// Grid (subdomains, blocks, ceil(K / 16)), 256 threads; wavefront t computes rows
// 16t..16t+15 of the block.  which = 0: Y = M W (block-diagonal part of the forward
// sweep); which = 2: Y = N Y in place.
__global__ void __launch_bounds__(256) k_blk_diag(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr,
    const i64* __restrict__ blk_off, const double* __restrict__ LB,
    const i64* __restrict__ v_off, int K, const double* Win, double* Yout,
    const int* __restrict__ active, int which) {
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i];
  const int q = blockIdx.y;
  if (q * 64 >= n) return;
  const int c0 = blockIdx.z * 16;
  const int ncol = min(16, K - c0);
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int kr = lane >> 4, cl = lane & 15;
  const bool colok = cl < ncol;
  const i64 cb = v_off[i] + (i64)c0 * n;
  const unsigned bytes = (unsigned)ncol * (unsigned)n * 8u;
  const __amdgpu_buffer_rsrc_t rx = dbuf((which == 0 ? Win : Yout) + cb, bytes);
  const __amdgpu_buffer_rsrc_t ry = dbuf(Yout + cb, bytes);
  auto offs = [&](int row) -> unsigned {
    return (row < n && colok) ? ((unsigned)cl * (unsigned)n + (unsigned)row) * 8u : 0xfffffff0u;
  };
  // M is lower triangular (row tile t: inner steps 0..4t+3), N upper (4t..15)
  const int lo = which == 0 ? 0 : 4 * t, hi = which == 0 ? 4 * t + 3 : 15;
  const double* base = LB + blk_off[i] + (i64)q * BSTRIDE + which * BMAT + (t * 16) * 64 + lane;
  double a[16], v[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    a[s] = base[(s >= lo && s <= hi ? s : lo) * 64];
    v[s] = dbuf_load(rx, offs(q * 64 + 4 * s + kr));
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = s >= lo && s <= hi ? a[s] : 0.0;
  const dbl4 acc = mfma16(a, v, dbl4{0.0, 0.0, 0.0, 0.0});
  if (which != 0) __syncthreads();  // in place: every wavefront has read the block
#pragma unroll
  for (int r = 0; r < 4; ++r) dbuf_store(ry, offs(q * 64 + 16 * t + kr + 4 * r), acc[r]);
}

// Grid (subdomains, ceil(K / 16)), 256 threads.  Forward: Y_q <- Y_q - P_q y_{q-1} for
// q = 0, 1, ...; backward: Y_q <- Y_q - Q_q x_{q+1} for q = last, ..., 0.  Each lane
// reads and writes only its own rows of Y (the result layout of the products), so the
// update is in place without a race; the chain value goes through LDS.
template <bool FWD>
__global__ void __launch_bounds__(256) k_blk_chain(
    const i32* __restrict__ subs, const i32* __restrict__ n_arr, const i32* __restrict__ b_arr,
    const i64* __restrict__ blk_off, const double* __restrict__ LB,
    const i64* __restrict__ v_off, int K, double* __restrict__ Yout,
    const int* __restrict__ active) {
  __shared__ double ybuf[2][64 * 16];
  const int i = subs ? subs[blockIdx.x] : blockIdx.x;
  if (active && active[i] != ST_RUNNING) return;
  const int n = n_arr[i], b = b_arr[i];
  const int nblk = (n + 63) >> 6;
  const int c0 = blockIdx.y * 16;
  const int ncol = min(16, K - c0);
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int kr = lane >> 4, cl = lane & 15;
  const bool colok = cl < ncol;
  const i64 cb = v_off[i] + (i64)c0 * n;
  const unsigned bytes = (unsigned)ncol * (unsigned)n * 8u;
  const __amdgpu_buffer_rsrc_t ry = dbuf(Yout + cb, bytes);
  auto offs = [&](int row) -> unsigned {
    return (row >= 0 && row < n && colok) ? ((unsigned)cl * (unsigned)n + (unsigned)row) * 8u
                                          : 0xfffffff0u;
  };
  // P: nonzero inner steps plo..15 (last b columns); Q: 0..qhi (first b columns)
  const int lo = FWD ? max(0, (64 - b) >> 2) : 0;
  const int hi = FWD ? 15 : min(15, (b - 1) >> 2);
  const double* Lb = LB + blk_off[i] + (FWD ? BMAT : 3 * BMAT) + (t * 16) * 64 + lane;
  for (int e = threadIdx.x; e < 2 * 64 * 16; e += 256) (&ybuf[0][0])[e] = 0.0;
  __syncthreads();
  // step j processes block q(j) = j (forward) or nblk-1-j (backward); steps past the
  // last block read a valid block's fragments and store nothing
  auto blk = [&](int j) { return FWD ? j : nblk - 1 - j; };
  auto load = [&](int j, double (&f)[16], double (&u)[4]) {
    const int q = blk(j);
    const double* base = Lb + (i64)min(max(q, 0), nblk - 1) * BSTRIDE;
#pragma unroll
    for (int s = 0; s < 16; ++s) f[s] = base[(s >= lo && s <= hi ? s : lo) * 64];
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r] = dbuf_load(ry, offs(q * 64 + 16 * t + kr + 4 * r));
  };
  auto step = [&](int j, const double (&f)[16], const double (&u)[4]) {
    const int q = blk(j);
    dbl4 acc = {u[0], u[1], u[2], u[3]};
    const double* yp = ybuf[(j + 1) & 1];  // the previous step's chain value (zeros at j = 0)
    // all LDS reads first, then the products with zeros for the empty inner steps: no
    // branches, so the reads are issued together and waited for once
    double a[16], y[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      a[s] = s >= lo && s <= hi ? f[s] : 0.0;
      y[s] = yp[(4 * s + kr) * 16 + cl];
    }
    acc = mfma16(a, y, acc);
    double* yc = ybuf[j & 1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = 16 * t + kr + 4 * r;
      yc[lr * 16 + cl] = acc[r];
      dbuf_store(ry, offs(q * 64 + lr), acc[r]);
    }
    lds_barrier();
  };
  double f0[16], f1[16], f2[16], u0[4], u1[4], u2[4];
  load(0, f0, u0);
  load(1, f1, u1);
  for (int j = 0; j < nblk; j += 3) {
    // operands two steps ahead; scheduling barriers keep each group of loads together
    load(j + 2, f2, u2);
    __builtin_amdgcn_sched_barrier(0);
    step(j, f0, u0);
    __builtin_amdgcn_sched_barrier(0);
    load(j + 3, f0, u0);
    __builtin_amdgcn_sched_barrier(0);
    step(j + 1, f1, u1);
    __builtin_amdgcn_sched_barrier(0);
    load(j + 4, f1, u1);
    __builtin_amdgcn_sched_barrier(0);
    step(j + 2, f2, u2);
    __builtin_amdgcn_sched_barrier(0);
  }
}

void launch_band_solve_blk4(hipStream_t s, int nsubs, const i32* subs, int nmax,
                            const i32* n_arr, const i32* b_arr, const i64* blk_off,
                            const double* LB, const i64* v_off, int K, const double* W,
                            double* Y, const int* active) {
  // the caller guarantees W != Y and a blocked factor built from half-bandwidths <= 64
  if (nsubs == 0 || K == 0 || nmax == 0) return;
  const dim3 gd(nsubs, (nmax + 63) / 64, (K + 15) / 16), gc(nsubs, (K + 15) / 16);
  hipLaunchKernelGGL(k_blk_diag, gd, dim3(256), 0, s, subs, n_arr, blk_off, LB, v_off, K, W, Y,
                     active, 0);
  hipLaunchKernelGGL(k_blk_chain<true>, gc, dim3(256), 0, s, subs, n_arr, b_arr, blk_off, LB,
                     v_off, K, Y, active);
  hipLaunchKernelGGL(k_blk_diag, gd, dim3(256), 0, s, subs, n_arr, blk_off, LB, v_off, K, Y, Y,
                     active, 2);
  hipLaunchKernelGGL(k_blk_chain<false>, gc, dim3(256), 0, s, subs, n_arr, b_arr, blk_off, LB,
                     v_off, K, Y, active);
}

void launch_band_solve_blk(hipStream_t s, int nsubs, const i32* subs, const i32* n_arr,
                           const i32* b_arr, const i64* blk_off, const double* LB,
                           const i64* v_off, int K, const double* W, double* Y,
                           const int* active) {
  // the caller guarantees W != Y and a blocked factor built from half-bandwidths <= 64
  if (nsubs == 0 || K == 0) return;
  hipLaunchKernelGGL(k_band_solve_blk, dim3(nsubs, (K + 15) / 16), dim3(256), 0, s, subs, n_arr,
                     b_arr, blk_off, LB, v_off, K, W, Y, active);
}
