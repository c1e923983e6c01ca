// Band solves with an LDL^T factor (A = Lt D Lt^T, Lt unit lower triangular) for
// gfx950: a one-wavefront blocked variant for any half-bandwidth and rolling-window
// variants for half-bandwidths below 64 (one or many right-hand sides).  The factor
// layouts (ld w = b+1):
//   column layout Fc[c*w + d] = Lt(c+d, c),  row layout Fr[j*w + d] = Lt(j, j-d),
//   and the diagonal slot (d = 0) holds 1/D.
// wave_bcast broadcasts one lane's value to the wavefront (v_readlane).
#pragma once
#include "common.h"

__device__ inline double wave_bcast(double v, int lane) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_readlane(lo, lane);
  hi = __builtin_amdgcn_readlane(hi, lane);
  return __hiloint2double(hi, lo);
}
__device__ inline float wave_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// ---------------------------------------------------------------------------
// Solves with an LDL^T band factor (one or many right-hand sides).
//   F (row layout, ld w = b+1): F[j*w + d] = Lt(j, j-d) for 1 <= d <= b, where
//   Lt is the unit lower triangular factor of A = Lt D Lt^T, and F[j*w] = 1/D_jj.
// Forward sweep Lt y = v (unit diagonal: the diagonal-block chain is one
// broadcast and one FMA per row), then y <- D^{-1} y folded into the first
// touch of each row in the backward sweep Lt^T x = y.
// ---------------------------------------------------------------------------

// Unstaged variant for any b (factor read from global memory), one wavefront.  Forward:
// for each 64-row block, lane l owns row j0 + l; it first subtracts the contributions of
// the rows before the block (up to b back), then the block's own rows by a chain of
// broadcasts, the factor entries of the chain read a 16-step chunk ahead into registers
// (unconditional loads, masked afterwards).  Backward: the same on the reversed order with
// the column entries Lt(j0 + k, row), 1/D folded into each row's first touch.
constexpr int WV_CH = 16;  // steps per prefetched chunk of the in-block chains

// The vector lives in global memory and only a ring of the last (forward) or next
// (backward) M >= b + 64 values in LDS (M a power of two, rmask = M - 1), so that
// LDS no longer bounds the subdomain size or the number of resident wavefronts.  vin is
// read once (times scale, if given) by the forward sweep, which writes y = Lt^{-1} v to
// vout; the backward sweep reads y back from vout (made visible by the barrier between
// the sweeps) and overwrites it with x (times scale).  vin may equal vout.  One wavefront.
template <typename T, typename V, typename G>
__device__ __forceinline__ void wave_ldl_solve_ring(int n, int b, const T* __restrict__ F,
                                                    const G* vin, G* vout,
                                                    const double* __restrict__ scale, V* ring,
                                                    int rmask) {
  const int lane = threadIdx.x & 63;
  const int w = b + 1;
  for (int j0 = 0; j0 < n; j0 += 64) {
    const int nb = min(64, n - j0);
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0;
    if (act) {
      const T* Fr = F + (i64)row * w;
      a = scale ? (V)((double)vin[row] * scale[row]) : (V)vin[row];
      for (int d0 = lane + 1; d0 <= b && row - d0 >= 0; d0 += 16) {
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int dd = d0 + t;
          const bool ok = dd <= b && row - dd >= 0;
          const V lv = (V)Fr[ok ? dd : 0];
          const V xv = ring[(ok ? row - dd : row) & rmask];
          acc += ok ? lv * xv : (V)0;
        }
        a -= acc;
      }
    }
    {
      const int nch = (nb + WV_CH - 1) / WV_CH;
      auto load = [&](int c, V* buf) {
#pragma unroll
        for (int t = 0; t < WV_CH; ++t) {
          const int dd = lane - (WV_CH * c + t);
          const bool ok = act && dd > 0 && dd <= b;
          const V val = (V)F[ok ? (i64)row * w + dd : (i64)0];
          buf[t] = ok ? val : (V)0;
        }
      };
      auto run = [&](int c, const V* buf) {
#pragma unroll
        for (int t = 0; t < WV_CH; ++t) {
          const V yk = wave_bcast(a, WV_CH * c + t);
          a -= buf[t] * yk;
        }
      };
      V l0[WV_CH], l1[WV_CH];
      load(0, l0);
      if (nch > 1) load(1, l1);
      run(0, l0);
      if (nch > 2) load(2, l0);
      if (nch > 1) run(1, l1);
      if (nch > 3) load(3, l1);
      if (nch > 2) run(2, l0);
      if (nch > 3) run(3, l1);
    }
    if (act) {
      ring[row & rmask] = a;
      vout[row] = (G)a;
    }
    __syncthreads();
  }
  for (int j1 = n; j1 > 0; j1 -= 64) {
    const int j0 = max(0, j1 - 64);
    const int nb = j1 - j0;
    const int row = j0 + lane;
    const bool act = lane < nb;
    V a = 0;
    if (act) {
      a = (V)vout[row] * (V)F[(i64)row * w];
      const int imax = min(n - 1, row + b);
      for (int i0 = j1; i0 <= imax; i0 += 16) {
        V acc = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int i = i0 + t;
          const bool ok = i <= imax;
          const int ic = ok ? i : row;
          const V lv = ok ? (V)F[(i64)ic * w + (ic - row)] : (V)0;
          acc += lv * ring[ic & rmask];
        }
        a -= acc;
      }
    }
    {
      const int nch = (nb + WV_CH - 1) / WV_CH;
      auto load = [&](int c, V* buf) {
#pragma unroll
        for (int t = 0; t < WV_CH; ++t) {
          const int k = nb - 1 - (WV_CH * c + t);
          const int dd = k - lane;
          const bool ok = act && k >= 0 && dd > 0 && dd <= b;
          const V val = (V)F[ok ? (i64)(j0 + k) * w + dd : (i64)0];
          buf[t] = ok ? val : (V)0;
        }
      };
      auto run = [&](int c, const V* buf) {
#pragma unroll
        for (int t = 0; t < WV_CH; ++t) {
          const int k = max(nb - 1 - (WV_CH * c + t), 0);
          const V xk = wave_bcast(a, k);
          a -= buf[t] * xk;
        }
      };
      V l0[WV_CH], l1[WV_CH];
      load(0, l0);
      if (nch > 1) load(1, l1);
      run(0, l0);
      if (nch > 2) load(2, l0);
      if (nch > 1) run(1, l1);
      if (nch > 3) load(3, l1);
      if (nch > 2) run(2, l0);
      if (nch > 3) run(3, l1);
    }
    if (act) {
      ring[row & rmask] = a;
      vout[row] = scale ? (G)((double)a * scale[row]) : (G)a;
    }
    __syncthreads();
  }
}

// ring size for wave_ldl_solve_ring: the power of two at or above b + 64
__host__ __device__ inline int wave_ring_size(int b) {
  int m = 64;
  while (m < b + 64) m <<= 1;
  return m;
}

// ---------------------------------------------------------------------------
// Rolling-window LDL^T band solve for b < 64 with one workgroup of ROT_NT
// threads: wavefront 0 runs the substitution, six others stage the factor.
//
//   Fc (column layout, ld w = b+1): Fc[c*w + d] = Lt(c+d, c) for 1 <= d <= b;
//   Fr (row layout):                Fr[j*w + d] = Lt(j, j-d) for 1 <= d <= b,
//                                   Fr[j*w] = 1/D_jj,
//   where A = Lt D Lt^T with Lt unit lower triangular (entries outside the
//   matrix are stored as 0).
//
// Forward sweep Lt y = v: lane l owns the rows r = l (mod 64).  At step j (one
// per row) y_j is final in lane j mod 64; it is broadcast (v_readlane) and every
// lane subtracts Lt(r, j) y_j for its row r.  Because b < 64 a row receives
// contributions only from the 63 rows before it, so a lane carries two
// accumulators: a for its row in the current 64-row block and a2 for its row in
// the next block.  Per block (rows j0..j0+63) the tables
//   Tc[k][l] = Lt(j0+l, j0+k)      (l > k: the row in this block),
//   Tn[k][l] = Lt(j0+64+l, j0+k)   (l < k: the row in the next block),
// zero elsewhere, make step k two FMAs without any lane selection:
//   y = bcast(a, k);  a -= Tc[k][l] y;  a2 -= Tn[k][l] y.
// At the end of a block a holds the block's final y, a <- a2, and a2 <- the
// right-hand side of the block after next.  Entry (column k, offset d) of the
// block's column segment goes to position (k, (k+d) mod 64).
// Backward sweep Lt^T x = D^{-1} y: the same recurrence on the reversed row
// order rho = N-1-j (N = 64 * number of blocks), where it is lower triangular
// with entries Lt(j, j-d); reversed block q' is row block nblk-1-q', whose row
// segment entry (local row kk, offset d) goes to position (63-kk, (63-kk+d) mod
// 64).  Both sweeps thus write the same table positions, which are zeroed once.
// The staging wavefronts build the tables of the next step in the other LDS
// buffer from the contiguous band segment (read into registers one step ahead),
// so the substitution reads only LDS.
//   v:     the right-hand side (LDS, n entries), overwritten by the solution;
//   tiles: 2 * ROT_TILE entries of V in LDS.
// All ROT_NT threads must call it.
// ---------------------------------------------------------------------------
constexpr int ROT_NT = 512;
constexpr int ROT_TILE = 2 * 4096 + 64;          // Tc, Tn, 1/D of the next block's rows
// Staging threads: in FP64, wavefronts 1-3 and 5-7, wavefront 4 (which shares the
// substitution's SIMD: wavefront w runs on SIMD w mod 4) only taking part in the barriers
// (measured on 1225-row subdomains: 61.3 -> 58.6 us per apply); in FP32, whose faster
// substitution leaves the staging the longer part, all seven.
template <typename V>
struct RotStage {
  static constexpr bool skip4 = sizeof(V) == 8;
  static constexpr int ns = skip4 ? ROT_NT - 128 : ROT_NT - 64;
  static constexpr int per = (64 * 64 + ns - 1) / ns;  // segment entries per stager
};

// 64 substitution steps of one block, in chunks of CH; the table entries of chunk
// c+1 are read while chunk c runs (scheduling barriers keep the reads ahead).
// Registers: 4*CH values of V for the table entries.
template <typename V, int CH = 16>
__device__ __forceinline__ void rot_block(const V* buf, int lane, V& a, V& a2) {
  constexpr int NC = 64 / CH;
  const V* Tc = buf;
  const V* Tn = buf + 4096;
  V tc[2][CH], tn[2][CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    tc[0][t] = Tc[t * 64 + lane];
    tn[0][t] = Tn[t * 64 + lane];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c + 1 < NC) {
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        tc[(c + 1) & 1][t] = Tc[(CH * (c + 1) + t) * 64 + lane];
        tn[(c + 1) & 1][t] = Tn[(CH * (c + 1) + t) * 64 + lane];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const V y = wave_bcast(a, CH * c + t);
      a -= tc[c & 1][t] * y;
      a2 -= tn[c & 1][t] * y;
    }
    // keep the a2 updates inside their chunk (otherwise they are sunk to the end
    // of the block, holding 64 broadcast values in scalar registers)
    asm volatile("" : "+v"(a2));
    __builtin_amdgcn_sched_barrier(0);
  }
}

//   init(): called by all threads once the first table segment's reads are in flight;
//   fills v (the reads of the segment and of the vector then overlap).
template <typename T, typename V, typename Init>
__device__ __forceinline__ void wg_ldl_solve_rot(int n, int b, const T* __restrict__ Fc,
                                                 const T* __restrict__ Fr, V* v, V* tiles,
                                                 Init init) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = b + 1;
  const int nblk = (n + 63) >> 6;
  const int nsteps = 2 * nblk;
  const int N = nblk * 64;
  const int seg = 64 * w;
  constexpr int NS = RotStage<V>::ns;
  constexpr int ROT_PER = RotStage<V>::per;
  const bool stager = wave > 0 && !(RotStage<V>::skip4 && wave == 4);
  // staging thread index
  const int tl = (RotStage<V>::skip4 && wave > 4) ? threadIdx.x - 128 : threadIdx.x - 64;
  // staging registers: one segment of the step after next
  T gv[ROT_PER];
  int gpos[ROT_PER];  // table position (k*64 + l) + 1, 0 = no entry; bit 30 = Tn
  T gd = 0;
  auto stage_load = [&](int s) {
    const bool fwd = s < nblk;
    const int q = fwd ? s : nsteps - 1 - s;  // row block
    const int j0 = q * 64;
    const T* src = (fwd ? Fc : Fr) + (i64)j0 * w;
    const int cnt = min(64, n - j0) * w;
#pragma unroll
    for (int u = 0; u < ROT_PER; ++u) {
      const int e = tl + u * NS;
      const int kk = e / w, d = e - kk * w;
      int pos = 0;
      if (e < cnt && d > 0) {
        const int k = fwd ? kk : 63 - kk;
        const int l = (k + d) & 63;
        pos = (k * 64 + l + 1) | ((l > k) ? 0 : (1 << 30));
      }
      gpos[u] = pos;
      gv[u] = src[min(e, cnt - 1)];
    }
    gd = 0;
    // 1/D of the rows of the next reversed block (row block q-1), lane order of
    // the reversed rows: lane l <-> row j0 - 1 - l
    if (!fwd && tl < 64 && q > 0) gd = Fr[(i64)(j0 - 1 - tl) * w];
  };
  auto stage_store = [&](V* buf) {
#pragma unroll
    for (int u = 0; u < ROT_PER; ++u) {
      const int pos = gpos[u];
      if (pos) {
        const int p = (pos & ((1 << 30) - 1)) - 1;
        buf[(pos >> 30) ? 4096 + p : p] = (V)gv[u];
      }
    }
    if (tl < 64) buf[8192 + tl] = (V)gd;
  };
  // read step 0's segment, zero both buffers (positions without an entry stay zero) and
  // fill the vector while it is in flight, then stage step 0
  if (stager) stage_load(0);
  for (int t = threadIdx.x; t < 2 * ROT_TILE; t += ROT_NT) tiles[t] = (V)0;
  init();
  __syncthreads();
  if (stager) {
    stage_store(tiles);
    if (nsteps > 1) stage_load(1);
  }
  __syncthreads();
  V a = 0, a2 = 0;
  for (int s = 0; s < nsteps; ++s) {
    V* buf = tiles + (s & 1) * ROT_TILE;
    if (wave > 0) {
      if (stager && s + 1 < nsteps) {
        stage_store(tiles + ((s + 1) & 1) * ROT_TILE);
        if (s + 2 < nsteps) stage_load(s + 2);
      }
    } else if (s < nblk) {  // forward, row block s
      const int row = s * 64 + lane;
      if (s == 0) a = row < n ? v[row] : (V)0;
      a2 = row + 64 < n ? v[row + 64] : (V)0;
      rot_block<V>(buf, lane, a, a2);
      if (row < n) v[row] = a;
      a = a2;
    } else {  // backward, reversed block s - nblk: lane l <-> row N-1-(64(s-nblk)+l)
      const int row = N - 1 - (64 * (s - nblk) + lane);
      if (s == nblk) a = row < n ? v[row] * (V)Fr[(i64)row * w] : (V)0;
      a2 = (row - 64 >= 0 && row - 64 < n) ? v[row - 64] * buf[8192 + lane] : (V)0;
      rot_block<V>(buf, lane, a, a2);
      if (row < n) v[row] = a;
      a = a2;
    }
    // the solution vector and the tables are in LDS; the staging loads of the block
    // after next stay in flight across the barrier
    lds_barrier();
  }
}

// ---------------------------------------------------------------------------
// Many right-hand sides (b < 64): one workgroup of NW wavefronts, wavefront w runs
// the rolling-window recurrence of wg_ldl_solve_rot on column w of V (global
// memory, column-major, ld = n; overwritten by the solution), and all threads
// stage the shared tables (ceil(w / NW) band entries each per block).  The column
// values a block needs (right-hand side of the next block, or D^{-1} y of the next
// reversed block) are read from global memory one block ahead.  Columns w >= ncol
// run on zeros.  The forward results are made visible to the backward sweep, which
// reads them in another lane order, by a workgroup barrier with a memory fence.
//   tiles: 2 * ROT_TILE entries of V in LDS (the 1/D slots are unused here).
// ---------------------------------------------------------------------------
template <typename T, typename V, int NW>
__device__ __forceinline__ void wg_ldl_solve_rot_cols(int n, int b, const T* __restrict__ Fc,
                                                      const T* __restrict__ Fr, V* __restrict__ X,
                                                      int ncol, V* tiles) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  constexpr int NTH = 64 * NW;
  constexpr int PER = (64 * 64 + NTH - 1) / NTH;
  const int w = b + 1;
  const int nblk = (n + 63) >> 6;
  const int nsteps = 2 * nblk;
  const int N = nblk * 64;
  const bool has = wave < ncol;
  V* v = X + (i64)(has ? wave : 0) * n;
  T gv[PER];
  int gpos[PER];
  auto stage_load = [&](int s) {
    const bool fwd = s < nblk;
    const int q = fwd ? s : nsteps - 1 - s;
    const int j0 = q * 64;
    const T* src = (fwd ? Fc : Fr) + (i64)j0 * w;
    const int cnt = min(64, n - j0) * w;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NTH;
      const int kk = e / w, d = e - kk * w;
      int pos = 0;
      if (e < cnt && d > 0) {
        const int k = fwd ? kk : 63 - kk;
        const int l = (k + d) & 63;
        pos = (k * 64 + l + 1) | ((l > k) ? 0 : (1 << 30));
      }
      gpos[u] = pos;
      gv[u] = src[min(e, cnt - 1)];
    }
  };
  auto stage_store = [&](V* buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int pos = gpos[u];
      if (pos) {
        const int p = (pos & ((1 << 30) - 1)) - 1;
        buf[(pos >> 30) ? 4096 + p : p] = (V)gv[u];
      }
    }
  };
  for (int t = tid; t < 2 * ROT_TILE; t += NTH) tiles[t] = (V)0;
  __syncthreads();
  stage_load(0);
  stage_store(tiles);
  if (nsteps > 1) stage_load(1);
  V a = 0, a2 = 0, nxt = 0;
  // value for the first block's a2 (forward: right-hand side of rows 64..127)
  {
    const int row = 64 + lane;
    nxt = (has && row < n) ? v[row] : (V)0;
  }
  if (has && lane < n) a = v[lane];
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    V* buf = tiles + (s & 1) * ROT_TILE;
    if (s + 1 < nsteps) {
      stage_store(tiles + ((s + 1) & 1) * ROT_TILE);
      if (s + 2 < nsteps) stage_load(s + 2);
    }
    if (s < nblk) {  // forward, row block s
      const int row = s * 64 + lane;
      a2 = nxt;
      // prefetch the next block's a2 (rows of the block after next)
      nxt = (has && row + 128 < n) ? v[row + 128] : (V)0;
      rot_block<V, (NW > 8 ? 8 : 16)>(buf, lane, a, a2);
      if (has && row < n) v[row] = a;
      a = a2;
      if (s == nblk - 1) {
        // forward done: make y visible, then start the reversed sweep
        __threadfence_block();
        __syncthreads();
        const int r0 = N - 1 - lane;
        a = (has && r0 < n) ? v[r0] * (V)Fr[(i64)r0 * w] : (V)0;
        const int r1 = r0 - 64;
        nxt = (has && r1 >= 0 && r1 < n) ? v[r1] * (V)Fr[(i64)r1 * w] : (V)0;
      }
    } else {  // backward, reversed block s - nblk: lane l <-> row N-1-(64(s-nblk)+l)
      const int row = N - 1 - (64 * (s - nblk) + lane);
      a2 = nxt;
      const int r2 = row - 128;
      nxt = (has && r2 >= 0 && r2 < n) ? v[r2] * (V)Fr[(i64)r2 * w] : (V)0;
      rot_block<V, (NW > 8 ? 8 : 16)>(buf, lane, a, a2);
      if (has && row < n) v[row] = a;
      a = a2;
    }
    // tables in LDS; each lane's global rows are its own until the sweep changes
    // direction (full barrier above), so prefetches stay in flight across this one
    lds_barrier();
  }
}

// ---------------------------------------------------------------------------
// Rolling-window step for NC right-hand sides per wavefront: each table entry read
// from LDS feeds NC independent chains (NC broadcasts and 2 NC FMAs per row), which
// divides the LDS traffic per right-hand side by NC.  With one column per wavefront
// and 16 wavefronts per workgroup the table reads (16 KB per row step) bound the solve.
// ---------------------------------------------------------------------------
template <typename V, int CH, int NC>
__device__ __forceinline__ void rot_block_m(const V* buf, int lane, V (&a)[NC], V (&a2)[NC]) {
  constexpr int NCH = 64 / CH;
  const V* Tc = buf;
  const V* Tn = buf + 4096;
  V tc[2][CH], tn[2][CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    tc[0][t] = Tc[t * 64 + lane];
    tn[0][t] = Tn[t * 64 + lane];
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    if (c + 1 < NCH) {
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        tc[(c + 1) & 1][t] = Tc[(CH * (c + 1) + t) * 64 + lane];
        tn[(c + 1) & 1][t] = Tn[(CH * (c + 1) + t) * 64 + lane];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const V y = wave_bcast(a[q], CH * c + t);
        a[q] -= tc[c & 1][t] * y;
        a2[q] -= tn[c & 1][t] * y;
      }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) asm volatile("" : "+v"(a2[q]));
    __builtin_amdgcn_sched_barrier(0);
  }
}

// As wg_ldl_solve_rot_cols, with NW wavefronts of NC columns each (wavefront w owns
// columns w*NC .. w*NC+NC-1 of X; columns >= ncol run on zeros).
template <typename T, typename V, int NW, int NC>
__device__ __forceinline__ void wg_ldl_solve_rot_mcols(int n, int b, const T* __restrict__ Fc,
                                                       const T* __restrict__ Fr,
                                                       V* __restrict__ X, int ncol, V* tiles) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  constexpr int NTH = 64 * NW;
  constexpr int PER = (64 * 64 + NTH - 1) / NTH;
  const int w = b + 1;
  const int nblk = (n + 63) >> 6;
  const int nsteps = 2 * nblk;
  const int N = nblk * 64;
  bool has[NC];
  V* v[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int col = wave * NC + q;
    has[q] = col < ncol;
    v[q] = X + (i64)(has[q] ? col : 0) * n;
  }
  T gv[PER];
  int gpos[PER];
  auto stage_load = [&](int s) {
    const bool fwd = s < nblk;
    const int qb = fwd ? s : nsteps - 1 - s;
    const int j0 = qb * 64;
    const T* src = (fwd ? Fc : Fr) + (i64)j0 * w;
    const int cnt = min(64, n - j0) * w;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NTH;
      const int kk = e / w, d = e - kk * w;
      int pos = 0;
      if (e < cnt && d > 0) {
        const int k = fwd ? kk : 63 - kk;
        const int l = (k + d) & 63;
        pos = (k * 64 + l + 1) | ((l > k) ? 0 : (1 << 30));
      }
      gpos[u] = pos;
      gv[u] = src[min(e, cnt - 1)];
    }
  };
  auto stage_store = [&](V* buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int pos = gpos[u];
      if (pos) {
        const int p = (pos & ((1 << 30) - 1)) - 1;
        buf[(pos >> 30) ? 4096 + p : p] = (V)gv[u];
      }
    }
  };
  for (int t = tid; t < 2 * ROT_TILE; t += NTH) tiles[t] = (V)0;
  __syncthreads();
  stage_load(0);
  stage_store(tiles);
  if (nsteps > 1) stage_load(1);
  V a[NC], a2[NC], nxt[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int row = 64 + lane;
    nxt[q] = (has[q] && row < n) ? v[q][row] : (V)0;
    a[q] = (has[q] && lane < n) ? v[q][lane] : (V)0;
    a2[q] = 0;
  }
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    V* buf = tiles + (s & 1) * ROT_TILE;
    if (s + 1 < nsteps) {
      stage_store(tiles + ((s + 1) & 1) * ROT_TILE);
      if (s + 2 < nsteps) stage_load(s + 2);
    }
    if (s < nblk) {  // forward, row block s
      const int row = s * 64 + lane;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        a2[q] = nxt[q];
        nxt[q] = (has[q] && row + 128 < n) ? v[q][row + 128] : (V)0;
      }
      rot_block_m<V, 8, NC>(buf, lane, a, a2);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (has[q] && row < n) v[q][row] = a[q];
        a[q] = a2[q];
      }
      if (s == nblk - 1) {
        // forward done: make y visible, then start the reversed sweep
        __threadfence_block();
        __syncthreads();
        const int r0 = N - 1 - lane;
        const int r1 = r0 - 64;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          a[q] = (has[q] && r0 < n) ? v[q][r0] * (V)Fr[(i64)r0 * w] : (V)0;
          nxt[q] = (has[q] && r1 >= 0 && r1 < n) ? v[q][r1] * (V)Fr[(i64)r1 * w] : (V)0;
        }
      }
    } else {  // backward, reversed block s - nblk: lane l <-> row N-1-(64(s-nblk)+l)
      const int row = N - 1 - (64 * (s - nblk) + lane);
      const int r2 = row - 128;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        a2[q] = nxt[q];
        nxt[q] = (has[q] && r2 >= 0 && r2 < n) ? v[q][r2] * (V)Fr[(i64)r2 * w] : (V)0;
      }
      rot_block_m<V, 8, NC>(buf, lane, a, a2);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (has[q] && row < n) v[q][row] = a[q];
        a[q] = a2[q];
      }
    }
    lds_barrier();  // as in wg_ldl_solve_rot_cols
  }
}

// As wg_ldl_solve_rot_mcols with NS more wavefronts that only stage the tables, so
// the NW computing wavefronts run nothing but the recurrence (workgroup of
// 64 (NW + NS) threads).  The change of sweep direction is a full barrier that every
// thread executes.
template <typename T, typename V, int NW, int NC, int NS>
__device__ __forceinline__ void wg_ldl_solve_rot_mcols_st(int n, int b, const T* __restrict__ Fc,
                                                          const T* __restrict__ Fr,
                                                          V* __restrict__ X, int ncol, V* tiles) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  constexpr int NST = 64 * NS;
  constexpr int PER = (64 * 64 + NST - 1) / NST;
  const bool stager = wave >= NW;
  const int tl = tid - 64 * NW;  // staging thread index
  const int w = b + 1;
  const int nblk = (n + 63) >> 6;
  const int nsteps = 2 * nblk;
  const int N = nblk * 64;
  bool has[NC];
  V* v[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int col = wave * NC + q;
    has[q] = !stager && col < ncol;
    v[q] = X + (i64)(has[q] ? col : 0) * n;
  }
  T gv[PER];
  int gpos[PER];
  auto stage_load = [&](int s) {
    const bool fwd = s < nblk;
    const int qb = fwd ? s : nsteps - 1 - s;
    const int j0 = qb * 64;
    const T* src = (fwd ? Fc : Fr) + (i64)j0 * w;
    const int cnt = min(64, n - j0) * w;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tl + u * NST;
      const int kk = e / w, d = e - kk * w;
      int pos = 0;
      if (e < cnt && d > 0) {
        const int k = fwd ? kk : 63 - kk;
        const int l = (k + d) & 63;
        pos = (k * 64 + l + 1) | ((l > k) ? 0 : (1 << 30));
      }
      gpos[u] = pos;
      gv[u] = src[min(e, cnt - 1)];
    }
  };
  auto stage_store = [&](V* buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int pos = gpos[u];
      if (pos) {
        const int p = (pos & ((1 << 30) - 1)) - 1;
        buf[(pos >> 30) ? 4096 + p : p] = (V)gv[u];
      }
    }
  };
  for (int t = tid; t < 2 * ROT_TILE; t += 64 * (NW + NS)) tiles[t] = (V)0;
  __syncthreads();
  if (stager) {
    stage_load(0);
    stage_store(tiles);
    if (nsteps > 1) stage_load(1);
  }
  V a[NC], a2[NC], nxt[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int row = 64 + lane;
    nxt[q] = (has[q] && row < n) ? v[q][row] : (V)0;
    a[q] = (has[q] && lane < n) ? v[q][lane] : (V)0;
    a2[q] = 0;
  }
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    V* buf = tiles + (s & 1) * ROT_TILE;
    if (stager) {
      if (s + 1 < nsteps) {
        stage_store(tiles + ((s + 1) & 1) * ROT_TILE);
        if (s + 2 < nsteps) stage_load(s + 2);
      }
    } else if (s < nblk) {  // forward, row block s
      const int row = s * 64 + lane;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        a2[q] = nxt[q];
        nxt[q] = (has[q] && row + 128 < n) ? v[q][row + 128] : (V)0;
      }
      rot_block_m<V, 4, NC>(buf, lane, a, a2);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (has[q] && row < n) v[q][row] = a[q];
        a[q] = a2[q];
      }
    } else {  // backward, reversed block s - nblk: lane l <-> row N-1-(64(s-nblk)+l)
      const int row = N - 1 - (64 * (s - nblk) + lane);
      const int r2 = row - 128;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        a2[q] = nxt[q];
        nxt[q] = (has[q] && r2 >= 0 && r2 < n) ? v[q][r2] * (V)Fr[(i64)r2 * w] : (V)0;
      }
      rot_block_m<V, 4, NC>(buf, lane, a, a2);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (has[q] && row < n) v[q][row] = a[q];
        a[q] = a2[q];
      }
    }
    if (s == nblk - 1) {
      // forward done (every thread takes this barrier): make y visible, then start the
      // reversed sweep, which reads rows written by other lanes
      __threadfence_block();
      __syncthreads();
      const int r0 = N - 1 - lane;
      const int r1 = r0 - 64;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        a[q] = (has[q] && r0 < n) ? v[q][r0] * (V)Fr[(i64)r0 * w] : (V)0;
        nxt[q] = (has[q] && r1 >= 0 && r1 < n) ? v[q][r1] * (V)Fr[(i64)r1 * w] : (V)0;
      }
    }
    lds_barrier();
  }
}
