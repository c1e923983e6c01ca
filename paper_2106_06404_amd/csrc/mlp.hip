// Warm-start network of the local eigensolver: a three-layer perceptron
//   h1 = relu(x W1 + b1),  h2 = relu(h1 W2 + b2),  y = h2 W3 + b3,
// whose output, read as n_vec vectors on a subdomain's node frame, starts the
// block iteration for the GEVP of Sec. 2.3.  Training minimises the share of the
// method's own eigenvectors that lies outside the span of the output block (a
// least-squares projection loss), with Adam.
//
// Kernels:
//   k_sgemm       FP32 tiled GEMM (64x64 tiles, 4x4 per thread, LDS staging of 16-deep
//                 k slices), operands optionally transposed, split-K into partial sums
//   k_splitk_epi  sum of the split-K partials + bias + relu, or times relu'(h)
//   k_colsum      bias gradients (column sums)
//   k_proj_loss   per-sample projection loss and its gradient w.r.t. the output
//   k_adam        Adam update of all parameters
//   k_hgemm       BF16 inference GEMM on the matrix cores (v_mfma_f32_16x16x16_bf16),
//                 FP32 accumulation, fused bias + relu
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// FP32 GEMM: C_z = sum_{k in split z} opA(A)[m,k] opB(B)[k,n]
//   TA = 0: A is M x K row-major (A[m*lda + k]); TA = 1: A is stored K x M (A[k*lda + m])
//   TB = 0: B is K x N row-major (B[k*ldb + n]); TB = 1: B is stored N x K (B[n*ldb + k])
// C_z = C + z*M*N (row-major, ldc = N).  Grid: (ceil(N/64), ceil(M/64), splits).
// ---------------------------------------------------------------------------
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, int kchunk,
                                               const float* __restrict__ A, int lda,
                                               const float* __restrict__ B, int ldb,
                                               float* __restrict__ C) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int t = threadIdx.x;
  const int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int tx = t & 15, ty = t >> 4;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u;
      int r, c;
      if (TA) {
        r = e & 63;
        c = e >> 6;
      } else {
        c = e & 15;
        r = e >> 4;
      }
      const int m = m0 + r, k = k0 + c;
      float v = 0.f;
      if (m < M && k < ke) v = TA ? A[(i64)k * lda + m] : A[(i64)m * lda + k];
      As[c][r] = v;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u;
      int r, c;
      if (TB) {
        c = e & 15;
        r = e >> 4;
      } else {
        r = e & 63;
        c = e >> 6;
      }
      const int n = n0 + r, k = k0 + c;
      float v = 0.f;
      if (n < N && k < ke) v = TB ? B[(i64)n * ldb + k] : B[(i64)k * ldb + n];
      Bs[c][r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  float* Cz = C + (i64)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n < N) Cz[(i64)m * N + n] = acc[i][j];
    }
  }
}

// out[m,n] = epilogue(sum_z part[z][m,n]):
//   mode 0: + bias[n] (bias may be null);  mode 1: + bias, relu;
//   mode 2: times [h[m,n] > 0] (relu' of the layer output h)
__global__ void k_splitk_epi(int M, int N, int splits, const float* __restrict__ part,
                             const float* __restrict__ bias, const float* __restrict__ h, int mode,
                             float* __restrict__ out) {
  const i64 MN = (i64)M * N;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < MN; e += (i64)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[z * MN + e];
    const int n = (int)(e % N);
    if (mode <= 1 && bias) s += bias[n];
    if (mode == 1) s = fmaxf(s, 0.f);
    if (mode == 2) s = h[e] > 0.f ? s : 0.f;
    out[e] = s;
  }
}

// g[n] = sum_m D[m, n]  (one thread per column; M is the batch size)
__global__ void k_colsum(int M, int N, const float* __restrict__ D, float* __restrict__ g) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += D[(i64)m * N + n];
  g[n] = s;
}

// rows x[idx[b]] of a sample matrix (n_in wide) into a batch
__global__ void k_gather_rows(int B, int w, const int* __restrict__ idx, const float* __restrict__ src,
                              float* __restrict__ dst) {
  const i64 tot = (i64)B * w;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (i64)gridDim.x * blockDim.x) {
    const int b = (int)(e / w), c = (int)(e % w);
    dst[e] = src[(i64)idx[b] * w + c];
  }
}

// ---------------------------------------------------------------------------
// Projection loss of one sample per workgroup (256 threads):
//   Ys = diag(s) Y (n_pos x V, vector v = y[v*n_pos ...]), T = first m targets,
//   G = Ys^T Ys + ridge I, C = Ys^T T, loss = 1 - tr(C^T G^{-1} C)/m,
//   dy = diag(s) (-(2/m)) (T (G^{-1}C)^T - Ys (G^{-1}C)(G^{-1}C)^T) / B.
// G and C are accumulated in FP32 over the frame; the V x V algebra runs in FP64.
// ---------------------------------------------------------------------------
constexpr int LOSS_CH = 128;  // frame rows staged per chunk

__global__ __launch_bounds__(256) void k_proj_loss(
    int B, int V, int n_pos, int m_cap, const int* __restrict__ idx, const float* __restrict__ y,
    const float* __restrict__ tgt, const float* __restrict__ mask, const int* __restrict__ cnt,
    double ridge, float* __restrict__ dy, float* __restrict__ loss_b) {
  const int b = blockIdx.x;
  const int s_id = idx ? idx[b] : b;
  const int m = min(cnt[s_id], m_cap);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int out = V * n_pos;
  const float* yb = y + (i64)b * out;
  const float* tb = tgt + (i64)s_id * m_cap * n_pos;
  const float* sb = mask + (i64)s_id * n_pos;
  float* dyb = dy + (i64)b * out;
  __shared__ float Ych[16][LOSS_CH], Tch[16][LOSS_CH];
  __shared__ double G[16 * 16], Cm[16 * 16], Q[16 * 16], L[16 * 16], GiC[16 * 16];
  __shared__ double sh_loss;
  if (m <= 0) {
    for (i64 e = tid; e < out; e += nt) dyb[e] = 0.f;
    if (tid == 0) loss_b[b] = 0.f;
    return;
  }
  // each thread owns up to two of the V*V + V*m sums
  const int nG = V * V, nC = V * m, nsum = nG + nC;
  float acc[2] = {0.f, 0.f};
  for (int r0 = 0; r0 < n_pos; r0 += LOSS_CH) {
    const int rn = min(LOSS_CH, n_pos - r0);
    for (int e = tid; e < V * LOSS_CH; e += nt) {
      const int v = e / LOSS_CH, r = e % LOSS_CH;
      Ych[v][r] = r < rn ? yb[(i64)v * n_pos + r0 + r] * sb[r0 + r] : 0.f;
    }
    for (int e = tid; e < m * LOSS_CH; e += nt) {
      const int j = e / LOSS_CH, r = e % LOSS_CH;
      Tch[j][r] = r < rn ? tb[(i64)j * n_pos + r0 + r] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = tid + u * nt;
      if (q >= nsum) continue;
      float s = 0.f;
      if (q < nG) {
        const int a = q / V, c = q % V;
        for (int r = 0; r < rn; ++r) s += Ych[a][r] * Ych[c][r];
      } else {
        const int a = (q - nG) / m, j = (q - nG) % m;
        for (int r = 0; r < rn; ++r) s += Ych[a][r] * Tch[j][r];
      }
      acc[u] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = tid + u * nt;
    if (q >= nsum) continue;
    if (q < nG) {
      const int a = q / V, c = q % V;
      G[a * V + c] = (double)acc[u] + (a == c ? ridge : 0.0);
    } else {
      const int a = (q - nG) / m, j = (q - nG) % m;
      Cm[a * m + j] = (double)acc[u];
    }
  }
  __syncthreads();
  // Cholesky G = L L^T and GiC = G^{-1} C (thread 0; V <= 16)
  if (tid == 0) {
    for (int j = 0; j < V; ++j) {
      double d = G[j * V + j];
      for (int k = 0; k < j; ++k) d -= L[j * V + k] * L[j * V + k];
      d = d > 0.0 ? sqrt(d) : 1e-300;
      L[j * V + j] = d;
      for (int i = j + 1; i < V; ++i) {
        double s = G[i * V + j];
        for (int k = 0; k < j; ++k) s -= L[i * V + k] * L[j * V + k];
        L[i * V + j] = s / d;
      }
    }
    double tr = 0.0;
    for (int j = 0; j < m; ++j) {
      double w[16];
      for (int i = 0; i < V; ++i) {  // L w = C[:, j]
        double s = Cm[i * m + j];
        for (int k = 0; k < i; ++k) s -= L[i * V + k] * w[k];
        w[i] = s / L[i * V + i];
      }
      for (int i = V - 1; i >= 0; --i) {  // L^T g = w
        double s = w[i];
        for (int k = i + 1; k < V; ++k) s -= L[k * V + i] * GiC[k * m + j];
        GiC[i * m + j] = s / L[i * V + i];
      }
      for (int i = 0; i < V; ++i) tr += Cm[i * m + j] * GiC[i * m + j];
    }
    sh_loss = 1.0 - tr / m;
  }
  __syncthreads();
  // Q = GiC GiC^T (V x V)
  for (int q = tid; q < V * V; q += nt) {
    const int a = q / V, c = q % V;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += GiC[a * m + j] * GiC[c * m + j];
    Q[q] = s;
  }
  __syncthreads();
  const double f = -2.0 / (double)m / (double)B;
  // one frame row per thread: all V outputs of the row from its m targets and V values
  for (int r = tid; r < n_pos; r += nt) {
    const float sr = sb[r];
    float tv[16], yv[16];
    for (int j = 0; j < m; ++j) tv[j] = sr != 0.f ? tb[(i64)j * n_pos + r] : 0.f;
    for (int u = 0; u < V; ++u) yv[u] = yb[(i64)u * n_pos + r] * sr;
    for (int v = 0; v < V; ++v) {
      double acc2 = 0.0;
      for (int j = 0; j < m; ++j) acc2 += (double)tv[j] * GiC[v * m + j];
      for (int u = 0; u < V; ++u) acc2 -= (double)yv[u] * Q[u * V + v];
      dyb[(i64)v * n_pos + r] = sr != 0.f ? (float)(f * acc2) * sr : 0.f;
    }
  }
  if (tid == 0) loss_b[b] = (float)sh_loss;
}

// Adam with bias correction (step counts from 1)
__global__ void k_adam(i64 n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ mo, float* __restrict__ ve, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (i64)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * mo[e] + (1.f - b1) * gi;
    const float vi = b2 * ve[e] + (1.f - b2) * gi * gi;
    mo[e] = mi;
    ve[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Glorot-uniform weights from a counter-based generator (splitmix64 finaliser of
// seed ^ index); biases zero.  w[e] for e in [lo, hi) gets U(-a, a).
__global__ void k_init_uniform(i64 lo, i64 hi, float a, unsigned long long seed, float* __restrict__ w) {
  for (i64 e = lo + (i64)blockIdx.x * blockDim.x + threadIdx.x; e < hi; e += (i64)gridDim.x * blockDim.x) {
    unsigned long long x = seed ^ (unsigned long long)e;
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    const double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
    w[e] = (float)((2.0 * u - 1.0) * a);
  }
}

// ---------------------------------------------------------------------------
// BF16 inference
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  // round to nearest even; NaN stays NaN
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// dst[r*ldd + c] = bf16(src[r*lds + c]) for c < cols, 0 for cols <= c < ldd  (rows x ldd)
__global__ void k_to_bf16(int rows, int cols, int ldd, const float* __restrict__ src, int lds,
                          unsigned short* __restrict__ dst) {
  const i64 tot = (i64)rows * ldd;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (i64)gridDim.x * blockDim.x) {
    const int r = (int)(e / ldd), c = (int)(e % ldd);
    dst[e] = c < cols ? f32_to_bf16(src[(i64)r * lds + c]) : (unsigned short)0;
  }
}

// dst[c*ldd + r] = bf16(src[r*lds + c]) (transpose; rows r < rows, zero pad to ldd)
__global__ void k_to_bf16_t(int rows, int cols, int ldd, const float* __restrict__ src, int lds,
                            unsigned short* __restrict__ dst) {
  const i64 tot = (i64)cols * ldd;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (i64)gridDim.x * blockDim.x) {
    const int c = (int)(e / ldd), r = (int)(e % ldd);
    dst[e] = r < rows ? f32_to_bf16(src[(i64)r * lds + c]) : (unsigned short)0;
  }
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// C[m, n] = act(sum_k A[m, k] Bt[n, k] + bias[n]), A: M x Kp, Bt: N x Kp (bf16, Kp a
// multiple of 16, zero padded).  One wave computes a 32 x 32 block as 2 x 2 MFMA tiles
// of 16 x 16; a workgroup of 4 waves covers 64 x 64.  MFMA operand layout (16x16x16):
// lane l supplies A[l % 16][4*(l/16) + 0..3] and B[4*(l/16) + 0..3][l % 16]; the result
// lane l holds D[4*(l/16) + j][l % 16], j = 0..3.
// out_bf16: write bf16 (hidden layers, row stride ldc) else fp32 (row stride ldc).
__global__ __launch_bounds__(256) void k_hgemm(int M, int N, int Kp, const unsigned short* __restrict__ A,
                                               const unsigned short* __restrict__ Bt,
                                               const float* __restrict__ bias, int relu,
                                               int out_bf16, void* __restrict__ Cout, int ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (w & 1) * 32;
  const int lr = lane & 15, lk = (lane >> 4) * 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // clamped rows keep every load in bounds; their results are not stored
  const int ma0 = min(m0 + lr, M - 1), ma1 = min(m0 + 16 + lr, M - 1);
  const int nb0 = min(n0 + lr, N - 1), nb1 = min(n0 + 16 + lr, N - 1);
  const unsigned short* a0p = A + (i64)ma0 * Kp + lk;
  const unsigned short* a1p = A + (i64)ma1 * Kp + lk;
  const unsigned short* b0p = Bt + (i64)nb0 * Kp + lk;
  const unsigned short* b1p = Bt + (i64)nb1 * Kp + lk;
  for (int k = 0; k < Kp; k += 16) {
    const bf16x4 a0 = *reinterpret_cast<const bf16x4*>(a0p + k);
    const bf16x4 a1 = *reinterpret_cast<const bf16x4*>(a1p + k);
    const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(b0p + k);
    const bf16x4 b1 = *reinterpret_cast<const bf16x4*>(b1p + k);
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc[1][1], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + 16 * j + lr;
      if (n >= N) continue;
      const float bn = bias ? bias[n] : 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 16 * i + lk + q;
        if (m >= M) continue;
        float v = acc[i][j][q] + bn;
        if (relu) v = fmaxf(v, 0.f);
        if (out_bf16)
          reinterpret_cast<unsigned short*>(Cout)[(i64)m * ldc + n] = f32_to_bf16(v);
        else
          reinterpret_cast<float*>(Cout)[(i64)m * ldc + n] = v;
      }
    }
}

// ---------------------------------------------------------------------------
// Eigensolver start block from the network output (K columns, column-major per
// subdomain like k_eig_init): column c < n_vec of a warm subdomain takes
// y[sample, c*n_pos + pos[row]]; other columns, cold subdomains and non-finite
// network values take the counter-based random start.  Rows with zero weight get 0.
// ---------------------------------------------------------------------------
__device__ inline double warm_hash_uniform(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_eig_init_warm(i64 total_rows, const i32* __restrict__ row_sub,
                                const i64* __restrict__ voff, const i32* __restrict__ nb,
                                const i64* __restrict__ kvoff, int K, const double* __restrict__ dv,
                                double* __restrict__ X, unsigned long long seed,
                                const i32* __restrict__ seed_id, const int* __restrict__ warm,
                                const float* __restrict__ yw, int n_vec, int n_pos,
                                const i32* __restrict__ pos) {
  i64 g = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total_rows) return;
  const int i = row_sub[g];
  const int r = (int)(g - voff[i]);
  const int n = nb[i];
  double* Xi = X + kvoff[i];
  const bool z = dv[g] == 0.0;
  const unsigned long long sid = (unsigned long long)seed_id[i];
  const bool wi = warm[i] != 0;
  const int pr = pos[g];
  for (int c = 0; c < K; ++c) {
    double v;
    float yv = 0.f;
    const bool use = wi && c < n_vec && pr >= 0;
    if (use) yv = yw[(i64)i * n_vec * n_pos + (i64)c * n_pos + pr];
    if (use && isfinite(yv)) {
      v = (double)yv;
    } else {
      const unsigned long long key = seed ^ (sid << 40) ^ ((unsigned long long)r << 12) ^
                                     (unsigned long long)c;
      v = warm_hash_uniform(key);
    }
    Xi[r + (i64)c * n] = z ? 0.0 : v;
  }
}

// Training targets from converged Ritz vectors: for subdomain i (one workgroup) with
// t_i = min(m_i + 1, m_cap, K) columns, write column j / ||column j|| at frame
// positions pos[row] of tgt[i][j][.], set mask[i][pos] = 1 and cnt[i] = t_i.
__global__ void k_warm_targets(const int* __restrict__ sel, const i32* __restrict__ nb,
                               const i64* __restrict__ voff, const i64* __restrict__ kvoff, int K,
                               const double* __restrict__ X, const int* __restrict__ mcount,
                               int m_cap, int n_pos, const i32* __restrict__ pos,
                               float* __restrict__ tgt, float* __restrict__ mask,
                               int* __restrict__ cnt) {
  const int i = sel[blockIdx.x];
  const int n = nb[i];
  const int t = min(min(mcount[i] + 1, m_cap), K);
  const double* Xi = X + kvoff[i];
  const i32* pi = pos + voff[i];
  __shared__ double red[16];
  for (int r = threadIdx.x; r < n; r += blockDim.x)
    if (pi[r] >= 0) mask[(i64)i * n_pos + pi[r]] = 1.f;
  for (int j = 0; j < t; ++j) {
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      const double v = pi[r] >= 0 ? Xi[r + (i64)j * n] : 0.0;
      s += v * v;
    }
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    float* tj = tgt + ((i64)i * m_cap + j) * n_pos;
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      if (pi[r] >= 0) tj[pi[r]] = (float)(Xi[r + (i64)j * n] * inv);
  }
  if (threadIdx.x == 0) cnt[i] = t;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int grid_1d(i64 n, int bs = 256, int cap = 16384) {
  i64 g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

int launch_sgemm(hipStream_t s, int ta, int tb, int M, int N, int K, int splits, const float* A,
                 int lda, const float* B, int ldb, float* C) {
  // k chunks are multiples of 16; the count actually launched (<= splits) is returned
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + 15) / 16 * 16;
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_sgemm<0, 0>), grid, dim3(256), 0, s, M, N, K, kchunk, A, lda, B, ldb, C);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_sgemm<1, 0>), grid, dim3(256), 0, s, M, N, K, kchunk, A, lda, B, ldb, C);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_sgemm<0, 1>), grid, dim3(256), 0, s, M, N, K, kchunk, A, lda, B, ldb, C);
  else
    hipLaunchKernelGGL((k_sgemm<1, 1>), grid, dim3(256), 0, s, M, N, K, kchunk, A, lda, B, ldb, C);
  return splits;
}

int sgemm_splits(int K, int splits) {
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + 15) / 16 * 16;
  return (K + kchunk - 1) / kchunk;
}

void launch_splitk_epi(hipStream_t s, int M, int N, int splits, const float* part, const float* bias,
                       const float* h, int mode, float* out) {
  hipLaunchKernelGGL(k_splitk_epi, dim3(grid_1d((i64)M * N)), dim3(256), 0, s, M, N, splits, part,
                     bias, h, mode, out);
}

void launch_colsum(hipStream_t s, int M, int N, const float* D, float* g) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, M, N, D, g);
}

void launch_gather_rows(hipStream_t s, int B, int w, const int* idx, const float* src, float* dst) {
  hipLaunchKernelGGL(k_gather_rows, dim3(grid_1d((i64)B * w)), dim3(256), 0, s, B, w, idx, src, dst);
}

void launch_proj_loss(hipStream_t s, int B, int V, int n_pos, int m_cap, const int* idx,
                      const float* y, const float* tgt, const float* mask, const int* cnt,
                      double ridge, float* dy, float* loss_b) {
  hipLaunchKernelGGL(k_proj_loss, dim3(B), dim3(256), 0, s, B, V, n_pos, m_cap, idx, y, tgt, mask,
                     cnt, ridge, dy, loss_b);
}

void launch_adam(hipStream_t s, i64 n, float* p, const float* g, float* m, float* v, float lr,
                 int step) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_1d(n)), dim3(256), 0, s, n, p, g, m, v, lr, b1, b2, 1e-8f,
                     c1, c2);
}

void launch_init_uniform(hipStream_t s, i64 lo, i64 hi, float a, unsigned long long seed, float* w) {
  hipLaunchKernelGGL(k_init_uniform, dim3(grid_1d(hi - lo)), dim3(256), 0, s, lo, hi, a, seed, w);
}

void launch_to_bf16(hipStream_t s, int rows, int cols, int ldd, const float* src, int lds,
                    unsigned short* dst) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_1d((i64)rows * ldd)), dim3(256), 0, s, rows, cols, ldd, src,
                     lds, dst);
}

void launch_to_bf16_t(hipStream_t s, int rows, int cols, int ldd, const float* src, int lds,
                      unsigned short* dst) {
  hipLaunchKernelGGL(k_to_bf16_t, dim3(grid_1d((i64)cols * ldd)), dim3(256), 0, s, rows, cols, ldd,
                     src, lds, dst);
}

void launch_hgemm(hipStream_t s, int M, int N, int Kp, const unsigned short* A, const unsigned short* Bt,
                  const float* bias, int relu, int out_bf16, void* C, int ldc) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(k_hgemm, grid, dim3(256), 0, s, M, N, Kp, A, Bt, bias, relu, out_bf16, C, ldc);
}

void launch_eig_init_warm(hipStream_t s, i64 total_rows, const i32* row_sub, const i64* voff,
                          const i32* nb, const i64* kvoff, int K, const double* dv, double* X,
                          unsigned long long seed, const i32* seed_id, const int* warm,
                          const float* yw, int n_vec, int n_pos, const i32* pos) {
  hipLaunchKernelGGL(k_eig_init_warm, dim3((unsigned)((total_rows + 255) / 256)), dim3(256), 0, s,
                     total_rows, row_sub, voff, nb, kvoff, K, dv, X, seed, seed_id, warm, yw, n_vec,
                     n_pos, pos);
}

void launch_warm_targets(hipStream_t s, int nsel, const int* sel, const i32* nb, const i64* voff,
                         const i64* kvoff, int K, const double* X, const int* mcount, int m_cap,
                         int n_pos, const i32* pos, float* tgt, float* mask, int* cnt) {
  if (nsel <= 0) return;
  hipLaunchKernelGGL(k_warm_targets, dim3(nsel), dim3(256), 0, s, sel, nb, voff, kvoff, K, X, mcount,
                     m_cap, n_pos, pos, tgt, mask, cnt);
}
