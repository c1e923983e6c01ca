// Shared declarations of the msdd HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

typedef int64_t i64;
typedef int32_t i32;

#define MSDD_WG 256

// Status words written by kernels (per subdomain unless noted).
enum : int {
  ST_RUNNING = 0,
  ST_DONE = 1,
  ST_GROW = 2,      // eigensolver needs a larger block
  ST_NOTSPD = 3,    // non-positive pivot
  ST_BADINPUT = 4,  // entry outside the planned band, NaN, ...
  ST_NOCONV = 5,    // eigensolver iteration limit
};

// Workgroup barrier that orders LDS accesses only: the fences are limited to the local
// address space, so global loads still in flight (prefetches held in registers) are
// not waited for.  For use where threads communicate through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum over a workgroup of blockDim.x threads (blockDim.x a multiple of 64, <= 1024).
template <typename T>
__device__ inline T block_sum(T v, T* sh /* >= 16 entries */) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
