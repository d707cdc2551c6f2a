// Small device helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdet {

// Exclusive scan of one uint32 per thread over a workgroup of NT threads.
// sh must hold NT/64 + 1 words. Contains barriers: call from every thread.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < NT / 64; ++w) {
      const uint32_t t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[NT / 64] = acc;
  }
  __syncthreads();
  const uint32_t r = sh[wave] + x - v;
  *total = sh[NT / 64];
  __syncthreads();
  return r;
}

__device__ inline uint32_t lanes_below_mask(uint64_t mask) {
  const int lane = threadIdx.x & 63;
  return (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

}  // namespace pdet
