// Small device helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdet {

// A value every lane of the wave holds (read from LDS after a barrier, say), moved to a
// scalar register so that arithmetic on it stays scalar.
__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int32_t uni(int32_t v) { return (int32_t)__builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t uni(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan over a whole wave (every lane active): scans of the 16-lane rows by
// row_shr:1,2,4,8 (a lane without a source adds 0), then the row totals carried on by
// row_bcast:15 (into rows 1 and 3) and row_bcast:31 (into rows 2 and 3).
__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}

// Exclusive scan of one uint32 per thread over a workgroup of NT threads (NT a multiple of
// 64; every thread calls it, with all lanes of its wave active). sh must hold NT/64 + 1
// words. Wave scans by DPP, the wave totals through LDS, each wave adding those before it;
// two barriers.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  static_assert(NT % 64 == 0, "whole waves");
  const int wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if ((threadIdx.x & 63) == 63) sh[wave] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t t = sh[w];
    before += (w < wave) ? t : 0u;
    tot += t;
  }
  *total = uni(tot);
  __syncthreads();   // sh is free for the next scan
  return uni(before) + incl - v;
}

// A double moved across lanes with a DPP control (both 32-bit halves; every lane of the
// row must be active).
template <int CTRL>
__device__ inline double dpp_double(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum of x over each aligned group of `width` lanes (a power of two <= 64); lane 0 of a
// group holds the exact group sum of its order, other lanes a sum in another order.
// Within a 16-lane row the steps are DPP moves (quad swaps, half-row mirror, row mirror);
// across rows they are lane shuffles.
__device__ inline double group_sum(double x, int width) {
  if (width > 1) x += dpp_double<0xB1>(x);    // quad_perm [1,0,3,2]
  if (width > 2) x += dpp_double<0x4E>(x);    // quad_perm [2,3,0,1]
  if (width > 4) x += dpp_double<0x141>(x);   // row_half_mirror
  if (width > 8) x += dpp_double<0x140>(x);   // row_mirror
  if (width > 16) x += __shfl_xor(x, 16);
  if (width > 32) x += __shfl_xor(x, 32);
  return x;
}

// The same sum for a width fixed at compile time (no per-level tests).
template <int W>
__device__ inline double group_sum(double x) {
  if constexpr (W > 1) x += dpp_double<0xB1>(x);
  if constexpr (W > 2) x += dpp_double<0x4E>(x);
  if constexpr (W > 4) x += dpp_double<0x141>(x);
  if constexpr (W > 8) x += dpp_double<0x140>(x);
  if constexpr (W > 16) x += __shfl_xor(x, 16);
  if constexpr (W > 32) x += __shfl_xor(x, 32);
  return x;
}

// Set bits of `mask` in the lanes below the calling one (v_mbcnt: no per-lane 64-bit
// mask to keep in registers).
__device__ inline uint32_t lanes_below_mask(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace pdet
