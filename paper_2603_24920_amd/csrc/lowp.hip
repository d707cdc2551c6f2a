// Low-precision copies of the data for the verification forms that read fewer bytes
// per candidate: bf16 (round to nearest even) and fp8 e4m3 with a per-row power-of-two
// scale. Rows are padded with zeros to `dpad` (a multiple of 16) so every candidate
// row is read with 16-byte loads. The float32 data stays the reference for re-ranking.
#include "internal.h"

namespace pdet {
namespace {

__device__ inline uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

// One row by one wave: the bf16 copy and / or the fp8 copy with its power-of-two scale.
__device__ inline void lowp_row(const float* X, int64_t row, int d, int dpad, int lane,
                                uint16_t* xbf, uint8_t* xf8, float* xscale) {
  const float* xr = X + row * d;
  if (xbf) {
    for (int t = lane; t < dpad; t += 64) xbf[row * dpad + t] = (t < d) ? to_bf16(xr[t]) : 0;
  }
  if (xf8) {
    float mx = 0.0f;
    for (int t = lane; t < d; t += 64) mx = fmaxf(mx, fabsf(xr[t]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    // scale 2^e with max|x| / 2^e <= 224, inside the e4m3 range of either encoding
    int e = 0;
    if (mx > 0.0f) e = (int)ceilf(log2f(mx / 224.0f));
    const float sc = ldexpf(1.0f, e), inv = ldexpf(1.0f, -e);
    if (lane == 0) xscale[row] = sc;
    for (int t = lane * 4; t < dpad; t += 256) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (t + u < d) ? xr[t + u] * inv : 0.0f;
      int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
      w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
      *reinterpret_cast<int*>(xf8 + row * dpad + t) = w;
    }
  }
}

// One wave per row; the grid strides over the rows (a dispatch holds fewer than 2^32
// work-items, so a wave per row of a 100M-row set cannot be one launch).
constexpr int64_t LOWP_MAX_BLOCKS = int64_t(1) << 20;

__global__ __launch_bounds__(256) void lowp_rows(const float* X, int64_t n, int d, int dpad,
                                                 uint16_t* xbf, uint8_t* xf8, float* xscale) {
  const int lane = threadIdx.x & 63;
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n;
       row += (int64_t)gridDim.x * 4)
    lowp_row(X, row, d, dpad, lane, xbf, xf8, xscale);
}

}  // namespace

void build_lowp_copies(Index& ix, hipStream_t s) {
  const bool bf = ix.lowp & (1u << PDET_BF16);
  const bool f8 = ix.lowp & (1u << PDET_FP8_E4M3);
  if (!bf && !f8) return;
  if (bf) ix.xbf16.alloc((size_t)ix.n * ix.dpad * 2);
  if (f8) {
    ix.xfp8.alloc((size_t)ix.n * ix.dpad);
    ix.xscale.alloc((size_t)ix.n * 4);
  }
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(ix.n, 4), LOWP_MAX_BLOCKS);
  hipLaunchKernelGGL(lowp_rows, dim3(grid), dim3(256), 0, s, ix.X, ix.n, ix.d, ix.dpad,
                     bf ? ix.xbf16.as<uint16_t>() : nullptr, f8 ? ix.xfp8.as<uint8_t>() : nullptr,
                     f8 ? ix.xscale.as<float>() : nullptr);
  PDET_HIP(hipGetLastError());
}

void extend_lowp_copies(Index& ix, int64_t n_old, std::vector<DevBuf>& keep, hipStream_t s) {
  const bool bf = ix.lowp & (1u << PDET_BF16);
  const bool f8 = ix.lowp & (1u << PDET_FP8_E4M3);
  const int64_t m = ix.n - n_old;
  if ((!bf && !f8) || m <= 0) return;
  auto grow = [&](DevBuf& b, size_t row_bytes) {
    DevBuf nb((size_t)ix.n * row_bytes);
    PDET_HIP(hipMemcpyAsync(nb.p, b.p, (size_t)n_old * row_bytes, hipMemcpyDeviceToDevice, s));
    keep.push_back(std::move(b));
    b = std::move(nb);
  };
  if (bf) grow(ix.xbf16, (size_t)ix.dpad * 2);
  if (f8) {
    grow(ix.xfp8, (size_t)ix.dpad);
    grow(ix.xscale, 4);
  }
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(m, 4), LOWP_MAX_BLOCKS);
  hipLaunchKernelGGL(lowp_rows, dim3(grid), dim3(256), 0, s, ix.X + n_old * ix.d, m, ix.d,
                     ix.dpad, bf ? ix.xbf16.as<uint16_t>() + n_old * ix.dpad : nullptr,
                     f8 ? ix.xfp8.as<uint8_t>() + n_old * ix.dpad : nullptr,
                     f8 ? ix.xscale.as<float>() + n_old : nullptr);
  PDET_HIP(hipGetLastError());
}

}  // namespace pdet
