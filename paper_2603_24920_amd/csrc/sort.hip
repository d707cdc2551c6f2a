// Breakpoint selection (encoding phase, dynamic breakpoints) and device scans.
//
// The paper selects the Nr-1 interior order statistics of each sampled column with
// rounds of QuickSelect. On the GPU every column is sorted instead (a bitonic
// network: tiles sorted in LDS, cross-tile merge steps in global memory), then the
// breakpoint ranks are read off: B(z) = C-up(m*(z-1)), m = floor(ns/Nr). Sorting gives
// the same order statistics as selection.
#include "internal.h"

namespace pdet {
namespace {

constexpr int TILE = 4096;         // keys per LDS tile (16 KB)
constexpr int SORT_THREADS = 512;

__device__ inline void cas(float& a, float& b, bool asc) {
  if ((a > b) == asc) { float t = a; a = b; b = t; }
}

// Stages k = 2..tile of the network on one tile; directions from the global index.
__global__ __launch_bounds__(SORT_THREADS) void bitonic_tile_sort(float* keys, int64_t npad,
                                                                  int tile) {
  __shared__ float sk[TILE];
  const int64_t tiles_per_col = npad / tile;
  const int64_t col = blockIdx.x / tiles_per_col;
  const int64_t base = col * npad + (blockIdx.x % tiles_per_col) * tile;
  const int64_t gbase = (blockIdx.x % tiles_per_col) * tile;    // index inside the column
  for (int e = threadIdx.x; e < tile; e += blockDim.x) sk[e] = keys[base + e];
  __syncthreads();
  for (int k = 2; k <= tile; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < tile / 2; t += blockDim.x) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const bool asc = (((gbase + i) & k) == 0);
        cas(sk[i], sk[i | j], asc);
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < tile; e += blockDim.x) keys[base + e] = sk[e];
}

// Full tiles (TILE keys) run the same network with each of TILE_T threads holding KPT
// consecutive keys: steps with stride j < KPT stay in registers, strides up to a wave's
// 64*KPT keys go through lane shuffles, and only the larger ones through LDS (laid out
// key-major so that consecutive threads hit consecutive banks).
constexpr int KPT = 16;
constexpr int TILE_T = TILE / KPT;   // 256 threads

__device__ inline void tile_step(float (&x)[KPT], int t, int64_t gidx0, int64_t k, int j,
                                 float* sk) {
  if (j < KPT) {
#pragma unroll
    for (int e = 0; e < KPT; ++e)
      if (!(e & j)) cas(x[e], x[e | j], ((gidx0 + e) & k) == 0);
  } else if (j < 64 * KPT) {
    const int m = j / KPT;                       // partner lane: t ^ m, same wave
    const bool lower = (t & m) == 0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
      const float y = __shfl_xor(x[e], m);
      const bool asc = ((gidx0 + e) & k) == 0;
      x[e] = (lower == asc) ? fminf(x[e], y) : fmaxf(x[e], y);
    }
  } else {
#pragma unroll
    for (int e = 0; e < KPT; ++e) sk[e * TILE_T + t] = x[e];
    __syncthreads();
    const int tp = t ^ (j / KPT);
    const bool lower = (t & (j / KPT)) == 0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
      const float y = sk[e * TILE_T + tp];
      const bool asc = ((gidx0 + e) & k) == 0;
      x[e] = (lower == asc) ? fminf(x[e], y) : fmaxf(x[e], y);
    }
    __syncthreads();
  }
}

// MERGE false: stages k = 2..TILE of each tile; true: steps j = TILE/2..1 of stage `kst`.
template <bool MERGE>
__global__ __launch_bounds__(TILE_T) void bitonic_tile_reg(float* keys, int64_t npad,
                                                           int64_t kst) {
  __shared__ float sk[TILE];
  const int64_t tiles_per_col = npad / TILE;
  const int64_t col = blockIdx.x / tiles_per_col;
  const int64_t gbase = (blockIdx.x % tiles_per_col) * TILE;
  const int t = threadIdx.x;
  float4* src = reinterpret_cast<float4*>(keys + col * npad + gbase + (int64_t)t * KPT);
  float x[KPT];
#pragma unroll
  for (int q = 0; q < KPT / 4; ++q) {
    const float4 v = src[q];
    x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
  }
  const int64_t gidx0 = gbase + (int64_t)t * KPT;   // index inside the column of x[0]
  if constexpr (MERGE) {
    for (int j = TILE >> 1; j > 0; j >>= 1) tile_step(x, t, gidx0, kst, j, sk);
  } else {
    for (int k = 2; k <= TILE; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) tile_step(x, t, gidx0, k, j, sk);
  }
#pragma unroll
  for (int q = 0; q < KPT / 4; ++q)
    src[q] = make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
}

// S consecutive steps j = J, J/2, .., J/2^(S-1) (all >= tile) of stage k in one pass: a
// thread holds the 2^S keys whose indices differ only in those S bits, applies the S
// compare-exchange levels in registers (largest stride first, as the network does), and
// writes them back. All of a group's keys share bit k, hence one direction.
template <int S>
__global__ void bitonic_global_steps(float* keys, int64_t npad, int64_t k, int p0,
                                     int64_t groups_total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= groups_total) return;
  const int64_t per_col = npad >> S;
  const int64_t col = g / per_col, t = g % per_col;
  const int64_t base = ((t >> p0) << (p0 + S)) | (t & ((int64_t(1) << p0) - 1));
  float* c = keys + col * npad;
  constexpr int G = 1 << S;
  float x[G];
#pragma unroll
  for (int a = 0; a < G; ++a) x[a] = c[base + ((int64_t)a << p0)];
  const bool asc = ((base & k) == 0);
#pragma unroll
  for (int l = S - 1; l >= 0; --l) {
#pragma unroll
    for (int a = 0; a < G; ++a)
      if (!(a & (1 << l))) cas(x[a], x[a | (1 << l)], asc);
  }
#pragma unroll
  for (int a = 0; a < G; ++a) c[base + ((int64_t)a << p0)] = x[a];
}

// Steps j = tile/2 .. 1 of stage k > tile inside each tile.
__global__ __launch_bounds__(SORT_THREADS) void bitonic_tile_merge(float* keys, int64_t npad,
                                                                   int tile, int64_t k) {
  __shared__ float sk[TILE];
  const int64_t tiles_per_col = npad / tile;
  const int64_t col = blockIdx.x / tiles_per_col;
  const int64_t gbase = (blockIdx.x % tiles_per_col) * tile;
  const int64_t base = col * npad + gbase;
  const bool asc = ((gbase & k) == 0);
  for (int e = threadIdx.x; e < tile; e += blockDim.x) sk[e] = keys[base + e];
  __syncthreads();
  for (int j = tile >> 1; j > 0; j >>= 1) {
    for (int t = threadIdx.x; t < tile / 2; t += blockDim.x) {
      const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
      cas(sk[i], sk[i | j], asc);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < tile; e += blockDim.x) keys[base + e] = sk[e];
}

__global__ void fill_kernel(float* p, int64_t count, float v) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < count) p[g] = v;
}

// B[col][u] = sorted[col][m*u - 1] for u = 1..Nr-1 (1-based rank m*u).
__global__ void pick_kernel(const float* sorted, int ncols, int64_t npad, int64_t m, int Nr,
                            float* B) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncols * (Nr - 1)) return;
  const int col = g / (Nr - 1), u = 1 + g % (Nr - 1);
  B[(int64_t)col * (Nr + 1) + u] = sorted[(int64_t)col * npad + m * u - 1];
}

__global__ void outer_kernel(float* B, const uint32_t* colmm, int ncols, int Nr) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  B[(int64_t)col * (Nr + 1)] = ordered_to_float(colmm[col]);
  B[(int64_t)col * (Nr + 1) + Nr] = ordered_to_float(colmm[ncols + col]);
}

// ---- exclusive scan of uint32 rows: block sums, scan of sums, local scan + offset
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_ITEMS;

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: [SCAN_THREADS/64 + 1]
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
    for (int w = 0; w < SCAN_THREADS / 64; ++w) { const uint32_t t = sh[w]; sh[w] = acc; acc += t; }
    sh[SCAN_THREADS / 64] = acc;
  }
  __syncthreads();
  const uint32_t r = sh[wave] + x - v;
  *total = sh[SCAN_THREADS / 64];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_sums(const uint32_t* in, int64_t len,
                                                          int64_t nblk, uint32_t* sums) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  const int64_t row = blockIdx.x / nblk, b = blockIdx.x % nblk;
  const uint32_t* r = in + row * len;
  uint32_t s = 0;
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    const int64_t i = b * SCAN_BLOCK + it * SCAN_THREADS + threadIdx.x;
    if (i < len) s += r[i];
  }
  uint32_t tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) sums[row * nblk + b] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_of_sums(uint32_t* sums, int64_t nblk,
                                                             uint32_t* totals) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  uint32_t* r = sums + (int64_t)blockIdx.x * nblk;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblk; b0 += SCAN_THREADS) {
    const int64_t i = b0 + threadIdx.x;
    const uint32_t v = i < nblk ? r[i] : 0;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, sh, &tot);
    if (i < nblk) r[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && totals) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_apply(const uint32_t* in, uint32_t* out,
                                                           int64_t len, int64_t nblk,
                                                           const uint32_t* sums) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  const int64_t row = blockIdx.x / nblk, b = blockIdx.x % nblk;
  const uint32_t* r = in + row * len;
  uint32_t* o = out + row * len;
  // each thread owns SCAN_ITEMS consecutive entries
  const int64_t i0 = b * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    v[it] = (i0 + it < len) ? r[i0 + it] : 0;
    s += v[it];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, sh, &tot) + sums[row * nblk + b];
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    if (i0 + it < len) o[i0 + it] = run;
    run += v[it];
  }
}

}  // namespace

void sort_columns(float* keys, int ncols, int64_t npad, hipStream_t s) {
  const int tile = (int)std::min<int64_t>(npad, TILE);
  const int64_t tiles = ncols * (npad / tile);
  const bool full = tile == TILE;   // register / shuffle form for full tiles
  if (full)
    hipLaunchKernelGGL(bitonic_tile_reg<false>, dim3((unsigned)tiles), dim3(TILE_T), 0, s, keys,
                       npad, (int64_t)0);
  else
    hipLaunchKernelGGL(bitonic_tile_sort, dim3((unsigned)tiles), dim3(SORT_THREADS), 0, s, keys,
                       npad, tile);
  PDET_HIP(hipGetLastError());
  for (int64_t k = 2 * (int64_t)tile; k <= npad; k <<= 1) {
    // the steps j = k/2 .. tile, up to four per pass
    int hi = 0;
    while ((int64_t(1) << (hi + 1)) <= (k >> 1)) ++hi;   // log2(k/2)
    int lo = 0;
    while ((int64_t(1) << (lo + 1)) <= tile) ++lo;        // log2(tile)
    while (hi >= lo) {
      const int S = std::min(4, hi - lo + 1);
      const int p0 = hi - S + 1;
      const int64_t groups = (int64_t)ncols * (npad >> S);
      const dim3 gr(cdiv(groups, 256));
      switch (S) {
        case 1: hipLaunchKernelGGL(bitonic_global_steps<1>, gr, dim3(256), 0, s, keys, npad, k, p0, groups); break;
        case 2: hipLaunchKernelGGL(bitonic_global_steps<2>, gr, dim3(256), 0, s, keys, npad, k, p0, groups); break;
        case 3: hipLaunchKernelGGL(bitonic_global_steps<3>, gr, dim3(256), 0, s, keys, npad, k, p0, groups); break;
        default: hipLaunchKernelGGL(bitonic_global_steps<4>, gr, dim3(256), 0, s, keys, npad, k, p0, groups); break;
      }
      PDET_HIP(hipGetLastError());
      hi -= S;
    }
    if (full)
      hipLaunchKernelGGL(bitonic_tile_reg<true>, dim3((unsigned)tiles), dim3(TILE_T), 0, s, keys,
                         npad, k);
    else
      hipLaunchKernelGGL(bitonic_tile_merge, dim3((unsigned)tiles), dim3(SORT_THREADS), 0, s,
                         keys, npad, tile, k);
    PDET_HIP(hipGetLastError());
  }
}

void fill_f32(float* p, int64_t count, float v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv(count, 256)), dim3(256), 0, s, p, count, v);
  PDET_HIP(hipGetLastError());
}

void pick_breakpoints(const float* sorted, int ncols, int64_t npad, int64_t ns, int Nr, float* B,
                      hipStream_t s) {
  const int64_t m = ns / Nr;
  const int tot = ncols * (Nr - 1);
  hipLaunchKernelGGL(pick_kernel, dim3(cdiv(tot, 256)), dim3(256), 0, s, sorted, ncols, npad, m,
                     Nr, B);
  PDET_HIP(hipGetLastError());
}

void set_outer_breakpoints(float* B, const uint32_t* colmm, int ncols, int Nr, hipStream_t s) {
  hipLaunchKernelGGL(outer_kernel, dim3(cdiv(ncols, 64)), dim3(64), 0, s, B, colmm, ncols, Nr);
  PDET_HIP(hipGetLastError());
}

void scan_rows(const uint32_t* in, uint32_t* out, uint32_t* totals, int rows, int64_t len,
               DevBuf& tmp, hipStream_t s) {
  const int64_t nblk = (len + SCAN_BLOCK - 1) / SCAN_BLOCK;
  const size_t need = (size_t)rows * nblk * sizeof(uint32_t);
  if (tmp.bytes < need) tmp.alloc(need);
  uint32_t* sums = tmp.as<uint32_t>();
  hipLaunchKernelGGL(scan_sums, dim3((unsigned)(rows * nblk)), dim3(SCAN_THREADS), 0, s, in, len,
                     nblk, sums);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_of_sums, dim3(rows), dim3(SCAN_THREADS), 0, s, sums, nblk, totals);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)(rows * nblk)), dim3(SCAN_THREADS), 0, s, in, out,
                     len, nblk, sums);
  PDET_HIP(hipGetLastError());
}

}  // namespace pdet
