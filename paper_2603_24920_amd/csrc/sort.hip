// Breakpoint selection (encoding phase, dynamic breakpoints) and device scans.
//
// The paper selects the Nr-1 interior order statistics of each sampled column with rounds
// of QuickSelect. Here each column's order statistics B(z) = C-up(m*(z-1)), m = floor(ns/Nr)
// (1-based ranks) are selected without sorting the column:
//  1. the column's sample min and max (reduced by the sample projection);
//  2. a histogram of NB equal-width value buckets between them (bucket index is a
//     monotone function of the value, so bucket order is value order);
//  3. per target rank, its bucket and its rank inside the bucket (a scan of the histogram);
//  4. the keys of the buckets that hold a target are gathered, bucket by bucket;
//  5. per target, an exact radix select (four 8-bit passes over the order-preserving
//     integer image of the floats) inside its bucket.
// The result is the exact order statistic whatever the distribution (a bucket may hold
// any number of keys; large ones only take longer).
#include "internal.h"
#include "devutil.h"

namespace pdet {
namespace {

constexpr int NB = 4096;            // value buckets per column
constexpr int SEL_THREADS = 256;
constexpr int GATHER_KEYS = 4096;   // keys per gather block
constexpr int HIST_KEYS_MAX = 32768;   // keys per histogram block at most: several per
                                       // bucket before the block adds its counts to the
                                       // column's (one atomic per bucket it saw), while a
                                       // column still spans at least 64 blocks

__device__ inline int bucket_of(float v, float lo, float scale) {
  const int b = (int)__fmul_rn(__fsub_rn(v, lo), scale);   // no contraction: one rounding each
  return b < 0 ? 0 : (b >= NB ? NB - 1 : b);
}

__device__ inline void col_range(const uint32_t* mm, int ncols, int col, float& lo, float& scale) {
  lo = ordered_to_float(mm[col]);
  const float hi = ordered_to_float(mm[ncols + col]);
  scale = (hi > lo) ? (float)NB / (hi - lo) : 0.0f;
}

// Bucket histogram of every column, counted in LDS per block.
__global__ __launch_bounds__(256) void col_hist(const float* keys, int64_t ld, int64_t ns,
                                                int ncols, const uint32_t* mm, int kpb,
                                                uint32_t* hist) {
  __shared__ uint32_t h[NB];
  const int col = blockIdx.y;
  for (int i = threadIdx.x; i < NB; i += 256) h[i] = 0;
  __syncthreads();
  float lo, scale;
  col_range(mm, ncols, col, lo, scale);
  const float* c = keys + (int64_t)col * ld;
  const int64_t k0 = (int64_t)blockIdx.x * kpb;
  for (int u = threadIdx.x; u < kpb; u += 256) {
    const int64_t i = k0 + u;
    if (i < ns) atomicAdd(&h[bucket_of(c[i], lo, scale)], 1u);
  }
  __syncthreads();
  uint32_t* g = hist + (int64_t)col * NB;
  for (int i = threadIdx.x; i < NB; i += 256)
    if (h[i]) atomicAdd(&g[i], h[i]);
}

// Per column (one block): the bucket and in-bucket rank of every target rank m*u, and the
// gather offset of every bucket that holds a target (-1 for the others).
__global__ __launch_bounds__(1024) void col_targets(const uint32_t* hist, int Nr, int64_t m,
                                                    int32_t* tbucket, uint32_t* trank,
                                                    int32_t* boff, uint32_t* needbits) {
  __shared__ uint32_t cum[NB];      // inclusive prefix of the histogram
  __shared__ uint32_t need[NB];
  __shared__ uint32_t wsum[1024 / 64 + 1];
  const int col = blockIdx.x;
  const uint32_t* h = hist + (int64_t)col * NB;
  constexpr int PER = NB / 1024;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // inclusive scan of the histogram (each thread PER consecutive buckets)
  auto scan = [&](const uint32_t* in_lds_or_null, const uint32_t* in_glob, uint32_t* out) {
    uint32_t v[PER], s = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      v[e] = in_lds_or_null ? in_lds_or_null[threadIdx.x * PER + e] : in_glob[threadIdx.x * PER + e];
      s += v[e];
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      for (int w = 0; w < 1024 / 64; ++w) { const uint32_t t = wsum[w]; wsum[w] = acc; acc += t; }
    }
    __syncthreads();
    uint32_t run = wsum[wave] + x - s;
#pragma unroll
    for (int e = 0; e < PER; ++e) { run += v[e]; out[threadIdx.x * PER + e] = run; }
    __syncthreads();
  };
  scan(nullptr, h, cum);
  for (int i = threadIdx.x; i < NB; i += 1024) need[i] = 0;
  __syncthreads();
  for (int u = 1 + threadIdx.x; u < Nr; u += 1024) {
    const uint32_t r = (uint32_t)(m * u);      // 1-based rank, r <= ns
    int lo = 0, hi = NB - 1;                    // first bucket with cum >= r
    while (lo < hi) {
      const int md = (lo + hi) >> 1;
      if (cum[md] >= r) hi = md; else lo = md + 1;
    }
    const uint32_t before = lo ? cum[lo - 1] : 0u;
    tbucket[(int64_t)col * (Nr - 1) + u - 1] = lo;
    trank[(int64_t)col * (Nr - 1) + u - 1] = r - before;
    need[lo] = 1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += 1024) need[i] = need[i] ? (cum[i] - (i ? cum[i - 1] : 0u)) : 0u;
  __syncthreads();
  scan(need, nullptr, cum);                     // inclusive: end offset of each needed bucket
  int32_t* bo = boff + (int64_t)col * NB;
  for (int i = threadIdx.x; i < NB; i += 1024)
    bo[i] = need[i] ? (int32_t)(cum[i] - need[i]) : -1;
  // the same choice as a bit mask (bit b of word b / 32: bucket b is gathered)
  if (threadIdx.x < NB / 32) {
    uint32_t w = 0;
    for (int j = 0; j < 32; ++j) w |= (need[threadIdx.x * 32 + j] ? 1u : 0u) << j;
    needbits[(int64_t)col * (NB / 32) + threadIdx.x] = w;
  }
}

// Keys of the needed buckets, gathered per column bucket by bucket (order inside a bucket
// unspecified) as order-preserving uints: a block counts its keys per bucket in LDS, takes
// one global reservation per bucket, then writes. Whether a key's bucket is needed comes
// from the column's bit mask, held in LDS.
__global__ __launch_bounds__(256) void col_gather(const float* keys, int64_t ld, int64_t ns,
                                                  int ncols, const uint32_t* mm,
                                                  const int32_t* boff, const uint32_t* needbits,
                                                  uint32_t* fill, uint32_t* gbuf) {
  __shared__ uint32_t cntl[NB];
  __shared__ uint32_t basel[NB];
  __shared__ uint32_t needl[NB / 32];
  constexpr int PER = GATHER_KEYS / 256;
  const int col = blockIdx.y;
  for (int i = threadIdx.x; i < NB; i += 256) cntl[i] = 0;
  if (threadIdx.x < NB / 32) needl[threadIdx.x] = needbits[(int64_t)col * (NB / 32) + threadIdx.x];
  __syncthreads();
  float lo, scale;
  col_range(mm, ncols, col, lo, scale);
  const float* c = keys + (int64_t)col * ld;
  const int32_t* bo = boff + (int64_t)col * NB;
  const int64_t k0 = (int64_t)blockIdx.x * GATHER_KEYS;
  int bk[PER];
  uint32_t rk[PER];
  float kv[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int64_t i = k0 + e * 256 + threadIdx.x;
    bk[e] = -1;
    if (i < ns) {
      kv[e] = c[i];
      const int b = bucket_of(kv[e], lo, scale);
      if ((needl[b >> 5] >> (b & 31)) & 1u) {
        bk[e] = b;
        rk[e] = atomicAdd(&cntl[b], 1u);
      }
    }
  }
  __syncthreads();
  uint32_t* fl = fill + (int64_t)col * NB;
  for (int i = threadIdx.x; i < NB; i += 256)
    if (cntl[i]) basel[i] = (uint32_t)bo[i] + atomicAdd(&fl[i], cntl[i]);
  __syncthreads();
  uint32_t* g = gbuf + (int64_t)col * ns;
#pragma unroll
  for (int e = 0; e < PER; ++e)
    if (bk[e] >= 0) g[basel[bk[e]] + rk[e]] = float_to_ordered(kv[e]);
}

// B[col][u] = the trank-th smallest key of target u's bucket: radix select, 8 bits a pass.
__global__ __launch_bounds__(SEL_THREADS) void col_select(const uint32_t* hist,
                                                          const int32_t* tbucket,
                                                          const uint32_t* trank,
                                                          const int32_t* boff,
                                                          const uint32_t* gbuf, int64_t ns,
                                                          int Nr, float* B) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t wsum[SEL_THREADS / 64 + 1];
  __shared__ uint32_t s_pick, s_rem;
  const int u = blockIdx.x + 1, col = blockIdx.y;
  const int b = tbucket[(int64_t)col * (Nr - 1) + u - 1];
  uint32_t r = trank[(int64_t)col * (Nr - 1) + u - 1];
  const uint32_t size = hist[(int64_t)col * NB + b];
  const uint32_t* keys = gbuf + (int64_t)col * ns + boff[(int64_t)col * NB + b];
  uint32_t prefix = 0;
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = 24 - 8 * pass;
    h[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < size; i += SEL_THREADS) {
      const uint32_t k = keys[i];
      if (pass == 0 || (k >> (sh + 8)) == prefix) atomicAdd(&h[(k >> sh) & 255u], 1u);
    }
    __syncthreads();
    // the bin where the remaining rank falls (inclusive prefix over bins)
    const uint32_t v = h[threadIdx.x];
    uint32_t x = v;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      for (int w = 0; w < SEL_THREADS / 64; ++w) { const uint32_t t = wsum[w]; wsum[w] = acc; acc += t; }
    }
    __syncthreads();
    const uint32_t incl = wsum[wave] + x;
    if (incl - v < r && r <= incl) { s_pick = (uint32_t)threadIdx.x; s_rem = r - (incl - v); }
    __syncthreads();
    prefix = (prefix << 8) | s_pick;
    r = s_rem;
    __syncthreads();
  }
  if (threadIdx.x == 0) B[(int64_t)col * (Nr + 1) + u] = ordered_to_float(prefix);
}

__global__ void fill_kernel(float* p, int64_t count, float v) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < count) p[g] = v;
}

// range blockIdx.y of the list, grid-stride
__global__ void fill_words_kernel(FillList f) {
  const int r = blockIdx.y;
  uint32_t* p = f.p[r];
  const uint32_t v = f.value[r], nw = f.nwords[r];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- column moments of the sample (static encoding), in a fixed summation order
constexpr int MOM_THREADS = 256;

// part[col][b]: block b's sum over its share of column col of x (mean == nullptr) or of
// (x - mean[col])^2, in FP64.
__global__ __launch_bounds__(MOM_THREADS) void col_partial(const float* keys, int64_t ld,
                                                           int64_t ns, int nblk,
                                                           const double* mean, double* part) {
  __shared__ double sh[MOM_THREADS / 64];
  const int col = blockIdx.y, b = blockIdx.x;
  const float* c = keys + (int64_t)col * ld;
  const double mu = mean ? mean[col] : 0.0;
  double s = 0.0;
  for (int64_t i = (int64_t)b * MOM_THREADS + threadIdx.x; i < ns;
       i += (int64_t)nblk * MOM_THREADS) {
    const double x = (double)c[i] - mu;
    s += mean ? x * x : x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < MOM_THREADS / 64; ++w) t += sh[w];
    part[(int64_t)col * nblk + b] = t;
  }
}

// out[col] = (sum of part[col][0..nblk)) / ns, summed in block order.
__global__ void col_finish(const double* part, int nblk, int ncols, int64_t ns, double* out) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += part[(int64_t)col * nblk + b];
  out[col] = t / (double)ns;
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

// NZ: the scanned value of an entry is 1 if it is not zero, else 0
template <bool NZ>
__global__ __launch_bounds__(SCAN_THREADS) void scan_sums(const uint32_t* in, int64_t len,
                                                          int64_t nblk, uint32_t* sums) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  const int64_t row = blockIdx.x / nblk, b = blockIdx.x % nblk;
  const uint32_t* r = in + row * len;
  uint32_t s = 0;
  auto val = [](uint32_t x) { return NZ ? (x != 0u ? 1u : 0u) : x; };
  if ((len & 3) == 0 && (b + 1) * SCAN_BLOCK <= len) {
    // a whole block of a row of length divisible by 4: 16-byte loads, consecutive per lane
    const uint4* r4 = reinterpret_cast<const uint4*>(r + b * SCAN_BLOCK);
#pragma unroll
    for (int u = 0; u < SCAN_ITEMS / 4; ++u) {
      const uint4 w = r4[u * SCAN_THREADS + threadIdx.x];
      s += val(w.x) + val(w.y) + val(w.z) + val(w.w);
    }
  } else {
    for (int it = 0; it < SCAN_ITEMS; ++it) {
      const int64_t i = b * SCAN_BLOCK + it * SCAN_THREADS + threadIdx.x;
      if (i < len) s += val(r[i]);
    }
  }
  uint32_t tot;
  block_excl_scan<SCAN_THREADS>(s, sh, &tot);
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
    const uint32_t ex = block_excl_scan<SCAN_THREADS>(v, sh, &tot);
    if (i < nblk) r[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && totals) totals[blockIdx.x] = carry;
}

template <bool NZ>
__global__ __launch_bounds__(SCAN_THREADS) void scan_apply(const uint32_t* in, uint32_t* out,
                                                           int64_t len, int64_t nblk,
                                                           const uint32_t* sums) {
  __shared__ uint32_t sh[SCAN_THREADS / 64 + 1];
  const int64_t row = blockIdx.x / nblk, b = blockIdx.x % nblk;
  const uint32_t* r = in + row * len;
  uint32_t* o = out + row * len;
  // each thread owns SCAN_ITEMS consecutive entries, read and written as 16-byte vectors
  // when the row is (rows of a length divisible by 4 start 16-byte aligned)
  const int64_t i0 = b * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_ITEMS;
  const bool vec = (len & 3) == 0 && i0 + SCAN_ITEMS <= len;
  uint32_t v[SCAN_ITEMS];
  if (vec) {
#pragma unroll
    for (int u = 0; u < SCAN_ITEMS / 4; ++u) {
      const uint4 w = reinterpret_cast<const uint4*>(r + i0)[u];
      v[4 * u] = w.x; v[4 * u + 1] = w.y; v[4 * u + 2] = w.z; v[4 * u + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) v[it] = (i0 + it < len) ? r[i0 + it] : 0;
  }
  uint32_t s = 0;
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    if (NZ) v[it] = v[it] != 0u ? 1u : 0u;
    s += v[it];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan<SCAN_THREADS>(s, sh, &tot) + sums[row * nblk + b];
  uint32_t ov[SCAN_ITEMS];
#pragma unroll
  for (int it = 0; it < SCAN_ITEMS; ++it) {
    ov[it] = run;
    run += v[it];
  }
  if (vec) {
#pragma unroll
    for (int u = 0; u < SCAN_ITEMS / 4; ++u)
      reinterpret_cast<uint4*>(o + i0)[u] =
          make_uint4(ov[4 * u], ov[4 * u + 1], ov[4 * u + 2], ov[4 * u + 3]);
  } else {
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it)
      if (i0 + it < len) o[i0 + it] = ov[it];
  }
}

}  // namespace

void fill_words(const FillList& f, hipStream_t s) {
  if (f.n == 0) return;
  uint32_t most = 0;
  for (int r = 0; r < f.n; ++r) most = std::max(most, f.nwords[r]);
  const unsigned gx = (unsigned)std::min<int64_t>(std::max<int64_t>(cdiv(most, 256), 1), 1024);
  hipLaunchKernelGGL(fill_words_kernel, dim3(gx, f.n), dim3(256), 0, s, f);
  PDET_HIP(hipGetLastError());
}

void fill_f32(float* p, int64_t count, float v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv(count, 256)), dim3(256), 0, s, p, count, v);
  PDET_HIP(hipGetLastError());
}

void select_breakpoints(const float* keys, int ncols, int64_t ld, int64_t ns, int Nr, float* B,
                        const uint32_t* mm, std::vector<PooledBuf>& keep, hipStream_t s) {
  const int64_t m = ns / Nr;
  PooledBuf hist((size_t)ncols * NB * 4), fill((size_t)ncols * NB * 4);
  PooledBuf boff((size_t)ncols * NB * 4), tb((size_t)ncols * (Nr - 1) * 4);
  PooledBuf needbits((size_t)ncols * (NB / 32) * 4);
  PooledBuf tr((size_t)ncols * (Nr - 1) * 4), gbuf((size_t)ncols * ns * 4);
  FillList fz;
  fz.add(hist.ptr(), 0u, hist.bytes());
  fz.add(fill.ptr(), 0u, fill.bytes());
  fill_words(fz, s);
  const dim3 kg(cdiv(ns, GATHER_KEYS), ncols);
  const int kpb = (int)std::min<int64_t>(
      HIST_KEYS_MAX, std::max<int64_t>(GATHER_KEYS, (ns / 64 + GATHER_KEYS - 1) / GATHER_KEYS *
                                                         GATHER_KEYS));
  hipLaunchKernelGGL(col_hist, dim3(cdiv(ns, kpb), ncols), dim3(256), 0, s, keys, ld, ns, ncols,
                     mm, kpb, hist.as<uint32_t>());
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(col_targets, dim3(ncols), dim3(1024), 0, s, hist.as<uint32_t>(), Nr, m,
                     tb.as<int32_t>(), tr.as<uint32_t>(), boff.as<int32_t>(),
                     needbits.as<uint32_t>());
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(col_gather, kg, dim3(256), 0, s, keys, ld, ns, ncols, mm,
                     boff.as<int32_t>(), needbits.as<uint32_t>(), fill.as<uint32_t>(),
                     gbuf.as<uint32_t>());
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(col_select, dim3(Nr - 1, ncols), dim3(SEL_THREADS), 0, s,
                     hist.as<uint32_t>(), tb.as<int32_t>(), tr.as<uint32_t>(), boff.as<int32_t>(),
                     gbuf.as<uint32_t>(), ns, Nr, B);
  PDET_HIP(hipGetLastError());
  // the kernels above still use the temporaries: the caller keeps them until it synchronises
  for (PooledBuf* t : {&hist, &fill, &boff, &needbits, &tb, &tr, &gbuf})
    keep.push_back(std::move(*t));
}

double normal_quantile(double p) {
  // Phi(x) = erfc(-x / sqrt 2) / 2. The lower half is solved directly (the upper half by
  // symmetry, which keeps relative accuracy in both tails): bisection brackets the root,
  // then Newton steps with Phi'(x) = exp(-x^2 / 2) / sqrt(2 pi) polish it.
  if (!(p > 0.0 && p < 1.0)) return std::numeric_limits<double>::quiet_NaN();
  if (p == 0.5) return 0.0;   // Phi(0) = 1/2 exactly
  if (p > 0.5) return -normal_quantile(1.0 - p);
  auto Phi = [](double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); };
  double lo = -40.0, hi = 0.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (Phi(mid) < p) lo = mid; else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  const double inv_sqrt_2pi = 0.3989422804014327;   // 1 / sqrt(2 pi)
  for (int it = 0; it < 8; ++it) {
    const double pdf = inv_sqrt_2pi * std::exp(-0.5 * x * x);
    if (pdf <= 0.0) break;
    const double dx = (Phi(x) - p) / pdf;
    x -= dx;
    if (std::fabs(dx) <= 1e-16 * std::fabs(x)) break;
  }
  return x;
}

void static_breakpoints(const float* keys, int ncols, int64_t ld, int64_t ns, int Nr, float* B,
                        std::vector<PooledBuf>& keep, hipStream_t s) {
  const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(ns, MOM_THREADS * 16), 256));
  keep.emplace_back((size_t)ncols * nblk * 8);
  keep.emplace_back((size_t)2 * ncols * 8);
  double* part = keep[keep.size() - 2].as<double>();
  double* mom = keep.back().as<double>();   // [0, ncols): mean, [ncols, 2 ncols): variance
  hipLaunchKernelGGL(col_partial, dim3(nblk, ncols), dim3(MOM_THREADS), 0, s, keys, ld, ns, nblk,
                     nullptr, part);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(col_finish, dim3(cdiv(ncols, 64)), dim3(64), 0, s, part, nblk, ncols, ns,
                     mom);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(col_partial, dim3(nblk, ncols), dim3(MOM_THREADS), 0, s, keys, ld, ns, nblk,
                     mom, part);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(col_finish, dim3(cdiv(ncols, 64)), dim3(64), 0, s, part, nblk, ncols, ns,
                     mom + ncols);
  PDET_HIP(hipGetLastError());
  std::vector<double> hm((size_t)2 * ncols);
  PDET_HIP(hipMemcpyAsync(hm.data(), mom, hm.size() * 8, hipMemcpyDeviceToHost, s));
  PDET_HIP(hipStreamSynchronize(s));
  std::vector<double> zq(Nr);
  for (int u = 1; u < Nr; ++u) zq[u] = normal_quantile((double)u / Nr);
  std::vector<float> hb((size_t)ncols * (Nr - 1));
  for (int c = 0; c < ncols; ++c) {
    const double mu = hm[c], sd = std::sqrt(std::max(0.0, hm[ncols + c]));
    for (int u = 1; u < Nr; ++u) hb[(size_t)c * (Nr - 1) + u - 1] = (float)(mu + sd * zq[u]);
  }
  // interior entries 1 .. Nr-1 of each row of B (the outer ones come from the encode pass)
  PDET_HIP(hipMemcpy2DAsync(B + 1, (size_t)(Nr + 1) * 4, hb.data(), (size_t)(Nr - 1) * 4,
                            (size_t)(Nr - 1) * 4, ncols, hipMemcpyHostToDevice, s));
  PDET_HIP(hipStreamSynchronize(s));
}

void set_outer_breakpoints(float* B, const uint32_t* colmm, int ncols, int Nr, hipStream_t s) {
  hipLaunchKernelGGL(outer_kernel, dim3(cdiv(ncols, 64)), dim3(64), 0, s, B, colmm, ncols, Nr);
  PDET_HIP(hipGetLastError());
}

template <bool NZ>
void scan_rows_t(const uint32_t* in, uint32_t* out, uint32_t* totals, int rows, int64_t len,
                 DevBuf& tmp, hipStream_t s) {
  const int64_t nblk = (len + SCAN_BLOCK - 1) / SCAN_BLOCK;
  const size_t need = (size_t)rows * nblk * sizeof(uint32_t);
  if (tmp.bytes < need) tmp.alloc(need);
  uint32_t* sums = tmp.as<uint32_t>();
  hipLaunchKernelGGL(scan_sums<NZ>, dim3((unsigned)(rows * nblk)), dim3(SCAN_THREADS), 0, s, in, len,
                     nblk, sums);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_of_sums, dim3(rows), dim3(SCAN_THREADS), 0, s, sums, nblk, totals);
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_apply<NZ>, dim3((unsigned)(rows * nblk)), dim3(SCAN_THREADS), 0, s, in, out,
                     len, nblk, sums);
  PDET_HIP(hipGetLastError());
}

void scan_rows(const uint32_t* in, uint32_t* out, uint32_t* totals, int rows, int64_t len,
               DevBuf& tmp, hipStream_t s) {
  scan_rows_t<false>(in, out, totals, rows, len, tmp, s);
}

void scan_rows_nonzero(const uint32_t* in, uint32_t* out, uint32_t* totals, int rows,
                       int64_t len, DevBuf& tmp, hipStream_t s) {
  scan_rows_t<true>(in, out, totals, rows, len, tmp, s);
}

}  // namespace pdet
