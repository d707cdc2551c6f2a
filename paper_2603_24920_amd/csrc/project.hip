// Projection (Eq. 1) and dynamic encoding (Algorithm 1) for gfx950.
//
// P = X . A is a thin contraction (m x d) . (d x 16L). Each wave computes a 16-point
// tile against all 16-column tiles of A on the bf16 matrix cores with FP32 accumulation:
// every float32 operand is split exactly into three bf16 parts (hi + mid + lo: 3 x 8
// significant bits), and the six products whose weight is at least 2^-16 of hi * hi are
// accumulated (v_mfma_f32_16x16x32_bf16; each bf16 product is exact in FP32). The dropped
// terms are below 2^-24 relative, so the result stays within the float32 dot-product error
// bound, at a sixth of the matrix-core cycles of v_mfma_f32_16x16x4_f32. A tile whose rows
// are exact in bf16 (e.g. byte-valued data: mid = lo = 0) needs only the three hi * (A part)
// products. The same routine serves the sampled projection, the full encode pass and the
// query projection, so a point gets bit-identical hash values in all three.
//
// MFMA 16x16x32 bf16 lane layout: lane l supplies A[l%16][8*(l/16) .. +7] and
// B[8*(l/16) .. +7][l%16]; accumulator element i of lane l is D[4*(l/16)+i][l%16].
#include "internal.h"

namespace pdet {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// x = hi + mid + lo, each part bf16 (round to nearest even; the differences are exact).
__device__ inline void split3(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = (__bf16)x;
  const float r1 = x - (float)hi;
  mid = (__bf16)r1;
  lo = (__bf16)(r1 - (float)mid);
}

enum Mode { MODE_PROJECT = 0, MODE_SAMPLE = 1, MODE_ENCODE = 2 };

constexpr int PROJ_THREADS = 1024;
constexpr int PROJ_WAVES = PROJ_THREADS / 64;
constexpr int DK_MAX = 128;              // rows of A staged per chunk (at most)
constexpr int KB_MAX = DK_MAX / 32;      // 32-row MFMA steps per chunk

struct ProjArgs {
  const float* X;          // [rows of X][d]
  int64_t m;               // points in this launch
  int d;
  const int64_t* rows;     // MODE_SAMPLE: X row of point p; else nullptr (p itself)
  const float* A;          // [d][NC] padded columns for the trees of this launch
  int tree0;               // first tree of this launch
  int ntrees;              // trees of this launch (<= NT)
  int L, K, Nr, bits;
  int dk;                  // rows of A staged per chunk
  // MODE_PROJECT: out[p][L*K]; MODE_SAMPLE: out[col][ld] (column-major)
  float* out;
  int64_t ld;
  // MODE_ENCODE
  const float* Btab;       // [L*K][Nr+1]
  uint8_t* codes;          // [L][n][KP]
  uint16_t* flkey;         // [L][n]: first-layer key (leading code bit of each dimension,
                           // dimension 0 most significant)
  int64_t n;
  uint32_t* colmin;        // [L*K] ordered-uint min / max
  uint32_t* colmax;
  uint32_t* nonfinite;     // set to 1 if some projection is NaN or infinite
};

template <int NT, bool VEC4, int MODE>
__global__ __launch_bounds__(PROJ_THREADS) void project_kernel(ProjArgs a) {
  constexpr int NC = NT * 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // A as bf16 parts, [part][32-row step][lane group][column] of 8 consecutive rows (16
  // bytes): the 16 lanes of a group read 256 consecutive bytes per operand
  uint4* As = reinterpret_cast<uint4*>(smem_raw);
  const int kbc = (a.dk + 31) / 32;        // 32-row steps per chunk
  // [NT*K][Nr + 1]: interior breakpoints + inf, one padding word per column so that the
  // 16 columns a wave searches at once sit in different LDS banks
  float* Bs = reinterpret_cast<float*>(As + 3 * kbc * 4 * NC);
  const int bstride = a.Nr + 1;
  // the code staging area starts 16-byte aligned (rounded table size)
  uint8_t* stage = reinterpret_cast<uint8_t*>(
      Bs + (MODE == MODE_ENCODE ? ((NT * a.K * bstride + 3) & ~3) : 0));

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col16 = lane & 15;
  const int grp = lane >> 4;
  const int nchunks = (a.d + a.dk - 1) / a.dk;

  if constexpr (MODE == MODE_ENCODE) {
    // the Nr - 1 interior breakpoints B(2..Nr) of every column of this launch, in
    // breadth-first order of the implicit search tree (slot k = 1 .. Nr-1 holds the
    // in-order element (2j+1) 2^(bits-1-depth) - 1, j = k - 2^depth): the candidates of one
    // search step are neighbours, so the lanes searching a column spread over the banks
    const int tot = NT * a.K * (a.Nr - 1);
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int c = e / (a.Nr - 1), k = e % (a.Nr - 1) + 1;
      const int depth = 31 - __clz(k), j = k - (1 << depth);
      const int inorder = ((2 * j + 1) << (a.bits - 1 - depth)) - 1;
      const int gcol = (a.tree0 + c / a.K) * a.K + c % a.K;
      Bs[c * bstride + k] =
          (c / a.K < a.ntrees) ? a.Btab[(int64_t)gcol * (a.Nr + 1) + 1 + inorder] : INFINITY;
    }
  }

  auto load_A = [&](int chunk) {
    const int k0 = chunk * a.dk;
    const int tot = kbc * 4 * NC;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int c = e % NC, g = (e / NC) & 3, kb = e / (4 * NC);
      bf16x8 hi, mid, lo;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int r = k0 + 32 * kb + 8 * g + j;
        __bf16 h, m, l;
        split3((r < a.d && 32 * kb + 8 * g + j < a.dk) ? a.A[(int64_t)r * NC + c] : 0.0f, h, m,
               l);
        hi[j] = h; mid[j] = m; lo[j] = l;
      }
      As[(0 * kbc * 4 + kb * 4 + g) * NC + c] = *reinterpret_cast<const uint4*>(&hi);
      As[(1 * kbc * 4 + kb * 4 + g) * NC + c] = *reinterpret_cast<const uint4*>(&mid);
      As[(2 * kbc * 4 + kb * 4 + g) * NC + c] = *reinterpret_cast<const uint4*>(&lo);
    }
  };
  // column min / max of this workgroup (ordered uints), reduced in LDS before one global
  // atomic per column: all workgroups update the same few cache lines
  __shared__ uint32_t wg_min[NT * 16], wg_max[NT * 16];
  if ((MODE == MODE_ENCODE || MODE == MODE_SAMPLE) && threadIdx.x < NT * 16) {
    wg_min[threadIdx.x] = float_to_ordered(INFINITY);
    wg_max[threadIdx.x] = float_to_ordered(-INFINITY);
  }
  if (nchunks == 1) load_A(0);
  __syncthreads();

  float vmin[NT], vmax[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) { vmin[t] = INFINITY; vmax[t] = -INFINITY; }
  bool nonfin = false;   // a projection of this lane's points was NaN or infinite

  const int64_t ntiles = (a.m + 15) / 16;
  const int64_t tiles_per_iter = (int64_t)gridDim.x * PROJ_WAVES;
  const int64_t iters = (ntiles + tiles_per_iter - 1) / tiles_per_iter;
  // this lane's 8 consecutive values of its point per 32-row step of a chunk
  float4 xb[2 * KB_MAX];
  auto load_x = [&](int64_t tile, int k0) {
    const int64_t p_load = tile * 16 + col16;           // point whose X row this lane reads
    const bool load_ok = p_load < a.m;
    int64_t xrow = 0;
    if (load_ok) xrow = (MODE == MODE_SAMPLE) ? a.rows[p_load] : p_load;
    const float* xr = a.X + xrow * (int64_t)a.d;
    const int kend = min(a.dk, a.d - k0);
#pragma unroll
    for (int u = 0; u < 2 * KB_MAX; ++u) {
      const int kk = k0 + (u >> 1) * 32 + 8 * grp + 4 * (u & 1);   // first of 4 values
      if ((u >> 1) * 32 < kend) {
        if (VEC4 && load_ok && kk + 3 < a.d) {
          xb[u] = *reinterpret_cast<const float4*>(xr + kk);
        } else {
          xb[u].x = (load_ok && kk + 0 < a.d) ? xr[kk + 0] : 0.0f;
          xb[u].y = (load_ok && kk + 1 < a.d) ? xr[kk + 1] : 0.0f;
          xb[u].z = (load_ok && kk + 2 < a.d) ? xr[kk + 2] : 0.0f;
          xb[u].w = (load_ok && kk + 3 < a.d) ? xr[kk + 3] : 0.0f;
        }
      }
    }
  };
  // with one chunk, the next tile's values are loaded while this tile's hash values are
  // searched and written
  const bool single = nchunks == 1;
  const int64_t tile0 = (int64_t)blockIdx.x * PROJ_WAVES + wave;
  if (single && iters > 0) load_x(tile0, 0);
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t tile = it * tiles_per_iter + tile0;

    floatx4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int chunk = 0; chunk < nchunks; ++chunk) {
      if (nchunks > 1) {
        __syncthreads();
        load_A(chunk);
        __syncthreads();
      }
      const int k0 = chunk * a.dk;
      const int kend = min(a.dk, a.d - k0);
      if (!single) load_x(tile, k0);
#pragma unroll
      for (int kb = 0; kb < KB_MAX; ++kb) {
        if (kb * 32 < kend) {
          const float xv[8] = {xb[2 * kb].x, xb[2 * kb].y, xb[2 * kb].z, xb[2 * kb].w,
                               xb[2 * kb + 1].x, xb[2 * kb + 1].y, xb[2 * kb + 1].z,
                               xb[2 * kb + 1].w};
          // hi parts first; mid and lo (split3's remaining steps) only when some value of
          // the wave is not exact in bf16 (otherwise both are zero and their products drop)
          bf16x8 xh, xm = {}, xl = {};
          bool inexact = false;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            xh[j] = (__bf16)xv[j];
            inexact = inexact || (float)xh[j] != xv[j];
          }
          const bool full = __ballot(inexact) != 0;   // wave-uniform
          if (full) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const float r1 = xv[j] - (float)xh[j];
              xm[j] = (__bf16)r1;
              xl[j] = (__bf16)(r1 - (float)xm[j]);
            }
          }
          const uint4* ab = As + (kb * 4 + grp) * NC + col16;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const uint4 h4 = ab[t * 16], m4 = ab[kbc * 4 * NC + t * 16],
                        l4 = ab[2 * kbc * 4 * NC + t * 16];
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&h4);
            const bf16x8 am = *reinterpret_cast<const bf16x8*>(&m4);
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(&l4);
            // smallest terms first
            if (full) {
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, ah, acc[t], 0, 0, 0);
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xm, am, acc[t], 0, 0, 0);
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, al, acc[t], 0, 0, 0);
            if (full) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xm, ah, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, am, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ah, acc[t], 0, 0, 0);
          }
        }
      }
    }
    if (single && it + 1 < iters) load_x(tile + tiles_per_iter, 0);

    // acc[t][i] = P[tile*16 + 4*grp + i][t*16 + col16]
    const int64_t pbase = tile * 16 + 4 * grp;
    if constexpr (MODE == MODE_PROJECT || MODE == MODE_SAMPLE) {
      if (col16 < a.K) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (t >= a.ntrees) break;
          const int gcol = (a.tree0 + t) * a.K + col16;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t p = pbase + i;
            if (p < a.m) {
              if (MODE == MODE_PROJECT) {
                a.out[p * (int64_t)(a.L * a.K) + gcol] = acc[t][i];
              } else {
                a.out[(int64_t)gcol * a.ld + p] = acc[t][i];
                vmin[t] = fminf(vmin[t], acc[t][i]);
                vmax[t] = fmaxf(vmax[t], acc[t][i]);
              }
            }
          }
        }
      }
    } else {
      uint8_t* st = stage + wave * (16 * NT * KP);          // [16 points][NT][KP]
      // descend the implicit search trees of the lane's NT x 4 hash values together, one
      // level per step: the 4*NT table reads of a step are issued before any compare (one
      // search after another would wait for every read). After bits steps,
      // node - Nr = #{B(z) <= h}. Lanes past the K columns search column K-1 and discard it.
      int node[NT][4];
      const int ccol = min(col16, a.K - 1);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) node[t][i] = 1;
      for (int step = 0; step < a.bits; ++step) {
        float b[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float* tab = Bs + (t * a.K + ccol) * bstride;
#pragma unroll
          for (int i = 0; i < 4; ++i) b[t][i] = tab[node[t][i]];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) node[t][i] = 2 * node[t][i] + (b[t][i] <= acc[t][i] ? 1 : 0);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pl = 4 * grp + i;
          uint8_t code = 0;
          if (col16 < a.K && t < a.ntrees) {
            const float h = acc[t][i];
            code = static_cast<uint8_t>(node[t][i] - a.Nr);
            if (pbase + i < a.m) {
              vmin[t] = fminf(vmin[t], h);
              vmax[t] = fmaxf(vmax[t], h);
              nonfin = nonfin || !isfinite(h);
            }
          }
          st[(pl * NT + t) * KP + col16] = code;
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      // lane e < 16*NT writes the 16-byte code row of point e%16 in tree e/16
      if (lane < 16 * a.ntrees) {
        const int pl = lane & 15, t = lane >> 4;
        const int64_t p = tile * 16 + pl;
        if (p < a.m) {
          const uint4 v = *reinterpret_cast<const uint4*>(st + (pl * NT + t) * KP);
          *reinterpret_cast<uint4*>(a.codes + ((int64_t)(a.tree0 + t) * a.n + p) * KP) = v;
          const uint32_t w[4] = {v.x, v.y, v.z, v.w};
          uint32_t key = 0;
          for (int j = 0; j < a.K; ++j)
            key |= ((w[j >> 2] >> (8 * (j & 3) + a.bits - 1)) & 1u) << (a.K - 1 - j);
          a.flkey[(int64_t)(a.tree0 + t) * a.n + p] = (uint16_t)key;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  if constexpr (MODE == MODE_ENCODE || MODE == MODE_SAMPLE) {
    if (MODE == MODE_ENCODE && __ballot(nonfin) && lane == 0) atomicOr(a.nonfinite, 1u);
    // column min / max over all points (outer breakpoints B(1), B(Nr+1)), or over the
    // sampled points (the range of the breakpoint selection's buckets)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float lo = vmin[t], hi = vmax[t];
      lo = fminf(lo, __shfl_xor(lo, 16)); hi = fmaxf(hi, __shfl_xor(hi, 16));
      lo = fminf(lo, __shfl_xor(lo, 32)); hi = fmaxf(hi, __shfl_xor(hi, 32));
      if (lane < a.K && t < a.ntrees && lo <= hi) {
        atomicMin(&wg_min[t * 16 + lane], float_to_ordered(lo));
        atomicMax(&wg_max[t * 16 + lane], float_to_ordered(hi));
      }
    }
    __syncthreads();
    if (threadIdx.x < NT * 16) {
      const int t = threadIdx.x >> 4, j = threadIdx.x & 15;
      const uint32_t lo = wg_min[threadIdx.x], hi = wg_max[threadIdx.x];
      if (j < a.K && t < a.ntrees && lo <= hi) {
        const int gcol = (a.tree0 + t) * a.K + j;
        atomicMin(&a.colmin[gcol], lo);
        atomicMax(&a.colmax[gcol], hi);
      }
    }
  }
}

template <int NT, bool VEC4, int MODE>
void launch_t(const ProjArgs& a, hipStream_t s, size_t smem, int grid) {
  auto k = project_kernel<NT, VEC4, MODE>;
  PDET_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  hipLaunchKernelGGL(k, dim3(grid), dim3(PROJ_THREADS), smem, s, a);
  PDET_HIP(hipGetLastError());
}

template <int MODE>
void launch_mode(int nt, bool vec4, const ProjArgs& a, hipStream_t s, size_t smem, int grid) {
#define PDET_CASE(N)                                                   \
  case N:                                                              \
    if (vec4) launch_t<N, true, MODE>(a, s, smem, grid);               \
    else launch_t<N, false, MODE>(a, s, smem, grid);                   \
    break;
  switch (nt) {
    PDET_CASE(1) PDET_CASE(2) PDET_CASE(4)
    default: throw Error{PDET_EUNSUPPORTED, "projection tile count"};
  }
#undef PDET_CASE
}

int grid_for(int64_t m, int dev_cus) {
  const int64_t tiles = (m + 15) / 16;
  const int64_t wg = (tiles + PROJ_WAVES - 1) / PROJ_WAVES;
  return (int)std::max<int64_t>(1, std::min<int64_t>(wg, (int64_t)dev_cus * 2));
}

}  // namespace

// Trees per launch: 4 (64 columns), the LDS budget of the encode tables.
constexpr int TREES_PER_LAUNCH = 4;

static int group_nt(int trees) { return trees <= 1 ? 1 : (trees <= 2 ? 2 : 4); }

// Encoded rows go to codes [L][stride][KP] and keys [L][stride] (the index's own arrays
// unless given).
// MODE_SAMPLE: the column min / max of the sampled hash values go to mm ([2][L*K] ordered).
void run_projection(const Index& ix, const float* X, int64_t m, const int64_t* rows, int mode,
                    float* out, int64_t ld, hipStream_t s, uint8_t* codes = nullptr,
                    uint16_t* keys = nullptr, int64_t stride = 0, uint32_t* mm = nullptr) {
  for (int t0 = 0; t0 < ix.L; t0 += TREES_PER_LAUNCH) {
    const int trees = std::min(TREES_PER_LAUNCH, ix.L - t0);
    const int nt = group_nt(trees);
    ProjArgs a{};
    a.X = X; a.m = m; a.d = ix.d; a.rows = rows;
    a.tree0 = t0; a.ntrees = trees; a.L = ix.L; a.K = ix.K; a.Nr = ix.Nr; a.bits = ix.bits;
    a.n = codes ? stride : ix.n;
    a.out = out; a.ld = ld;
    a.Btab = ix.B.as<float>();
    a.codes = codes ? codes : ix.codes.as<uint8_t>();
    a.flkey = codes ? keys : ix.flkey.as<uint16_t>();
    a.colmin = mode == MODE_SAMPLE ? mm : ix.colmm.as<uint32_t>();
    a.colmax = (mode == MODE_SAMPLE ? mm : ix.colmm.as<uint32_t>()) + ix.L * ix.K;
    a.nonfinite = ix.nonfinite.as<uint32_t>();
    // A is stored per launch group: [group][d][NC]
    a.A = ix.A.as<float>() + (int64_t)(t0 / TREES_PER_LAUNCH) * ix.d * (TREES_PER_LAUNCH * 16);
    const int NC = nt * 16;
    a.dk = std::min(((ix.d + 31) / 32) * 32, DK_MAX);
    size_t smem = (size_t)3 * ((a.dk + 31) / 32) * 4 * NC * 16;
    if (mode == MODE_ENCODE)
      smem += (size_t)((nt * ix.K * (ix.Nr + 1) + 3) & ~3) * 4 + (size_t)PROJ_WAVES * 16 * nt * KP;
    const bool vec4 = (ix.d % 4) == 0;
    const int grid = grid_for(m, ix.num_cus);
    if (mode == MODE_PROJECT) launch_mode<MODE_PROJECT>(nt, vec4, a, s, smem, grid);
    else if (mode == MODE_SAMPLE) launch_mode<MODE_SAMPLE>(nt, vec4, a, s, smem, grid);
    else launch_mode<MODE_ENCODE>(nt, vec4, a, s, smem, grid);
  }
}

void project_points(const Index& ix, const float* X, int64_t m, float* out, hipStream_t s) {
  run_projection(ix, X, m, nullptr, MODE_PROJECT, out, 0, s);
}
void project_sample(const Index& ix, const int64_t* rows, int64_t m, float* out, int64_t ld,
                    uint32_t* mm, hipStream_t s) {
  run_projection(ix, ix.X, m, rows, MODE_SAMPLE, out, ld, s, nullptr, nullptr, 0, mm);
}
void encode_points(const Index& ix, hipStream_t s) {
  run_projection(ix, ix.X, ix.n, nullptr, MODE_ENCODE, nullptr, 0, s);
}
void encode_rows(const Index& ix, const float* X, int64_t m, uint8_t* codes, uint16_t* keys,
                 hipStream_t s) {
  run_projection(ix, X, m, nullptr, MODE_ENCODE, nullptr, 0, s, codes, keys, m);
}

// Padded device layout of A: for each group of 4 trees, [d][64] with column
// 16*t + j = a_{(g*4+t), j} for j < K and zeros elsewhere.
std::vector<float> pad_projection(const float* proj, int d, int L, int K) {
  const int groups = (L + TREES_PER_LAUNCH - 1) / TREES_PER_LAUNCH;
  const int NCg = TREES_PER_LAUNCH * 16;
  std::vector<float> out((size_t)groups * d * NCg, 0.0f);
  for (int g = 0; g < groups; ++g) {
    const int trees = std::min(TREES_PER_LAUNCH, L - g * TREES_PER_LAUNCH);
    const int nc = group_nt(trees) * 16;   // the launch reads NC = nt*16 columns per row
    for (int r = 0; r < d; ++r)
      for (int t = 0; t < trees; ++t)
        for (int j = 0; j < K; ++j)
          out[(size_t)g * d * NCg + (size_t)r * nc + t * 16 + j] =
              proj[(size_t)r * L * K + (g * TREES_PER_LAUNCH + t) * K + j];
  }
  return out;
}

}  // namespace pdet
