// DE-Tree creation (Algorithm 2, node split rule of the indexing phase), bulk form.
//
// A tree is flattened over a point permutation `perm`: every node owns a contiguous
// range, a split partitions its range by the chosen bit (bit-0 child first), so the
// final leaf order along `perm` is the depth-first order of the tree.
//
//  1. first layer: counting sort of the points by the K-bit first-layer keys the encoder
//     wrote (2^K nodes); the scatter also moves each point's 16-byte code row next to its
//     id, so later passes read contiguous (row, id) ranges instead of gathering rows;
//  2. nodes larger than LDS_SEG_CAP: level-synchronous global passes (bit counts per
//     dimension over the node's contiguous rows, the most balanced dimension, a partition
//     into the other of two (row, id) buffers); a node keeps the index of the buffer that
//     holds it, and a leaf that ends up in the second buffer has its ids copied back;
//  3. nodes of (max_leaf, LDS_SEG_CAP] points: one workgroup loads the node into LDS and
//     splits every open node of a level at once (bit counts by wave ballots, one
//     workgroup-wide scan for the partition), level after level; for very small max_leaf
//     (more open nodes than the workgroup tracks) a depth-first variant splits one node at
//     a time;
//  4. leaves are recorded at their start position, numbered by a prefix scan, and written
//     as flat tables with their breakpoint boxes.
// A node is a leaf iff it has at most max_leaf points or every dimension is fully
// refined. Empty nodes are dropped. Inside a leaf the point order is unspecified.
#include "devutil.h"
#include "internal.h"

namespace pdet {
namespace {

struct Seg {
  int32_t tree, start, count;
  uint8_t buf, pad[3];        // buffer (0 or 1) that holds the node's rows and ids
  uint8_t depth[KP];
  uint8_t prefix[KP];
};

// Row and id buffers, [L][n] each, in permutation order. ids[0] is the index's perm (the
// final output); rows[1] / ids[1] are build temporaries.
struct Bufs {
  uint4* rows[2];
  int32_t* ids[2];
};

struct Copy {
  int32_t tree, start, count;
};

struct LeafOut {
  uint32_t* cnt_at;     // [L][n] leaf size recorded at the leaf's first position
  uint16_t* hidx_at;    // [L][n][KP]
};

// Nodes finished in LDS come in size classes (CLS_BELOW[c], CLS_CAP[c]], one list each.
constexpr int NCLS = 4;
constexpr int CLS_CAP[NCLS] = {256, 512, 1024, LDS_SEG_CAP};
constexpr int CLS_BELOW[NCLS] = {0, 256, 512, 1024};

__host__ __device__ inline int size_class(int count) {
  return count <= 256 ? 0 : count <= 512 ? 1 : count <= 1024 ? 2 : 3;
}

struct Lists {
  Seg* big_next; uint32_t* n_big_next; uint32_t* pts_big_next;   // and their total size
  Seg* mid[NCLS]; uint32_t* n_mid;                              // n_mid[c]: class c
  Copy* copies; uint32_t* n_copies;   // leaves whose ids sit in buffer 1
  uint32_t* cnt_next = nullptr;   // [big_next index][KP]: next-bit counts, if known
};

// A global pass over the nodes larger than LDS_SEG_CAP gives each workgroup one unit: at
// most SEG_CHUNK consecutive positions of one node (so the grid follows the points, not
// the largest node).
constexpr int SEG_CHUNK = 4096;
struct Unit {
  uint32_t seg;      // node index in the level's list
  uint32_t first;    // first position within the node
};

__device__ inline uint32_t code_byte(const uint4& v, int j) {
  const uint32_t w = (j < 8) ? ((j < 4) ? v.x : v.y) : ((j < 12) ? v.z : v.w);
  return (w >> (8 * (j & 3))) & 255u;
}

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over a whole wave (every lane active): row sums by DPP moves (quad swaps, half-row and
// row mirrors), then the four row totals read into scalar registers; the result is uniform.
__device__ inline uint32_t wave_total(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// 1 in every byte of w that is not zero, 0 in the others.
__device__ inline uint32_t nonzero_bytes(uint32_t w) {
  return ((((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u) >> 7;
}

__device__ inline uint32_t lanes_below(uint64_t mask) { return lanes_below_mask(mask); }

// A leaf record: the leaf's size at its first position and its 16 index words
// ((1 << depth) | prefix per dimension, 0 past K) in two 16-byte stores.
__device__ inline void store_leaf(const LeafOut& lo, int64_t n, int tree, int64_t start, int count,
                                  const uint32_t (&hv)[KP]) {
  lo.cnt_at[(int64_t)tree * n + start] = (uint32_t)count;
  uint4* h = reinterpret_cast<uint4*>(lo.hidx_at + ((int64_t)tree * n + start) * KP);
  h[0] = make_uint4(hv[0] | (hv[1] << 16), hv[2] | (hv[3] << 16), hv[4] | (hv[5] << 16),
                    hv[6] | (hv[7] << 16));
  h[1] = make_uint4(hv[8] | (hv[9] << 16), hv[10] | (hv[11] << 16), hv[12] | (hv[13] << 16),
                    hv[14] | (hv[15] << 16));
}

__device__ void emit_leaf(const LeafOut& lo, int64_t n, int tree, int64_t start, int count,
                          const uint8_t* depth, const uint8_t* prefix, int K) {
  uint32_t hv[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) hv[j] = (j < K) ? ((1u << depth[j]) | prefix[j]) & 0xffffu : 0u;
  store_leaf(lo, n, tree, start, count, hv);
}

// The leaf record of child `bit` of a node split on dimension j (depth and prefix of the
// parent, read in place).
__device__ void emit_child_leaf(const LeafOut& lo, int64_t n, int tree, int64_t start, int count,
                                const uint8_t* depth, const uint8_t* prefix, int j, int bit,
                                int K) {
  uint32_t hv[KP];
#pragma unroll
  for (int jj = 0; jj < KP; ++jj) {
    const uint32_t d = depth[jj] + (jj == j ? 1u : 0u);
    const uint32_t p = (jj == j) ? prefix[jj] * 2u + (uint32_t)bit : prefix[jj];
    hv[jj] = (jj < K) ? ((1u << d) | p) & 0xffffu : 0u;
  }
  store_leaf(lo, n, tree, start, count, hv);
}

__device__ inline bool fully_refined(const uint8_t* depth, int K, int bits) {
  bool f = true;
  for (int j = 0; j < K; ++j) f = f && (depth[j] >= bits);
  return f;
}

// A node to its place: a leaf (records at its start; ids copied later if they sit in buffer
// 1), an LDS size class, or the next global level (with its bit counts, if known). Called by
// every lane of the wave; lanes with active == false take no place.
__device__ void route(const Seg& s, int K, int bits, int max_leaf, int64_t n, const LeafOut& lo,
                      const Lists& li, bool active, const uint32_t* counts = nullptr) {
  active = active && s.count > 0;
  const bool leaf = active && (s.count <= max_leaf || fully_refined(s.depth, K, bits));
  const bool mid = active && !leaf && s.count <= LDS_SEG_CAP;
  const bool big = active && !leaf && !mid;
  const int c = mid ? size_class(s.count) : -1;
  const bool copy = leaf && s.buf == 1;
  if (leaf) emit_leaf(lo, n, s.tree, s.start, s.count, s.depth, s.prefix, K);
  // the wave's places in every list it appends to: lane 0 reserves the copies, lane 1 + cl
  // size class cl, lane 5 the next level, lane 6 adds its points; the reservations are all
  // in flight together (one after another, each would wait for the one before)
  const uint64_t m_copy = __ballot(copy);
  uint64_t m_mid[NCLS];
#pragma unroll
  for (int cl = 0; cl < NCLS; ++cl) m_mid[cl] = __ballot(c == cl);
  const uint64_t m_big = __ballot(big);
  uint32_t pts = big ? (uint32_t)s.count : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pts += __shfl_xor(pts, o);
  const int lane = threadIdx.x & 63;
  uint32_t* ctr = nullptr;
  uint32_t add = 0;
  if (lane == 0) { ctr = li.n_copies; add = (uint32_t)__popcll(m_copy); }
#pragma unroll
  for (int cl = 0; cl < NCLS; ++cl)
    if (lane == 1 + cl) { ctr = &li.n_mid[cl]; add = (uint32_t)__popcll(m_mid[cl]); }
  if (lane == 1 + NCLS) { ctr = li.n_big_next; add = (uint32_t)__popcll(m_big); }
  if (lane == 2 + NCLS) { ctr = li.pts_big_next; add = pts; }
  uint32_t got = 0;
  if (add) got = atomicAdd(ctr, add);
  if (copy) {
    const uint32_t cp = (uint32_t)__builtin_amdgcn_readlane((int)got, 0) + lanes_below_mask(m_copy);
    li.copies[cp] = Copy{s.tree, s.start, s.count};
  }
#pragma unroll
  for (int cl = 0; cl < NCLS; ++cl) {
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)got, 1 + cl);
    if (c == cl) li.mid[cl][b + lanes_below_mask(m_mid[cl])] = s;
  }
  if (big) {
    const uint32_t k =
        (uint32_t)__builtin_amdgcn_readlane((int)got, 1 + NCLS) + lanes_below_mask(m_big);
    li.big_next[k] = s;
    if (counts && li.cnt_next)
      for (int j = 0; j < KP; ++j) li.cnt_next[(int64_t)k * KP + j] = counts[j];
  }
}

// First layer: a stable LSD radix sort of each tree's 16-bit keys in two 8-bit passes
// (one for K <= 8). A workgroup takes RK_TILE consecutive items of one tree in RK_ROUNDS
// rounds of 256, in order; the lanes of a wave holding the same digit find each other with
// eight ballots, so an item's place is its digit's running offset (the exclusive scan of the
// [tree][digit][tile] counts, plus the tile's earlier rounds) plus the same-digit items of
// the earlier waves and lanes of its round. The output keeps input order within a digit.
constexpr int RK_THREADS = 256;
constexpr int RK_ROUNDS = 8;
constexpr int RK_TILE = RK_THREADS * RK_ROUNDS;
constexpr int RK_WAVES = RK_THREADS / 64;

// The lanes of the wave that hold the same 8-bit digit as this one (valid lanes only).
__device__ inline uint64_t same_digit_lanes(uint32_t dgt, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool set = (dgt >> bit) & 1u;
    const uint64_t bb = __ballot(valid && set);
    m &= set ? bb : ~bb;
  }
  return m;
}

// h[tree][digit][tile]: items of the tile whose key has `digit` at bits SHIFT..SHIFT+7.
template <int SHIFT>
__global__ __launch_bounds__(RK_THREADS) void rk_hist(const uint16_t* keys, int64_t n, int nblk,
                                                      uint32_t* h) {
  __shared__ uint32_t cnt[256];
  const int tree = blockIdx.y, blk = blockIdx.x;
  cnt[threadIdx.x] = 0;
  const uint16_t* kt = keys + (int64_t)tree * n;
  const int64_t p0 = (int64_t)blk * RK_TILE;
  // the tile's keys, 8 per thread (one 16-byte load for a whole tile of a row whose length
  // is a multiple of 8); only the counts matter here, so any key may go to any thread
  static_assert(RK_TILE == 8 * RK_THREADS, "8 keys per thread");
  uint32_t kv[8];
  bool ok[8];
  if ((n & 7) == 0 && p0 + RK_TILE <= n) {
    const uint4 w = reinterpret_cast<const uint4*>(kt + p0)[threadIdx.x];
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) { kv[2 * e] = ws[e] & 0xffffu; kv[2 * e + 1] = ws[e] >> 16; }
#pragma unroll
    for (int e = 0; e < 8; ++e) ok[e] = true;
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int64_t p = p0 + r * RK_THREADS + threadIdx.x;
      ok[r] = p < n;
      kv[r] = ok[r] ? kt[p] : 0u;
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (ok[e]) atomicAdd(&cnt[(kv[e] >> SHIFT) & 255u], 1u);
  __syncthreads();
  h[((int64_t)tree * 256 + threadIdx.x) * nblk + blk] = cnt[threadIdx.x];
}

// One pass: items (key, code row, id) of each tree to their places. FIRST: the input is
// the encoder's output in point order (ids are positions). The tile is first sorted by
// digit in LDS (stable: rounds, then waves, then lanes, in input order), then written out
// in tile order, so that the items of one digit leave as one contiguous run (whole cache
// lines instead of one 16-byte row per digit and round).
template <int SHIFT, bool FIRST>
__global__ __launch_bounds__(RK_THREADS) void rk_scatter(const uint16_t* kin, const uint4* rin,
                                                         const int32_t* iin, int64_t n, int nblk,
                                                         const uint32_t* off, uint16_t* kout,
                                                         uint4* rout, int32_t* iout) {
  __shared__ uint4 srow[RK_TILE];
  __shared__ int32_t sid[RK_TILE];
  __shared__ uint16_t skey[RK_TILE];
  __shared__ uint32_t lcur[256];    // running local position of each digit
  __shared__ uint32_t lbase[256];   // first local position of each digit
  __shared__ uint32_t gbase[256];   // first global position of each digit's run of this tile
  __shared__ uint32_t wc[RK_WAVES][256];
  __shared__ uint32_t sh[RK_THREADS / 64 + 1];
  const int tree = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x, wave = tid >> 6;
  const int64_t tb = (int64_t)tree * n;
  const int64_t p0 = (int64_t)blk * RK_TILE;
  const int m = (int)min<int64_t>(RK_TILE, n - p0);   // items of this tile
  // the tile's keys (rows and ids are loaded one round ahead of their placement)
  uint32_t key[RK_ROUNDS];
#pragma unroll
  for (int r = 0; r < RK_ROUNDS; ++r) {
    const int q = r * RK_THREADS + tid;
    key[r] = q < m ? kin[tb + p0 + q] : 0u;
  }
  auto load = [&](int r, uint4& row, int32_t& id) {
    const int q = r * RK_THREADS + tid;
    row = make_uint4(0, 0, 0, 0);
    id = 0;
    if (q < m) {
      row = rin[tb + p0 + q];
      id = FIRST ? (int32_t)(p0 + q) : iin[tb + p0 + q];
    }
  };
  uint4 row, nrow;
  int32_t id, nid;
  load(0, row, id);
  // local digit counts -> local bases (an exclusive scan over the 256 digits)
  {
    const uint32_t gb = off[((int64_t)tree * 256 + tid) * nblk + blk];
    gbase[tid] = gb;
    lcur[tid] = 0;
  }
#pragma unroll
  for (int w = 0; w < RK_WAVES; ++w) wc[w][tid] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RK_ROUNDS; ++r)
    if (r * RK_THREADS + tid < m) atomicAdd(&lcur[(key[r] >> SHIFT) & 255u], 1u);
  __syncthreads();
  {
    uint32_t tot;
    const uint32_t ex = block_excl_scan<RK_THREADS>(lcur[tid], sh, &tot);
    __syncthreads();
    lbase[tid] = ex;
    lcur[tid] = ex;
  }
  __syncthreads();
  // stable local placement, round by round
#pragma unroll
  for (int r = 0; r < RK_ROUNDS; ++r) {
    if (r + 1 < RK_ROUNDS) load(r + 1, nrow, nid);
    const bool v = r * RK_THREADS + tid < m;
    const uint32_t d = (key[r] >> SHIFT) & 255u;
    const uint64_t mk = same_digit_lanes(d, v);
    const uint32_t rank = lanes_below_mask(mk);
    if (v && rank == 0) wc[wave][d] = (uint32_t)__popcll(mk);
    __syncthreads();
    if (v) {
      uint32_t pos = lcur[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wc[w][d];
      srow[pos] = row;
      sid[pos] = id;
      skey[pos] = (uint16_t)key[r];
    }
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < RK_WAVES; ++w) { t += wc[w][tid]; wc[w][tid] = 0; }
    lcur[tid] += t;
    __syncthreads();
    row = nrow;
    id = nid;
  }
  // out in tile order: consecutive local positions of one digit go to consecutive places
#pragma unroll 2
  for (int q = tid; q < m; q += RK_THREADS) {
    const uint32_t k = skey[q];
    const uint32_t d = (k >> SHIFT) & 255u;
    const uint32_t pos = gbase[d] + (uint32_t)q - lbase[d];
    kout[tb + pos] = (uint16_t)k;
    rout[tb + pos] = srow[q];
    iout[tb + pos] = sid[q];
  }
}

// First-layer nodes from the sorted keys: start[tree][key] and end[tree][key] at the
// boundaries of each key's run (both zero for keys that do not occur).
// 8 consecutive keys per thread (one 16-byte load when the row allows) and their neighbours;
// a run of equal keys starts where the key before differs and ends where the key after does
// (0xffffffff stands for the missing neighbours of the row's ends).
__global__ void rk_bounds(const uint16_t* keys, int64_t n, int K, uint32_t* start,
                          uint32_t* end) {
  const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  const int tree = blockIdx.y;
  if (p0 >= n) return;
  const uint16_t* kt = keys + (int64_t)tree * n;
  uint32_t k[10];
  k[0] = p0 > 0 ? kt[p0 - 1] : 0xffffffffu;
  if ((n & 7) == 0) {   // rows start 16-byte aligned and hold whole groups of 8
    const uint4 w = *reinterpret_cast<const uint4*>(kt + p0);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) { k[1 + 2 * e] = ws[e] & 0xffffu; k[2 + 2 * e] = ws[e] >> 16; }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) k[1 + e] = p0 + e < n ? kt[p0 + e] : 0xffffffffu;
  }
  k[9] = p0 + 8 < n ? kt[p0 + 8] : 0xffffffffu;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t p = p0 + e;
    if (p >= n) break;
    const uint32_t key = k[1 + e];
    const int64_t g = ((int64_t)tree << K) + key;
    if (k[e] != key) start[g] = (uint32_t)p;
    if (k[e + 2] != key) end[g] = (uint32_t)(p + 1);
  }
}

__global__ void rk_counts(const uint32_t* start, const uint32_t* end, int64_t total,
                          uint32_t* hist) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < total) hist[g] = end[g] - start[g];
}

__global__ void fl_segments(const uint32_t* hist, const uint32_t* off, int L, int K, int bits,
                            int max_leaf, int64_t n, LeafOut lo, Lists li) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = g < ((int64_t)L << K);   // (every lane routes: the appends are per wave)
  const uint32_t c = in ? hist[g] : 0u;
  const uint32_t key = (uint32_t)(g & ((1ll << K) - 1));
  Seg s;
  s.tree = (int32_t)(g >> K);
  s.start = in ? (int32_t)off[g] : 0;
  s.count = (int32_t)c;
  s.buf = 0;
  s.pad[0] = s.pad[1] = s.pad[2] = 0;
  for (int j = 0; j < KP; ++j) {
    s.depth[j] = (j < K) ? 1 : (uint8_t)bits;
    s.prefix[j] = (j < K) ? (uint8_t)((key >> (K - 1 - j)) & 1) : 0;
  }
  route(s, K, bits, max_leaf, n, lo, li, in && c > 0);
}

// ---- global passes over nodes larger than LDS_SEG_CAP (contiguous rows, no gathers)
// The units of every listed node, in no particular order.
__global__ __launch_bounds__(256) void seg_units(const Seg* segs, int nseg, Unit* units,
                                                 uint32_t* n_units) {
  __shared__ uint32_t sh[256 / 64 + 1];
  __shared__ uint32_t base;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const uint32_t m = (i < nseg) ? (uint32_t)((segs[i].count + SEG_CHUNK - 1) / SEG_CHUNK) : 0u;
  uint32_t tot;
  const uint32_t ex = block_excl_scan<256>(m, sh, &tot);
  if (threadIdx.x == 0) base = atomicAdd(n_units, tot);
  __syncthreads();
  for (uint32_t t = 0; t < m; ++t) units[base + ex + t] = Unit{(uint32_t)i, t * (uint32_t)SEG_CHUNK};
}

__global__ __launch_bounds__(256) void seg_count(const Seg* segs, const Unit* units,
                                                 const uint32_t* n_units, Bufs b, int64_t n,
                                                 int K, int bits, uint32_t* cnt) {
  if (blockIdx.x >= *n_units) return;
  const Unit u = units[blockIdx.x];
  const Seg s = segs[u.seg];
  uint32_t local[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) local[j] = 0;
  const uint4* rows = b.rows[s.buf] + (int64_t)s.tree * n + s.start;
  const int end = min(s.count, (int)u.first + SEG_CHUNK);
  for (int p = (int)u.first + threadIdx.x; p < end; p += 256) {
    const uint4 v = rows[p];
#pragma unroll
    for (int j = 0; j < KP; ++j)
      if (j < K && s.depth[j] < bits) local[j] += (code_byte(v, j) >> (bits - 1 - s.depth[j])) & 1;
  }
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const uint32_t v = wave_sum(local[j]);
    if ((threadIdx.x & 63) == 0 && v && j < K) atomicAdd(&cnt[(int64_t)u.seg * KP + j], v);
  }
}

// The most balanced dimension of each node (ties to the smallest), the size of its bit-0
// child, the children's write cursors, and whether each child is a leaf (bit 0 / bit 1).
__global__ void seg_choose(const Seg* segs, int nseg, const uint32_t* cnt, int K, int bits,
                           int max_leaf, int32_t* split, uint32_t* c0, uint32_t* cur0,
                           uint32_t* cur1, uint8_t* leafs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nseg) return;
  const Seg s = segs[i];
  int best = -1;
  int64_t best_score = 0;
  for (int j = 0; j < K; ++j) {
    if (s.depth[j] >= bits) continue;
    const int64_t sc = llabs(2 * (int64_t)cnt[(int64_t)i * KP + j] - s.count);
    if (best < 0 || sc < best_score) { best = j; best_score = sc; }
  }
  // a node routed here is never fully refined, so best >= 0
  split[i] = best;
  // (a count never exceeds the node's size; the bound keeps the cursors inside the node
  // whatever the counts hold)
  const uint32_t z = (uint32_t)s.count - min(cnt[(int64_t)i * KP + best], (uint32_t)s.count);
  c0[i] = z;
  cur0[i] = (uint32_t)s.start;
  cur1[i] = (uint32_t)s.start + z;
  uint8_t d[KP];
  for (int j = 0; j < KP; ++j) d[j] = s.depth[j];
  d[best] = (uint8_t)(d[best] + 1);
  const bool full = fully_refined(d, K, bits);
  const uint32_t z1 = (uint32_t)s.count - z;
  leafs[i] = (uint8_t)(((z <= (uint32_t)max_leaf || full) ? 1 : 0) |
                       ((z1 <= (uint32_t)max_leaf || full) ? 2 : 0));
}

// Partition of each node's rows and ids into the other buffer, bit-0 child first. A
// child that is a leaf needs no rows any more: only its ids are written. A child that
// stays above LDS_SEG_CAP points gets its next-bit counts here (cntn[node][bit][dim]), so
// the next level needs no counting pass: a thread sums its rows' masked bits as byte
// counters (16 rows per unit and thread), each wave adds them up as 16-bit fields.
__global__ __launch_bounds__(256) void seg_split(const Seg* segs, const Unit* units,
                                                 const uint32_t* n_units, const int32_t* split,
                                                 const uint8_t* leafs, const uint32_t* c0,
                                                 Bufs b, int64_t n, int K, int bits,
                                                 uint32_t* cur0, uint32_t* cur1,
                                                 uint32_t* cntn) {
  static_assert(SEG_CHUNK / 256 <= 255, "byte counters");
  if (blockIdx.x >= *n_units) return;
  const Unit u = units[blockIdx.x];
  const Seg s = segs[u.seg];
  const int j = split[u.seg];
  const int sh = bits - 1 - s.depth[j];
  const uint8_t lf = leafs[u.seg];
  const uint32_t z = c0[u.seg];
  const bool need0 = !(lf & 1) && z > (uint32_t)LDS_SEG_CAP;
  const bool need1 = !(lf & 2) && (uint32_t)s.count - z > (uint32_t)LDS_SEG_CAP;
  // the children's next unrefined bit of every dimension (dimension j one deeper)
  uint32_t M[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int jj = 0; jj < KP; ++jj) {
    const int cd = s.depth[jj] + (jj == j ? 1 : 0);
    if (jj < K && cd < bits) M[jj >> 2] |= 1u << (8 * (jj & 3) + bits - 1 - cd);
  }
  // the split bit of a code row (one bit set)
  const uint32_t sbit = 1u << (8 * (j & 3) + sh);
  const uint4 SB = make_uint4((j >> 2) == 0 ? sbit : 0u, (j >> 2) == 1 ? sbit : 0u,
                              (j >> 2) == 2 ? sbit : 0u, (j >> 2) == 3 ? sbit : 0u);
  uint32_t acc0[4] = {0u, 0u, 0u, 0u}, acc1[4] = {0u, 0u, 0u, 0u};
  const int64_t tb = (int64_t)s.tree * n;
  const uint4* rs = b.rows[s.buf] + tb + s.start;
  const int32_t* is = b.ids[s.buf] + tb + s.start;
  uint4* rd = b.rows[1 - s.buf] + tb;
  int32_t* id_d = b.ids[1 - s.buf] + tb;
  const int end = min(s.count, (int)u.first + SEG_CHUNK);
  // SPLIT_G steps of 256 points at a time: their loads are all in flight together, and a
  // wave reserves its places in each child once per group
  constexpr int SPLIT_G = 8;
  for (int b0 = (int)u.first; b0 < end; b0 += 256 * SPLIT_G) {
    uint4 row[SPLIT_G];
    int32_t id[SPLIT_G];
    bool valid[SPLIT_G], bit[SPLIT_G];
#pragma unroll
    for (int i = 0; i < SPLIT_G; ++i) {
      const int p = b0 + i * 256 + (int)threadIdx.x;
      valid[i] = p < end;
      row[i] = valid[i] ? rs[p] : make_uint4(0, 0, 0, 0);
      id[i] = valid[i] ? is[p] : 0;
    }
    uint64_t mz[SPLIT_G], mo[SPLIT_G];
    uint32_t nz = 0, no = 0;
#pragma unroll
    for (int i = 0; i < SPLIT_G; ++i) {
      bit[i] = ((row[i].x & SB.x) | (row[i].y & SB.y) | (row[i].z & SB.z) | (row[i].w & SB.w)) != 0u;
      mz[i] = __ballot(valid[i] && !bit[i]);
      mo[i] = __ballot(valid[i] && bit[i]);
      nz += (uint32_t)__popcll(mz[i]);
      no += (uint32_t)__popcll(mo[i]);
    }
    uint32_t bz = 0, bo = 0;
    if ((threadIdx.x & 63) == 0) {
      if (nz) bz = atomicAdd(&cur0[u.seg], nz);
      if (no) bo = atomicAdd(&cur1[u.seg], no);
    }
    bz = uni(bz);   // lane 0 holds them
    bo = uni(bo);
#pragma unroll
    for (int i = 0; i < SPLIT_G; ++i) {
      if (valid[i]) {
        const int bt = bit[i] ? 1 : 0;
        const uint32_t pos = bt ? bo + lanes_below(mo[i]) : bz + lanes_below(mz[i]);
        id_d[pos] = id[i];
        if (!((lf >> bt) & 1)) rd[pos] = row[i];
        if (bt ? need1 : need0) {
          uint32_t* acc = bt ? acc1 : acc0;
          acc[0] += nonzero_bytes(row[i].x & M[0]);
          acc[1] += nonzero_bytes(row[i].y & M[1]);
          acc[2] += nonzero_bytes(row[i].z & M[2]);
          acc[3] += nonzero_bytes(row[i].w & M[3]);
        }
      }
      bz += (uint32_t)__popcll(mz[i]);
      bo += (uint32_t)__popcll(mo[i]);
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (!(c ? need1 : need0)) continue;
    const uint32_t* acc = c ? acc1 : acc0;
    // bytes 0 and 2 (even dimensions), bytes 1 and 3 (odd) as 16-bit fields
    uint32_t w[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      w[2 * i] = wave_sum(acc[i] & 0x00ff00ffu);
      w[2 * i + 1] = wave_sum((acc[i] >> 8) & 0x00ff00ffu);
    }
    if ((threadIdx.x & 63) == 0)
      for (int jj = 0; jj < K; ++jj) {
        const uint32_t v = (w[2 * (jj >> 2) + (jj & 1)] >> (16 * ((jj >> 1) & 1))) & 0xffffu;
        if (v) atomicAdd(&cntn[((int64_t)u.seg * 2 + c) * KP + jj], v);
      }
  }
}

__global__ void seg_children(const Seg* segs, int nseg, const int32_t* split, const uint32_t* c0,
                             const uint32_t* cntn, int K, int bits, int max_leaf, int64_t n,
                             LeafOut lo, Lists li) {
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i0 < nseg;   // (every lane routes: the appends are per wave)
  const int i = in ? i0 : 0;
  const Seg s = segs[i];
  const int j = split[i];
  Seg a = s, b = s;
  a.buf = b.buf = (uint8_t)(1 - s.buf);
  a.count = (int32_t)c0[i];
  b.start = s.start + a.count;
  b.count = s.count - a.count;
  // (every field written with a fixed index: a runtime index would put the copies in
  // scratch memory)
#pragma unroll
  for (int jj = 0; jj < KP; ++jj) {
    if (jj == j) {
      a.depth[jj] = b.depth[jj] = (uint8_t)(s.depth[jj] + 1);
      a.prefix[jj] = (uint8_t)(s.prefix[jj] * 2);
      b.prefix[jj] = (uint8_t)(s.prefix[jj] * 2 + 1);
    }
  }
  route(a, K, bits, max_leaf, n, lo, li, in, cntn + (int64_t)i * 2 * KP);
  route(b, K, bits, max_leaf, n, lo, li, in, cntn + ((int64_t)i * 2 + 1) * KP);
}

// Ids of leaves whose data sits in buffer 1 go to the permutation (buffer 0).
__global__ void seg_copy(const Copy* cp, Bufs b, int64_t n) {
  const Copy c = cp[blockIdx.x];
  const int64_t base = (int64_t)c.tree * n + c.start;
  for (int t = threadIdx.x; t < c.count; t += blockDim.x) b.ids[0][base + t] = b.ids[1][base + t];
}

// ---- one workgroup finishes a node of at most LDS_SEG_CAP points in LDS

// Frontier form: every open node of a level is split at once. Open nodes hold more than
// max_leaf points each, so a workgroup of capacity CAP tracks at most CAP / (max_leaf + 1)
// of them; the host takes this form (with MAXS of 16 or 64, the smaller LDS footprint when it
// suffices) when that is at most 64.
constexpr int FR_MAXS = 64;

struct SegL {
  int16_t start, count;       // range within the workgroup's node
  uint8_t depth[KP];
  uint8_t prefix[KP];
};

// Instantiated per size class (count in (below, CAP], NT threads): LDS and threads scale
// with the node, so small nodes run many workgroups per CU. Blocks whose node is outside
// the class return at once.
//
// A level: each thread finds the open node of each of its PER consecutive positions and
// reads their rows once (kept in registers through the level); 1. next-bit counts per open
// node and dimension; 2. split dimension per node; 3. stable partition of every node by its
// split bit (a workgroup scan of the bit-0 flags); 4. children, open ones listed for the next
// level. The position order lives in one of two LDS arrays, the partition writing the other.
// Six waves per SIMD for the classes whose LDS allows them (three workgroups of the largest
// class share a CU); the others are limited by LDS first.
constexpr int frontier_waves(int cap, int maxs) {
  return (cap >= 512 && (maxs == 16 || cap == 2048)) ? 6 : 1;
}

template <int CAP, int NT, int MAXS>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(frontier_waves(CAP, MAXS))))
void seg_lds_frontier(
    const Seg* mid, Bufs b, int64_t n, int K, int bits, int max_leaf, int below, LeafOut lo) {
  constexpr int PER = CAP / NT;           // consecutive positions per thread in the scan
  static_assert(PER * NT == CAP && PER <= 32 && MAXS <= NT, "class shape");
  __shared__ uint4 rows[CAP];
  __shared__ uint16_t ordb[2][CAP];
  __shared__ __align__(16) SegL segs[2][MAXS];   // (depth bytes read as words)
  __shared__ uint4 smask[MAXS];
  __shared__ uint32_t cnt[MAXS][KP];
  __shared__ uint32_t zstart[MAXS];
  __shared__ uint16_t c0s[MAXS];
  __shared__ uint8_t jsel[MAXS];
  __shared__ uint4 bmask[MAXS];   // the split bit of a node's code rows (one bit set)
  __shared__ uint32_t sh_scan[NT / 64 + 1];
  __shared__ uint32_t s_nact;

  const Seg s = mid[blockIdx.x];
  if (s.count <= below || s.count > CAP) return;
  const int count = s.count;
  const int64_t tb = (int64_t)s.tree * n;
  const uint4* rsrc = b.rows[s.buf] + tb + s.start;
  const int32_t* isrc = b.ids[s.buf] + tb + s.start;
  for (int t = threadIdx.x; t < count; t += NT) {
    rows[t] = rsrc[t];
    ordb[0][t] = (uint16_t)t;
  }
  if (threadIdx.x == 0) {
    SegL r;
    r.start = 0;
    r.count = (int16_t)count;
    for (int j = 0; j < KP; ++j) { r.depth[j] = s.depth[j]; r.prefix[j] = s.prefix[j]; }
    segs[0][0] = r;
    s_nact = 1;   // routed here: more than max_leaf points and not fully refined
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int p0 = threadIdx.x * PER;
  int cur = 0, co = 0;   // node list and position order of this level
  for (;;) {
    const int nact = (int)uni(s_nact);
    if (nact == 0) break;
    const SegL* S = segs[cur];
    // thread i < nact handles open node i: its depth bytes stay in registers for the level
    uint32_t dw[4] = {0u, 0u, 0u, 0u};
    auto dep = [&](int j) { return (dw[j >> 2] >> (8 * (j & 3))) & 255u; };   // j constant
    if ((int)threadIdx.x < nact) {
      const uint32_t* gd = reinterpret_cast<const uint32_t*>(S[threadIdx.x].depth);
#pragma unroll
      for (int q = 0; q < 4; ++q) dw[q] = gd[q];
      uint32_t m[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int j = 0; j < KP; ++j)
        if (j < K && dep(j) < (uint32_t)bits) m[j >> 2] |= 1u << (8 * (j & 3) + bits - 1 - dep(j));
      smask[threadIdx.x] = make_uint4(m[0], m[1], m[2], m[3]);
#pragma unroll
      for (int j = 0; j < KP; ++j) cnt[threadIdx.x][j] = 0;
    }
    // the open node of each of the thread's positions (-1: none): the node holding p0 by
    // binary search over the sorted starts, then the boundaries met in order
    int se[PER];
    {
      int lo2 = 0, hi2 = nact;   // first node starting after p0
      while (lo2 < hi2) {
        const int md = (lo2 + hi2) >> 1;
        if (S[md].start <= p0) lo2 = md + 1; else hi2 = md;
      }
      int snext = lo2, sg = lo2 - 1;   // sg: last node starting at or before p0
      int send = (sg >= 0) ? S[sg].start + S[sg].count : 0;
      int nstart = (snext < nact) ? S[snext].start : CAP;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int p = p0 + e;
        if (p == nstart) {
          sg = snext++;
          send = S[sg].start + S[sg].count;
          nstart = (snext < nact) ? S[snext].start : CAP;
        }
        se[e] = (sg >= 0 && p < send && p < count) ? sg : -1;
      }
    }
    // the thread's rows, all read before any is used, and their current order entries
    int oi[PER];
    uint4 rv[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      oi[e] = ordb[co][p0 + e];
      rv[e] = rows[se[e] >= 0 ? oi[e] : 0];
    }
    __syncthreads();   // masks and zeroed counts visible
    // 1. next-bit counts per open node and dimension. Byte j of a code row is dimension
    //    j's code; a node's mask keeps the next unrefined bit of each of its dimensions, so
    //    a masked row has at most one bit per byte. A thread sums its positions as byte
    //    counters, one per dimension; each wave then adds up the counters of its lanes in
    //    one node (as 16-bit fields) and adds them to the node's counts.
    {
      uint32_t acc[4] = {0u, 0u, 0u, 0u};
      uint4 M = make_uint4(0u, 0u, 0u, 0u);
      int run = -1;   // node whose counts acc holds
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int g = se[e];
        if (g != run) {
          // a node boundary inside the thread's positions: the finished run's counts go
          // to its node directly
          if (run >= 0) {
#pragma unroll
            for (int j = 0; j < KP; ++j) {
              const uint32_t c = (acc[j >> 2] >> (8 * (j & 3))) & 255u;
              if (j < K && c) atomicAdd(&cnt[run][j], c);
            }
          }
          acc[0] = acc[1] = acc[2] = acc[3] = 0u;
          run = g;
          if (g >= 0) M = smask[g];
        }
        if (g >= 0) {
          acc[0] += nonzero_bytes(rv[e].x & M.x);
          acc[1] += nonzero_bytes(rv[e].y & M.y);
          acc[2] += nonzero_bytes(rv[e].z & M.z);
          acc[3] += nonzero_bytes(rv[e].w & M.w);
        }
      }
      uint64_t pending = __ballot(run >= 0);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int s0 = __builtin_amdgcn_readlane(run, leader);
        const bool mine = run == s0;
        // bytes 0 and 2 (even dimensions), bytes 1 and 3 (odd) as 16-bit fields, summed
        // over the wave (uniform results)
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          w[2 * i] = wave_total(mine ? (acc[i] & 0x00ff00ffu) : 0u);
          w[2 * i + 1] = wave_total(mine ? ((acc[i] >> 8) & 0x00ff00ffu) : 0u);
        }
        if (lane < K) {
          const int wi = 2 * (lane >> 2) + (lane & 1);
          uint32_t ww = w[0];
#pragma unroll
          for (int i = 1; i < 8; ++i) ww = (wi == i) ? w[i] : ww;
          const uint32_t c = (ww >> (16 * ((lane >> 1) & 1))) & 0xffffu;
          if (c) atomicAdd(&cnt[s0][lane], c);
        }
        pending &= ~__ballot(mine);
      }
    }
    __syncthreads();
    // 2. split dimension of every open node: the most balanced one, ties to the smallest
    if ((int)threadIdx.x < nact) {
      const SegL& g = S[threadIdx.x];
      int best = -1, best_score = 0, best_cnt = 0;
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        const int dj = (int)dep(j);
        const int cj = (int)cnt[threadIdx.x][j];
        const int sc = abs(2 * cj - g.count);
        if (j < K && dj < bits && (best < 0 || sc < best_score)) {
          best = j; best_score = sc; best_cnt = cj;
        }
      }
      jsel[threadIdx.x] = (uint8_t)best;
      const int bj = max(best, 0);
      const uint32_t wsel = (bj >> 2) == 0 ? dw[0] : (bj >> 2) == 1 ? dw[1] : (bj >> 2) == 2 ? dw[2] : dw[3];
      const uint32_t bit = 1u << (8 * (bj & 3) + bits - 1 - ((wsel >> (8 * (bj & 3))) & 255u));
      bmask[threadIdx.x] = make_uint4((bj >> 2) == 0 ? bit : 0u, (bj >> 2) == 1 ? bit : 0u,
                                      (bj >> 2) == 2 ? bit : 0u, (bj >> 2) == 3 ? bit : 0u);
      c0s[threadIdx.x] = (uint16_t)(g.count - best_cnt);
    }
    __syncthreads();
    // 3. stable partition of every open node: a workgroup-wide scan of the bit-0 flags
    //    over consecutive position runs gives each point its rank among its node's zeros
    uint32_t zmask = 0;
    {
      int jg = -1;
      uint4 B = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int g = se[e];
        if (g >= 0 && g != jg) { jg = g; B = bmask[g]; }
        const bool one = ((rv[e].x & B.x) | (rv[e].y & B.y) | (rv[e].z & B.z) | (rv[e].w & B.w)) != 0u;
        if (g >= 0 && !one) zmask |= 1u << e;
      }
    }
    uint32_t ztot;
    const uint32_t zbase = block_excl_scan<NT>((uint32_t)__popc(zmask), sh_scan, &ztot);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int g = se[e];
      if (g >= 0 && p0 + e == S[g].start)
        zstart[g] = zbase + (uint32_t)__popc(zmask & ((1u << e) - 1u));
    }
    __syncthreads();
    {
      int gs = -1, gstart = 0, gc0 = 0;
      uint32_t gz = 0;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int p = p0 + e;
        if (p >= count) continue;
        const int g = se[e];
        if (g < 0) { ordb[co ^ 1][p] = (uint16_t)oi[e]; continue; }
        if (g != gs) { gs = g; gstart = S[g].start; gc0 = c0s[g]; gz = zstart[g]; }
        const uint32_t zb = zbase + (uint32_t)__popc(zmask & ((1u << e) - 1u)) - gz;
        const int off = p - gstart;
        const int np = ((zmask >> e) & 1u) ? gstart + (int)zb : gstart + gc0 + (off - (int)zb);
        ordb[co ^ 1][np] = (uint16_t)oi[e];
      }
    }
    // 4. children: leaves are emitted, open ones form the next level's list (in position
    //    order: children of a node are adjacent, bit 0 first)
    //    The children are read and written field by field from the parent in LDS: a
    //    private copy indexed by the runtime split dimension would live in scratch memory.
    uint32_t nopen = 0;
    bool oa = false, ob = false;
    int za = 0, zb = 0, jc = 0;
    if ((int)threadIdx.x < nact) {
      const SegL& g = S[threadIdx.x];
      jc = jsel[threadIdx.x];
      za = c0s[threadIdx.x];
      zb = g.count - za;
      bool full = true;   // every dimension fully refined after the split
#pragma unroll
      for (int jj = 0; jj < KP; ++jj)
        full = full && (jj >= K || (int)dep(jj) + (jj == jc ? 1 : 0) >= bits);
      oa = za > max_leaf && !full;
      ob = zb > max_leaf && !full;
      if (!oa && za > 0)
        emit_child_leaf(lo, n, s.tree, (int64_t)s.start + g.start, za, g.depth, g.prefix, jc, 0,
                        K);
      if (!ob && zb > 0)
        emit_child_leaf(lo, n, s.tree, (int64_t)s.start + g.start + za, zb, g.depth, g.prefix,
                        jc, 1, K);
      nopen = (oa ? 1u : 0u) + (ob ? 1u : 0u);
    }
    uint32_t total;
    const uint32_t at = block_excl_scan<NT>(nopen, sh_scan, &total);
    if ((int)threadIdx.x < nact) {
      const SegL& g = S[threadIdx.x];
      SegL* Nx = segs[cur ^ 1];
      uint32_t w = at;
      for (int bit = 0; bit < 2; ++bit) {
        if (!(bit ? ob : oa)) continue;
        SegL& c = Nx[w++];
        c.start = (int16_t)(g.start + (bit ? za : 0));
        c.count = (int16_t)(bit ? zb : za);
        for (int jj = 0; jj < KP; ++jj) {
          c.depth[jj] = (uint8_t)(g.depth[jj] + (jj == jc ? 1 : 0));
          c.prefix[jj] = (uint8_t)(jj == jc ? g.prefix[jj] * 2 + bit : g.prefix[jj]);
        }
      }
    }
    if (threadIdx.x == 0) s_nact = total;
    __syncthreads();
    cur ^= 1;
    co ^= 1;
  }
  // the ids in leaf order: every read (the node's ids may sit in the output array) before
  // any write; an order entry is below count (clamped all the same, so that the reads stay
  // inside the node)
  int32_t outv[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int t = threadIdx.x + e * NT;
    outv[e] = (t < count) ? isrc[min((int)ordb[co][t], count - 1)] : 0;
  }
  __syncthreads();
  int32_t* out = b.ids[0] + tb + s.start;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int t = threadIdx.x + e * NT;
    if (t < count) out[t] = outv[e];
  }
}

// Depth-first form for small max_leaf (more open nodes than the frontier form tracks):
// one node split at a time, with an explicit stack.
constexpr int STACK_MAX = KP * 8 + 8;

struct Node {
  int16_t lstart, lcount;
  uint8_t depth[KP];
  uint8_t prefix[KP];
};

template <int CAP, int NT>
__global__ __launch_bounds__(NT) void seg_lds_dfs(const Seg* mid, Bufs b, int64_t n, int K,
                                                  int bits, int max_leaf, int below,
                                                  LeafOut lo) {
  __shared__ int32_t ids[CAP];
  __shared__ uint4 rows[CAP];
  __shared__ uint16_t idx[CAP];
  __shared__ uint16_t tmp[CAP];
  __shared__ Node stack[STACK_MAX];
  __shared__ Node cur;
  __shared__ int sp;
  __shared__ int state;          // 0 done, 2 split
  __shared__ uint32_t cnt[KP];
  __shared__ uint32_t cz, co;
  __shared__ int jsplit;

  const Seg s = mid[blockIdx.x];
  if (s.count <= below || s.count > CAP) return;
  const int64_t tb = (int64_t)s.tree * n;
  const uint4* rsrc = b.rows[s.buf] + tb + s.start;
  const int32_t* isrc = b.ids[s.buf] + tb + s.start;
  for (int t = threadIdx.x; t < s.count; t += blockDim.x) {
    ids[t] = isrc[t];
    rows[t] = rsrc[t];
    idx[t] = (uint16_t)t;
  }
  if (threadIdx.x == 0) {
    Node r;
    r.lstart = 0;
    r.lcount = (int16_t)s.count;
    for (int j = 0; j < KP; ++j) { r.depth[j] = s.depth[j]; r.prefix[j] = s.prefix[j]; }
    stack[0] = r;
    sp = 1;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (;;) {
    if (threadIdx.x == 0) {
      // pop until a node to split (state 2) or an empty stack (state 0); leaves met on the
      // way are emitted here
      state = 0;
      while (sp > 0) {
        cur = stack[--sp];
        if (cur.lcount <= max_leaf || fully_refined(cur.depth, K, bits)) {
          emit_leaf(lo, n, s.tree, (int64_t)s.start + cur.lstart, cur.lcount, cur.depth,
                    cur.prefix, K);
          continue;
        }
        state = 2;
        break;
      }
    }
    if (threadIdx.x < KP) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int st = state;
    __syncthreads();            // every thread has read `state` before thread 0 pops again
    if (st == 0) break;

    uint32_t local[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) local[j] = 0;
    for (int t = threadIdx.x; t < cur.lcount; t += blockDim.x) {
      const uint4 v = rows[idx[cur.lstart + t]];
#pragma unroll
      for (int j = 0; j < KP; ++j)
        if (j < K && cur.depth[j] < bits) local[j] += (code_byte(v, j) >> (bits - 1 - cur.depth[j])) & 1;
    }
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const uint32_t v = wave_sum(local[j]);
      if (lane == 0 && v && j < K) atomicAdd(&cnt[j], v);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int best = -1;
      int best_score = 0;
      for (int j = 0; j < K; ++j) {
        if (cur.depth[j] >= bits) continue;
        const int sc = abs(2 * (int)cnt[j] - cur.lcount);
        if (best < 0 || sc < best_score) { best = j; best_score = sc; }
      }
      const int c0 = cur.lcount - (int)cnt[best];
      Node a = cur, bn = cur;
      a.lcount = (int16_t)c0;
      bn.lstart = (int16_t)(cur.lstart + c0);
      bn.lcount = (int16_t)(cur.lcount - c0);
      a.depth[best] = bn.depth[best] = cur.depth[best] + 1;
      a.prefix[best] = (uint8_t)(cur.prefix[best] * 2);
      bn.prefix[best] = (uint8_t)(cur.prefix[best] * 2 + 1);
      if (bn.lcount > 0) stack[sp++] = bn;     // popped after the bit-0 child
      if (a.lcount > 0) stack[sp++] = a;
      jsplit = best;
      cz = (uint32_t)cur.lstart;
      co = (uint32_t)(cur.lstart + c0);
    }
    __syncthreads();
    const int j = jsplit;
    const int sh = bits - 1 - cur.depth[j];
    for (int b0 = 0; b0 < cur.lcount; b0 += blockDim.x) {
      const int t = b0 + threadIdx.x;
      const bool valid = t < cur.lcount;
      uint16_t e = 0;
      int bit = 0;
      if (valid) {
        e = idx[cur.lstart + t];
        bit = (code_byte(rows[e], j) >> sh) & 1;
      }
      const uint64_t mz = __ballot(valid && bit == 0);
      const uint64_t mo = __ballot(valid && bit == 1);
      uint32_t bz = 0, bo = 0;
      if (lane == 0) {
        if (mz) bz = atomicAdd(&cz, (uint32_t)__popcll(mz));
        if (mo) bo = atomicAdd(&co, (uint32_t)__popcll(mo));
      }
      bz = __shfl(bz, 0);
      bo = __shfl(bo, 0);
      if (valid) tmp[bit ? bo + lanes_below(mo) : bz + lanes_below(mz)] = e;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cur.lcount; t += blockDim.x) idx[cur.lstart + t] = tmp[cur.lstart + t];
    __syncthreads();
  }
  __syncthreads();
  int32_t* out = b.ids[0] + tb + s.start;
  for (int t = threadIdx.x; t < s.count; t += blockDim.x) out[t] = ids[idx[t]];
}

// ---- leaf tables
struct LeafTables {
  int32_t* start[PDET_MAX_L];
  int32_t* count[PDET_MAX_L];
  uint16_t* hidx[PDET_MAX_L];
  float* box[PDET_MAX_L];
  int64_t nl[PDET_MAX_L];
};

// Leaf tables in two steps: every recorded start position goes to its leaf's slot (one
// sparse write per leaf), then one thread per leaf fills the rest (all lanes busy).
// 4 consecutive positions per thread (16-byte loads when the row allows).
__global__ void leaf_starts(const uint32_t* cnt_at, const uint32_t* ord, int64_t n,
                            LeafTables t) {
  const int64_t p0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const int tree = blockIdx.y;
  if (p0 >= n) return;
  const int64_t g0 = (int64_t)tree * n + p0;
  uint32_t c[4], o[4];
  if ((n & 3) == 0) {   // rows start 16-byte aligned and hold whole groups of 4
    const uint4 cw = *reinterpret_cast<const uint4*>(cnt_at + g0);
    const uint4 ow = *reinterpret_cast<const uint4*>(ord + g0);
    c[0] = cw.x; c[1] = cw.y; c[2] = cw.z; c[3] = cw.w;
    o[0] = ow.x; o[1] = ow.y; o[2] = ow.z; o[3] = ow.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      c[e] = p0 + e < n ? cnt_at[g0 + e] : 0u;
      o[e] = p0 + e < n ? ord[g0 + e] : 0u;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (c[e]) t.start[tree][o[e]] = (int32_t)(p0 + e);
}

__global__ void leaf_fill(const uint32_t* cnt_at, const uint16_t* hidx_at, int64_t n, int K,
                          int bits, int Nr, const float* B, LeafTables t) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int tree = blockIdx.y;
  const int64_t nl = t.nl[tree];
  if (o >= nl) return;
  const int64_t g = (int64_t)tree * n + t.start[tree][o];
  t.count[tree][o] = (int32_t)cnt_at[g];
  const uint4* hs = reinterpret_cast<const uint4*>(hidx_at + g * KP);
  const uint4 h0 = hs[0], h1 = hs[1];
  uint4* hd = reinterpret_cast<uint4*>(t.hidx[tree] + o * KP);
  hd[0] = h0;
  hd[1] = h1;
  const uint32_t hw[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    if (j < K) {
      const int h = (int)((hw[j >> 1] >> (16 * (j & 1))) & 0xffffu);
      const int dep = 31 - __clz(h);
      const int pre = h & ((1 << dep) - 1);
      const int lo_code = pre << (bits - dep);
      const int hi_code = ((pre + 1) << (bits - dep)) - 1;
      const float* Bc = B + (int64_t)(tree * K + j) * (Nr + 1);
      t.box[tree][(int64_t)j * nl + o] = Bc[lo_code];
      t.box[tree][(int64_t)(K + j) * nl + o] = Bc[hi_code + 1];
    }
  }
}

// Leaf ordinal of every point: position p lies in the leaf that starts at the last
// recorded start <= p, whose ordinal is the exclusive start count at p, plus one if p
// itself starts a leaf, minus one.
// Per-point leaf ordinals, tree-major: leaf_soa[tree][id]. One launch covers the points whose
// id lies in window `win` of 2^LEAF_WIN ids, so its writes stay within 4 * 2^LEAF_WIN bytes of
// each tree's array (small enough for the last-level cache to gather the 4-byte writes into
// whole lines); every window's launch reads the permutation in full, the rest only for its ids.
constexpr int LEAF_WIN = 25;

__global__ void leaf_of_kernel(const uint32_t* cnt_at, const uint32_t* ord, const int32_t* perm,
                               int64_t n, int win, int32_t* leaf_soa) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int tree = blockIdx.y;
  if (p >= n) return;
  const int64_t g = (int64_t)tree * n + p;
  const int32_t id = perm[g];
  if ((id >> LEAF_WIN) != win) return;
  leaf_soa[(int64_t)tree * n + id] = (int32_t)ord[g] + (cnt_at[g] ? 1 : 0) - 1;
}

// leaf_of[id][tree] from the tree-major form: coalesced reads of every tree's array, one
// row of L ordinals written per point.
__global__ void leaf_rows_by_id(const int32_t* leaf_soa, int64_t n, int L, int32_t* leaf_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (L == 4) {
    const int4 v = make_int4(leaf_soa[i], leaf_soa[n + i], leaf_soa[2 * n + i],
                             leaf_soa[3 * n + i]);
    *reinterpret_cast<int4*>(leaf_of + i * 4) = v;
    return;
  }
  for (int t = 0; t < L; ++t) leaf_of[i * L + t] = leaf_soa[(int64_t)t * n + i];
}

// leafrow[i][p] = leaf_of[perm_i[p]]: the leaf ordinals of a point in every tree, stored in
// the order the query walks tree i's leaves, so the dedupe test reads them contiguously.
__global__ void leafrow_kernel(const int32_t* perm, const int32_t* leaf_of, int64_t n, int L,
                               int32_t* leafrow) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int tree = blockIdx.y;
  if (p >= n) return;
  const int32_t* src = leaf_of + (int64_t)perm[(int64_t)tree * n + p] * L;
  int32_t* dst = leafrow + ((int64_t)tree * n + p) * L;
  if (L == 4) {   // one 16-byte row
    *reinterpret_cast<int4*>(dst) = *reinterpret_cast<const int4*>(src);
    return;
  }
  for (int j = 0; j < L; ++j) dst[j] = src[j];
}

// Union box of each group of 16 consecutive leaves (depth-first neighbours share most
// of their code prefixes, so the union stays tight). One thread per leaf (coalesced reads of
// the box table); the 16 lanes of a group reduce with shuffles. All trees in one launch.
struct GroupArgs {
  const float* box[PDET_MAX_L];
  float* gbox[PDET_MAX_L];
  int64_t nl[PDET_MAX_L];
  int K;
};

__global__ __launch_bounds__(256) void group_boxes(GroupArgs a) {
  const int i = blockIdx.y;
  const int64_t nl = a.nl[i], ng = (nl + 15) / 16;
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ng * 16) return;   // whole groups: the 16 lanes of a group stay together
  const int64_t g = l >> 4;
  const float* box = a.box[i];
  float* gbox = a.gbox[i];
  for (int j = 0; j < a.K; ++j) {
    float lo = (l < nl) ? box[(int64_t)j * nl + l] : INFINITY;
    float hi = (l < nl) ? box[(int64_t)(a.K + j) * nl + l] : -INFINITY;
    for (int o = 8; o > 0; o >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, o, 16));
      hi = fmaxf(hi, __shfl_xor(hi, o, 16));
    }
    if ((l & 15) == 0) {
      gbox[(int64_t)j * ng + g] = lo;
      gbox[(int64_t)(a.K + j) * ng + g] = hi;
    }
  }
}

}  // namespace

// A small pinned host area per thread for counter readbacks (kept until the thread ends).
uint32_t* readback_words() {
  struct Words {
    uint32_t* p = nullptr;
    ~Words() { if (p) (void)hipHostFree(p); }
  };
  static thread_local Words w;
  if (!w.p) PDET_HIP(hipHostMalloc((void**)&w.p, 64 * sizeof(uint32_t), hipHostMallocDefault));
  return w.p;
}

// Three streams (default priority) and their fork / join events per thread and device, kept
// until the thread ends.
struct SideStreams {
  int dev = -1;
  hipStream_t st[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
  void clear() {
    for (auto& x : st) if (x) { (void)hipStreamDestroy(x); x = nullptr; }
    for (auto& e : join) if (e) { (void)hipEventDestroy(e); e = nullptr; }
    if (fork) { (void)hipEventDestroy(fork); fork = nullptr; }
  }
  ~SideStreams() { clear(); }
};
SideStreams& side_streams() {
  static thread_local SideStreams ss;
  int dev = 0;
  PDET_HIP(hipGetDevice(&dev));
  if (ss.dev != dev) {
    ss.clear();
    for (auto& x : ss.st) PDET_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    PDET_HIP(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
    for (auto& e : ss.join) PDET_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ss.dev = dev;
  }
  return ss;
}

void first_layer_sort(int L, int K, int64_t n, uint16_t* keys, const uint4* codes, uint4* rows0,
                      int32_t* ids0, uint4* rows1, int32_t* ids1, uint16_t* keys1,
                      uint32_t* start, uint32_t* end, PooledBuf& h8, PooledBuf& o8,
                      DevBuf& scan_tmp, hipStream_t s) {
  const int nblk = (int)cdiv(n, RK_TILE);
  h8.alloc((size_t)L * 256 * nblk * 4);
  o8.alloc((size_t)L * 256 * nblk * 4);
  const dim3 grid((unsigned)nblk, (unsigned)L);
  const bool two = K > 8;
  // sorted keys: back in `keys` after two passes, in keys1 after one (a pass never writes
  // the buffer it reads)
  uint16_t* kfin = two ? keys : keys1;
  hipLaunchKernelGGL(rk_hist<0>, grid, dim3(RK_THREADS), 0, s, keys, n, nblk, h8.as<uint32_t>());
  PDET_HIP(hipGetLastError());
  scan_rows(h8.as<uint32_t>(), o8.as<uint32_t>(), nullptr, L, (int64_t)256 * nblk, scan_tmp, s);
  // one pass (K <= 8): straight to the final buffers; two: through buffer 1
  hipLaunchKernelGGL((rk_scatter<0, true>), grid, dim3(RK_THREADS), 0, s, keys, codes, nullptr, n,
                     nblk, o8.as<uint32_t>(), keys1, two ? rows1 : rows0, two ? ids1 : ids0);
  PDET_HIP(hipGetLastError());
  if (two) {
    hipLaunchKernelGGL(rk_hist<8>, grid, dim3(RK_THREADS), 0, s, keys1, n, nblk,
                       h8.as<uint32_t>());
    PDET_HIP(hipGetLastError());
    scan_rows(h8.as<uint32_t>(), o8.as<uint32_t>(), nullptr, L, (int64_t)256 * nblk, scan_tmp, s);
    hipLaunchKernelGGL((rk_scatter<8, false>), grid, dim3(RK_THREADS), 0, s, keys1, rows1, ids1,
                       n, nblk, o8.as<uint32_t>(), keys, rows0, ids0);
    PDET_HIP(hipGetLastError());
  }
  FillList fz;
  fz.add(start, 0u, (size_t)L * ((size_t)1 << K) * 4);
  fz.add(end, 0u, (size_t)L * ((size_t)1 << K) * 4);
  fill_words(fz, s);
  hipLaunchKernelGGL(rk_bounds, dim3(cdiv(n, 256 * 8), L), dim3(256), 0, s, kfin, n, K, start,
                     end);
  PDET_HIP(hipGetLastError());
}

void build_trees(Index& ix, hipStream_t s) {
  const hipStream_t s_main = s;
  const int64_t n = ix.n;
  const int L = ix.L, K = ix.K, bits = ix.bits;
  const int64_t NK = 1ll << K;

  // allocated first, while the encoder still runs: its size does not depend on the trees
  ix.leafrow.alloc((size_t)L * n * L * 4);
  PooledBuf hist((size_t)L * NK * 4), off((size_t)L * NK * 4), cursor((size_t)L * NK * 4);
  DevBuf scan_tmp;
  DevBuf rows0((size_t)L * n * KP);   // code rows in permutation order (buffer 0)
  Bufs bf{};
  bf.rows[0] = rows0.as<uint4>();
  bf.ids[0] = ix.perm.as<int32_t>();

  // first layer: radix sort of the keys carrying code rows and ids, then the nodes' starts
  // and sizes from the runs of equal keys. The pass buffers double as the split phase's
  // second row / id buffers.
  DevBuf rows1((size_t)L * n * KP);
  PooledBuf ids1((size_t)L * n * 4), keys1((size_t)L * n * 2);
  bf.rows[1] = rows1.as<uint4>();
  bf.ids[1] = ids1.as<int32_t>();
  PooledBuf h8, o8;   // live until the final synchronisation, like every temporary here
  first_layer_sort(L, K, n, ix.flkey.as<uint16_t>(),
                   reinterpret_cast<const uint4*>(ix.codes.as<uint8_t>()), bf.rows[0], bf.ids[0],
                   bf.rows[1], bf.ids[1], keys1.as<uint16_t>(), off.as<uint32_t>(),
                   cursor.as<uint32_t>(), h8, o8, scan_tmp, s);
  hipLaunchKernelGGL(rk_counts, dim3(cdiv(L * NK, 256)), dim3(256), 0, s, off.as<uint32_t>(),
                     cursor.as<uint32_t>(), L * NK, hist.as<uint32_t>());
  PDET_HIP(hipGetLastError());

  // leaf records at start positions
  PooledBuf cnt_at((size_t)L * n * 4), hidx_at((size_t)L * n * KP * 2);
  PDET_HIP(hipMemsetAsync(cnt_at.ptr(), 0, cnt_at.bytes(), s));
  LeafOut lo{cnt_at.as<uint32_t>(), hidx_at.as<uint16_t>()};

  // node lists; counters: [0] n_big_a [1] pts_big_a [2] n_big_b [3] pts_big_b
  // [4..7] n_mid per size class [8] n_copies [9] n_units. A class-c node has more than
  // max(CLS_BELOW[c], max_leaf) points, which bounds its list.
  int64_t mid_off[NCLS + 1] = {0};
  for (int cl = 0; cl < NCLS; ++cl)
    mid_off[cl + 1] = mid_off[cl] +
                      (int64_t)L * (n / (std::max(CLS_BELOW[cl], ix.max_leaf) + 1) + 1);
  const int64_t big_cap = (int64_t)L * (n / (LDS_SEG_CAP + 1) + 1);
  PooledBuf mid((size_t)mid_off[NCLS] * sizeof(Seg));
  PooledBuf bigA((size_t)big_cap * sizeof(Seg)), bigB((size_t)big_cap * sizeof(Seg));
  PooledBuf copies((size_t)2 * big_cap * sizeof(Copy));
  PooledBuf ctr(16 * 4);
  {
    FillList fz;
    fz.add(ctr.ptr(), 0u, ctr.bytes());
    fill_words(fz, s);
  }
  uint32_t* c = ctr.as<uint32_t>();
  Lists li{bigA.as<Seg>(), c + 0, c + 1, {}, c + 4, copies.as<Copy>(), c + 8};
  for (int cl = 0; cl < NCLS; ++cl) li.mid[cl] = mid.as<Seg>() + mid_off[cl];
  hipLaunchKernelGGL(fl_segments, dim3(cdiv(L * NK, 256)), dim3(256), 0, s, hist.as<uint32_t>(),
                     off.as<uint32_t>(), L, K, bits, ix.max_leaf, n, lo, li);
  PDET_HIP(hipGetLastError());

  uint32_t* hc = readback_words();
  PDET_HIP(hipMemcpyAsync(hc, c, 16 * 4, hipMemcpyDeviceToHost, s));
  PDET_HIP(hipStreamSynchronize(s));
  uint32_t nbig = hc[0], ptsbig = hc[1];
  Seg* cur_big = bigA.as<Seg>();
  Seg* nxt_big = bigB.as<Seg>();
  int cur_slot = 0;   // counters of the current list at c[2*cur_slot]
  // next-bit counts of the current level's nodes (counted at the first level, carried from
  // the split pass after it), of the next level's, and of every node's children
  PooledBuf cntbuf, cntnext, cntn, split, c0, cur0, cur1, leafs, units;
  if (nbig) {
    units.alloc(((size_t)L * n / SEG_CHUNK + (size_t)big_cap) * sizeof(Unit));
    cntbuf.alloc((size_t)big_cap * KP * 4);
    cntnext.alloc((size_t)big_cap * KP * 4);
    cntn.alloc((size_t)big_cap * 2 * KP * 4);
    split.alloc((size_t)big_cap * 4); c0.alloc((size_t)big_cap * 4);
    cur0.alloc((size_t)big_cap * 4); cur1.alloc((size_t)big_cap * 4);
    leafs.alloc((size_t)big_cap);
  }
  uint32_t* cur_cnt = cntbuf.as<uint32_t>();
  uint32_t* nxt_cnt = cntnext.as<uint32_t>();
  for (int level = 0; nbig > 0; ++level) {
    const int nxt_slot = 1 - cur_slot;
    {
      FillList fz;
      if (level == 0) fz.add(cur_cnt, 0u, (size_t)nbig * KP * 4);
      fz.add(cntn.ptr(), 0u, (size_t)nbig * 2 * KP * 4);
      fz.add(c + 2 * nxt_slot, 0u, 8);
      fz.add(c + 8, 0u, 8);   // copies, units
      fill_words(fz, s);
    }
    // every node gives at most count / SEG_CHUNK + 1 units
    const unsigned nu = (unsigned)(ptsbig / SEG_CHUNK + nbig);
    hipLaunchKernelGGL(seg_units, dim3(cdiv(nbig, 256)), dim3(256), 0, s, cur_big, (int)nbig,
                       units.as<Unit>(), c + 9);
    PDET_HIP(hipGetLastError());
    if (level == 0) {
      hipLaunchKernelGGL(seg_count, dim3(nu), dim3(256), 0, s, cur_big, units.as<Unit>(), c + 9,
                         bf, n, K, bits, cur_cnt);
      PDET_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(seg_choose, dim3(cdiv(nbig, 64)), dim3(64), 0, s, cur_big, (int)nbig,
                       cur_cnt, K, bits, ix.max_leaf, split.as<int32_t>(),
                       c0.as<uint32_t>(), cur0.as<uint32_t>(), cur1.as<uint32_t>(),
                       leafs.as<uint8_t>());
    PDET_HIP(hipGetLastError());
    hipLaunchKernelGGL(seg_split, dim3(nu), dim3(256), 0, s, cur_big, units.as<Unit>(), c + 9,
                       split.as<int32_t>(), leafs.as<uint8_t>(), c0.as<uint32_t>(), bf, n, K,
                       bits, cur0.as<uint32_t>(), cur1.as<uint32_t>(), cntn.as<uint32_t>());
    PDET_HIP(hipGetLastError());
    Lists ln = li;
    ln.big_next = nxt_big;
    ln.n_big_next = c + 2 * nxt_slot;
    ln.pts_big_next = c + 2 * nxt_slot + 1;
    ln.cnt_next = nxt_cnt;
    hipLaunchKernelGGL(seg_children, dim3(cdiv(nbig, 64)), dim3(64), 0, s, cur_big, (int)nbig,
                       split.as<int32_t>(), c0.as<uint32_t>(), cntn.as<uint32_t>(), K, bits,
                       ix.max_leaf, n, lo, ln);
    PDET_HIP(hipGetLastError());
    PDET_HIP(hipMemcpyAsync(hc, c, 16 * 4, hipMemcpyDeviceToHost, s));
    PDET_HIP(hipStreamSynchronize(s));
    if (hc[8]) {
      hipLaunchKernelGGL(seg_copy, dim3(hc[8]), dim3(256), 0, s, copies.as<Copy>(), bf, n);
      PDET_HIP(hipGetLastError());
    }
    nbig = hc[2 * nxt_slot];
    ptsbig = hc[2 * nxt_slot + 1];
    std::swap(cur_big, nxt_big);
    std::swap(cur_cnt, nxt_cnt);
    cur_slot = nxt_slot;
  }
  {
    // one launch per size class, one node per block, in the frontier form when the class
    // holds at most FR_MAXS open nodes. The classes touch disjoint nodes: classes 0-2 run on
    // side streams beside class 3 on the build's stream, so that one class's tail overlaps
    // the others' work.
    SideStreams& ss = side_streams();
    PDET_HIP(hipEventRecord(ss.fork, s));
    for (int k = 0; k < 3; ++k) PDET_HIP(hipStreamWaitEvent(ss.st[k], ss.fork, 0));
    auto finish = [&](auto cap_c, auto nt_c, int cl) {
      constexpr int CAP = decltype(cap_c)::value, NT = decltype(nt_c)::value;
      static_assert(CAP <= LDS_SEG_CAP, "class");
      const uint32_t nm = hc[4 + cl];
      if (!nm) return;
      const hipStream_t s = cl < 3 ? ss.st[cl] : s_main;
      const Seg* list = mid.as<Seg>() + mid_off[cl];
      const int below = CLS_BELOW[cl];
      const int open_max = CAP / (ix.max_leaf + 1);
      if (open_max <= 16)
        hipLaunchKernelGGL((seg_lds_frontier<CAP, NT, 16>), dim3(nm), dim3(NT), 0, s, list, bf,
                           n, K, bits, ix.max_leaf, below, lo);
      else if (open_max <= FR_MAXS)
        hipLaunchKernelGGL((seg_lds_frontier<CAP, NT, FR_MAXS>), dim3(nm), dim3(NT), 0, s, list,
                           bf, n, K, bits, ix.max_leaf, below, lo);
      else
        hipLaunchKernelGGL((seg_lds_dfs<CAP, NT>), dim3(nm), dim3(NT), 0, s, list, bf, n, K,
                           bits, ix.max_leaf, below, lo);
      PDET_HIP(hipGetLastError());
    };
    finish(std::integral_constant<int, LDS_SEG_CAP>{}, std::integral_constant<int, 512>{}, 3);
    finish(std::integral_constant<int, 1024>{}, std::integral_constant<int, 256>{}, 2);
    finish(std::integral_constant<int, 512>{}, std::integral_constant<int, 128>{}, 1);
    finish(std::integral_constant<int, 256>{}, std::integral_constant<int, 64>{}, 0);
    for (int k = 0; k < 3; ++k) {
      PDET_HIP(hipEventRecord(ss.join[k], ss.st[k]));
      PDET_HIP(hipStreamWaitEvent(s, ss.join[k], 0));
    }
  }

  finish_trees(ix, cnt_at.as<uint32_t>(), hidx_at.as<uint16_t>(), scan_tmp, s);
  ix.flkey.release();
}

void finish_trees(Index& ix, const uint32_t* cnt_at, const uint16_t* hidx_at, DevBuf& scan_tmp,
                  hipStream_t s) {
  const int64_t n = ix.n;
  const int L = ix.L, K = ix.K, bits = ix.bits;
  // number the leaves in position (= depth-first) order
  PooledBuf flags((size_t)L * n * 4), totals((size_t)L * 4);
  scan_rows_nonzero(cnt_at, flags.as<uint32_t>(), totals.as<uint32_t>(), L, n, scan_tmp, s);
  std::vector<uint32_t> nl(L);
  // per-point leaf ordinals and the leaf-row table need only the scan: they run while the
  // host reads the leaf counts back (into pinned memory, so the copy does not wait for
  // them) and sizes the leaf tables
  uint32_t* hp = readback_words() + 32;   // apart from the level counters (words 0..7)
  PDET_HIP(hipMemcpyAsync(hp, totals.ptr(), L * 4, hipMemcpyDeviceToHost, s));
  hipEvent_t counts_ready;
  PDET_HIP(hipEventCreateWithFlags(&counts_ready, hipEventDisableTiming));
  PDET_HIP(hipEventRecord(counts_ready, s));
  PooledBuf leaf_of((size_t)n * L * 4), leaf_soa((size_t)n * L * 4);
  const int nwin = (int)((n + (int64_t(1) << LEAF_WIN) - 1) >> LEAF_WIN);
  for (int w = 0; w < nwin; ++w)
    hipLaunchKernelGGL(leaf_of_kernel, dim3(cdiv(n, 256), L), dim3(256), 0, s, cnt_at,
                       flags.as<uint32_t>(), ix.perm.as<int32_t>(), n, w, leaf_soa.as<int32_t>());
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(leaf_rows_by_id, dim3(cdiv(n, 256)), dim3(256), 0, s, leaf_soa.as<int32_t>(),
                     n, L, leaf_of.as<int32_t>());
  PDET_HIP(hipGetLastError());
  hipLaunchKernelGGL(leafrow_kernel, dim3(cdiv(n, 256), L), dim3(256), 0, s,
                     ix.perm.as<int32_t>(), leaf_of.as<int32_t>(), n, L, ix.leafrow.as<int32_t>());
  PDET_HIP(hipGetLastError());
  const hipError_t ce = hipEventSynchronize(counts_ready);
  (void)hipEventDestroy(counts_ready);
  PDET_HIP(ce);
  for (int i = 0; i < L; ++i) nl[i] = hp[i];
  LeafTables t{};
  ix.nl_max = 0;
  // every tree's leaf tables and group boxes in one allocation (256-byte aligned parts)
  auto part = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
  size_t arena = 0;
  for (int i = 0; i < L; ++i) {
    const size_t ng = (size_t)std::max<int64_t>((nl[i] + 15) / 16, 1);
    arena += part((size_t)nl[i] * 4) * 2 + part((size_t)nl[i] * KP * 2) +
             part((size_t)nl[i] * 2 * K * 4) + part(ng * 2 * K * 4);
  }
  // a whole number of MiB: the next index of this shape (whose leaf counts differ a little)
  // then gets the same block from the block cache
  ix.leaf_arena.alloc((arena + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1));
  char* cur = ix.leaf_arena.as<char>();
  auto take = [&](DevBuf& v, size_t b) { v.view(cur, b); cur += part(b); };
  for (int i = 0; i < L; ++i) {
    ix.nl[i] = nl[i];
    ix.nl_max = std::max<int64_t>(ix.nl_max, nl[i]);
    take(ix.leaf_start[i], (size_t)nl[i] * 4);
    take(ix.leaf_count[i], (size_t)nl[i] * 4);
    take(ix.leaf_hidx[i], (size_t)nl[i] * KP * 2);
    take(ix.box[i], (size_t)nl[i] * 2 * K * 4);
    take(ix.gbox[i], (size_t)std::max<int64_t>((nl[i] + 15) / 16, 1) * 2 * K * 4);
    t.start[i] = ix.leaf_start[i].as<int32_t>();
    t.count[i] = ix.leaf_count[i].as<int32_t>();
    t.hidx[i] = ix.leaf_hidx[i].as<uint16_t>();
    t.box[i] = ix.box[i].as<float>();
    t.nl[i] = nl[i];
  }
  hipLaunchKernelGGL(leaf_starts, dim3(cdiv(n, 256 * 4), L), dim3(256), 0, s, cnt_at,
                     flags.as<uint32_t>(), n, t);
  PDET_HIP(hipGetLastError());
  int64_t nl_max = 0;
  for (int i = 0; i < L; ++i) nl_max = std::max<int64_t>(nl_max, nl[i]);
  if (nl_max) {
    hipLaunchKernelGGL(leaf_fill, dim3(cdiv(nl_max, 256), L), dim3(256), 0, s,
                       cnt_at, hidx_at, n, K, bits, ix.Nr,
                       ix.B.as<float>(), t);
    PDET_HIP(hipGetLastError());
  }
  GroupArgs ga{};
  int64_t nl_pad = 0;
  for (int i = 0; i < L; ++i) {
    const int64_t ng = (nl[i] + 15) / 16;
    ga.box[i] = ix.box[i].as<float>();
    ga.gbox[i] = ix.gbox[i].as<float>();
    ga.nl[i] = nl[i];
    nl_pad = std::max<int64_t>(nl_pad, ng * 16);
  }
  ga.K = K;
  if (nl_pad) {
    hipLaunchKernelGGL(group_boxes, dim3(cdiv(nl_pad, 256), L), dim3(256), 0, s, ga);
    PDET_HIP(hipGetLastError());
  }
  PDET_HIP(hipStreamSynchronize(s));   // temporaries are freed on return
}

}  // namespace pdet
