// c^2-k-ANN query (Algorithm 5) with the optimised range query of Section 6.2.2
// (relaxed whole-leaf admission when the leaf's lower bound is within eps*r, and
// admission in ascending lower-bound order), batched on gfx950.
//
// Kernels:
//  q_setup  per query: radius ladder r_rho = r_min*c^rho, thresholds (eps*r_rho)^2
//           and c*r_rho, computed with the same double operations as the definition.
//  q_rho    batched over (leaf block, tree, query tiles): the first round whose threshold
//           admits each leaf (its squared lower bound to q' <= (eps r_rho)^2), for rounds
//           up to rcap. Groups of 16 consecutive leaves are tested first with their union
//           box (a lower bound of every member's bound, as a subtree prunes in the range
//           query). Only leaves admitted by round rcap are written, as (round, leaf)
//           entries of a per-query, per-tree list; later rounds are found by q_main if a
//           query ever reaches them. Two forms: one query tile per workgroup (q_rho_tile),
//           or runs of tiles per workgroup in two passes (q_rho_runs) when the chunk has
//           enough tiles and leaf blocks to fill the device that way.
//  q_main   one workgroup per query, one pass per round over the admitted leaves of all
//           trees (the list entries of that round): an admitted point is new iff none of
//           its leaves in the other trees was admitted earlier in the (round, tree) order
//           (closed form of the candidate union, read from leafrow and the admission
//           rounds of the leaves admitted so far, kept in an LDS hash, or in a dense table
//           in device memory past 512 leaves). When stop rule A can fire in a round,
//           exact new-point counts per leaf give the tree where |S| reaches T, and a
//           weighted select over that tree's (LB^2, leaf ordinal) keys gives the leaf;
//           trees before it are admitted whole. New points are verified by exact distance
//           and offered to a top-k list in LDS; stop rule B checks the k-th distance
//           against c*r after each round.
#include <type_traits>

#include "devutil.h"
#include "internal.h"

namespace pdet {
namespace {

constexpr int QM = 256;          // threads of q_main
constexpr int CBMIN = 384;       // least pending-candidate buffer beside the top-k list (>= QM)
constexpr int QT = 64;           // queries per q_rho block (group tests in sub-tiles of 16)
constexpr int QR_THREADS = 256;  // leaves per q_rho block (one per thread)
constexpr int NXCD = 8;          // accelerator dies; workgroup i runs on die i % NXCD
constexpr int NRHO = NRHO_TABLE; // threshold table length (255 rounds + sentinel)
constexpr int GL = 16;           // leaves per pruning group
constexpr int RCAP_MAX = 8;      // most rounds q_rho resolves (the index's rcap <= this)
constexpr int QR_TILES_MAX = 64; // query tiles one q_rho workgroup runs through
constexpr int QR_TARGET_WG = 32768;  // q_rho workgroups a chunk aims for
constexpr int RWIN = 3;          // rounds resolved per refinement step inside q_main
constexpr int GCH = 2048;        // groups per refinement chunk (LDS bitmap of GCH bits)
constexpr int TREE_SHIFT = 28;   // admitted-leaf entries pack (tree << 28) | leaf
constexpr int LEAF_BITS = 24;    // leaf-list entries pack (round << 24) | leaf
constexpr int HSZ = 1024;        // LDS hash of (tree, leaf) -> round for the dedupe test
constexpr int HMAX = HSZ / 2;    // most entries it takes; beyond, a dense table in HBM
constexpr uint32_t HEMPTY = 0xffffffffu;
constexpr uint32_t NO_CUT = 0xffffffffu;
constexpr int WALK_VERIFY = 0, WALK_COUNT = 1, WALK_CUT = 2;
constexpr int STOP_OVERFLOW = 3; // query-stat stop code: leaf lists overflowed (answered again)
constexpr float BAND_REL = 1e-5f; // near-tie band: |LB^2 - (eps r)^2| <= BAND_REL (eps r)^2, and
                                 // the k-th squared distance within 2 BAND_REL of (c r)^2
constexpr double LOWP_SLACK_BF16 = 0.125;  // relative distance slack of the low-precision
constexpr double LOWP_SLACK_FP8 = 0.5;     // pre-test of stop rule B (bf16 / fp8 e4m3 copies)
constexpr int LBCH = 4;          // box dimensions q_main loads at a time for a lower bound
constexpr int RLBCH = 2;         // the same in the (rare) refinement, which is kept lean

struct QArgs {
  int64_t n;
  int d, L, K, dpad;
  const float* X;
  const uint16_t* xbf;
  const uint8_t* xf8;
  const float* xscale;
  const int32_t* perm;
  const int32_t* lstart[PDET_MAX_L];
  const int32_t* lcount[PDET_MAX_L];
  const float* box[PDET_MAX_L];
  const float* gbox[PDET_MAX_L];
  int64_t nl[PDET_MAX_L];
  int64_t nlo[PDET_MAX_L];   // first slot of tree i's region in a per-query leaf list
  uint32_t lcap[PDET_MAX_L]; // entries tree i's region holds (min(nl_i, the slot's cap))
  int64_t ng[PDET_MAX_L];
  int64_t nlpad;
  int lb_per_die;            // q_rho leaf blocks (256 leaves) of a tree that each die takes
  int qr_tiles;              // query tiles per q_rho workgroup
  const float* Q;
  const float* qp;           // [nq][L*K]
  const int32_t* qk;         // per-query k, T, offsets and c
  const int64_t* qT;
  const int64_t* qoff;
  const double* qc;
  int32_t uk;                // uniform: the batch shares k and c, and q_setup writes the
  int64_t uT;                // per-query arrays of its slots from these (no upload)
  double uc;
  int uniform;
  const float* t2;           // [slots][NRHO]
  const double* crr;         // [slots][NRHO]: (c*r)^2, compared with squared distances
  uint8_t* rho;              // [slots][L][nlpad] dense round table (0xff: not admitted)
  uint32_t* lcnt;            // [slots][PDET_MAX_L] leaf-list lengths
  uint32_t* bandc;           // [slots][NRHO]: leaves whose LB^2 lies in the band of round
                             // rho's threshold (counted where the leaf's bound is computed)
  const int32_t* leafrow;    // [L][n][L]
  uint32_t* adm_leaf;        // [slots][admcap] leaf lists: tree i from nlo[i]
  uint32_t* adm_w;
  float* adm_lb;             // [slots][admcap] the listed leaf's squared lower bound
  uint32_t* adm2_leaf;       // [slots][admcap + 1] a round's admitted leaves
  uint32_t* adm2_pre;
  int32_t* adm_start;
  float* adm2_lb;            // their squared lower bounds
  int64_t admcap;
  int64_t* ids;
  float* dists;
  int32_t* qstats;
  int rescore, NM;
  int rcap;                  // rounds resolved by q_rho; later ones are refined per query
  int lpc, lpc32;            // lanes per candidate row: verification form, float32 re-rank
  int64_t q0;
  int nslots;
  double r_min, eps;
  const int32_t* qmap;       // null: slot s answers query q0 + s; else query qmap[q0 + s]
  uint32_t* ovf;             // [1 + nq]: count of queries whose leaf lists overflowed, their ids
  int32_t* cand;             // optional [nq][cand_cap]: the ids of S in admission order of
  int64_t cand_cap;          // the walk (the first cand_cap of them)
};

__device__ inline int64_t slot_query(const QArgs& a, int slot) {
  return a.qmap ? (int64_t)a.qmap[a.q0 + slot] : a.q0 + slot;
}

__global__ void q_setup(QArgs a) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= a.nslots) return;
  const int64_t q = slot_query(a, slot);
  // the overflow count of the batch starts at zero (written before any q_main of the batch)
  if (!a.qmap && a.q0 == 0 && slot == 0) a.ovf[0] = 0;
  if (a.uniform) {
    const_cast<int32_t*>(a.qk)[q] = a.uk;
    const_cast<int64_t*>(a.qT)[q] = a.uT;
    const_cast<int64_t*>(a.qoff)[q] = q * (int64_t)a.uk;
    const_cast<double*>(a.qc)[q] = a.uc;
  }
  const double c = a.uniform ? a.uc : a.qc[q];
  float* t2 = const_cast<float*>(a.t2) + (int64_t)slot * NRHO;
  double* crr = const_cast<double*>(a.crr) + (int64_t)slot * NRHO;
  double r = a.r_min;
  for (int rho = 0; rho < NRHO - 1; ++rho) {
    const double t = a.eps * r;
    const double tt = t * t;
    t2[rho] = (float)tt;
    crr[rho] = (c * r) * (c * r);
    r = c * r;
  }
  t2[NRHO - 1] = INFINITY;
  crr[NRHO - 1] = INFINITY;
  for (int i = 0; i < PDET_MAX_L; ++i) a.lcnt[(int64_t)slot * PDET_MAX_L + i] = 0;
  for (int rho = 0; rho < NRHO; ++rho) a.bandc[(int64_t)slot * NRHO + rho] = 0;
}

// float in the global address space (a pointer rebuilt from scalar registers keeps it)
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) const char gchar;

// Box `b` of a structure-of-arrays box table [2][K][nb] (lower corners, then upper). The
// loop runs over the largest K so that all 2K loads are issued before the first is used.
// Column starts are uniform and the row offset is a 32-bit lane value (2K*nb < 2^30 since a
// tree has fewer than 2^24 leaves), so each load is a scalar base plus one vector offset.
__device__ inline void load_box(const float* box, int64_t nb, uint32_t b, int K,
                                float (&lo)[PDET_MAX_K], float (&hi)[PDET_MAX_K]) {
#pragma unroll
  for (int j = 0; j < PDET_MAX_K; ++j) {
    const gchar* cl = (const gchar*)uni((uint64_t)(box + (int64_t)j * nb));
    const gchar* ch = (const gchar*)uni((uint64_t)(box + (int64_t)(K + j) * nb));
    lo[j] = (j < K) ? *(const gfloat*)(cl + b * 4u) : 0.0f;
    hi[j] = (j < K) ? *(const gfloat*)(ch + b * 4u) : 0.0f;
  }
}

// Union of the 16 group boxes of a 256-leaf block (lanes 16i..16i+15 of each wave hold group
// i of the wave's four), into bbox: within waves by lane shuffles, across them through red.
// Every thread calls it; a barrier must follow before bbox is read. The union's bound to any
// query is never above a group's (each term of box_lb2 only shrinks, and FP32 fma and
// subtraction are monotone), so a query the block's box does not admit opens none of its
// groups.
__device__ inline void block_box(const float (&lo)[PDET_MAX_K], const float (&hi)[PDET_MAX_K],
                                 float (*red)[2][PDET_MAX_K], float (*bbox)[PDET_MAX_K]) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < PDET_MAX_K; ++j) {
    float l = lo[j], h = hi[j];
    l = fminf(l, __shfl_xor(l, 16));
    l = fminf(l, __shfl_xor(l, 32));
    h = fmaxf(h, __shfl_xor(h, 16));
    h = fmaxf(h, __shfl_xor(h, 32));
    if ((threadIdx.x & 63) == 0) { red[w][0][j] = l; red[w][1][j] = h; }
  }
  __syncthreads();
  if (threadIdx.x < 2 * PDET_MAX_K) {
    const int side = threadIdx.x / PDET_MAX_K, j = threadIdx.x % PDET_MAX_K;
    float v = red[0][side][j];
    for (int u = 1; u < (int)(blockDim.x >> 6); ++u)
      v = side ? fmaxf(v, red[u][side][j]) : fminf(v, red[u][side][j]);
    bbox[side][j] = v;
  }
}

// box_lb2 (below) of a box held in LDS, in a loop that keeps few values in registers: the
// same fma sequence in dimension order, so the same value.
__device__ inline float box_lb2_lds(const float* blo, const float* bhi, const float* q, int K) {
  float acc = 0.0f;
#pragma unroll 2
  for (int j = 0; j < K; ++j) {
    const float g = fmaxf(0.0f, fmaxf(blo[j] - q[j], q[j] - bhi[j]));
    acc = __fmaf_rn(g, g, acc);
  }
  return acc;
}

// Squared lower-bound distance from q' to a box; explicit fma in dimension order keeps it
// identical wherever it is evaluated.
__device__ inline float box_lb2(const float (&lo)[PDET_MAX_K], const float (&hi)[PDET_MAX_K],
                                const float* q, int K) {
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < PDET_MAX_K; ++j) {
    if (j < K) {
      const float g = fmaxf(0.0f, fmaxf(lo[j] - q[j], q[j] - hi[j]));
      acc = __fmaf_rn(g, g, acc);
    }
  }
  return acc;
}

// The same bound with the box read CH dimensions at a time (fewer registers; the same
// fma sequence, so the same value).
template <int CH>
__device__ inline float leaf_lb2(const float* box, int64_t nl, int64_t leaf, const float* q,
                                 int K) {
  float acc = 0.0f;
  for (int j0 = 0; j0 < K; j0 += CH) {
    float lo[CH], hi[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int j = j0 + u;
      lo[u] = (j < K) ? box[(int64_t)j * nl + leaf] : 0.0f;
      hi[u] = (j < K) ? box[(int64_t)(K + j) * nl + leaf] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int j = j0 + u;
      if (j < K) {
        const float g = fmaxf(0.0f, fmaxf(lo[u] - q[j], q[j] - hi[u]));
        acc = __fmaf_rn(g, g, acc);
      }
    }
  }
  return acc;
}

// KT: the projection width K when it is fixed at compile time (16, the usual case), else 0.
// One workgroup per block of 256 leaves of one tree and one query tile (taken when runs of
// tiles would leave too few workgroups to fill the device).
template <int KT>
__global__ __launch_bounds__(QR_THREADS) void q_rho_tile(QArgs a) {
  const int K = KT ? KT : a.K;
  // one padding word per query row: the 16 queries a wave tests at once read 16 banks
  __shared__ float sq[QT][PDET_MAX_K + 1];
  __shared__ float st[QT][RCAP_MAX + 1];
  // Grid (NXCD * query tiles, lb_per_die, L): the row length is a multiple of NXCD, so
  // blockIdx.x % NXCD is the die a workgroup runs on. Each die takes a fixed share of every
  // tree's leaf blocks and runs through the query tiles of one leaf block after another,
  // which keeps its share of the box tables and the tile's queries in its own L2.
  const int die = blockIdx.x % NXCD;
  const int slot0 = (blockIdx.x / NXCD) * QT;
  const int tree = blockIdx.z;
  const int64_t nl = a.nl[tree], ng = a.ng[tree];
  const int64_t lb = (int64_t)die * a.lb_per_die + blockIdx.y;
  if (lb * QR_THREADS >= nl) return;
  const int rcap = a.rcap;
  const int64_t leaf = lb * QR_THREADS + threadIdx.x;
  const int64_t g = leaf / GL;
  const int sl = threadIdx.x & 15;
  // the group box does not depend on the staged queries: its loads are issued first and
  // are in flight while the query tile is staged
  float lo[PDET_MAX_K], hi[PDET_MAX_K];
  load_box(a.gbox[tree], ng, (uint32_t)std::min(g, ng - 1), K, lo, hi);   // tested if g < ng
  // thresholds and projected queries of the tile: every load issued before any is stored
  constexpr int NST = (QT * (RCAP_MAX + 1) + QR_THREADS - 1) / QR_THREADS;
  constexpr int NSQ = QT * PDET_MAX_K / QR_THREADS;   // rows of PDET_MAX_K, K used
  float stv[NST], sqv[NSQ];
#pragma unroll
  for (int u = 0; u < NST; ++u) {
    const int e = threadIdx.x + u * QR_THREADS;
    const int qi = e / (RCAP_MAX + 1), r = e % (RCAP_MAX + 1);
    stv[u] = (e < QT * (RCAP_MAX + 1) && slot0 + qi < a.nslots)
                 ? a.t2[(int64_t)(slot0 + qi) * NRHO + r] : INFINITY;
  }
  if (!a.qmap) {
    const float* qpt = a.qp + (a.q0 + slot0) * (int64_t)(a.L * K) + tree * K;
#pragma unroll
    for (int u = 0; u < NSQ; ++u) {
      const int e = threadIdx.x + u * QR_THREADS;
      const int qi = e / PDET_MAX_K, j = e % PDET_MAX_K;
      sqv[u] = (j < K && slot0 + qi < a.nslots) ? qpt[(uint32_t)(qi * a.L * K + j)] : 0.0f;
    }
  } else {
#pragma unroll
    for (int u = 0; u < NSQ; ++u) {
      const int e = threadIdx.x + u * QR_THREADS;
      const int qi = e / PDET_MAX_K, j = e % PDET_MAX_K;
      const bool ok = j < K && slot0 + qi < a.nslots;
      sqv[u] = ok ? a.qp[slot_query(a, slot0 + qi) * (int64_t)(a.L * K) + tree * K + j] : 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < NST; ++u) {
    const int e = threadIdx.x + u * QR_THREADS;
    if (e < QT * (RCAP_MAX + 1)) st[e / (RCAP_MAX + 1)][e % (RCAP_MAX + 1)] = stv[u];
  }
#pragma unroll
  for (int u = 0; u < NSQ; ++u) {
    const int e = threadIdx.x + u * QR_THREADS;
    sq[e / PDET_MAX_K][e % PDET_MAX_K] = sqv[u];
  }
  __syncthreads();
  // lane sl of the 16 lanes sharing group g tests that group against query 16*sub + sl (one
  // tile per workgroup: a block-box test first, as in q_rho_runs, would cost more here than
  // it saves)
  uint64_t open_mask = 0;
  for (int sub = 0; sub < QT / 16; ++sub) {
    const int qi = sub * 16 + sl;
    bool open = false;
    if (g < ng && slot0 + qi < a.nslots)
      open = box_lb2(lo, hi, sq[qi], K) <= st[qi][rcap] * (1.0f + BAND_REL);
    const uint64_t mask = __ballot(open);
    open_mask |= (uint64_t)((uint32_t)(mask >> (threadIdx.x & 48)) & 0xffffu) << (16 * sub);
  }
  if (leaf >= nl || open_mask == 0) return;
  load_box(a.box[tree], nl, (uint32_t)leaf, K, lo, hi);
  for (uint64_t mq = open_mask; mq; mq &= mq - 1) {
    const int qi = __ffsll((unsigned long long)mq) - 1;   // open only for slots < nslots
    const int slot = slot0 + qi;
    const float acc = box_lb2(lo, hi, sq[qi], K);
    int c = 0;   // #thresholds < lb2 among rounds 0..rcap: the leaf's first round if <= rcap
#pragma unroll
    for (int rr = 0; rr <= RCAP_MAX; ++rr) c += (rr <= rcap && st[qi][rr] < acc) ? 1 : 0;
    // a near tie can only be with the thresholds on either side of the bound
#pragma unroll
    for (int rr = c - 1; rr <= c; ++rr)
      if (rr >= 0 && rr <= rcap && fabsf(acc - st[qi][rr]) <= BAND_REL * st[qi][rr])
        atomicAdd(&a.bandc[(int64_t)slot * NRHO + rr], 1u);
    if (c <= rcap) {
      const uint32_t pos = atomicAdd(&a.lcnt[(int64_t)slot * PDET_MAX_L + tree], 1u);
      // past the region's capacity only the count grows: q_main sees the overflow
      if (pos < a.lcap[tree]) {
        const int64_t at = (int64_t)slot * a.admcap + a.nlo[tree] + pos;
        a.adm_leaf[at] = ((uint32_t)c << LEAF_BITS) | (uint32_t)leaf;
        a.adm_lb[at] = acc;
      }
    }
  }
}

// One workgroup per block of 256 leaves (16 groups) of one tree and run of a.qr_tiles query
// tiles (the host sizes runs so that the grid still fills the device), in two passes over
// them. Pass 1 holds each lane's group box in registers and tests it against every query,
// keeping the open-query bits of each group and tile in LDS. Pass 2 holds the lane's leaf
// box in the same registers and bounds the leaf for the queries that opened its group, on
// the tiles where some group of the block is open. A wave takes the list positions for one
// query with one atomic.
template <int KT>
__global__ __launch_bounds__(QR_THREADS) void q_rho_runs(QArgs a) {
  const int K = KT ? KT : a.K;
  constexpr int NGB = QR_THREADS / GL;   // groups per leaf block
  static_assert(64 % GL == 0 && 64 / GL == 4 && QR_THREADS % 64 == 0, "a wave holds 4 groups");
  // one padding word per query row: the 16 queries a wave tests at once read 16 banks
  __shared__ float sq[2][QT][PDET_MAX_K + 1];
  __shared__ float st[2][QT][RCAP_MAX + 1];
  __shared__ uint64_t gmask[QR_TILES_MAX][NGB];   // pass 1: open queries per tile and group
  __shared__ uint8_t open_tiles[QR_TILES_MAX];    // tiles where some group is open, in order
  __shared__ uint32_t n_open;
  __shared__ float bred[QR_THREADS / 64][2][PDET_MAX_K];
  __shared__ float bbox[2][PDET_MAX_K];
  // Grid (NXCD * lb_per_die, L, runs of a.qr_tiles tiles): blockIdx.x % NXCD is the die a
  // workgroup runs on. Each die takes a fixed share of every tree's leaf blocks, which keeps
  // its share of the box tables in its own L2.
  const int die = blockIdx.x % NXCD;
  const int tree = blockIdx.y;
  const int64_t nl = a.nl[tree], ng = a.ng[tree];
  const int64_t lb = (int64_t)die * a.lb_per_die + blockIdx.x / NXCD;
  if (lb * QR_THREADS >= nl) return;
  const int rcap = a.rcap;
  const int64_t leaf = lb * QR_THREADS + threadIdx.x;
  const int gl = threadIdx.x / GL;
  const int64_t g = lb * NGB + gl;
  const int sl = threadIdx.x & 15;
  const int t0 = blockIdx.z * a.qr_tiles;
  const int ntiles = std::min((a.nslots + QT - 1) / QT - t0, a.qr_tiles);
  if (threadIdx.x == 0) n_open = 0;
  constexpr int NST = (QT * (RCAP_MAX + 1) + QR_THREADS - 1) / QR_THREADS;
  constexpr int NSQ = QT * PDET_MAX_K / QR_THREADS;   // rows of PDET_MAX_K, K used
  float stv[NST], sqv[NSQ];
  // thresholds and projected queries of a tile into registers (every load issued first),
  // then into LDS buffer b
  auto fetch = [&](int slot0) {
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int e = threadIdx.x + u * QR_THREADS;
      const int qi = e / (RCAP_MAX + 1), r = e % (RCAP_MAX + 1);
      stv[u] = (e < QT * (RCAP_MAX + 1) && slot0 + qi < a.nslots)
                   ? a.t2[(int64_t)(slot0 + qi) * NRHO + r] : INFINITY;
    }
#pragma unroll
    for (int u = 0; u < NSQ; ++u) {
      const int e = threadIdx.x + u * QR_THREADS;
      const int qi = e / PDET_MAX_K, j = e % PDET_MAX_K;
      const bool ok = j < K && slot0 + qi < a.nslots;
      sqv[u] = !ok ? 0.0f
               : !a.qmap ? a.qp[(a.q0 + slot0 + qi) * (int64_t)(a.L * K) + tree * K + j]
                         : a.qp[slot_query(a, slot0 + qi) * (int64_t)(a.L * K) + tree * K + j];
    }
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int e = threadIdx.x + u * QR_THREADS;
      if (e < QT * (RCAP_MAX + 1)) st[b][e / (RCAP_MAX + 1)][e % (RCAP_MAX + 1)] = stv[u];
    }
#pragma unroll
    for (int u = 0; u < NSQ; ++u) {
      const int e = threadIdx.x + u * QR_THREADS;
      sq[b][e / PDET_MAX_K][e % PDET_MAX_K] = sqv[u];
    }
  };
  float lo[PDET_MAX_K], hi[PDET_MAX_K];
  load_box(a.gbox[tree], ng, (uint32_t)std::min(g, ng - 1), K, lo, hi);   // tested if g < ng
  fetch(t0 * QT);
  block_box(lo, hi, bred, bbox);   // read after the first tile's barrier
  // pass 1: group tests (double buffered: past a tile's barrier, a thread has finished
  // reading the other buffer)
  for (int tile = 0; tile < ntiles; ++tile) {
    const int b = tile & 1, slot0 = (t0 + tile) * QT;
    stage(b);
    __syncthreads();
    if (tile + 1 < ntiles) fetch(slot0 + QT);
    // the block's box first (lane l: query l of the tile, in every wave); then lane sl of
    // the 16 lanes sharing group gl tests that group against query 16*sub + sl, for the
    // queries the block's box admits
    const int ql = threadIdx.x & 63;
    const bool bopen = slot0 + ql < a.nslots &&
                       box_lb2_lds(bbox[0], bbox[1], sq[b][ql], K) <=
                           st[b][ql][rcap] * (1.0f + BAND_REL);
    const uint64_t bmask = __ballot(bopen);
    uint64_t open_mask = 0;
#pragma unroll
    for (int sub = 0; sub < QT / 16; ++sub) {
      if (!((bmask >> (16 * sub)) & 0xffffull)) continue;
      const int qi = sub * 16 + sl;
      bool open = false;
      if (g < ng && ((bmask >> qi) & 1ull))
        open = box_lb2(lo, hi, sq[b][qi], K) <= st[b][qi][rcap] * (1.0f + BAND_REL);
      const uint64_t mask = __ballot(open);
      open_mask |= (uint64_t)((uint32_t)(mask >> (threadIdx.x & 48)) & 0xffffu) << (16 * sub);
    }
    if (sl == 0) gmask[tile][gl] = open_mask;
    // the tiles where some group of the block is open, listed in order
    const uint32_t any = __syncthreads_or(open_mask != 0);
    if (threadIdx.x == 0 && any) open_tiles[n_open++] = (uint8_t)tile;
  }
  __syncthreads();
  // pass 2: leaf bounds for the queries that opened the leaf's group, over the open tiles
  // (the next one's queries and thresholds load while the current one is tested; a run
  // that is one tile long, the chunk's last, still holds it in buffer 0)
  const int nop = (int)n_open;
  if (nop == 0) return;
  if (leaf < nl) load_box(a.box[tree], nl, (uint32_t)leaf, K, lo, hi);
  const bool resident = ntiles == 1;
  if (!resident) fetch((t0 + open_tiles[0]) * QT);
  for (int oi = 0; oi < nop; ++oi) {
    const int tile = open_tiles[oi], b = resident ? 0 : (oi & 1);
    const int slot0 = (t0 + tile) * QT;
    if (!resident) {
      stage(b);
      __syncthreads();
      if (oi + 1 < nop) fetch((t0 + open_tiles[oi + 1]) * QT);
    }
    const uint64_t open_mask = (leaf < nl) ? gmask[tile][gl] : 0ull;
    // the queries that open one of the wave's 4 groups, one at a time for the whole wave
    // (the same sequence in every lane: the ballot below counts lanes of one query)
    const int wg0 = (threadIdx.x >> 6) * (64 / GL);
    const uint64_t wave_open =
        gmask[tile][wg0] | gmask[tile][wg0 + 1] | gmask[tile][wg0 + 2] | gmask[tile][wg0 + 3];
    for (uint64_t mq = wave_open; mq; mq &= mq - 1) {
      const int qi = __ffsll((unsigned long long)mq) - 1;   // open only for slots < nslots
      const int slot = slot0 + qi;
      bool adm = false;
      int c = 0;   // #thresholds < lb2 among rounds 0..rcap: the leaf's first round if <= rcap
      float acc = 0.0f;
      if ((open_mask >> qi) & 1u) {
        acc = box_lb2(lo, hi, sq[b][qi], K);
#pragma unroll
        for (int rr = 0; rr <= RCAP_MAX; ++rr) c += (rr <= rcap && st[b][qi][rr] < acc) ? 1 : 0;
        // a near tie can only be with the thresholds on either side of the bound
#pragma unroll
        for (int rr = c - 1; rr <= c; ++rr)
          if (rr >= 0 && rr <= rcap && fabsf(acc - st[b][qi][rr]) <= BAND_REL * st[b][qi][rr])
            atomicAdd(&a.bandc[(int64_t)slot * NRHO + rr], 1u);
        adm = c <= rcap;
      }
      const uint64_t am = __ballot(adm);
      if (!am) continue;
      const int leader = __ffsll((unsigned long long)am) - 1;
      uint32_t base = 0;
      if ((threadIdx.x & 63) == leader)
        base = atomicAdd(&a.lcnt[(int64_t)slot * PDET_MAX_L + tree], (uint32_t)__popcll(am));
      base = __shfl(base, leader);
      if (adm) {
        const uint32_t pos = base + lanes_below_mask(am);
        // past the region's capacity only the count grows: q_main sees the overflow
        if (pos < a.lcap[tree]) {
          const int64_t at = (int64_t)slot * a.admcap + a.nlo[tree] + pos;
          a.adm_leaf[at] = ((uint32_t)c << LEAF_BITS) | (uint32_t)leaf;
          a.adm_lb[at] = acc;
        }
      }
    }
  }
}

__device__ inline bool lex_less(double a, int32_t ia, double b, int32_t ib) {
  return a < b || (a == b && ia < ib);
}

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// 16-byte loads a lane keeps in flight per candidate row: float32 rows (FP64 accumulation
// needs more registers per load) and the low-precision copies
constexpr int NCH32 = 2;
constexpr int NCHLP = 4;
constexpr int NR32 = 1;          // float32 candidate rows per lane group per trip

// Squared Euclidean distances of NR candidates `id[r]` to the query, computed by a group of
// `lpc` lanes (a power of two; every lane of the group must call it; rows with valid[r]
// false are not read; LPC > 0 fixes lpc at compile time). Each lane issues all its 16-byte loads of the NR rows (up to NCH per
// row) before using them. PREC 0: float32 data against the query held in FP64 (qd), FP64
// accumulation; 1: bf16 copy; 2: fp8 e4m3 copy with a per-row scale (both against the
// float32 query qv, FP32 accumulation). Candidates are ranked by squared distance (the
// square root is monotone) and the root is taken once, for the returned k.
template <int PREC, int NR, int LPC = 0>
__device__ inline void cand_dist(const QArgs& a, const int32_t (&id)[NR], const bool (&valid)[NR],
                                 const float* qv, const double* qd, int lg, int lpc_rt,
                                 double (&out)[NR]) {
  const int lpc = LPC ? LPC : lpc_rt;
  double accd[NR];
  float accf[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { accd[r] = 0.0; accf[r] = 0.0f; }
  if constexpr (PREC == PDET_FP32) {
    if ((a.d & 3) == 0) {
      const double2* q2 = reinterpret_cast<const double2*>(qd);
      const int n4 = a.d >> 2;
      constexpr int NCH = NCH32;
      for (int base = 0; base < n4; base += NCH * lpc) {
        // Every load is issued, unconditionally, before any is used (a lane without a row
        // or past the row's end reads a valid address and discards it): loads under a
        // branch would each wait for the one before.
        float4 buf[NR][NCH];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const float4* x4 = reinterpret_cast<const float4*>(a.X + (int64_t)id[r] * a.d);
#pragma unroll
          for (int u = 0; u < NCH; ++u) buf[r][u] = x4[min(base + lg + u * lpc, n4 - 1)];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
          for (int u = 0; u < NCH; ++u) {
            // no branch around the arithmetic either (one would let the compiler move the
            // load into it): a discarded row contributes zeros
            const int c = min(base + lg + u * lpc, n4 - 1);
            const bool ok = valid[r] && base + lg + u * lpc < n4;
            const float4 x = buf[r][u];
            const double2 qa = q2[2 * c], qb = q2[2 * c + 1];
            const double d0 = ok ? (double)x.x - qa.x : 0.0, d1 = ok ? (double)x.y - qa.y : 0.0;
            const double d2 = ok ? (double)x.z - qb.x : 0.0, d3 = ok ? (double)x.w - qb.y : 0.0;
            accd[r] = fma(d0, d0, accd[r]); accd[r] = fma(d1, d1, accd[r]);
            accd[r] = fma(d2, d2, accd[r]); accd[r] = fma(d3, d3, accd[r]);
          }
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (!valid[r]) continue;
        const float* xr = a.X + (int64_t)id[r] * a.d;
        for (int t = lg; t < a.d; t += lpc) {
          const double df = (double)xr[t] - qd[t];
          accd[r] = fma(df, df, accd[r]);
        }
      }
    }
  } else {
    const int nv = (PREC == PDET_BF16) ? (a.dpad >> 3) : (a.dpad >> 4);
    constexpr int NCH = NCHLP;
    for (int base = 0; base < nv; base += NCH * lpc) {
      // bf16: loads issued unconditionally before use, as for float32 rows; fp8 keeps
      // them under the row test (issuing all four first costs more in spilled registers)
      uint4 buf[NR][NCH];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint4* xr = (PREC == PDET_BF16)
                              ? reinterpret_cast<const uint4*>(a.xbf + (int64_t)id[r] * a.dpad)
                              : reinterpret_cast<const uint4*>(a.xf8 + (int64_t)id[r] * a.dpad);
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          const int c = base + lg + u * lpc;
          if constexpr (PREC == PDET_BF16) {
            buf[r][u] = xr[min(c, nv - 1)];
          } else {
            if (valid[r] && c < nv) buf[r][u] = xr[c];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const float sc = (PREC == PDET_BF16 || !valid[r]) ? 1.0f : a.xscale[id[r]];
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          // no branch around the arithmetic (see the float32 form): a discarded row
          // contributes zeros
          const int c = min(base + lg + u * lpc, nv - 1);
          const bool ok = valid[r] && base + lg + u * lpc < nv;
          const uint4 v = buf[r][u];
          if constexpr (PREC == PDET_BF16) {
            const float* q = qv + c * 8;
            const float xs[8] = {bf16_lo(v.x), bf16_hi(v.x), bf16_lo(v.y), bf16_hi(v.y),
                                 bf16_lo(v.z), bf16_hi(v.z), bf16_lo(v.w), bf16_hi(v.w)};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float df = ok ? xs[e] - q[e] : 0.0f;
              accf[r] = fmaf(df, df, accf[r]);
            }
          } else {
            if (!ok) continue;
            const float* q = qv + c * 16;
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              const int wi = (int)w[h];
              const float x0 = __builtin_amdgcn_cvt_f32_fp8(wi, 0) * sc - q[h * 4 + 0];
              const float x1 = __builtin_amdgcn_cvt_f32_fp8(wi, 1) * sc - q[h * 4 + 1];
              const float x2 = __builtin_amdgcn_cvt_f32_fp8(wi, 2) * sc - q[h * 4 + 2];
              const float x3 = __builtin_amdgcn_cvt_f32_fp8(wi, 3) * sc - q[h * 4 + 3];
              accf[r] = fmaf(x0, x0, accf[r]); accf[r] = fmaf(x1, x1, accf[r]);
              accf[r] = fmaf(x2, x2, accf[r]); accf[r] = fmaf(x3, x3, accf[r]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) accd[r] = (double)accf[r];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if constexpr (LPC > 0) out[r] = group_sum<LPC>(accd[r]);
    else out[r] = group_sum(accd[r], lpc);
  }
}

// Bitonic sort of (distance, id) pairs, ascending, over `len` (a power of two) entries.
__device__ void sort_pairs(double* ld, int32_t* li, int len) {
  for (int k = 2; k <= len; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < (len >> 1); t += QM) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int p = i | j;
        const bool asc = (i & k) == 0;
        const double di = ld[i], dp = ld[p];
        const int32_t ii = li[i], ip = li[p];
        if (lex_less(dp, ip, di, ii) == asc) {
          ld[i] = dp; li[i] = ip; ld[p] = di; li[p] = ii;
        }
      }
      __syncthreads();
    }
  }
}

// Round in which leaf `key` = (tree << 28) | leaf was admitted, from the LDS hash of the
// admitted leaves (linear probing; never more than half full), or 255 if it was not.
__device__ inline int hash_round(const uint32_t* hk, const uint8_t* hr, uint32_t key) {
  uint32_t h = mix32(key) & (HSZ - 1);
  for (;;) {
    const uint32_t k = hk[h];
    if (k == key) return hr[h];
    if (k == HEMPTY) return 255;
    h = (h + 1) & (HSZ - 1);
  }
}

// Closed form of the candidate union: before step (rho, i) a point is in S iff its leaf in
// some tree i2 < i is admitted in a round <= rho, or its leaf in some tree i2 > i in a round
// < rho (every earlier step was admitted whole, or the query would have stopped). `lr` is
// the point's row of leaf ordinals; the admission rounds come from the LDS hash, or from
// the dense table rr [L][nlpad] once the hash has overflowed.
__device__ inline bool is_new(const QArgs& a, bool dense, const uint8_t* rr, const uint32_t* hk,
                              const uint8_t* hr, const int32_t* lr, int i, int rho) {
  for (int i2 = 0; i2 < a.L; ++i2) {
    if (i2 == i) continue;
    const int r2 = dense ? rr[(int64_t)i2 * a.nlpad + lr[i2]]
                         : hash_round(hk, hr, ((uint32_t)i2 << TREE_SHIFT) | (uint32_t)lr[i2]);
    if (i2 < i ? (r2 <= rho) : (r2 < rho)) return false;
  }
  return true;
}

// is_new for L = 4 trees, with the point's leaf row already in registers.
__device__ inline bool is_new4(bool dense, int64_t nlpad, const uint8_t* rr, const uint32_t* hk,
                               const uint8_t* hr, const int32_t (&lr)[4], int i, int rho) {
#pragma unroll
  for (int i2 = 0; i2 < 4; ++i2) {
    if (i2 == i) continue;
    const int r2 = dense ? rr[(int64_t)i2 * nlpad + lr[i2]]
                         : hash_round(hk, hr, ((uint32_t)i2 << TREE_SHIFT) | (uint32_t)lr[i2]);
    if (i2 < i ? (r2 <= rho) : (r2 < rho)) return false;
  }
  return true;
}

// One workgroup per query (see the file header). The kernels below instantiate it with the
// occupancy each form reaches: float32 verification keeps a small top-k list and runs eight
// workgroups per CU (a few registers spill; the latency-bound kernel gains more from the
// extra queries in flight); the low-precision forms keep k * rescore candidates and run six.
template <int PREC>
__device__ __forceinline__ void q_main_body(const QArgs& a) {
  extern __shared__ __align__(16) unsigned char sm[];
  double* ld = reinterpret_cast<double*>(sm);     // squared distances of the top-k buffer
  int32_t* li = reinterpret_cast<int32_t*>(ld + a.NM);
  const int dq = (PREC == PDET_FP32) ? ((a.d + 3) & ~3) : a.dpad;
  double* qd = reinterpret_cast<double*>(li + a.NM);   // NM is a multiple of 4: 16-byte aligned
  float* qv = reinterpret_cast<float*>(qd + dq);
  float* qps = qv + dq;

  // the walk's window (traverse) and the select scratch (select_key) are never live at once
  __shared__ __align__(16) uint32_t wbuf[3 * QM + 2];
  uint32_t* w_pre = wbuf;                                       // [QM + 1]
  int32_t* w_start = reinterpret_cast<int32_t*>(wbuf + QM + 2);  // [QM], 8-byte aligned
  int32_t* idbuf = w_start + QM;                                // [QM]
  unsigned long long* sel_key = reinterpret_cast<unsigned long long*>(w_start);  // [QM]
  uint32_t* sel_w = w_pre;                                      // [QM]
  __shared__ uint8_t w_tree[QM];
  __shared__ uint32_t sh_scan[QM / 64 + 1];
  __shared__ uint32_t hist[256];
  uint32_t* wcnt = hist;   // per-entry counts of a WALK_CUT chunk (hist: radix select only)
  __shared__ float st2[NRHO];
  __shared__ uint32_t gopen[GCH / 32];
  __shared__ uint32_t ent_off[PDET_MAX_L + 1];
  __shared__ uint32_t s_mt[PDET_MAX_L];
  __shared__ uint32_t s_pt[PDET_MAX_L];          // points of the round's leaves per tree
  __shared__ uint32_t ent_pre[PDET_MAX_L + 1];   // pre2 at the tree boundaries ent_off[i]
  __shared__ uint32_t s_lc[PDET_MAX_L];          // leaf-list lengths per tree
  __shared__ uint32_t s_lco[PDET_MAX_L + 1];     // their prefix (lists in tree order)
  __shared__ uint32_t hkey[HSZ];
  __shared__ uint8_t hrnd[HSZ];
  __shared__ uint32_t s_nb, s_ncb, s_newtot, s_ef, s_hsum, s_hmix, s_cnt, s_cute, s_clo, s_chi, s_cl;
  __shared__ unsigned long long s_cut;

  const int slot = blockIdx.x;
  const int64_t q = slot_query(a, slot);
  const int tid = threadIdx.x, lane = tid & 63;
  const int lpc = a.lpc;                          // lanes per candidate (power of two)
  const int lg = tid & (lpc - 1), grp = tid / lpc;
  const int k = a.qk[q];
  const int64_t T = a.qT[q];
  const int KL = (PREC == PDET_FP32) ? k : k * a.rescore;
  const int CBcap = a.NM - KL;   // pending candidates beside the list (>= CBMIN >= QM)
  const int LK = a.L * a.K;

  for (int e = tid; e < a.NM; e += QM) { ld[e] = INFINITY; li[e] = INT32_MAX; }
  for (int t = tid; t < dq; t += QM) {
    const float v = (t < a.d) ? a.Q[q * a.d + t] : 0.0f;
    qv[t] = v;
    qd[t] = (double)v;
  }
  for (int t = tid; t < LK; t += QM) qps[t] = a.qp[q * LK + t];
  for (int t = tid; t < NRHO; t += QM) st2[t] = a.t2[(int64_t)slot * NRHO + t];
  uint8_t* rq = a.rho + (int64_t)slot * a.L * a.nlpad;
  for (int e = tid; e < HSZ; e += QM) hkey[e] = HEMPTY;
  if (tid < a.L) s_lc[tid] = a.lcnt[(int64_t)slot * PDET_MAX_L + tid];
  if (tid == 0) { s_ncb = 0; s_hsum = 0; s_hmix = 0; }
  __syncthreads();

  uint32_t* adm = a.adm_leaf + (int64_t)slot * a.admcap;
  uint32_t* admw = a.adm_w + (int64_t)slot * a.admcap;
  float* lstlb = a.adm_lb + (int64_t)slot * a.admcap;   // bounds of the list entries
  uint32_t* adm2 = a.adm2_leaf + (int64_t)slot * (a.admcap + 1);
  uint32_t* pre2 = a.adm2_pre + (int64_t)slot * (a.admcap + 1);
  int32_t* ast = a.adm_start + (int64_t)slot * (a.admcap + 1);
  float* admlb = a.adm2_lb + (int64_t)slot * (a.admcap + 1);  // bounds of the round's leaves

  int64_t nS = 0, leaves = 0, visits = 0;
  uint32_t hn = 0;             // leaves in the hash (all admitted in rounds <= rho)
  bool dense = false;          // the hash overflowed: rounds live in the dense table rq
  uint32_t hsum = 0, hmix = 0;
  int stop = -1, rounds = 0;
  uint32_t band_b = 0;         // rounds whose stop-rule-B count was a near tie
  int cap = a.rcap;            // rounds whose leaf indices are resolved
  // Leaf lists past their slot's capacity (a large index caps them): the query is flagged
  // and answered again with full-capacity slots. STOP_OVERFLOW leaves the round loop;
  // the lists written so far are whole, so the dense table is restored from them.
  auto overflowed = [&]() -> bool {
    bool o = false;
    for (int i = 0; i < a.L; ++i) o = o || s_lc[i] > a.lcap[i];
    return o;
  };
  if (overflowed()) stop = STOP_OVERFLOW;
  const uint64_t t_start = wall_clock64();

  // Sorts the kept list and the pending buffer together (over the power of two that holds
  // them; entries past that are stale and never read); the first KL are the new list.
  auto merge = [&]() {
    const int used = KL + (int)uni(s_ncb);
    int len = 1;
    while (len < used) len <<= 1;
    for (int e = used + tid; e < len; e += QM) { ld[e] = INFINITY; li[e] = INT32_MAX; }
    __syncthreads();
    sort_pairs(ld, li, len);
    if (tid == 0) s_ncb = 0;
    __syncthreads();
  };

  // Walk the points of list entries [e_lo, e_hi), 256 at a time. A point's leaf is found
  // by a binary search in an LDS window of the prefix list. WALK_COUNT adds every new point
  // to its leaf's count admw[]; WALK_VERIFY verifies the new points and offers them to the
  // top-k; WALK_CUT (entries in admission order) does the same up to and including the
  // first leaf after which R new points have been admitted, whose entry goes to cut_e
  // (NO_CUT if the range holds fewer). Returns the number of new points admitted (uniform).
  // P0, P1: the prefix values pre2[e_lo], pre2[e_hi] (uniform; passed in from LDS copies).
  auto traverse = [&](int mode, int rho, uint32_t e_lo, uint32_t e_hi, uint32_t P0,
                      uint32_t P1, uint32_t R, uint32_t& cut_e) -> uint32_t {
    uint32_t newc = 0;
    cut_e = NO_CUT;
    if (tid == 0) s_ef = e_lo;
    __syncthreads();
    // The window holds QM list entries from ef on (their prefixes up to w_pre[QM]) and is
    // reloaded only when a chunk reaches past it: a window covers many chunks' points.
    uint32_t ef = 0, wend = 0;
    bool have = false;
    for (uint32_t base = P0; base < P1; base += QM) {
      visits += std::min<uint32_t>(QM, P1 - base);
      const bool reload = !have || wend < std::min(base + (uint32_t)QM, P1);
      if (reload) {
        ef = uni(s_ef);   // the entry holding `base`
        const uint32_t e = ef + tid;
        w_pre[tid] = (e <= e_hi) ? pre2[e] : 0xffffffffu;
        if (e < e_hi) {
          w_tree[tid] = (uint8_t)(adm2[e] >> TREE_SHIFT);
          w_start[tid] = ast[e];
        }
        if (tid == 0) w_pre[QM] = (ef + QM <= e_hi) ? pre2[ef + QM] : 0xffffffffu;
      }
      wcnt[tid] = 0;
      if (tid == 0) {
        s_nb = 0;
        s_cute = NO_CUT;
      }
      __syncthreads();
      if (reload) {
        wend = uni(w_pre[QM]);
        have = true;
      }
      const uint32_t p = base + tid;
      bool nw = false;
      int32_t id = 0;
      int lo = 0;
      if (p < P1) {
        int hi = QM;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_pre[mid] <= p) lo = mid; else hi = mid;
        }
        const int tr = w_tree[lo];
        const int64_t pos = (int64_t)tr * a.n + w_start[lo] + (p - w_pre[lo]);
        if (a.L == 4) {
          // the point's leaf row and id loaded together, before either is used
          const int4 r4 = *reinterpret_cast<const int4*>(a.leafrow + pos * 4);
          id = a.perm[pos];
          const int32_t lr[4] = {r4.x, r4.y, r4.z, r4.w};
          nw = is_new4(dense, a.nlpad, rq, hkey, hrnd, lr, tr, rho);
        } else {
          id = a.perm[pos];
          nw = is_new(a, dense, rq, hkey, hrnd, a.leafrow + pos * a.L, tr, rho);
        }
      }
      if (mode == WALK_CUT && cut_e == NO_CUT) {
        // new points per window entry; the first entry whose inclusive count reaches R
        if (nw) atomicAdd(&wcnt[lo], 1u);
        __syncthreads();
        const uint32_t c = wcnt[tid];
        uint32_t tot;
        const uint32_t ex = block_excl_scan<QM>(c, sh_scan, &tot);
        if (ef + tid < e_hi && newc + ex + c >= R) atomicMin(&s_cute, ef + tid);
        __syncthreads();
        cut_e = uni(s_cute);
        // the rest of that leaf (its end prefix is in the window: cut_e - ef < QM)
        if (cut_e != NO_CUT) P1 = std::min(P1, uni(w_pre[cut_e + 1 - ef]));
      }
      if (mode == WALK_CUT && cut_e != NO_CUT) nw = nw && ef + lo <= cut_e;
      const uint64_t mask = __ballot(nw);
      uint32_t wbase = 0;
      if (lane == 0 && mask) wbase = atomicAdd(&s_nb, (uint32_t)__popcll(mask));
      wbase = __shfl(wbase, 0);
      if (nw) {
        if (mode == WALK_COUNT) {
          atomicAdd(&admw[ef + lo], 1u);
        } else {
          idbuf[wbase + lanes_below_mask(mask)] = id;
          hsum += (uint32_t)id;
          hmix += mix32((uint32_t)id);
          if (a.cand) {
            const int64_t at = nS + newc + wbase + lanes_below_mask(mask);
            if (at < a.cand_cap) a.cand[q * a.cand_cap + at] = id;
          }
        }
      }
      __syncthreads();
      const uint32_t nb = uni(s_nb);
      newc += nb;
      if (tid == QM - 1 && p < P1) {
        // first window entry of the next chunk (the one holding base + QM): this thread's
        // entry or, when that ends here, the next (every entry holds at least one point)
        s_ef = ef + lo + (w_pre[lo + 1] <= base + QM ? 1 : 0);
      }
      if (mode != WALK_COUNT) {
        constexpr int NRV = (PREC == PDET_FP32) ? NR32 : 1;
        // the low-precision forms take one instance of the loop per lane-group width, so the
        // reduction has no tests (for float32 the extra instances cost more in spills)
        auto dist_rows = [&](auto lpc_c) {
          constexpr int LPC = decltype(lpc_c)::value;   // 0: the runtime width
          const uint32_t G = QM / (LPC ? LPC : lpc);   // lane groups: candidates per row
          for (uint32_t c0 = 0; c0 < nb; c0 += NRV * G) {
            int32_t cid[NRV];
            bool valid[NRV];
            double dd[NRV];
#pragma unroll
            for (int r = 0; r < NRV; ++r) {
              const uint32_t c = c0 + r * G + grp;
              valid[r] = c < nb;
              cid[r] = valid[r] ? idbuf[c] : 0;
            }
            cand_dist<PREC, NRV, LPC>(a, cid, valid, qv, qd, lg, lpc, dd);
#pragma unroll
            for (int r = 0; r < NRV; ++r) {
              if (valid[r] && lg == 0 && lex_less(dd[r], cid[r], ld[KL - 1], li[KL - 1])) {
                const uint32_t pos = atomicAdd(&s_ncb, 1u);
                ld[KL + pos] = dd[r];
                li[KL + pos] = cid[r];
              }
            }
          }
        };
        if constexpr (PREC == PDET_FP32) {
          dist_rows(std::integral_constant<int, 0>{});
        } else {
          switch (lpc) {   // lanes_for gives a power of two in [4, 64]
            case 4: dist_rows(std::integral_constant<int, 4>{}); break;
            case 8: dist_rows(std::integral_constant<int, 8>{}); break;
            case 16: dist_rows(std::integral_constant<int, 16>{}); break;
            case 32: dist_rows(std::integral_constant<int, 32>{}); break;
            default: dist_rows(std::integral_constant<int, 64>{}); break;
          }
        }
      }
      __syncthreads();
      if (mode != WALK_COUNT && uni(s_ncb) > (uint32_t)(CBcap - QM)) merge();
    }
    return newc;
  };

  // Puts the entries [e0, e1) of tree i (at most QM) in admission order, ascending
  // (LB^2, leaf ordinal) (keys are distinct within a tree), with their prefix list rebuilt.
  auto order_entries = [&](uint32_t e0, uint32_t e1, uint32_t P0) {
    const uint32_t mi = e1 - e0, e = e0 + tid;
    unsigned long long key = ~0ull;
    uint32_t en = 0, cnt = 0;
    int32_t st0 = 0;
    float lb = 0.0f;
    if (tid < mi) {
      en = adm2[e];
      st0 = ast[e];
      cnt = pre2[e + 1] - pre2[e];
      lb = admlb[e];
      key = ((unsigned long long)__float_as_uint(lb) << 32) | (en & ((1u << TREE_SHIFT) - 1));
    }
    sel_key[tid] = key;
    __syncthreads();
    uint32_t rank = 0;
    if (tid < mi)
      for (uint32_t u = 0; u < mi; ++u) rank += (sel_key[u] < key) ? 1u : 0u;
    __syncthreads();
    if (tid < mi) {
      adm2[e0 + rank] = en;
      ast[e0 + rank] = st0;
      admlb[e0 + rank] = lb;
      sel_w[rank] = cnt;
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t ex = block_excl_scan<QM>(tid < mi ? sel_w[tid] : 0u, sh_scan, &tot);
    if (tid < mi) pre2[e0 + tid] = P0 + ex;   // pre2[e1] = P0 + tot is unchanged
    __syncthreads();
  };

  // Weighted radix select over list entries [e0, e1) keyed by (LB^2 bits, leaf ordinal):
  // the smallest key whose inclusive weight prefix reaches R. Weights: the leaf sizes
  // (by_counts) or the exact new-point counts admw[].
  auto select_key = [&](uint32_t e0, uint32_t e1, uint32_t R, bool by_counts) {
    if (e1 - e0 <= (uint32_t)QM) {
      // at most one entry per thread: each entry's inclusive prefix in key order is a sum
      // over all entries (keys are distinct within a tree); the cut is the least key whose
      // prefix reaches R, the same key the radix passes find
      const uint32_t m = e1 - e0, e = e0 + tid;
      unsigned long long key = ~0ull;
      uint32_t wgt = 0;
      if (e < e1) {
        key = ((unsigned long long)__float_as_uint(admlb[e]) << 32) |
              (adm2[e] & ((1u << TREE_SHIFT) - 1));
        wgt = by_counts ? pre2[e + 1] - pre2[e]
                        : __hip_atomic_load(&admw[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      sel_key[tid] = key;
      sel_w[tid] = wgt;
      if (tid == 0) s_cut = ~0ull;
      __syncthreads();
      if (e < e1) {
        uint32_t pref = 0;
        for (uint32_t u = 0; u < m; ++u) pref += (sel_key[u] <= key) ? sel_w[u] : 0u;
        if (pref >= R) atomicMin(&s_cut, key);
      }
      __syncthreads();
      const unsigned long long cut = uni((uint64_t)s_cut);
      __syncthreads();
      return cut;
    }
    unsigned long long prefix = 0;
    for (int pass = 0; pass < 8; ++pass) {
      const int shift = 56 - 8 * pass;
      hist[tid] = 0;
      __syncthreads();
      for (uint32_t e = e0 + tid; e < e1; e += QM) {
        const unsigned long long key = ((unsigned long long)__float_as_uint(admlb[e]) << 32) |
                                       (adm2[e] & ((1u << TREE_SHIFT) - 1));
        if (pass == 0 || (key >> (shift + 8)) == prefix) {
          const uint32_t wgt =
              by_counts ? pre2[e + 1] - pre2[e]
                        : __hip_atomic_load(&admw[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (wgt) atomicAdd(&hist[(key >> shift) & 255], wgt);
        }
      }
      __syncthreads();
      const uint32_t h = hist[tid];
      uint32_t tot;
      const uint32_t ex = block_excl_scan<QM>(h, sh_scan, &tot);
      if (ex < R && ex + h >= R) {
        s_cut = (prefix << 8) | (unsigned long long)tid;
        s_newtot = R - ex;
      }
      __syncthreads();
      prefix = uni((uint64_t)s_cut);
      R = uni(s_newtot);
      __syncthreads();
    }
    return prefix;
  };

  // Keeps the entries of [e0, e1) whose key is <= cut, compacted in place (writes never pass
  // the read position), with their prefix sums; returns how many remain.
  auto keep_upto = [&](uint32_t e0, uint32_t e1, unsigned long long cut) -> uint32_t {
    const uint32_t P0 = uni(pre2[e0]);
    uint32_t nm = 0, nP = 0;
    for (uint32_t b = e0; b < e1; b += QM) {
      const uint32_t e = b + tid;
      bool inc = false;
      uint32_t cnt = 0, en = 0;
      int32_t st0 = 0;
      float lb = 0.0f;
      if (e < e1) {
        en = adm2[e];
        st0 = ast[e];
        lb = admlb[e];
        inc = ((((unsigned long long)__float_as_uint(lb)) << 32) |
               (en & ((1u << TREE_SHIFT) - 1))) <= cut;
        if (inc) cnt = pre2[e + 1] - pre2[e];
      }
      uint32_t t1, t2;
      const uint32_t pos = block_excl_scan<QM>(inc ? 1u : 0u, sh_scan, &t1);
      const uint32_t pre = block_excl_scan<QM>(cnt, sh_scan, &t2);
      if (inc) {
        adm2[e0 + nm + pos] = en;
        ast[e0 + nm + pos] = st0;
        admlb[e0 + nm + pos] = lb;
        pre2[e0 + nm + pos] = P0 + nP + pre;
      }
      nm += t1;
      nP += t2;
      __syncthreads();   // pre2[e + 1] of this chunk's last entry is read before it moves
    }
    if (tid == 0) pre2[e0 + nm] = P0 + nP;
    __syncthreads();
    return nm;
  };

  for (int rho = 0; rho < NRHO - 1 && stop == -1; ++rho) {
    rounds = rho + 1;
    if (rho == cap + 1) {
      // The lists hold every leaf whose first round is <= cap. Leaves whose first round is
      // within the next RWIN rounds are appended: per chunk of groups, group tests into an
      // LDS bitmap, then one leaf per thread for the open groups.
      const int ncap = std::min(NRHO - 2, cap + RWIN);
      for (int i = 0; i < a.L; ++i) {
        const int64_t nl = a.nl[i], ng = a.ng[i];
        const float* gb = a.gbox[i];
        const float* qi = qps + i * a.K;
        uint32_t* lst = adm + a.nlo[i];
        for (int64_t g0 = 0; g0 < ng; g0 += GCH) {
          for (int w = tid; w < GCH / 32; w += QM) gopen[w] = 0u;
          __syncthreads();
          for (int64_t g = g0 + tid; g < std::min<int64_t>(ng, g0 + GCH); g += QM) {
            if (leaf_lb2<RLBCH>(gb, ng, g, qi, a.K) <= st2[ncap] * (1.0f + BAND_REL))
              atomicOr(&gopen[(g - g0) >> 5], 1u << ((g - g0) & 31));
          }
          __syncthreads();
          const int64_t l1 = std::min<int64_t>(nl, (g0 + GCH) * GL);
          for (int64_t leaf = g0 * GL + tid; leaf < l1; leaf += QM) {
            const int64_t gl = leaf / GL - g0;
            if (!((gopen[gl >> 5] >> (gl & 31)) & 1u)) continue;
            const float lb2 = leaf_lb2<RLBCH>(a.box[i], nl, leaf, qi, a.K);
            int pos = 0;   // first round whose threshold admits the leaf
#pragma unroll
            for (int sft = NRHO / 2; sft > 0; sft >>= 1)
              if (st2[pos + sft - 1] < lb2) pos += sft;
            for (int rr = pos - 1; rr <= pos; ++rr)
              if (rr > cap && rr <= ncap && fabsf(lb2 - st2[rr]) <= BAND_REL * st2[rr])
                atomicAdd(&a.bandc[(int64_t)slot * NRHO + rr], 1u);
            if (pos > cap && pos <= ncap) {
              const uint32_t at = atomicAdd(&s_lc[i], 1u);
              if (at < a.lcap[i]) {
                lst[at] = ((uint32_t)pos << LEAF_BITS) | (uint32_t)leaf;
                lstlb[a.nlo[i] + at] = lb2;
              }
            }
          }
          __syncthreads();
        }
      }
      cap = ncap;
      if (overflowed()) {
        // s_lco still holds the prefix of the lists before this append: every entry the
        // dense table may hold lies in it
        stop = STOP_OVERFLOW;
        break;
      }
    }
    // admitted leaves of this round, from the lists in tree order: entries, their sizes'
    // prefix sums and their perm start positions
    if (tid < a.L) { s_mt[tid] = 0; s_pt[tid] = 0; }
    if (tid == 0) {
      s_cnt = 0;
      s_clo = 0;
      s_chi = 0;
      s_cl = 0;
      s_lco[0] = 0;
      for (int i = 0; i < a.L; ++i) s_lco[i + 1] = s_lco[i] + s_lc[i];
    }
    __syncthreads();
    const uint32_t E = uni(s_lco[a.L]);
    uint32_t m = 0, P = 0;
    for (uint32_t v0 = 0; v0 < E; v0 += QM) {
      const uint32_t v = v0 + tid;
      bool match = false;
      uint32_t en = 0, cnt = 0;
      int32_t st0 = 0;
      float lbv = 0.0f;
      if (v < E) {
        int tr = 0;
        while (tr + 1 < a.L && s_lco[tr + 1] <= v) ++tr;
        const uint32_t ent = adm[a.nlo[tr] + (v - s_lco[tr])];
        if ((ent >> LEAF_BITS) == (uint32_t)rho) {
          lbv = lstlb[a.nlo[tr] + (v - s_lco[tr])];
          const uint32_t leaf = ent & ((1u << LEAF_BITS) - 1);
          match = true;
          en = ((uint32_t)tr << TREE_SHIFT) | leaf;
          cnt = (uint32_t)a.lcount[tr][leaf];
          st0 = a.lstart[tr][leaf];
          atomicAdd(&s_mt[tr], 1u);
          atomicAdd(&s_pt[tr], cnt);
        }
      }
      uint32_t t1, t2;
      const uint32_t pos = block_excl_scan<QM>(match ? 1u : 0u, sh_scan, &t1);
      const uint32_t pre = block_excl_scan<QM>(cnt, sh_scan, &t2);
      if (match) {
        adm2[m + pos] = en;
        pre2[m + pos] = P + pre;
        ast[m + pos] = st0;
        admlb[m + pos] = lbv;
      }
      m += t1;
      P += t2;
    }
    if (tid == 0) {
      pre2[m] = P;
      ent_off[0] = 0;   // tree i's entries are [ent_off[i], ent_off[i+1]) of the list
      ent_pre[0] = 0;
      for (int i = 0; i < a.L; ++i) {
        ent_off[i + 1] = ent_off[i] + s_mt[i];
        ent_pre[i + 1] = ent_pre[i] + s_pt[i];
      }
    }
    __syncthreads();
    // this round's leaves join the dedupe state (every thread reads the lists and hn alike)
    if (!dense && hn + m > (uint32_t)HMAX) {
      dense = true;   // every leaf admitted so far, this round's included, into the table
      for (uint32_t v = tid; v < E; v += QM) {
        int tr = 0;
        while (tr + 1 < a.L && s_lco[tr + 1] <= v) ++tr;
        const uint32_t ent = adm[a.nlo[tr] + (v - s_lco[tr])];
        if ((ent >> LEAF_BITS) <= (uint32_t)rho)
          rq[(int64_t)tr * a.nlpad + (ent & ((1u << LEAF_BITS) - 1))] = (uint8_t)(ent >> LEAF_BITS);
      }
    } else if (dense) {
      for (uint32_t e = tid; e < m; e += QM) {
        const uint32_t en = adm2[e];
        rq[(int64_t)(en >> TREE_SHIFT) * a.nlpad + (en & ((1u << TREE_SHIFT) - 1))] =
            (uint8_t)rho;
      }
    } else {
      for (uint32_t e = tid; e < m; e += QM) {
        const uint32_t key = adm2[e];
        uint32_t h = mix32(key) & (HSZ - 1);
        while (atomicCAS(&hkey[h], HEMPTY, key) != HEMPTY) h = (h + 1) & (HSZ - 1);
        hrnd[h] = (uint8_t)rho;
      }
    }
    hn += m;
    __syncthreads();
    const int64_t pts = (int64_t)P;

    if (m > 0) {

      uint32_t ce;
      if (nS + pts < T) {
        // stop rule A cannot fire in this round: admit every tree's leaves in one pass
        leaves += m;
        nS += traverse(WALK_VERIFY, rho, 0, m, 0, P, 0, ce);
      } else {
        // trees in order; exact counts decide the tree (and leaf) where |S| reaches T
        for (int i = 0; i < a.L && stop == -1; ++i) {
          const uint32_t e0 = uni(ent_off[i]), e1 = uni(ent_off[i + 1]);
          if (e0 == e1) continue;
          const uint32_t p0 = uni(ent_pre[i]), p1 = uni(ent_pre[i + 1]);
          const int64_t pts_i = (int64_t)p1 - (int64_t)p0;
          if (nS + pts_i < T || e1 - e0 <= (uint32_t)QM) {
            // whole tree, or its leaves in admission order up to the one where |S| reaches T
            const bool may_stop = nS + pts_i >= T;
            if (may_stop) order_entries(e0, e1, p0);
            nS += traverse(may_stop ? WALK_CUT : WALK_VERIFY, rho, e0, e1, p0, p1,
                           (uint32_t)(T - nS), ce);
            if (ce != NO_CUT) {
              leaves += ce - e0 + 1;
              stop = 1;
            } else {
              leaves += e1 - e0;
            }
            continue;
          }
          if (nS == 0) {
            // S is empty, so every point of this tree's leaves is new (a tree's leaves are
            // disjoint): the leaf sizes are the new-point counts and the cut they select
            // is the leaf where |S| reaches T
            const unsigned long long cut = select_key(e0, e1, (uint32_t)T, true);
            const uint32_t e_end = e0 + keep_upto(e0, e1, cut);
            stop = 1;
            leaves += e_end - e0;
            nS += traverse(WALK_VERIFY, rho, e0, e_end, p0, uni(pre2[e_end]), 0, ce);
            continue;
          }
          // more leaves than one ordering pass takes: count new points per leaf over a
          // bounded prefix, then select the leaf by key
          uint32_t e1c = e1;
          if (pts_i >= T) {
            // A tree's leaves are disjoint, so at most |S| of their points are already in S:
            // the shortest (LB^2, ordinal) prefix holding >= T points has >= T - |S| new
            // points, and the leaf where |S| reaches T lies in it. Only it is counted.
            const unsigned long long kap = select_key(e0, e1, (uint32_t)T, true);
            e1c = e0 + keep_upto(e0, e1, kap);
          }
          for (uint32_t e = e0 + tid; e < e1c; e += QM) admw[e] = 0;
          __syncthreads();
          const uint32_t new_i =
              traverse(WALK_COUNT, rho, e0, e1c, p0, uni(pre2[e1c]), 0, ce);
          uint32_t e_end = e1;
          if (nS + (int64_t)new_i < T) {
            // contradicts the bound above: the query ends with stop = -2 (an internal
            // error the statistics report; it leaves the round loop)
            if (e1c != e1) { stop = -2; break; }
          } else {
            // the smallest key whose inclusive new-point prefix reaches R = T - |S|
            const unsigned long long cut = select_key(e0, e1c, (uint32_t)(T - nS), false);
            e_end = e0 + keep_upto(e0, e1c, cut);
            stop = 1;
          }
          leaves += e_end - e0;
          nS += traverse(WALK_VERIFY, rho, e0, e_end, p0, uni(pre2[e_end]), 0, ce);
        }
      }
      if (stop != -1) break;
    }
    if (nS >= k) {
      // stop rule B: at least k points of S within c*r (compared squared, with (c*r)^2);
      // the counts at (c r)^2 (1 -+ 2 BAND_REL) flag a near tie of the k-th distance
      const double crr = a.crr[(int64_t)slot * NRHO + rho];
      const double blo = crr * (1.0 - 2.0 * BAND_REL), bhi = crr * (1.0 + 2.0 * BAND_REL);
      uint32_t cnt = 0, clo = 0, chi = 0;
      if constexpr (PREC == PDET_FP32) {
        // the k-th smallest distance of the kept list and the pending buffer is <= c*r
        // iff at least k of them are
        const uint32_t tot = (uint32_t)KL + uni(s_ncb);
        for (uint32_t e = tid; e < tot; e += QM) {
          const double v = ld[e];
          cnt += (v <= crr) ? 1u : 0u;
          clo += (v <= blo) ? 1u : 0u;
          chi += (v <= bhi) ? 1u : 0u;
        }
      } else {
        // Low-precision distances rank the candidates. The rule is tested on them first,
        // against (c r)^2 widened by the format's error (LOWP_SLACK); when that count
        // reaches k, the rule is decided on exact float32 distances of the kept list (the
        // best k * rescore of S by low-precision distance), so quantisation error neither
        // stops a query that the exact count would not stop nor, unless a kept candidate's
        // error exceeds the slack, keeps one running that it would stop.
        const double slack = (PREC == PDET_BF16) ? LOWP_SLACK_BF16 : LOWP_SLACK_FP8;
        const double crr_wide = crr * (1.0 + slack) * (1.0 + slack);
        const uint32_t tot = (uint32_t)KL + uni(s_ncb);
        uint32_t cl = 0;
        for (uint32_t e = tid; e < tot; e += QM) cl += (ld[e] <= crr_wide) ? 1u : 0u;
        if (cl) atomicAdd(&s_cl, cl);
        __syncthreads();
        const bool fires = uni(s_cl) >= (uint32_t)k;
        if (fires && uni(s_ncb) > 0) merge();
        const int lpc32 = a.lpc32, lg32 = tid & (lpc32 - 1), grp32 = tid / lpc32;
        const int G32 = QM / lpc32;
        for (int t0 = 0; fires && t0 < KL; t0 += 2 * G32) {
          int32_t id[2];
          bool valid[2];
          double dd[2];
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const int t = t0 + r * G32 + grp32;
            valid[r] = t < KL && li[t] != INT32_MAX;
            id[r] = valid[r] ? li[t] : 0;
          }
          cand_dist<PDET_FP32, 2>(a, id, valid, qv, qd, lg32, lpc32, dd);
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            if (valid[r] && lg32 == 0) {
              cnt += (dd[r] <= crr) ? 1u : 0u;
              clo += (dd[r] <= blo) ? 1u : 0u;
              chi += (dd[r] <= bhi) ? 1u : 0u;
            }
          }
        }
      }
      if (cnt) atomicAdd(&s_cnt, cnt);
      if (clo) atomicAdd(&s_clo, clo);
      if (chi) atomicAdd(&s_chi, chi);
      __syncthreads();
      if (uni(s_cnt) >= (uint32_t)k) stop = 2;
      if (uni(s_clo) < (uint32_t)k && uni(s_chi) >= (uint32_t)k) ++band_b;
    }
    __syncthreads();
  }
  if (uni(s_ncb) > 0) merge();
  if (dense) {
    // leave the dense table all 0xff for the slot's next query: every entry written was a
    // listed leaf
    __syncthreads();
    const uint32_t E = uni(s_lco[a.L]);
    for (uint32_t v = tid; v < E; v += QM) {
      int tr = 0;
      while (tr + 1 < a.L && s_lco[tr + 1] <= v) ++tr;
      const uint32_t ent = adm[a.nlo[tr] + (v - s_lco[tr])];
      rq[(int64_t)tr * a.nlpad + (ent & ((1u << LEAF_BITS) - 1))] = 0xff;
    }
  }

  if constexpr (PREC != PDET_FP32) {
    // re-rank the kept low-precision candidates with exact float32 distances
    const int lpc32 = a.lpc32, lg32 = tid & (lpc32 - 1), grp32 = tid / lpc32;
    const int G32 = QM / lpc32;
    for (int t0 = 0; t0 < KL; t0 += 2 * G32) {
      int32_t id[2];
      bool valid[2];
      double dd[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int t = t0 + r * G32 + grp32;
        valid[r] = t < KL && li[t] != INT32_MAX;
        id[r] = valid[r] ? li[t] : 0;
      }
      cand_dist<PDET_FP32, 2>(a, id, valid, qv, qd, lg32, lpc32, dd);
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (valid[r] && lg32 == 0) ld[t0 + r * G32 + grp32] = dd[r];
    }
    __syncthreads();
    int len = 1;
    while (len < KL) len <<= 1;
    for (int e = KL + tid; e < len; e += QM) { ld[e] = INFINITY; li[e] = INT32_MAX; }
    __syncthreads();
    sort_pairs(ld, li, len);
  }

  // (full-capacity slots never overflow; the guard keeps a retry from touching its own map)
  if (stop == STOP_OVERFLOW && tid == 0 && !a.qmap)
    a.ovf[1 + atomicAdd(&a.ovf[0], 1u)] = (uint32_t)q;
  const int64_t off = a.qoff[q];
  for (int t = tid; t < k; t += QM) {
    a.ids[off + t] = (li[t] == INT32_MAX) ? -1 : (int64_t)li[t];
    a.dists[off + t] = (float)sqrt(ld[t]);
  }
  atomicAdd(&s_hsum, hsum);
  atomicAdd(&s_hmix, hmix);
  __syncthreads();
  if (tid == 0 && a.qstats) {
    int32_t* st = a.qstats + q * PDET_QSTAT_WORDS;
    st[PDET_QSTAT_ROUNDS] = rounds;
    st[PDET_QSTAT_NCAND] = (int32_t)nS;
    st[PDET_QSTAT_STOP] = stop;
    st[PDET_QSTAT_LEAVES] = (int32_t)leaves;
    st[PDET_QSTAT_HSUM] = (int32_t)s_hsum;
    st[PDET_QSTAT_HMIX] = (int32_t)s_hmix;
    st[PDET_QSTAT_TIME] = (int32_t)std::min<uint64_t>(wall_clock64() - t_start, INT32_MAX);
    st[PDET_QSTAT_VISITS] = (int32_t)std::min<int64_t>(visits, INT32_MAX);
    uint32_t bl = 0;
    for (int rr = 0; rr < rounds; ++rr) bl += a.bandc[(int64_t)slot * NRHO + rr];
    st[PDET_QSTAT_BAND_LEAF] = (int32_t)bl;
    st[PDET_QSTAT_BAND_STOPB] = (int32_t)band_b;
  }
}

__global__ __launch_bounds__(QM) __attribute__((amdgpu_waves_per_eu(8))) void q_main_f32(QArgs a) {
  q_main_body<PDET_FP32>(a);
}

template <int PREC>
__global__ __launch_bounds__(QM) __attribute__((amdgpu_waves_per_eu(6))) void q_main_lowp(QArgs a) {
  q_main_body<PREC>(a);
}

// The same search for batches with long candidate walks (see use_long_walk): eight
// workgroups per CU hide more of the walk's latency than the register spills cost there,
// while short searches run faster at six (measured on 1M and 100M points).
template <int PREC>
__global__ __launch_bounds__(QM) __attribute__((amdgpu_waves_per_eu(8))) void q_main_lowp_long(QArgs a) {
  q_main_body<PREC>(a);
}

}  // namespace

// Per-query parameters of a batch into the workspace's pinned staging arrays.
double query_beta(const Index& ix, const QueryConfig& qc, double c, double& memo_c,
                  double& memo_b) {
  if (qc.beta >= 0.0) return qc.beta;
  if (c != memo_c) { memo_c = c; memo_b = theoretical_beta(ix.K, ix.L, c); }
  return memo_b;
}

int stage_params(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws) {
  int maxKL = 1;
  int64_t acc = 0;
  bool uniform = qc.nq > 0;
  double memo_c = 0.0, memo_b = 0.0;   // theoretical beta of the last c (batches mix few c)
  for (int64_t q = 0; q < qc.nq; ++q) {
    const int k = qc.k_host[q];
    uniform = uniform && k == qc.k_host[0] && qc.c_host[q] == qc.c_host[0];
    ws.h_k.as<int32_t>()[q] = k;
    ws.h_c.as<double>()[q] = qc.c_host[q];
    const double beta = query_beta(ix, qc, qc.c_host[q], memo_c, memo_b);
    ws.h_T.as<int64_t>()[q] = (int64_t)std::ceil(beta * (double)ix.n) + k;
    ws.h_off.as<int64_t>()[q] = acc;
    acc += k;
    maxKL = std::max(maxKL, qc.precision == PDET_FP32 ? k : k * qc.rescore);
  }
  ws.uniform = uniform;
  if (uniform) {
    ws.uk = qc.k_host[0];
    ws.uc = qc.c_host[0];
    ws.uT = ws.h_T.as<int64_t>()[0];
  }
  return maxKL;
}

// Query slots a capped workspace aims for: one q_main workgroup per slot, eight resident
// per compute unit.
constexpr int64_t TARGET_SLOTS = 2048;
// Least per-tree leaf-list capacity of a capped slot, and the full-capacity slots that
// answer overflowed queries again.
constexpr int64_t MIN_LIST_CAP = 16384;
constexpr int64_t LIST_CAP_DIV = 16;
constexpr int64_t RETRY_SLOTS = 16;

int64_t total_leaves(const Index& ix) {
  int64_t t = 0;
  for (int i = 0; i < ix.L; ++i) t += ix.nl[i];
  return std::max<int64_t>(t, 1);
}

// Entries of a slot's leaf lists when every tree's region holds min(nl_i, cap) of them.
int64_t list_entries(const Index& ix, int64_t cap) {
  int64_t t = 0;
  for (int i = 0; i < ix.L; ++i) t += std::min<int64_t>(ix.nl[i], cap);
  return std::max<int64_t>(t, 1);
}

size_t slot_bytes_at(const Index& ix, int64_t admcap) {
  const int64_t nlpad = ((ix.nl_max + 15) / 16) * 16;
  return (size_t)ix.L * nlpad + (size_t)admcap * 12 + (size_t)(admcap + 1) * 16 + NRHO * 16 +
         PDET_MAX_L * 4;
}

size_t slot_bytes(const Index& ix) { return slot_bytes_at(ix, total_leaves(ix)); }

namespace {
// (Re)allocates `want` slots whose lists hold min(nl_i, cap) entries per tree.
void alloc_slots(const Index& ix, QueryWorkspace& ws, int64_t want, int64_t cap, hipStream_t s) {
  const int64_t nlpad = ((ix.nl_max + 15) / 16) * 16;
  const int64_t admcap = list_entries(ix, cap);
  ws.rho.release(); ws.admb.release(); ws.adm2.release(); ws.t2.release(); ws.crr.release();
  ws.lcnt.release(); ws.bandc.release();
  ws.rho.alloc((size_t)want * ix.L * nlpad);
  ws.admb.alloc((size_t)want * admcap * 12);
  ws.adm2.alloc((size_t)want * (admcap + 1) * 16);
  ws.t2.alloc((size_t)want * NRHO * 4);
  ws.crr.alloc((size_t)want * NRHO * 8);
  ws.lcnt.alloc((size_t)want * PDET_MAX_L * 4);
  ws.bandc.alloc((size_t)want * NRHO * 4);
  // the dense round table starts "never admitted"; a query that writes it restores it
  PDET_HIP(hipMemsetAsync(ws.rho.p, 0xff, ws.rho.bytes, s));
  ws.nslots = want;
  ws.list_cap = cap;
}
}  // namespace

// Sizes the workspace for a batch of nq queries: per-query arrays, and as many query slots
// (concurrent per-query scratch) as `budget` bytes allow (0: a third of free memory, at
// most 48 GiB; memory held by the block cache counts as free). Slots normally hold every
// leaf of every tree. With cap_lists, an index whose full-capacity slots would number fewer
// than min(nq, TARGET_SLOTS) in that budget caps each tree's list at
// max(MIN_LIST_CAP, nl_max / LIST_CAP_DIV) entries instead (the default budget may then
// grow to a third of free memory) and keeps RETRY_SLOTS full-capacity slots for the
// queries that overflow them. Allocation happens here, never during a launch sequence.
void reserve_workspace(const Index& ix, QueryWorkspace& ws, int64_t nq, size_t budget,
                       hipStream_t s, bool cap_lists) {
  const int64_t nl_all = std::max<int64_t>(ix.nl_max, 1);
  const bool resize = cap_lists && ws.cap_req != ix.list_cap;
  if (resize || ws.nslots == 0 || (ws.nslots < nq && ws.nslots < ws.nslots_max)) {
    size_t avail = 0;
    const bool dflt = budget == 0;
    if (dflt) {
      size_t freeb = 0, totalb = 0;
      PDET_HIP(hipMemGetInfo(&freeb, &totalb));
      avail = freeb + ws.bytes() + cache_held();
      budget = std::min<size_t>(avail / 3, (size_t)48 << 30);
    }
    const int64_t target = std::max<int64_t>(1, std::min<int64_t>(nq, TARGET_SLOTS));
    int64_t cap = nl_all;
    if (cap_lists && ix.list_cap > 0) {
      cap = std::min<int64_t>(ix.list_cap, nl_all);
      if (cap < nl_all) {
        const size_t retry = (size_t)RETRY_SLOTS * slot_bytes(ix);
        budget = budget > retry ? budget - retry : slot_bytes_at(ix, list_entries(ix, cap));
      }
    } else if (cap_lists && (int64_t)(budget / slot_bytes(ix)) < target) {
      // The capacity depends on the index alone (a sixteenth of the largest tree's leaves,
      // at least MIN_LIST_CAP), so repeated calls size the same blocks.
      const int64_t c = std::max<int64_t>(MIN_LIST_CAP, nl_all / LIST_CAP_DIV);
      if (c < nl_all) {
        if (dflt) budget = std::max<size_t>(budget, avail / 3);
        // full-capacity retry slots come out of the same budget
        const size_t retry = (size_t)RETRY_SLOTS * slot_bytes(ix);
        cap = c;
        budget = budget > retry ? budget - retry : 0;
      }
    }
    const size_t per_slot = slot_bytes_at(ix, list_entries(ix, cap));
    int64_t slots_cap = std::max<int64_t>(1, (int64_t)(budget / per_slot));
    // capped slots: TARGET_SLOTS fill the device; more would only change the block sizes
    if (cap < nl_all) slots_cap = std::min<int64_t>(slots_cap, TARGET_SLOTS);
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(nq, slots_cap));
    if (want > ws.nslots || cap != ws.list_cap) alloc_slots(ix, ws, want, cap, s);
    ws.nslots_max = slots_cap;
    if (cap_lists) ws.cap_req = ix.list_cap;
    if (cap < nl_all) {
      if (!ws.full) ws.full.reset(new QueryWorkspace());
      if (ws.full->nslots == 0) alloc_slots(ix, *ws.full, RETRY_SLOTS, nl_all, s);
    } else {
      ws.full.reset();
    }
  }
  if (ws.nq_cap < nq) {
    ws.dk.alloc((size_t)nq * 4); ws.dc.alloc((size_t)nq * 8);
    ws.dT.alloc((size_t)nq * 8); ws.doff.alloc((size_t)nq * 8);
    ws.qp.alloc((size_t)nq * PDET_MAX_L * PDET_MAX_K * 4);
    ws.ovf.alloc((size_t)(nq + 1) * 4);
    ws.h_k.alloc((size_t)nq * 4); ws.h_c.alloc((size_t)nq * 8);
    ws.h_T.alloc((size_t)nq * 8); ws.h_off.alloc((size_t)nq * 8);
    ws.nq_cap = nq;
  }
  if (!ws.h_ovf.p) ws.h_ovf.alloc(4);
  PDET_HIP(hipStreamSynchronize(s));
}

namespace {
// Points the per-slot arrays of `a` at the slots of workspace `sw`: tree i's leaf-list
// region holds min(nl_i, sw.list_cap) entries.
void bind_slots(const Index& ix, QArgs& a, QueryWorkspace& sw) {
  const int64_t cap = sw.list_cap;
  const int64_t admcap = list_entries(ix, cap);
  const int64_t nslots = sw.nslots;
  int64_t o = 0;
  for (int i = 0; i < ix.L; ++i) {
    const int64_t li = std::min<int64_t>(ix.nl[i], cap);
    a.nlo[i] = o;
    a.lcap[i] = (uint32_t)li;
    o += li;
  }
  a.t2 = sw.t2.as<float>();
  a.crr = sw.crr.as<double>();
  a.rho = sw.rho.as<uint8_t>();
  a.lcnt = sw.lcnt.as<uint32_t>();
  a.bandc = sw.bandc.as<uint32_t>();
  a.adm_leaf = sw.admb.as<uint32_t>();
  a.adm_w = a.adm_leaf + nslots * admcap;
  a.adm_lb = reinterpret_cast<float*>(a.adm_w + nslots * admcap);
  a.adm2_leaf = sw.adm2.as<uint32_t>();
  a.adm2_pre = a.adm2_leaf + nslots * (admcap + 1);
  a.adm_start = reinterpret_cast<int32_t*>(a.adm2_pre + nslots * (admcap + 1));
  a.adm2_lb = reinterpret_cast<float*>(a.adm_start + nslots * (admcap + 1));
  a.admcap = admcap;
}

// Everything of a batch's kernel arguments except the slot arrays; `smem` gets q_main's
// dynamic LDS.
QArgs batch_args(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws, int maxKL,
                 size_t& smem) {
  const int LK = ix.L * ix.K;
  const int64_t nlpad = ((ix.nl_max + 15) / 16) * 16;
  QArgs a{};
  a.n = ix.n; a.d = ix.d; a.L = ix.L; a.K = ix.K; a.dpad = ix.dpad;
  a.X = ix.X;
  a.xbf = ix.xbf16.as<uint16_t>();
  a.xf8 = ix.xfp8.as<uint8_t>();
  a.xscale = ix.xscale.as<float>();
  a.perm = ix.perm.as<int32_t>();
  a.leafrow = ix.leafrow.as<int32_t>();
  for (int i = 0; i < ix.L; ++i) {
    a.lstart[i] = ix.leaf_start[i].as<int32_t>();
    a.lcount[i] = ix.leaf_count[i].as<int32_t>();
    a.box[i] = ix.box[i].as<float>();
    a.gbox[i] = ix.gbox[i].as<float>();
    a.nl[i] = ix.nl[i];
    a.ng[i] = (ix.nl[i] + GL - 1) / GL;
  }
  a.nlpad = nlpad;
  a.lb_per_die = (int)cdiv(cdiv(ix.nl_max, QR_THREADS), NXCD);
  a.Q = qc.Q;
  a.qp = ws.qp.as<float>();
  a.qk = ws.dk.as<int32_t>();
  a.qT = ws.dT.as<int64_t>();
  a.qoff = ws.doff.as<int64_t>();
  a.qc = ws.dc.as<double>();
  a.uniform = ws.uniform ? 1 : 0;
  a.uk = ws.uk;
  a.uT = ws.uT;
  a.uc = ws.uc;
  a.ids = qc.ids;
  a.dists = qc.dists;
  a.qstats = qc.qstats;
  a.rescore = qc.rescore;
  a.rcap = std::max(0, std::min(RCAP_MAX, ix.rcap));
  // lanes per candidate: enough that each lane's share of a row is at most nch 16-byte loads
  auto lanes_for = [](int64_t chunks, int nch) {
    int l = 4;
    while (l < 64 && (int64_t)l * nch < chunks) l <<= 1;
    return l;
  };
  const int64_t ch32 = (ix.d % 4 == 0) ? ix.d / 4 : ix.d;
  a.lpc32 = lanes_for(ch32, NCH32);
  a.lpc = qc.precision == PDET_FP32
              ? a.lpc32
              : lanes_for(qc.precision == PDET_BF16 ? ix.dpad / 8 : ix.dpad / 16, NCHLP);
  a.r_min = qc.r_min;
  a.eps = qc.eps;
  int NM = 1;
  while (NM < maxKL + CBMIN) NM <<= 1;
  a.NM = NM;
  const int dq = (qc.precision == PDET_FP32) ? ((ix.d + 3) & ~3) : ix.dpad;
  smem = (size_t)NM * 12 + (size_t)dq * 12 + (size_t)LK * 4;
  // with the kernel's static LDS (under 16 KiB) a workgroup stays within 64 KiB
  PDET_REQUIRE(smem <= 48 * 1024, PDET_EUNSUPPORTED,
               "d and k * rescore too large for the query workgroup's LDS");
  a.qmap = nullptr;
  a.ovf = ws.ovf.as<uint32_t>();
  a.cand = qc.cand;
  a.cand_cap = qc.cand_cap;
  return a;
}

// Candidate target beta * n from which the low-precision search runs as q_main_lowp_long,
// if that kernel then fits at least a third more workgroups per CU (a large top-k buffer or
// a long query row can make LDS the limit instead; seven against six did not pay for the
// spills on 10M points of d = 256).
constexpr double LONG_WALK_T = 50000.0;

template <int PREC>
bool use_long_walk(const Index& ix, const QueryConfig& qc, size_t smem) {
  if (qc.beta * (double)ix.n < LONG_WALK_T) return false;
  int wg_long = 0, wg_short = 0;
  PDET_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &wg_long, reinterpret_cast<const void*>(&q_main_lowp_long<PREC>), QM, smem));
  PDET_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &wg_short, reinterpret_cast<const void*>(&q_main_lowp<PREC>), QM, smem));
  return 3 * wg_long >= 4 * wg_short;
}

// Per chunk of `nslots` queries of the nq the arguments select: thresholds, round
// indices, search.
void launch_chunks(const Index& ix, const QueryConfig& qc, QArgs a, int64_t nq, int64_t nslots,
                   size_t smem, hipStream_t s, bool timed, pdet_timing& tm) {
  const bool long_walk =
      qc.precision == PDET_BF16       ? use_long_walk<PDET_BF16>(ix, qc, smem)
      : qc.precision == PDET_FP8_E4M3 ? use_long_walk<PDET_FP8_E4M3>(ix, qc, smem)
                                      : false;
  for (int64_t q0 = 0; q0 < nq; q0 += nslots) {
    a.q0 = q0;
    a.nslots = (int)std::min<int64_t>(nslots, nq - q0);
    {
      Span sp(s, timed ? &tm.query_rho_ms : nullptr);
      hipLaunchKernelGGL(q_setup, dim3(cdiv(a.nslots, 64)), dim3(64), 0, s, a);
      PDET_HIP(hipGetLastError());
      // runs of query tiles per workgroup: long enough to amortise the block's group boxes,
      // short enough that the chunk still gives about QR_TARGET_WG workgroups
      const int64_t ntile = cdiv(a.nslots, QT);
      const int64_t nblk = (int64_t)NXCD * a.lb_per_die * ix.L;
      a.qr_tiles = (int)std::max<int64_t>(
          1, std::min<int64_t>(QR_TILES_MAX, ntile * nblk / QR_TARGET_WG));
      if (a.qr_tiles == 1) {
        const dim3 grid((uint32_t)(NXCD * ntile), (uint32_t)a.lb_per_die, (uint32_t)ix.L);
        if (ix.K == 16)
          hipLaunchKernelGGL(q_rho_tile<16>, grid, dim3(QR_THREADS), 0, s, a);
        else
          hipLaunchKernelGGL(q_rho_tile<0>, grid, dim3(QR_THREADS), 0, s, a);
      } else {
        const dim3 grid((uint32_t)(NXCD * a.lb_per_die), (uint32_t)ix.L,
                        (uint32_t)cdiv(ntile, a.qr_tiles));
        if (ix.K == 16)
          hipLaunchKernelGGL(q_rho_runs<16>, grid, dim3(QR_THREADS), 0, s, a);
        else
          hipLaunchKernelGGL(q_rho_runs<0>, grid, dim3(QR_THREADS), 0, s, a);
      }
      PDET_HIP(hipGetLastError());
      sp.finish();
    }
    Span sp(s, timed ? &tm.query_main_ms : nullptr);
    switch (qc.precision) {
      case PDET_FP32:
        hipLaunchKernelGGL(q_main_f32, dim3(a.nslots), dim3(QM), smem, s, a);
        break;
      case PDET_BF16:
        if (long_walk)
          hipLaunchKernelGGL(q_main_lowp_long<PDET_BF16>, dim3(a.nslots), dim3(QM), smem, s, a);
        else
          hipLaunchKernelGGL(q_main_lowp<PDET_BF16>, dim3(a.nslots), dim3(QM), smem, s, a);
        break;
      default:
        if (long_walk)
          hipLaunchKernelGGL(q_main_lowp_long<PDET_FP8_E4M3>, dim3(a.nslots), dim3(QM), smem, s,
                             a);
        else
          hipLaunchKernelGGL(q_main_lowp<PDET_FP8_E4M3>, dim3(a.nslots), dim3(QM), smem, s, a);
        break;
    }
    PDET_HIP(hipGetLastError());
    sp.finish();
    if (timed) ++tm.query_main_launches;
  }
}
}  // namespace

// Enqueues the whole query sequence on stream s (parameter upload from the pinned staging,
// query projection, then per chunk of slots: thresholds, round indices, search). No host
// synchronisation unless `timed` (HIP events per kernel family).
void enqueue_query(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws, int maxKL,
                   hipStream_t s, bool timed) {
  const int64_t nq = qc.nq;
  if (!ws.uniform) {
    PDET_HIP(hipMemcpyAsync(ws.dk.p, ws.h_k.p, nq * 4, hipMemcpyHostToDevice, s));
    PDET_HIP(hipMemcpyAsync(ws.dc.p, ws.h_c.p, nq * 8, hipMemcpyHostToDevice, s));
    PDET_HIP(hipMemcpyAsync(ws.dT.p, ws.h_T.p, nq * 8, hipMemcpyHostToDevice, s));
    PDET_HIP(hipMemcpyAsync(ws.doff.p, ws.h_off.p, nq * 8, hipMemcpyHostToDevice, s));
  }

  pdet_timing scratch_tm{};
  pdet_timing& tm = timed ? timer().t : scratch_tm;
  if (timed) {
    tm.query_project_ms = tm.query_rho_ms = tm.query_main_ms = 0.0;
    tm.query_main_launches = 0;
    tm.query_retried = 0;
  }
  {
    Span sp(s, timed ? &tm.query_project_ms : nullptr);
    project_points(ix, qc.Q, nq, ws.qp.as<float>(), s);
    sp.finish();
  }
  size_t smem = 0;
  QArgs a = batch_args(ix, qc, ws, maxKL, smem);
  bind_slots(ix, a, ws);
  launch_chunks(ix, qc, a, nq, ws.nslots, smem, s, timed, tm);
}

void retry_overflowed(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws, int maxKL,
                      hipStream_t s, bool timed) {
  if (!ws.capped() || qc.nq == 0) return;
  uint32_t* h = ws.h_ovf.as<uint32_t>();
  PDET_HIP(hipMemcpyAsync(h, ws.ovf.p, 4, hipMemcpyDeviceToHost, s));
  PDET_HIP(hipStreamSynchronize(s));
  const int64_t n_ovf = *h;
  if (n_ovf == 0) return;
  PDET_REQUIRE(n_ovf <= qc.nq, PDET_EDEVICE, "overflow count exceeds the batch");
  pdet_timing scratch_tm{};
  pdet_timing& tm = timed ? timer().t : scratch_tm;
  size_t smem = 0;
  QArgs a = batch_args(ix, qc, ws, maxKL, smem);
  bind_slots(ix, a, *ws.full);
  // full-capacity slots: the lists hold every leaf, so none of these overflows
  a.qmap = reinterpret_cast<const int32_t*>(ws.ovf.as<uint32_t>() + 1);
  launch_chunks(ix, qc, a, n_ovf, ws.full->nslots, smem, s, timed, tm);
  ws.retried += n_ovf;
  if (timed) tm.query_retried = n_ovf;
}

void run_query(const Index& ix, const QueryConfig& qc, hipStream_t s) {
  if (qc.nq == 0) return;
  WorkspaceLease lease(ix);
  QueryWorkspace& ws = lease.get();
  reserve_workspace(ix, ws, qc.nq, 0, s, true);
  const int maxKL = stage_params(ix, qc, ws);
  enqueue_query(ix, qc, ws, maxKL, s, timer().on);
  retry_overflowed(ix, qc, ws, maxKL, s, timer().on);
  // the workspace goes back to the pool when this returns: wait for the kernels first
  PDET_HIP(hipStreamSynchronize(s));
}

}  // namespace pdet
