// The query of Algorithm 5 as printed, without the query-phase optimisations that Section
// 6.2.2 evaluates, and the (r,c)-ANN query of Algorithm 4 - on gfx950.
//
// DET Range Query (Algorithm 3) on tree i at radius r' = eps*r: a leaf whose lower bound
// exceeds r' is pruned (16-leaf union boxes prune first, as subtrees do), a leaf whose upper
// bound is at most r' contributes all of its points, any other admitted leaf contributes the
// points whose projected distance to q' is smaller than r'. Every round re-runs the range
// query on every tree at the round's radius; S is the union of the results; stop rule A
// (|S| >= ceil(beta n) + k) is checked after each tree, stop rule B after all L trees.
//
// One workgroup per query. S is a bitmap of n bits in the query's slot (cleared by the
// workgroup first); a point is new iff its bit was clear (atomic or). New points are verified
// by exact distance (float32 data, FP64 accumulation) into a top-k list in LDS. Projected
// distances read the index's float32 hash values (kept once computed, see
// ensure_hash_values), compared in float32 with the same threshold as the optimised query.
#include "devutil.h"
#include "internal.h"

namespace pdet {
namespace {

constexpr int QL = 256;           // threads per query
constexpr int LGRP = 16;          // leaves per union box
constexpr int LPC = 16;           // lanes per candidate row in verification
constexpr int CBL = 512;          // pending candidates beside the top-k list (>= QL)
constexpr float BANDL = 1e-5f;

struct LArgs {
  int64_t n;
  int d, L, K, LK;
  const float* X;
  const float* H;               // [n][L*K] float32 hash values
  const int32_t* perm;          // [L][n]
  const int32_t* lstart[PDET_MAX_L];
  const int32_t* lcount[PDET_MAX_L];
  const float* box[PDET_MAX_L];
  const float* gbox[PDET_MAX_L];
  int64_t nl[PDET_MAX_L], ng[PDET_MAX_L];
  const float* Q;
  const float* qp;              // [nq][L*K]
  int k;
  int64_t T;
  double c, r_min, eps;
  int max_rounds;
  int rc_mode;                  // Algorithm 4: one radius, the closest point or none
  uint32_t* bitmap;             // [slots][bwords]
  int64_t bwords;
  int64_t q0;
  int NM;                       // top-k list + pending entries (power of two)
  int64_t* ids;
  float* dists;
  int32_t* qstats;
};

__device__ inline void box_bounds(const float* box, int64_t nb, int64_t b, const float* q, int K,
                                  float& lb2, float& ub2) {
  float a = 0.0f, u = 0.0f;
  for (int j = 0; j < K; ++j) {
    const float lo = box[(int64_t)j * nb + b], hi = box[(int64_t)(K + j) * nb + b];
    const float g = fmaxf(0.0f, fmaxf(lo - q[j], q[j] - hi));
    const float f = fmaxf(fabsf(q[j] - lo), fabsf(q[j] - hi));
    a = __fmaf_rn(g, g, a);
    u = __fmaf_rn(f, f, u);
  }
  lb2 = a;
  ub2 = u;
}

__device__ inline bool less_pair(double a, int32_t ia, double b, int32_t ib) {
  return a < b || (a == b && ia < ib);
}

// Bitonic sort of (distance, id) pairs, ascending, over `len` (a power of two) entries.
__device__ void sort_pairs_l(double* ld, int32_t* li, int len) {
  for (int k = 2; k <= len; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < (len >> 1); t += QL) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int p = i | j;
        const bool asc = (i & k) == 0;
        const double di = ld[i], dp = ld[p];
        const int32_t ii = li[i], ip = li[p];
        if (less_pair(dp, ip, di, ii) == asc) {
          ld[i] = dp; li[i] = ip; ld[p] = di; li[p] = ii;
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(QL) void q_literal(LArgs a) {
  extern __shared__ __align__(16) unsigned char sm[];
  double* ld = reinterpret_cast<double*>(sm);          // [NM] squared distances
  int32_t* li = reinterpret_cast<int32_t*>(ld + a.NM);  // [NM] ids
  double* qd = reinterpret_cast<double*>(li + a.NM);    // [d] the query (NM is a multiple of 2)
  float* qps = reinterpret_cast<float*>(qd + a.d);      // [L*K] projected query
  __shared__ uint32_t og[QL];                           // open groups of a chunk
  __shared__ uint32_t lv_leaf[QL];                      // admitted leaves of a chunk
  __shared__ uint32_t lv_pre[QL + 1];
  __shared__ int32_t lv_start[QL];
  __shared__ uint8_t lv_whole[QL];
  __shared__ int32_t idbuf[QL];
  __shared__ uint32_t sh_scan[QL / 64 + 1];
  __shared__ uint32_t s_nb, s_ncb, s_cnt, s_band, s_hsum, s_hmix;

  const int slot = blockIdx.x;
  const int64_t q = a.q0 + slot;
  const int tid = threadIdx.x, lane = tid & 63;
  const int k = a.k, KL = k;
  uint32_t* bm = a.bitmap + (int64_t)slot * a.bwords;
  for (int64_t w = tid; w < a.bwords; w += QL) bm[w] = 0u;
  for (int e = tid; e < a.NM; e += QL) { ld[e] = INFINITY; li[e] = INT32_MAX; }
  for (int t = tid; t < a.d; t += QL) qd[t] = (double)a.Q[q * a.d + t];
  for (int t = tid; t < a.LK; t += QL) qps[t] = a.qp[q * a.LK + t];
  if (tid == 0) { s_ncb = 0; s_band = 0; s_hsum = 0; s_hmix = 0; }
  __syncthreads();
  const uint64_t t_start = wall_clock64();

  auto merge = [&]() {
    const int used = KL + (int)uni(s_ncb);
    int len = 1;
    while (len < used) len <<= 1;
    for (int e = used + tid; e < len; e += QL) { ld[e] = INFINITY; li[e] = INT32_MAX; }
    __syncthreads();
    sort_pairs_l(ld, li, len);
    if (tid == 0) s_ncb = 0;
    __syncthreads();
  };

  int64_t nS = 0, examined = 0, visits = 0;
  uint32_t hsum = 0, hmix = 0, band = 0;
  int stop = -1, rounds = 0;
  double r = a.r_min;
  for (int rho = 0; rho < a.max_rounds && stop == -1; ++rho) {
    rounds = rho + 1;
    const double tt = a.eps * r;
    const float t2 = (float)(tt * tt);
    for (int i = 0; i < a.L && stop == -1; ++i) {
      const float* qi = qps + i * a.K;
      const int64_t nl = a.nl[i], ng = a.ng[i];
      for (int64_t g0 = 0; g0 < ng; g0 += QL) {
        // open union boxes of this chunk
        const int64_t g = g0 + tid;
        bool open = false;
        if (g < ng) {
          float lb2, ub2;
          box_bounds(a.gbox[i], ng, g, qi, a.K, lb2, ub2);
          open = lb2 <= t2 * (1.0f + BANDL);
        }
        uint32_t nog;
        const uint32_t opos = block_excl_scan<QL>(open ? 1u : 0u, sh_scan, &nog);
        if (open) og[opos] = (uint32_t)g;
        __syncthreads();
        // their leaves, QL at a time: bounds, admission, then the admitted leaves' points
        for (uint32_t j0 = 0; j0 < nog * LGRP; j0 += QL) {
          const uint32_t j = j0 + tid;
          bool adm = false, whole = false;
          int64_t leaf = 0;
          uint32_t cnt = 0;
          if (j < nog * LGRP) {
            leaf = (int64_t)og[j / LGRP] * LGRP + (j % LGRP);
            if (leaf < nl) {
              float lb2, ub2;
              box_bounds(a.box[i], nl, leaf, qi, a.K, lb2, ub2);
              if (fabsf(lb2 - t2) <= BANDL * t2 || fabsf(ub2 - t2) <= BANDL * t2) ++band;
              adm = lb2 <= t2;
              whole = ub2 <= t2;
              if (adm) cnt = (uint32_t)a.lcount[i][leaf];
            }
          }
          uint32_t nlv, P;
          const uint32_t lpos = block_excl_scan<QL>(adm ? 1u : 0u, sh_scan, &nlv);
          const uint32_t ppos = block_excl_scan<QL>(cnt, sh_scan, &P);
          if (adm) {
            lv_leaf[lpos] = (uint32_t)leaf;
            lv_pre[lpos] = ppos;
            lv_start[lpos] = a.lstart[i][leaf];
            lv_whole[lpos] = whole ? 1 : 0;
          }
          if (tid == 0) lv_pre[nlv] = P;
          __syncthreads();
          examined += nlv;
          // the admitted leaves' points, QL at a time
          for (uint32_t base = 0; base < P; base += QL) {
            visits += std::min<uint32_t>(QL, P - base);
            const uint32_t p = base + tid;
            bool nw = false;
            int32_t id = 0;
            if (tid == 0) s_nb = 0;
            __syncthreads();
            if (p < P) {
              int lo = 0, hi = (int)nlv;
              while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (lv_pre[mid] <= p) lo = mid; else hi = mid;
              }
              const int64_t pos = (int64_t)i * a.n + lv_start[lo] + (p - lv_pre[lo]);
              id = a.perm[pos];
              bool cand = lv_whole[lo] != 0;
              if (!cand) {
                // projected distance in tree i, smaller than r' (Algorithm 3)
                const float* h = a.H + (int64_t)id * a.LK + i * a.K;
                float acc = 0.0f;
                for (int jj = 0; jj < a.K; ++jj) {
                  const float df = h[jj] - qi[jj];
                  acc = __fmaf_rn(df, df, acc);
                }
                if (fabsf(acc - t2) <= BANDL * t2) ++band;
                cand = acc < t2;
              }
              if (cand) {
                const uint32_t bit = 1u << (id & 31);
                nw = (atomicOr(&bm[id >> 5], bit) & bit) == 0u;
              }
            }
            const uint64_t mask = __ballot(nw);
            uint32_t wbase = 0;
            if (lane == 0 && mask) wbase = atomicAdd(&s_nb, (uint32_t)__popcll(mask));
            wbase = __shfl(wbase, 0);
            if (nw) {
              idbuf[wbase + lanes_below_mask(mask)] = id;
              hsum += (uint32_t)id;
              hmix += mix32((uint32_t)id);
            }
            __syncthreads();
            const uint32_t nb = uni(s_nb);
            nS += nb;
            // exact distances of the new points, LPC lanes per row
            const int lg = tid & (LPC - 1), grp = tid / LPC;
            for (uint32_t c0 = 0; c0 < nb; c0 += QL / LPC) {
              const uint32_t cix = c0 + grp;
              const bool valid = cix < nb;
              const int32_t cid = valid ? idbuf[cix] : 0;
              double acc = 0.0;
              if (valid) {
                const float* xr = a.X + (int64_t)cid * a.d;
                for (int t = lg; t < a.d; t += LPC) {
                  const double df = (double)xr[t] - qd[t];
                  acc = fma(df, df, acc);
                }
              }
#pragma unroll
              for (int o = LPC / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LPC);
              if (valid && lg == 0 && less_pair(acc, cid, ld[KL - 1], li[KL - 1])) {
                const uint32_t at = atomicAdd(&s_ncb, 1u);
                ld[KL + at] = acc;
                li[KL + at] = cid;
              }
            }
            __syncthreads();
            if (uni(s_ncb) > (uint32_t)(a.NM - KL - QL)) merge();
          }
        }
      }
      if (nS >= a.T) stop = 1;   // stop rule A, checked after each tree (Algorithm 5 / 4)
    }
    if (stop == -1) {
      if (uni(s_ncb) > 0) merge();
      const double cr = a.c * r;
      if (a.rc_mode) {
        // Algorithm 4: the closest point of S if it lies within c r, else none
        stop = (ld[0] <= cr * cr) ? 2 : 0;
      } else if (nS >= k) {
        // stop rule B: at least k points of S within c r
        uint32_t cnt = 0;
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        for (int e = tid; e < KL; e += QL) cnt += (ld[e] <= cr * cr) ? 1u : 0u;
        if (cnt) atomicAdd(&s_cnt, cnt);
        __syncthreads();
        if (uni(s_cnt) >= (uint32_t)k) stop = 2;
      }
    }
    r = a.c * r;
  }
  if (uni(s_ncb) > 0) merge();
  atomicAdd(&s_hsum, hsum);
  atomicAdd(&s_hmix, hmix);
  if (band) atomicAdd(&s_band, band);
  __syncthreads();
  const bool none = a.rc_mode && stop == 0;
  for (int t = tid; t < k; t += QL) {
    a.ids[q * k + t] = (none || li[t] == INT32_MAX) ? -1 : (int64_t)li[t];
    a.dists[q * k + t] = none ? INFINITY : (float)sqrt(ld[t]);
  }
  if (tid == 0 && a.qstats) {
    int32_t* st = a.qstats + q * PDET_QSTAT_WORDS;
    st[PDET_QSTAT_ROUNDS] = rounds;
    st[PDET_QSTAT_NCAND] = (int32_t)nS;
    st[PDET_QSTAT_STOP] = stop;
    st[PDET_QSTAT_LEAVES] = (int32_t)std::min<int64_t>(examined, INT32_MAX);
    st[PDET_QSTAT_HSUM] = (int32_t)s_hsum;
    st[PDET_QSTAT_HMIX] = (int32_t)s_hmix;
    st[PDET_QSTAT_TIME] = (int32_t)std::min<uint64_t>(wall_clock64() - t_start, INT32_MAX);
    st[PDET_QSTAT_VISITS] = (int32_t)std::min<int64_t>(visits, INT32_MAX);
    st[PDET_QSTAT_BAND_LEAF] = (int32_t)s_band;
    st[PDET_QSTAT_BAND_STOPB] = 0;
  }
}

}  // namespace

// The float32 hash values of every point (the encoder's arithmetic), computed on the first
// literal query of an index and kept with it.
const float* ensure_hash_values(const Index& ix, hipStream_t s) {
  std::lock_guard<std::mutex> g(ix.hash_mu);
  if (!ix.H.p) {
    ix.H.alloc((size_t)ix.n * ix.L * ix.K * 4);
    project_points(ix, ix.X, ix.n, ix.H.as<float>(), s);
  }
  return ix.H.as<float>();
}

void run_query_literal(const Index& ix, const QueryConfig& qc, int32_t k, double c, bool rc_mode,
                       hipStream_t s) {
  const int64_t nq = qc.nq;
  const float* H = ensure_hash_values(ix, s);
  const int LK = ix.L * ix.K;
  PooledBuf qp((size_t)nq * LK * 4);
  project_points(ix, qc.Q, nq, qp.as<float>(), s);
  const int64_t bwords = (ix.n + 31) / 32;
  // query slots: one bitmap of n bits each, at most a quarter of free memory
  size_t freeb = 0, totalb = 0;
  PDET_HIP(hipMemGetInfo(&freeb, &totalb));
  const int64_t per = bwords * 4;
  const int64_t slots = std::max<int64_t>(1, std::min<int64_t>({nq, (int64_t)2048,
                                                                (int64_t)(freeb / 4 / per)}));
  PooledBuf bitmap((size_t)slots * per);
  LArgs a{};
  a.n = ix.n; a.d = ix.d; a.L = ix.L; a.K = ix.K; a.LK = LK;
  a.X = ix.X; a.H = H; a.perm = ix.perm.as<int32_t>();
  for (int i = 0; i < ix.L; ++i) {
    a.lstart[i] = ix.leaf_start[i].as<int32_t>();
    a.lcount[i] = ix.leaf_count[i].as<int32_t>();
    a.box[i] = ix.box[i].as<float>();
    a.gbox[i] = ix.gbox[i].as<float>();
    a.nl[i] = ix.nl[i];
    a.ng[i] = (ix.nl[i] + LGRP - 1) / LGRP;
  }
  a.Q = qc.Q;
  a.qp = qp.as<float>();
  a.k = k;
  const double beta = qc.beta >= 0.0 ? qc.beta : theoretical_beta(ix.K, ix.L, c);
  a.T = (int64_t)std::ceil(beta * (double)ix.n) + (rc_mode ? 1 : k);
  a.c = c;
  a.r_min = qc.r_min;
  a.eps = qc.eps;
  a.max_rounds = rc_mode ? 1 : PDET_MAX_ROUNDS;
  a.rc_mode = rc_mode ? 1 : 0;
  a.bitmap = bitmap.as<uint32_t>();
  a.bwords = bwords;
  int NM = 1;
  while (NM < k + CBL) NM <<= 1;
  a.NM = NM;
  a.ids = qc.ids;
  a.dists = qc.dists;
  a.qstats = qc.qstats;
  const size_t smem = (size_t)NM * 12 + (size_t)ix.d * 8 + (size_t)LK * 4;
  PDET_REQUIRE(smem <= 56 * 1024, PDET_EUNSUPPORTED, "d and k too large for the literal query");
  for (int64_t q0 = 0; q0 < nq; q0 += slots) {
    a.q0 = q0;
    const int64_t m = std::min<int64_t>(slots, nq - q0);
    hipLaunchKernelGGL(q_literal, dim3((unsigned)m), dim3(QL), smem, s, a);
    PDET_HIP(hipGetLastError());
  }
  // the temporaries go back to the pool when this returns
  PDET_HIP(hipStreamSynchronize(s));
}

}  // namespace pdet

using namespace pdet;

extern "C" {

pdet_status pdet_query_literal(const pdet_index* idx, const float* queries, int64_t nq,
                               const pdet_query_params* p, int64_t* ids, float* dists,
                               int32_t* qstats, void* stream) {
  return guarded([&] {
    PDET_REQUIRE(idx && p, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(!p->k_per_query && !p->c_per_query, PDET_EINVAL,
                 "pdet_query_literal takes uniform k and c");
    PDET_REQUIRE(p->precision == PDET_FP32, PDET_EINVAL,
                 "pdet_query_literal verifies in float32 only");
    PDET_REQUIRE(nq >= 0, PDET_EINVAL, "nq must be >= 0");
    PDET_REQUIRE(nq == 0 || (queries && ids && dists), PDET_EINVAL, "NULL queries or outputs");
    PDET_REQUIRE(std::isfinite(p->beta), PDET_EINVAL, "beta must be finite");
    PDET_REQUIRE(p->k >= 1 && p->k <= idx->n && p->k <= PDET_MAX_TOPK, PDET_EINVAL,
                 "k must be in [1, min(n, 1024)]");
    PDET_REQUIRE(p->c > 1.0 && std::isfinite(p->c), PDET_EINVAL, "c must be > 1");
    double r_min = p->r_min;
    if (r_min <= 0.0) {
      PDET_REQUIRE(idx->tuned_r_min > 0.0, PDET_EINVAL,
                   "r_min <= 0 selects the tuned radius, but the index has not been tuned");
      r_min = idx->tuned_r_min;
    }
    PDET_REQUIRE(std::isfinite(r_min), PDET_EINVAL, "r_min must be finite");
    if (nq == 0) return;
    QueryConfig qc{};
    qc.Q = queries;
    qc.nq = nq;
    qc.beta = p->beta;
    qc.r_min = r_min;
    qc.eps = (p->eps > 0.0) ? p->eps : epsilon(idx->K, idx->L);
    qc.precision = PDET_FP32;
    qc.rescore = 1;
    qc.ids = ids;
    qc.dists = dists;
    qc.qstats = qstats;
    run_query_literal(*idx, qc, p->k, p->c, false, static_cast<hipStream_t>(stream));
  });
}

pdet_status pdet_rc_ann(const pdet_index* idx, const float* queries, int64_t nq, double r,
                        double c, double beta, double eps, int64_t* ids, float* dists,
                        int32_t* qstats, void* stream) {
  return guarded([&] {
    PDET_REQUIRE(idx, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(nq >= 0, PDET_EINVAL, "nq must be >= 0");
    PDET_REQUIRE(nq == 0 || (queries && ids && dists), PDET_EINVAL, "NULL queries or outputs");
    PDET_REQUIRE(r > 0.0 && std::isfinite(r), PDET_EINVAL, "r must be > 0");
    PDET_REQUIRE(c > 1.0 && std::isfinite(c), PDET_EINVAL, "c must be > 1");
    PDET_REQUIRE(std::isfinite(beta), PDET_EINVAL, "beta must be finite");
    if (nq == 0) return;
    QueryConfig qc{};
    qc.Q = queries;
    qc.nq = nq;
    qc.beta = beta;
    qc.r_min = r;
    qc.eps = (eps > 0.0) ? eps : epsilon(idx->K, idx->L);
    qc.precision = PDET_FP32;
    qc.rescore = 1;
    qc.ids = ids;
    qc.dists = dists;
    qc.qstats = qstats;
    run_query_literal(*idx, qc, 1, c, true, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
