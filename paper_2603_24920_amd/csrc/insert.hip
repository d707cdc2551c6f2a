// Online insertion into the resident DE-Trees (Algorithm 2's insertion loop, Section 3.2).
//
// Points are inserted one at a time, in id order: each goes to the leaf whose region holds
// its code; a target that already holds max_leaf points is split (on the dimension the
// node-split rule picks over the points it holds) until the point finds room, unless it is
// fully refined. The resident tree is the bulk tree with the empty children of its splits
// kept as empty leaves, and every first-layer node exists from the start.
//
// Points of different first-layer nodes never meet, so one wave takes one touched
// first-layer node (tree, key) and inserts its new points in order. It works on the node's
// complete leaf list (empty leaves included) in depth-first order:
//  * a node that an earlier insertion touched has its empty leaves stored (ix.empt);
//  * an untouched node is still a bulk subtree, and its empty leaves follow from its
//    non-empty ones. In the bulk rule a split leaves a child empty only when the points
//    agree on the next bit of every unrefined dimension (a one-sided division is the worst
//    the rule can pick), and then the split takes the smallest unrefined dimension. A split
//    with two non-empty children is on a dimension that every leaf below refines and whose
//    next bit orders the leaves as a run of 0s then a run of 1s; among such dimensions the
//    split one has the smallest (|#1 - #0|, dimension), since a smaller one would have been
//    picked instead. The counts come from the leaves' sizes.
// The trees are then laid out again (untouched nodes shifted, touched ones written from
// their lists) and the leaf tables rebuilt by the build's own final stage.
#include <cstring>

#include "devutil.h"
#include "internal.h"

namespace pdet {
namespace {

constexpr int STK = 128;   // replay stack: deeper than K * (bits - 1) + 1 for every K, Nr

struct LRec {              // a leaf of a touched first-layer node (48 bytes)
  uint16_t h[KP];          // node id per dimension
  int32_t win_lo, win_hi;  // old permutation positions its old points come from
  int32_t count;           // points it holds
  int32_t old_leaf;        // >= 0: an old leaf not split since (its window is all its own)
};

struct Touch {             // a first-layer node that receives points in this call
  int32_t tree, key;
  int32_t nlo, nhi;        // its new points: sorted positions nlo..nhi-1 of the tree
  int32_t la, lb;          // its old non-empty leaves (ordinals)
  int32_t ps, pe;          // its old permutation positions
  int32_t elo, ehi;        // its stored empty leaves (records of ix.empt)
  int32_t mat;             // 1: the empty leaves are stored
  int32_t cap;             // records (and list slots) of its region
  uint32_t rec0, lid0;     // its region in the record and lid pools
  int32_t len, nonempty, status, pad;   // results; status 1: capacity, 2: inconsistent
};

struct InsArgs {
  Touch* touch;
  LRec* rec;
  int32_t* dfs;
  int32_t* lid;              // pool: record of each old position of a split old leaf
  int32_t* nlid;             // [L][m]: record of each sorted new point
  const uint4* nrows;        // [L][m] sorted new code rows
  const int32_t* nids;       // [L][m] sorted new point (0-based among the new ones)
  const int32_t* perm;       // old [L][n_old]
  const uint8_t* codes;      // [L][n_total][KP]
  const uint16_t* leaf_hidx[PDET_MAX_L];
  const int32_t* leaf_start[PDET_MAX_L];
  const int32_t* leaf_count[PDET_MAX_L];
  const EmptyRec* empt;
  uint32_t* worst;           // largest status over the nodes
  int64_t n_old, n_total, m;
  int K, bits, max_leaf;
};

__device__ inline uint32_t code_at(const uint4& v, int j) {
  const uint32_t w = (j < 8) ? ((j < 4) ? v.x : v.y) : ((j < 12) ? v.z : v.w);
  return (w >> (8 * (j & 3))) & 255u;
}
__device__ inline uint32_t h_at(const uint4& a, const uint4& b, int j) {
  const uint4& v = (j < 8) ? a : b;
  const int q = (j & 7) >> 1;
  const uint32_t w = (q < 2) ? (q == 0 ? v.x : v.y) : (q == 2 ? v.z : v.w);
  return (w >> (16 * (j & 1))) & 0xffffu;
}
__device__ inline int depth_of(uint32_t h) { return 31 - __clz((int)h); }

__device__ inline int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Does the node (h0, h1) hold the code row?
__device__ inline bool holds(const uint4& h0, const uint4& h1, const uint4& row, int K,
                             int bits) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    if (j < K) {
      const uint32_t h = h_at(h0, h1, j);
      const int dep = depth_of(h);
      ok = ok && ((code_at(row, j) >> (bits - dep)) == (h ^ (1u << dep)));
    }
  }
  return ok;
}

__device__ inline void load_h(const uint16_t* p, uint4& h0, uint4& h1) {
  h0 = reinterpret_cast<const uint4*>(p)[0];
  h1 = reinterpret_cast<const uint4*>(p)[1];
}

// The first-layer node of key `key`: one refined bit per dimension.
__device__ inline void root_h(int key, int K, uint16_t* h) {
  for (int j = 0; j < KP; ++j)
    h[j] = (j < K) ? (uint16_t)(2u | ((uint32_t)(key >> (K - 1 - j)) & 1u)) : (uint16_t)0;
}

// ---- per touched first-layer node: complete leaf list, then the sequential insertion
__global__ __launch_bounds__(64) void ins_subtree(InsArgs a) {
  Touch& tc = a.touch[blockIdx.x];
  const int lane = threadIdx.x;
  const int t = tc.tree;
  LRec* R = a.rec + tc.rec0;
  int32_t* D = a.dfs + tc.rec0;
  int32_t* lid = a.lid + tc.lid0;
  const int cap = tc.cap;
  const uint16_t* LH = a.leaf_hidx[t];
  const int32_t* LS = a.leaf_start[t];
  const int32_t* LC = a.leaf_count[t];
  int len = 0, status = 0;

  __shared__ __align__(16) uint16_t st_h[STK][KP];
  __shared__ int st_a[STK], st_b[STK];

  // -- 1. the complete leaf list in depth-first order
  if (tc.mat) {
    const int E = tc.ehi - tc.elo, N = tc.lb - tc.la;
    len = E + N;
    if (len > cap) {
      status = 1;
    } else {
      for (int e = lane; e < E; e += 64) {
        const EmptyRec& er = a.empt[tc.elo + e];
        if (er.local < 0 || er.local >= len) { status = 2; continue; }
        LRec r;
        for (int j = 0; j < KP; ++j) r.h[j] = er.h[j];
        r.win_lo = r.win_hi = 0; r.count = 0; r.old_leaf = -1;
        R[er.local] = r;
        D[er.local] = er.local;
      }
      for (int i = lane; i < N; i += 64) {
        // empty leaves before non-empty leaf i: those e with (local_e - e) <= i, a
        // non-decreasing quantity in e
        int lo = 0, hi = E;
        while (lo < hi) {
          const int md = (lo + hi) >> 1;
          if (a.empt[tc.elo + md].local - md <= i) lo = md + 1; else hi = md;
        }
        const int pos = i + lo, l = tc.la + i;
        LRec r;
        for (int j = 0; j < KP; ++j) r.h[j] = LH[(int64_t)l * KP + j];
        r.win_lo = LS[l]; r.win_hi = LS[l] + LC[l]; r.count = LC[l]; r.old_leaf = l;
        R[pos] = r;
        D[pos] = pos;
      }
    }
    if (__ballot(status == 2)) status = 2;   // a stored empty leaf out of place
  } else {
    // replay of the bulk splits from the non-empty leaves
    if (lane == 0) {
      root_h(tc.key, a.K, st_h[0]);
      st_a[0] = tc.la;
      st_b[0] = tc.lb;
    }
    int sp = 1;
    __syncthreads();
    while (sp > 0 && status == 0) {
      --sp;
      const int na = st_a[sp], nb = st_b[sp];
      uint4 h0, h1;
      load_h(st_h[sp], h0, h1);
      __syncthreads();
      bool same = false;
      if (nb == na + 1) {
        uint4 g0, g1;
        load_h(LH + (int64_t)na * KP, g0, g1);
        same = g0.x == h0.x && g0.y == h0.y && g0.z == h0.z && g0.w == h0.w && g1.x == h1.x &&
               g1.y == h1.y && g1.z == h1.z && g1.w == h1.w;
      }
      if (nb == na || same) {
        if (len >= cap) { status = 1; break; }
        if (lane == 0) {
          LRec r;
          *reinterpret_cast<uint4*>(r.h) = h0;
          *reinterpret_cast<uint4*>(r.h + 8) = h1;
          if (same) {
            r.win_lo = LS[na]; r.win_hi = LS[na] + LC[na]; r.count = LC[na]; r.old_leaf = na;
          } else {
            r.win_lo = r.win_hi = 0; r.count = 0; r.old_leaf = -1;
          }
          R[len] = r;
          D[len] = len;
        }
        ++len;
        continue;
      }
      // an internal node: find its split. Per dimension (bit j of the masks): some leaf
      // does not refine it further, some leaf has its next bit 0 / 1, a 1 precedes a 0;
      // and the leaves' point counts (bit 1) and leaf counts (bit 0). Every leaf row is
      // read once per node.
      uint32_t unref_m = 0;
#pragma unroll
      for (int j = 0; j < KP; ++j)
        if (j < a.K && depth_of(h_at(h0, h1, j)) < a.bits) unref_m |= 1u << j;
      uint32_t notref_m = 0, any0_m = 0, any1_m = 0, dec_m = 0;
      int c1[KP], n0[KP], msum = 0;
#pragma unroll
      for (int j = 0; j < KP; ++j) { c1[j] = 0; n0[j] = 0; }
      for (int base = na; base < nb; base += 64) {
        const int l = base + lane;
        if (l < nb) {
          uint4 r0, r1, p0 = make_uint4(0, 0, 0, 0), p1 = make_uint4(0, 0, 0, 0);
          load_h(LH + (int64_t)l * KP, r0, r1);
          if (l > na) load_h(LH + (int64_t)(l - 1) * KP, p0, p1);
          const int cnt = LC[l];
          msum += cnt;
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            if ((unref_m >> j) & 1u) {
              const int dep = depth_of(h_at(h0, h1, j));
              const uint32_t lh = h_at(r0, r1, j);
              const int ld = depth_of(lh);
              if (ld <= dep) {
                notref_m |= 1u << j;
              } else if ((lh >> (ld - dep - 1)) & 1u) {
                any1_m |= 1u << j;
                c1[j] += cnt;
              } else {
                any0_m |= 1u << j;
                n0[j] += 1;
                if (l > na) {
                  const uint32_t ph = h_at(p0, p1, j);
                  const int pd = depth_of(ph);
                  if (pd > dep && ((ph >> (pd - dep - 1)) & 1u)) dec_m |= 1u << j;
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        notref_m |= __shfl_xor(notref_m, o);
        any0_m |= __shfl_xor(any0_m, o);
        any1_m |= __shfl_xor(any1_m, o);
        dec_m |= __shfl_xor(dec_m, o);
      }
      msum = wave_sum_i(msum);
      const uint32_t cand = unref_m & ~notref_m & ~dec_m & any0_m & any1_m;
      int best = -1, best_score = 0, best_n0 = 0;
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        if ((cand >> j) & 1u) {
          const int cj = wave_sum_i(c1[j]), nj = wave_sum_i(n0[j]);
          const int score = abs(2 * cj - msum);
          if (best < 0 || score < best_score) { best = j; best_score = score; best_n0 = nj; }
        }
      }
      const int first = unref_m ? __ffs((int)unref_m) - 1 : -1;
      const bool f_ok = first >= 0 && !((notref_m >> first) & 1u) &&
                        (((any0_m >> first) & 1u) != ((any1_m >> first) & 1u));
      const int f_bit = first >= 0 ? (int)((any1_m >> first) & 1u) : 0;
      if (sp + 2 > STK || first < 0 || (best < 0 && !f_ok)) { status = 2; break; }
      const int j = best >= 0 ? best : first;
      // children: push bit 1 first so that bit 0 comes off the stack first
      int a1, b1, a0, b0;
      if (best >= 0) {
        a0 = na; b0 = na + best_n0; a1 = b0; b1 = nb;
      } else if (f_bit == 0) {
        a0 = na; b0 = nb; a1 = nb; b1 = nb;
      } else {
        a0 = na; b0 = na; a1 = na; b1 = nb;
      }
      if (lane < KP) {
        const uint32_t hv = h_at(h0, h1, lane);
        const uint32_t ch = (lane == j) ? (hv << 1) : hv;
        st_h[sp][lane] = (uint16_t)(lane == j ? (ch | 1u) : ch);
        st_h[sp + 1][lane] = (uint16_t)ch;
      }
      if (lane == 0) {
        st_a[sp] = a1; st_b[sp] = b1;
        st_a[sp + 1] = a0; st_b[sp + 1] = b0;
      }
      sp += 2;
      __syncthreads();
    }
  }
  __syncthreads();
  int nrec = len;

  // -- 2. the new points, in order
  const int64_t tm = (int64_t)t * a.m;
  for (int q = tc.nlo; q < tc.nhi && status == 0; ++q) {
    const uint4 row = a.nrows[tm + q];
    int pos = -1;
    for (int base = 0; base < len; base += 64) {
      const int p = base + lane;
      bool hit = false;
      if (p < len) {
        uint4 h0, h1;
        load_h(R[D[p]].h, h0, h1);
        hit = holds(h0, h1, row, a.K, a.bits);
      }
      const uint64_t bal = __ballot(hit);
      if (bal) { pos = base + __ffsll((long long)bal) - 1; break; }
    }
    if (pos < 0) { status = 2; break; }
    int X = D[pos];
    while (true) {
      const LRec rx = R[X];
      if (rx.count < a.max_leaf) break;
      uint4 h0, h1;
      load_h(rx.h, h0, h1);
      const bool whole = rx.old_leaf >= 0;
      // count the next bit of every unrefined dimension over the points X holds
      int c[KP];
#pragma unroll
      for (int j = 0; j < KP; ++j) c[j] = 0;
      auto add = [&](const uint4& cr) {
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          if (j < a.K) {
            const int dep = depth_of(h_at(h0, h1, j));
            if (dep < a.bits) c[j] += (int)((code_at(cr, j) >> (a.bits - 1 - dep)) & 1u);
          }
        }
      };
      for (int p = rx.win_lo + lane; p < rx.win_hi; p += 64) {
        if (whole || lid[p - tc.ps] == X) {
          const int32_t id = a.perm[(int64_t)t * a.n_old + p];
          add(*reinterpret_cast<const uint4*>(a.codes + ((int64_t)t * a.n_total + id) * KP));
        }
      }
      for (int k = tc.nlo + lane; k < q; k += 64)
        if (a.nlid[tm + k] == X) add(a.nrows[tm + k]);
      int best = -1, best_score = 0, best_c1 = 0;
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        if (j < a.K) {
          const int dep = depth_of(h_at(h0, h1, j));
          const int cj = wave_sum_i(c[j]);
          if (dep < a.bits) {
            const int score = abs(2 * cj - rx.count);
            if (best < 0 || score < best_score) { best = j; best_score = score; best_c1 = cj; }
          }
        }
      }
      if (best < 0) break;   // fully refined: the point goes in regardless
      if (nrec + 2 > cap || len + 1 > cap) { status = 1; break; }
      const int A = nrec, B = nrec + 1;
      nrec += 2;
      const int dep = depth_of(h_at(h0, h1, best));
      if (lane < 2) {
        LRec r;
        *reinterpret_cast<uint4*>(r.h) = h0;
        *reinterpret_cast<uint4*>(r.h + 8) = h1;
        r.h[best] = (uint16_t)((h_at(h0, h1, best) << 1) | (uint32_t)lane);
        r.win_lo = rx.win_lo; r.win_hi = rx.win_hi;
        r.count = lane ? best_c1 : rx.count - best_c1;
        r.old_leaf = -1;
        R[lane ? B : A] = r;
      }
      // the points of X move to the child of their bit
      for (int p = rx.win_lo + lane; p < rx.win_hi; p += 64) {
        if (whole || lid[p - tc.ps] == X) {
          const int32_t id = a.perm[(int64_t)t * a.n_old + p];
          const uint4 cr = *reinterpret_cast<const uint4*>(a.codes + ((int64_t)t * a.n_total + id) * KP);
          lid[p - tc.ps] = ((code_at(cr, best) >> (a.bits - 1 - dep)) & 1u) ? B : A;
        }
      }
      for (int k = tc.nlo + lane; k < q; k += 64)
        if (a.nlid[tm + k] == X)
          a.nlid[tm + k] = ((code_at(a.nrows[tm + k], best) >> (a.bits - 1 - dep)) & 1u) ? B : A;
      // X's slot of the list becomes A, B
      for (int top = len - 1; top > pos; top -= 64) {
        const int idx = top - lane;
        const int32_t v = (idx > pos) ? D[idx] : 0;
        __syncthreads();
        if (idx > pos) D[idx + 1] = v;
        __syncthreads();
      }
      if (lane == 0) { D[pos] = A; D[pos + 1] = B; }
      ++len;
      __syncthreads();
      const int bq = (int)((code_at(row, best) >> (a.bits - 1 - dep)) & 1u);
      X = bq ? B : A;
      pos += bq;
    }
    if (status) break;
    if (lane == 0) {
      a.nlid[tm + q] = X;
      R[X].count += 1;
    }
    __syncthreads();
  }

  // -- 3. results
  int nonempty = 0;
  if (status == 0)
    for (int p = lane; p < len; p += 64) nonempty += R[D[p]].count > 0 ? 1 : 0;
  nonempty = wave_sum_i(nonempty);
  if (lane == 0) {
    tc.len = len;
    tc.nonempty = nonempty;
    tc.status = status;
    if (status) atomicMax(a.worst, (uint32_t)status);
  }
}

// ---- layout of the grown trees
struct FlatArgs {
  const Touch* touch;
  const LRec* rec;
  const int32_t* dfs;
  const int32_t* lid;
  const int32_t* nlid;
  const int32_t* nids;
  const int32_t* perm;       // old
  int32_t* perm_new;
  uint32_t* cnt_at;          // [L][n_total]
  uint16_t* hidx_at;         // [L][n_total][KP]
  const uint32_t* fstart;    // [L][2^K] old start of each first-layer node
  const uint32_t* nshift;    // [L][2^K] new points of the nodes before it
  const uint32_t* eoff_new;
  EmptyRec* empt_new;
  int64_t n_old, n_total, m;
  int K;
};

__global__ __launch_bounds__(64) void ins_flatten(FlatArgs a) {
  const Touch& tc = a.touch[blockIdx.x];
  const int lane = threadIdx.x;
  const int t = tc.tree;
  const int64_t g = ((int64_t)t << a.K) + tc.key;
  const LRec* R = a.rec + tc.rec0;
  const int32_t* D = a.dfs + tc.rec0;
  const int32_t* lid = a.lid + tc.lid0;
  const int64_t tm = (int64_t)t * a.m;
  const int32_t* po = a.perm + (int64_t)t * a.n_old;
  int32_t* pn = a.perm_new + (int64_t)t * a.n_total;
  int64_t cur = (int64_t)a.fstart[g] + a.nshift[g];
  uint32_t e = a.eoff_new[g];
  for (int p = 0; p < tc.len; ++p) {
    const int r = D[p];
    const LRec rr = R[r];
    if (rr.count == 0) {
      if (lane == 0) {
        EmptyRec er;
        er.local = p; er.tree = t; er.key = tc.key; er.pad = 0;
        for (int j = 0; j < KP; ++j) er.h[j] = rr.h[j];
        a.empt_new[e] = er;
      }
      ++e;
      continue;
    }
    if (lane == 0) {
      a.cnt_at[(int64_t)t * a.n_total + cur] = (uint32_t)rr.count;
      uint4* hd = reinterpret_cast<uint4*>(a.hidx_at + ((int64_t)t * a.n_total + cur) * KP);
      hd[0] = *reinterpret_cast<const uint4*>(rr.h);
      hd[1] = *reinterpret_cast<const uint4*>(rr.h + 8);
    }
    if (cur + rr.count > a.n_total) return;   // (never, for consistent leaf counts)
    int64_t w = cur;
    if (rr.old_leaf >= 0) {
      for (int i = lane; i < rr.win_hi - rr.win_lo; i += 64) pn[w + i] = po[rr.win_lo + i];
      w += rr.win_hi - rr.win_lo;
    } else {
      for (int base = rr.win_lo; base < rr.win_hi; base += 64) {
        const int q = base + lane;
        const bool in = q < rr.win_hi && lid[q - tc.ps] == r;
        const uint64_t bal = __ballot(in);
        if (in && w + lanes_below_mask(bal) < cur + rr.count) pn[w + lanes_below_mask(bal)] = po[q];
        w += __popcll(bal);
      }
    }
    if (w - cur < rr.count) {
      for (int base = tc.nlo; base < tc.nhi; base += 64) {
        const int k = base + lane;
        const bool in = k < tc.nhi && a.nlid[tm + k] == r;
        const uint64_t bal = __ballot(in);
        if (in && w + lanes_below_mask(bal) < cur + rr.count)
          pn[w + lanes_below_mask(bal)] = (int32_t)(a.n_old + a.nids[tm + k]);
        w += __popcll(bal);
      }
    }
    cur += rr.count;
  }
}

__device__ inline int fkey_of(const uint16_t* h, int K) {
  int key = 0;
  for (int j = 0; j < K; ++j) {
    const uint32_t v = h[j];
    const int dep = depth_of(v);
    key |= (int)((v >> (dep - 1)) & 1u) << (K - 1 - j);
  }
  return key;
}

struct LeafArgs {
  const uint16_t* hidx[PDET_MAX_L];
  const int32_t* start[PDET_MAX_L];
  const int32_t* count[PDET_MAX_L];
  int64_t nl[PDET_MAX_L];
};

// Size, leaf count and first leaf of every first-layer node, from the leaf tables.
__global__ void ins_stats(LeafArgs la, int K, uint32_t* fsize, uint32_t* fleaves,
                          uint32_t* ffirst) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (o >= la.nl[t]) return;
  const int64_t g = ((int64_t)t << K) + fkey_of(la.hidx[t] + o * KP, K);
  atomicAdd(&fsize[g], (uint32_t)la.count[t][o]);
  atomicAdd(&fleaves[g], 1u);
  atomicMin(&ffirst[g], (uint32_t)o);
}

// Per first-layer node: new point count, whether it is touched, its region sizes.
// Region capacity of a touched node: its known leaves and 4 slots per new point, times its
// multiplier (2 at first; after an overflow, enough for K * (bits - 1) splits below every
// leaf and every new point). A bulk node's empty leaves are not known before its replay,
// so its leaves are scaled too. cap_total[0] (64-bit) sums the capacities (a grid-stride
// loop with one atomic per block).
__global__ __launch_bounds__(256) void ins_plan(const uint32_t* nstart, const uint32_t* nend,
                                                const uint32_t* fsize, const uint32_t* fleaves,
                                                const uint32_t* eoff, const uint8_t* emat,
                                                const uint32_t* multg, int64_t total,
                                                uint32_t* ncount, uint32_t* tflag,
                                                uint32_t* capg, uint32_t* lidg,
                                                unsigned long long* cap_total) {
  __shared__ unsigned long long part[4];
  unsigned long long sum = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = nend[g] - nstart[g];
    ncount[g] = c;
    tflag[g] = c ? 1u : 0u;
    uint64_t cap = 0;
    if (c) {
      const uint64_t ec = eoff ? eoff[g + 1] - eoff[g] : 0u;
      const bool mat = emat && emat[g];
      const uint64_t base = fleaves[g] + ec, mult = multg[g];
      cap = (mat ? base : base * mult) + 4u * (uint64_t)c * mult + 64u;
    }
    capg[g] = (uint32_t)std::min<uint64_t>(cap, 0xffffffffu);
    lidg[g] = c ? fsize[g] : 0u;
    sum += cap;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long b = part[0] + part[1] + part[2] + part[3];
    if (b) atomicAdd(cap_total, b);
  }
}

__global__ void ins_widen(const Touch* touch, int64_t T, int K, uint32_t mult, uint32_t* multg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T || touch[i].status != 1) return;
  multg[((int64_t)touch[i].tree << K) + touch[i].key] = mult;
}

__global__ void ins_fill(const uint32_t* tflag_scan, const uint32_t* ncount,
                         const uint32_t* nstart, const uint32_t* fsize, const uint32_t* fleaves,
                         const uint32_t* ffirst, const uint32_t* fstart, const uint32_t* eoff,
                         const uint8_t* emat, const uint32_t* capg, const uint32_t* cap_scan,
                         const uint32_t* lid_scan, int64_t total, int K, Touch* touch) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total || ncount[g] == 0) return;
  Touch tc{};
  tc.tree = (int32_t)(g >> K);
  tc.key = (int32_t)(g & ((1ll << K) - 1));
  tc.nlo = (int32_t)nstart[g];
  tc.nhi = (int32_t)(nstart[g] + ncount[g]);
  tc.la = fleaves[g] ? (int32_t)ffirst[g] : 0;
  tc.lb = tc.la + (int32_t)fleaves[g];
  tc.ps = (int32_t)fstart[g];
  tc.pe = tc.ps + (int32_t)fsize[g];
  tc.elo = eoff ? (int32_t)eoff[g] : 0;
  tc.ehi = eoff ? (int32_t)eoff[g + 1] : 0;
  tc.mat = (emat && emat[g]) ? 1 : 0;
  tc.cap = (int32_t)capg[g];
  tc.rec0 = cap_scan[g];
  tc.lid0 = lid_scan[g];
  touch[tflag_scan[g]] = tc;
}

// Points of untouched first-layer nodes: shifted by the new points before their node.
__global__ void ins_copy_untouched(const int32_t* perm, const int32_t* leafrow, LeafArgs la,
                                   const uint32_t* ncount, const uint32_t* nshift, int64_t n_old,
                                   int64_t n_total, int L, int K, int32_t* perm_new,
                                   uint32_t* cnt_at, uint16_t* hidx_at) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (p >= n_old) return;
  const int32_t leaf = leafrow[((int64_t)t * n_old + p) * L + t];
  const uint16_t* h = la.hidx[t] + (int64_t)leaf * KP;
  const int64_t g = ((int64_t)t << K) + fkey_of(h, K);
  if (ncount[g]) return;
  const int64_t np = p + nshift[g];
  perm_new[(int64_t)t * n_total + np] = perm[(int64_t)t * n_old + p];
  if (la.start[t][leaf] == p) {
    cnt_at[(int64_t)t * n_total + np] = (uint32_t)la.count[t][leaf];
    uint4* hd = reinterpret_cast<uint4*>(hidx_at + ((int64_t)t * n_total + np) * KP);
    hd[0] = reinterpret_cast<const uint4*>(h)[0];
    hd[1] = reinterpret_cast<const uint4*>(h)[1];
  }
}

__global__ void ins_empty_counts(const uint32_t* ncount, const uint32_t* tflag_scan,
                                 const Touch* touch, const uint32_t* eoff, const uint8_t* emat,
                                 int64_t total, uint32_t* ecnt, uint8_t* emat_new) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  if (ncount[g]) {
    const Touch& tc = touch[tflag_scan[g]];
    ecnt[g] = (uint32_t)(tc.len - tc.nonempty);
    emat_new[g] = 1;
  } else {
    ecnt[g] = eoff ? eoff[g + 1] - eoff[g] : 0u;
    emat_new[g] = emat ? emat[g] : 0;
  }
}

__global__ void ins_copy_empties(const EmptyRec* old, int64_t n, const uint32_t* eoff_old,
                                 const uint32_t* eoff_new, const uint32_t* ncount, int K,
                                 EmptyRec* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const EmptyRec r = old[e];
  const int64_t g = ((int64_t)r.tree << K) + r.key;
  if (ncount[g]) return;
  out[eoff_new[g] + (e - eoff_old[g])] = r;
}

}  // namespace

void insert_points(pdet_index& ix, const float* data, int64_t n_total, hipStream_t s) {
  const int64_t n_old = ix.n, m = n_total - n_old;
  const int L = ix.L, K = ix.K;
  const int64_t NK = int64_t(1) << K, G = L * NK;
  DevBuf scan_tmp;
  std::vector<DevBuf> keep;   // old buffers, released after the final synchronisation

  // -- encode the new rows (the index is unchanged if they hold a non-finite value)
  PooledBuf ncodes((size_t)L * m * KP), nkeys((size_t)L * m * 2), mm_save(ix.colmm.bytes);
  PDET_HIP(hipMemcpyAsync(mm_save.ptr(), ix.colmm.p, ix.colmm.bytes, hipMemcpyDeviceToDevice, s));
  PDET_HIP(hipMemsetAsync(ix.nonfinite.p, 0, 4, s));
  encode_rows(ix, data + n_old * ix.d, m, ncodes.as<uint8_t>(), nkeys.as<uint16_t>(), s);
  // (checked at the first readback below: every step before the swap at the end writes
  // temporaries only, and codes are in range whatever the projections)
  uint32_t* hw = readback_words() + 48;

  // -- group the new points by (tree, first-layer node), in id order
  PooledBuf srows((size_t)L * m * KP), sids((size_t)L * m * 4), rows1((size_t)L * m * KP),
      ids1((size_t)L * m * 4), keys1((size_t)L * m * 2), nstart((size_t)G * 4),
      nend((size_t)G * 4), h8, o8;
  first_layer_sort(L, K, m, nkeys.as<uint16_t>(), reinterpret_cast<const uint4*>(ncodes.ptr()),
                   srows.as<uint4>(), sids.as<int32_t>(), rows1.as<uint4>(), ids1.as<int32_t>(),
                   keys1.as<uint16_t>(), nstart.as<uint32_t>(), nend.as<uint32_t>(), h8, o8,
                   scan_tmp, s);

  // -- all codes: the old rows, then the new ones
  DevBuf codes((size_t)L * n_total * KP);
  PDET_HIP(hipMemcpy2DAsync(codes.p, (size_t)n_total * KP, ix.codes.p, (size_t)n_old * KP,
                            (size_t)n_old * KP, L, hipMemcpyDeviceToDevice, s));
  PDET_HIP(hipMemcpy2DAsync(codes.as<uint8_t>() + (size_t)n_old * KP, (size_t)n_total * KP,
                            ncodes.ptr(), (size_t)m * KP, (size_t)m * KP, L,
                            hipMemcpyDeviceToDevice, s));

  // -- per first-layer node: old size, leaves, first leaf, start
  LeafArgs la{};
  int64_t nl_max = 0;
  for (int i = 0; i < L; ++i) {
    la.hidx[i] = ix.leaf_hidx[i].as<uint16_t>();
    la.start[i] = ix.leaf_start[i].as<int32_t>();
    la.count[i] = ix.leaf_count[i].as<int32_t>();
    la.nl[i] = ix.nl[i];
    nl_max = std::max<int64_t>(nl_max, ix.nl[i]);
  }
  PooledBuf fsize((size_t)G * 4), fleaves((size_t)G * 4), ffirst((size_t)G * 4),
      fstart((size_t)G * 4), ncount((size_t)G * 4), nshift((size_t)G * 4), tflag((size_t)G * 4),
      tscan((size_t)G * 4), capg((size_t)G * 4), capscan((size_t)G * 4), lidg((size_t)G * 4),
      lidscan((size_t)G * 4), totals(16 * 4), flags(8);
  PDET_HIP(hipMemsetAsync(fsize.ptr(), 0, fsize.bytes(), s));
  PDET_HIP(hipMemsetAsync(fleaves.ptr(), 0, fleaves.bytes(), s));
  PDET_HIP(hipMemsetAsync(ffirst.ptr(), 0xff, ffirst.bytes(), s));
  if (nl_max) {
    hipLaunchKernelGGL(ins_stats, dim3(cdiv(nl_max, 256), L), dim3(256), 0, s, la, K,
                       fsize.as<uint32_t>(), fleaves.as<uint32_t>(), ffirst.as<uint32_t>());
    PDET_HIP(hipGetLastError());
  }
  scan_rows(fsize.as<uint32_t>(), fstart.as<uint32_t>(), nullptr, L, NK, scan_tmp, s);
  const uint32_t* eoff = ix.eoff.p ? ix.eoff.as<uint32_t>() : nullptr;
  const uint8_t* emat = ix.emat.p ? ix.emat.as<uint8_t>() : nullptr;

  // -- the touched nodes, their new lists, then the layout
  PooledBuf touch, recs, dfs, lidp, nlid((size_t)L * m * 4), multg((size_t)G * 4),
      cap_total(8), ecnt((size_t)G * 4);
  DevBuf eoff_new((size_t)(G + 1) * 4), emat_new((size_t)G);
  PDET_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(multg.ptr()), 2, (size_t)G, s));
  uint32_t T = 0;
  int64_t n_empty = 0;
  for (int attempt = 0;; ++attempt) {
    PDET_HIP(hipMemsetAsync(cap_total.ptr(), 0, 8, s));
    hipLaunchKernelGGL(ins_plan, dim3((unsigned)std::min<int64_t>(cdiv(G, 256), 128)), dim3(256),
                       0, s, nstart.as<uint32_t>(),
                       nend.as<uint32_t>(), fsize.as<uint32_t>(), fleaves.as<uint32_t>(), eoff,
                       emat, multg.as<uint32_t>(), G, ncount.as<uint32_t>(),
                       tflag.as<uint32_t>(), capg.as<uint32_t>(), lidg.as<uint32_t>(),
                       cap_total.as<unsigned long long>());
    PDET_HIP(hipGetLastError());
    scan_rows(tflag.as<uint32_t>(), tscan.as<uint32_t>(), totals.as<uint32_t>(), 1, G, scan_tmp, s);
    scan_rows(capg.as<uint32_t>(), capscan.as<uint32_t>(), totals.as<uint32_t>() + 1, 1, G,
              scan_tmp, s);
    scan_rows(lidg.as<uint32_t>(), lidscan.as<uint32_t>(), totals.as<uint32_t>() + 2, 1, G,
              scan_tmp, s);
    PDET_HIP(hipMemcpyAsync(hw, totals.ptr(), 3 * 4, hipMemcpyDeviceToHost, s));
    PDET_HIP(hipMemcpyAsync(hw + 4, cap_total.ptr(), 8, hipMemcpyDeviceToHost, s));
    PDET_HIP(hipMemcpyAsync(hw + 6, ix.nonfinite.p, 4, hipMemcpyDeviceToHost, s));
    PDET_HIP(hipStreamSynchronize(s));
    if (hw[6]) {
      PDET_HIP(hipMemcpyAsync(ix.colmm.p, mm_save.ptr(), ix.colmm.bytes, hipMemcpyDeviceToDevice,
                              s));
      PDET_HIP(hipStreamSynchronize(s));
      throw Error{PDET_EINVAL, "the inserted rows hold non-finite values"};
    }
    T = hw[0];
    const uint32_t total_cap = hw[1], total_lid = hw[2];
    uint64_t cap64 = 0;
    std::memcpy(&cap64, hw + 4, 8);
    PDET_REQUIRE(cap64 < (uint64_t(1) << 31), PDET_EUNSUPPORTED,
                 "insertion: the work area of this batch exceeds 2^31 leaf records");
    touch.alloc((size_t)std::max<uint32_t>(T, 1) * sizeof(Touch));
    recs.alloc((size_t)std::max<uint32_t>(total_cap, 1) * sizeof(LRec));
    dfs.alloc((size_t)std::max<uint32_t>(total_cap, 1) * 4);
    lidp.alloc((size_t)std::max<uint32_t>(total_lid, 1) * 4);
    hipLaunchKernelGGL(ins_fill, dim3(cdiv(G, 256)), dim3(256), 0, s, tscan.as<uint32_t>(),
                       ncount.as<uint32_t>(), nstart.as<uint32_t>(), fsize.as<uint32_t>(),
                       fleaves.as<uint32_t>(), ffirst.as<uint32_t>(), fstart.as<uint32_t>(), eoff,
                       emat, capg.as<uint32_t>(), capscan.as<uint32_t>(), lidscan.as<uint32_t>(),
                       G, K, touch.as<Touch>());
    PDET_HIP(hipGetLastError());
    InsArgs a{};
    a.touch = touch.as<Touch>();
    a.rec = recs.as<LRec>();
    a.dfs = dfs.as<int32_t>();
    a.lid = lidp.as<int32_t>();
    a.nlid = nlid.as<int32_t>();
    a.nrows = srows.as<uint4>();
    a.nids = sids.as<int32_t>();
    a.perm = ix.perm.as<int32_t>();
    a.codes = codes.as<uint8_t>();
    for (int i = 0; i < L; ++i) {
      a.leaf_hidx[i] = la.hidx[i];
      a.leaf_start[i] = la.start[i];
      a.leaf_count[i] = la.count[i];
    }
    a.empt = ix.empt.p ? ix.empt.as<EmptyRec>() : nullptr;
    a.worst = flags.as<uint32_t>();
    a.n_old = n_old; a.n_total = n_total; a.m = m;
    a.K = K; a.bits = ix.bits; a.max_leaf = ix.max_leaf;
    PDET_HIP(hipMemsetAsync(flags.ptr(), 0, 4, s));
    if (T) {
      hipLaunchKernelGGL(ins_subtree, dim3(T), dim3(64), 0, s, a);
      PDET_HIP(hipGetLastError());
    }
    // empty leaves per node (valid when every node succeeded), read back with the status
    hipLaunchKernelGGL(ins_empty_counts, dim3(cdiv(G, 256)), dim3(256), 0, s,
                       ncount.as<uint32_t>(), tscan.as<uint32_t>(), touch.as<Touch>(), eoff, emat,
                       G, ecnt.as<uint32_t>(), emat_new.as<uint8_t>());
    PDET_HIP(hipGetLastError());
    scan_rows(ecnt.as<uint32_t>(), eoff_new.as<uint32_t>(), eoff_new.as<uint32_t>() + G, 1, G,
              scan_tmp, s);
    PDET_HIP(hipMemcpyAsync(hw, flags.ptr(), 4, hipMemcpyDeviceToHost, s));
    PDET_HIP(hipMemcpyAsync(hw + 1, eoff_new.as<uint32_t>() + G, 4, hipMemcpyDeviceToHost, s));
    PDET_HIP(hipStreamSynchronize(s));
    const int worst = (int)hw[0];
    n_empty = hw[1];
    PDET_REQUIRE(worst != 2, PDET_EDEVICE, "insertion: a tree's leaves are not consistent");
    if (worst == 0) break;
    PDET_REQUIRE(attempt == 0, PDET_EDEVICE, "insertion: node capacity exceeded");
    hipLaunchKernelGGL(ins_widen, dim3(cdiv(T, 256)), dim3(256), 0, s, touch.as<Touch>(),
                       (int64_t)T, K, (uint32_t)(K * (ix.bits - 1) + 2), multg.as<uint32_t>());
    PDET_HIP(hipGetLastError());
  }

  // -- new layout
  scan_rows(ncount.as<uint32_t>(), nshift.as<uint32_t>(), nullptr, L, NK, scan_tmp, s);
  DevBuf perm_new((size_t)L * n_total * 4);
  PooledBuf cnt_at((size_t)L * n_total * 4), hidx_at((size_t)L * n_total * KP * 2);
  PDET_HIP(hipMemsetAsync(cnt_at.ptr(), 0, cnt_at.bytes(), s));
  hipLaunchKernelGGL(ins_copy_untouched, dim3(cdiv(n_old, 256), L), dim3(256), 0, s,
                     ix.perm.as<int32_t>(), ix.leafrow.as<int32_t>(), la, ncount.as<uint32_t>(),
                     nshift.as<uint32_t>(), n_old, n_total, L, K, perm_new.as<int32_t>(),
                     cnt_at.as<uint32_t>(), hidx_at.as<uint16_t>());
  PDET_HIP(hipGetLastError());
  // empty leaves: untouched nodes' records copied, touched ones written by the layout
  DevBuf empt_new((size_t)std::max<int64_t>(n_empty, 1) * sizeof(EmptyRec));
  if (ix.n_empty) {
    hipLaunchKernelGGL(ins_copy_empties, dim3(cdiv(ix.n_empty, 256)), dim3(256), 0, s,
                       ix.empt.as<EmptyRec>(), ix.n_empty, eoff, eoff_new.as<uint32_t>(),
                       ncount.as<uint32_t>(), K, empt_new.as<EmptyRec>());
    PDET_HIP(hipGetLastError());
  }
  if (T) {
    FlatArgs f{};
    f.touch = touch.as<Touch>();
    f.rec = recs.as<LRec>();
    f.dfs = dfs.as<int32_t>();
    f.lid = lidp.as<int32_t>();
    f.nlid = nlid.as<int32_t>();
    f.nids = sids.as<int32_t>();
    f.perm = ix.perm.as<int32_t>();
    f.perm_new = perm_new.as<int32_t>();
    f.cnt_at = cnt_at.as<uint32_t>();
    f.hidx_at = hidx_at.as<uint16_t>();
    f.fstart = fstart.as<uint32_t>();
    f.nshift = nshift.as<uint32_t>();
    f.eoff_new = eoff_new.as<uint32_t>();
    f.empt_new = empt_new.as<EmptyRec>();
    f.n_old = n_old; f.n_total = n_total; f.m = m; f.K = K;
    hipLaunchKernelGGL(ins_flatten, dim3(T), dim3(64), 0, s, f);
    PDET_HIP(hipGetLastError());
  }

  // -- swap in the grown index and rebuild the leaf tables
  keep.push_back(std::move(ix.perm));
  keep.push_back(std::move(ix.codes));
  keep.push_back(std::move(ix.leafrow));
  keep.push_back(std::move(ix.leaf_arena));
  keep.push_back(std::move(ix.empt));
  keep.push_back(std::move(ix.eoff));
  keep.push_back(std::move(ix.emat));
  ix.perm = std::move(perm_new);
  ix.codes = std::move(codes);
  ix.empt = std::move(empt_new);
  ix.eoff = std::move(eoff_new);
  ix.emat = std::move(emat_new);
  ix.n_empty = n_empty;
  ix.n = n_total;
  ix.X = data;
  ix.H.release();   // hash values of the literal query, for the old rows
  set_outer_breakpoints(ix.B.as<float>(), ix.colmm.as<uint32_t>(), L * K, ix.Nr, s);
  ix.leafrow.alloc((size_t)L * n_total * L * 4);
  finish_trees(ix, cnt_at.as<uint32_t>(), hidx_at.as<uint16_t>(), scan_tmp, s);
  extend_lowp_copies(ix, n_old, keep, s);
  PDET_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < L; ++i)
    PDET_REQUIRE(ix.nl[i] < (int64_t(1) << 24), PDET_EUNSUPPORTED,
                 "a tree has 2^24 leaves or more (raise max_leaf)");
  {
    std::lock_guard<std::mutex> g(ix.ws_mu);
    ix.ws_free.clear();   // workspaces were sized for the old leaf counts
  }
}

}  // namespace pdet
