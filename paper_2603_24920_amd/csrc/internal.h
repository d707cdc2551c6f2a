// Index layout and the host-side entry points of each kernel family.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <vector>

#include "common.h"

namespace pdet {
// Length of the per-slot radius tables (255 rounds r_min * c^rho and a sentinel).
constexpr int NRHO_TABLE = 256;

// Query scratch, kept by the index and reused across calls (see run_query).
struct QueryWorkspace {
  DevBuf rho, admb, adm2, t2, crr, lcnt, bandc, qp, dk, dc, dT, doff;
  PinnedBuf h_k, h_c, h_T, h_off;   // staging of the per-query parameters
  int64_t nslots = 0, nslots_max = 0, nq_cap = 0;
  // Leaf-list capacity of a slot per tree: tree i holds min(nl_i, list_cap) entries. A
  // large index caps it so that more slots fit; a query whose lists would overflow is
  // flagged in `ovf` (count, then query indices) and answered again in `full`, whose
  // slots hold every leaf.
  int64_t list_cap = 0;
  int64_t cap_req = -1;            // the index's requested capacity when this was sized
  DevBuf ovf;
  PinnedBuf h_ovf;
  std::unique_ptr<QueryWorkspace> full;
  int64_t retried = 0;             // queries answered again in `full` (all batches)
  // a batch whose queries share k and c passes them as scalars (no per-query upload)
  bool uniform = false;
  int32_t uk = 0;
  int64_t uT = 0;
  double uc = 0.0;
  size_t bytes() const {
    return rho.bytes + admb.bytes + adm2.bytes + t2.bytes + crr.bytes + lcnt.bytes + bandc.bytes +
           (full ? full->bytes() : 0);
  }
  bool capped() const { return full != nullptr; }
};
}  // namespace pdet

struct pdet_index {
  int64_t n = 0, n_sample = 0;
  int d = 0, K = 0, L = 0, Nr = 0, bits = 0, max_leaf = 0;
  uint32_t lowp = 0;
  int num_cus = 256;
  int device = 0;
  const float* X = nullptr;        // borrowed float32 [n][d]
  std::vector<float> proj_host;    // the projection [d][L*K] (given or drawn)
  pdet::DevBuf sample_dev;         // int64 [n_sample]: the sampled ids (given or drawn)

  pdet::DevBuf small;              // one block holding the views A, B, colmm and nonfinite
  pdet::DevBuf A;                  // float32 padded projection, see pad_projection()
  pdet::DevBuf B;                  // float32 [L*K][Nr+1] breakpoints
  pdet::DevBuf colmm;              // uint32 [2][L*K] ordered min / max of every column
  pdet::DevBuf nonfinite;          // uint32: set by the encoder if a projection is not finite
  pdet::DevBuf codes;              // uint8 [L][n][KP]
  mutable pdet::DevBuf H;          // float32 [n][L*K] hash values (first literal query, kept)
  mutable std::mutex hash_mu;
  pdet::DevBuf flkey;              // uint16 [L][n] first-layer keys (during the build only)
  pdet::DevBuf perm;               // int32 [L][n]
  pdet::DevBuf leafrow;            // int32 [L][n][L]: for the point at perm position p of tree
                                   // i, its leaf ordinal in every tree (read along leaves)
  // per tree, leaves in depth-first order (views into leaf_arena)
  pdet::DevBuf leaf_arena;
  pdet::DevBuf leaf_start[PDET_MAX_L];   // int32 [nl]
  pdet::DevBuf leaf_count[PDET_MAX_L];   // int32 [nl]
  pdet::DevBuf leaf_hidx[PDET_MAX_L];    // uint16 [nl][KP]
  pdet::DevBuf box[PDET_MAX_L];          // float32 [2][K][nl]: lower / upper edge per dim
  pdet::DevBuf gbox[PDET_MAX_L];         // float32 [2][K][ceil(nl/16)]: union box of 16 leaves
  int64_t nl[PDET_MAX_L] = {};
  int64_t nl_max = 0;
  // radius schedule chosen by pdet_autotune (r_min <= 0 in a query selects tuned_r_min)
  double tuned_r_min = 0.0;
  int rcap = 4;                    // rounds resolved by the batched bound kernel
  int64_t list_cap = 0;            // per-tree leaf-list capacity of query slots (0: automatic)
  // low-precision copies for verification
  int dpad = 0;                    // row length of the copies (multiple of 16)
  pdet::DevBuf xbf16;              // bf16 [n][dpad]
  pdet::DevBuf xfp8;               // fp8 e4m3 [n][dpad]
  pdet::DevBuf xscale;             // float32 [n]: fp8 row scale (power of two)

  // online insertion (absent until the first pdet_insert): the empty leaves of every
  // first-layer node an insertion has touched, in CSR order of (tree, first-layer key)
  pdet::DevBuf empt;               // pdet::EmptyRec [n_empty]
  pdet::DevBuf eoff;               // uint32 [L * 2^K + 1]
  pdet::DevBuf emat;               // uint8 [L * 2^K]: 1 where the empty leaves are stored
  int64_t n_empty = 0;
  mutable std::atomic<int> users{0};   // live plans and servers (an insertion needs none)

  // query workspaces: one per concurrent pdet_query call
  mutable std::mutex ws_mu;
  mutable std::vector<std::unique_ptr<pdet::QueryWorkspace>> ws_free;

  int64_t device_bytes() const;
};

namespace pdet {
// An empty leaf of a first-layer node (48 bytes): a split child that holds no point.
struct EmptyRec {
  int32_t local;      // its position among the node's leaves, empty ones included, depth first
  int32_t tree, key, pad;
  uint16_t h[KP];     // node id per dimension: (1 << refined bits) | their value; 0 beyond K
};
// Inserts rows ix.n .. n_total-1 of `data` (which also holds the indexed rows, unchanged)
// into every tree; the index then borrows `data`.
void insert_points(pdet_index& ix, const float* data, int64_t n_total, hipStream_t s);

// Takes a workspace from the index's pool for the duration of one call.
class WorkspaceLease {
 public:
  explicit WorkspaceLease(const pdet_index& ix) : ix_(ix) {
    std::lock_guard<std::mutex> g(ix_.ws_mu);
    if (!ix_.ws_free.empty()) {
      ws_ = std::move(ix_.ws_free.back());
      ix_.ws_free.pop_back();
    } else {
      ws_ = std::make_unique<QueryWorkspace>();
    }
  }
  ~WorkspaceLease() {
    std::lock_guard<std::mutex> g(ix_.ws_mu);
    ix_.ws_free.push_back(std::move(ws_));
  }
  QueryWorkspace& get() { return *ws_; }
 private:
  const pdet_index& ix_;
  std::unique_ptr<QueryWorkspace> ws_;
};
}  // namespace pdet

namespace pdet {
using Index = pdet_index;

// Counts a plan or a server as a user of its index for as long as it lives.
struct IndexUse {
  const pdet_index* ix = nullptr;
  void hold(const pdet_index* i) {
    ix = i;
    ix->users.fetch_add(1);
  }
  ~IndexUse() {
    if (ix) ix->users.fetch_sub(1);
  }
};

// Build temporaries come from a process-wide pool (api.hip): they go back only after the
// build has synchronised its stream (or are freed if an error unwinds the build), so a later
// build of the same size reuses them without hipMalloc / hipFree. At most 2 GiB are kept.
DevBuf pool_take(size_t bytes);
void pool_give(DevBuf&& d);

// A build temporary with DevBuf's interface, taken from and returned to the pool.
struct PooledBuf {
  DevBuf d;
  PooledBuf() = default;
  explicit PooledBuf(size_t b) { alloc(b); }
  PooledBuf(PooledBuf&& o) noexcept : d(std::move(o.d)) {}
  PooledBuf& operator=(PooledBuf&& o) noexcept {
    if (this != &o) { pool_give(std::move(d)); d = std::move(o.d); }
    return *this;
  }
  ~PooledBuf() { pool_give(std::move(d)); }
  void alloc(size_t b) {
    pool_give(std::move(d));
    if (b) d = pool_take(b);
  }
  size_t bytes() const { return d.bytes; }
  void* ptr() const { return d.p; }
  template <class T> T* as() const { return d.as<T>(); }
};

// Per-thread kernel timing (see pdet_set_timing).
struct Timer {
  bool on = false;
  pdet_timing t{};
  struct Pending { hipEvent_t a, b; double* acc; };
  std::vector<Pending> pending;   // finished spans whose events are read at the next flush
};
Timer& timer();
// Reads the events of every finished span into its accumulator (waits for them).
void flush_timing();

// Records HIP events around a region on stream `s` when timing is on. finish() records
// the end event without waiting; flush_timing() later adds the elapsed milliseconds to
// *acc, so timed runs keep their kernels back to back.
class Span {
 public:
  Span(hipStream_t s, double* acc);
  ~Span();
  void finish();
 private:
  hipStream_t s_;
  double* acc_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// project.hip
std::vector<float> pad_projection(const float* proj, int d, int L, int K);
void project_points(const Index& ix, const float* X, int64_t m, float* out, hipStream_t s);
// The sampled rows' hash values (column-major, ld) and their column min / max in mm
// ([2][L*K] ordered uints, initialised by the caller to the empty range).
void project_sample(const Index& ix, const int64_t* rows, int64_t m, float* out, int64_t ld,
                    uint32_t* mm, hipStream_t s);
void encode_points(const Index& ix, hipStream_t s);
// Encodes the m rows of X (points being inserted) with the index's breakpoints into
// codes [L][m][KP] and first-layer keys [L][m], widening the column extremes (ix.colmm) and
// raising ix.nonfinite for a non-finite projection.
void encode_rows(const Index& ix, const float* X, int64_t m, uint8_t* codes, uint16_t* keys,
                 hipStream_t s);

// sort.hip
// Interior breakpoints B[col][u] (u = 1..Nr-1) of the sampled hash values keys[col][0..ns)
// (column stride ld): the exact order statistics of 1-based rank floor(ns/Nr)*u. mm holds
// the columns' min / max ([2][ncols] ordered uints, from the sample projection).
// Temporaries go to `keep`, which the caller holds until its stream has synchronised.
void select_breakpoints(const float* keys, int ncols, int64_t ld, int64_t ns, int Nr, float* B,
                        const uint32_t* mm, std::vector<PooledBuf>& keep, hipStream_t s);
// Static (iSAX-style) interior breakpoints mu + sigma * Phi^-1((u)/Nr), u = 1..Nr-1, from the
// columns' sampled mean and population standard deviation (synchronises `s`).
void static_breakpoints(const float* keys, int ncols, int64_t ld, int64_t ns, int Nr, float* B,
                        std::vector<PooledBuf>& keep, hipStream_t s);
// Phi^-1(p) for p in (0, 1): the standard normal quantile, to double precision.
double normal_quantile(double p);
void fill_f32(float* p, int64_t count, float v, hipStream_t s);

// Up to FILL_MAX ranges of 32-bit words, each set to its own value by one launch (in place of
// a memset per small buffer: counters, extremes, flags).
constexpr int FILL_MAX = 8;
struct FillList {
  uint32_t* p[FILL_MAX];
  uint32_t value[FILL_MAX];
  uint32_t nwords[FILL_MAX];
  int n = 0;
  void add(void* ptr, uint32_t v, size_t bytes) {
    if (n >= FILL_MAX) throw std::logic_error("fill list full");
    p[n] = static_cast<uint32_t*>(ptr);
    value[n] = v;
    nwords[n] = (uint32_t)(bytes / 4);
    ++n;
  }
};
void fill_words(const FillList& f, hipStream_t s);
void set_outer_breakpoints(float* B, const uint32_t* colmm, int ncols, int Nr, hipStream_t s);
void scan_rows(const uint32_t* in, uint32_t* out, uint32_t* totals, int rows, int64_t len,
               DevBuf& tmp, hipStream_t s);
// The same over the indicator (entry != 0) of each entry.
void scan_rows_nonzero(const uint32_t* in, uint32_t* out, uint32_t* totals, int rows,
                       int64_t len, DevBuf& tmp, hipStream_t s);

// tree.hip
// 64 words of pinned host memory per thread for small readbacks (kept until the thread ends):
// words 0..31 serve the tree build, 32..47 its leaf counts, 48..63 an insertion.
uint32_t* readback_words();
void build_trees(Index& ix, hipStream_t s);
// Stable sort of each tree's n first-layer keys (LSD radix over 8-bit digits) carrying the
// points' 16-byte code rows and ids (the position of each point). Sorted rows and ids end in
// rows0 / ids0; `keys` is overwritten; start[tree][key] / end[tree][key] bound each key's run
// (both 0 for absent keys). h8 / o8 are temporaries that must outlive the stream's work.
void first_layer_sort(int L, int K, int64_t n, uint16_t* keys, const uint4* codes, uint4* rows0,
                      int32_t* ids0, uint4* rows1, int32_t* ids1, uint16_t* keys1,
                      uint32_t* start, uint32_t* end, PooledBuf& h8, PooledBuf& o8,
                      DevBuf& scan_tmp, hipStream_t s);
// The per-tree leaf tables, per-point leaf ordinals, leaf rows and group boxes of an index
// whose perm (ix.perm, [L][ix.n]) is final, from the leaf records at their start positions
// (cnt_at [L][n]: the leaf's size at its first position, 0 elsewhere; hidx_at [L][n][KP]).
// ix.leafrow must be allocated ([L][n][L]). Waits for the stream before returning.
void finish_trees(Index& ix, const uint32_t* cnt_at, const uint16_t* hidx_at, DevBuf& scan_tmp,
                  hipStream_t s);

// lowp.hip
void build_lowp_copies(Index& ix, hipStream_t s);
// After an insertion (ix.n and ix.X already the new ones): the copies grow to ix.n rows,
// the first n_old copied, the rest converted; the old buffers move into `keep` (they must
// outlive the stream's work).
void extend_lowp_copies(Index& ix, int64_t n_old, std::vector<DevBuf>& keep, hipStream_t s);

// query.hip
struct QueryConfig {
  const float* Q;
  int64_t nq;
  const int32_t* k_host;   // [nq]
  const double* c_host;    // [nq]
  double beta, r_min, eps;
  int precision, rescore;
  int64_t* ids;
  float* dists;
  int32_t* qstats;
  int32_t* cand = nullptr;   // optional [nq][cand_cap]: the candidate set S of each query
  int64_t cand_cap = 0;
};
void run_query(const Index& ix, const QueryConfig& qc, hipStream_t s);
int stage_params(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws);
size_t slot_bytes(const Index& ix);
// cap_lists: a large index may cap the slots' leaf lists (see QueryWorkspace); the
// caller then runs retry_overflowed() after the batch.
void reserve_workspace(const Index& ix, QueryWorkspace& ws, int64_t nq, size_t budget,
                       hipStream_t s, bool cap_lists = false);
void enqueue_query(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws, int maxKL,
                   hipStream_t s, bool timed);
// For a workspace with capped lists: waits for stream s, then answers the batch's flagged
// queries again with full-capacity slots (a no-op for uncapped workspaces).
// pdet_query_noalloc (noalloc.hip): the batch in chunks of slots laid out in the library's
// static scratch array; uniform k and c.
void run_query_noalloc(const Index& ix, const QueryConfig& qc, int32_t k, double c,
                       hipStream_t s);
// literal.hip: Algorithm 5 as printed (rc_mode false) or Algorithm 4 (rc_mode true, k = 1)
void run_query_literal(const Index& ix, const QueryConfig& qc, int32_t k, double c, bool rc_mode,
                       hipStream_t s);

// Looks up this device's copy of the scratch array (once per device; pdet_build calls it, so
// that the runtime has placed the array before any allocation-free query runs).
void noalloc_setup(int dev);
void retry_overflowed(const Index& ix, const QueryConfig& qc, QueryWorkspace& ws, int maxKL,
                      hipStream_t s, bool timed);

// api.hip
double epsilon(int K, int L);
double theoretical_beta(int K, int L, double c);
void clear_error();
QueryConfig check_query(const pdet_index* idx, const float* queries, int64_t nq,
                        const pdet_query_params* p, int64_t* ids, float* dists, int32_t* qstats,
                        std::vector<int32_t>& k, std::vector<double>& c);

// Runs f, converting library failures into a status and the thread's error message.
template <class F>
pdet_status guarded(F&& f) {
  try {
    clear_error();
    f();
    return PDET_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return PDET_ENOMEM;
  } catch (...) {
    set_error("unexpected failure");
    return PDET_EDEVICE;
  }
}

}  // namespace pdet
