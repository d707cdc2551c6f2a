/*
 * pdet.h - DET-LSH index build and c^2-k-ANN search on AMD Instinct MI355X (gfx950).
 *
 * Method: arxiv 2603.24920 (DET-LSH / PDET-LSH). Section 2.1 defines the problem
 * (dataset D of n points in R^d, query q, approximation ratio c > 1, k); Section 3
 * defines the encoding phase (3.1: Eq. 1 projections, dynamic breakpoints, Algorithm 1),
 * the indexing phase (3.2: DE-Trees, Algorithm 2) and the query phase (3.3: Algorithms
 * 3-5), with the query-phase optimisations of Section 6.2.2; Section 4.3 gives the node
 * bound distances, Section 5 (Lemma 3, Eq. 2) the parameters.
 *
 * Conventions for every entry point:
 *  - Plain C types only. "device" pointers are HIP device allocations on the
 *    current device; "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).
 *    Calls are stream-ordered: device outputs are valid once the stream reaches
 *    the call's end. Host outputs are valid when the call returns.
 *  - Every call returns a pdet_status. On failure nothing is leaked, output
 *    handles are set to NULL, and pdet_last_error() describes the failure
 *    (thread-local, valid until the next call on the same thread).
 *  - No exception crosses this boundary.
 */
#ifndef PDET_H
#define PDET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdet_index pdet_index; /* opaque; owned by the library */

typedef enum {
  PDET_OK = 0,
  PDET_EINVAL = -1,       /* an argument is out of range or inconsistent          */
  PDET_ENOMEM = -2,       /* a device allocation failed                            */
  PDET_EDEVICE = -3,      /* a HIP runtime call failed                             */
  PDET_EUNSUPPORTED = -4  /* valid in the method but beyond this build's limits    */
} pdet_status;

typedef enum { PDET_FP32 = 0, PDET_BF16 = 1, PDET_FP8_E4M3 = 2 } pdet_precision;

/* Limits of this build. */
#define PDET_MAX_K 16          /* projections per space: first-layer keys fit 16 bits   */
#define PDET_MAX_L 16          /* projected spaces (trees)                               */
#define PDET_MAX_TOPK 1024     /* k * rescore per query                                  */
#define PDET_MAX_ROUNDS 255    /* radius rounds r_min * c^rho, rho < 255                 */

/*
 * Index build parameters (encoding phase and indexing phase, Sections 3.1-3.2).
 *   K, L        projections per space and number of spaces (Eq. 1: K*L Gaussian vectors).
 *   Nr          regions per dimension, a power of two in [2, 256] (8-bit symbols).
 *   max_leaf    leaf capacity ("max_size" of Algorithm 2), >= 1.
 *   proj        host, float32 [d][L*K] row-major; column i*K+j is the hash vector a_ij
 *               (entries i.i.d. N(0,1)); it is copied. NULL: the library draws it from
 *               `seed` (pdet_draw_params).
 *   sample_ids  host, int64 [n_sample], distinct ids in [0,n): the points whose
 *               projections give the interior breakpoints. floor(n_sample/Nr) >= 1.
 *               NULL: the library draws min(n, max(ceil(sample_frac * n), Nr^2)) distinct
 *               ids uniformly from `seed` (n_sample is then ignored).
 *   sample_frac fraction of n sampled when sample_ids is NULL, in (0, 1] (Section 3.1
 *               uses 0.1); ignored otherwise.
 *   seed        seed of the library's draws (used only where proj or sample_ids is NULL).
 *   lowp_copies bit mask: (1u<<PDET_BF16) and/or (1u<<PDET_FP8_E4M3) build the
 *               low-precision copies of the data used by those verification forms.
 *   encoding    PDET_ENC_DYNAMIC (0): interior breakpoints are the order statistics of the
 *               sampled projections (Algorithm 1, the method's encoding). PDET_ENC_STATIC
 *               (1): the iSAX-style static breakpoints the encoding phase contrasts with
 *               (Section 3.1): each column's sampled projections are normalised by their
 *               mean mu and population standard deviation sigma (FP64 over the float32
 *               values) and B(z) = mu + sigma * Phi^-1((z-1)/Nr) for z = 2..Nr, the
 *               equal-mass quantiles of N(0,1). Both take B(1) and B(Nr+1) from the column
 *               extremes over all points. Everything after the breakpoints is the same.
 */
typedef enum { PDET_ENC_DYNAMIC = 0, PDET_ENC_STATIC = 1 } pdet_encoding;

typedef struct {
  int32_t K, L, Nr, max_leaf;
  const float* proj;
  const int64_t* sample_ids;
  int64_t n_sample;
  uint32_t lowp_copies;
  int32_t encoding;
  double sample_frac;
  uint64_t seed;
} pdet_build_params;

/*
 * The library's seeded draws for pdet_build (host only, no device): proj (if not NULL)
 * receives float32 [d][L*K] entries i.i.d. N(0,1) (mt19937_64 from `seed`, Box-Muller on
 * 53-bit uniforms, row-major order); *n_sample receives min(n, max(ceil(sample_frac * n),
 * Nr^2)); sample_ids (if not NULL) receives that many distinct ids in [0, n), ascending,
 * uniformly drawn (Floyd's algorithm on a second stream of the same seed). A build with
 * proj or sample_ids NULL uses exactly these draws, and exports them (PDET_X_PROJ,
 * PDET_X_SAMPLE). EINVAL for n < 1, d < 1, L or K outside [1,16], Nr outside [2,256], or
 * sample_frac outside (0, 1].
 */
pdet_status pdet_draw_params(int64_t n, int32_t d, int32_t L, int32_t K, int32_t Nr,
                             double sample_frac, uint64_t seed, float* proj,
                             int64_t* sample_ids, int64_t* n_sample);

/*
 * Build an index over `data` (device, float32 [n][d] row-major, n < 2^28).
 * The data pointer is BORROWED: it must stay allocated and unchanged until
 * pdet_free(), because verification reads it. Everything derived from it
 * (breakpoints, codes, trees, low-precision copies) is owned by the index.
 * Errors: EINVAL if the data holds a non-finite value (found by the encoder; nothing is
 * returned); EUNSUPPORTED for n >= 2^28, L*K*n_sample (rounded up to a power of two)
 * >= 2^32, or a tree with 2^24 leaves or more; EINVAL for
 * n < 1, d < 1, K outside [1,16], L outside [1,16], Nr not a power of two in [2,256],
 * max_leaf < 1, NULL sample_ids with sample_frac outside (0, 1], n_sample < Nr, ids out of
 * range, an unknown encoding;
 * ENOMEM/EDEVICE from the runtime. On error *out is NULL.
 * Synchronises `stream` once (to size the leaf tables), and once more with the static
 * encoding (the column moments go to the host, which evaluates Phi^-1).
 */
pdet_status pdet_build(const float* data, int64_t n, int32_t d, const pdet_build_params* p,
                       void* stream, pdet_index** out);

/* Release an index and all device memory it owns. NULL is a no-op. */
void pdet_free(pdet_index* idx);

/*
 * Online insertion (Algorithm 2's insertion loop, Section 3.2): rows idx->n .. n_total-1 of
 * `data` (device, float32 [n_total][d]; its first idx->n rows must be the indexed points,
 * unchanged) are inserted into every tree, one point at a time in row order. A point goes
 * to the leaf whose region holds its code (encoded with the index's interior breakpoints;
 * the outer ones widen to the new column extremes); while that leaf holds max_leaf points
 * or more and is not fully refined, it is split on the dimension the node-split rule picks
 * over the points it holds, and the point follows its bit. The resident tree before the
 * first insertion is the bulk tree with the empty children of its splits kept as empty
 * leaves (and every first-layer node present); empty leaves never appear in the exported
 * leaf tables. Afterwards the index borrows `data` (the old pointer is no longer read),
 * n = n_total, and the codes, permutations, leaf tables and low-precision copies cover
 * every point; the sample and the interior breakpoints stay as built.
 * n_total == idx->n only replaces the data pointer.
 * Must not overlap any other call on the index. EINVAL: NULL idx or data, n_total < n, a
 * live plan or server on the index (free them first), or non-finite values in the new
 * rows (then the index is unchanged); EUNSUPPORTED: n_total >= 2^28, a tree with 2^24
 * leaves or more, or a batch whose work area exceeds 2^31 leaf records; ENOMEM / EDEVICE
 * from the runtime (after such an error the index must be freed). Synchronises `stream`.
 */
pdet_status pdet_insert(pdet_index* idx, const float* data, int64_t n_total, void* stream);

/*
 * Query parameters (c^2-k-ANN query, Algorithm 5, Section 3.3).
 *   k, c          uniform k >= 1 and c > 1, used when the per-query arrays are NULL.
 *   k_per_query   host int32 [nq] or NULL; c_per_query host double [nq] or NULL.
 *   beta          stop rule A fires once |S| >= ceil(beta*n) + k (beta >= 0). beta < 0
 *                 selects the theoretical value of Lemma 3 for each query's c,
 *                 2 - 2 alpha2^L with c^2 chi2_{alpha2}(K) = eps^2 (pdet_theoretical_beta).
 *   r_min         first search radius; radii r_min*c^rho for rho < 255. <= 0 selects the
 *                 index's tuned value (pdet_autotune).
 *   eps           projected-radius factor; <= 0 selects sqrt(chi2 upper quantile of
 *                 exp(-1/L) with K degrees of freedom) (Eq. 2 and Lemma 3).
 *   precision     pdet_precision of candidate verification. FP32 reads the float32
 *                 data; BF16 / FP8_E4M3 read the index's low-precision copy and
 *                 re-rank the best rescore*k candidates from the float32 data.
 *   rescore       >= 1; ignored for FP32.
 */
typedef struct {
  int32_t k;
  double c;
  const int32_t* k_per_query;
  const double* c_per_query;
  double beta;
  double r_min;
  double eps;
  int32_t precision;
  int32_t rescore;
} pdet_query_params;

/* Per-query statistics words written to `qstats` (int32 [nq][PDET_QSTAT_WORDS]). */
#define PDET_QSTAT_WORDS 10
#define PDET_QSTAT_ROUNDS 0   /* radius rounds started                                      */
#define PDET_QSTAT_NCAND 1    /* |S| at termination                                         */
#define PDET_QSTAT_STOP 2     /* 1: stop rule A (|S| >= T), 2: stop rule B, -1: radius       */
                              /* ladder exhausted, -2: internal inconsistency (a bug)       */
#define PDET_QSTAT_LEAVES 3   /* leaves admitted                                            */
#define PDET_QSTAT_HSUM 4     /* sum of candidate ids mod 2^32                               */
#define PDET_QSTAT_HMIX 5     /* sum of mix32(id) mod 2^32, mix32 = murmur3 finaliser        */
#define PDET_QSTAT_TIME 6     /* device time of the query's search in wall-clock ticks       */
                              /* (pdet_index_info.wall_clock_khz ticks per millisecond)      */
#define PDET_QSTAT_VISITS 7   /* point occurrences examined (a point counts once per leaf)   */
#define PDET_QSTAT_BAND_LEAF 8  /* (leaf, round) pairs, over the rounds the query ran, whose */
                              /* squared lower bound lies within 1e-5 relative of that      */
                              /* round's threshold (eps r)^2: FP32-vs-FP64 admission ties   */
#define PDET_QSTAT_BAND_STOPB 9 /* rounds whose stop-rule-B test was a near tie: the k-th   */
                              /* squared distance within 2e-5 relative of (c r)^2           */

/*
 * Answer nq queries (device float32 [nq][d]).
 * Outputs (device, caller-owned) are laid out CSR in query order: query q owns
 * entries [off_q, off_q + k_q) with off_q = sum of k over earlier queries.
 *   ids    int64: neighbour ids sorted by (distance, id) ascending, the distance taken
 *          as the FP64 squared distance (the same order up to ties of the root).
 *   dists  float32: Euclidean distances (not squared) of those neighbours.
 *   qstats int32 [nq][PDET_QSTAT_WORDS] or NULL.
 * Errors: EINVAL for k < 1, k > n, c <= 1, beta < 0, r_min <= 0 on an untuned index, a low-precision form
 * whose copy the index lacks, rescore < 1; EUNSUPPORTED for k*rescore > PDET_MAX_TOPK, or
 * for d and k*rescore together too large for the query workgroup's LDS
 * (12*d + 12*pow2(k*rescore + 384) bytes above 48 KiB).
 * A query whose radius ladder runs out before a stop rule fires gets stop = -1.
 * Concurrent calls on one index are allowed on different streams (the index is
 * read-only after build).
 */
pdet_status pdet_query(const pdet_index* idx, const float* queries, int64_t nq,
                       const pdet_query_params* p, int64_t* ids, float* dists,
                       int32_t* qstats, void* stream);

/*
 * pdet_query, and in addition the candidate set S of every query (Algorithm 5: the union
 * of the points the range queries admitted, up to the step where a stop rule fired), for
 * step-by-step checking. cand (device int32 [nq][cand_cap], caller-owned) receives the
 * distinct ids of S of query q in entries [q*cand_cap, q*cand_cap + min(|S|, cand_cap));
 * their order is unspecified, |S| is qstats word PDET_QSTAT_NCAND, and ids past cand_cap
 * are not written. Errors: those of pdet_query; EINVAL for cand NULL or cand_cap < 1.
 */
pdet_status pdet_query_candidates(const pdet_index* idx, const float* queries, int64_t nq,
                                  const pdet_query_params* p, int64_t* ids, float* dists,
                                  int32_t* qstats, int32_t* cand, int64_t cand_cap, void* stream);

/*
 * pdet_query without device allocation. For callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same arguments,
 * results and errors as pdet_query, except that k and c must be uniform (k_per_query and
 * c_per_query NULL, else EINVAL), and the per-query scratch lives in one static device
 * array of PDET_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends. The array holds the batch's per-query arrays (4*L*K + 32 bytes
 * per query) and as many query slots as then fit (a slot holds every leaf of every tree:
 * about L*nl + 28*(sum of the trees' leaves) bytes); the batch runs in chunks of that many
 * queries. A batch for which the per-query arrays and one slot exceed the array gets
 * EUNSUPPORTED with the sizes in the message. The call makes no hipMalloc / hipFree and no
 * allocating library call, and never synchronises the stream (pdet_build looked the array
 * up on its device, so the runtime placed it there before). Calls that overlap on one
 * device share the array and race: serialise them (one stream, or wait between calls).
 * Must run with the index's device current.
 */
#define PDET_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pdet_status pdet_query_noalloc(const pdet_index* idx, const float* queries, int64_t nq,
                               const pdet_query_params* p, int64_t* ids, float* dists,
                               int32_t* qstats, void* stream);

/*
 * The c^2-k-ANN query of Algorithm 5 as printed, without the optimisations that Section
 * 6.2.2 evaluates: every round re-runs the DET Range Query (Algorithm 3) on each tree at
 * radius eps*r - a leaf whose lower bound exceeds eps*r is pruned, a leaf whose upper bound
 * is at most eps*r contributes all its points, any other admitted leaf contributes the
 * points whose projected distance to q' is smaller than eps*r - and stop rule A
 * (|S| >= ceil(beta n) + k) is checked after each tree. For comparing the two forms of the
 * query. Arguments, outputs and errors as pdet_query, except: k and c uniform
 * (k_per_query / c_per_query non-NULL: EINVAL), FP32 verification only (EINVAL
 * otherwise), k <= 1024; qstats word PDET_QSTAT_LEAVES counts the leaves examined (LB
 * within the radius) and PDET_QSTAT_BAND_LEAF the leaf bounds and projected distances that
 * lie within 1e-5 relative of the threshold. The first call on an index computes and keeps
 * the float32 hash values of every point (4*L*K bytes per point, the encoder's arithmetic),
 * which the per-point filter reads. Synchronises `stream`.
 */
pdet_status pdet_query_literal(const pdet_index* idx, const float* queries, int64_t nq,
                               const pdet_query_params* p, int64_t* ids, float* dists,
                               int32_t* qstats, void* stream);

/*
 * (r,c)-ANN query (Algorithm 4) at one radius r > 0 for each of nq queries: the literal range
 * query at eps*r tree by tree, the candidate set S their union; once |S| >= ceil(beta n) + 1
 * the point of S closest to q is returned; after all L trees the closest point of S is
 * returned if it lies within c*r, else none. ids int64 [nq] (-1: none), dists float32 [nq]
 * (+inf: none); qstats as pdet_query_literal, with PDET_QSTAT_STOP 1 (|S| reached beta n + 1),
 * 2 (a point within c r) or 0 (none). beta < 0 takes Lemma 3's beta for c; eps <= 0 takes
 * Eq. 2's. Synchronises `stream`.
 */
pdet_status pdet_rc_ann(const pdet_index* idx, const float* queries, int64_t nq, double r,
                        double c, double beta, double eps, int64_t* ids, float* dists,
                        int32_t* qstats, void* stream);

/* Sizes the index's query workspace (per-query scratch: round-index tables, admitted-leaf
 * lists, thresholds) for batches of up to nq queries, so that a later pdet_query of at most
 * nq queries allocates nothing. Not an operation of the method itself: the search of
 * Algorithm 5 needs this scratch, and a caller that serves a resident index wants it sized
 * once, before the first batch. Device memory is taken with hipMalloc (or from the block
 * cache, see pdet_release_cache) and kept until pdet_free; at most a third of free device
 * memory (and 48 GiB, unless the index is large enough for capped leaf lists, see
 * pdet_set_list_cap) is used, so large batches are then run in chunks of query slots.
 * Waits for `stream`. nq < 0 -> PDET_EINVAL. */
pdet_status pdet_reserve(pdet_index* idx, int64_t nq, void* stream);

/* Per-tree capacity of the admitted-leaf lists in each query slot of pdet_query,
 * pdet_reserve, plans and servers created after the call. Not an operation of the
 * method: it trades slot memory for concurrency. 0 (the default) holds every leaf unless
 * the index is so large that fewer than min(nq, 2048) such slots fit the workspace budget;
 * then each tree's list is capped at max(16384, a sixteenth of the largest tree's leaves)
 * entries, and at most 2048 slots are used.
 * cap > 0 sets the capacity (trees with fewer leaves hold all of theirs). A query whose
 * lists would exceed the capacity is answered again, after the batch, with slots that
 * hold every leaf; results are the same either way, and pdet_get_timing counts such
 * queries (query_retried). Drops the index's pooled query workspaces: must not run
 * concurrently with queries on the same index. cap < 0 -> PDET_EINVAL. */
pdet_status pdet_set_list_cap(pdet_index* idx, int64_t cap);

/* Device memory recycling. Not an operation of the method: freeing device blocks that
 * kernels have touched and allocating them again is slow in the driver, and a process that
 * rebuilds indexes or re-sizes query scratch would pay it on every cycle. Blocks of 32 MiB
 * or more that the library releases (pdet_free, temporaries, re-sized scratch) are
 * therefore kept, up to 60% of each device's memory, and reused for a later allocation of
 * exactly the same size on the same device. Releasing a block waits for the device to be
 * idle, as hipFree does. A failed allocation returns every cached block to the driver and
 * tries once more. Build temporaries (up to 2 GiB in all) are kept for the next build of
 * the same size. pdet_release_cache returns every cached block and kept temporary now (e.g.
 * before handing the memory to another library); it must not run concurrently with other
 * calls. */
void pdet_release_cache(void);

/* Description of a built index. */
typedef struct {
  int64_t n, n_sample;
  int32_t d, K, L, Nr, max_leaf;
  uint32_t lowp_copies;
  int64_t leaves[PDET_MAX_L];   /* non-empty leaves per tree                          */
  int64_t device_bytes;         /* device memory owned by the index                   */
  int32_t wall_clock_khz;       /* device wall-clock rate (query timing stats)        */
} pdet_index_info;

pdet_status pdet_info(const pdet_index* idx, pdet_index_info* out);

/*
 * Copy index contents to host memory (introspection and step-by-step checking).
 *   PDET_X_BREAKPOINTS float32 [L*K][Nr+1]; entry [i*K+j][u] is B_ij(u+1): u=0 the
 *                      column min over all points, u=Nr the max, interior from the sample.
 *   PDET_X_CODES       uint8 [L][n][16]: region index of dimension j in column j (j<K).
 *   PDET_X_PERM        int32 [n] for `tree`: point ids leaf by leaf (depth-first leaf
 *                      order; order inside a leaf unspecified).
 *   PDET_X_LEAF_START  int32 [leaves] for `tree`; PDET_X_LEAF_COUNT likewise.
 *   PDET_X_LEAF_HIDX   uint16 [leaves][16] for `tree`: (1 << t_j) | prefix_j, where the
 *                      leaf fixes the t_j leading bits prefix_j of dimension j's code.
 *   PDET_X_LEAF_OF     int32 [n] for `tree`: the leaf ordinal of every point id.
 *   PDET_X_PROJ        float32 [d][L*K]: the projection the index uses (given or drawn).
 *   PDET_X_SAMPLE      int64 [n_sample]: the sampled ids (given or drawn).
 * `bytes` must equal the exact size; otherwise EINVAL. Synchronises the device.
 */
enum {
  PDET_X_BREAKPOINTS = 0, PDET_X_CODES = 1, PDET_X_PERM = 2,
  PDET_X_LEAF_START = 3, PDET_X_LEAF_COUNT = 4, PDET_X_LEAF_HIDX = 5, PDET_X_LEAF_OF = 6,
  PDET_X_PROJ = 7, PDET_X_SAMPLE = 8
};
pdet_status pdet_export(const pdet_index* idx, int32_t what, int32_t tree, void* host,
                        size_t bytes);

/*
 * Hash values of m points (device float32 [m][d]) with the index's projection
 * (Eq. 1): out device float32 [m][L*K], column i*K+j = a_ij . x. Same arithmetic
 * as the build's encoder and the query projection.
 */
pdet_status pdet_project(const pdet_index* idx, const float* x, int64_t m, float* out,
                         void* stream);

/*
 * Kernel timing (HIP events on the call's stream). When switched on for the calling
 * thread, pdet_build and pdet_query record the device time of each kernel family and
 * pdet_get_timing returns the figures of the last build and the last query on this
 * thread. Off by default; switching it on adds no synchronisation beyond the calls' own.
 */
typedef struct {
  double build_sample_ms;   /* projection of the sampled points                        */
  double build_sort_ms;     /* column sort and breakpoint pick                          */
  double build_encode_ms;   /* projection + region encoding of all points               */
  double build_tree_ms;     /* DE-Tree creation, leaf tables                            */
  double build_lowp_ms;     /* low-precision copies                                     */
  double query_project_ms;  /* query projection                                         */
  double query_rho_ms;      /* leaf lower bounds -> first admitting round               */
  double query_main_ms;     /* search, dedupe, verification, top-k                      */
  int64_t query_main_launches;
  int64_t query_retried;    /* queries answered again after their leaf lists overflowed */
} pdet_timing;
void pdet_set_timing(int32_t on);
pdet_status pdet_get_timing(pdet_timing* out);

/*
 * Radius-schedule autotuner (the dataset-level "magic" r_min of the parameter-setting
 * section, which the paper takes from PM-LSH: at r_min the candidate set reaches
 * beta*n + k, at r_min/c it does not). Runs the pilot queries (device float32
 * [n_pilot][d]) from a tiny first radius, sets the index's tuned r_min one ladder step
 * below the median terminating radius, then sets how many rounds the batched bound kernel
 * resolves (rounds_resolved, 1..8) to cover the rounds every pilot query needed. Queries passing r_min <= 0
 * use the tuned value. Must not run concurrently with queries on the same index.
 */
typedef struct {
  double r_min;
  int32_t rounds_resolved;
  double median_rounds, p95_rounds;
} pdet_tuning;
pdet_status pdet_autotune(pdet_index* idx, const float* pilot, int64_t n_pilot, int32_t k,
                          double c, double beta, int32_t precision, void* stream,
                          pdet_tuning* out);
/* Sets the tuned schedule directly (e.g. a saved pdet_tuning): r_min > 0, 1 <= rounds <= 8. */
pdet_status pdet_set_tuning(pdet_index* idx, double r_min, int32_t rounds_resolved);

/*
 * Query plans (batching form): the whole launch sequence of one batch - parameter upload,
 * query projection, round indices, search - captured once into a HIP graph. The query,
 * output and per-query k / c arguments are fixed at creation (same meaning as pdet_query);
 * the caller may rewrite the query buffer between launches. pdet_plan_launch replays the
 * graph on `stream`; outputs are valid when the stream reaches the end of the launch.
 * If the plan's query slots hold capped leaf lists (see pdet_set_list_cap), the launch
 * also waits for the stream once and answers overflowed queries again on it.
 * Launches of one plan must not overlap. The plan holds its own scratch until freed.
 */
typedef struct pdet_plan pdet_plan;
pdet_status pdet_plan_create(const pdet_index* idx, const float* queries, int64_t nq,
                             const pdet_query_params* p, int64_t* ids, float* dists,
                             int32_t* qstats, pdet_plan** out);
pdet_status pdet_plan_launch(pdet_plan* plan, void* stream);
void pdet_plan_free(pdet_plan* plan);

/*
 * Serving form: a continuous-batching request loop over a resident index. submit() copies
 * a host query (float32 [d]) into the queue and returns at once; a worker thread admits
 * queued requests into batches of at most min(max_batch, slots the memory budget holds)
 * queries and keeps up to `lanes` batches in flight on separate streams, so requests that
 * arrive while others run are admitted as lanes free up. wait() blocks until a request is
 * done and returns its k ids and distances (host) and its latency (submit to completion).
 * A result is the same whatever batch it was served in (each query has its own
 * workgroup). Slots of a large index hold capped leaf lists (see pdet_set_list_cap); a
 * batch whose queries overflowed them answers those again on its lane before its results
 * are returned. memory_budget 0 takes a quarter of the free device memory; r_min <= 0
 * takes the tuned value; eps <= 0 takes Eq. 2.
 */
typedef struct pdet_server pdet_server;
typedef struct {
  int32_t max_batch;      /* 1..1024                                      */
  int32_t lanes;          /* batches in flight, 1..4                      */
  int32_t k_max;          /* largest k a request may ask for             */
  int32_t precision;      /* pdet_precision                               */
  int32_t rescore;
  double beta, r_min, eps;
  int64_t memory_budget;  /* bytes of query scratch over all lanes       */
} pdet_server_params;
typedef struct {
  int64_t completed, batches, batch_cap;
  double mean_batch, p50_ms, p99_ms, qps;
} pdet_server_stats;
pdet_status pdet_server_create(const pdet_index* idx, const pdet_server_params* p,
                               pdet_server** out);
pdet_status pdet_server_submit(pdet_server* sv, const float* query, int32_t k, double c,
                               int64_t* request_id);
pdet_status pdet_server_wait(pdet_server* sv, int64_t request_id, int64_t* ids, float* dists,
                             double* latency_ms);
pdet_status pdet_server_get_stats(pdet_server* sv, pdet_server_stats* out);
void pdet_server_free(pdet_server* sv);   /* drains queued requests first */

/* Load generator for measuring a server (not part of the method): a native client that
 * submits nreq requests at the arrival times of a Poisson process of rate_qps requests per
 * second (exponential gaps drawn from a 64-bit Mersenne twister seeded with `seed`),
 * request i being host query (i mod m) of queries (float32 [m][d]) with the given k and c,
 * then waits for every one of them (results are discarded; the server's statistics hold
 * their latencies). offered_qps (may be NULL) receives the rate actually offered, measured
 * between the first and the last submission. Blocks the calling thread until all are done. */
pdet_status pdet_server_offer_poisson(pdet_server* sv, const float* queries, int64_t m,
                                      int64_t nreq, double rate_qps, int32_t k, double c,
                                      uint64_t seed, double* offered_qps);

/* beta = 2 - 2 alpha2^L of Lemma 3 (Section 5.1), where alpha2 = Pr[chi2(K) > eps^2 / c^2] and
 * eps^2 = chi2_{alpha1}(K), alpha1 = exp(-1/L): the theoretical false-positive fraction that
 * queries use when beta < 0 (Section 5.2.1, Figure "betal"). NaN for K < 1, L < 1, c <= 1. */
double pdet_theoretical_beta(int32_t K, int32_t L, double c);

/* Phi^-1(p), the standard normal quantile, to double precision, as the static encoding
 * (PDET_ENC_STATIC) evaluates it on the host; NaN outside (0, 1). */
double pdet_normal_quantile(double p);

/* eps = sqrt(chi2 upper exp(-1/L) quantile, K dof) from Eq. 2 / Lemma 3; NaN if invalid. */
double pdet_epsilon(int32_t K, int32_t L);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* pdet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PDET_H */
