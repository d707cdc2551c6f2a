// C ABI of libpdet (declared in include/pdet.h): argument checks, the build pipeline
// (encoding phase then indexing phase) and the query entry point.
#include <cmath>
#include <cstring>
#include <exception>
#include <limits>
#include <new>
#include <random>
#include <thread>

#include "internal.h"

namespace pdet {

namespace {
thread_local std::string g_last_error;
// Regularised lower incomplete gamma P(a, x): power series for x < a + 1, otherwise
// 1 - Q from the continued fraction of Q (modified Lentz).
double gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  const double lg = std::lgamma(a);
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int i = 1; i < 10000; ++i) {
      term *= x / (a + i);
      sum += term;
      if (std::fabs(term) < std::fabs(sum) * 1e-17) break;
    }
    return sum * std::exp(-x + a * std::log(x) - lg);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 10000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-17) break;
  }
  return 1.0 - std::exp(-x + a * std::log(x) - lg) * h;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {
// The block cache behind DevBuf (declared in common.h). Lives until the process ends, so
// buffers released by static objects at exit still find it.
struct BlockCache {
  struct Block { void* p; size_t bytes; int dev; };
  std::mutex mu;
  std::vector<Block> blocks;
  std::vector<size_t> held;    // per device
  std::vector<size_t> cap;     // per device: 60% of its memory (0: not yet read)
  size_t& at(std::vector<size_t>& v, int dev) {
    if ((int)v.size() <= dev) v.resize((size_t)dev + 1, 0);
    return v[(size_t)dev];
  }
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();
  return *c;
}
}  // namespace

bool cache_take(size_t bytes, void** p) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  for (size_t i = 0; i < c.blocks.size(); ++i) {
    if (c.blocks[i].bytes == bytes && c.blocks[i].dev == dev) {
      *p = c.blocks[i].p;
      c.blocks.erase(c.blocks.begin() + (int64_t)i);
      c.at(c.held, dev) -= bytes;
      return true;
    }
  }
  return false;
}

bool cache_give(void* p, size_t bytes, int dev) {
  if (std::uncaught_exceptions() > 0) return false;   // error paths free at once
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != dev) return false;
  BlockCache& c = block_cache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    size_t& cp = c.at(c.cap, dev);
    if (cp == 0) {
      size_t total = 0;
      if (hipDeviceTotalMem(&total, dev) != hipSuccess) return false;
      cp = total / 10 * 6;
    }
    if (c.at(c.held, dev) + bytes > cp) return false;
  }
  // as hipFree does: no kernel may still use the block when it is handed out again
  if (hipDeviceSynchronize() != hipSuccess) return false;
  std::lock_guard<std::mutex> g(c.mu);
  c.blocks.push_back({p, bytes, dev});
  c.at(c.held, dev) += bytes;
  return true;
}

void cache_flush() {
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  for (const auto& b : c.blocks) (void)hipFree(b.p);
  c.blocks.clear();
  std::fill(c.held.begin(), c.held.end(), 0);
}

size_t cache_held() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  return c.at(c.held, dev);
}
void clear_error() { g_last_error.clear(); }

// Checks query arguments and fills per-query k and c (host) and the query configuration.
QueryConfig check_query(const pdet_index* idx, const float* queries, int64_t nq,
                        const pdet_query_params* p, int64_t* ids, float* dists, int32_t* qstats,
                        std::vector<int32_t>& k, std::vector<double>& c) {
  PDET_REQUIRE(idx && p, PDET_EINVAL, "NULL argument");
  PDET_REQUIRE(nq >= 0, PDET_EINVAL, "nq must be >= 0");
  PDET_REQUIRE(nq == 0 || (queries && ids && dists), PDET_EINVAL, "NULL queries or outputs");
  PDET_REQUIRE(std::isfinite(p->beta), PDET_EINVAL, "beta must be finite");
  double r_min = p->r_min;
  if (r_min <= 0.0) {
    PDET_REQUIRE(idx->tuned_r_min > 0.0, PDET_EINVAL,
                 "r_min <= 0 selects the tuned radius, but the index has not been tuned");
    r_min = idx->tuned_r_min;
  }
  PDET_REQUIRE(std::isfinite(r_min), PDET_EINVAL, "r_min must be finite");
  PDET_REQUIRE(p->precision >= PDET_FP32 && p->precision <= PDET_FP8_E4M3, PDET_EINVAL,
               "unknown precision");
  if (p->precision != PDET_FP32) {
    PDET_REQUIRE(idx->lowp & (1u << p->precision), PDET_EINVAL,
                 "index was built without this low-precision copy");
    PDET_REQUIRE(p->rescore >= 1, PDET_EINVAL, "rescore must be >= 1");
  }
  k.resize(nq);
  c.resize(nq);
  for (int64_t q = 0; q < nq; ++q) {
    k[q] = p->k_per_query ? p->k_per_query[q] : p->k;
    c[q] = p->c_per_query ? p->c_per_query[q] : p->c;
    PDET_REQUIRE(k[q] >= 1 && k[q] <= idx->n, PDET_EINVAL, "k must be in [1, n]");
    PDET_REQUIRE(c[q] > 1.0 && std::isfinite(c[q]), PDET_EINVAL, "c must be > 1");
    const int64_t kl = (p->precision == PDET_FP32) ? k[q] : (int64_t)k[q] * p->rescore;
    PDET_REQUIRE(kl <= PDET_MAX_TOPK, PDET_EUNSUPPORTED, "k * rescore exceeds 1024");
  }
  QueryConfig qc{};
  qc.Q = queries;
  qc.nq = nq;
  qc.k_host = k.data();
  qc.c_host = c.data();
  qc.beta = p->beta;
  qc.r_min = r_min;
  qc.eps = (p->eps > 0.0) ? p->eps : epsilon(idx->K, idx->L);
  qc.precision = p->precision;
  qc.rescore = p->precision == PDET_FP32 ? 1 : p->rescore;
  qc.ids = ids;
  qc.dists = dists;
  qc.qstats = qstats;
  return qc;
}

Timer& timer() {
  static thread_local Timer t;
  return t;
}

Span::Span(hipStream_t s, double* acc) : s_(s), acc_(acc) {
  if (!timer().on || !acc) return;
  PDET_HIP(hipEventCreate(&a_));
  PDET_HIP(hipEventCreate(&b_));
  PDET_HIP(hipEventRecord(a_, s_));
}

void Span::finish() {
  if (!a_) return;
  PDET_HIP(hipEventRecord(b_, s_));
  timer().pending.push_back({a_, b_, acc_});
  a_ = b_ = nullptr;
}

void flush_timing() {
  Timer& tm = timer();
  for (const Timer::Pending& pd : tm.pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(pd.b) == hipSuccess && hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess)
      *pd.acc += ms;
    (void)hipEventDestroy(pd.a);
    (void)hipEventDestroy(pd.b);
  }
  tm.pending.clear();
}

Span::~Span() {
  if (a_) (void)hipEventDestroy(a_);
  if (b_) (void)hipEventDestroy(b_);
}

// Lemma 3 / Eq. 2: with eps^2 = chi2_{alpha1}(K) and c^2 chi2_{alpha2}(K) = eps^2, the false
// positive fraction is beta = 2 - 2 alpha2^L, alpha2 = Pr[chi2(K) > eps^2 / c^2].
double theoretical_beta(int K, int L, double c) {
  const double e = epsilon(K, L);
  const double alpha2 = 1.0 - gamma_p(0.5 * K, 0.5 * e * e / (c * c));
  return 2.0 - 2.0 * std::pow(alpha2, (double)L);
}

// eps^2 is the upper alpha1 quantile of chi2(K), alpha1 = exp(-1/L) (Eq. 2, Lemma 3):
// solve 1 - P(K/2, x/2) = alpha1 by bisection.
double epsilon(int K, int L) {
  const double alpha = std::exp(-1.0 / L);
  double lo = 0.0, hi = 1.0;
  while (1.0 - gamma_p(0.5 * K, 0.5 * hi) > alpha) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (1.0 - gamma_p(0.5 * K, 0.5 * mid) > alpha) lo = mid; else hi = mid;
  }
  return std::sqrt(0.5 * (lo + hi));
}

namespace {
class ScratchPool {
 public:
  DevBuf take(size_t b) {
    {
      std::lock_guard<std::mutex> g(mu_);
      for (size_t i = 0; i < free_.size(); ++i)
        if (free_[i].bytes == b) {
          DevBuf d = std::move(free_[i]);
          free_.erase(free_.begin() + (int64_t)i);
          held_ -= b;
          return d;
        }
    }
    return DevBuf(b);
  }
  void give(DevBuf&& d) {
    if (!d.p) return;
    if (std::uncaught_exceptions() > 0) { d.release(); return; }
    std::lock_guard<std::mutex> g(mu_);
    if (held_ + d.bytes > kPoolCap) { d.release(); return; }
    held_ += d.bytes;
    free_.push_back(std::move(d));
  }
  void drain() {
    std::vector<DevBuf> out;
    {
      std::lock_guard<std::mutex> g(mu_);
      out.swap(free_);
      held_ = 0;
    }
  }
 private:
  static constexpr size_t kPoolCap = size_t(2) << 30;
  std::mutex mu_;
  std::vector<DevBuf> free_;
  size_t held_ = 0;
};

ScratchPool& scratch_pool() {
  static ScratchPool* p = new ScratchPool();   // lives until the process ends
  return *p;
}
}  // namespace

DevBuf pool_take(size_t bytes) { return scratch_pool().take(bytes); }
void pool_give(DevBuf&& d) { scratch_pool().give(std::move(d)); }

}  // namespace pdet

int64_t pdet_index::device_bytes() const {
  int64_t b = A.bytes + B.bytes + colmm.bytes + codes.bytes + H.bytes + perm.bytes + leafrow.bytes +
              xbf16.bytes + xfp8.bytes + xscale.bytes + leaf_arena.bytes + sample_dev.bytes +
              nonfinite.bytes + empt.bytes + eoff.bytes + emat.bytes;
  b += small.bytes - A.bytes - B.bytes - colmm.bytes - nonfinite.bytes;   // (views of small)
  auto own = [](const pdet::DevBuf& x) { return x.owned ? (int64_t)x.bytes : 0; };
  for (int i = 0; i < PDET_MAX_L; ++i)
    b += own(leaf_start[i]) + own(leaf_count[i]) + own(leaf_hidx[i]) + own(box[i]) +
         own(gbox[i]);
  return b;
}

using namespace pdet;

extern "C" {

const char* pdet_last_error(void) { return g_last_error.c_str(); }

double pdet_normal_quantile(double p) { return pdet::normal_quantile(p); }

double pdet_theoretical_beta(int32_t K, int32_t L, double c) {
  if (K < 1 || L < 1 || !(c > 1.0) || !std::isfinite(c)) return std::numeric_limits<double>::quiet_NaN();
  return pdet::theoretical_beta(K, L, c);
}

double pdet_epsilon(int32_t K, int32_t L) {
  if (K < 1 || L < 1) return std::numeric_limits<double>::quiet_NaN();
  return pdet::epsilon(K, L);
}

extern "C++" {
namespace {
// A pass over [0, count) split into contiguous parts on up to 16 host threads (one below
// 2^20 items): f(begin, end, part) for each part.
template <class F>
void host_parallel(int64_t count, F&& f) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int parts = count < (int64_t(1) << 20) ? 1 : std::min(16, hw);
  if (parts == 1) {
    f(int64_t(0), count, 0);
    return;
  }
  std::vector<std::thread> th;
  const int64_t per = (count + parts - 1) / parts;
  for (int t = 0; t < parts; ++t)
    th.emplace_back([&, t] { f(std::min(count, t * per), std::min(count, (t + 1) * per), t); });
  for (auto& x : th) x.join();
}

// Pinned staging for the sample ids of a build (per thread, grown as needed, kept): the
// upload is then one asynchronous DMA.
PinnedBuf& sample_staging(size_t bytes) {
  static thread_local PinnedBuf buf;
  if (buf.bytes < bytes) buf.alloc(bytes);
  return buf;
}

// The seeded draws of pdet_draw_params: two mt19937_64 streams of one seed (projection and
// sample), Box-Muller normals from 53-bit uniforms in (0, 1), Floyd's algorithm for the
// sample (a bit per id marks the drawn ones; the ids come out ascending).
uint64_t bounded(std::mt19937_64& g, uint64_t range) {   // uniform in [0, range)
  const uint64_t lim = ~uint64_t(0) - (~uint64_t(0) % range);
  uint64_t x;
  do { x = g(); } while (x >= lim);
  return x % range;
}

int64_t sample_count(int64_t n, int32_t Nr, double frac) {
  const int64_t want = std::max<int64_t>((int64_t)std::ceil(frac * (double)n), (int64_t)Nr * Nr);
  return std::min<int64_t>(n, want);
}

void draw(int64_t n, int32_t d, int32_t LK, int32_t Nr, double frac, uint64_t seed, float* proj,
          int64_t* ids, int64_t* n_sample) {
  if (proj) {
    std::mt19937_64 g(seed);
    const double two_pi = 6.283185307179586;
    auto unit = [&]() { return ((double)(g() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    const int64_t total = (int64_t)d * LK;
    for (int64_t e = 0; e < total; e += 2) {
      const double rad = std::sqrt(-2.0 * std::log(unit())), ang = two_pi * unit();
      proj[e] = (float)(rad * std::cos(ang));
      if (e + 1 < total) proj[e + 1] = (float)(rad * std::sin(ang));
    }
  }
  const int64_t m = sample_count(n, Nr, frac);
  if (n_sample) *n_sample = m;
  if (ids) {
    std::mt19937_64 g(seed ^ 0x9e3779b97f4a7c15ull);
    std::vector<uint64_t> bits((size_t)((n + 63) / 64), 0);
    auto has = [&](int64_t v) { return (bits[v >> 6] >> (v & 63)) & 1u; };
    auto put = [&](int64_t v) { bits[v >> 6] |= uint64_t(1) << (v & 63); };
    for (int64_t j = n - m; j < n; ++j) {
      const int64_t t = (int64_t)bounded(g, (uint64_t)j + 1);
      put(has(t) ? j : t);
    }
    int64_t at = 0;
    for (int64_t v = 0; v < n; ++v)
      if (has(v)) ids[at++] = v;
  }
}
}  // namespace
}  // extern "C++"

pdet_status pdet_draw_params(int64_t n, int32_t d, int32_t L, int32_t K, int32_t Nr,
                             double sample_frac, uint64_t seed, float* proj,
                             int64_t* sample_ids, int64_t* n_sample) {
  return guarded([&] {
    PDET_REQUIRE(n >= 1 && d >= 1, PDET_EINVAL, "n and d must be >= 1");
    PDET_REQUIRE(L >= 1 && L <= PDET_MAX_L && K >= 1 && K <= PDET_MAX_K, PDET_EINVAL,
                 "L and K must be in [1, 16]");
    PDET_REQUIRE(Nr >= 2 && Nr <= 256, PDET_EINVAL, "Nr must be in [2, 256]");
    PDET_REQUIRE(sample_frac > 0.0 && sample_frac <= 1.0, PDET_EINVAL,
                 "sample_frac must be in (0, 1]");
    draw(n, d, L * K, Nr, sample_frac, seed, proj, sample_ids, n_sample);
  });
}

pdet_status pdet_build(const float* data, int64_t n, int32_t d, const pdet_build_params* p,
                       void* stream, pdet_index** out) {
  if (out) *out = nullptr;
  pdet_index* ix = nullptr;
  const pdet_status st = guarded([&] {
    PDET_REQUIRE(out && p && data, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(n >= 1, PDET_EINVAL, "n must be >= 1");
    PDET_REQUIRE(n < (int64_t(1) << 28), PDET_EUNSUPPORTED, "n must be below 2^28");
    PDET_REQUIRE(d >= 1, PDET_EINVAL, "d must be >= 1");
    PDET_REQUIRE(p->K >= 1 && p->K <= PDET_MAX_K, PDET_EINVAL, "K must be in [1, 16]");
    PDET_REQUIRE(p->L >= 1 && p->L <= PDET_MAX_L, PDET_EINVAL, "L must be in [1, 16]");
    PDET_REQUIRE(p->Nr >= 2 && p->Nr <= 256 && (p->Nr & (p->Nr - 1)) == 0, PDET_EINVAL,
                 "Nr must be a power of two in [2, 256]");
    PDET_REQUIRE(p->max_leaf >= 1, PDET_EINVAL, "max_leaf must be >= 1");
    if (!p->sample_ids)
      PDET_REQUIRE(p->sample_frac > 0.0 && p->sample_frac <= 1.0, PDET_EINVAL,
                   "sample_frac must be in (0, 1] when sample_ids is NULL");
    const int64_t n_sample =
        p->sample_ids ? p->n_sample : sample_count(n, p->Nr, p->sample_frac);
    PDET_REQUIRE(n_sample >= p->Nr && n_sample <= n, PDET_EINVAL,
                 "n_sample must be in [Nr, n]");
    PDET_REQUIRE((p->lowp_copies & ~((1u << PDET_BF16) | (1u << PDET_FP8_E4M3))) == 0,
                 PDET_EINVAL, "unknown lowp_copies bit");
    PDET_REQUIRE(p->encoding == PDET_ENC_DYNAMIC || p->encoding == PDET_ENC_STATIC, PDET_EINVAL,
                 "unknown encoding");
    // a given sample is checked on several host threads (branch-free: an id is out of range
    // iff, as unsigned, >= n) while it is copied to the pinned staging of its upload; without
    // staging (no device) it is only checked, so that the error is still reported first
    PinnedBuf* staging = nullptr;
    if (p->sample_ids) {
      try {
        staging = &sample_staging((size_t)n_sample * 8);
      } catch (const Error&) {
        staging = nullptr;
      }
      int64_t* dst = staging ? staging->as<int64_t>() : nullptr;
      uint64_t bad[16] = {};
      host_parallel(n_sample, [&](int64_t b, int64_t e, int part) {
        uint64_t x = 0;
        for (int64_t i = b; i < e; ++i) {
          const int64_t v = p->sample_ids[i];
          x |= (uint64_t)((uint64_t)v >= (uint64_t)n);
          if (dst) dst[i] = v;
        }
        bad[part] = x;
      });
      uint64_t any = 0;
      for (uint64_t x : bad) any |= x;
      PDET_REQUIRE(any == 0, PDET_EINVAL, "sample id out of range");
      PDET_REQUIRE(staging, PDET_ENOMEM, "pinned staging for the sample ids failed");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);

    ix = new pdet_index();
    ix->n = n; ix->d = d; ix->K = p->K; ix->L = p->L; ix->Nr = p->Nr;
    ix->bits = ilog2(p->Nr);
    ix->max_leaf = p->max_leaf;
    ix->n_sample = n_sample;
    // the projection and the sample, given or drawn, kept for export
    ix->proj_host.resize((size_t)d * p->L * p->K);
    if (p->proj)
      std::copy(p->proj, p->proj + ix->proj_host.size(), ix->proj_host.begin());
    else
      draw(n, d, p->L * p->K, p->Nr, 1.0, p->seed, ix->proj_host.data(), nullptr, nullptr);
    std::vector<int64_t> drawn;   // the drawn sample (a given one is uploaded directly)
    if (!p->sample_ids) {
      drawn.resize((size_t)n_sample);
      draw(n, d, p->L * p->K, p->Nr, p->sample_frac, p->seed, nullptr, drawn.data(), nullptr);
    }
    const int64_t* sample_src = p->sample_ids ? p->sample_ids : drawn.data();
    ix->lowp = p->lowp_copies;
    ix->X = data;
    ix->dpad = ((d + 15) / 16) * 16;
    PDET_HIP(hipGetDevice(&ix->device));
    noalloc_setup(ix->device);
    PDET_HIP(hipDeviceGetAttribute(&ix->num_cus, hipDeviceAttributeMultiprocessorCount,
                                   ix->device));
    const int LK = ix->L * ix->K;

    // projection matrix and sampled projections
    const std::vector<float> Ap = pad_projection(ix->proj_host.data(), d, ix->L, ix->K);
    {
      // the small per-index arrays share one block (a whole number of MiB, so that the
      // block cache hands the same block to the next index of this shape)
      auto part = [](size_t b) { return (b + 255) & ~size_t(255); };
      const size_t a_b = Ap.size() * 4, b_b = (size_t)LK * (ix->Nr + 1) * 4,
                   mm_b = (size_t)2 * LK * 4;
      const size_t tot = part(a_b) + part(b_b) + part(mm_b) + part(4);
      ix->small.alloc((tot + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1));
      char* q = ix->small.as<char>();
      ix->A.view(q, a_b); q += part(a_b);
      ix->B.view(q, b_b); q += part(b_b);
      ix->colmm.view(q, mm_b); q += part(mm_b);
      ix->nonfinite.view(q, 4);
    }
    PDET_HIP(hipMemcpyAsync(ix->A.p, Ap.data(), Ap.size() * 4, hipMemcpyHostToDevice, s));
    std::vector<PooledBuf> temps;   // build temporaries, held until the final synchronisation
    ix->sample_dev.alloc((size_t)n_sample * 8);   // kept for export
    {
      if (!staging) {   // a drawn sample
        staging = &sample_staging((size_t)n_sample * 8);
        std::memcpy(staging->as<int64_t>(), sample_src, (size_t)n_sample * 8);
      }
      PDET_HIP(hipMemcpyAsync(ix->sample_dev.p, staging->p, ix->sample_dev.bytes,
                              hipMemcpyHostToDevice, s));
    }
    const DevBuf& sid = ix->sample_dev;
    PooledBuf ps((size_t)LK * n_sample * 4);   // sampled hash values, column-major
    PooledBuf smm((size_t)2 * LK * 4);          // their column min / max
    pdet_timing& tm = timer().t;
    if (timer().on) {
      tm.build_sample_ms = tm.build_sort_ms = tm.build_encode_ms = 0.0;
      tm.build_tree_ms = tm.build_lowp_ms = 0.0;
    }
    {
      Span sp(s, &tm.build_sample_ms);
      // the sample's and the encode's column extremes (ordered-uint min / max) and the
      // non-finite flag start in one launch
      FillList fz;
      fz.add(smm.ptr(), 0xffffffffu, (size_t)LK * 4);
      fz.add(smm.as<uint32_t>() + LK, 0u, (size_t)LK * 4);
      fz.add(ix->nonfinite.p, 0u, 4);
      fz.add(ix->colmm.p, 0xffffffffu, (size_t)LK * 4);
      fz.add(ix->colmm.as<uint32_t>() + LK, 0u, (size_t)LK * 4);
      fill_words(fz, s);
      project_sample(*ix, sid.as<int64_t>(), n_sample, ps.as<float>(), n_sample,
                     smm.as<uint32_t>(), s);
      sp.finish();
    }
    {
      Span sp(s, &tm.build_sort_ms);
      if (p->encoding == PDET_ENC_STATIC)
        static_breakpoints(ps.as<float>(), LK, n_sample, n_sample, ix->Nr,
                           ix->B.as<float>(), temps, s);
      else
        select_breakpoints(ps.as<float>(), LK, n_sample, n_sample, ix->Nr,
                           ix->B.as<float>(), smm.as<uint32_t>(), temps, s);
      sp.finish();
    }

    // encode every point; column extremes give the outer breakpoints
    ix->codes.alloc((size_t)ix->L * n * KP);
    ix->flkey.alloc((size_t)ix->L * n * 2);
    ix->perm.alloc((size_t)ix->L * n * 4);
    {
      Span sp(s, &tm.build_encode_ms);
      encode_points(*ix, s);
      set_outer_breakpoints(ix->B.as<float>(), ix->colmm.as<uint32_t>(), LK, ix->Nr, s);
      sp.finish();
    }
    {
      Span sp(s, &tm.build_tree_ms);
      build_trees(*ix, s);
      sp.finish();
    }
    for (int i = 0; i < ix->L; ++i)   // per-query leaf lists pack (round << 24) | leaf
      PDET_REQUIRE(ix->nl[i] < (int64_t(1) << 24), PDET_EUNSUPPORTED,
                   "a tree has 2^24 leaves or more (raise max_leaf)");
    {
      Span sp(s, &tm.build_lowp_ms);
      build_lowp_copies(*ix, s);
      sp.finish();
    }
    PDET_HIP(hipStreamSynchronize(s));
    flush_timing();
    uint32_t nonfinite = 0;
    PDET_HIP(hipMemcpy(&nonfinite, ix->nonfinite.p, 4, hipMemcpyDeviceToHost));
    PDET_REQUIRE(nonfinite == 0, PDET_EINVAL, "the data holds non-finite values");
    *out = ix;
    ix = nullptr;
  });
  delete ix;
  return st;
}

void pdet_free(pdet_index* idx) { delete idx; }

pdet_status pdet_insert(pdet_index* idx, const float* data, int64_t n_total, void* stream) {
  return guarded([&] {
    PDET_REQUIRE(idx && data, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(n_total >= idx->n, PDET_EINVAL, "n_total is below the indexed count");
    PDET_REQUIRE(n_total < (int64_t(1) << 28), PDET_EUNSUPPORTED, "n must be below 2^28");
    PDET_REQUIRE(idx->users.load() == 0, PDET_EINVAL,
                 "the index has live plans or servers (free them before inserting)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n_total > idx->n) insert_points(*idx, data, n_total, s);
    idx->X = data;
    flush_timing();
  });
}

pdet_status pdet_query(const pdet_index* idx, const float* queries, int64_t nq,
                       const pdet_query_params* p, int64_t* ids, float* dists, int32_t* qstats,
                       void* stream) {
  return guarded([&] {
    std::vector<int32_t> k;
    std::vector<double> c;
    const QueryConfig qc = check_query(idx, queries, nq, p, ids, dists, qstats, k, c);
    if (nq == 0) return;
    run_query(*idx, qc, static_cast<hipStream_t>(stream));
    flush_timing();
  });
}

pdet_status pdet_query_candidates(const pdet_index* idx, const float* queries, int64_t nq,
                                  const pdet_query_params* p, int64_t* ids, float* dists,
                                  int32_t* qstats, int32_t* cand, int64_t cand_cap, void* stream) {
  return guarded([&] {
    std::vector<int32_t> k;
    std::vector<double> c;
    QueryConfig qc = check_query(idx, queries, nq, p, ids, dists, qstats, k, c);
    PDET_REQUIRE(cand && cand_cap >= 1, PDET_EINVAL, "cand must be non-NULL and cand_cap >= 1");
    if (nq == 0) return;
    qc.cand = cand;
    qc.cand_cap = cand_cap;
    run_query(*idx, qc, static_cast<hipStream_t>(stream));
    flush_timing();
  });
}

pdet_status pdet_reserve(pdet_index* idx, int64_t nq, void* stream) {
  return guarded([&] {
    PDET_REQUIRE(idx, PDET_EINVAL, "NULL index");
    PDET_REQUIRE(nq >= 0, PDET_EINVAL, "nq must be >= 0");
    if (nq == 0) return;
    WorkspaceLease lease(*idx);
    reserve_workspace(*idx, lease.get(), nq, 0, static_cast<hipStream_t>(stream), true);
  });
}

pdet_status pdet_set_list_cap(pdet_index* idx, int64_t cap) {
  return guarded([&] {
    PDET_REQUIRE(idx, PDET_EINVAL, "NULL index");
    PDET_REQUIRE(cap >= 0, PDET_EINVAL, "cap must be >= 0");
    std::lock_guard<std::mutex> g(idx->ws_mu);
    idx->list_cap = cap;
    idx->ws_free.clear();
  });
}

void pdet_release_cache(void) {
  scratch_pool().drain();   // its buffers go back to the block cache, which is then emptied
  cache_flush();
}

void pdet_set_timing(int32_t on) { timer().on = on != 0; }

pdet_status pdet_get_timing(pdet_timing* out) {
  return guarded([&] {
    PDET_REQUIRE(out, PDET_EINVAL, "NULL argument");
    flush_timing();
    *out = timer().t;
  });
}

pdet_status pdet_info(const pdet_index* idx, pdet_index_info* out) {
  return guarded([&] {
    PDET_REQUIRE(idx && out, PDET_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->n = idx->n;
    out->n_sample = idx->n_sample;
    out->d = idx->d;
    out->K = idx->K;
    out->L = idx->L;
    out->Nr = idx->Nr;
    out->max_leaf = idx->max_leaf;
    out->lowp_copies = idx->lowp;
    for (int i = 0; i < idx->L; ++i) out->leaves[i] = idx->nl[i];
    out->device_bytes = idx->device_bytes();
    int khz = 0;
    PDET_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, idx->device));
    out->wall_clock_khz = khz;
  });
}

pdet_status pdet_export(const pdet_index* idx, int32_t what, int32_t tree, void* host,
                        size_t bytes) {
  return guarded([&] {
    PDET_REQUIRE(idx && host, PDET_EINVAL, "NULL argument");
    const void* src = nullptr;
    size_t want = 0;
    const bool per_tree = what >= PDET_X_PERM && what <= PDET_X_LEAF_OF;
    if (per_tree) PDET_REQUIRE(tree >= 0 && tree < idx->L, PDET_EINVAL, "tree out of range");
    switch (what) {
      case PDET_X_BREAKPOINTS:
        src = idx->B.p; want = (size_t)idx->L * idx->K * (idx->Nr + 1) * 4; break;
      case PDET_X_CODES:
        src = idx->codes.p; want = (size_t)idx->L * idx->n * KP; break;
      case PDET_X_PERM:
        src = idx->perm.as<int32_t>() + (int64_t)tree * idx->n; want = (size_t)idx->n * 4; break;
      case PDET_X_LEAF_START:
        src = idx->leaf_start[tree].p; want = (size_t)idx->nl[tree] * 4; break;
      case PDET_X_LEAF_COUNT:
        src = idx->leaf_count[tree].p; want = (size_t)idx->nl[tree] * 4; break;
      case PDET_X_LEAF_HIDX:
        src = idx->leaf_hidx[tree].p; want = (size_t)idx->nl[tree] * KP * 2; break;
      case PDET_X_PROJ: {   // the host copy
        want = idx->proj_host.size() * 4;
        PDET_REQUIRE(bytes == want, PDET_EINVAL,
                     "export size mismatch: expected " + std::to_string(want) + " bytes");
        std::copy(idx->proj_host.begin(), idx->proj_host.end(), static_cast<float*>(host));
        return;
      }
      case PDET_X_SAMPLE:
        src = idx->sample_dev.p; want = (size_t)idx->n_sample * 8; break;
      case PDET_X_LEAF_OF: {
        // from the first tree's permutation and leaf rows: the point at position p of
        // tree 0 is perm_0[p], and its leaf in `tree` is leafrow[0][p][tree]
        want = (size_t)idx->n * 4;
        PDET_REQUIRE(bytes == want, PDET_EINVAL,
                     "export size mismatch: expected " + std::to_string(want) + " bytes");
        std::vector<int32_t> perm0(idx->n), rows((size_t)idx->n * idx->L);
        PDET_HIP(hipDeviceSynchronize());
        PDET_HIP(hipMemcpy(perm0.data(), idx->perm.p, (size_t)idx->n * 4, hipMemcpyDeviceToHost));
        PDET_HIP(hipMemcpy(rows.data(), idx->leafrow.p, rows.size() * 4, hipMemcpyDeviceToHost));
        int32_t* out = static_cast<int32_t*>(host);
        for (int64_t pos = 0; pos < idx->n; ++pos)
          out[perm0[pos]] = rows[(size_t)pos * idx->L + tree];
        return;
      }
      default:
        throw Error{PDET_EINVAL, "unknown export item"};
    }
    PDET_REQUIRE(bytes == want, PDET_EINVAL,
                 "export size mismatch: expected " + std::to_string(want) + " bytes");
    PDET_HIP(hipDeviceSynchronize());
    if (want) PDET_HIP(hipMemcpy(host, src, want, hipMemcpyDeviceToHost));
  });
}

pdet_status pdet_project(const pdet_index* idx, const float* x, int64_t m, float* out,
                         void* stream) {
  return guarded([&] {
    PDET_REQUIRE(idx && x && out, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(m >= 0, PDET_EINVAL, "m must be >= 0");
    if (m == 0) return;
    project_points(*idx, x, m, out, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
