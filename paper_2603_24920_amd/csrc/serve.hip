// Batching and serving forms around the c^2-k-ANN query (Algorithm 5):
//  - query plans: the whole launch sequence of a batch (uneven k and c per query) captured
//    once into a HIP graph and replayed;
//  - the autotuner of the radius schedule (the dataset-level "magic" r_min of the
//    parameter-setting section, and how many rounds the batched bound kernel resolves);
//  - a continuous-batching server: requests queue on the host, a worker thread admits
//    them into batches sized by the device-memory budget, keeps up to `lanes` batches in
//    flight on separate streams, and records per-request latency.
// Every query is computed by its own workgroup from the same inputs, so a result does not
// depend on the batch it lands in.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <random>
#include <thread>
#include <unordered_map>

#include "internal.h"

using namespace pdet;

struct pdet_plan {
  const pdet_index* ix = nullptr;
  IndexUse use;
  QueryWorkspace ws;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t nq = 0;
  QueryConfig qc{};   // the captured batch (host arrays of k and c are not kept)
  int maxKL = 0;
  ~pdet_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Rounds each pilot query needed (stats word 0) for a first radius r.
std::vector<int32_t> pilot_rounds(const pdet_index* ix, const float* Q, int64_t np, int32_t k,
                                  double c, double beta, int32_t precision, double r,
                                  hipStream_t s) {
  pdet_query_params p{};
  p.k = k; p.c = c; p.beta = beta; p.r_min = r; p.eps = 0.0; p.precision = precision;
  p.rescore = 4;
  DevBuf ids((size_t)np * k * 8), dists((size_t)np * k * 4), st((size_t)np * PDET_QSTAT_WORDS * 4);
  std::vector<int32_t> kk;
  std::vector<double> cc;
  const QueryConfig qc = check_query(ix, Q, np, &p, ids.as<int64_t>(), dists.as<float>(),
                                     st.as<int32_t>(), kk, cc);
  run_query(*ix, qc, s);
  std::vector<int32_t> h((size_t)np * PDET_QSTAT_WORDS);
  PDET_HIP(hipMemcpy(h.data(), st.p, h.size() * 4, hipMemcpyDeviceToHost));
  std::vector<int32_t> rounds;
  for (int64_t q = 0; q < np; ++q)
    if (h[q * PDET_QSTAT_WORDS + PDET_QSTAT_STOP] > 0)
      rounds.push_back(h[q * PDET_QSTAT_WORDS + PDET_QSTAT_ROUNDS]);
  PDET_REQUIRE(!rounds.empty(), PDET_EINVAL, "every pilot query exhausted the radius ladder");
  std::sort(rounds.begin(), rounds.end());
  return rounds;
}

}  // namespace

// ---------------------------------------------------------------- server
struct pdet_server {
  struct Req {
    std::vector<float> q;
    int32_t k = 0;
    double c = 0.0;
    double t_in = 0.0, t_out = 0.0;
    std::vector<int64_t> ids;
    std::vector<float> dists;
    bool done = false;
  };
  struct Lane {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    QueryWorkspace ws;
    DevBuf dq, dids, ddists;
    PinnedBuf hq, hids, hdists;
    std::vector<int64_t> batch;
    std::vector<int64_t> off;
    QueryConfig qc{};   // the batch in flight (host arrays of k and c are not kept)
    int maxKL = 0;
    int64_t tot = 0;    // its output entries
    bool busy = false;
    ~Lane() {
      if (ev) (void)hipEventDestroy(ev);
      if (s) (void)hipStreamDestroy(s);
    }
  };

  const pdet_index* ix = nullptr;
  IndexUse use;
  pdet_server_params prm{};
  double eps = 0.0, r_min = 0.0;
  int64_t cap = 0;                 // queries per batch admitted by the memory budget
  std::mutex mu;
  std::condition_variable cv_done, cv_work;
  std::unordered_map<int64_t, Req> reqs;
  std::deque<int64_t> pending;
  int64_t next_id = 0;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::thread worker;
  bool stopping = false;
  std::string failure;
  // statistics
  std::vector<double> lat_ms;
  int64_t completed = 0, batches = 0, batched_queries = 0;
  double t_first = -1.0, t_last = 0.0;

  void run();
  ~pdet_server() {
    {
      std::lock_guard<std::mutex> g(mu);
      stopping = true;
    }
    cv_work.notify_all();
    if (worker.joinable()) worker.join();
  }
};

void pdet_server::run() {
  try {
    PDET_HIP(hipSetDevice(ix->device));
    for (;;) {
      bool progressed = false;
      for (auto& lp : lanes) {
        Lane& ln = *lp;
        if (!ln.busy) continue;
        const hipError_t e = hipEventQuery(ln.ev);
        if (e == hipErrorNotReady) continue;
        PDET_HIP(e);
        if (ln.ws.capped()) {
          // capped leaf lists: queries that overflowed them are answered again, then the
          // outputs are copied once more (a rare, blocking path of this lane)
          const int64_t before = ln.ws.retried;
          retry_overflowed(*ix, ln.qc, ln.ws, ln.maxKL, ln.s, false);
          if (ln.ws.retried != before) {
            PDET_HIP(hipMemcpyAsync(ln.hids.p, ln.dids.p, (size_t)ln.tot * 8,
                                    hipMemcpyDeviceToHost, ln.s));
            PDET_HIP(hipMemcpyAsync(ln.hdists.p, ln.ddists.p, (size_t)ln.tot * 4,
                                    hipMemcpyDeviceToHost, ln.s));
            PDET_HIP(hipStreamSynchronize(ln.s));
          }
        }
        const double t = now_ms();
        {
          std::lock_guard<std::mutex> g(mu);
          for (size_t j = 0; j < ln.batch.size(); ++j) {
            Req& r = reqs[ln.batch[j]];
            r.ids.assign(ln.hids.as<int64_t>() + ln.off[j], ln.hids.as<int64_t>() + ln.off[j] + r.k);
            r.dists.assign(ln.hdists.as<float>() + ln.off[j],
                           ln.hdists.as<float>() + ln.off[j] + r.k);
            r.done = true;
            r.t_out = t;
            lat_ms.push_back(t - r.t_in);
          }
          completed += (int64_t)ln.batch.size();
          t_last = t;
        }
        ln.busy = false;
        ln.batch.clear();
        progressed = true;
        cv_done.notify_all();
      }
      for (auto& lp : lanes) {
        Lane& ln = *lp;
        if (ln.busy) continue;
        std::vector<int32_t> k;
        std::vector<double> c;
        {
          std::lock_guard<std::mutex> g(mu);
          if (pending.empty()) break;
          const int64_t b = std::min<int64_t>((int64_t)pending.size(), cap);
          ln.off.clear();
          int64_t tot = 0;
          for (int64_t j = 0; j < b; ++j) {
            const int64_t id = pending.front();
            pending.pop_front();
            Req& r = reqs[id];
            std::copy(r.q.begin(), r.q.end(), ln.hq.as<float>() + j * ix->d);
            ln.batch.push_back(id);
            k.push_back(r.k);
            c.push_back(r.c);
            ln.off.push_back(tot);
            tot += r.k;
          }
          ++batches;
          batched_queries += b;
        }
        const int64_t b = (int64_t)ln.batch.size();
        QueryConfig qc{};
        qc.Q = ln.dq.as<float>();
        qc.nq = b;
        qc.k_host = k.data();
        qc.c_host = c.data();
        qc.beta = prm.beta;
        qc.r_min = r_min;
        qc.eps = eps;
        qc.precision = prm.precision;
        qc.rescore = prm.precision == PDET_FP32 ? 1 : prm.rescore;
        qc.ids = ln.dids.as<int64_t>();
        qc.dists = ln.ddists.as<float>();
        qc.qstats = nullptr;
        PDET_HIP(hipMemcpyAsync(ln.dq.p, ln.hq.p, (size_t)b * ix->d * 4, hipMemcpyHostToDevice,
                                ln.s));
        const int maxKL = stage_params(*ix, qc, ln.ws);
        enqueue_query(*ix, qc, ln.ws, maxKL, ln.s, false);
        const int64_t tot = ln.off.back() + k.back();
        ln.qc = qc;
        ln.qc.k_host = nullptr;
        ln.qc.c_host = nullptr;
        ln.maxKL = maxKL;
        ln.tot = tot;
        PDET_HIP(hipMemcpyAsync(ln.hids.p, ln.dids.p, (size_t)tot * 8, hipMemcpyDeviceToHost, ln.s));
        PDET_HIP(hipMemcpyAsync(ln.hdists.p, ln.ddists.p, (size_t)tot * 4, hipMemcpyDeviceToHost,
                                ln.s));
        PDET_HIP(hipEventRecord(ln.ev, ln.s));
        ln.busy = true;
        progressed = true;
      }
      bool idle = true;
      for (auto& lp : lanes) idle = idle && !lp->busy;
      std::unique_lock<std::mutex> lk(mu);
      if (stopping && pending.empty() && idle) break;
      if (!progressed) {
        if (idle && pending.empty())
          cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
        else
          cv_work.wait_for(lk, std::chrono::microseconds(20));
      }
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(mu);
    failure = e.msg;
  }
  cv_done.notify_all();
}

extern "C" {

pdet_status pdet_autotune(pdet_index* idx, const float* pilot, int64_t n_pilot, int32_t k,
                          double c, double beta, int32_t precision, void* stream,
                          pdet_tuning* out) {
  return guarded([&] {
    PDET_REQUIRE(idx && pilot && out, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(n_pilot >= 1, PDET_EINVAL, "need at least one pilot query");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // first radius: its projected threshold is 1e-4 of the median breakpoint range
    const int LK = idx->L * idx->K;
    std::vector<float> B((size_t)LK * (idx->Nr + 1));
    PDET_HIP(hipStreamSynchronize(s));
    PDET_HIP(hipMemcpy(B.data(), idx->B.p, B.size() * 4, hipMemcpyDeviceToHost));
    std::vector<double> rng(LK);
    for (int col = 0; col < LK; ++col)
      rng[col] = (double)B[(size_t)col * (idx->Nr + 1) + idx->Nr] - B[(size_t)col * (idx->Nr + 1)];
    std::nth_element(rng.begin(), rng.begin() + LK / 2, rng.end());
    const double eps = epsilon(idx->K, idx->L);
    const double r0 = std::max(1e-30, 1e-4 * rng[LK / 2] / eps);
    const int rcap_saved = idx->rcap;
    std::vector<int32_t> rounds;
    try {
      rounds = pilot_rounds(idx, pilot, n_pilot, k, c, beta, precision, r0, s);
      const int32_t med = rounds[rounds.size() / 2];
      const int steps = std::max(0, med - 2);
      double r = r0;
      for (int i = 0; i < steps; ++i) r = c * r;
      // rounds a tuned query needs: the batched kernel resolves every round a pilot query
      // reached, so per-query refinement stays rare
      rounds = pilot_rounds(idx, pilot, n_pilot, k, c, beta, precision, r, s);
      const int32_t p95 = rounds[std::min(rounds.size() - 1, (size_t)(0.95 * rounds.size()))];
      idx->tuned_r_min = r;
      idx->rcap = std::max(1, std::min(8, (int)rounds.back() - 1));
      out->r_min = r;
      out->rounds_resolved = idx->rcap;
      out->median_rounds = rounds[rounds.size() / 2];
      out->p95_rounds = p95;
    } catch (...) {
      idx->rcap = rcap_saved;
      throw;
    }
  });
}

pdet_status pdet_set_tuning(pdet_index* idx, double r_min, int32_t rounds_resolved) {
  return guarded([&] {
    PDET_REQUIRE(idx, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(r_min > 0.0 && std::isfinite(r_min), PDET_EINVAL, "r_min must be > 0");
    PDET_REQUIRE(rounds_resolved >= 1 && rounds_resolved <= 8, PDET_EINVAL,
                 "rounds_resolved must be in [1, 8]");
    idx->tuned_r_min = r_min;
    idx->rcap = rounds_resolved;
  });
}

pdet_status pdet_plan_create(const pdet_index* idx, const float* queries, int64_t nq,
                             const pdet_query_params* p, int64_t* ids, float* dists,
                             int32_t* qstats, pdet_plan** out) {
  if (out) *out = nullptr;
  pdet_plan* plan = nullptr;
  const pdet_status st = guarded([&] {
    PDET_REQUIRE(out, PDET_EINVAL, "NULL argument");
    std::vector<int32_t> k;
    std::vector<double> c;
    const QueryConfig qc = check_query(idx, queries, nq, p, ids, dists, qstats, k, c);
    PDET_REQUIRE(nq >= 1, PDET_EINVAL, "a plan needs at least one query");
    plan = new pdet_plan();
    plan->ix = idx;
    plan->use.hold(idx);
    plan->nq = nq;
    hipStream_t cs = nullptr;
    PDET_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    try {
      reserve_workspace(*idx, plan->ws, nq, 0, cs, true);
      const int maxKL = stage_params(*idx, qc, plan->ws);
      plan->qc = qc;
      plan->qc.k_host = nullptr;
      plan->qc.c_host = nullptr;
      plan->maxKL = maxKL;
      PDET_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_query(*idx, qc, plan->ws, maxKL, cs, false);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      PDET_HIP(hipStreamEndCapture(cs, &plan->graph));
      PDET_HIP(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
    } catch (...) {
      (void)hipStreamDestroy(cs);
      throw;
    }
    PDET_HIP(hipStreamDestroy(cs));
    *out = plan;
    plan = nullptr;
  });
  delete plan;
  return st;
}

pdet_status pdet_plan_launch(pdet_plan* plan, void* stream) {
  return guarded([&] {
    PDET_REQUIRE(plan, PDET_EINVAL, "NULL argument");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    PDET_HIP(hipGraphLaunch(plan->exec, s));
    // capped leaf lists: wait for the graph, answer overflowed queries again
    retry_overflowed(*plan->ix, plan->qc, plan->ws, plan->maxKL, s, false);
  });
}

void pdet_plan_free(pdet_plan* plan) { delete plan; }

pdet_status pdet_server_create(const pdet_index* idx, const pdet_server_params* p,
                               pdet_server** out) {
  if (out) *out = nullptr;
  pdet_server* sv = nullptr;
  const pdet_status st = guarded([&] {
    PDET_REQUIRE(idx && p && out, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(p->max_batch >= 1 && p->max_batch <= 1024, PDET_EINVAL,
                 "max_batch must be in [1, 1024]");
    PDET_REQUIRE(p->lanes >= 1 && p->lanes <= 4, PDET_EINVAL, "lanes must be in [1, 4]");
    PDET_REQUIRE(p->k_max >= 1 && p->k_max <= idx->n, PDET_EINVAL, "k_max must be in [1, n]");
    PDET_REQUIRE(std::isfinite(p->beta), PDET_EINVAL, "beta must be finite");
    PDET_REQUIRE(p->precision >= PDET_FP32 && p->precision <= PDET_FP8_E4M3, PDET_EINVAL,
                 "unknown precision");
    if (p->precision != PDET_FP32) {
      PDET_REQUIRE(idx->lowp & (1u << p->precision), PDET_EINVAL,
                   "index was built without this low-precision copy");
      PDET_REQUIRE(p->rescore >= 1 && (int64_t)p->k_max * p->rescore <= PDET_MAX_TOPK,
                   PDET_EINVAL, "rescore must be >= 1 with k_max * rescore <= 1024");
    }
    const double r_min = p->r_min > 0.0 ? p->r_min : idx->tuned_r_min;
    PDET_REQUIRE(r_min > 0.0, PDET_EINVAL, "r_min <= 0 needs a tuned index");
    sv = new pdet_server();
    sv->ix = idx;
    sv->use.hold(idx);
    sv->prm = *p;
    sv->r_min = r_min;
    sv->eps = p->eps > 0.0 ? p->eps : epsilon(idx->K, idx->L);
    size_t budget = (size_t)std::max<int64_t>(0, p->memory_budget);
    if (budget == 0) {
      size_t freeb = 0, totalb = 0;
      PDET_HIP(hipMemGetInfo(&freeb, &totalb));
      budget = (freeb + cache_held()) / 4;
    }
    // admission: the batch size the per-lane share of the budget holds in query slots
    // (capped leaf lists for a large index, as in pdet_query)
    const size_t per_lane = budget / p->lanes;
    for (int l = 0; l < p->lanes; ++l) {
      auto ln = std::make_unique<pdet_server::Lane>();
      PDET_HIP(hipStreamCreateWithFlags(&ln->s, hipStreamNonBlocking));
      PDET_HIP(hipEventCreateWithFlags(&ln->ev, hipEventDisableTiming));
      reserve_workspace(*idx, ln->ws, p->max_batch, per_lane, ln->s, true);
      if (l == 0) sv->cap = std::max<int64_t>(1, std::min<int64_t>(p->max_batch, ln->ws.nslots));
      ln->dq.alloc((size_t)sv->cap * idx->d * 4);
      ln->hq.alloc((size_t)sv->cap * idx->d * 4);
      ln->dids.alloc((size_t)sv->cap * p->k_max * 8);
      ln->ddists.alloc((size_t)sv->cap * p->k_max * 4);
      ln->hids.alloc((size_t)sv->cap * p->k_max * 8);
      ln->hdists.alloc((size_t)sv->cap * p->k_max * 4);
      sv->lanes.push_back(std::move(ln));
    }
    sv->worker = std::thread([sv] { sv->run(); });
    *out = sv;
    sv = nullptr;
  });
  delete sv;
  return st;
}

pdet_status pdet_server_submit(pdet_server* sv, const float* query, int32_t k, double c,
                               int64_t* request_id) {
  return guarded([&] {
    PDET_REQUIRE(sv && query && request_id, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(k >= 1 && k <= sv->prm.k_max, PDET_EINVAL, "k must be in [1, k_max]");
    PDET_REQUIRE(c > 1.0 && std::isfinite(c), PDET_EINVAL, "c must be > 1");
    pdet_server::Req r;
    r.q.assign(query, query + sv->ix->d);
    r.k = k;
    r.c = c;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      PDET_REQUIRE(sv->failure.empty(), PDET_EDEVICE, "server failed: " + sv->failure);
      r.t_in = now_ms();
      if (sv->t_first < 0) sv->t_first = r.t_in;
      *request_id = sv->next_id++;
      sv->reqs.emplace(*request_id, std::move(r));
      sv->pending.push_back(*request_id);
    }
    sv->cv_work.notify_one();
  });
}

pdet_status pdet_server_wait(pdet_server* sv, int64_t request_id, int64_t* ids, float* dists,
                             double* latency_ms) {
  return guarded([&] {
    PDET_REQUIRE(sv, PDET_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    PDET_REQUIRE(sv->reqs.count(request_id), PDET_EINVAL, "unknown request id");
    // look the request up on every wake-up: submissions may rehash the table
    sv->cv_done.wait(lk, [&] { return sv->reqs.at(request_id).done || !sv->failure.empty(); });
    auto it = sv->reqs.find(request_id);
    PDET_REQUIRE(it->second.done, PDET_EDEVICE, "server failed: " + sv->failure);
    if (ids) std::copy(it->second.ids.begin(), it->second.ids.end(), ids);
    if (dists) std::copy(it->second.dists.begin(), it->second.dists.end(), dists);
    if (latency_ms) *latency_ms = it->second.t_out - it->second.t_in;
    sv->reqs.erase(it);
  });
}

pdet_status pdet_server_get_stats(pdet_server* sv, pdet_server_stats* out) {
  return guarded([&] {
    PDET_REQUIRE(sv && out, PDET_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(sv->mu);
    std::vector<double> l = sv->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double f) { return l.empty() ? 0.0 : l[std::min(l.size() - 1, (size_t)(f * l.size()))]; };
    out->completed = sv->completed;
    out->batches = sv->batches;
    out->mean_batch = sv->batches ? (double)sv->batched_queries / sv->batches : 0.0;
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->qps = (sv->completed && sv->t_last > sv->t_first)
                   ? sv->completed / ((sv->t_last - sv->t_first) * 1e-3) : 0.0;
    out->batch_cap = sv->cap;
  });
}

pdet_status pdet_server_offer_poisson(pdet_server* sv, const float* queries, int64_t m,
                                      int64_t nreq, double rate_qps, int32_t k, double c,
                                      uint64_t seed, double* offered_qps) {
  return guarded([&] {
    PDET_REQUIRE(sv && queries, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(m >= 1 && nreq >= 1, PDET_EINVAL, "m and nreq must be >= 1");
    PDET_REQUIRE(rate_qps > 0.0 && std::isfinite(rate_qps), PDET_EINVAL, "rate must be > 0");
    const int d = sv->ix->d;
    // arrival times: cumulative exponential gaps of mean 1 / rate (a Poisson process)
    std::mt19937_64 gen(seed);
    std::exponential_distribution<double> gap(rate_qps);
    std::vector<double> t_arr((size_t)nreq);
    double t = 0.0;
    for (int64_t i = 0; i < nreq; ++i) { t += gap(gen); t_arr[(size_t)i] = t; }
    std::vector<int64_t> rid((size_t)nreq);
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] {
      return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    double t_last = 0.0;
    for (int64_t i = 0; i < nreq; ++i) {
      while (elapsed() < t_arr[(size_t)i]) {
      }
      t_last = elapsed();
      const pdet_status st = pdet_server_submit(sv, queries + (size_t)(i % m) * d, k, c,
                                                &rid[(size_t)i]);
      PDET_REQUIRE(st == PDET_OK, st, std::string("submit failed: ") + pdet_last_error());
    }
    for (int64_t i = 0; i < nreq; ++i) {
      const pdet_status st = pdet_server_wait(sv, rid[(size_t)i], nullptr, nullptr, nullptr);
      PDET_REQUIRE(st == PDET_OK, st, std::string("wait failed: ") + pdet_last_error());
    }
    if (offered_qps) *offered_qps = (nreq > 1 && t_last > 0.0) ? (double)(nreq - 1) / t_last : 0.0;
  });
}

void pdet_server_free(pdet_server* sv) { delete sv; }

}  // extern "C"
