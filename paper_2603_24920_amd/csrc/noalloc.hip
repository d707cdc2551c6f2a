// pdet_query_noalloc: the c^2-k-ANN query of pdet_query without any device allocation,
// for callers that cannot allocate (code under HIP graph capture, tight serving loops).
//
// Every buffer of the search beyond the caller's inputs and outputs - the batch's projected
// queries and per-query parameters, and the query slots (round tables, admitted-leaf lists,
// thresholds, counters) - lives in `scratch`, a file-scope device array of
// PDET_NOALLOC_SCRATCH_BYTES that each device holds until the process ends. Its device
// address is looked up once per device (hipGetSymbolAddress, with that device current) and
// only that address is handed to kernels. Slots hold every leaf of every tree (no capped
// lists, so no second pass); a batch runs in chunks of as many slots as the array holds
// after the per-query arrays. Calls that overlap on one device share the array and race.
#include "internal.h"

namespace pdet {
namespace {

static __device__ __align__(256) unsigned char scratch[PDET_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (looked up on first use).
void* scratch_address(int dev) {
  PDET_REQUIRE(dev >= 0 && dev < MAX_DEVICES, PDET_EUNSUPPORTED, "device index beyond 64");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    PDET_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PDET_REQUIRE(p != nullptr, PDET_EDEVICE, "the scratch array has no device address");
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// Fills `words` 32-bit words with v (a kernel, not a memset node, so a captured graph
// replays it like any other launch).
__global__ void fill_words(uint32_t* p, int64_t words, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

constexpr size_t ALIGN = 256;
size_t up(size_t b) { return (b + ALIGN - 1) & ~(ALIGN - 1); }

// Bytes of the per-query arrays of a batch of nq queries (projections [nq][L*K] float32,
// k int32, c double, T int64, output offset int64, overflow list uint32 [nq + 1]).
size_t batch_bytes(const Index& ix, int64_t nq) {
  return up((size_t)nq * ix.L * ix.K * 4) + up((size_t)nq * 4) + 3 * up((size_t)nq * 8) +
         up((size_t)(nq + 1) * 4);
}

// Bytes of `slots` query slots whose leaf lists hold every leaf.
size_t slots_bytes(const Index& ix, int64_t slots, int64_t nlpad, int64_t admcap) {
  return up((size_t)slots * ix.L * nlpad) + up((size_t)slots * admcap * 12) +
         up((size_t)slots * (admcap + 1) * 16) + up((size_t)slots * NRHO_TABLE * 4) +
         up((size_t)slots * NRHO_TABLE * 8) + up((size_t)slots * PDET_MAX_L * 4) +
         up((size_t)slots * NRHO_TABLE * 4);
}

}  // namespace

void noalloc_setup(int dev) { (void)scratch_address(dev); }

void run_query_noalloc(const Index& ix, const QueryConfig& qc, int32_t k, double c,
                       hipStream_t s) {
  int dev = -1;
  PDET_HIP(hipGetDevice(&dev));
  PDET_REQUIRE(dev == ix.device, PDET_EINVAL,
               "the current device is not the device the index was built on");
  char* base = static_cast<char*>(scratch_address(dev));
  const int64_t nq = qc.nq;
  const int64_t nl_all = std::max<int64_t>(ix.nl_max, 1);
  const int64_t nlpad = ((ix.nl_max + 15) / 16) * 16;
  int64_t admcap = 0;
  for (int i = 0; i < ix.L; ++i) admcap += ix.nl[i];
  admcap = std::max<int64_t>(admcap, 1);
  const size_t cap_bytes = PDET_NOALLOC_SCRATCH_BYTES;
  const size_t fixed = batch_bytes(ix, nq);
  const size_t one = slots_bytes(ix, 1, nlpad, admcap);
  PDET_REQUIRE(fixed + one <= cap_bytes, PDET_EUNSUPPORTED,
               "pdet_query_noalloc: a batch of " + std::to_string(nq) + " queries needs " +
                   std::to_string(fixed + one) + " bytes of scratch (per-query arrays and one "
                   "query slot of this index); the array holds " + std::to_string(cap_bytes));
  // as many slots as fit: s slots take at most s times the bytes of one (each of the seven
  // regions rounds up to ALIGN bytes once)
  const int64_t slots = std::max<int64_t>(1, std::min<int64_t>((int64_t)((cap_bytes - fixed) / one), nq));

  QueryWorkspace ws;
  size_t off = 0;
  auto take = [&](DevBuf& b, size_t bytes) {
    b.view(base + off, bytes);
    off += up(bytes);
  };
  take(ws.qp, (size_t)nq * ix.L * ix.K * 4);
  take(ws.dk, (size_t)nq * 4);
  take(ws.dc, (size_t)nq * 8);
  take(ws.dT, (size_t)nq * 8);
  take(ws.doff, (size_t)nq * 8);
  take(ws.ovf, (size_t)(nq + 1) * 4);
  take(ws.rho, (size_t)slots * ix.L * nlpad);
  take(ws.admb, (size_t)slots * admcap * 12);
  take(ws.adm2, (size_t)slots * (admcap + 1) * 16);
  take(ws.t2, (size_t)slots * NRHO_TABLE * 4);
  take(ws.crr, (size_t)slots * NRHO_TABLE * 8);
  take(ws.lcnt, (size_t)slots * PDET_MAX_L * 4);
  take(ws.bandc, (size_t)slots * NRHO_TABLE * 4);
  PDET_REQUIRE(off <= cap_bytes, PDET_EDEVICE, "scratch layout exceeds the array");
  ws.nslots = ws.nslots_max = slots;
  ws.nq_cap = nq;
  ws.list_cap = nl_all;
  ws.uniform = true;
  ws.uk = k;
  ws.uc = c;
  const double beta = qc.beta >= 0.0 ? qc.beta : theoretical_beta(ix.K, ix.L, c);
  ws.uT = (int64_t)std::ceil(beta * (double)ix.n) + k;

  // The array keeps the last call's contents (possibly of another index): the dense round
  // tables must start "never admitted" (0xff). Everything else is written before it is read
  // (q_setup clears the per-slot counters and writes the thresholds of each chunk).
  const int64_t words = (int64_t)(ws.rho.bytes / 4);
  hipLaunchKernelGGL(fill_words, dim3((unsigned)std::min<int64_t>(cdiv(words, 256), 4096)),
                     dim3(256), 0, s, ws.rho.as<uint32_t>(), words, 0xffffffffu);
  PDET_HIP(hipGetLastError());
  const int maxKL = qc.precision == PDET_FP32 ? k : k * qc.rescore;
  enqueue_query(ix, qc, ws, maxKL, s, false);
}

}  // namespace pdet

using namespace pdet;

extern "C" pdet_status pdet_query_noalloc(const pdet_index* idx, const float* queries,
                                          int64_t nq, const pdet_query_params* p, int64_t* ids,
                                          float* dists, int32_t* qstats, void* stream) {
  return guarded([&] {
    PDET_REQUIRE(idx && p, PDET_EINVAL, "NULL argument");
    PDET_REQUIRE(!p->k_per_query && !p->c_per_query, PDET_EINVAL,
                 "pdet_query_noalloc takes uniform k and c (per-query arrays need pdet_query)");
    PDET_REQUIRE(nq >= 0, PDET_EINVAL, "nq must be >= 0");
    PDET_REQUIRE(nq == 0 || (queries && ids && dists), PDET_EINVAL, "NULL queries or outputs");
    PDET_REQUIRE(std::isfinite(p->beta), PDET_EINVAL, "beta must be finite");
    PDET_REQUIRE(p->k >= 1 && p->k <= idx->n, PDET_EINVAL, "k must be in [1, n]");
    PDET_REQUIRE(p->c > 1.0 && std::isfinite(p->c), PDET_EINVAL, "c must be > 1");
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
    const int64_t kl = (p->precision == PDET_FP32) ? p->k : (int64_t)p->k * p->rescore;
    PDET_REQUIRE(kl <= PDET_MAX_TOPK, PDET_EUNSUPPORTED, "k * rescore exceeds 1024");
    if (nq == 0) return;
    QueryConfig qc{};
    qc.Q = queries;
    qc.nq = nq;
    qc.beta = p->beta;
    qc.r_min = r_min;
    qc.eps = (p->eps > 0.0) ? p->eps : epsilon(idx->K, idx->L);
    qc.precision = p->precision;
    qc.rescore = p->precision == PDET_FP32 ? 1 : p->rescore;
    qc.ids = ids;
    qc.dists = dists;
    qc.qstats = qstats;
    run_query_noalloc(*idx, qc, p->k, p->c, static_cast<hipStream_t>(stream));
  });
}
