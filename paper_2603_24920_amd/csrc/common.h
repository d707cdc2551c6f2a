// Internal definitions shared by the HIP translation units of libpdet.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "pdet.h"

namespace pdet {

// Code rows are padded to 16 bytes (one 128-bit load per point per tree).
constexpr int KP = 16;
// Segments up to this many points finish their subtree inside one workgroup's LDS.
constexpr int LDS_SEG_CAP = 2048;

// Failure carrying a status; thrown only inside the library, caught at the ABI.
struct Error {
  pdet_status status;
  std::string msg;
};

void set_error(const std::string& msg);

#define PDET_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      throw ::pdet::Error{e_ == hipErrorOutOfMemory ? PDET_ENOMEM : PDET_EDEVICE,      \
                          std::string(#call) + ": " + hipGetErrorString(e_)};          \
    }                                                                                  \
  } while (0)

#define PDET_REQUIRE(cond, status, msg)                     \
  do {                                                      \
    if (!(cond)) throw ::pdet::Error{(status), (msg)};      \
  } while (0)

// Process-wide cache of large device blocks (api.hip). Freeing a block that kernels have
// touched and allocating again costs the driver tens of milliseconds per GiB here, which a
// process that rebuilds indexes or re-sizes query scratch pays on every cycle; blocks of at
// least CACHE_MIN_BYTES (1 MiB) are therefore kept on release and handed out again for a request of
// exactly their size on the same device. A cached block is taken only after its device was
// idle (as hipFree waits), so no kernel still uses it. hipMalloc failures flush the cache and
// retry; pdet_release_cache() returns every cached block to the driver.
constexpr size_t CACHE_MIN_BYTES = size_t(1) << 20;
bool cache_take(size_t bytes, void** p);
bool cache_give(void* p, size_t bytes, int device);
void cache_flush();
size_t cache_held();   // bytes cached for the current device

// Device buffer owned by RAII; freed with hipFree (or kept by the block cache). A view
// (view()) points into another buffer and is never freed through itself.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned), dev(o.dev) {
    o.p = nullptr; o.bytes = 0; o.owned = true;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; owned = o.owned; dev = o.dev;
      o.p = nullptr; o.bytes = 0; o.owned = true;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    (void)hipGetDevice(&dev);
    if (b >= CACHE_MIN_BYTES && cache_take(b, &p)) {
      bytes = b;
      return;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e == hipErrorOutOfMemory && cache_held() > 0) {
      (void)hipGetLastError();
      cache_flush();
      e = hipMalloc(&p, b);
    }
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{PDET_ENOMEM, "hipMalloc(" + std::to_string(b) + " bytes) failed: " +
                                   hipGetErrorString(e)};
    }
    bytes = b;
  }
  void view(void* q, size_t b) {
    release();
    p = q;
    bytes = b;
    owned = false;
  }
  void release() {
    if (p && owned && !(bytes >= CACHE_MIN_BYTES && cache_give(p, bytes, dev))) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    owned = true;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
  int dev = 0;   // device of the allocation
};

// Pinned host buffer (hipHostMalloc), for asynchronous copies and graph memcpy nodes.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{PDET_ENOMEM, "hipHostMalloc(" + std::to_string(b) + " bytes) failed"};
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Total-order mapping float -> uint32 (for atomic min/max on floats).
__host__ __device__ inline uint32_t float_to_ordered(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ordered_to_float(uint32_t u) {
  return __builtin_bit_cast(float, (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__host__ __device__ inline uint32_t mix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
  return h;
}

inline int ilog2(int x) { int b = 0; while ((1 << b) < x) ++b; return b; }

inline unsigned cdiv(int64_t a, int64_t b) { return static_cast<unsigned>((a + b - 1) / b); }

}  // namespace pdet
