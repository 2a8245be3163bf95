// Host-side utilities shared by the library's translation units: error
// reporting for the C ABI, device allocation tracking, a counter-based fill.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sfista.h"

namespace sf {

inline std::string& last_error_slot() {
  static thread_local std::string msg;
  return msg;
}

inline void clear_error() { last_error_slot().clear(); }

inline int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error_slot() = buf;
  return code;
}

inline int hip_fail(hipError_t e, const char* where) {
  return set_error(SFISTA_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

inline long round_up(long v, long m) { return (v + m - 1) / m * m; }

// The library's device memory pool on device `dev` (created on first use).
// Freed blocks stay cached in it, up to kPoolKeep bytes, so that handles made
// and dropped in a loop reuse mapped memory instead of mapping and unmapping
// it each time; sfista_release_cached() hands the cache back.
constexpr uint64_t kPoolKeep = uint64_t(8) << 30;

inline hipMemPool_t library_pool(int dev, hipError_t* err) {
  static std::mutex mu;
  static std::vector<hipMemPool_t> pools;
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0) { *err = hipErrorInvalidDevice; return nullptr; }
  if ((size_t)dev >= pools.size()) pools.resize(dev + 1, nullptr);
  if (!pools[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t p = nullptr;
    if ((*err = hipMemPoolCreate(&p, &props)) != hipSuccess) return nullptr;
    uint64_t keep = kPoolKeep;
    if ((*err = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess) {
      (void)hipMemPoolDestroy(p);
      return nullptr;
    }
    pools[dev] = p;
  }
  *err = hipSuccess;
  return pools[dev];
}

// Releases the cached blocks of every pool made so far.
inline hipError_t release_cached_pools() {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return e;
  for (int d = 0; d < ndev; ++d) {
    hipError_t pe;
    hipMemPool_t p = library_pool(d, &pe);
    if (!p) return pe;
    if ((e = hipMemPoolTrimTo(p, 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Owns device allocations; everything is released when the arena dies.
// Requests are carved from a few large chunks (each cleared once when it is
// made): a new chunk is at least twice the request and grows geometrically
// up to kMaxChunk, so an arena holds O(log size) blocks, because every block
// released costs a runtime call of about a quarter of a millisecond whatever
// its size.  Requests above kMaxChunk get a block of their own.  Blocks come
// from the library pool through the stream-ordered allocator, so making and
// dropping a plan neither stalls the device nor remaps memory.  All requests
// of one arena are made on one stream; the clears and, when the arena dies,
// the frees are ordered on that stream, which therefore has to outlive the
// arena.
class DeviceArena {
 public:
  DeviceArena() = default;
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  ~DeviceArena() { release(); }
  // Queues the frees of every block on the arena's stream.
  void release() {
    for (void* p : blocks_) (void)hipFreeAsync(p, stream_);
    blocks_.clear();
    base_ = nullptr;
    used_ = cap_ = 0;
  }
  // Allocates `bytes` of cleared device memory (256-byte aligned); nullptr
  // on failure.
  void* alloc_zero(size_t bytes, hipStream_t s) {
    bytes = (bytes < 256 ? 256 : bytes + 255) & ~static_cast<size_t>(255);
    if (bytes > kMaxChunk) return fresh(bytes, s);   // a block of its own
    if (used_ + bytes > cap_) {
      size_t chunk = next_;
      while (chunk < 2 * bytes && chunk < kMaxChunk) chunk *= 2;
      if (chunk > kMaxChunk) chunk = kMaxChunk;
      char* c = static_cast<char*>(fresh(chunk, s));
      if (!c) return nullptr;
      base_ = c;
      cap_ = chunk;
      used_ = 0;
      next_ = chunk < kMaxChunk ? 2 * chunk : kMaxChunk;
    }
    void* p = base_ + used_;
    used_ += bytes;
    return p;
  }
  const char* last_error() const { return err_.c_str(); }

 private:
  static constexpr size_t kMaxChunk = size_t(1) << 30;
  void* fresh(size_t bytes, hipStream_t s) {
    void* p = nullptr;
    stream_ = s;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    hipMemPool_t pool = e == hipSuccess ? library_pool(dev, &e) : nullptr;
    if (pool) e = hipMallocFromPoolAsync(&p, bytes, pool, s);
    if (e != hipSuccess) {
      err_ = hipGetErrorString(e);
      (void)hipGetLastError();
      return nullptr;
    }
    blocks_.push_back(p);
    e = hipMemsetAsync(p, 0, bytes, s);
    if (e != hipSuccess) {
      err_ = hipGetErrorString(e);
      return nullptr;
    }
    return p;
  }
  std::vector<void*> blocks_;
  hipStream_t stream_ = nullptr;
  char* base_ = nullptr;
  size_t used_ = 0, cap_ = 0, next_ = size_t(8) << 20;
  std::string err_;
};

// splitmix64 (Steele, Lea, Flood 2014) of (seed + index), mapped to [-1, 1).
__device__ __forceinline__ double hash_uniform(uint64_t seed, uint64_t idx) {
  uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static __global__ void hash_fill_kernel(double* out, long count, uint64_t seed) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
    out[e] = hash_uniform(seed, static_cast<uint64_t>(e));
}

}  // namespace sf

