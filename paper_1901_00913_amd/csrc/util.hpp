// Host-side utilities shared by the library's translation units: error
// reporting for the C ABI, device allocation tracking, a counter-based fill.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

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

// Owns device allocations; everything is released when the arena dies.
class DeviceArena {
 public:
  DeviceArena() = default;
  DeviceArena(const DeviceArena&) = delete;
  DeviceArena& operator=(const DeviceArena&) = delete;
  ~DeviceArena() {
    for (void* p : ptrs_) (void)hipFree(p);
  }
  // Allocates and clears `bytes` (at least 256) on `s`; nullptr on failure.
  void* alloc_zero(size_t bytes, hipStream_t s) {
    if (bytes < 256) bytes = 256;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      err_ = hipGetErrorString(e);
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs_.push_back(p);
    e = hipMemsetAsync(p, 0, bytes, s);
    if (e != hipSuccess) {
      err_ = hipGetErrorString(e);
      return nullptr;
    }
    return p;
  }
  const char* last_error() const { return err_.c_str(); }

 private:
  std::vector<void*> ptrs_;
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

