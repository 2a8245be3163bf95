// Shared device helpers: operand-plane formats, float-float arithmetic,
// deterministic FP64 reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sf {

// GEMM arithmetic modes (values match sfista_precision).
enum Mode : int { M_F64 = 0, M_F32 = 1, M_BF16 = 2, M_F16 = 3, M_BF16X3 = 4 };

template <int MODE> struct ModeTraits;
template <> struct ModeTraits<M_F64>    { using Acc = double; static constexpr int esize = 8; static constexpr int planes = 1; };
template <> struct ModeTraits<M_F32>    { using Acc = float;  static constexpr int esize = 4; static constexpr int planes = 1; };
template <> struct ModeTraits<M_BF16>   { using Acc = float;  static constexpr int esize = 2; static constexpr int planes = 1; };
template <> struct ModeTraits<M_F16>    { using Acc = float;  static constexpr int esize = 2; static constexpr int planes = 1; };
template <> struct ModeTraits<M_BF16X3> { using Acc = float;  static constexpr int esize = 2; static constexpr int planes = 2; };

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));     // round to nearest even
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
__device__ __forceinline__ uint16_t f32_to_f16(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<_Float16>(f));
}

// GEMM operand layout in device memory.  An operand is a (rows x ld) matrix
// whose K index runs along ld (a multiple of 64 elements).  It is stored in
// blocks of 16 rows x 64 bytes of K (1 KB); blocks run along K first, then
// down the rows.  Inside a block the layout is chunk-major: the 16-byte
// chunk g (K bytes [16 g, 16 g + 16)) of row r sits at byte 16 (16 g + r).
// A block is then exactly what one MFMA fragment load wants (lane l holds row
// l % 16, chunk l / 16 at byte 16 l), and the GEMM moves it from memory to
// LDS with one contiguous 1 KB transfer per wave.
template <int MODE>
__device__ __forceinline__ long op_index(long row, long k, long ld) {
  constexpr int ES = ModeTraits<MODE>::esize;
  constexpr int KSEG = 64 / ES;   // K elements per block
  constexpr int CE = 16 / ES;     // K elements per chunk
  const long blk = (row >> 4) * (ld / KSEG) + k / KSEG;
  const int kin = (int)(k % KSEG);
  return blk * (1024 / ES) + ((kin / CE) * 16 + (row & 15)) * CE + (kin % CE);
}

// Store one value into the operand planes of a GEMM mode.  BF16X3 keeps
// v = hi + lo with hi = bf16(v), lo = bf16(v - hi); `vlo` carries the low
// word of a float-float value when there is one.
template <int MODE>
__device__ __forceinline__ void store_planes(void* const* p, long idx, double v, float vlo = 0.f) {
  if constexpr (MODE == M_F64) {
    static_cast<double*>(p[0])[idx] = v;
  } else if constexpr (MODE == M_F32) {
    static_cast<float*>(p[0])[idx] = static_cast<float>(v);
  } else if constexpr (MODE == M_BF16) {
    static_cast<uint16_t*>(p[0])[idx] = f32_to_bf16(static_cast<float>(v));
  } else if constexpr (MODE == M_F16) {
    static_cast<uint16_t*>(p[0])[idx] = f32_to_f16(static_cast<float>(v));
  } else {
    float vf = static_cast<float>(v);
    uint16_t hi = f32_to_bf16(vf);
    float rest = static_cast<float>(v - static_cast<double>(bf16_to_f32(hi))) + vlo;
    static_cast<uint16_t*>(p[0])[idx] = hi;
    static_cast<uint16_t*>(p[1])[idx] = f32_to_bf16(rest);
  }
}

template <int MODE>
__device__ __forceinline__ void store_planes_f(void* const* p, long idx, float v, float vlo = 0.f) {
  if constexpr (MODE == M_BF16X3) {
    uint16_t hi = f32_to_bf16(v);
    float rest = (v - bf16_to_f32(hi)) + vlo;     // exact: v - hi is representable
    static_cast<uint16_t*>(p[0])[idx] = hi;
    static_cast<uint16_t*>(p[1])[idx] = f32_to_bf16(rest);
  } else if constexpr (MODE == M_F32) {
    static_cast<float*>(p[0])[idx] = v;
  } else if constexpr (MODE == M_BF16) {
    static_cast<uint16_t*>(p[0])[idx] = f32_to_bf16(v);
  } else if constexpr (MODE == M_F16) {
    static_cast<uint16_t*>(p[0])[idx] = f32_to_f16(v);
  } else {
    static_cast<double*>(p[0])[idx] = static_cast<double>(v);
  }
}

// Eight consecutive K values of one operand row, starting at element idx of
// a chunk-aligned K index (a multiple of 8): one 16-byte chunk per plane for
// the 2-byte modes, two 16-byte chunks (16 rows apart) for FP32.  `vlo`
// carries the low words of float-float values (BF16X3 only).
template <int MODE>
__device__ __forceinline__ void store8_planes(void* const* p, long idx, const float (&v)[8], const float (&vlo)[8]) {
  if constexpr (MODE == M_F32) {
    float* d = static_cast<float*>(p[0]) + idx;
    *reinterpret_cast<float4*>(d) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4*>(d + 64) = make_float4(v[4], v[5], v[6], v[7]);   // next chunk: 16 rows x 4 values on
  } else if constexpr (MODE == M_BF16 || MODE == M_F16 || MODE == M_BF16X3) {
    uint32_t w0[4], w1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint16_t h0, h1, l0 = 0, l1 = 0;
      if constexpr (MODE == M_F16) {
        h0 = f32_to_f16(v[2 * q]);
        h1 = f32_to_f16(v[2 * q + 1]);
      } else {
        h0 = f32_to_bf16(v[2 * q]);
        h1 = f32_to_bf16(v[2 * q + 1]);
        if constexpr (MODE == M_BF16X3) {
          l0 = f32_to_bf16((v[2 * q] - bf16_to_f32(h0)) + vlo[2 * q]);
          l1 = f32_to_bf16((v[2 * q + 1] - bf16_to_f32(h1)) + vlo[2 * q + 1]);
        }
      }
      w0[q] = static_cast<uint32_t>(h0) | (static_cast<uint32_t>(h1) << 16);
      w1[q] = static_cast<uint32_t>(l0) | (static_cast<uint32_t>(l1) << 16);
    }
    *reinterpret_cast<uint4*>(static_cast<uint16_t*>(p[0]) + idx) = make_uint4(w0[0], w0[1], w0[2], w0[3]);
    if constexpr (MODE == M_BF16X3)
      *reinterpret_cast<uint4*>(static_cast<uint16_t*>(p[1]) + idx) = make_uint4(w1[0], w1[1], w1[2], w1[3]);
  }
}

// ---------------------------------------------------------------- float-float
// Error-free transformations (Knuth two-sum, Dekker/FMA two-product).  The
// pragmas keep the compiler from contracting the exact sums.
struct ff { float hi, lo; };

#pragma clang fp contract(off)
__device__ __forceinline__ ff two_sum(float a, float b) {
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ ff fast_two_sum(float a, float b) {
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}
__device__ __forceinline__ ff two_prod(float a, float b) {
  float p = a * b;
  float e = __builtin_fmaf(a, b, -p);
  return {p, e};
}
__device__ __forceinline__ ff ff_add(ff a, ff b) {
  ff s = two_sum(a.hi, b.hi);
  ff t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ ff ff_neg(ff a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ ff ff_mul(ff a, ff b) {
  ff p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ ff ff_mul_f(ff a, float b) {
  ff p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
#pragma clang fp contract(on)

__device__ __forceinline__ ff ff_from_double(double d) {
  float hi = static_cast<float>(d);
  float lo = static_cast<float>(d - static_cast<double>(hi));
  return {hi, lo};
}

}  // namespace sf
