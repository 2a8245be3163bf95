// Term-stacked "NT" GEMM on gfx950 MFMA:  C[M x N] = A[M x K] * B[N x K]^T.
//
// Both operands are row-major with K contiguous, so every GEMM of the sFISTA
// iteration reads 16-byte chunks along K from LDS for both operands.  The
// caller guarantees the padding contract:
//   * A has at least round_up(M, BM) rows and B at least round_up(N, BN) rows;
//   * lda, ldb >= round_up(K, 64 elements) and the entries in [K, lda) are 0,
// so the main loop needs no bounds checks; only the epilogue masks rows >= M
// and columns >= N.
//
// One workgroup computes a BM x BN tile with (BM/WM) x (BN/WN) wavefronts of
// 64 lanes; each wave owns a WM x WN sub-tile made of 16x16 MFMA blocks.  K is
// walked in stages of 128 bytes per row, double-buffered in LDS with a
// 16-byte row pad (rows 144 bytes apart), which keeps the 16-lane column
// reads of a fragment on distinct banks.
//
// Every mode consumes a 16-byte chunk per lane per 64-byte K segment:
//   BF16/FP16 : 8 values  -> one v_mfma_f32_16x16x32_{bf16,f16}
//   BF16X3    : hi and lo chunks of both operands -> three bf16 MFMAs
//               (a_hi b_hi + a_hi b_lo + a_lo b_hi)
//   FP32      : 4 values  -> four v_mfma_f32_16x16x4_f32
//   FP64      : 2 values  -> two v_mfma_f64_16x16x4_f64
// Lane l feeds row/column (l % 16) and the chunk (l / 16) of the segment for
// both operands, so the k-index assignment is identical on both sides and
// the hardware's internal k order is immaterial.  The accumulator of a 16x16
// block holds, in lane l, column (l % 16) and four rows: 4*(l/16) + t for
// the f32-accumulating instructions, (l/16) + 4*t for the f64 one
// (t = 0..3, the accumulator register).
#pragma once

#include "common.hpp"

namespace sf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

struct GemmArgs {
  const void* a[2];   // A planes (hi, lo for BF16X3)
  const void* b[2];   // B planes
  long lda, ldb;      // leading dimensions in elements
  int M, N, K;
};

template <int MODE> struct AccVec { using T = f32x4_t; };
template <> struct AccVec<M_F64> { using T = f64x4_t; };

template <int MODE>
__device__ __forceinline__ void mma_chunk(typename AccVec<MODE>::T& acc, const uint4* a, const uint4* b) {
  if constexpr (MODE == M_BF16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a[0]),
                                                  __builtin_bit_cast(bf16x8_t, b[0]), acc, 0, 0, 0);
  } else if constexpr (MODE == M_F16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a[0]),
                                                 __builtin_bit_cast(f16x8_t, b[0]), acc, 0, 0, 0);
  } else if constexpr (MODE == M_BF16X3) {
    const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, a[0]);
    const bf16x8_t al = __builtin_bit_cast(bf16x8_t, a[1]);
    const bf16x8_t bh = __builtin_bit_cast(bf16x8_t, b[0]);
    const bf16x8_t bl = __builtin_bit_cast(bf16x8_t, b[1]);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  } else if constexpr (MODE == M_F32) {
    const float4 av = __builtin_bit_cast(float4, a[0]);
    const float4 bv = __builtin_bit_cast(float4, b[0]);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc, 0, 0, 0);
  } else {
    const double2 av = __builtin_bit_cast(double2, a[0]);
    const double2 bv = __builtin_bit_cast(double2, b[0]);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, acc, 0, 0, 0);
  }
}

// Workgroup -> tile.  Workgroups are dispatched round-robin over the 8 XCDs
// (id % 8); the first remap gives every XCD a contiguous range of tile ids so
// that tiles sharing A or B panels share that XCD's L2.  Within the range,
// tiles are walked in column groups of GROUP_M tile-rows.
__device__ __forceinline__ void map_tile(int bid, int nblk, int tiles_m, int tiles_n, int& tm, int& tn) {
  int t = bid;
  if ((nblk & 7) == 0) {
    const int per = nblk >> 3;
    t = (bid & 7) * per + (bid >> 3);
  }
  constexpr int GROUP_M = 8;
  const int width = GROUP_M * tiles_n;
  const int group = t / width;
  const int first_m = group * GROUP_M;
  const int gm = min(tiles_m - first_m, GROUP_M);
  const int inner = t - group * width;
  tm = first_m + inner % gm;
  tn = inner / gm;
}

template <int MODE, int BM, int BN, int WM, int WN, class Epi>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64, 1)
void gemm_nt_kernel(GemmArgs g, Epi epi) {
  using Tr = ModeTraits<MODE>;
  using AccT = typename AccVec<MODE>::T;
  constexpr int P = Tr::planes;
  constexpr int WAVES_N = BN / WN;
  constexpr int NT = (BM / WM) * WAVES_N * 64;
  constexpr int ROWB = 128;                 // K bytes per row per stage
  constexpr int PITCH = ROWB + 16;          // padded LDS row
  constexpr int TILEB = (BM + BN) * PITCH;  // bytes per plane per stage
  constexpr int CA = BM * (ROWB / 16) / NT; // A chunks per thread per plane
  constexpr int CB = BN * (ROWB / 16) / NT;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(BM * (ROWB / 16) % NT == 0 && BN * (ROWB / 16) % NT == 0, "tile/threads");

  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];

  const int tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  int tm, tn;
  map_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WAVES_N;
  const int wn = wave - wm * WAVES_N;

  const long lda_b = g.lda * Tr::esize;
  const long ldb_b = g.ldb * Tr::esize;
  const int ktiles = (g.K * Tr::esize + ROWB - 1) / ROWB;

  // Per-thread global source pointers (advance by ROWB per stage).
  const unsigned char* pa[P][CA];
  const unsigned char* pb[P][CB];
  int la[CA], lb[CB];
#pragma unroll
  for (int i = 0; i < CA; ++i) {
    const int c = tid + i * NT;
    const int row = c >> 3, cc = c & 7;
    la[i] = row * PITCH + cc * 16;
#pragma unroll
    for (int p = 0; p < P; ++p)
      pa[p][i] = static_cast<const unsigned char*>(g.a[p]) + (long)(tm * BM + row) * lda_b + cc * 16;
  }
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    const int c = tid + i * NT;
    const int row = c >> 3, cc = c & 7;
    lb[i] = (BM + row) * PITCH + cc * 16;
#pragma unroll
    for (int p = 0; p < P; ++p)
      pb[p][i] = static_cast<const unsigned char*>(g.b[p]) + (long)(tn * BN + row) * ldb_b + cc * 16;
  }

  uint4 sa[P][CA], sb[P][CB];
  auto gload = [&](int kt) {
    const long off = (long)kt * ROWB;
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
      for (int i = 0; i < CA; ++i) sa[p][i] = *reinterpret_cast<const uint4*>(pa[p][i] + off);
#pragma unroll
      for (int i = 0; i < CB; ++i) sb[p][i] = *reinterpret_cast<const uint4*>(pb[p][i] + off);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      unsigned char* base = lds + (buf * P + p) * TILEB;
#pragma unroll
      for (int i = 0; i < CA; ++i) *reinterpret_cast<uint4*>(base + la[i]) = sa[p][i];
#pragma unroll
      for (int i = 0; i < CB; ++i) *reinterpret_cast<uint4*>(base + lb[i]) = sb[p][i];
    }
  };

  AccT acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = AccT{0, 0, 0, 0};

  // fragment read offsets inside a stage
  const int frow = lane & 15;
  const int fchunk = (lane >> 4) * 16;
  const int a_off = (wm * WM + frow) * PITCH + fchunk;
  const int b_off = (BM + wn * WN + frow) * PITCH + fchunk;

  gload(0);
  lstore(0);
  __syncthreads();

  for (int kt = 0; kt < ktiles; ++kt) {
    const int buf = kt & 1;
    const bool more = (kt + 1) < ktiles;
    if (more) gload(kt + 1);
#pragma unroll
    for (int seg = 0; seg < ROWB / 64; ++seg) {
      uint4 fa[FM][P], fb[FN][P];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const unsigned char* base = lds + (buf * P + p) * TILEB + seg * 64;
#pragma unroll
        for (int i = 0; i < FM; ++i)
          fa[i][p] = *reinterpret_cast<const uint4*>(base + a_off + i * 16 * PITCH);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          fb[j][p] = *reinterpret_cast<const uint4*>(base + b_off + j * 16 * PITCH);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) mma_chunk<MODE>(acc[i][j], fa[i], fb[j]);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue
  constexpr int RSTEP = (MODE == M_F64) ? 4 : 1;          // row stride between accumulator registers
  const int row0 = tm * BM + wm * WM + (lane >> 4) * (MODE == M_F64 ? 1 : 4);
  const int col0 = tn * BN + wn * WN + (lane & 15);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = col0 + j * 16;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = row0 + i * 16 + t * RSTEP;
        if (row < g.M && col < g.N) epi(row, col, acc[i][j][t]);
      }
    }
}

// Tile configuration of the single kernel family.
struct TileCfg {
  static constexpr int BM = 128, BN = 128, WM = 64, WN = 64;
  static constexpr int ROW_PAD = 256;   // operand row allocations are multiples of this
  static constexpr int K_PAD = 64;      // operand leading dimensions are multiples of this
};

template <int MODE>
constexpr size_t gemm_lds_bytes() {
  return 2ull * ModeTraits<MODE>::planes * (TileCfg::BM + TileCfg::BN) * (128 + 16);
}

template <int MODE, class Epi>
hipError_t launch_gemm(const GemmArgs& g, const Epi& epi, hipStream_t s) {
  constexpr int BM = TileCfg::BM, BN = TileCfg::BN, WM = TileCfg::WM, WN = TileCfg::WN;
  auto kern = gemm_nt_kernel<MODE, BM, BN, WM, WN, Epi>;
  static bool attr_set = false;
  constexpr size_t lds = gemm_lds_bytes<MODE>();
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  constexpr int threads = (BM / WM) * (BN / WN) * 64;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(threads), lds, s, g, epi);
  return hipGetLastError();
}

}  // namespace sf
