// Term-stacked "NT" GEMM on gfx950 MFMA:  C[M x N] = A[M x K] * B[N x K]^T.
//
// Both operands are stored in the blocked K-major operand layout of
// op_index (common.hpp), so every GEMM of the sFISTA iteration streams whole
// 1 KB blocks (16 rows x 64 K-bytes) into LDS.  The caller guarantees the
// padding contract:
//   * A has at least round_up(M, BM) rows and B at least round_up(N, BN) rows;
//   * lda, ldb >= round_up(K, 64 elements) and the entries in [K, lda) are 0,
// so the main loop needs no bounds checks; only the epilogue masks rows >= M
// and columns >= N.
//
// One workgroup computes a BM x BN tile with (BM/WM) x (BN/WN) wavefronts of
// 64 lanes; each wave owns a WM x WN sub-tile made of 16x16 MFMA blocks.  K is
// walked in stages of 64 bytes per row through two LDS buffers filled by
// direct global-to-LDS loads (see gemm_tile).
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

#include <algorithm>
#include <type_traits>
#include <vector>

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
  int kchunk;         // K stages (64 bytes) per split; split z = blockIdx.y covers [z kchunk, (z+1) kchunk)
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

// Epilogues that also take eight consecutive columns of a row at once
// (store8) get their outputs staged through LDS (see gemm_tile).
template <class E, class = void>
struct HasStore8 : std::false_type {};
template <class E>
struct HasStore8<E, std::void_t<decltype(&E::store8)>> : std::true_type {};
// Epilogues whose per-element work is dominated by element-wise state
// traffic opt out of the eight-column grouping in the split reduction
// (there one element per thread keeps those accesses coalesced).
template <class E, class = void>
struct ReduceVec8 : std::true_type {};
template <class E>
struct ReduceVec8<E, std::void_t<decltype(E::kElementwiseReduce)>> : std::false_type {};

// s_waitcnt immediate that waits until at most N vector-memory operations
// are outstanding (expcnt and lgkmcnt left at their no-wait maxima).
template <int N>
constexpr int vmcnt_imm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  return (N & 0xF) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14);
}

// Staged epilogue of fragment row I and the rows after it (a compile-time
// recursion, so every accumulator index is a constant even when the
// epilogue body is too large for the compiler to unroll a loop over rows).
template <int I, int FM, int FN, int GPR, int GPL, int SP, class AccT, class Epi>
__device__ __forceinline__ void stage_rows(const AccT (&acc)[FM][FN], float* stg, int lane, int rbase, int cbase,
                                           int M, int N, const Epi& epi) {
  if constexpr (I < FM) {
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) stg[((lane >> 4) * 4 + t) * SP + j * 16 + (lane & 15)] = acc[I][j][t];
    for (int q = 0; q < GPL; ++q) {
      const int gi = q * 64 + lane;
      const int lr = gi / GPR, lc = (gi - lr * GPR) * 8;
      const float4 u0 = *reinterpret_cast<const float4*>(stg + lr * SP + lc);
      const float4 u1 = *reinterpret_cast<const float4*>(stg + lr * SP + lc + 4);
      const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
      const int row = rbase + I * 16 + lr, col = cbase + lc;
      if (row < M && col < N) epi.store8(row, col, v, min(8, N - col));
    }
    stage_rows<I + 1, FM, FN, GPR, GPL, SP>(acc, stg, lane, rbase, cbase, M, N, epi);
  }
}

// LDS staging: two buffers (two distinct __shared__ arrays, so the compiler
// can tell the global-to-LDS copy into one from the fragment reads of the
// other), each holding one stage of 64 K-bytes for the BM + BN rows of every
// plane, as the 1 KB blocks of the operand layout (op_index: 16 rows x 64
// K-bytes, chunk-major inside).  An MFMA fragment wants lane l to hold row
// l % 16, chunk l / 16, i.e. byte 16 l of a block, so every fragment read is
// one contiguous 1 KB wave access, the pattern the LDS serves at full rate
// (16-row gathers from a row-major tile run at half rate on gfx950, with or
// without padding or XOR swizzles).
//
// Global -> LDS uses gfx950's global_load_lds_dwordx4: one instruction copies
// one contiguous 1 KB block (lane L moves bytes [16 L, 16 L + 16)).  Stage kt
// lives in buffer kt % 2.  At the top of a stage each wave waits for its own
// copies of that stage, a workgroup barrier publishes every wave's copies
// (and retires all reads of the other buffer), and the copies of the next
// stage into the other buffer are issued before this stage's MFMAs.  The
// fragment reads are ordinary LDS loads, so the compiler interleaves them
// with the MFMAs and waits for each fragment only where it is first used.
template <int MODE, class T, class Epi>
__device__ __forceinline__ void gemm_tile(unsigned char* lds0, unsigned char* lds1, const GemmArgs& g, int tm,
                                          int tn, int kt0, int ktiles, const Epi& epi) {
  using Tr = ModeTraits<MODE>;
  using AccT = typename AccVec<MODE>::T;
  constexpr int BM = T::BM, BN = T::BN, WM = T::WM, WN = T::WN;
  constexpr int P = Tr::planes;
  constexpr int WAVES_N = BN / WN;
  constexpr int NW = (BM / WM) * WAVES_N;
  constexpr int SEGB = 64;                    // K bytes per row per stage
  constexpr int ROWS = BM + BN;
  constexpr int PLANEB = ROWS * SEGB;         // bytes per plane per stage
  constexpr int NINS = P * ROWS / 16;         // 1 KB copy instructions per stage
  constexpr int IPI = NINS / NW;              // copy instructions per wave per stage
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(NINS % NW == 0 && BM % 16 == 0 && BN % 16 == 0, "tile/waves");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WAVES_N;
  const int wn = wave - wm * WAVES_N;

  // This wave's copy instructions for one stage: wave-uniform global source
  // (stage kt0; lane L adds 16 L) and LDS offset inside a buffer.
  const unsigned char* src[IPI];
  int dst[IPI];
  const int voff = lane * 16;
  {
    const long nseg_a = g.lda * Tr::esize / SEGB;   // K blocks per 16-row block of A
    const long nseg_b = g.ldb * Tr::esize / SEGB;
#pragma unroll
    for (int i = 0; i < IPI; ++i) {
      const int q = wave + NW * i;
      const int p = q / (ROWS / 16);
      const int rg = q - p * (ROWS / 16);
      const unsigned char* base;
      if (rg < BM / 16)
        base = static_cast<const unsigned char*>(p == 0 ? g.a[0] : g.a[1]) +
               ((long)(tm * (BM / 16) + rg) * nseg_a + kt0) * 1024;
      else
        base = static_cast<const unsigned char*>(p == 0 ? g.b[0] : g.b[1]) +
               ((long)(tn * (BN / 16) + rg - BM / 16) * nseg_b + kt0) * 1024;
      src[i] = base;
      dst[i] = p * PLANEB + rg * 16 * SEGB;
    }
  }

  // copies of stage ST into buffer BUF (a stage past the end re-reads the
  // last one into a buffer that is never consumed)
#define SF_ISSUE(BUF, ST)                                                                            \
  {                                                                                                  \
    const long st_ = (long)min((ST), ktiles - 1) * 1024;                                             \
    _Pragma("unroll") for (int i_ = 0; i_ < IPI; ++i_) {                                             \
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)(src[i_] + st_ + voff), \
                                       (void __attribute__((address_space(3)))*)((BUF) + dst[i_]), 16, 0, 0); \
    }                                                                                                \
  }
  // MFMAs of one stage from buffer BUF: block i of this wave's A rows and
  // block j of its B rows, byte 16 lane of each 1 KB block.  The B
  // fragments stay in registers for the stage; the A fragments of block
  // row i + 1 are read while the MFMAs of row i run (scheduling barriers keep
  // the compiler from hoisting more reads than registers allow).
#define SF_LD(PTR) (*reinterpret_cast<const uint4*>(PTR))
#define SF_STAGE(BUF)                                                                                \
  {                                                                                                  \
    const unsigned char* sb_ = (BUF);                                                                \
    uint4 fb_[FN][P], fa_[2][P];                                                                     \
    _Pragma("unroll") for (int j = 0; j < FN; ++j)                                                   \
      _Pragma("unroll") for (int p = 0; p < P; ++p) fb_[j][p] = SF_LD(sb_ + p * PLANEB + b_off + j * 1024); \
    _Pragma("unroll") for (int p = 0; p < P; ++p) fa_[0][p] = SF_LD(sb_ + p * PLANEB + a_off);      \
    _Pragma("unroll") for (int i = 0; i < FM; ++i) {                                                 \
      if (i + 1 < FM) {                                                                              \
        _Pragma("unroll") for (int p = 0; p < P; ++p)                                                \
          fa_[(i + 1) & 1][p] = SF_LD(sb_ + p * PLANEB + a_off + (i + 1) * 1024);                   \
      }                                                                                              \
      _Pragma("unroll") for (int j = 0; j < FN; ++j) mma_chunk<MODE>(acc[i][j], fa_[i & 1], fb_[j]); \
      __builtin_amdgcn_sched_barrier(0);                                                             \
    }                                                                                                \
  }
#define SF_TOP()                                                                                     \
  __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());                                                        \
  __builtin_amdgcn_s_barrier();                                                                      \
  asm volatile("" ::: "memory");

  AccT acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = AccT{0, 0, 0, 0};

  const int a_off = wm * WM * SEGB + lane * 16;
  const int b_off = (BM + wn * WN) * SEGB + lane * 16;

  // ktiles is even (gemm_kstages, plan_gemm), so both buffers are used
  // once per trip and the accumulators stay in place
  SF_ISSUE(lds0, 0);
  for (int kt = 0; kt < ktiles; kt += 2) {
    SF_TOP();
    SF_ISSUE(lds1, kt + 1);
    SF_STAGE(lds0);
    SF_TOP();
    SF_ISSUE(lds0, kt + 2);
    SF_STAGE(lds1);
  }
  // no copy may still target this workgroup's LDS when it exits
  __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
#undef SF_ISSUE
#undef SF_STAGE
#undef SF_LD
#undef SF_TOP

  // Staged epilogue: each wave writes one 16-row fragment row of its
  // accumulators to a private LDS area (row-major), then every lane takes
  // eight consecutive columns of a row, so the epilogue stores whole 16-byte
  // chunks of the operand layout instead of single elements.  Both stage
  // buffers are free once every wave's copies have landed and all waves have
  // passed the barrier below.
  if constexpr (std::is_same<typename Tr::Acc, float>::value && HasStore8<Epi>::value) {
    __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    constexpr int SP = WN + 4;                  // padded staging row (floats)
    constexpr int HALF = NW / 2;
    constexpr int GPR = WN / 8;                 // groups of 8 per staged row
    constexpr int GPL = 16 * GPR / 64;          // groups per lane per fragment row
    static_assert(NW % 2 == 0 && (16 * GPR) % 64 == 0, "staging shape");
    static_assert(HALF * 16 * SP * 4 <= T::template buf_bytes<MODE>(), "staging fits one stage buffer");
    float* stg = reinterpret_cast<float*>((wave < HALF ? lds0 : lds1) + (wave % HALF) * (16 * SP * 4));
    stage_rows<0, FM, FN, GPR, GPL, SP>(acc, stg, lane, tm * BM + wm * WM, tn * BN + wn * WN, g.M, g.N, epi);
    return;
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

// Tile configurations.  Tile256 (256 x 256, 8 waves of 128 x 64, two 64 KB
// LDS stages for bf16x3, one workgroup per CU) is the single-image shape of
// the 2-byte and FP32 modes; FP64 accumulators (8 registers per 16 x 16
// block) need the smaller Tile128.  TileS (64 x 64, 4 waves of 32 x 32)
// serves small images in the batched form.
template <int BM_, int BN_, int WM_, int WN_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int THREADS = (BM / WM) * (BN / WN) * 64;
  // bytes of one of the two LDS stage buffers
  template <int MODE>
  static constexpr int buf_bytes() { return ModeTraits<MODE>::planes * (BM + BN) * 64; }
};
#ifdef SF_TILE_BM
using Tile256 = Tile<SF_TILE_BM, SF_TILE_BN, SF_TILE_WM, SF_TILE_WN>;
#else
using Tile256 = Tile<256, 256, 128, 64>;
#endif
using Tile128 = Tile<128, 128, 64, 32>;
using Tile320 = Tile<320, 256, 160, 64>;   // 2-plane modes only (72 copies per stage over 8 waves)
using TileS = Tile<64, 64, 32, 32>;

template <int MODE> struct BigTile { using T = Tile256; };
template <> struct BigTile<M_F64> { using T = Tile128; };

struct TileCfg {
  static constexpr int ROW_PAD = 256;     // operand row allocations are multiples of this
  static constexpr int K_PAD = 64;        // operand leading dimensions are multiples of this
  static_assert(Tile256::BM <= ROW_PAD && Tile256::BN <= ROW_PAD, "row padding must cover a tile");
};

// K stages of 64 bytes, rounded up to an even count: the K padding of the
// operands (a multiple of 64 elements, zero-filled) always covers it.
template <int MODE>
__host__ __device__ inline int gemm_kstages(int K) { return 2 * ((K * ModeTraits<MODE>::esize + 127) / 128); }

// One tile of one product of a batch: the product index selects the GEMM
// arguments and the epilogue parameters.
struct WorkItem {
  int prod, tm, tn, pad;
};

// Grouped launch: every workgroup computes the tile of the batch's work list
// that its (XCD-grouped) id names.
template <int MODE, class T, class Epi>
__global__ __launch_bounds__(T::THREADS, 1) void gemm_grouped_kernel(const GemmArgs* args, const Epi* epis,
                                                                     const WorkItem* work) {
  __shared__ __attribute__((aligned(16))) unsigned char lds0[T::template buf_bytes<MODE>()];
  __shared__ __attribute__((aligned(16))) unsigned char lds1[T::template buf_bytes<MODE>()];
  int bid = blockIdx.x;
  if ((gridDim.x & 7) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  const WorkItem w = work[bid];
  // the arguments stay in global memory (uniform scalar loads); a private
  // copy would put their small arrays in scratch
  const GemmArgs& g = args[w.prod];
  const Epi& e = epis[w.prod];
  gemm_tile<MODE, T>(lds0, lds1, g, w.tm, w.tn, 0, gemm_kstages<MODE>(g.K), e);
}

// ------------------------------------------------------------ planned launch
// A single product runs from a work list built on the host (plan_gemm): item
// i is workgroup i's tile, either over the whole K range (the GEMM's own
// epilogue runs) or over one of S K-splits (the partial goes to a per-tile
// workspace slot and tile_reduce_kernel adds the splits in order and runs the
// epilogue).  Workgroups are dispatched round-robin over the XCDs (id % 8), so
// the list interleaves eight per-XCD sequences, each a compact block of tiles
// over one K range, sharing that XCD's L2.
struct PlanItem {
  int tm, tn;
  int z;      // K split, or -1 for the whole K range
  int slot;   // workspace slot of a split tile
};

template <class Acc>
struct EpiSlot {
  Acc* ws;      // BM x BN partial of this (tile, split)
  int r0, c0, bn;
  __device__ __forceinline__ void operator()(int row, int col, Acc v) const {
    ws[(long)(row - r0) * bn + (col - c0)] = v;
  }
  __device__ __forceinline__ void store8(int row, int col, const float (&v)[8], int cnt) const {
    if constexpr (std::is_same<Acc, float>::value) {
      Acc* d = ws + (long)(row - r0) * bn + (col - c0);
      if (cnt == 8) {
        *reinterpret_cast<float4*>(d) = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4*>(d + 4) = make_float4(v[4], v[5], v[6], v[7]);
        return;
      }
      for (int q = 0; q < cnt; ++q) d[q] = v[q];
    }
  }
};

template <int MODE, class T, class Epi>
__global__ __launch_bounds__(T::THREADS, 1) void gemm_planned_kernel(GemmArgs g, Epi epi,
                                                                     typename ModeTraits<MODE>::Acc* ws, int S,
                                                                     const PlanItem* work) {
  __shared__ __attribute__((aligned(16))) unsigned char lds0[T::template buf_bytes<MODE>()];
  __shared__ __attribute__((aligned(16))) unsigned char lds1[T::template buf_bytes<MODE>()];
  const PlanItem w = work[blockIdx.x];
  const int ktot = gemm_kstages<MODE>(g.K);
  if (w.z < 0) {
    gemm_tile<MODE, T>(lds0, lds1, g, w.tm, w.tn, 0, ktot, epi);
  } else {
    const int kt0 = w.z * g.kchunk;
    EpiSlot<typename ModeTraits<MODE>::Acc> part{ws + (long)(w.slot * S + w.z) * (T::BM * T::BN), w.tm * T::BM,
                                                 w.tn * T::BN, T::BN};
    gemm_tile<MODE, T>(lds0, lds1, g, w.tm, w.tn, kt0, min(ktot - kt0, g.kchunk), part);
  }
}

// Adds the S partials of every split tile in split order (deterministic) and
// applies the product's epilogue.  Block x handles split tile x.
template <class Acc, class Epi, int BM, int BN>
__global__ void tile_reduce_kernel(const Acc* ws, int S, int M, int N, const int2* tiles, Epi epi) {
  const int2 t = tiles[blockIdx.x];
  const Acc* base = ws + (long)blockIdx.x * S * (BM * BN);
  if constexpr (std::is_same<Acc, float>::value && HasStore8<Epi>::value && ReduceVec8<Epi>::value) {
    // eight consecutive columns per thread: vector loads of every split, one
    // vector store through the epilogue
    for (int q = blockIdx.y * blockDim.x + threadIdx.x; q < BM * BN / 8; q += gridDim.y * blockDim.x) {
      const int lr = q / (BN / 8), lc = (q - lr * (BN / 8)) * 8;
      const int row = t.x * BM + lr, col = t.y * BN + lc;
      if (row >= M || col >= N) continue;
      const float* p = base + lr * BN + lc;
      float4 a = *reinterpret_cast<const float4*>(p);
      float4 b = *reinterpret_cast<const float4*>(p + 4);
      for (int z = 1; z < S; ++z) {
        const float4 a2 = *reinterpret_cast<const float4*>(p + (long)z * (BM * BN));
        const float4 b2 = *reinterpret_cast<const float4*>(p + (long)z * (BM * BN) + 4);
        a.x += a2.x; a.y += a2.y; a.z += a2.z; a.w += a2.w;
        b.x += b2.x; b.y += b2.y; b.z += b2.z; b.w += b2.w;
      }
      const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      epi.store8(row, col, v, min(8, N - col));
    }
    return;
  }
  for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < BM * BN; e += gridDim.y * blockDim.x) {
    const int lr = e / BN, lc = e - lr * BN;
    const int row = t.x * BM + lr, col = t.y * BN + lc;
    if (row < M && col < N) {
      Acc v = base[e];
      for (int z = 1; z < S; ++z) v += base[(long)z * (BM * BN) + e];
      epi(row, col, v);
    }
  }
}

// Host-side plan of one product shape.
struct GemmPlan {
  std::vector<PlanItem> items;     // in workgroup order
  std::vector<int2> split_tiles;   // (tm, tn) per workspace slot
  int S = 1;                       // K splits of the split tiles
  int kchunk = 0;                  // K stages per split
  size_t ws_elems() const { return split_tiles.size() * (size_t)S; }   // x BM x BN accumulator values
};

// Full tiles fill whole rounds of `slots` resident workgroups; the tiles of
// a last, partial round are split along K so that they fill one more round
// (at least 4 K stages per split).  Inside a round, tiles are taken in groups
// of 8 tile rows walked column by column, and consecutive runs of that order
// go to the same XCD.
template <class T>
GemmPlan plan_gemm(int M, int N, int kst, int slots) {
  GemmPlan pl;
  const int tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
  constexpr int GROUP_M = 8;
  std::vector<int2> order;
  for (int g0 = 0; g0 < tiles_m; g0 += GROUP_M)
    for (int tn = 0; tn < tiles_n; ++tn)
      for (int tm = g0; tm < std::min(tiles_m, g0 + GROUP_M); ++tm) order.push_back(make_int2(tm, tn));
  const int tiles = (int)order.size();
  const int full = slots > 0 ? (tiles / slots) * slots : tiles;
  const int tail = tiles - full;
  int S = 1;
  if (tail > 0)
    while (S < 16 && tail * S * 2 <= slots && kst / (S * 2) >= 4) S *= 2;
  pl.kchunk = 2 * ((kst + 2 * S - 1) / (2 * S));   // even, like kst
  S = (kst + pl.kchunk - 1) / pl.kchunk;           // every split non-empty
  pl.S = S;
  auto place = [&](const std::vector<PlanItem>& ph) {
    const int n = (int)ph.size();
    if (n % 8 != 0) {
      pl.items.insert(pl.items.end(), ph.begin(), ph.end());
      return;
    }
    const int per = n / 8;
    const size_t base = pl.items.size();
    pl.items.resize(base + n);
    for (int x = 0; x < 8; ++x)
      for (int j = 0; j < per; ++j) pl.items[base + (size_t)8 * j + x] = ph[(size_t)x * per + j];
  };
  for (int r0 = 0; r0 < full; r0 += slots) {
    std::vector<PlanItem> ph;
    for (int i = r0; i < r0 + slots; ++i) ph.push_back(PlanItem{order[i].x, order[i].y, -1, 0});
    place(ph);
  }
  if (tail > 0) {
    std::vector<PlanItem> ph;
    if (S == 1) {
      for (int i = full; i < tiles; ++i) ph.push_back(PlanItem{order[i].x, order[i].y, -1, 0});
    } else {
      for (int i = full; i < tiles; ++i) pl.split_tiles.push_back(order[i]);
      for (int z = 0; z < S; ++z)
        for (int i = full; i < tiles; ++i) ph.push_back(PlanItem{order[i].x, order[i].y, z, i - full});
    }
    place(ph);
  }
  return pl;
}

// Device copy of a plan (arrays owned by the caller's arena).
struct GemmPlanDev {
  const PlanItem* items = nullptr;
  const int2* split_tiles = nullptr;
  int nitems = 0, nsplit = 0, S = 1, kchunk = 0;
  int tile320 = 0;
};

// Launch of a planned product: the tile pass, then (with split tiles) the
// reduction that applies `epi`.  `ws` holds nsplit x S x BM x BN values.
template <int MODE, class Epi>
hipError_t launch_planned(GemmArgs g, const Epi& epi, const GemmPlanDev& pl, typename ModeTraits<MODE>::Acc* ws,
                          hipStream_t s, hipEvent_t mid = nullptr) {
  using T = typename BigTile<MODE>::T;
  using Acc = typename ModeTraits<MODE>::Acc;
  if (g.M <= 0 || g.N <= 0 || pl.nitems == 0) return hipSuccess;
  g.kchunk = pl.kchunk;
  if constexpr (ModeTraits<MODE>::planes == 2) {
    if (pl.tile320) {
      hipLaunchKernelGGL((gemm_planned_kernel<MODE, Tile320, Epi>), dim3(pl.nitems), dim3(Tile320::THREADS), 0, s, g,
                         epi, ws, pl.S, pl.items);
      if (mid) (void)hipEventRecord(mid, s);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((gemm_planned_kernel<MODE, T, Epi>), dim3(pl.nitems), dim3(T::THREADS), 0, s, g, epi, ws,
                     pl.S, pl.items);
  if (mid) (void)hipEventRecord(mid, s);
  if (pl.nsplit > 0) {
    // about 2048 blocks whatever the number of split tiles, up to one work
    // item (eight columns or one element) per thread; each element's sum
    // over the splits keeps its order
    constexpr bool vec8 = std::is_same<Acc, float>::value && HasStore8<Epi>::value && ReduceVec8<Epi>::value;
    constexpr int per_tile = T::BM * T::BN / (vec8 ? 8 : 1) / 256;
    const int ry = std::min(per_tile, std::max(32, 2048 / pl.nsplit));
    hipLaunchKernelGGL((tile_reduce_kernel<Acc, Epi, T::BM, T::BN>), dim3(pl.nsplit, ry), dim3(256), 0, s, ws,
                       pl.S, g.M, g.N, pl.split_tiles, epi);
  }
  return hipGetLastError();
}

}  // namespace sf
