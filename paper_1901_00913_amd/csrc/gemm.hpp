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
// walked in stages of 64 bytes per row through an NS-deep ring of LDS
// buffers filled by direct global-to-LDS loads (see gemm_nt_kernel).
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


// Fragment loads of one stage: P planes x (FM A + FN B) 16-byte LDS reads,
// issued back to back in one asm block that ends with its own lgkmcnt wait,
// so every read has retired when the block ends.  Keeping these reads out of
// the compiler's sight stops its conservative wait on the in-flight
// global-to-LDS loads of later stages (their ordering is enforced by the
// explicit vmcnt wait and barrier at the top of each stage).
template <int P, int FM, int FN> struct FragLoad;

#define SF_R(o, a, off) "ds_read_b128 %" #o ", %" #a " offset:" #off "\n\t"
template <> struct FragLoad<1, 4, 2> {
  static __device__ __forceinline__ void run(uint4 (&fa)[4][1], uint4 (&fb)[2][1], const unsigned (&ra)[1],
                                             const unsigned (&rb)[1]) {
    asm volatile(SF_R(0, 6, 0) SF_R(1, 6, 1024) SF_R(2, 6, 2048) SF_R(3, 6, 3072) SF_R(4, 7, 0) SF_R(5, 7, 1024)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fa[2][0]), "=&v"(fa[3][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0])
                 : "v"(ra[0]), "v"(rb[0])
                 : "memory");
  }
};
template <> struct FragLoad<2, 4, 2> {
  static __device__ __forceinline__ void run(uint4 (&fa)[4][2], uint4 (&fb)[2][2], const unsigned (&ra)[2],
                                             const unsigned (&rb)[2]) {
    asm volatile(SF_R(0, 12, 0) SF_R(1, 12, 1024) SF_R(2, 12, 2048) SF_R(3, 12, 3072) SF_R(4, 13, 0)
                 SF_R(5, 13, 1024) SF_R(6, 14, 0) SF_R(7, 14, 1024) SF_R(8, 14, 2048) SF_R(9, 14, 3072)
                 SF_R(10, 15, 0) SF_R(11, 15, 1024)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fa[2][0]), "=&v"(fa[3][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0]),
                   "=&v"(fa[0][1]), "=&v"(fa[1][1]), "=&v"(fa[2][1]), "=&v"(fa[3][1]), "=&v"(fb[0][1]), "=&v"(fb[1][1])
                 : "v"(ra[0]), "v"(rb[0]), "v"(ra[1]), "v"(rb[1])
                 : "memory");
  }
};
template <> struct FragLoad<1, 4, 4> {
  static __device__ __forceinline__ void run(uint4 (&fa)[4][1], uint4 (&fb)[4][1], const unsigned (&ra)[1],
                                             const unsigned (&rb)[1]) {
    asm volatile(SF_R(0, 8, 0) SF_R(1, 8, 1024) SF_R(2, 8, 2048) SF_R(3, 8, 3072) SF_R(4, 9, 0) SF_R(5, 9, 1024)
                 SF_R(6, 9, 2048) SF_R(7, 9, 3072)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fa[2][0]), "=&v"(fa[3][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0]),
                   "=&v"(fb[2][0]), "=&v"(fb[3][0])
                 : "v"(ra[0]), "v"(rb[0])
                 : "memory");
  }
};
template <> struct FragLoad<2, 4, 4> {
  static __device__ __forceinline__ void run(uint4 (&fa)[4][2], uint4 (&fb)[4][2], const unsigned (&ra)[2],
                                             const unsigned (&rb)[2]) {
    asm volatile(SF_R(0, 16, 0) SF_R(1, 16, 1024) SF_R(2, 16, 2048) SF_R(3, 16, 3072) SF_R(4, 17, 0)
                 SF_R(5, 17, 1024) SF_R(6, 17, 2048) SF_R(7, 17, 3072) SF_R(8, 18, 0) SF_R(9, 18, 1024)
                 SF_R(10, 18, 2048) SF_R(11, 18, 3072) SF_R(12, 19, 0) SF_R(13, 19, 1024) SF_R(14, 19, 2048)
                 SF_R(15, 19, 3072)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fa[2][0]), "=&v"(fa[3][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0]),
                   "=&v"(fb[2][0]), "=&v"(fb[3][0]), "=&v"(fa[0][1]), "=&v"(fa[1][1]), "=&v"(fa[2][1]), "=&v"(fa[3][1]),
                   "=&v"(fb[0][1]), "=&v"(fb[1][1]), "=&v"(fb[2][1]), "=&v"(fb[3][1])
                 : "v"(ra[0]), "v"(rb[0]), "v"(ra[1]), "v"(rb[1])
                 : "memory");
  }
};
template <> struct FragLoad<1, 2, 4> {
  static __device__ __forceinline__ void run(uint4 (&fa)[2][1], uint4 (&fb)[4][1], const unsigned (&ra)[1],
                                             const unsigned (&rb)[1]) {
    asm volatile(SF_R(0, 6, 0) SF_R(1, 6, 1024) SF_R(2, 7, 0) SF_R(3, 7, 1024) SF_R(4, 7, 2048) SF_R(5, 7, 3072)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0]), "=&v"(fb[2][0]), "=&v"(fb[3][0])
                 : "v"(ra[0]), "v"(rb[0])
                 : "memory");
  }
};
template <> struct FragLoad<2, 2, 4> {
  static __device__ __forceinline__ void run(uint4 (&fa)[2][2], uint4 (&fb)[4][2], const unsigned (&ra)[2],
                                             const unsigned (&rb)[2]) {
    asm volatile(SF_R(0, 12, 0) SF_R(1, 12, 1024) SF_R(2, 13, 0) SF_R(3, 13, 1024) SF_R(4, 13, 2048)
                 SF_R(5, 13, 3072) SF_R(6, 14, 0) SF_R(7, 14, 1024) SF_R(8, 15, 0) SF_R(9, 15, 1024)
                 SF_R(10, 15, 2048) SF_R(11, 15, 3072)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0]), "=&v"(fb[2][0]), "=&v"(fb[3][0]),
                   "=&v"(fa[0][1]), "=&v"(fa[1][1]), "=&v"(fb[0][1]), "=&v"(fb[1][1]), "=&v"(fb[2][1]), "=&v"(fb[3][1])
                 : "v"(ra[0]), "v"(rb[0]), "v"(ra[1]), "v"(rb[1])
                 : "memory");
  }
};
template <> struct FragLoad<1, 2, 2> {
  static __device__ __forceinline__ void run(uint4 (&fa)[2][1], uint4 (&fb)[2][1], const unsigned (&ra)[1],
                                             const unsigned (&rb)[1]) {
    asm volatile(SF_R(0, 4, 0) SF_R(1, 4, 1024) SF_R(2, 5, 0) SF_R(3, 5, 1024)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0])
                 : "v"(ra[0]), "v"(rb[0])
                 : "memory");
  }
};
template <> struct FragLoad<2, 2, 2> {
  static __device__ __forceinline__ void run(uint4 (&fa)[2][2], uint4 (&fb)[2][2], const unsigned (&ra)[2],
                                             const unsigned (&rb)[2]) {
    asm volatile(SF_R(0, 8, 0) SF_R(1, 8, 1024) SF_R(2, 9, 0) SF_R(3, 9, 1024) SF_R(4, 10, 0) SF_R(5, 10, 1024)
                 SF_R(6, 11, 0) SF_R(7, 11, 1024)
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0][0]), "=&v"(fa[1][0]), "=&v"(fb[0][0]), "=&v"(fb[1][0]), "=&v"(fa[0][1]), "=&v"(fa[1][1]),
                   "=&v"(fb[0][1]), "=&v"(fb[1][1])
                 : "v"(ra[0]), "v"(rb[0]), "v"(ra[1]), "v"(rb[1])
                 : "memory");
  }
};
#undef SF_R

// 32-bit LDS address of a pointer into __shared__ memory.
__device__ __forceinline__ unsigned lds_addr(const void* p) {
  return static_cast<unsigned>(reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) void*)p));
}

// s_waitcnt immediate that waits until at most N vector-memory operations
// are outstanding (expcnt and lgkmcnt left at their no-wait maxima).
template <int N>
constexpr int vmcnt_imm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  return (N & 0xF) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14);
}

// LDS staging: NS stages, each holding 64 bytes of K for the BM + BN rows of
// every plane, as the 1 KB blocks of the operand layout (op_index: 16 rows x
// 64 K-bytes, chunk-major inside).  An MFMA fragment wants lane l to hold row
// l % 16, chunk l / 16, i.e. byte 16 l of a block, so every fragment read is
// one contiguous 1 KB wave access, the pattern the LDS serves at full rate
// (16-row gathers from a row-major tile run at half rate on gfx950, with or
// without padding or XOR swizzles).
//
// Global -> LDS uses gfx950's global_load_lds_dwordx4: one instruction copies
// one contiguous 1 KB block (lane L moves bytes [16 L, 16 L + 16)).  Loads run
// NS - 1 stages ahead; each stage starts with a wait until the wave's loads of
// that stage have landed and a workgroup barrier that publishes all waves'
// loads (and retires every wave's reads of the stage about to be refilled).
// Workgroup layout: KG groups of (BM/WM) x (BN/WN) waves.  Every group
// covers the whole BM x BN tile; per barrier the workgroup consumes G
// stages and group q computes the stages gg = q (mod KG) of them, so the K
// range is split inside the workgroup.  After the loop the groups add their
// accumulators through LDS and group 0 runs the epilogue.  KG = 2 lets eight
// waves share a 128 x 128 tile with 64 x 64 sub-tiles, which halves the LDS
// fragment traffic per MFMA compared with 64 x 32 sub-tiles.
template <int MODE, class T, class Epi>
__device__ __forceinline__ void gemm_tile(unsigned char* lds, const GemmArgs& g, int tm, int tn, int kz,
                                          const Epi& epi) {
  using Tr = ModeTraits<MODE>;
  using AccT = typename AccVec<MODE>::T;
  using Acc = typename Tr::Acc;
  constexpr int BM = T::BM, BN = T::BN, WM = T::WM, WN = T::WN, NS = T::NS, G = T::G, KG = T::KG;
  constexpr int P = Tr::planes;
  constexpr int WAVES_N = BN / WN;
  constexpr int NWG = (BM / WM) * WAVES_N;    // waves per K group
  constexpr int NW = KG * NWG;
  constexpr int SEGB = 64;                    // K bytes per row per stage
  constexpr int ROWS = BM + BN;
  constexpr int PLANEB = ROWS * SEGB;         // bytes per plane per stage
  constexpr int STAGEB = P * PLANEB;
  constexpr int NINS = P * ROWS / 16;         // 16-row load instructions per stage
  constexpr int IPI = G * NINS / NW;          // load instructions per wave per barrier interval
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert((G * NINS) % NW == 0 && BM % 16 == 0 && BN % 16 == 0, "tile/waves");
  static_assert(G >= 1 && NS >= 2 * G && NS % G == 0 && G % KG == 0, "stages per barrier");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int grp = wave / NWG;
  const int wig = wave - grp * NWG;
  const int wm = wig / WAVES_N;
  const int wn = wig - wm * WAVES_N;
  const int ktot = (g.K * Tr::esize + SEGB - 1) / SEGB;
  const int kt0 = kz * g.kchunk;
  const int ktiles = min(ktot - kt0, g.kchunk);   // >= 1 by construction of the split

  // This wave's load instructions for one barrier interval: stage offset
  // (0..G-1), global source of its lane, LDS offset inside a stage.
  const unsigned char* src[IPI];
  int dst[IPI], sof[IPI];
  {
    const long nseg_a = g.lda * Tr::esize / SEGB;   // K blocks per 16-row block of A
    const long nseg_b = g.ldb * Tr::esize / SEGB;
#pragma unroll
    for (int i = 0; i < IPI; ++i) {
      const int q = wave + NW * i;
      const int gg = q / NINS;
      const int r = q - gg * NINS;
      const int p = r / (ROWS / 16);
      const int rg = r - p * (ROWS / 16);
      const unsigned char* base;
      if (rg < BM / 16)
        base = static_cast<const unsigned char*>(g.a[p]) + ((long)(tm * (BM / 16) + rg) * nseg_a + kt0) * 1024;
      else
        base = static_cast<const unsigned char*>(g.b[p]) +
               ((long)(tn * (BN / 16) + rg - BM / 16) * nseg_b + kt0) * 1024;
      src[i] = base + lane * 16;
      dst[i] = p * PLANEB + rg * 16 * SEGB;
      sof[i] = gg;
    }
  }

  // issue the G stages [J G, J G + G) into their ring buffers (indices past
  // the end are clamped; the re-read lands in a buffer never consumed again)
#define SF_ISSUE_GROUP(J)                                                                            \
  {                                                                                                  \
    _Pragma("unroll") for (int i_ = 0; i_ < IPI; ++i_) {                                             \
      const int st_ = (J) * G + sof[i_];                                                             \
      __builtin_amdgcn_global_load_lds(                                                              \
          (const void __attribute__((address_space(1)))*)(src[i_] + (long)min(st_, ktiles - 1) * 1024), \
          (void __attribute__((address_space(3)))*)(lds + (st_ % NS) * STAGEB + dst[i_]), 16, 0, 0); \
    }                                                                                                \
  }

  AccT acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = AccT{0, 0, 0, 0};

  // fragment reads: 16-row block i of this wave's rows, byte 16 lane of it
  const int a_off = wm * WM * SEGB + lane * 16;
  const int b_off = (BM + wn * WN) * SEGB + lane * 16;

  // Loads run NS - G stages ahead of the first stage consumed; at the top of
  // an interval NS - 2G stages may remain in flight.
  constexpr int AHEAD = (NS - G) / G;
#pragma unroll
  for (int j = 0; j < AHEAD; ++j) SF_ISSUE_GROUP(j);

  const int iters = (ktiles + G - 1) / G;
  for (int it = 0; it < iters; ++it) {
    __builtin_amdgcn_s_waitcnt(vmcnt_imm<(AHEAD - 1) * IPI>());
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    SF_ISSUE_GROUP(it + AHEAD);
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      if (KG > 1 && (gg % KG) != grp) continue;
      const int kt = it * G + gg;
      if (G > 1 && kt >= ktiles) break;
      const unsigned char* sbase = lds + (kt % NS) * STAGEB;
      uint4 fa[FM][P], fb[FN][P];
      {
        unsigned ra[P], rb[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          ra[p] = lds_addr(sbase + p * PLANEB + a_off);
          rb[p] = lds_addr(sbase + p * PLANEB + b_off);
        }
        FragLoad<P, FM, FN>::run(fa, fb, ra, rb);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) mma_chunk<MODE>(acc[i][j], fa[i], fb[j]);
    }
    asm volatile("" ::: "memory");
  }
  __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());
#undef SF_ISSUE_GROUP

  if constexpr (KG > 1) {
    // groups 1.. hand their partial sums to group 0 through LDS (fixed order)
    Acc* red = reinterpret_cast<Acc*>(lds);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    for (int q = 1; q < KG; ++q) {
      if (grp == q) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) red[(((wig * FM + i) * FN + j) * 4 + t) * 64 + lane] = acc[i][j][t];
      }
      __syncthreads();
      if (grp == 0) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[i][j][t] += red[(((wig * FM + i) * FN + j) * 4 + t) * 64 + lane];
      }
      __syncthreads();
    }
    if (grp != 0) return;
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

// Tile configurations.  TileL (128 x 128, 8 waves of 64 x 32, two 64 KB
// LDS stages for bf16x3) is the single-image shape; TileS (64 x 64, 4 waves
// of 32 x 32) serves small images in the batched form.
#ifndef SF_TILE_BM
#define SF_TILE_BM 128
#define SF_TILE_BN 128
#define SF_TILE_WM 64
#define SF_TILE_WN 32
#define SF_TILE_NS 2
#endif
#ifndef SF_TILE_G
#define SF_TILE_G 1
#endif
#ifndef SF_TILE_KG
#define SF_TILE_KG 1
#endif
template <int BM_, int BN_, int WM_, int WN_, int NS_, int G_, int KG_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int NS = NS_;   // LDS pipeline stages of 64 K-bytes
  static constexpr int G = G_;     // stages consumed per barrier
  static constexpr int KG = KG_;   // K groups of waves inside a workgroup
  static constexpr int THREADS = KG * (BM / WM) * (BN / WN) * 64;
  template <int MODE>
  static constexpr int lds_bytes() {
    using Acc = typename ModeTraits<MODE>::Acc;
    constexpr int stages = NS * ModeTraits<MODE>::planes * (BM + BN) * 64;
    constexpr int red = KG > 1 ? BM * BN * (int)sizeof(Acc) : 0;
    return stages > red ? stages : red;
  }
};
using TileL = Tile<SF_TILE_BM, SF_TILE_BN, SF_TILE_WM, SF_TILE_WN, SF_TILE_NS, SF_TILE_G, SF_TILE_KG>;
using TileS = Tile<64, 64, 32, 32, 4, 1, 1>;

struct TileCfg {
  static constexpr int ROW_PAD = 256;     // operand row allocations are multiples of this
  static constexpr int K_PAD = 64;        // operand leading dimensions are multiples of this
  static_assert(TileL::BM <= ROW_PAD && TileL::BN <= ROW_PAD, "row padding must cover a tile");
};

template <int MODE, class T = TileL>
constexpr size_t gemm_lds_bytes() { return (size_t)T::template lds_bytes<MODE>(); }

template <int MODE, class T, class Epi>
__global__ __launch_bounds__(T::THREADS, 1) void gemm_nt_kernel(GemmArgs g, Epi epi) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[T::template lds_bytes<MODE>()];
  const int tiles_m = (g.M + T::BM - 1) / T::BM;
  const int tiles_n = (g.N + T::BN - 1) / T::BN;
  int tm, tn;
  map_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
  gemm_tile<MODE, T>(lds, g, tm, tn, blockIdx.y, epi);
}

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
  __shared__ __attribute__((aligned(16))) unsigned char lds[T::template lds_bytes<MODE>()];
  int bid = blockIdx.x;
  if ((gridDim.x & 7) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  const WorkItem w = work[bid];
  const GemmArgs g = args[w.prod];
  const Epi e = epis[w.prod];
  gemm_tile<MODE, T>(lds, g, w.tm, w.tn, 0, e);
}

// Partial product of one K split, stored for the reduction.
template <int MODE>
struct EpiPartial {
  typename ModeTraits<MODE>::Acc* ws;
  int M, N;
  __device__ __forceinline__ void operator()(int row, int col, typename ModeTraits<MODE>::Acc v) const {
    ws[((long)blockIdx.y * M + row) * N + col] = v;
  }
};

// Sums the K-split partials in split order (deterministic) and applies the
// GEMM's own epilogue element-wise.
template <class Acc, class Epi>
__global__ void splitk_reduce_kernel(const Acc* ws, int S, int M, int N, Epi epi) {
  const long total = (long)M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    Acc v = ws[e];
    for (int z = 1; z < S; ++z) v += ws[z * total + e];
    const int row = (int)(e / N);
    epi(row, (int)(e - (long)row * N), v);
  }
}

template <int MODE>
inline int gemm_kstages(int K) { return (K * ModeTraits<MODE>::esize + 63) / 64; }

// Number of K splits for an M x N x K product: enough workgroups to fill
// `slots` (CUs x resident blocks per CU), keeping at least 16 K stages per split.
template <int MODE>
inline int choose_splitk(int M, int N, int K, int slots) {
  const int tiles = ((M + TileL::BM - 1) / TileL::BM) * ((N + TileL::BN - 1) / TileL::BN);
  const int kst = gemm_kstages<MODE>(K);
  int S = 1;
  while (S < 16 && tiles * S * 2 <= slots && kst / (S * 2) >= 16) S *= 2;
  return S;
}

// Launch; with S > 1 the partials go to `ws` (S x M x N accumulator values)
// and the reduction applies `epi`.
template <int MODE, class Epi>
hipError_t launch_gemm(GemmArgs g, const Epi& epi, hipStream_t s, int S = 1,
                       typename ModeTraits<MODE>::Acc* ws = nullptr) {
  using T = TileL;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int tiles = ((g.M + T::BM - 1) / T::BM) * ((g.N + T::BN - 1) / T::BN);
  constexpr int threads = T::THREADS;
  const int kst = gemm_kstages<MODE>(g.K);
  if (S <= 1 || !ws) {
    g.kchunk = kst;
    hipLaunchKernelGGL((gemm_nt_kernel<MODE, T, Epi>), dim3(tiles),
                       dim3(threads), 0, s, g, epi);
    return hipGetLastError();
  }
  g.kchunk = (kst + S - 1) / S;
  S = (kst + g.kchunk - 1) / g.kchunk;   // every split non-empty
  EpiPartial<MODE> part{ws, g.M, g.N};
  hipLaunchKernelGGL((gemm_nt_kernel<MODE, T, EpiPartial<MODE>>),
                     dim3(tiles, S), dim3(threads), 0, s, g, part);
  hipLaunchKernelGGL((splitk_reduce_kernel<typename ModeTraits<MODE>::Acc, Epi>), dim3(2048), dim3(256), 0, s,
                     ws, S, g.M, g.N, epi);
  return hipGetLastError();
}

}  // namespace sf
