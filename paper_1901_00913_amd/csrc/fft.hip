// Structured-FFT form of Algorithm 2: the Kronecker factors are applied
// through their generator vectors with 1-D FFTs (Section 3.3) instead of as
// dense GEMMs.
//
// A factor F = toep(c, c0 + 1) [+ hank(c, c0 + 1)] (Section 2; Hankel part
// for the reflexive boundary) applied to a line z of length M is a linear
// convolution:  (F z)[i] = sum_t c[t] z_ext[i + c0 - t], where z_ext extends
// z by zeros or by its half-sample mirror image.  With w[p] = z_ext[p + c0 -
// (M - 1)] for p < 2M - 1, (F z)[i] is entry i + M - 1 of the circular
// convolution of w and c, both zero-padded to N >= 2M - 1 points, so one FFT
// of the line, a product with the generator's spectrum and one inverse FFT
// give it.  F^T z is the adjoint chain: z placed at M - 1 .. 2M - 2, the
// circular correlation with c (conjugate spectrum), and the extension folded
// back onto the entries it copied.
//
// Two real lines share one complex transform (one as the real part, one as
// the imaginary part); the product with the spectrum of a real generator and
// the inverse transform keep them apart.  The transform is a mixed-radix
// Stockham FFT (radix 16, then 2, 4 or 8) held in LDS: each pass reads its
// butterflies' inputs into registers, synchronises, and writes the outputs in
// place.  At 4096 points (256 threads) each thread's first-pass inputs and
// last-pass outputs are the points it loads and stores itself, so those two
// passes run from and to registers and a transform takes two LDS exchanges.
// Twiddles come from a table, three reads per pass, the other powers by
// products.  Transforms are FP32; the iterates are FP64.
//
// One iteration is four line passes over the image (m x n, row-major), in
// three kernels (F2 and G1 run along the same lines and share one):
//   F1  T_k = Y A_k^T      rows of Y, one transform in, r out (stored T_k^T)
//   F2  R = sum_k B_k T_k - Bobs   rows of T_k^T, r in, one out
//   G1  S_k = B_k^T R      the same lines, one in, r out (S_k^T)
//   G2  G = sum_k S_k A_k  rows of S_k (columns of S_k^T), r in, one out,
//       fused with Steps 1 and 3 (X_k and Y_{k+1}).
// C ABI declared in include/sfista.h.
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sfista.h"
#include "kernels.hpp"
#include "util.hpp"

using namespace sf;

namespace {

constexpr int FFT_NMIN = 64;
constexpr int FFT_NMAX = 8192;   // lines of up to 4096 entries
constexpr int FFT_RMAX = 64;     // Kronecker terms
constexpr int EW_BLOCKS_FFT = 2048;

struct DiffSq64 {        // ||a - b||^2 term
  const double* a; const double* b;
  __device__ double operator()(long e) const { return a[e] - b[e]; }
};

__host__ __device__ constexpr int fft_threads(int N) { return N / 16 < 64 ? 64 : (N / 16 > 512 ? 512 : N / 16); }

inline int fft_size(int M) {
  int N = FFT_NMIN;
  while (N < 2 * M - 1) N *= 2;
  return N;
}

// ------------------------------------------------------------ complex math
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {   // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 mul_negi(float2 a) { return make_float2(a.y, -a.x); }   // -i a

// exp(-2 pi i e / 16) for a compile-time e in [0, 16)
template <int E>
__device__ __forceinline__ float2 w16() {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
  constexpr double cs[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
  constexpr double sn[16] = {0, s1, h, c1, 1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1};
  return make_float2((float)cs[E % 16], (float)-sn[E % 16]);
}

template <int E>
__device__ __forceinline__ float2 rot16(float2 a) {
  if constexpr (E % 16 == 0) return a;
  else if constexpr (E % 16 == 4) return mul_negi(a);
  else return cmul(a, w16<E>());
}

// Forward DFTs in registers, natural order in and out.
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const float2 s13 = cadd(a1, a3), d13 = mul_negi(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

// Two-step split N = N1 N2 with n = n1 + N1 n2 and k = k2 + N2 k1: DFTs of
// length N2 over n2, twiddles W_N^(n1 k2), DFTs of length N1 over n1.
template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R]);

template <>
__device__ __forceinline__ void dft<2>(float2 (&v)[2]) { dft2(v[0], v[1]); }

template <>
__device__ __forceinline__ void dft<4>(float2 (&v)[4]) { dft4(v[0], v[1], v[2], v[3]); }

template <>
__device__ __forceinline__ void dft<8>(float2 (&v)[8]) {   // N1 = 2, N2 = 4
  dft4(v[0], v[2], v[4], v[6]);
  dft4(v[1], v[3], v[5], v[7]);
  // y[n1][k2] sits at v[n1 + 2 k2]; twiddle W8^(n1 k2) = W16^(2 n1 k2)
  v[3] = rot16<2>(v[3]);
  v[5] = rot16<4>(v[5]);
  v[7] = rot16<6>(v[7]);
  float2 o[8];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 a = v[2 * k2], b = v[2 * k2 + 1];
    dft2(a, b);
    o[k2] = a;
    o[k2 + 4] = b;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = o[k];
}

template <>
__device__ __forceinline__ void dft<16>(float2 (&v)[16]) {   // N1 = N2 = 4
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) dft4(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
  // y[n1][k2] sits at v[n1 + 4 k2]; twiddle W16^(n1 k2)
  v[5] = rot16<1>(v[5]);   v[6] = rot16<2>(v[6]);   v[7] = rot16<3>(v[7]);
  v[9] = rot16<2>(v[9]);   v[10] = rot16<4>(v[10]); v[11] = rot16<6>(v[11]);
  v[13] = rot16<3>(v[13]); v[14] = rot16<6>(v[14]); v[15] = rot16<9>(v[15]);
  float2 o[16];
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 a0 = v[4 * k2], a1 = v[4 * k2 + 1], a2 = v[4 * k2 + 2], a3 = v[4 * k2 + 3];
    dft4(a0, a1, a2, a3);
    o[k2] = a0;
    o[k2 + 4] = a1;
    o[k2 + 8] = a2;
    o[k2 + 12] = a3;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}

// w[r] = W_N^(t r) for r < R from three table reads (W^t, W^4t, W^8t) and
// products: each power is at most three roundings away from the table, while
// the pass needs no more than three loads instead of R - 1.
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 (&w)[R], const float2* __restrict__ tw, int t) {
  w[0] = make_float2(1.f, 0.f);
  w[1] = tw[t];
  if constexpr (R >= 4) {
    w[2] = cmul(w[1], w[1]);
    w[3] = cmul(w[2], w[1]);
  } else {
    return;
  }
  if constexpr (R >= 8) {
    w[4] = tw[4 * t];
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
  }
  if constexpr (R >= 16) {
    w[8] = tw[8 * t];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
  }
}

// Stockham passes, radix 16 first, then 2, 4 or 8; pass (NS, R) works on
// sub-transforms of size NS already done: butterfly j reads points
// j + r N/R (twiddled by W_N^((j mod NS) r N/(NS R))) and writes points
// (j / NS) NS R + j mod NS + r NS.  Thread t takes butterflies t + u FT.
// A transform may start from registers and end in registers: thread t then
// holds points t + v FT (x[v], v < N / FT).  The first pass reads exactly
// those points (butterfly t + u FT, input r is point t + (u + r U) FT with
// U = N / (R FT)), and the last pass writes them, whenever N / R is a
// multiple of FT; otherwise the points go through LDS.
template <int N, int R>
constexpr bool regs_ok() { return (N / R) % fft_threads(N) == 0; }

constexpr int last_radix(int N) {
  int ns = 1;
  while (N / ns > 16) ns *= 16;
  return N / ns;
}

template <int N, int NS, bool IN_REGS, bool OUT_REGS>
__device__ __forceinline__ void fft_passes(float2 (&x)[N / fft_threads(N)], float2* buf,
                                           const float2* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = N / NS >= 16 ? 16 : N / NS;
    constexpr int FT = fft_threads(N);
    constexpr int NB = N / R;
    constexpr int U = (NB + FT - 1) / FT;
    constexpr bool LAST = NS * R == N;
    constexpr bool FROM_REGS = NS == 1 && IN_REGS;
    constexpr bool TO_REGS = LAST && OUT_REGS;
    static_assert(!FROM_REGS || regs_ok<N, R>(), "first pass cannot start from registers");
    static_assert(!TO_REGS || regs_ok<N, R>(), "last pass cannot end in registers");
    float2 v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = (int)threadIdx.x + u * FT;
      if (NB % FT == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (FROM_REGS) v[u][r] = x[u + r * U];
          else v[u][r] = buf[j + r * NB];
        }
        if constexpr (NS > 1) {
          float2 w[R];
          twiddle_powers<R>(w, tw, (j % NS) * (N / (NS * R)));
#pragma unroll
          for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], w[r]);
        }
        dft<R>(v[u]);
      }
    }
    if constexpr (TO_REGS) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) x[u + r * U] = v[u][r];
    } else {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = (int)threadIdx.x + u * FT;
        if (NB % FT == 0 || j < NB) {
          const int d = (j / NS) * NS * R + j % NS;
#pragma unroll
          for (int r = 0; r < R; ++r) buf[d + r * NS] = v[u][r];
        }
      }
      __syncthreads();
      fft_passes<N, NS * R, IN_REGS, OUT_REGS>(x, buf, tw);
    }
  }
}

// Forward FFT of N points.  IN: the points are x (thread t holds t + v FT)
// rather than buf (complete and synchronised).  OUT: the result is left in
// x rather than in buf (then synchronised).  A transform that starts from
// registers begins with a barrier, so buf may still be read by the caller's
// previous loop; one that ends in registers leaves buf to be written only
// after a barrier.  The register forms fall back to LDS when the pass
// shapes do not allow them.
template <int N, bool IN, bool OUT>
__device__ __forceinline__ void fft(float2 (&x)[N / fft_threads(N)], float2* buf, const float2* __restrict__ tw) {
  constexpr int FT = fft_threads(N);
  constexpr bool IN_OK = IN && regs_ok<N, (N >= 16 ? 16 : N)>();
  constexpr bool OUT_OK = OUT && regs_ok<N, last_radix(N)>();
  if constexpr (IN && !IN_OK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < N / FT; ++u) buf[threadIdx.x + u * FT] = x[u];
    __syncthreads();
  }
  fft_passes<N, 1, IN_OK, OUT_OK>(x, buf, tw);
  if constexpr (OUT && !OUT_OK) {
#pragma unroll
    for (int u = 0; u < N / FT; ++u) x[u] = buf[threadIdx.x + u * FT];
  }
}

// Workgroup -> line pair: consecutive pairs on one XCD (workgroups are
// dealt to the 8 XCDs in turn), so the L2 of that XCD sees whole lines of
// the transposed arrays.
__device__ __forceinline__ int line_group() {
  const int b = (int)blockIdx.x, nb = (int)gridDim.x;
  if (nb % 8) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

// Source index of extended position e of a line of length M (-1: zero).
__device__ __forceinline__ int ext_src(int e, int M, int refl) {
  if (e >= 0 && e < M) return e;
  if (!refl) return -1;
  return e < 0 ? -1 - e : 2 * M - 1 - e;
}

// ------------------------------------------------------------ line access
// FP64 rows (an image m x n), optionally scaled by 1 / sqrt(*ss).
struct RowsF64 {
  const double* p;
  long ld;
  const double* ss;
  __device__ float2 get2(int /*k*/, int a, bool bv, int e, double scale) const {
    const double va = p[(long)a * ld + e] * scale;
    const double vb = bv ? p[(long)(a + 1) * ld + e] * scale : 0.0;
    return make_float2((float)va, (float)vb);
  }
};

// FP32 lines of r arrays: element (k, line, e) at p[k ks + line ls + e es].
// ADJ: the two lines of a pair are adjacent in memory (ls = 1).
template <bool ADJ>
struct LinesF32 {
  const float* p;
  long ls, es, ks;
  const double* ss;   // unused
  __device__ float2 get2(int k, int a, bool bv, int e, double) const {
    const float* q = p + (long)k * ks + (long)e * es;
    if constexpr (ADJ) {
      if (bv) return *reinterpret_cast<const float2*>(q + a);
      return make_float2(q[a], 0.f);
    } else {
      return make_float2(q[(long)a * ls], bv ? q[(long)(a + 1) * ls] : 0.f);
    }
  }
};

// Fan-out outputs: term k, lines a and a + 1 (valid when bv), entry e.
struct OutTransposed {   // T_k^T[e][line]
  float* p;
  long ld, ks;
  __device__ void put2(int k, int a, bool bv, int e, float va, float vb) const {
    float* q = p + (long)k * ks + (long)e * ld + a;
    if (bv) *reinterpret_cast<float2*>(q) = make_float2(va, vb);
    else *q = va;
  }
};

struct OutRows {         // S_k^T[line][e]
  float* p;
  long ld, ks;
  __device__ void put2(int k, int a, bool bv, int e, float va, float vb) const {
    float* q = p + (long)k * ks + (long)a * ld + e;
    q[0] = va;
    if (bv) q[ld] = vb;
  }
};

// Fan-in epilogues: line L, entry e, value v of the summed product.
struct EpiResidT {       // R^T[line][e] = v - Bobs^T (when given); optional FP64 copy
  float* rt;
  long ld;
  const float* bobst;
  double* out64;
  long o_line, o_e;
  __device__ void put(int L, int e, float v) const {
    const float r = bobst ? v - bobst[(long)L * ld + e] : v;
    rt[(long)L * ld + e] = r;
    if (out64) out64[(long)L * o_line + (long)e * o_e] = (double)r;
  }
};

struct EpiUpdate {       // Steps 1 and 3 of Algorithm 2 on row L
  const double* xprev;
  double* xout;
  double* y;             // Y_k in, Y_{k+1} out
  long ld;
  double c1, c2, beta;   // c1 = L / (L + lambda^2), c2 = 1 / (L + lambda^2)
  int nonneg;
  __device__ void put(int L, int e, float g) const {
    const long i = (long)L * ld + e;
    double x = c1 * y[i] - c2 * (double)g;
    if (nonneg) x = x > 0.0 ? x : 0.0;
    xout[i] = x;
    y[i] = x + beta * (x - xprev[i]);
  }
};

struct EpiStore64 {      // the product itself, FP64 rows
  double* out;
  long ld;
  __device__ void put(int L, int e, float g) const { out[(long)L * ld + e] = (double)g; }
};

// Entry s of the fold of the extension (adjoint of the load of a line of
// length M into w): the correlated line u is in buf.
__device__ __forceinline__ float2 fold_at(const float2* buf, int s, int M, int c0, int refl) {
  float2 w = buf[s + M - 1 - c0];
  if (refl) {
    const int p1 = M - 2 - s - c0;
    if (p1 >= 0) w = cadd(w, buf[p1]);
    const int p2 = 3 * M - 2 - s - c0;
    if (p2 <= 2 * M - 2) w = cadd(w, buf[p2]);
  }
  return w;
}

// Point e of the transform input for lines a, a + 1 of term k: the
// extension w (CONV) or the line at M - 1 .. 2M - 2 (CORR), zero elsewhere.
template <bool CORR, class In>
__device__ __forceinline__ float2 input_point(const In& in, int k, int a, bool bv, int e, int M, int c0, int refl,
                                              double scale) {
  float2 v = make_float2(0.f, 0.f);
  if constexpr (CORR) {
    if (e >= M - 1 && e < 2 * M - 1) v = in.get2(k, a, bv, e - (M - 1), scale);
  } else {
    if (e < 2 * M - 1) {
      const int src = ext_src(e + c0 - (M - 1), M, refl);
      if (src >= 0) v = in.get2(k, a, bv, src, scale);
    }
  }
  return v;
}

// The input points a thread holds: x[u] = point t + u FT.
template <int N, bool CORR, class In>
__device__ __forceinline__ void fetch_pair(float2 (&x)[N / fft_threads(N)], const In& in, int k, int a, bool bv, int M,
                                           int c0, int refl, double scale) {
  constexpr int FT = fft_threads(N);
#pragma unroll
  for (int u = 0; u < N / FT; ++u)
    x[u] = input_point<CORR>(in, k, a, bv, (int)threadIdx.x + u * FT, M, c0, refl, scale);
}

// One line pair in, one out per term (F1, G1).
template <int N, bool CORR, class In, class Out>
__global__ __launch_bounds__(fft_threads(N)) void fan_out_kernel(In in, Out out, const float2* __restrict__ spec,
                                                               const float2* __restrict__ tw, int M, int nlines,
                                                               int c0, int refl, int r) {
  constexpr int FT = fft_threads(N);
  constexpr int PER = N / FT;
  __shared__ float2 buf[N];
  const int a = 2 * line_group();
  if (a >= nlines) return;
  const bool bv = a + 1 < nlines;
  const double scale = in.ss ? 1.0 / sqrt(*in.ss) : 1.0;
  float2 z[PER];
  fetch_pair<N, CORR>(z, in, 0, a, bv, M, c0, refl, scale);
  fft<N, true, true>(z, buf, tw);   // the spectrum, point t + u FT in z[u]
  const float inv = 1.0f / (float)N;
  for (int k = 0; k < r; ++k) {
    const float2* sk = spec + (long)k * N;
    float2 x[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = (int)threadIdx.x + u * FT;
      const float2 p = CORR ? cmulconj(z[u], sk[e]) : cmul(z[u], sk[e]);
      x[u] = make_float2(p.x, -p.y);   // conjugate: the inverse runs as a forward FFT
    }
    if constexpr (CORR) {            // the fold gathers points of other threads: through LDS
      fft<N, true, false>(x, buf, tw);
      for (int e = (int)threadIdx.x; e < M; e += FT) {
        const float2 w = fold_at(buf, e, M, c0, refl);
        out.put2(k, a, bv, e, w.x * inv, -w.y * inv);
      }
    } else {                         // the crop keeps points M - 1 .. 2M - 2 where they are
      fft<N, true, true>(x, buf, tw);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int p = (int)threadIdx.x + u * FT;
        if (p >= M - 1 && p < 2 * M - 1) out.put2(k, a, bv, p - (M - 1), x[u].x * inv, -x[u].y * inv);
      }
    }
  }
}

// r line pairs in (one per term), their products summed, one out (F2, G2).
template <int N, bool CORR, class In, class Epi>
__global__ __launch_bounds__(fft_threads(N)) void fan_in_kernel(In in, Epi epi, const float2* __restrict__ spec,
                                                              const float2* __restrict__ tw, int M, int nlines,
                                                              int c0, int refl, int r) {
  constexpr int FT = fft_threads(N);
  constexpr int PER = N / FT;
  __shared__ float2 buf[N];
  const int a = 2 * line_group();
  if (a >= nlines) return;
  const bool bv = a + 1 < nlines;
  float2 acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = make_float2(0.f, 0.f);
  for (int k = 0; k < r; ++k) {
    float2 x[PER];
    fetch_pair<N, CORR>(x, in, k, a, bv, M, c0, refl, 1.0);
    fft<N, true, true>(x, buf, tw);
    const float2* sk = spec + (long)k * N;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = (int)threadIdx.x + u * FT;
      acc[u] = cadd(acc[u], CORR ? cmulconj(x[u], sk[e]) : cmul(x[u], sk[e]));
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = make_float2(acc[u].x, -acc[u].y);
  const float inv = 1.0f / (float)N;
  if constexpr (CORR) {
    fft<N, true, false>(acc, buf, tw);
    for (int e = (int)threadIdx.x; e < M; e += FT) {
      const float2 w = fold_at(buf, e, M, c0, refl);
      epi.put(a, e, w.x * inv);
      if (bv) epi.put(a + 1, e, -w.y * inv);
    }
  } else {
    fft<N, true, true>(acc, buf, tw);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int p = (int)threadIdx.x + u * FT;
      if (p >= M - 1 && p < 2 * M - 1) {
        epi.put(a, p - (M - 1), acc[u].x * inv);
        if (bv) epi.put(a + 1, p - (M - 1), -acc[u].y * inv);
      }
    }
  }
}

// Column pass of an iteration, F2 then G1 on the same pair of columns:
// R = sum_k B_k T_k - Bobs (fan-in convolution), whose cropped points are
// already in registers at the positions the correlation of G1 reads them, so
// R goes from the inverse transform of F2 straight into the forward
// transform of G1 as FP32 values (the separate passes exchange the same
// values through memory, up to the compiler's contraction of the scaling
// into the subtraction of Bobs); then S_k = B_k^T R (fan-out correlation
// and fold).
template <int N>
__global__ __launch_bounds__(fft_threads(N)) void column_pass_kernel(LinesF32<false> in, const float* __restrict__ bobst,
                                                                   long ldb, OutRows out,
                                                                   const float2* __restrict__ spec,
                                                                   const float2* __restrict__ tw, int M, int nlines,
                                                                   int c0, int refl, int r) {
  constexpr int FT = fft_threads(N);
  constexpr int PER = N / FT;
  __shared__ float2 buf[N];
  const int a = 2 * line_group();
  if (a >= nlines) return;
  const bool bv = a + 1 < nlines;
  float2 acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = make_float2(0.f, 0.f);
  for (int k = 0; k < r; ++k) {
    float2 x[PER];
    fetch_pair<N, false>(x, in, k, a, bv, M, c0, refl, 1.0);
    fft<N, true, true>(x, buf, tw);
    const float2* sk = spec + (long)k * N;
#pragma unroll
    for (int u = 0; u < PER; ++u) acc[u] = cadd(acc[u], cmul(x[u], sk[(int)threadIdx.x + u * FT]));
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = make_float2(acc[u].x, -acc[u].y);
  fft<N, true, true>(acc, buf, tw);
  const float inv = 1.0f / (float)N;
#pragma unroll
  for (int u = 0; u < PER; ++u) {   // the residual, placed as G1's correlation input
    const int p = (int)threadIdx.x + u * FT;
    float2 v = make_float2(0.f, 0.f);
    if (p >= M - 1 && p < 2 * M - 1) {
      const int e = p - (M - 1);
      v.x = acc[u].x * inv - bobst[(long)a * ldb + e];
      if (bv) v.y = -acc[u].y * inv - bobst[(long)(a + 1) * ldb + e];
    }
    acc[u] = v;
  }
  fft<N, true, true>(acc, buf, tw);
  for (int k = 0; k < r; ++k) {
    const float2* sk = spec + (long)k * N;
    float2 x[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const float2 q = cmulconj(acc[u], sk[(int)threadIdx.x + u * FT]);
      x[u] = make_float2(q.x, -q.y);
    }
    fft<N, true, false>(x, buf, tw);
    for (int e = (int)threadIdx.x; e < M; e += FT) {
      const float2 w = fold_at(buf, e, M, c0, refl);
      out.put2(k, a, bv, e, w.x * inv, -w.y * inv);
    }
  }
}

// Spectrum of generator k (length M, zero-padded to N): spec[k N + e].
template <int N>
__global__ __launch_bounds__(fft_threads(N)) void spectrum_kernel(const double* gen, int M, float2* spec,
                                                                const float2* __restrict__ tw) {
  constexpr int FT = fft_threads(N);
  __shared__ float2 buf[N];
  const int k = (int)blockIdx.x;
  float2 x[N / FT];
#pragma unroll
  for (int u = 0; u < N / FT; ++u) {
    const int e = (int)threadIdx.x + u * FT;
    x[u] = make_float2(e < M ? (float)gen[(long)k * M + e] : 0.f, 0.f);
  }
  fft<N, true, true>(x, buf, tw);
#pragma unroll
  for (int u = 0; u < N / FT; ++u) spec[(long)k * N + threadIdx.x + u * FT] = x[u];
}

// Bobs (m x n, FP64) -> Bobs^T (n x ld, FP32).
static __global__ void transpose_f32_kernel(const double* src, float* dst, int m, int n, long ld) {
  __shared__ float tile[32][33];
  const int j0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
  for (int t = threadIdx.y; t < 32; t += blockDim.y) {
    const int i = i0 + t, j = j0 + threadIdx.x;
    if (i < m && j < n) tile[t][threadIdx.x] = (float)src[(long)i * n + j];
  }
  __syncthreads();
  for (int t = threadIdx.y; t < 32; t += blockDim.y) {
    const int j = j0 + t, i = i0 + threadIdx.x;
    if (j < n && i < m) dst[(long)j * ld + i] = tile[threadIdx.x][t];
  }
}

static __global__ void fill_f64_kernel(double* a, double* b, double* c, const double* src, long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
    const double v = src ? src[e] : 0.0;
    a[e] = v;
    b[e] = v;
    c[e] = v;
  }
}

// Runs f.template operator()<N>() for the runtime FFT size N.
template <class F>
hipError_t with_size(int N, F&& f) {
  switch (N) {
    case 64: return f.template operator()<64>();
    case 128: return f.template operator()<128>();
    case 256: return f.template operator()<256>();
    case 512: return f.template operator()<512>();
    case 1024: return f.template operator()<1024>();
    case 2048: return f.template operator()<2048>();
    case 4096: return f.template operator()<4096>();
    case 8192: return f.template operator()<8192>();
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

struct sfista_fft {
  int m = 0, n = 0, r = 0, l = 0, q = 0, refl = 0, nonneg = 0;
  double lam = 0.0, L = 0.0, bobs_norm = 0.0;
  hipStream_t s = nullptr;
  long iter = 0;          // iterations completed (k)
  double tk = 1.0;        // t_{k+1}
  int Nm = 0, Nn = 0;     // transform sizes along columns (m) and rows (n)
  long ldt = 0;           // leading dimension of the transposed arrays (>= m, even)
  float2 *twm = nullptr, *twn = nullptr;      // W_N^t tables
  float2 *specH = nullptr, *specK = nullptr;  // r x Nm spectra of h_k, r x Nn of k_k
  double* Y = nullptr;                        // Y_{k+1}, FP64 m x n
  double* X[2] = {};                          // X_k in X[k & 1]
  double* aux = nullptr;                      // m x n FP64 scratch (power iterate, residual)
  double* red = nullptr;                      // reduction partials + scalars
  double* v0buf = nullptr;
  double* lzq[2] = {};           // Lanczos vectors (made on first use)
  double* lzcoef = nullptr;      // Lanczos coefficients
  float *Tt = nullptr, *St = nullptr, *Rt = nullptr, *BobsT = nullptr;
  DeviceArena arena;
};

namespace {

// The four line passes.  `in` is the F1 input (FP64 rows, optionally scaled).
hipError_t pass_f1(sfista_fft* h, const double* x, const double* ss) {
  return with_size(h->Nn, [&]<int N>() -> hipError_t {
    hipLaunchKernelGGL((fan_out_kernel<N, false, RowsF64, OutTransposed>), dim3((h->m + 1) / 2),
                       dim3(fft_threads(N)), 0, h->s, RowsF64{x, h->n, ss},
                       OutTransposed{h->Tt, h->ldt, (long)h->n * h->ldt}, h->specK, h->twn, h->n, h->m, h->q, h->refl,
                       h->r);
    return hipGetLastError();
  });
}

hipError_t pass_f2(sfista_fft* h, bool with_bobs, double* out64, long o_line, long o_e) {
  return with_size(h->Nm, [&]<int N>() -> hipError_t {
    hipLaunchKernelGGL((fan_in_kernel<N, false, LinesF32<false>, EpiResidT>), dim3((h->n + 1) / 2),
                       dim3(fft_threads(N)), 0, h->s,
                       LinesF32<false>{h->Tt, h->ldt, 1, (long)h->n * h->ldt, nullptr},
                       EpiResidT{h->Rt, h->ldt, with_bobs ? h->BobsT : nullptr, out64, o_line, o_e}, h->specH, h->twm,
                       h->m, h->n, h->l, h->refl, h->r);
    return hipGetLastError();
  });
}

hipError_t pass_g1(sfista_fft* h) {
  return with_size(h->Nm, [&]<int N>() -> hipError_t {
    hipLaunchKernelGGL((fan_out_kernel<N, true, LinesF32<false>, OutRows>), dim3((h->n + 1) / 2),
                       dim3(fft_threads(N)), 0, h->s, LinesF32<false>{h->Rt, h->ldt, 1, 0, nullptr},
                       OutRows{h->St, h->ldt, (long)h->n * h->ldt}, h->specH, h->twm, h->m, h->n, h->l, h->refl,
                       h->r);
    return hipGetLastError();
  });
}

template <class Epi>
hipError_t pass_g2(sfista_fft* h, const Epi& epi) {
  return with_size(h->Nn, [&]<int N>() -> hipError_t {
    hipLaunchKernelGGL((fan_in_kernel<N, true, LinesF32<true>, Epi>), dim3((h->m + 1) / 2), dim3(fft_threads(N)), 0,
                       h->s, LinesF32<true>{h->St, 1, h->ldt, (long)h->n * h->ldt, nullptr}, epi, h->specK, h->twn,
                       h->n, h->m, h->q, h->refl, h->r);
    return hipGetLastError();
  });
}

// A_s^T A_s x (x scaled by 1 / sqrt(*ss) when ss is given) into out;
// A_s x into ax when ax is given.
hipError_t normal_op(sfista_fft* h, const double* x, const double* ss, double* ax, double* out) {
  hipError_t e;
  if ((e = pass_f1(h, x, ss)) != hipSuccess) return e;
  if ((e = pass_f2(h, false, ax, 1, h->n)) != hipSuccess) return e;
  if (!out) return hipSuccess;
  if ((e = pass_g1(h)) != hipSuccess) return e;
  return pass_g2(h, EpiStore64{out, h->n});
}

// F2 and G1 in one pass over the column pairs.
hipError_t pass_columns(sfista_fft* h) {
  return with_size(h->Nm, [&]<int N>() -> hipError_t {
    hipLaunchKernelGGL((column_pass_kernel<N>), dim3((h->n + 1) / 2), dim3(fft_threads(N)), 0, h->s,
                       LinesF32<false>{h->Tt, h->ldt, 1, (long)h->n * h->ldt, nullptr}, h->BobsT, h->ldt,
                       OutRows{h->St, h->ldt, (long)h->n * h->ldt}, h->specH, h->twm, h->m, h->n, h->l, h->refl,
                       h->r);
    return hipGetLastError();
  });
}

hipError_t run_iteration(sfista_fft* h) {
  hipError_t e;
  const long k = h->iter + 1;
  const double tn = (1.0 + sqrt(1.0 + 4.0 * h->tk * h->tk)) / 2.0;   // t_{k+1}
  const double beta = (h->tk - 1.0) / tn;                            // Step 3
  const double den = h->L + h->lam * h->lam;
  if ((e = pass_f1(h, h->Y, nullptr)) != hipSuccess) return e;
  if ((e = pass_columns(h)) != hipSuccess) return e;
  if ((e = pass_g2(h, EpiUpdate{h->X[(k - 1) & 1], h->X[k & 1], h->Y, h->n, h->L / den, 1.0 / den, beta,
                                h->nonneg})) != hipSuccess)
    return e;
  h->tk = tn;
  h->iter = k;
  return hipSuccess;
}

template <class T>
bool take(DeviceArena& ar, T*& p, size_t count, hipStream_t s) {
  p = static_cast<T*>(ar.alloc_zero(count * sizeof(T), s));
  return p != nullptr;
}

// Lanczos estimate of L, the recurrence of the GEMM form's run_lanczos with
// A_s^T A_s applied by the transform passes.
hipError_t run_lanczos(sfista_fft* h, const double* v0, int steps, double* L_out) {
  const long mn = (long)h->m * h->n;
  double* scal = h->red + RED_BLOCKS;
  DeviceArena& ar = h->arena;
  if ((!h->lzq[0] && !take(ar, h->lzq[0], mn, h->s)) || (!h->lzq[1] && !take(ar, h->lzq[1], mn, h->s)) ||
      !take(ar, h->lzcoef, (size_t)steps * 2, h->s))
    return hipErrorOutOfMemory;
  double* coef = h->lzcoef;
  hipError_t e;
  if ((e = sumsq(DoubleSq{v0}, mn, h->red, scal, h->s)) != hipSuccess) return e;
  hipLaunchKernelGGL(lanczos_scale_kernel, dim3(EW_BLOCKS_FFT), dim3(256), 0, h->s, v0, scal, h->lzq[0], mn);
  int cur = 0;
  for (int j = 0; j < steps; ++j) {
    double* q = h->lzq[cur];
    double* qo = h->lzq[cur ^ 1];      // q_{j-1}, then q_{j+1}
    if ((e = normal_op(h, q, nullptr, nullptr, h->aux)) != hipSuccess) return e;
    if ((e = sumf(DoubleDot{q, h->aux}, mn, h->red, coef + 2 * j, h->s)) != hipSuccess) return e;
    hipLaunchKernelGGL(lanczos_orth_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, h->s, h->aux, q, qo, coef, j, mn,
                       h->red);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RED_THREADS), 0, h->s, h->red, RED_BLOCKS,
                       coef + 2 * j + 1);
    if (j + 1 < steps) {
      hipLaunchKernelGGL(lanczos_scale_kernel, dim3(EW_BLOCKS_FFT), dim3(256), 0, h->s, h->aux, coef + 2 * j + 1, qo,
                         mn);
      cur ^= 1;
    }
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<double> hc((size_t)steps * 2);
  if ((e = hipMemcpyAsync(hc.data(), coef, hc.size() * 8, hipMemcpyDeviceToHost, h->s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return e;
  *L_out = lanczos_ritz_max(hc.data(), steps);
  return hipSuccess;
}

hipError_t run_power(sfista_fft* h, const double* v0, int steps, double* L_out) {
  const long mn = (long)h->m * h->n;
  double* scal = h->red + RED_BLOCKS;
  hipError_t e;
  if ((e = sumsq(DoubleSq{v0}, mn, h->red, scal, h->s)) != hipSuccess) return e;
  const double* v = v0;
  for (int it = 0; it < steps; ++it) {
    if ((e = normal_op(h, v, scal, nullptr, h->aux)) != hipSuccess) return e;
    if ((e = sumsq(DoubleSq{h->aux}, mn, h->red, scal, h->s)) != hipSuccess) return e;
    v = h->aux;
  }
  double ss = 0.0;
  if ((e = hipMemcpyAsync(&ss, scal, sizeof(double), hipMemcpyDeviceToHost, h->s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return e;
  *L_out = sqrt(ss);
  return hipSuccess;
}


std::vector<float2> twiddles(int N) {
  std::vector<float2> t(N);
  for (int i = 0; i < N; ++i) {
    const double a = 2.0 * M_PI * (double)i / (double)N;
    t[i] = make_float2((float)cos(a), (float)-sin(a));
  }
  return t;
}

int fft_setup(sfista_fft* h, const double* Bobs, const double* hgen, const double* kgen, const sfista_params* p) {
  const int m = h->m, n = h->n, r = h->r;
  const long mn = (long)m * n;
  hipStream_t s = h->s;
  h->Nm = fft_size(m);
  h->Nn = fft_size(n);
  h->ldt = round_up(m, 64);
  DeviceArena& ar = h->arena;
  const size_t tsz = (size_t)r * n * h->ldt;
  if (!take(ar, h->twm, h->Nm, s) || !take(ar, h->twn, h->Nn, s) || !take(ar, h->specH, (size_t)r * h->Nm, s) ||
      !take(ar, h->specK, (size_t)r * h->Nn, s) || !take(ar, h->Y, mn, s) || !take(ar, h->X[0], mn, s) ||
      !take(ar, h->X[1], mn, s) || !take(ar, h->aux, mn, s) || !take(ar, h->red, RED_BLOCKS + 8, s) ||
      !take(ar, h->Tt, tsz, s) || !take(ar, h->St, tsz, s) || !take(ar, h->Rt, (size_t)n * h->ldt, s) ||
      !take(ar, h->BobsT, (size_t)n * h->ldt, s))
    return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", ar.last_error());
  const std::vector<float2> tm = twiddles(h->Nm), tn = twiddles(h->Nn);
  hipError_t e;
  if ((e = hipMemcpyAsync(h->twm, tm.data(), tm.size() * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(h->twn, tn.data(), tn.size() * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "twiddle upload");
  e = with_size(h->Nm, [&]<int N>() -> hipError_t {
    hipLaunchKernelGGL(spectrum_kernel<N>, dim3(r), dim3(fft_threads(N)), 0, s, hgen, m, h->specH, h->twm);
    return hipGetLastError();
  });
  if (e == hipSuccess)
    e = with_size(h->Nn, [&]<int N>() -> hipError_t {
      hipLaunchKernelGGL(spectrum_kernel<N>, dim3(r), dim3(fft_threads(N)), 0, s, kgen, n, h->specK, h->twn);
      return hipGetLastError();
    });
  if (e != hipSuccess) return hip_fail(e, "generator spectra");
  hipLaunchKernelGGL(transpose_f32_kernel, dim3((n + 31) / 32, (m + 31) / 32), dim3(32, 8), 0, s, Bobs, h->BobsT, m,
                     n, h->ldt);
  double* scal = h->red + RED_BLOCKS;
  if ((e = sumsq(DoubleSq{Bobs}, mn, h->red, scal, s)) != hipSuccess) return hip_fail(e, "norm");
  double ss = 0.0;
  if ((e = hipMemcpyAsync(&ss, scal, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "setup");
  h->bobs_norm = sqrt(ss);
  if (!(h->L > 0.0)) {
    const bool lanczos = p->l_estimate == SFISTA_L_LANCZOS;
    const int steps = p->power_iters > 0 ? p->power_iters : (lanczos ? 12 : 30);
    const double* v0 = p->v0;
    if (!v0) {
      if (!take(ar, h->v0buf, mn, s)) return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
      hipLaunchKernelGGL(hash_fill_kernel, dim3(EW_BLOCKS_FFT), dim3(256), 0, s, h->v0buf, mn, 0x5f15a7ull);
      v0 = h->v0buf;
    }
    double L = 0.0;
    if ((e = lanczos ? run_lanczos(h, v0, steps, &L) : run_power(h, v0, steps, &L)) != hipSuccess)
      return hip_fail(e, lanczos ? "Lanczos estimate of L" : "power iteration");
    if (!isfinite(L) || !(L > 0.0)) return set_error(SFISTA_ERR_NONFINITE, "Lipschitz estimate is %g", L);
    h->L = L;
  }
  hipLaunchKernelGGL(fill_f64_kernel, dim3(EW_BLOCKS_FFT), dim3(256), 0, s, h->X[0], h->X[1], h->Y, p->x0, mn);
  if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "state init");
  return SFISTA_OK;
}

}  // namespace

extern "C" {

int sfista_fft_setup(const double* Bobs, int m, int n, const double* h, const double* k, int r, int l, int q, int bc,
                     const sfista_params* p, hipStream_t stream, sfista_fft_handle* out) {
  clear_error();
  if (!out) return set_error(SFISTA_ERR_ARG, "out handle pointer is NULL");
  *out = nullptr;
  if (!Bobs || !h || !k || !p) return set_error(SFISTA_ERR_ARG, "NULL input pointer");
  if (m < 1 || n < 1) return set_error(SFISTA_ERR_ARG, "image size %d x %d must be positive", m, n);
  if (m > FFT_NMAX / 2 || n > FFT_NMAX / 2)
    return set_error(SFISTA_ERR_UNSUPPORTED, "the FFT form takes images of at most %d x %d", FFT_NMAX / 2,
                     FFT_NMAX / 2);
  if (r < 1 || r > (m < n ? m : n)) return set_error(SFISTA_ERR_ARG, "rank r=%d must lie in [1, min(m,n)]", r);
  if (r > FFT_RMAX) return set_error(SFISTA_ERR_UNSUPPORTED, "rank r=%d exceeds %d", r, FFT_RMAX);
  if (l < 0 || l >= m || q < 0 || q >= n) return set_error(SFISTA_ERR_ARG, "centre (%d, %d) outside the image", l, q);
  if (bc != SFISTA_BC_ZERO && bc != SFISTA_BC_REFLEXIVE) return set_error(SFISTA_ERR_ARG, "unknown boundary %d", bc);
  if (!isfinite(p->lambda) || p->lambda < 0.0) return set_error(SFISTA_ERR_ARG, "lambda must be finite and >= 0");
  if (!isfinite(p->L)) return set_error(SFISTA_ERR_ARG, "L must be finite");
  if (p->power_iters < 0) return set_error(SFISTA_ERR_ARG, "power_iters must be >= 0");
  if (p->l_estimate != SFISTA_L_POWER && p->l_estimate != SFISTA_L_LANCZOS)
    return set_error(SFISTA_ERR_ARG, "unknown l_estimate %d", p->l_estimate);
  sfista_fft* f = new (std::nothrow) sfista_fft();
  if (!f) return set_error(SFISTA_ERR_NOMEM, "host allocation failed");
  f->m = m; f->n = n; f->r = r; f->l = l; f->q = q; f->refl = bc == SFISTA_BC_REFLEXIVE ? 1 : 0;
  f->nonneg = p->nonneg ? 1 : 0; f->lam = p->lambda; f->L = p->L > 0.0 ? p->L : 0.0; f->s = stream;
  const int rc = fft_setup(f, Bobs, h, k, p);
  if (rc != SFISTA_OK) {
    (void)hipStreamSynchronize(stream);
    delete f;
    return rc;
  }
  *out = f;
  return SFISTA_OK;
}

int sfista_fft_step(sfista_fft_handle h, int iters) {
  clear_error();
  if (!h) return set_error(SFISTA_ERR_ARG, "NULL handle");
  if (iters < 0) return set_error(SFISTA_ERR_ARG, "iters must be >= 0");
  for (int i = 0; i < iters; ++i) {
    const hipError_t e = run_iteration(h);
    if (e != hipSuccess) return hip_fail(e, "sfista_fft_step");
  }
  return SFISTA_OK;
}

int sfista_fft_solve(sfista_fft_handle h, int max_iters, double tol, double* X_out, sfista_report* rep) {
  clear_error();
  if (!h) return set_error(SFISTA_ERR_ARG, "NULL handle");
  if (max_iters < 0 || !(tol >= 0.0)) return set_error(SFISTA_ERR_ARG, "max_iters >= 0 and tol >= 0 required");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return hip_fail(e, "event create");
  (void)hipEventRecord(e0, h->s);
  const long mn = (long)h->m * h->n;
  double* scal = h->red + RED_BLOCKS;
  int done = 0;
  e = hipSuccess;
  while (done < max_iters && e == hipSuccess) {
    int chunk = max_iters - done;
    if (tol > 0.0 && chunk > 10) chunk = 10;
    for (int i = 0; i < chunk && e == hipSuccess; ++i) e = run_iteration(h);
    if (e != hipSuccess) break;
    done += chunk;
    if (tol > 0.0 && h->iter >= 1) {
      const double* xa = h->X[h->iter & 1];
      const double* xb = h->X[(h->iter - 1) & 1];
      (void)sumsq(DiffSq64{xa, xb}, mn, h->red, scal + 2, h->s);
      (void)sumsq(DoubleSq{xa}, mn, h->red, scal + 3, h->s);
      double v[2];
      if ((e = hipMemcpyAsync(v, scal + 2, 16, hipMemcpyDeviceToHost, h->s)) != hipSuccess) break;
      if ((e = hipStreamSynchronize(h->s)) != hipSuccess) break;
      if (sqrt(v[0]) <= tol * sqrt(v[1])) break;
    }
  }
  (void)hipEventRecord(e1, h->s);
  const double* xk = h->X[h->iter & 1];
  double v[2] = {0.0, 0.0};
  if (e == hipSuccess) e = pass_f1(h, xk, nullptr);
  if (e == hipSuccess) e = pass_f2(h, true, h->aux, 1, h->n);
  if (e == hipSuccess) e = sumsq(DoubleSq{h->aux}, mn, h->red, scal, h->s);
  if (e == hipSuccess) e = sumsq(DoubleSq{xk}, mn, h->red, scal + 1, h->s);
  if (e == hipSuccess && X_out) e = hipMemcpyAsync(X_out, xk, mn * sizeof(double), hipMemcpyDeviceToDevice, h->s);
  if (e == hipSuccess) e = hipMemcpyAsync(v, scal, 16, hipMemcpyDeviceToHost, h->s);
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  float ms = 0.f;
  if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "sfista_fft_solve");
  int status = SFISTA_OK;
  const double phi = 0.5 * v[0] + 0.5 * h->lam * h->lam * v[1];
  if (!isfinite(phi)) status = set_error(SFISTA_ERR_NONFINITE, "objective is not finite after %ld iterations", h->iter);
  if (rep) {
    rep->iters = (int)h->iter;
    rep->seconds = ms * 1e-3;
    rep->L = h->L;
    rep->phi_s = phi;
    rep->resid_norm = sqrt(v[0]);
    rep->bobs_norm = h->bobs_norm;
    rep->x_norm = sqrt(v[1]);
    rep->resid_rel = h->bobs_norm > 0 ? sqrt(v[0]) / h->bobs_norm : 0.0;
    rep->status = status;
  }
  return status;
}

int sfista_fft_apply(sfista_fft_handle h, const double* X, double* AX, double* AtAX) {
  clear_error();
  if (!h || !X) return set_error(SFISTA_ERR_ARG, "NULL argument");
  hipError_t e = normal_op(h, X, nullptr, AX, AtAX);
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return hip_fail(e, "sfista_fft_apply");
  return SFISTA_OK;
}

int sfista_fft_get_L(sfista_fft_handle h, double* L) {
  clear_error();
  if (!h || !L) return set_error(SFISTA_ERR_ARG, "NULL argument");
  *L = h->L;
  return SFISTA_OK;
}

void sfista_fft_destroy(sfista_fft_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->s);
  delete h;
}

}  // extern "C"
