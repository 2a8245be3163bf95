// Element-wise kernels, GEMM epilogues and deterministic reductions of the
// sFISTA iteration (Algorithm 2).
#pragma once

#include <math.h>

#include <vector>

#include "common.hpp"

namespace sf {

// ------------------------------------------------------------- reductions
// Deterministic sum of squares: a fixed grid of RED_BLOCKS blocks writes one
// partial each (fixed lane/tree order), then one block adds the partials in
// index order.  No atomics, so results are bitwise reproducible.
constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += sh[w];
  }
  __syncthreads();
  return tot;   // valid in thread 0
}

// F(e) returns the value whose square is accumulated, for e in [0, count).
template <class F>
__global__ __launch_bounds__(RED_THREADS) void sumsq_partial_kernel(F f, long count, double* partial) {
  __shared__ double sh[RED_THREADS / 64];
  double acc = 0.0;
  for (long e = blockIdx.x * (long)RED_THREADS + threadIdx.x; e < count; e += (long)RED_BLOCKS * RED_THREADS) {
    const double v = f(e);
    acc += v * v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

static __global__ __launch_bounds__(RED_THREADS) void sum_partials_kernel(const double* partial, int count, double* out) {
  __shared__ double sh[RED_THREADS / 64];
  double acc = 0.0;
  for (int e = threadIdx.x; e < count; e += RED_THREADS) acc += partial[e];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = t;
}

// F(e) returns the value itself (a dot product when F multiplies two arrays).
template <class F>
__global__ __launch_bounds__(RED_THREADS) void sum_partial_kernel(F f, long count, double* partial) {
  __shared__ double sh[RED_THREADS / 64];
  double acc = 0.0;
  for (long e = blockIdx.x * (long)RED_THREADS + threadIdx.x; e < count; e += (long)RED_BLOCKS * RED_THREADS)
    acc += f(e);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <class F>
hipError_t sumf(F f, long count, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_partial_kernel<F>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, f, count, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RED_THREADS), 0, s, partial, RED_BLOCKS, out);
  return hipGetLastError();
}

template <class F>
hipError_t sumsq(F f, long count, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_partial_kernel<F>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, f, count, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RED_THREADS), 0, s, partial, RED_BLOCKS, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- Lanczos
// Symmetric Lanczos on M = A_s^T A_s for the estimate of L (Section 4 takes
// L from a Lanczos estimate of the operator norm).  Step j (0-based) keeps
// its coefficients on the device: coef[2j] = alpha_j = <q_j, M q_j> and
// coef[2j+1] = beta_j^2 = ||w_j||^2 after the three-term orthogonalisation.

// w <- w - alpha_j q_j - beta_{j-1} q_{j-1}, and the block partials of ||w||^2
// (launch with RED_BLOCKS x RED_THREADS, then sum_partials_kernel).
static __global__ __launch_bounds__(RED_THREADS) void lanczos_orth_kernel(double* w, const double* q,
                                                                          const double* qprev, const double* coef,
                                                                          int j, long count, double* partial) {
  __shared__ double sh[RED_THREADS / 64];
  const double a = coef[2 * j];
  const double b = j > 0 ? sqrt(coef[2 * j - 1]) : 0.0;
  double acc = 0.0;
  for (long e = blockIdx.x * (long)RED_THREADS + threadIdx.x; e < count; e += (long)RED_BLOCKS * RED_THREADS) {
    double v = w[e] - a * q[e];
    if (j > 0) v -= b * qprev[e];
    w[e] = v;
    acc += v * v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// q = w / sqrt(*ss); zero when ss is 0 (the Krylov space is invariant and
// the host stops reading coefficients there).
static __global__ void lanczos_scale_kernel(const double* w, const double* ss, double* q, long count) {
  const double s = *ss > 0.0 ? 1.0 / sqrt(*ss) : 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
    q[e] = w[e] * s;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a and off-diagonal b (Sylvester's law of inertia on the LDL^T
// pivots of T - x I).
inline int sturm_count_below(const double* a, const double* b, int k, double x) {
  int count = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    d = (a[i] - x) - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++count;
  }
  return count;
}

// Largest eigenvalue of that tridiagonal matrix by bisection inside its
// Gershgorin interval, to the last bit.  NaN if a coefficient is not finite.
inline double tridiag_max_eig(const double* a, const double* b, int k) {
  if (k < 1) return NAN;
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < k; ++i) {
    const double rad = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
    if (!isfinite(a[i]) || !isfinite(rad)) return NAN;
    lo = fmin(lo, a[i] - rad);
    hi = fmax(hi, a[i] + rad);
  }
  for (int it = 0; it < 4096; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (sturm_count_below(a, b, k, mid) == k) hi = mid;
    else lo = mid;
  }
  return hi;
}

// The estimate from the host copy of coef for `steps` steps: the largest
// Ritz value of the tridiagonal matrix of alpha_0.. and beta_0.., cut at
// the first vanishing beta_j (an invariant Krylov space).
inline double lanczos_ritz_max(const double* coef, int steps) {
  std::vector<double> a, b;
  for (int j = 0; j < steps; ++j) {
    a.push_back(coef[2 * j]);
    const double bb = coef[2 * j + 1];
    if (j + 1 == steps || !(bb > 0.0)) break;
    b.push_back(sqrt(bb));
  }
  return tridiag_max_eig(a.data(), b.data(), (int)a.size());
}

// ------------------------------------------------------------- state views
// Iterate-state storage: FP64 mode keeps doubles; other modes keep either
// float pairs (hi, lo) or plain floats.  Dense m x n, row-major.
enum StateKind : int { ST_F64 = 0, ST_PAIR = 1, ST_F32 = 2 };

__device__ __forceinline__ double state_get(const void* st, int kind, long e) {
  if (kind == ST_F64) return static_cast<const double*>(st)[e];
  if (kind == ST_PAIR) {
    const float2 p = static_cast<const float2*>(st)[e];
    return static_cast<double>(p.x) + static_cast<double>(p.y);
  }
  return static_cast<double>(static_cast<const float*>(st)[e]);
}

__device__ __forceinline__ void state_set(void* st, int kind, long e, double v) {
  if (kind == ST_F64) {
    static_cast<double*>(st)[e] = v;
  } else if (kind == ST_PAIR) {
    const float hi = static_cast<float>(v);
    static_cast<float2*>(st)[e] = make_float2(hi, static_cast<float>(v - static_cast<double>(hi)));
  } else {
    static_cast<float*>(st)[e] = static_cast<float>(v);
  }
}

struct StateSq {          // ||X||^2
  const void* st; int kind;
  __device__ double operator()(long e) const { return state_get(st, kind, e); }
};
struct StateDiffSq {      // ||X_a - X_b||^2
  const void* a; const void* b; int kind;
  __device__ double operator()(long e) const { return state_get(a, kind, e) - state_get(b, kind, e); }
};
struct DoubleSq {
  const double* p;
  __device__ double operator()(long e) const { return p[e]; }
};
struct DoubleDot {        // <a, b>
  const double* a; const double* b;
  __device__ double operator()(long e) const { return a[e] * b[e]; }
};

// ------------------------------------------------------------- element-wise
// X_0 -> both state buffers and the F1 operand planes of Y_1 = X_0.
template <int MODE>
__global__ void init_state_kernel(const double* x0, void* st0, void* st1, int kind,
                                  void* y0, void* y1, long ldy, int m, int n) {
  void* y[2] = {y0, y1};
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const double v = x0 ? x0[e] : 0.0;
    state_set(st0, kind, e, v);
    state_set(st1, kind, e, v);
    const long i = e / n, j = e - i * n;
    store_planes<MODE>(y, op_index<MODE>(i, j, ldy), v);
  }
}

// Dense m x n doubles, optionally scaled by 1/sqrt(*sumsq), -> operand planes.
template <int MODE>
__global__ void to_planes_kernel(const double* x, const double* sumsq, void* p0, void* p1, long ldp,
                                 int m, int n) {
  void* p[2] = {p0, p1};
  const double scale = sumsq ? 1.0 / sqrt(*sumsq) : 1.0;
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n, j = e - i * n;
    store_planes<MODE>(p, op_index<MODE>(i, j, ldp), x[e] * scale);
  }
}

// Iterate state -> operand planes (used to evaluate the residual at X_k).
template <int MODE>
__global__ void state_to_planes_kernel(const void* st, int kind, void* p0, void* p1, long ldp, int m, int n) {
  void* p[2] = {p0, p1};
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n, j = e - i * n;
    if (kind == ST_PAIR) {
      const float2 v = static_cast<const float2*>(st)[e];
      store_planes<MODE>(p, op_index<MODE>(i, j, ldp), static_cast<double>(v.x), v.y);
    } else {
      store_planes<MODE>(p, op_index<MODE>(i, j, ldp), state_get(st, kind, e));
    }
  }
}

static __global__ void state_to_double_kernel(const void* st, int kind, double* out, long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    out[e] = state_get(st, kind, e);
}

// Bobs (m x n, double) -> its transpose (n x m) in the accumulator type.
template <class T>
__global__ void transpose_to_kernel(const double* src, T* dst, int m, int n) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int i = bi + r, j = bj + threadIdx.x;
    if (i < m && j < n) tile[r][threadIdx.x] = src[(long)i * n + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int j = bj + r, i = bi + threadIdx.x;
    if (i < m && j < n) dst[(long)j * m + i] = static_cast<T>(tile[threadIdx.x][r]);
  }
}

// Factor packing into the four operand layouts of the iteration's GEMMs.
// d is the factor size (n for A_k, m for B_k); src holds r factors d x d.
enum PackKind : int {
  PK_STACK = 0,     // rows (k, a) of r*d, cols b:   F_k[a][b]     (F1's W = A stack)
  PK_CAT = 1,       // rows a, cols (k, b):          F_k[a][b]     (F2's [B_1 ... B_r])
  PK_STACK_T = 2,   // rows (k, a), cols b:          F_k[b][a]     (G1's [B_1^T; ...; B_r^T])
  PK_CAT_T = 3      // rows a, cols (k, b):          F_k[b][a]     (G2's [A_1; ...; A_r]^T)
};

template <int MODE>
__global__ void pack_kernel(const double* __restrict__ src, void* o0, void* o1, long ldo, int kind,
                            int d, long rows, long cols) {
  void* o[2] = {o0, o1};
  const long total = rows * cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / cols, col = e - row * cols;
    long s;
    if (kind == PK_STACK) {
      s = row * d + col;
    } else if (kind == PK_CAT) {
      const long k = col / d, b = col - k * d;
      s = (k * d + row) * d + b;
    } else if (kind == PK_STACK_T) {
      const long k = row / d, a = row - k * d;
      s = (k * d + col) * d + a;
    } else {
      const long k = col / d, b = col - k * d;
      s = (k * d + b) * d + row;
    }
    store_planes<MODE>(o, op_index<MODE>(row, col, ldo), src[s]);
  }
}

// ------------------------------------------------------------- epilogues
// F1 / G1: output row p = (k, a) of a term-stacked GEMM goes to row a and
// column block k of the next operand: element (a, k * colblk + col).
template <int MODE>
struct EpiStack {
  void* out[2];
  long ldo;
  int D, colblk;
  // optional copy into a gradient operand of the differentiable form: row
  // k colblk + col, K index koff + a (the same block seen with its two
  // indices exchanged)
  void* g[2] = {nullptr, nullptr};
  long ldg = 0, koff = 0;
  __device__ __forceinline__ void operator()(int row, int col, typename ModeTraits<MODE>::Acc v) const {
    const int k = row / D;
    const int a = row - k * D;
    const long idx = op_index<MODE>(a, (long)k * colblk + col, ldo);
    if constexpr (MODE == M_F64) store_planes<MODE>(out, idx, v);
    else store_planes_f<MODE>(out, idx, v);
    if (g[0]) {
      const long gi = op_index<MODE>((long)k * colblk + col, koff + a, ldg);
      if constexpr (MODE == M_F64) store_planes<MODE>(g, gi, v);
      else store_planes_f<MODE>(g, gi, v);
    }
  }
  // columns col .. col + cnt - 1 of one row (cnt <= 8): one vector store
  // when they fill a chunk-aligned group
  __device__ __forceinline__ void store8(int row, int col, const float (&v)[8], int cnt) const {
    if constexpr (MODE != M_F64) {
      const int k = row / D;
      const int a = row - k * D;
      const long k0 = (long)k * colblk + col;
      if (cnt == 8 && (k0 & 7) == 0 && !g[0]) {
        const float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        store8_planes<MODE>(out, op_index<MODE>(a, k0, ldo), v, z);
        return;
      }
    }
    for (int q = 0; q < cnt; ++q) (*this)(row, col + q, v[q]);
  }
};

// F2: R^T[j][i] = (sum_k B_k T_k)^T[j][i] - Bobs^T[j][i] (Step 1's inner
// residual); `copy` (optional) receives R[i][j] in FP64.
template <int MODE>
struct EpiResid {
  using Acc = typename ModeTraits<MODE>::Acc;
  void* out[2];
  long ldo;
  const Acc* bobs_t;   // n x m, nullable (normal-operator products only)
  int m;
  double* copy;        // m x n, nullable
  int n;
  // optional copy of R into a gradient operand: row i, K index koff + j
  void* g[2] = {nullptr, nullptr};
  long ldg = 0, koff = 0;
  __device__ __forceinline__ void operator()(int j, int i, Acc v) const {
    const Acc r = bobs_t ? v - bobs_t[(long)j * m + i] : v;
    const long idx = op_index<MODE>(j, i, ldo);
    if constexpr (MODE == M_F64) store_planes<MODE>(out, idx, r);
    else store_planes_f<MODE>(out, idx, r);
    if (copy) copy[(long)i * n + j] = static_cast<double>(r);
    if (g[0]) {
      const long gi = op_index<MODE>(i, koff + j, ldg);
      if constexpr (MODE == M_F64) store_planes<MODE>(g, gi, r);
      else store_planes_f<MODE>(g, gi, r);
    }
  }
  __device__ __forceinline__ void store8(int j, int i, const float (&v)[8], int cnt) const {
    if constexpr (MODE != M_F64) {
      if (cnt == 8 && (i & 7) == 0 && !copy && !g[0]) {
        float r[8];
        const float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (bobs_t && (m & 3) == 0) {   // rows start 16-byte aligned: two vector loads
          const float4* b4 = reinterpret_cast<const float4*>(bobs_t + (long)j * m + i);
          const float4 b0 = b4[0], b1 = b4[1];
          const float bb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) r[q] = v[q] - bb[q];
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) r[q] = bobs_t ? v[q] - bobs_t[(long)j * m + i + q] : v[q];
        }
        store8_planes<MODE>(out, op_index<MODE>(j, i, ldo), r, z);
        return;
      }
    }
    for (int q = 0; q < cnt; ++q) (*this)(j, i + q, v[q]);
  }
};

// G2 without update: raw FP64 copy of the normal-operator product.
template <int MODE>
struct EpiStore {
  double* out;
  int n;
  __device__ __forceinline__ void operator()(int i, int j, typename ModeTraits<MODE>::Acc v) const {
    out[(long)i * n + j] = static_cast<double>(v);
  }
};

// Steps 1 and 3 of Algorithm 2 at one pixel, given G = sum_j B_j^T R A_j:
//   Y_k     = X_{k-1} + beta_{k-1} (X_{k-1} - X_{k-2})
//   X_k     = (L Y_k - G) / (L + lambda^2)          [max(0, .) if nonneg]
//   Y_{k+1} = X_k + beta_k (X_k - X_{k-1})
// X_k overwrites X_{k-2} in place (state index s); the planes of Y_{k+1}
// (operand index o) feed the next iteration's F1.
// State update of one element for the float-state kinds (Steps 1 and 3 of
// Algorithm 2 with the Tikhonov scaling and the optional x >= 0 projection):
// reads X_{k-1} (x1) and X_{k-2} (x2), writes X_k over X_{k-2} and returns
// Y_{k+1} as a (hi, lo) float pair (lo = 0 for plain FP32 state).
template <int KIND>
__device__ __forceinline__ void update_state(const void* x1, void* x2, long s, float g, double c1, double c2,
                                             double bp, double bc, int nonneg, float& yh, float& yl) {
  if constexpr (KIND == ST_PAIR) {
    const float2 p1 = static_cast<const float2*>(x1)[s];
    const float2 p2 = static_cast<float2*>(x2)[s];
    const ff a1{p1.x, p1.y}, a2{p2.x, p2.y};
    const ff yk = ff_add(a1, ff_mul(ff_from_double(bp), ff_add(a1, ff_neg(a2))));
    ff xk = ff_add(ff_mul(ff_from_double(c1), yk), ff_neg(ff_mul_f(ff_from_double(c2), g)));
    if (nonneg && (xk.hi < 0.f || (xk.hi == 0.f && xk.lo < 0.f))) xk = ff{0.f, 0.f};
    const ff yn = ff_add(xk, ff_mul(ff_from_double(bc), ff_add(xk, ff_neg(a1))));
    static_cast<float2*>(x2)[s] = make_float2(xk.hi, xk.lo);
    yh = yn.hi;
    yl = yn.lo;
  } else {
    const float a1 = static_cast<const float*>(x1)[s];
    const float a2 = static_cast<float*>(x2)[s];
    const float yk = a1 + static_cast<float>(bp) * (a1 - a2);
    float xk = static_cast<float>(c1) * yk - static_cast<float>(c2) * g;
    if (nonneg) xk = fmaxf(xk, 0.f);
    const float yn = xk + static_cast<float>(bc) * (xk - a1);
    static_cast<float*>(x2)[s] = xk;
    yh = yn;
    yl = 0.f;
  }
}

template <int MODE, int KIND>
__device__ __forceinline__ void update_point(void* const* y, long o, const void* x1, void* x2, long s,
                                             typename ModeTraits<MODE>::Acc g, double c1, double c2, double bp,
                                             double bc, int nonneg) {
  if constexpr (KIND == ST_F64) {
    const double a1 = static_cast<const double*>(x1)[s];
    const double a2 = static_cast<double*>(x2)[s];
    const double yk = a1 + bp * (a1 - a2);
    double xk = c1 * yk - c2 * static_cast<double>(g);
    if (nonneg) xk = fmax(xk, 0.0);
    const double yn = xk + bc * (xk - a1);
    static_cast<double*>(x2)[s] = xk;
    store_planes<MODE>(y, o, yn);
  } else {
    float yh, yl;
    update_state<KIND>(x1, x2, s, static_cast<float>(g), c1, c2, bp, bc, nonneg, yh, yl);
    store_planes_f<MODE>(y, o, yh, yl);
  }
}

// Eight consecutive columns (j chunk-aligned) of the update with one vector
// store of Y_{k+1}; anything else falls back to single elements.
template <int MODE, int KIND, class E>
__device__ __forceinline__ void update_store8(const E& e, int i, int j, const float (&g)[8], int cnt, const void* x1,
                                              void* x2, double bp, double bc) {
  if constexpr (KIND != ST_F64 && MODE != M_F64) {
    if (cnt == 8 && (j & 7) == 0) {
      float yh[8], yl[8];
      const long s0 = (long)i * e.n + j;
#pragma unroll
      for (int q = 0; q < 8; ++q) update_state<KIND>(x1, x2, s0 + q, g[q], e.c1, e.c2, bp, bc, e.nonneg, yh[q], yl[q]);
      store8_planes<MODE>(e.y, op_index<MODE>(i, j, e.ldy), yh, yl);
      return;
    }
  }
  for (int q = 0; q < cnt; ++q)
    update_point<MODE, KIND>(e.y, op_index<MODE>(i, j + q, e.ldy), x1, x2, (long)i * e.n + j + q, g[q], e.c1, e.c2,
                             bp, bc, e.nonneg);
}

// G2 epilogue with the iteration's constants passed by the host.
template <int MODE, int KIND>
struct EpiUpdate {
  using Acc = typename ModeTraits<MODE>::Acc;
  void* y[2];
  long ldy;
  const void* x1;   // X_{k-1}
  void* x2;         // X_{k-2} in, X_k out
  int n;
  double c1, c2;    // L / (L + lambda^2), 1 / (L + lambda^2)
  double bp, bc;    // beta_{k-1}, beta_k
  int nonneg;
  __device__ __forceinline__ void operator()(int i, int j, Acc g) const {
    update_point<MODE, KIND>(y, op_index<MODE>(i, j, ldy), x1, const_cast<void*>(x2), (long)i * n + j, g, c1, c2,
                             bp, bc, nonneg);
  }
  __device__ __forceinline__ void store8(int i, int j, const float (&g)[8], int cnt) const {
    update_store8<MODE, KIND>(*this, i, j, g, cnt, x1, x2, bp, bc);
  }
  static constexpr bool kElementwiseReduce = true;
};

// G2 epilogue that reads the iteration number k = *counter + 1 and the
// momentum weights beta[k - 1], beta[k] from device memory, so that the same
// launch (for instance inside a captured graph) serves every iteration.
template <int MODE, int KIND>
struct EpiUpdateSeq {
  using Acc = typename ModeTraits<MODE>::Acc;
  void* y[2];
  long ldy;
  void* st[2];      // the two state buffers; X_k goes to st[k & 1]
  int n;
  double c1, c2;
  int nonneg;
  const double* beta;
  const int* counter;
  __device__ __forceinline__ void operator()(int i, int j, Acc g) const {
    const int k = *counter + 1;
    void* const x1 = (k & 1) ? st[0] : st[1];   // st[(k - 1) & 1], selected without indexing
    void* const x2 = (k & 1) ? st[1] : st[0];   // st[k & 1]
    update_point<MODE, KIND>(y, op_index<MODE>(i, j, ldy), x1, x2, (long)i * n + j, g, c1, c2,
                             beta[k - 1], beta[k], nonneg);
  }
  __device__ __forceinline__ void store8(int i, int j, const float (&g)[8], int cnt) const {
    const int k = *counter + 1;
    void* const x1 = (k & 1) ? st[0] : st[1];
    void* const x2 = (k & 1) ? st[1] : st[0];
    update_store8<MODE, KIND>(*this, i, j, g, cnt, x1, x2, beta[k - 1], beta[k]);
  }
  static constexpr bool kElementwiseReduce = true;
};

// ------------------------------------------------- differentiable form
// Step 1 and Step 3 of Algorithm 2 with FP64 iterates (G2 epilogue):
// X_k = c1 Y_k - c2 G, Y_{k+1} = X_k + beta (X_k - X_{k-1}), written as FP64
// (ynext may alias yin: each element is read and written by one thread) and
// as the F1 operand planes of Y_{k+1}.
template <int MODE>
struct EpiUpd64 {
  void* y[2];
  long ldy;
  const double* yin;
  const double* xprev;
  double* xout;
  double* ynext;
  int n;
  double c1, c2, beta;
  __device__ __forceinline__ void operator()(int i, int j, typename ModeTraits<MODE>::Acc g) const {
    const long e = (long)i * n + j;
    const double xk = c1 * yin[e] - c2 * static_cast<double>(g);
    const double yn = __builtin_fma(beta, xk - xprev[e], xk);   // same rounding as momentum_start_kernel
    xout[e] = xk;
    ynext[e] = yn;
    store_planes<MODE>(y, op_index<MODE>(i, j, ldy), yn);
  }
};

// Adjoint of Step 1 with respect to Y_k (G2 epilogue): Ybar = c1 Xbar + A_s^T Rbar.
template <int MODE>
struct EpiYbar {
  double* ybar;
  const double* xbar;
  int n;
  double c1;
  __device__ __forceinline__ void operator()(int i, int j, typename ModeTraits<MODE>::Acc v) const {
    const long e = (long)i * n + j;
    ybar[e] = c1 * xbar[e] + static_cast<double>(v);
  }
};

// Accumulation of a factor-gradient product:
// out[row rs + (col / cblk) cbs + col % cblk] += v.
template <int MODE>
struct EpiAcc64 {
  double* out;
  long rs, cbs;
  int cblk;
  __device__ __forceinline__ void operator()(int row, int col, typename ModeTraits<MODE>::Acc v) const {
    const int cb = col / cblk;
    const long o = (long)row * rs + (long)cb * cbs + (col - cb * cblk);
    out[o] += static_cast<double>(v);
  }
};

// Y_{c+1} = X_c + beta (X_c - X_{c-1}) from two stored iterates, as FP64 and
// as the F1 operand planes.
template <int MODE>
__global__ void momentum_start_kernel(const double* xprev, const double* xc, double beta, double* y, void* p0,
                                      void* p1, long ldp, int m, int n) {
  void* p[2] = {p0, p1};
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const double v = __builtin_fma(beta, xc[e] - xprev[e], xc[e]);   // as in EpiUpd64
    y[e] = v;
    const long i = e / n, j = e - i * n;
    store_planes<MODE>(p, op_index<MODE>(i, j, ldp), v);
  }
}

// Adjoint of Step 3 and the start of the adjoint of Step 1 at iteration k:
// Xbar_k = dX + a1 Ybar_{k+1} - a2 Ybar_{k+2} (dX nullable), Gbar = -c2 Xbar_k
// as FP64 (Xbar) and as F1 operand planes, and Gbar^T into the gradient
// operand gt (row j, K index koff + i).
template <int MODE>
__global__ void adjoint_step_kernel(const double* dx, const double* yb1, const double* yb2, double a1, double a2,
                                    double c2, double* xbar, void* p0, void* p1, long ldp, void* g0, void* g1,
                                    long ldg, long koff, int m, int n) {
  void* p[2] = {p0, p1};
  void* g[2] = {g0, g1};
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    double xb = a1 * yb1[e] - a2 * yb2[e];
    if (dx) xb += dx[e];
    xbar[e] = xb;
    const double gb = -c2 * xb;
    const long i = e / n, j = e - i * n;
    store_planes<MODE>(p, op_index<MODE>(i, j, ldp), gb);
    store_planes<MODE>(g, op_index<MODE>(j, koff + i, ldg), gb);
  }
}

// Transposed copy of an m x n FP64 matrix into a gradient operand: element
// (i, j) goes to row j, K index koff + i.
template <int MODE>
__global__ void pack_t_kernel(const double* src, void* g0, void* g1, long ldg, long koff, int m, int n) {
  void* g[2] = {g0, g1};
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n, j = e - i * n;
    store_planes<MODE>(g, op_index<MODE>(j, koff + i, ldg), src[e]);
  }
}

// Zeroes K indices [k0, k1) of rows [0, rows) of an operand.
template <int MODE>
__global__ void zero_k_kernel(void* g0, void* g1, long ldg, long rows, long k0, long k1) {
  void* g[2] = {g0, g1};
  const long w = k1 - k0;
  const long total = rows * w;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long r = e / w, k = k0 + (e - r * w);
    store_planes<MODE>(g, op_index<MODE>(r, k, ldg), 0.0);
  }
}

static __global__ void fill_zero_kernel(double* p, long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) p[e] = 0.0;
}

static __global__ void copy_kernel(const double* src, double* dst, long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) dst[e] = src[e];
}

// One-thread kernel advancing the device iteration counter.
static __global__ void advance_counter_kernel(int* counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) counter[0] = counter[0] + 1;
}

}  // namespace sf
