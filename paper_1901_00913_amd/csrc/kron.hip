// Kronecker approximation of the blur on the GPU, all in FP64 (Section 2,
// Theorem 1).
//
//   1. weighted PSF  P_bar = W_m P W_n  (zero boundary: W = diag(sqrt(d - |i - c|)))
//                    P_bar = S_m P S_n  (reflexive: S = M^{1/2}, the symmetric root
//                    of the Toeplitz matrix M with first row [d, 1, 0, 1, 0, ...]);
//   2. top-r SVD of P_bar by randomized subspace iteration with modified
//      Gram-Schmidt (twice) and a final one-sided Jacobi SVD of the small
//      projected problem;
//   3. signs: largest-magnitude entry of u_k positive (lowest index on ties);
//   4. generators h_k = sqrt(sigma_k) W_m^{-1} u_k, k_k = sqrt(sigma_k) W_n^{-1} v_k;
//   5. dense factors B_k = F(h_k, l), A_k = F(k_k, q), F = toep (+ hank);
//   6. eps_s = ||P_bar - sum_k sigma_k u_k v_k^T||_F (equal to ||A - A_s||_F).
//
// The reflexive root: M = d I + T with T[a][b] = 1 for odd |a - b|, so
// T = e_e e_o^T + e_o e_e^T (indicators of even / odd indices) has rank two.
// With ne = ceil(d/2), no = floor(d/2), c = sqrt(ne no) and
// w± = (e_e / sqrt(ne) ± e_o / sqrt(no)) / sqrt(2), the eigenvalues of M are
// d ± c on w± and d elsewhere, so
//   M^{±1/2} = d^{±1/2} I + ((d+c)^{±1/2} - d^{±1/2}) w+ w+^T + ((d-c)^{±1/2} - d^{±1/2}) w- w-^T.
// Any R with R^T R = M gives the same A_s (the factors only change by the
// orthogonal factor R S^{-1}), so no Cholesky factorisation is needed.
#include <math.h>

#include <algorithm>
#include <vector>

#include "../../include/sfista.h"
#include "kernels.hpp"
#include "util.hpp"

using namespace sf;

namespace {

constexpr int PMAX = 32;          // subspace width limit (rank + oversampling)
constexpr int OVERSAMPLE = 10;
constexpr int SUBSPACE_ITERS = 12;
constexpr int JACOBI_SWEEPS = 40;
constexpr int KT = 256;           // threads of the row kernels
constexpr int ST = 1024;          // threads of the single-block kernels
// internal streams of kron_approx_batch: more than the process's hardware
// queues still pays (on 64 images, 2 and 4 streams tie, 8 and 16 cut the
// setup by 40 and 56 ms, 32 by no more)
constexpr int KRON_STREAMS = 16;

struct Reflex {                   // closed-form M^{1/2} pieces for one side
  double sq_d, a_plus, a_minus;   // M^{1/2}:  sqrt(d), coefficients of w+ w+^T, w- w-^T
  double isq_d, g_plus, g_minus;  // M^{-1/2}
  double wpe, wpo, wme, wmo;      // entries of w+ / w- on even / odd indices
  int has_rank2;
};

Reflex make_reflex(int d) {
  Reflex r{};
  const double ne = (d + 1) / 2, no = d / 2;
  r.sq_d = sqrt((double)d);
  r.isq_d = 1.0 / r.sq_d;
  r.has_rank2 = no > 0;
  if (r.has_rank2) {
    const double c = sqrt(ne * no);
    r.a_plus = sqrt(d + c) - r.sq_d;
    r.a_minus = sqrt(d - c) - r.sq_d;
    r.g_plus = 1.0 / sqrt(d + c) - r.isq_d;
    r.g_minus = 1.0 / sqrt(d - c) - r.isq_d;
    r.wpe = 1.0 / sqrt(2.0 * ne);
    r.wpo = 1.0 / sqrt(2.0 * no);
    r.wme = r.wpe;
    r.wmo = -r.wpo;
  }
  return r;
}

__device__ __forceinline__ double wplus(const Reflex& r, long i) { return (i & 1) ? r.wpo : r.wpe; }
__device__ __forceinline__ double wminus(const Reflex& r, long i) { return (i & 1) ? r.wmo : r.wme; }

// sum over a wave then over the block; the result is broadcast to all threads
template <int NV>
__device__ void block_allreduce(double (&v)[NV], double* sh /* NV * 32 */) {
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q * 32 + wave] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += sh[q * 32 + w];
    v[q] = t;
  }
}

// ---------------------------------------------------------------- weighting
__global__ void weight_zero_kernel(const double* P, double* Pb, int m, int n, int l, int q) {
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long a = e / n, b = e - a * n;
    const double wa = sqrt((double)(m - labs(a - l)));
    const double wb = sqrt((double)(n - labs(b - q)));
    Pb[e] = wa * P[e] * wb;
  }
}

// Column sums of X (m x n) over even rows and odd rows, in two steps with a
// fixed order (deterministic): block (bx, by) sums rows [by RW, (by + 1) RW)
// of 64 columns, 4 row phases per column, into part[by][b][parity]; then
// colsum_finish_kernel adds the CS_RB chunks of each column in order.
constexpr int CS_RB = 16;

__global__ __launch_bounds__(256) void colsum_partial_kernel(const double* X, int m, int n, double* part) {
  __shared__ double sh[4][64][2];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  const int rw = (m + CS_RB - 1) / CS_RB;
  const int a0 = blockIdx.y * rw, a1 = min(m, a0 + rw);
  double v[2] = {0.0, 0.0};
  if (col < n)
    for (int a = a0 + g; a < a1; a += 4) v[a & 1] += X[(long)a * n + col];
  sh[g][threadIdx.x & 63][0] = v[0];
  sh[g][threadIdx.x & 63][1] = v[1];
  __syncthreads();
  if (g == 0 && col < n) {
    const int c = threadIdx.x;
    part[((long)blockIdx.y * n + col) * 2 + 0] = ((sh[0][c][0] + sh[1][c][0]) + sh[2][c][0]) + sh[3][c][0];
    part[((long)blockIdx.y * n + col) * 2 + 1] = ((sh[0][c][1] + sh[1][c][1]) + sh[2][c][1]) + sh[3][c][1];
  }
}

__global__ void colsum_finish_kernel(const double* part, int n, double* ev, double* od) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double se = 0.0, so = 0.0;
  for (int q = 0; q < CS_RB; ++q) {
    se += part[((long)q * n + b) * 2 + 0];
    so += part[((long)q * n + b) * 2 + 1];
  }
  ev[b] = se;
  od[b] = so;
}

// row sums of X over even and odd columns: ev[a], od[a]   (one block per row)
__global__ void rowsum_parity_kernel(const double* X, int m, int n, double* ev, double* od) {
  __shared__ double sh[2 * 32];
  const int a = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += blockDim.x) v[b & 1] += X[(long)a * n + b];
  block_allreduce<2>(v, sh);
  if (threadIdx.x == 0) { ev[a] = v[0]; od[a] = v[1]; }
}

// Q = S_m X :  Q[a][b] = sqrt(m) X[a][b] + a+ w+[a] (w+^T X)[b] + a- w-[a] (w-^T X)[b]
__global__ void left_root_kernel(const double* X, double* Q, int m, int n, Reflex rm, const double* ev,
                                 const double* od) {
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long a = e / n, b = e - a * n;
    double v = rm.sq_d * X[e];
    if (rm.has_rank2) {
      const double cp = rm.wpe * ev[b] + rm.wpo * od[b];
      const double cm = rm.wme * ev[b] + rm.wmo * od[b];
      v += rm.a_plus * wplus(rm, a) * cp + rm.a_minus * wminus(rm, a) * cm;
    }
    Q[e] = v;
  }
}

// Y = X S_n :  Y[a][b] = sqrt(n) X[a][b] + a+ (X w+)[a] w+[b] + a- (X w-)[a] w-[b]
__global__ void right_root_kernel(const double* X, double* Y, int m, int n, Reflex rn, const double* ev,
                                  const double* od) {
  const long total = (long)m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long a = e / n, b = e - a * n;
    double v = rn.sq_d * X[e];
    if (rn.has_rank2) {
      const double dp = rn.wpe * ev[a] + rn.wpo * od[a];
      const double dm = rn.wme * ev[a] + rn.wmo * od[a];
      v += rn.a_plus * dp * wplus(rn, b) + rn.a_minus * dm * wminus(rn, b);
    }
    Y[e] = v;
  }
}

__global__ void transpose_kernel(const double* src, double* dst, int m, int n) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int i = bi + r, j = bj + threadIdx.x;
    if (i < m && j < n) tile[r][threadIdx.x] = src[(long)i * n + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int j = bj + r, i = bi + threadIdx.x;
    if (i < m && j < n) dst[(long)j * m + i] = tile[threadIdx.x][r];
  }
}

// ---------------------------------------------------------------- subspace SVD
// out (p x rows, column-major) = X (rows x cols) * V (p x cols, column-major)^T
__global__ __launch_bounds__(KT) void mat_cols_kernel(const double* X, int rows, int cols, const double* V,
                                                      int p, double* out) {
  __shared__ double sh[PMAX * 4];
  const int a = blockIdx.x;
  double acc[PMAX];
#pragma unroll
  for (int c = 0; c < PMAX; ++c) acc[c] = 0.0;
  for (int b = threadIdx.x; b < cols; b += KT) {
    const double x = X[(long)a * cols + b];
#pragma unroll
    for (int c = 0; c < PMAX; ++c)
      if (c < p) acc[c] += x * V[(long)c * cols + b];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < PMAX; ++c) {
    if (c < p) {
      double v = acc[c];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if (lane == 0) sh[c * 4 + wave] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < p) {
    const int c = threadIdx.x;
    out[(long)c * rows + a] = ((sh[c * 4 + 0] + sh[c * 4 + 1]) + sh[c * 4 + 2]) + sh[c * 4 + 3];
  }
}

// The same product for p <= PC, RB rows per block: each V element loaded
// serves RB rows (the one-row kernel re-reads all of V from L2 per row).
// Every output keeps the one-row kernel's order of summation.
template <int PC, int RB>
__global__ __launch_bounds__(KT) void mat_cols_rows_kernel(const double* X, int rows, int cols, const double* V,
                                                           int p, double* out) {
  __shared__ double sh[RB * PC * 4];
  const int a0 = blockIdx.x * RB;
  double acc[RB][PC];
#pragma unroll
  for (int t = 0; t < RB; ++t)
#pragma unroll
    for (int c = 0; c < PC; ++c) acc[t][c] = 0.0;
  for (int b = threadIdx.x; b < cols; b += KT) {
    double v[PC];
#pragma unroll
    for (int c = 0; c < PC; ++c) v[c] = c < p ? V[(long)c * cols + b] : 0.0;
#pragma unroll
    for (int t = 0; t < RB; ++t) {
      if (a0 + t < rows) {
        const double x = X[(long)(a0 + t) * cols + b];
#pragma unroll
        for (int c = 0; c < PC; ++c) acc[t][c] += x * v[c];
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < RB; ++t)
#pragma unroll
    for (int c = 0; c < PC; ++c) {
      double w = acc[t][c];
      for (int o = 32; o > 0; o >>= 1) w += __shfl_down(w, o, 64);
      if (lane == 0) sh[(t * PC + c) * 4 + wave] = w;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < RB * p; i += KT) {
    const int t = i / p, c = i - t * p;
    if (a0 + t < rows) {
      const double* q = sh + (t * PC + c) * 4;
      out[(long)c * rows + a0 + t] = ((q[0] + q[1]) + q[2]) + q[3];
    }
  }
}

// out = X V^T through the multi-row kernel when p allows it.
void mat_cols(const double* X, int rows, int cols, const double* V, int p, double* out, hipStream_t s) {
  if (p <= 16) {
    constexpr int RB = 4;
    hipLaunchKernelGGL((mat_cols_rows_kernel<16, RB>), dim3((rows + RB - 1) / RB), dim3(KT), 0, s, X, rows, cols, V,
                       p, out);
  } else {
    hipLaunchKernelGGL(mat_cols_kernel, dim3(rows), dim3(KT), 0, s, X, rows, cols, V, p, out);
  }
}

// Modified Gram-Schmidt, applied twice, on p columns of length d (single
// block).  A column whose residual after projection falls below 1e-10 of its
// norm before projection is numerically dependent on the previous ones (the
// weighted PSF can have rank below p); it is set to zero instead of
// normalising rounding noise, which would not be orthogonal to the span.
__global__ __launch_bounds__(ST) void mgs2_kernel(double* Y, int p, int d) {
  __shared__ double sh[2 * 32];
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = 0; c < p; ++c) {
      double* yc = Y + (long)c * d;
      double v0[1] = {0.0};
      for (int t = threadIdx.x; t < d; t += ST) v0[0] += yc[t] * yc[t];
      block_allreduce<1>(v0, sh);
      for (int c2 = 0; c2 < c; ++c2) {
        const double* y2 = Y + (long)c2 * d;
        double v[1] = {0.0};
        for (int t = threadIdx.x; t < d; t += ST) v[0] += yc[t] * y2[t];
        block_allreduce<1>(v, sh);
        for (int t = threadIdx.x; t < d; t += ST) yc[t] -= v[0] * y2[t];
        __syncthreads();
      }
      double v[1] = {0.0};
      for (int t = threadIdx.x; t < d; t += ST) v[0] += yc[t] * yc[t];
      block_allreduce<1>(v, sh);
      const double inv = (v[0] > 1e-20 * v0[0] && v[0] > 0.0) ? 1.0 / sqrt(v[0]) : 0.0;
      for (int t = threadIdx.x; t < d; t += ST) yc[t] *= inv;
      __syncthreads();
    }
  }
}

// The same orthonormalisation for up to PC columns of length up to
// EPT * CT (CT = 512 threads), held in registers: classical Gram-Schmidt applied twice, so the
// projections of a column on all previous ones are one batched block
// reduction and its norm another (4p reductions, against about p^2 in the
// modified form, and no memory traffic between them).  Two passes give
// orthogonality at rounding level; dependent columns are zeroed by the same
// rule as mgs2_kernel.
// Column C of one pass (a compile-time recursion over the columns, so every
// register index is a constant).
template <int C, int PC, int EPT>
__device__ __forceinline__ void cgs2_column(double (&y)[PC][EPT], int p, double* sh) {
  if constexpr (C < PC) {
    if (C >= p) return;
    double dots[C + 1];   // dots[j], j < C: <y_C, y_j>; dots[C]: ||y_C||^2 before projection
#pragma unroll
    for (int j = 0; j <= C; ++j) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < EPT; ++q) a += y[C][q] * y[j][q];
      dots[j] = a;
    }
    block_allreduce<C + 1>(dots, sh);
    const double v0 = dots[C];
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int q = 0; q < EPT; ++q) y[C][q] -= dots[j] * y[j][q];
    double nv[1] = {0.0};
#pragma unroll
    for (int q = 0; q < EPT; ++q) nv[0] += y[C][q] * y[C][q];
    block_allreduce<1>(nv, sh);
    const double inv = (nv[0] > 1e-20 * v0 && nv[0] > 0.0) ? 1.0 / sqrt(nv[0]) : 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) y[C][q] *= inv;
    cgs2_column<C + 1, PC, EPT>(y, p, sh);
  }
}

constexpr int CT = 512;   // threads of the register Gram-Schmidt kernel

template <int PC, int EPT>
__global__ __launch_bounds__(CT) void cgs2_kernel(double* Y, int p, int d) {
  __shared__ double sh[(PC + 1) * 32];
  double y[PC][EPT];
#pragma unroll
  for (int c = 0; c < PC; ++c)
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int t = (int)threadIdx.x + q * CT;
      y[c][q] = (c < p && t < d) ? Y[(long)c * d + t] : 0.0;
    }
  cgs2_column<0, PC, EPT>(y, p, sh);
  cgs2_column<0, PC, EPT>(y, p, sh);
#pragma unroll
  for (int c = 0; c < PC; ++c)
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int t = (int)threadIdx.x + q * CT;
      if (c < p && t < d) Y[(long)c * d + t] = y[c][q];
    }
}

// Orthonormalises the p columns (length d) of Y in place.
void orthonormalise(double* Y, int p, int d, hipStream_t s) {
  if (p <= 16 && d <= CT)
    hipLaunchKernelGGL((cgs2_kernel<16, 1>), dim3(1), dim3(CT), 0, s, Y, p, d);
  else if (p <= 16 && d <= 2 * CT)
    hipLaunchKernelGGL((cgs2_kernel<16, 2>), dim3(1), dim3(CT), 0, s, Y, p, d);
  else if (p <= 16 && d <= 4 * CT)
    hipLaunchKernelGGL((cgs2_kernel<16, 4>), dim3(1), dim3(CT), 0, s, Y, p, d);
  else if (p <= 24 && d <= CT)
    hipLaunchKernelGGL((cgs2_kernel<24, 1>), dim3(1), dim3(CT), 0, s, Y, p, d);
  else if (p <= 24 && d <= 2 * CT)
    hipLaunchKernelGGL((cgs2_kernel<24, 2>), dim3(1), dim3(CT), 0, s, Y, p, d);
  else
    hipLaunchKernelGGL(mgs2_kernel, dim3(1), dim3(ST), 0, s, Y, p, d);
}

// One-sided (Hestenes) Jacobi on the p columns of Z (length d): rotates
// column pairs until all are orthogonal, accumulating the rotations in
// Wm (p x p, column-major).  Then writes the column norms (singular values)
// and the descending order.
__global__ __launch_bounds__(ST) void jacobi_kernel(double* Z, int p, int d, double* Wm, double* sig, int* order) {
  __shared__ double sh[3 * 32];
  __shared__ double w[PMAX * PMAX];
  __shared__ int rotated;
  for (int t = threadIdx.x; t < p * p; t += ST) w[t] = (t % (p + 1) == 0) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < JACOBI_SWEEPS; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int i = 0; i < p - 1; ++i) {
      for (int j = i + 1; j < p; ++j) {
        double* zi = Z + (long)i * d;
        double* zj = Z + (long)j * d;
        double v[3] = {0.0, 0.0, 0.0};
        for (int t = threadIdx.x; t < d; t += ST) {
          const double x = zi[t], y = zj[t];
          v[0] += x * x;
          v[1] += y * y;
          v[2] += x * y;
        }
        block_allreduce<3>(v, sh);
        const double alpha = v[0], beta = v[1], gam = v[2];
        if (alpha == 0.0 || beta == 0.0 || fabs(gam) <= 1e-15 * sqrt(alpha * beta)) {
          __syncthreads();
          continue;
        }
        const double zeta = (beta - alpha) / (2.0 * gam);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt);
        const double sn = cs * tt;
        for (int t = threadIdx.x; t < d; t += ST) {
          const double x = zi[t], y = zj[t];
          zi[t] = cs * x - sn * y;
          zj[t] = sn * x + cs * y;
        }
        if (threadIdx.x < p) {
          const double x = w[i * p + threadIdx.x], y = w[j * p + threadIdx.x];
          w[i * p + threadIdx.x] = cs * x - sn * y;
          w[j * p + threadIdx.x] = sn * x + cs * y;
        }
        if (threadIdx.x == 0) rotated = 1;
        __syncthreads();
      }
    }
    __syncthreads();
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  // column norms
  for (int c = 0; c < p; ++c) {
    double v[1] = {0.0};
    const double* zc = Z + (long)c * d;
    for (int t = threadIdx.x; t < d; t += ST) v[0] += zc[t] * zc[t];
    block_allreduce<1>(v, sh);
    if (threadIdx.x == 0) sig[c] = sqrt(v[0]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < p * p; t += ST) Wm[t] = w[t];
  if (threadIdx.x == 0) {
    for (int c = 0; c < p; ++c) order[c] = c;
    for (int a = 1; a < p; ++a) {           // insertion sort, descending, stable
      const int key = order[a];
      int b = a - 1;
      while (b >= 0 && sig[order[b]] < sig[key]) { order[b + 1] = order[b]; --b; }
      order[b + 1] = key;
    }
  }
}

// U[k] = Y * Wm[:, order[k]]  (length m),  V[k] = Z[order[k]] / sigma  (length n)
__global__ void finish_vectors_kernel(const double* Y, const double* Z, const double* Wm, const double* sig,
                                      const int* order, int p, int r, int m, int n, double* U, double* V,
                                      double* sig_out) {
  const int k = blockIdx.y;
  const int col = order[k];
  const double s = sig[col];
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < (m > n ? m : n); a += gridDim.x * blockDim.x) {
    if (a < m) {
      double u = 0.0;
      for (int c = 0; c < p; ++c) u += Y[(long)c * m + a] * Wm[col * p + c];
      U[(long)k * m + a] = u;
    }
    if (a < n) V[(long)k * n + a] = s > 0.0 ? Z[(long)col * n + a] / s : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sig_out[k] = s;
}

// Sign convention + generators, one block per term k.
__global__ __launch_bounds__(ST) void generators_kernel(double* U, double* V, const double* sig, int m, int n,
                                                        int l, int q, int bc, Reflex rm, Reflex rn, double* gh,
                                                        double* gk) {
  __shared__ double sh[4 * 32];
  __shared__ double bestv[ST / 64];
  __shared__ int besti[ST / 64];
  const int k = blockIdx.x;
  double* u = U + (long)k * m;
  double* v = V + (long)k * n;
  // argmax |u| with the lowest index on ties
  double bv = -1.0;
  int bi = 0x7fffffff;
  for (int a = threadIdx.x; a < m; a += ST) {
    const double x = fabs(u[a]);
    if (x > bv) { bv = x; bi = a; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_down(bv, o, 64);
    const int oi = __shfl_down(bi, o, 64);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { bestv[wave] = bv; besti[wave] = bi; }
  __syncthreads();
  __shared__ double flip;
  if (threadIdx.x == 0) {
    double v0 = bestv[0];
    int i0 = besti[0];
    for (int w2 = 1; w2 < (int)(blockDim.x >> 6); ++w2)
      if (bestv[w2] > v0 || (bestv[w2] == v0 && besti[w2] < i0)) { v0 = bestv[w2]; i0 = besti[w2]; }
    flip = (i0 < m && u[i0] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double f = flip;
  const double rs = sqrt(sig[k]);
  if (bc == SFISTA_BC_ZERO) {
    for (int a = threadIdx.x; a < m; a += ST) gh[(long)k * m + a] = f * rs * u[a] / sqrt((double)(m - abs(a - l)));
    for (int b = threadIdx.x; b < n; b += ST) gk[(long)k * n + b] = f * rs * v[b] / sqrt((double)(n - abs(b - q)));
    return;
  }
  // reflexive: M^{-1/2} x = x / sqrt(d) + g+ w+ (w+^T x) + g- w- (w-^T x)
  double s4[4] = {0.0, 0.0, 0.0, 0.0};   // even/odd sums of u and v
  for (int a = threadIdx.x; a < m; a += ST) s4[a & 1] += u[a];
  for (int b = threadIdx.x; b < n; b += ST) s4[2 + (b & 1)] += v[b];
  block_allreduce<4>(s4, sh);
  const double up = rm.wpe * s4[0] + rm.wpo * s4[1], um = rm.wme * s4[0] + rm.wmo * s4[1];
  const double vp = rn.wpe * s4[2] + rn.wpo * s4[3], vm = rn.wme * s4[2] + rn.wmo * s4[3];
  for (int a = threadIdx.x; a < m; a += ST) {
    double x = rm.isq_d * u[a];
    if (rm.has_rank2) x += rm.g_plus * wplus(rm, a) * up + rm.g_minus * wminus(rm, a) * um;
    gh[(long)k * m + a] = f * rs * x;
  }
  for (int b = threadIdx.x; b < n; b += ST) {
    double x = rn.isq_d * v[b];
    if (rn.has_rank2) x += rn.g_plus * wplus(rn, b) * vp + rn.g_minus * wminus(rn, b) * vm;
    gk[(long)k * n + b] = f * rs * x;
  }
  // keep the sign-fixed singular vectors for the eps_s evaluation
  __syncthreads();
  for (int a = threadIdx.x; a < m; a += ST) u[a] *= f;
  for (int b = threadIdx.x; b < n; b += ST) v[b] *= f;
}

// Dense factors: F[k][i][i'] = g[c + i - i'] (+ g[c + i + i' + 1] + g[c + i + i' + 1 - 2d]).
__global__ void expand_kernel(const double* g, int r, int d, int center, int bc, double* F) {
  const long total = (long)r * d * d;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long k = e / ((long)d * d);
    const long rem = e - k * d * d;
    const long i = rem / d, ip = rem - i * d;
    const double* gk = g + k * d;
    double v = 0.0;
    const long t = center + i - ip;
    if (t >= 0 && t < d) v += gk[t];
    if (bc == SFISTA_BC_REFLEXIVE) {
      const long h = center + i + ip + 1;
      if (h < d) v += gk[h];
      if (h - 2 * d >= 0) v += gk[h - 2 * d];
    }
    F[e] = v;
  }
}

struct TailSq {        // P_bar[a][b] - sum_k sigma_k u_k[a] v_k[b]
  const double* Pb; const double* U; const double* V; const double* sig; int r, m, n;
  __device__ double operator()(long e) const {
    const long a = e / n, b = e - a * n;
    double v = Pb[e];
    for (int k = 0; k < r; ++k) v -= sig[k] * U[(long)k * m + a] * V[(long)k * n + b];
    return v;
  }
};

// Argument checks shared by every entry point of the approximation.
int kron_check(int m, int n, int l, int q, int bc, int r) {
  if (m < 1 || n < 1) return set_error(SFISTA_ERR_ARG, "PSF size %d x %d must be positive", m, n);
  if (l < 0 || l >= m || q < 0 || q >= n) return set_error(SFISTA_ERR_ARG, "centre (%d, %d) outside the PSF", l, q);
  if (bc != SFISTA_BC_ZERO && bc != SFISTA_BC_REFLEXIVE) return set_error(SFISTA_ERR_ARG, "unknown boundary %d", bc);
  const int mn_min = m < n ? m : n;
  if (r < 1 || r > mn_min) return set_error(SFISTA_ERR_ARG, "rank r=%d must lie in [1, min(m,n)]", r);
  if (r > PMAX - OVERSAMPLE) return set_error(SFISTA_ERR_UNSUPPORTED, "rank r=%d exceeds %d", r, PMAX - OVERSAMPLE);
  if ((long)m * n > (1L << 31)) return set_error(SFISTA_ERR_UNSUPPORTED, "PSF too large");
  return SFISTA_OK;
}

// Queues the whole approximation of one (checked) PSF on s without waiting:
// dense factors (A, B) and generators (h, k) are each optional; res (device,
// 1 + r doubles) receives ||P_bar - sum_k sigma_k u_k v_k^T||_F^2 and then the
// r singular values.  The work buffers are freed in stream order.
int kron_enqueue(const double* P, int m, int n, int l, int q, int bc, int r, double* A, double* B, double* h_out,
                 double* k_out, double* res, hipStream_t s) {
  const int mn_min = m < n ? m : n;
  const int p = std::min(r + OVERSAMPLE, mn_min);
  const long mn = (long)m * n;

  DeviceArena ar;
  double* Pb = (double*)ar.alloc_zero(mn * 8, s);
  double* Pt = (double*)ar.alloc_zero(mn * 8, s);
  double* tmp = (double*)ar.alloc_zero(mn * 8, s);
  double* colpart = (double*)ar.alloc_zero((size_t)CS_RB * n * 2 * 8, s);
  double* vecs = (double*)ar.alloc_zero((size_t)4 * (m + n) * 8, s);
  double* Yc = (double*)ar.alloc_zero((size_t)PMAX * m * 8, s);
  double* Zc = (double*)ar.alloc_zero((size_t)PMAX * n * 8, s);
  double* Wm = (double*)ar.alloc_zero(PMAX * PMAX * 8, s);
  double* sig = (double*)ar.alloc_zero(PMAX * 8 * 2, s);
  int* order = (int*)ar.alloc_zero(PMAX * 4, s);
  double* U = (double*)ar.alloc_zero((size_t)r * m * 8, s);
  double* V = (double*)ar.alloc_zero((size_t)r * n * 8, s);
  double* gh = (double*)ar.alloc_zero((size_t)r * m * 8, s);
  double* gk = (double*)ar.alloc_zero((size_t)r * n * 8, s);
  double* red = (double*)ar.alloc_zero((RED_BLOCKS + 8) * 8, s);
  if (!(Pb && Pt && tmp && colpart && vecs && Yc && Zc && Wm && sig && order && U && V && gh && gk && red))
    return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", ar.last_error());
  double* sig_out = sig + PMAX;

  const dim3 ew(2048), et(256);
  const Reflex rm = make_reflex(m), rn = make_reflex(n);
  if (bc == SFISTA_BC_ZERO) {
    hipLaunchKernelGGL(weight_zero_kernel, ew, et, 0, s, P, Pb, m, n, l, q);
  } else {
    double *ev = vecs, *od = vecs + (m + n);
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((n + 63) / 64, CS_RB), dim3(256), 0, s, P, m, n, colpart);
    hipLaunchKernelGGL(colsum_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, s, colpart, n, ev, od);
    hipLaunchKernelGGL(left_root_kernel, ew, et, 0, s, P, tmp, m, n, rm, ev, od);
    hipLaunchKernelGGL(rowsum_parity_kernel, dim3(m), dim3(256), 0, s, tmp, m, n, ev, od);
    hipLaunchKernelGGL(right_root_kernel, ew, et, 0, s, tmp, Pb, m, n, rn, ev, od);
  }
  hipLaunchKernelGGL(transpose_kernel, dim3((n + 31) / 32, (m + 31) / 32), dim3(32, 8), 0, s, Pb, Pt, m, n);

  // randomized subspace iteration: Z <- orth(P_bar^T orth(P_bar Z))
  hipLaunchKernelGGL(hash_fill_kernel, ew, et, 0, s, Zc, (long)p * n, 0x51f15eedull);
  for (int it = 0; it < SUBSPACE_ITERS; ++it) {
    mat_cols(Pb, m, n, Zc, p, Yc, s);
    orthonormalise(Yc, p, m, s);
    mat_cols(Pt, n, m, Yc, p, Zc, s);
    if (it + 1 < SUBSPACE_ITERS) orthonormalise(Zc, p, n, s);
  }
  // Z = P_bar^T Y with Y orthonormal: P_bar ~ Y Z^T; SVD of Z by one-sided Jacobi
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(ST), 0, s, Zc, p, n, Wm, sig, order);
  hipLaunchKernelGGL(finish_vectors_kernel, dim3(16, r), dim3(256), 0, s, Yc, Zc, Wm, sig, order, p, r, m, n, U, V,
                     sig_out);
  hipLaunchKernelGGL(generators_kernel, dim3(r), dim3(ST), 0, s, U, V, sig_out, m, n, l, q, bc, rm, rn, gh, gk);
  if (B) hipLaunchKernelGGL(expand_kernel, ew, et, 0, s, gh, r, m, l, bc, B);
  if (A) hipLaunchKernelGGL(expand_kernel, ew, et, 0, s, gk, r, n, q, bc, A);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && h_out) e = hipMemcpyAsync(h_out, gh, (size_t)r * m * 8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && k_out) e = hipMemcpyAsync(k_out, gk, (size_t)r * n * 8, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "kron_approx launch");
  if ((e = sumsq(TailSq{Pb, U, V, sig_out, r, m, n}, mn, red, res, s)) != hipSuccess)
    return hip_fail(e, "kron_approx tail norm");
  if ((e = hipMemcpyAsync(res + 1, sig_out, (size_t)r * 8, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "kron_approx results");
  return SFISTA_OK;
}

// Host side of one result: sigma (r values) and eps_s from res (host copy).
int kron_results(const double* res, int r, double* sigma, double* eps_s) {
  if (sigma) for (int k = 0; k < r; ++k) sigma[k] = res[1 + k];
  if (eps_s) *eps_s = sqrt(res[0]);
  if (!isfinite(res[0])) return set_error(SFISTA_ERR_NONFINITE, "non-finite approximation error");
  return SFISTA_OK;
}

// The common body of kron_approx and kron_generators.
int kron_impl(const double* P, int m, int n, int l, int q, int bc, int r, double* A, double* B, double* h_out,
              double* k_out, double* sigma, double* eps_s, hipStream_t s) {
  int rc = kron_check(m, n, l, q, bc, r);
  if (rc != SFISTA_OK) return rc;
  DeviceArena rar;
  double* res = static_cast<double*>(rar.alloc_zero((size_t)(1 + r) * 8, s));
  if (!res) return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", rar.last_error());
  if ((rc = kron_enqueue(P, m, n, l, q, bc, r, A, B, h_out, k_out, res, s)) != SFISTA_OK) return rc;
  std::vector<double> hres((size_t)1 + r);
  hipError_t e;
  if ((e = hipMemcpyAsync(hres.data(), res, hres.size() * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "kron_approx");
  return kron_results(hres.data(), r, sigma, eps_s);
}

}  // namespace

extern "C" int kron_approx(const double* P, int m, int n, int l, int q, int bc, int r, double* A, double* B,
                           double* sigma, double* eps_s, hipStream_t s) {
  clear_error();
  if (!P || !A || !B) return set_error(SFISTA_ERR_ARG, "NULL device pointer");
  return kron_impl(P, m, n, l, q, bc, r, A, B, nullptr, nullptr, sigma, eps_s, s);
}

// Several PSFs at once: each image's sequence of kernels goes to one of a
// few internal streams (round robin), so that the latency-bound launches of
// different images overlap; results as kron_approx's, bit for bit.
extern "C" int kron_approx_batch(int count, const double* const* P, const int* m, const int* n, const int* l,
                                 const int* q, const int* bc, const int* r, double* const* A, double* const* B,
                                 double* sigma, double* eps_s, hipStream_t stream) {
  clear_error();
  if (count < 1) return set_error(SFISTA_ERR_ARG, "count must be >= 1");
  if (!P || !m || !n || !l || !q || !bc || !r || !A || !B) return set_error(SFISTA_ERR_ARG, "NULL argument array");
  std::vector<long> off((size_t)count + 1, 0);
  for (int i = 0; i < count; ++i) {
    if (!P[i] || !A[i] || !B[i]) return set_error(SFISTA_ERR_ARG, "image %d: NULL device pointer", i);
    const int rc = kron_check(m[i], n[i], l[i], q[i], bc[i], r[i]);
    if (rc != SFISTA_OK) {
      const std::string msg = last_error_slot();
      return set_error(rc, "image %d: %s", i, msg.c_str());
    }
    off[i + 1] = off[i] + 1 + r[i];
  }
  DeviceArena rar;
  double* res = static_cast<double*>(rar.alloc_zero((size_t)off[count] * 8, stream));
  if (!res) return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", rar.last_error());
  const int ns = std::min(count, KRON_STREAMS);
  std::vector<hipStream_t> st(ns, nullptr);
  std::vector<hipEvent_t> ev(ns + 1, nullptr);
  int rc = SFISTA_OK;
  hipError_t e = hipSuccess;
  for (int k = 0; k <= ns && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev[ns], stream);   // inputs and the cleared results are ready
  for (int k = 0; k < ns && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&st[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamWaitEvent(st[k], ev[ns], 0);
  }
  if (e != hipSuccess) rc = hip_fail(e, "kron_approx_batch streams");
  for (int i = 0; i < count && rc == SFISTA_OK; ++i)
    rc = kron_enqueue(P[i], m[i], n[i], l[i], q[i], bc[i], r[i], A[i], B[i], nullptr, nullptr, res + off[i],
                      st[i % ns]);
  // the caller's stream waits for every internal stream (also after a failure,
  // so that nothing queued outlives the call)
  for (int k = 0; k < ns; ++k) {
    if (!st[k] || !ev[k]) continue;
    if (hipEventRecord(ev[k], st[k]) != hipSuccess || hipStreamWaitEvent(stream, ev[k], 0) != hipSuccess)
      (void)hipStreamSynchronize(st[k]);
  }
  std::vector<double> hres((size_t)off[count]);
  if (rc == SFISTA_OK &&
      ((e = hipMemcpyAsync(hres.data(), res, hres.size() * 8, hipMemcpyDeviceToHost, stream)) != hipSuccess))
    rc = hip_fail(e, "kron_approx_batch results");
  if ((e = hipStreamSynchronize(stream)) != hipSuccess && rc == SFISTA_OK) rc = hip_fail(e, "kron_approx_batch");
  for (int k = 0; k < ns; ++k) if (st[k]) (void)hipStreamDestroy(st[k]);
  for (hipEvent_t x : ev) if (x) (void)hipEventDestroy(x);
  if (rc != SFISTA_OK) return rc;
  long so = 0;
  for (int i = 0; i < count; ++i) {
    const int ri = kron_results(hres.data() + off[i], r[i], sigma ? sigma + so : nullptr, eps_s ? eps_s + i : nullptr);
    if (ri != SFISTA_OK) {
      const std::string msg = last_error_slot();
      return set_error(ri, "image %d: %s", i, msg.c_str());
    }
    so += r[i];
  }
  return SFISTA_OK;
}

extern "C" int kron_generators(const double* P, int m, int n, int l, int q, int bc, int r, double* h, double* k,
                               double* sigma, double* eps_s, hipStream_t s) {
  clear_error();
  if (!P || !h || !k) return set_error(SFISTA_ERR_ARG, "NULL device pointer");
  return kron_impl(P, m, n, l, q, bc, r, nullptr, nullptr, h, k, sigma, eps_s, s);
}
