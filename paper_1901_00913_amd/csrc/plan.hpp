// The single-image plan of Algorithm 2 (packed factor operands, work
// planes, GEMM work lists, iterate state) and the host helpers shared by the
// translation units that build on it.
#pragma once

#include <math.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/sfista.h"
#include "gemm.hpp"
#include "kernels.hpp"
#include "util.hpp"

struct sfista_plan {
  int m = 0, n = 0, r = 0, mode = 0, nonneg = 0, kind = 0;
  double lam = 0.0, L = 0.0;
  hipStream_t s = nullptr;
  long iter = 0;          // iterations completed (k)
  double tk = 1.0;        // t_{k+1}: momentum parameter of the next iteration
  double beta_prev = 0.0; // beta_k = (t_k - 1) / t_{k+1} of the last iteration
  // leading dimensions (elements) of the packed operands
  long ldW = 0, ldBc = 0, ldBt = 0, ldAt = 0, ldY = 0, ldT = 0, ldR = 0, ldS = 0;
  void *W[2] = {}, *Bc[2] = {}, *Bt[2] = {}, *At[2] = {};
  void *Y[2] = {}, *T[2] = {}, *R[2] = {}, *S[2] = {}, *Xop[2] = {};
  void* bobs_t = nullptr;
  void* st[2] = {};
  double* aux = nullptr;      // m x n FP64 scratch (power iterate, copies)
  double* red = nullptr;      // reduction partials [RED_BLOCKS] + scalars
  double* v0buf = nullptr;    // m x n start of the estimate of L (made on first use)
  double* lzq[2] = {};        // m x n Lanczos vectors q_j, q_{j-1} (made on first use)
  double* lzcoef = nullptr;   // 2 x steps Lanczos coefficients (alpha_j, beta_j^2)
  int lzcap = 0;              // steps lzcoef holds
  void* ws = nullptr;         // K-split partials of the planned products
  sf::GemmPlanDev pl[4];      // work lists of F1, F2, G1, G2
  double bobs_norm = 0.0;
  // optional per-GEMM event timing
  int timing = 0;              // 0 off, k >= 1: the products of every k-th iteration
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;   // (gemm kind, index of the start event)
  hipEvent_t mid_ev = nullptr;                     // recorded between a GEMM and its split reduction
  double t_sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};      // GEMM kernels 0..3, their reductions 4..7
  long t_cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  sf::DeviceArena own_arena;
  sf::DeviceArena* mem = &own_arena;   // the owner's arena when the plan is part of a multi-image handle
  ~sfista_plan() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace sf {

constexpr int EW_BLOCKS = 2048;
constexpr int EW_THREADS = 256;

inline long ld_of(long k) { return round_up(k, TileCfg::K_PAD); }
inline long rows_of(long r) { return round_up(r, TileCfg::ROW_PAD); }

inline int state_kind(int mode, int pair) {
  if (mode == M_F64) return ST_F64;
  return pair ? ST_PAIR : ST_F32;
}

template <int MODE>
inline GemmArgs gargs(void* const* a, long lda, void* const* b, long ldb, int M, int N, int K) {
  GemmArgs g;
  g.a[0] = a[0]; g.a[1] = a[1];
  g.b[0] = b[0]; g.b[1] = b[1];
  g.lda = lda; g.ldb = ldb;
  g.M = M; g.N = N; g.K = K;
  g.kchunk = 0;
  return g;
}

template <int MODE>
inline typename ModeTraits<MODE>::Acc* ws_of(sfista_plan* h) {
  return static_cast<typename ModeTraits<MODE>::Acc*>(h->ws);
}

// Workgroups of the planned GEMM kernel resident per CU.
template <int MODE>
inline int resident_per_cu() {
  using T = typename BigTile<MODE>::T;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_planned_kernel<MODE, T, EpiStack<MODE>>, T::THREADS, 0) !=
          hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

// Host-side checks of one problem, before any device work.
inline int validate_problem(const double* Bobs, int m, int n, const double* A, const double* B, int r,
                            const sfista_params* p) {
  if (!Bobs || !A || !B || !p) return set_error(SFISTA_ERR_ARG, "NULL input pointer");
  if (m < 1 || n < 1) return set_error(SFISTA_ERR_ARG, "image size %d x %d must be positive", m, n);
  if (r < 1 || r > (m < n ? m : n)) return set_error(SFISTA_ERR_ARG, "rank r=%d must lie in [1, min(m,n)]", r);
  if ((long)r * m > (1L << 30) || (long)r * n > (1L << 30))
    return set_error(SFISTA_ERR_UNSUPPORTED, "r*m or r*n exceeds 2^30");
  if (!isfinite(p->lambda) || p->lambda < 0.0) return set_error(SFISTA_ERR_ARG, "lambda must be finite and >= 0");
  if (!isfinite(p->L)) return set_error(SFISTA_ERR_ARG, "L must be finite");
  if (p->precision < SFISTA_FP64 || p->precision > SFISTA_BF16X3)
    return set_error(SFISTA_ERR_UNSUPPORTED, "unknown precision %d", p->precision);
  if (p->power_iters < 0) return set_error(SFISTA_ERR_ARG, "power_iters must be >= 0");
  if (p->l_estimate != SFISTA_L_POWER && p->l_estimate != SFISTA_L_LANCZOS)
    return set_error(SFISTA_ERR_ARG, "unknown l_estimate %d", p->l_estimate);
  return SFISTA_OK;
}

// Validates and sets up one problem (the work of sfista_setup).  With
// `shared` non-null the plan's device buffers come from that arena, which
// has to outlive the plan.
int plan_create(const double* Bobs, int m, int n, const double* A, const double* B, int r, const sfista_params* p,
                hipStream_t stream, DeviceArena* shared, sfista_plan** out);

// Loads a new problem of the plan's sizes and rank into an existing plan:
// factors, observation, lambda, L (estimated again when L <= 0) and X_0 = 0.
// Allocates nothing after the first estimate of L; synchronises the stream.
int plan_refresh(sfista_plan* h, const double* Bobs, const double* A, const double* B, double lambda, double L);

}  // namespace sf
