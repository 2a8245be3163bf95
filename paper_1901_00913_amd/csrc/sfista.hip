// sFISTA solver plan: operand packing, the four term-stacked GEMMs of one
// iteration of Algorithm 2, the fused momentum/prox update, the power
// iteration for L, and the FP64 report.  C ABI declared in include/sfista.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/sfista.h"
#include "gemm.hpp"
#include "kernels.hpp"
#include "util.hpp"

using namespace sf;

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
  void* ws = nullptr;         // K-split partials of F2 and G2
  int split_f2 = 1, split_g2 = 1;
  double bobs_norm = 0.0;
  // optional per-GEMM event timing
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;   // (gemm kind, index of the start event)
  double t_sum[4] = {0, 0, 0, 0};
  long t_cnt[4] = {0, 0, 0, 0};
  DeviceArena arena;
  ~sfista_plan() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr int EW_BLOCKS = 2048;
constexpr int EW_THREADS = 256;

long ld_of(long k) { return round_up(k, TileCfg::K_PAD); }
long rows_of(long r) { return round_up(r, TileCfg::ROW_PAD); }

int state_kind(int mode, int pair) {
  if (mode == M_F64) return ST_F64;
  return pair ? ST_PAIR : ST_F32;
}

// ------------------------------------------------------------------ timing
hipEvent_t next_event(sfista_plan* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Brackets one GEMM launch with events when timing is enabled.
template <class F>
hipError_t timed(sfista_plan* h, int kind, F&& launch) {
  if (!h->timing) return launch();
  const size_t idx = h->ev_used;
  hipEvent_t a = next_event(h), b = next_event(h);
  if (!a || !b) return hipErrorOutOfMemory;
  (void)hipEventRecord(a, h->s);
  hipError_t e = launch();
  (void)hipEventRecord(b, h->s);
  h->ev_marks.push_back({kind, idx});
  return e;
}

hipError_t collect_times(sfista_plan* h) {
  if (h->ev_marks.empty()) return hipSuccess;
  hipError_t e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return e;
  for (auto& mk : h->ev_marks) {
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, h->ev_pool[mk.second], h->ev_pool[mk.second + 1])) != hipSuccess) return e;
    h->t_sum[mk.first] += ms;
    h->t_cnt[mk.first] += 1;
  }
  h->ev_marks.clear();
  h->ev_used = 0;
  return hipSuccess;
}

// ------------------------------------------------------------------ GEMMs
template <int MODE>
GemmArgs gargs(void* const* a, long lda, void* const* b, long ldb, int M, int N, int K) {
  GemmArgs g;
  g.a[0] = a[0]; g.a[1] = a[1];
  g.b[0] = b[0]; g.b[1] = b[1];
  g.lda = lda; g.ldb = ldb;
  g.M = M; g.N = N; g.K = K;
  g.kchunk = 0;
  return g;
}

// F1: T_k = Y A_k^T for all k, stored as T^T (n x rm):  Tt[j][k m + i].
template <int MODE>
hipError_t run_f1(sfista_plan* h, void* const* y, long ldy) {
  EpiStack<MODE> e;
  e.out[0] = h->T[0]; e.out[1] = h->T[1]; e.ldo = h->ldT; e.D = h->n; e.colblk = h->m;
  return launch_gemm<MODE>(gargs<MODE>(h->W, h->ldW, y, ldy, h->r * h->n, h->m, h->n), e, h->s);
}

// F2: R^T = (sum_k B_k T_k)^T - Bobs^T   (bobs optional)
template <int MODE>
hipError_t run_f2(sfista_plan* h, bool with_bobs, double* copy) {
  EpiResid<MODE> e;
  e.out[0] = h->R[0]; e.out[1] = h->R[1]; e.ldo = h->ldR;
  e.bobs_t = with_bobs ? static_cast<const typename ModeTraits<MODE>::Acc*>(h->bobs_t) : nullptr;
  e.m = h->m; e.copy = copy; e.n = h->n;
  return launch_gemm<MODE>(gargs<MODE>(h->T, h->ldT, h->Bc, h->ldBc, h->n, h->m, h->r * h->m), e, h->s,
                           h->split_f2, static_cast<typename ModeTraits<MODE>::Acc*>(h->ws));
}

// G1: S_k = B_k^T R for all k, stored side by side (m x rn): S[i][k n + j].
template <int MODE>
hipError_t run_g1(sfista_plan* h) {
  EpiStack<MODE> e;
  e.out[0] = h->S[0]; e.out[1] = h->S[1]; e.ldo = h->ldS; e.D = h->m; e.colblk = h->n;
  return launch_gemm<MODE>(gargs<MODE>(h->Bt, h->ldBt, h->R, h->ldR, h->r * h->m, h->n, h->m), e, h->s);
}

// G2 with an arbitrary epilogue: sum_k S_k A_k.
template <int MODE, class Epi>
hipError_t run_g2(sfista_plan* h, const Epi& e) {
  return launch_gemm<MODE>(gargs<MODE>(h->S, h->ldS, h->At, h->ldAt, h->m, h->n, h->r * h->n), e, h->s,
                           h->split_g2, static_cast<typename ModeTraits<MODE>::Acc*>(h->ws));
}

template <int MODE>
hipError_t run_iteration(sfista_plan* h) {
  const long k = h->iter + 1;
  const double t_next = (1.0 + sqrt(1.0 + 4.0 * h->tk * h->tk)) / 2.0;   // Step 2
  const double beta_k = (h->tk - 1.0) / t_next;                         // Step 3 weight
  hipError_t e;
  if ((e = timed(h, 0, [&] { return run_f1<MODE>(h, h->Y, h->ldY); })) != hipSuccess) return e;
  if ((e = timed(h, 1, [&] { return run_f2<MODE>(h, true, nullptr); })) != hipSuccess) return e;
  if ((e = timed(h, 2, [&] { return run_g1<MODE>(h); })) != hipSuccess) return e;
  const double inv = 1.0 / (h->L + h->lam * h->lam);
  void* x1 = h->st[(k - 1) & 1];
  void* x2 = h->st[k & 1];
  auto fill = [&](auto& u) {
    u.y[0] = h->Y[0]; u.y[1] = h->Y[1]; u.ldy = h->ldY;
    u.x1 = x1; u.x2 = x2; u.n = h->n;
    u.c1 = h->L * inv; u.c2 = inv; u.bp = h->beta_prev; u.bc = beta_k; u.nonneg = h->nonneg;
  };
  if (h->kind == ST_F64) {
    EpiUpdate<MODE, ST_F64> u; fill(u); e = timed(h, 3, [&] { return run_g2<MODE>(h, u); });
  } else if (h->kind == ST_PAIR) {
    EpiUpdate<MODE, ST_PAIR> u; fill(u); e = timed(h, 3, [&] { return run_g2<MODE>(h, u); });
  } else {
    EpiUpdate<MODE, ST_F32> u; fill(u); e = timed(h, 3, [&] { return run_g2<MODE>(h, u); });
  }
  if (e != hipSuccess) return e;
  h->beta_prev = beta_k;
  h->tk = t_next;
  h->iter = k;
  return hipSuccess;
}

// Normal operator on the planes in `src`: out = A_s^T A_s (src) in FP64;
// `ax` (optional) receives A_s(src) in FP64.
template <int MODE>
hipError_t run_normal(sfista_plan* h, void* const* src, long ldsrc, double* ax, double* out) {
  hipError_t e;
  if ((e = run_f1<MODE>(h, src, ldsrc)) != hipSuccess) return e;
  if ((e = run_f2<MODE>(h, false, ax)) != hipSuccess) return e;
  if (!out) return hipSuccess;
  if ((e = run_g1<MODE>(h)) != hipSuccess) return e;
  EpiStore<MODE> st;
  st.out = out; st.n = h->n;
  return run_g2<MODE>(h, st);
}

// Power iteration for L = lambda_max(A_s^T A_s):  V <- V / ||V||,
// W = A_s^T A_s V, estimate ||W||, V <- W.  Norms in FP64 on the device.
template <int MODE>
hipError_t run_power(sfista_plan* h, const double* v0, int steps, double* L_out) {
  const long mn = (long)h->m * h->n;
  double* partial = h->red;
  double* scal = h->red + RED_BLOCKS;
  hipError_t e;
  if ((e = sumsq(DoubleSq{v0}, mn, partial, scal, h->s)) != hipSuccess) return e;
  hipLaunchKernelGGL(to_planes_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, v0, scal,
                     h->Y[0], h->Y[1], h->ldY, h->m, h->n);
  for (int it = 0; it < steps; ++it) {
    if ((e = run_normal<MODE>(h, h->Y, h->ldY, nullptr, h->aux)) != hipSuccess) return e;
    if ((e = sumsq(DoubleSq{h->aux}, mn, partial, scal, h->s)) != hipSuccess) return e;
    if (it + 1 < steps)
      hipLaunchKernelGGL(to_planes_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, h->aux, scal,
                         h->Y[0], h->Y[1], h->ldY, h->m, h->n);
  }
  double ss = 0.0;
  if ((e = hipMemcpyAsync(&ss, scal, sizeof(double), hipMemcpyDeviceToHost, h->s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return e;
  *L_out = sqrt(ss);
  return hipSuccess;
}

template <int MODE>
hipError_t run_pack(sfista_plan* h, const double* A, const double* B) {
  const int m = h->m, n = h->n, r = h->r;
  auto pk = [&](const double* src, void* const* o, long ldo, int kind, int d, long rows, long cols) {
    hipLaunchKernelGGL(pack_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, src, o[0], o[1], ldo,
                       kind, d, rows, cols);
  };
  pk(A, h->W, h->ldW, PK_STACK, n, (long)r * n, n);
  pk(B, h->Bc, h->ldBc, PK_CAT, m, m, (long)r * m);
  pk(B, h->Bt, h->ldBt, PK_STACK_T, m, (long)r * m, m);
  pk(A, h->At, h->ldAt, PK_CAT_T, n, n, (long)r * n);
  return hipGetLastError();
}

template <int MODE>
int setup_mode(sfista_plan* h, const double* Bobs, const double* A, const double* B, const sfista_params* p) {
  using Acc = typename ModeTraits<MODE>::Acc;
  constexpr int P = ModeTraits<MODE>::planes;
  constexpr int es = ModeTraits<MODE>::esize;
  const int m = h->m, n = h->n, r = h->r;
  const long rm = (long)r * m, rn = (long)r * n;
  h->ldW = ld_of(n);  h->ldBc = ld_of(rm); h->ldBt = ld_of(m); h->ldAt = ld_of(rn);
  h->ldY = ld_of(n);  h->ldT = ld_of(rm);  h->ldR = ld_of(m);  h->ldS = ld_of(rn);
  auto planes = [&](void** dst, long rows, long ld) -> bool {
    for (int q = 0; q < P; ++q) {
      dst[q] = h->arena.alloc_zero((size_t)rows_of(rows) * ld * es, h->s);
      if (!dst[q]) return false;
    }
    return true;
  };
  bool ok = planes(h->W, rn, h->ldW) && planes(h->Bc, m, h->ldBc) && planes(h->Bt, rm, h->ldBt) &&
            planes(h->At, n, h->ldAt) && planes(h->Y, m, h->ldY) && planes(h->T, n, h->ldT) &&
            planes(h->R, n, h->ldR) && planes(h->S, m, h->ldS) && planes(h->Xop, m, h->ldY);
  const size_t st_bytes = (size_t)m * n * (h->kind == ST_F32 ? 4 : 8);
  ok = ok && (h->bobs_t = h->arena.alloc_zero((size_t)m * n * sizeof(Acc), h->s)) &&
       (h->st[0] = h->arena.alloc_zero(st_bytes, h->s)) && (h->st[1] = h->arena.alloc_zero(st_bytes, h->s)) &&
       (h->aux = static_cast<double*>(h->arena.alloc_zero((size_t)m * n * 8, h->s))) &&
       (h->red = static_cast<double*>(h->arena.alloc_zero((RED_BLOCKS + 8) * 8, h->s)));
  if (!ok) return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", h->arena.last_error());

  // K splits for the two square products (their tile count alone can leave CUs idle)
  {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const int per_cu = (int)(160 * 1024 / gemm_lds_bytes<MODE>()) > 1 ? 2 : 1;
    h->split_f2 = choose_splitk<MODE>(n, m, (int)rm, cus * per_cu);
    h->split_g2 = choose_splitk<MODE>(m, n, (int)rn, cus * per_cu);
    const int smax = h->split_f2 > h->split_g2 ? h->split_f2 : h->split_g2;
    if (smax > 1 && !(h->ws = h->arena.alloc_zero((size_t)smax * m * n * sizeof(Acc), h->s)))
      return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", h->arena.last_error());
  }

  hipError_t e;
  if ((e = run_pack<MODE>(h, A, B)) != hipSuccess) return hip_fail(e, "factor packing");
  {
    dim3 blk(32, 8), grd((n + 31) / 32, (m + 31) / 32);
    hipLaunchKernelGGL(transpose_to_kernel<Acc>, grd, blk, 0, h->s, Bobs, static_cast<Acc*>(h->bobs_t), m, n);
  }
  double* scal = h->red + RED_BLOCKS;
  if ((e = sumsq(DoubleSq{Bobs}, (long)m * n, h->red, scal, h->s)) != hipSuccess) return hip_fail(e, "norm");
  double ss = 0.0;
  if ((e = hipMemcpyAsync(&ss, scal, 8, hipMemcpyDeviceToHost, h->s)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return hip_fail(e, "setup");
  h->bobs_norm = sqrt(ss);

  if (!(h->L > 0.0)) {
    const int steps = p->power_iters > 0 ? p->power_iters : 30;
    const double* v0 = p->v0;
    if (!v0) {
      // fixed internal start: a deterministic hash pattern
      void* tmp = h->arena.alloc_zero((size_t)m * n * 8, h->s);
      if (!tmp) return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
      hipLaunchKernelGGL(hash_fill_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, static_cast<double*>(tmp),
                         (long)m * n, 0x5f15a7ull);
      v0 = static_cast<const double*>(tmp);
    }
    double L = 0.0;
    if ((e = run_power<MODE>(h, v0, steps, &L)) != hipSuccess) return hip_fail(e, "power iteration");
    if (!isfinite(L) || !(L > 0.0)) return set_error(SFISTA_ERR_NONFINITE, "Lipschitz estimate is %g", L);
    h->L = L;
  }
  hipLaunchKernelGGL(init_state_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, p->x0, h->st[0],
                     h->st[1], h->kind, h->Y[0], h->Y[1], h->ldY, m, n);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "state init");
  if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return hip_fail(e, "setup");
  return SFISTA_OK;
}

template <int MODE>
hipError_t steps_mode(sfista_plan* h, int iters) {
  for (int i = 0; i < iters; ++i) {
    hipError_t e = run_iteration<MODE>(h);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int MODE>
hipError_t report_mode(sfista_plan* h, double* rr, double* xx) {
  const long mn = (long)h->m * h->n;
  const void* xk = h->st[h->iter & 1];
  hipLaunchKernelGGL(state_to_planes_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, xk, h->kind,
                     h->Xop[0], h->Xop[1], h->ldY, h->m, h->n);
  hipError_t e;
  if ((e = run_f1<MODE>(h, h->Xop, h->ldY)) != hipSuccess) return e;
  if ((e = run_f2<MODE>(h, true, h->aux)) != hipSuccess) return e;
  double* partial = h->red;
  double* scal = h->red + RED_BLOCKS;
  if ((e = sumsq(DoubleSq{h->aux}, mn, partial, scal, h->s)) != hipSuccess) return e;
  if ((e = sumsq(StateSq{xk, h->kind}, mn, partial, scal + 1, h->s)) != hipSuccess) return e;
  double v[2];
  if ((e = hipMemcpyAsync(v, scal, 16, hipMemcpyDeviceToHost, h->s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return e;
  *rr = v[0];
  *xx = v[1];
  return hipSuccess;
}

template <int MODE>
hipError_t apply_mode(sfista_plan* h, const double* X, double* AX, double* AtAX) {
  hipLaunchKernelGGL(to_planes_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, X, nullptr, h->Xop[0],
                     h->Xop[1], h->ldY, h->m, h->n);
  hipError_t e = run_normal<MODE>(h, h->Xop, h->ldY, AX, AtAX);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(h->s);
}

#define SF_DISPATCH(mode, call)                       \
  switch (mode) {                                     \
    case M_F64: { constexpr int MD = M_F64; call; } break;       \
    case M_F32: { constexpr int MD = M_F32; call; } break;       \
    case M_BF16: { constexpr int MD = M_BF16; call; } break;     \
    case M_F16: { constexpr int MD = M_F16; call; } break;       \
    default: { constexpr int MD = M_BF16X3; call; } break;       \
  }

}  // namespace

// ====================================================================== C ABI
extern "C" {

int sfista_setup(const double* Bobs, int m, int n, const double* A, const double* B, int r,
                 const sfista_params* p, hipStream_t stream, sfista_handle* out) {
  clear_error();
  if (!out) return set_error(SFISTA_ERR_ARG, "out handle pointer is NULL");
  *out = nullptr;
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
  sfista_plan* h = new (std::nothrow) sfista_plan();
  if (!h) return set_error(SFISTA_ERR_NOMEM, "host allocation failed");
  h->m = m; h->n = n; h->r = r; h->mode = p->precision; h->nonneg = p->nonneg ? 1 : 0;
  h->kind = state_kind(h->mode, p->pair_state);
  h->lam = p->lambda; h->L = p->L > 0.0 ? p->L : 0.0; h->s = stream;
  int rc = SFISTA_OK;
  SF_DISPATCH(h->mode, rc = setup_mode<MD>(h, Bobs, A, B, p));
  if (rc != SFISTA_OK) {
    (void)hipStreamSynchronize(stream);
    delete h;
    return rc;
  }
  *out = h;
  return SFISTA_OK;
}

int sfista_step(sfista_handle h, int iters) {
  clear_error();
  if (!h) return set_error(SFISTA_ERR_ARG, "NULL handle");
  if (iters < 0) return set_error(SFISTA_ERR_ARG, "iters must be >= 0");
  hipError_t e = hipSuccess;
  SF_DISPATCH(h->mode, e = steps_mode<MD>(h, iters));
  if (e != hipSuccess) return hip_fail(e, "sfista_step");
  return SFISTA_OK;
}

int sfista_solve(sfista_handle h, int max_iters, double tol, double* X_out, sfista_report* rep) {
  clear_error();
  if (!h) return set_error(SFISTA_ERR_ARG, "NULL handle");
  if (max_iters < 0 || !(tol >= 0.0)) return set_error(SFISTA_ERR_ARG, "max_iters >= 0 and tol >= 0 required");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return hip_fail(e, "event create");
  (void)hipEventRecord(e0, h->s);
  const long mn = (long)h->m * h->n;
  int done = 0;
  while (done < max_iters) {
    int chunk = max_iters - done;
    if (tol > 0.0 && chunk > 10) chunk = 10;
    SF_DISPATCH(h->mode, e = steps_mode<MD>(h, chunk));
    if (e != hipSuccess) break;
    done += chunk;
    if (tol > 0.0 && h->iter >= 1) {
      double* scal = h->red + RED_BLOCKS;
      (void)sumsq(StateDiffSq{h->st[0], h->st[1], h->kind}, mn, h->red, scal + 2, h->s);
      (void)sumsq(StateSq{h->st[h->iter & 1], h->kind}, mn, h->red, scal + 3, h->s);
      double v[2];
      if ((e = hipMemcpyAsync(v, scal + 2, 16, hipMemcpyDeviceToHost, h->s)) != hipSuccess) break;
      if ((e = hipStreamSynchronize(h->s)) != hipSuccess) break;
      if (sqrt(v[0]) <= tol * sqrt(v[1])) break;
    }
  }
  (void)hipEventRecord(e1, h->s);
  if (e == hipSuccess) e = collect_times(h);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
    return hip_fail(e, "sfista_solve iterations");
  }
  double rr = 0.0, xx = 0.0;
  SF_DISPATCH(h->mode, e = report_mode<MD>(h, &rr, &xx));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0); (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "sfista_solve report");
  if (X_out) {
    hipLaunchKernelGGL(state_to_double_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, h->st[h->iter & 1],
                       h->kind, X_out, mn);
    if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return hip_fail(e, "copy X");
  }
  int status = SFISTA_OK;
  const double phi = 0.5 * rr + 0.5 * h->lam * h->lam * xx;
  if (!isfinite(phi)) status = set_error(SFISTA_ERR_NONFINITE, "objective is not finite after %ld iterations", h->iter);
  if (rep) {
    rep->iters = (int)h->iter;
    rep->seconds = ms * 1e-3;
    rep->L = h->L;
    rep->phi_s = phi;
    rep->resid_norm = sqrt(rr);
    rep->bobs_norm = h->bobs_norm;
    rep->x_norm = sqrt(xx);
    rep->resid_rel = h->bobs_norm > 0 ? sqrt(rr) / h->bobs_norm : 0.0;
    rep->status = status;
  }
  return status;
}

int sfista_apply(sfista_handle h, const double* X, double* AX, double* AtAX) {
  clear_error();
  if (!h || !X) return set_error(SFISTA_ERR_ARG, "NULL argument");
  hipError_t e = hipSuccess;
  SF_DISPATCH(h->mode, e = apply_mode<MD>(h, X, AX, AtAX));
  if (e != hipSuccess) return hip_fail(e, "sfista_apply");
  return SFISTA_OK;
}

int sfista_set_timing(sfista_handle h, int enable) {
  clear_error();
  if (!h) return set_error(SFISTA_ERR_ARG, "NULL handle");
  h->timing = enable ? 1 : 0;
  return SFISTA_OK;
}

int sfista_kernel_times(sfista_handle h, double* avg_ms, long* launches) {
  clear_error();
  if (!h || !avg_ms || !launches) return set_error(SFISTA_ERR_ARG, "NULL argument");
  hipError_t e = collect_times(h);
  if (e != hipSuccess) return hip_fail(e, "sfista_kernel_times");
  for (int k = 0; k < 4; ++k) {
    avg_ms[k] = h->t_cnt[k] ? h->t_sum[k] / h->t_cnt[k] : 0.0;
    launches[k] = h->t_cnt[k];
    h->t_sum[k] = 0.0;
    h->t_cnt[k] = 0;
  }
  return SFISTA_OK;
}

int sfista_get_L(sfista_handle h, double* L) {
  clear_error();
  if (!h || !L) return set_error(SFISTA_ERR_ARG, "NULL argument");
  *L = h->L;
  return SFISTA_OK;
}

void sfista_destroy(sfista_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->s);
  delete h;
}

const char* sfista_last_error(void) { return last_error_slot().c_str(); }

}  // extern "C"
