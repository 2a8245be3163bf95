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
#include "plan.hpp"
#include "util.hpp"

using namespace sf;


namespace {


// ------------------------------------------------------------------ timing
hipEvent_t next_event(sfista_plan* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Brackets one GEMM launch with events when timing is on for this iteration
// (every h->timing-th one): start, after the GEMM kernel (mid_ev, recorded by
// launch_planned) and after its split reduction.  Each event record leaves a
// gap of several microseconds before the next kernel, so sampling keeps the
// timed iterations close to untimed ones.
template <class F>
hipError_t timed(sfista_plan* h, int kind, F&& launch) {
  if (h->timing <= 0 || h->iter % h->timing != 0) return launch();
  const size_t idx = h->ev_used;
  hipEvent_t a = next_event(h), mid = next_event(h), b = next_event(h);
  if (!a || !mid || !b) return hipErrorOutOfMemory;
  (void)hipEventRecord(a, h->s);
  h->mid_ev = mid;
  hipError_t e = launch();
  h->mid_ev = nullptr;
  (void)hipEventRecord(b, h->s);
  h->ev_marks.push_back({kind, idx});
  return e;
}

hipError_t collect_times(sfista_plan* h) {
  if (h->ev_marks.empty()) return hipSuccess;
  hipError_t e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return e;
  for (auto& mk : h->ev_marks) {
    float g = 0.f, r = 0.f;
    if ((e = hipEventElapsedTime(&g, h->ev_pool[mk.second], h->ev_pool[mk.second + 1])) != hipSuccess) return e;
    if ((e = hipEventElapsedTime(&r, h->ev_pool[mk.second + 1], h->ev_pool[mk.second + 2])) != hipSuccess) return e;
    h->t_sum[mk.first] += g;
    h->t_cnt[mk.first] += 1;
    if (h->pl[mk.first].nsplit > 0) {   // products without split tiles launch no reduction
      h->t_sum[4 + mk.first] += r;
      h->t_cnt[4 + mk.first] += 1;
    }
  }
  h->ev_marks.clear();
  h->ev_used = 0;
  return hipSuccess;
}

// ------------------------------------------------------------------ GEMMs
// F1: T_k = Y A_k^T for all k, stored as T^T (n x rm):  Tt[j][k m + i].
template <int MODE>
hipError_t run_f1(sfista_plan* h, void* const* y, long ldy) {
  EpiStack<MODE> e;
  e.out[0] = h->T[0]; e.out[1] = h->T[1]; e.ldo = h->ldT; e.D = h->n; e.colblk = h->m;
  return launch_planned<MODE>(gargs<MODE>(h->W, h->ldW, y, ldy, h->r * h->n, h->m, h->n), e, h->pl[0], ws_of<MODE>(h),
                              h->s, h->mid_ev);
}

// F2: R^T = (sum_k B_k T_k)^T - Bobs^T   (bobs optional)
template <int MODE>
hipError_t run_f2(sfista_plan* h, bool with_bobs, double* copy) {
  EpiResid<MODE> e;
  e.out[0] = h->R[0]; e.out[1] = h->R[1]; e.ldo = h->ldR;
  e.bobs_t = with_bobs ? static_cast<const typename ModeTraits<MODE>::Acc*>(h->bobs_t) : nullptr;
  e.m = h->m; e.copy = copy; e.n = h->n;
  return launch_planned<MODE>(gargs<MODE>(h->T, h->ldT, h->Bc, h->ldBc, h->n, h->m, h->r * h->m), e, h->pl[1],
                              ws_of<MODE>(h), h->s, h->mid_ev);
}

// G1: S_k = B_k^T R for all k, stored side by side (m x rn): S[i][k n + j].
template <int MODE>
hipError_t run_g1(sfista_plan* h) {
  EpiStack<MODE> e;
  e.out[0] = h->S[0]; e.out[1] = h->S[1]; e.ldo = h->ldS; e.D = h->m; e.colblk = h->n;
  return launch_planned<MODE>(gargs<MODE>(h->Bt, h->ldBt, h->R, h->ldR, h->r * h->m, h->n, h->m), e, h->pl[2],
                              ws_of<MODE>(h), h->s, h->mid_ev);
}

// G2 with an arbitrary epilogue: sum_k S_k A_k.
template <int MODE, class Epi>
hipError_t run_g2(sfista_plan* h, const Epi& e) {
  return launch_planned<MODE>(gargs<MODE>(h->S, h->ldS, h->At, h->ldAt, h->m, h->n, h->r * h->n), e, h->pl[3],
                              ws_of<MODE>(h), h->s, h->mid_ev);
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

// Lanczos estimate of L (the coefficient recurrence of lanczos_orth_kernel):
// q_0 = v0 / ||v0||; step j forms w = A_s^T A_s q_j through the plan's four
// products, alpha_j = <q_j, w>, orthogonalises w against q_j and q_{j-1},
// stores ||w||^2 and normalises w into q_{j+1}.  The coefficients stay on the
// device until the end; the host takes the largest Ritz value.
template <int MODE>
hipError_t run_lanczos(sfista_plan* h, const double* v0, int steps, double* L_out) {
  const long mn = (long)h->m * h->n;
  double* partial = h->red;
  double* scal = h->red + RED_BLOCKS;
  for (int i = 0; i < 2; ++i)
    if (!h->lzq[i] && !(h->lzq[i] = static_cast<double*>(h->mem->alloc_zero((size_t)mn * 8, h->s))))
      return hipErrorOutOfMemory;
  if (h->lzcap < steps) {
    if (!(h->lzcoef = static_cast<double*>(h->mem->alloc_zero((size_t)steps * 2 * 8, h->s))))
      return hipErrorOutOfMemory;
    h->lzcap = steps;
  }
  double* coef = h->lzcoef;
  hipError_t e;
  if ((e = sumsq(DoubleSq{v0}, mn, partial, scal, h->s)) != hipSuccess) return e;
  hipLaunchKernelGGL(lanczos_scale_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, v0, scal, h->lzq[0], mn);
  int cur = 0;
  for (int j = 0; j < steps; ++j) {
    double* q = h->lzq[cur];
    double* qo = h->lzq[cur ^ 1];      // q_{j-1}, then q_{j+1}
    hipLaunchKernelGGL(to_planes_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, q, nullptr, h->Y[0],
                       h->Y[1], h->ldY, h->m, h->n);
    if ((e = run_normal<MODE>(h, h->Y, h->ldY, nullptr, h->aux)) != hipSuccess) return e;
    if ((e = sumf(DoubleDot{q, h->aux}, mn, partial, coef + 2 * j, h->s)) != hipSuccess) return e;
    hipLaunchKernelGGL(lanczos_orth_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, h->s, h->aux, q, qo, coef, j, mn,
                       partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RED_THREADS), 0, h->s, partial, RED_BLOCKS, coef + 2 * j + 1);
    if (j + 1 < steps) {
      hipLaunchKernelGGL(lanczos_scale_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, h->aux, coef + 2 * j + 1,
                         qo, mn);
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
int load_problem(sfista_plan* h, const double* Bobs, const double* A, const double* B, const sfista_params* p);

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
      dst[q] = h->mem->alloc_zero((size_t)rows_of(rows) * ld * es, h->s);
      if (!dst[q]) return false;
    }
    return true;
  };
  bool ok = planes(h->W, rn, h->ldW) && planes(h->Bc, m, h->ldBc) && planes(h->Bt, rm, h->ldBt) &&
            planes(h->At, n, h->ldAt) && planes(h->Y, m, h->ldY) && planes(h->T, n, h->ldT) &&
            planes(h->R, n, h->ldR) && planes(h->S, m, h->ldS) && planes(h->Xop, m, h->ldY);
  const size_t st_bytes = (size_t)m * n * (h->kind == ST_F32 ? 4 : 8);
  ok = ok && (h->bobs_t = h->mem->alloc_zero((size_t)m * n * sizeof(Acc), h->s)) &&
       (h->st[0] = h->mem->alloc_zero(st_bytes, h->s)) && (h->st[1] = h->mem->alloc_zero(st_bytes, h->s)) &&
       (h->aux = static_cast<double*>(h->mem->alloc_zero((size_t)m * n * 8, h->s))) &&
       (h->red = static_cast<double*>(h->mem->alloc_zero((RED_BLOCKS + 8) * 8, h->s)));
  if (!ok) return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", h->mem->last_error());

  // work lists of the four products (tile order, K splits of the last round)
  {
    using TB = typename BigTile<MODE>::T;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    const int slots = cus * resident_per_cu<MODE>();
    const GemmPlan plans[4] = {
        plan_gemm<TB>((int)rn, m, gemm_kstages<MODE>(n), slots), plan_gemm<TB>(n, m, gemm_kstages<MODE>((int)rm), slots),
        plan_gemm<TB>((int)rm, n, gemm_kstages<MODE>(m), slots), plan_gemm<TB>(m, n, gemm_kstages<MODE>((int)rn), slots)};
    size_t ws_elems = 0;
    GemmPlan alt[4];
    bool use320[4] = {false, false, false, false};
    if constexpr (ModeTraits<MODE>::planes == 2) {
      const int Ms[4] = {(int)rn, n, (int)rm, m}, Ns[4] = {m, m, n, n}, Ks[4] = {n, (int)rm, m, (int)rn};
      for (int q = 0; q < 4; ++q) {
        if (Ms[q] % 320) continue;
        alt[q] = plan_gemm<Tile320>(Ms[q], Ns[q], gemm_kstages<MODE>(Ks[q]), cus);
        use320[q] = alt[q].split_tiles.empty() && plans[q].split_tiles.size() > 0;
      }
    }
    for (int q = 0; q < 4; ++q) {
      const GemmPlan& gp = use320[q] ? alt[q] : plans[q];
      h->pl[q].tile320 = use320[q] ? 1 : 0;
      GemmPlanDev& pd = h->pl[q];
      PlanItem* items = static_cast<PlanItem*>(h->mem->alloc_zero(gp.items.size() * sizeof(PlanItem), h->s));
      int2* tiles = gp.split_tiles.empty()
                        ? nullptr
                        : static_cast<int2*>(h->mem->alloc_zero(gp.split_tiles.size() * sizeof(int2), h->s));
      if (!items || (!gp.split_tiles.empty() && !tiles))
        return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", h->mem->last_error());
      if (hipMemcpyAsync(items, gp.items.data(), gp.items.size() * sizeof(PlanItem), hipMemcpyHostToDevice, h->s) !=
              hipSuccess ||
          (tiles && hipMemcpyAsync(tiles, gp.split_tiles.data(), gp.split_tiles.size() * sizeof(int2),
                                   hipMemcpyHostToDevice, h->s) != hipSuccess))
        return set_error(SFISTA_ERR_HIP, "plan upload failed");
      pd.items = items;
      pd.split_tiles = tiles;
      pd.nitems = (int)gp.items.size();
      pd.nsplit = (int)gp.split_tiles.size();
      pd.S = gp.S;
      pd.kchunk = gp.kchunk;
      ws_elems = std::max(ws_elems, gp.ws_elems() * TB::BM * TB::BN);
    }
    if (ws_elems > 0 && !(h->ws = h->mem->alloc_zero(ws_elems * sizeof(Acc), h->s)))
      return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", h->mem->last_error());
  }

  return load_problem<MODE>(h, Bobs, A, B, p);
}

// Packs the factors, stores Bobs^T, takes ||Bobs||, estimates L unless h->L
// is set, and sets X_0; synchronises the stream.
template <int MODE>
int load_problem(sfista_plan* h, const double* Bobs, const double* A, const double* B, const sfista_params* p) {
  using Acc = typename ModeTraits<MODE>::Acc;
  const int m = h->m, n = h->n;
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
    const bool lanczos = p->l_estimate == SFISTA_L_LANCZOS;
    const int steps = p->power_iters > 0 ? p->power_iters : (lanczos ? 12 : 30);
    const double* v0 = p->v0;
    if (!v0) {
      // fixed internal start: a deterministic hash pattern
      if (!h->v0buf && !(h->v0buf = static_cast<double*>(h->mem->alloc_zero((size_t)m * n * 8, h->s))))
        return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
      hipLaunchKernelGGL(hash_fill_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, h->v0buf, (long)m * n,
                         0x5f15a7ull);
      v0 = h->v0buf;
    }
    double L = 0.0;
    if ((e = lanczos ? run_lanczos<MODE>(h, v0, steps, &L) : run_power<MODE>(h, v0, steps, &L)) != hipSuccess)
      return hip_fail(e, lanczos ? "Lanczos estimate of L" : "power iteration");
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

namespace sf {

int plan_create(const double* Bobs, int m, int n, const double* A, const double* B, int r, const sfista_params* p,
                hipStream_t stream, DeviceArena* shared, sfista_plan** out) {
  const int rc0 = validate_problem(Bobs, m, n, A, B, r, p);
  if (rc0 != SFISTA_OK) return rc0;
  sfista_plan* h = new (std::nothrow) sfista_plan();
  if (!h) return set_error(SFISTA_ERR_NOMEM, "host allocation failed");
  if (shared) h->mem = shared;
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

int plan_refresh(sfista_plan* h, const double* Bobs, const double* A, const double* B, double lambda, double L) {
  sfista_params p{};
  p.lambda = lambda; p.L = L; p.precision = h->mode; p.power_iters = 30; p.nonneg = h->nonneg;
  const int rc0 = validate_problem(Bobs, h->m, h->n, A, B, h->r, &p);
  if (rc0 != SFISTA_OK) return rc0;
  h->lam = lambda; h->L = L > 0.0 ? L : 0.0;
  h->iter = 0; h->tk = 1.0; h->beta_prev = 0.0;
  int rc = SFISTA_OK;
  SF_DISPATCH(h->mode, rc = load_problem<MD>(h, Bobs, A, B, &p));
  return rc;
}

}  // namespace sf

// ====================================================================== C ABI

extern "C" {

int sfista_setup(const double* Bobs, int m, int n, const double* A, const double* B, int r,
                 const sfista_params* p, hipStream_t stream, sfista_handle* out) {
  clear_error();
  if (!out) return set_error(SFISTA_ERR_ARG, "out handle pointer is NULL");
  *out = nullptr;
  return plan_create(Bobs, m, n, A, B, r, p, stream, nullptr, out);
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

int sfista_set_timing(sfista_handle h, int every) {
  clear_error();
  if (!h) return set_error(SFISTA_ERR_ARG, "NULL handle");
  if (every < 0) return set_error(SFISTA_ERR_ARG, "every must be >= 0");
  h->timing = every;
  return SFISTA_OK;
}

int sfista_kernel_times(sfista_handle h, double* avg_ms, long* launches) {
  clear_error();
  if (!h || !avg_ms || !launches) return set_error(SFISTA_ERR_ARG, "NULL argument");
  hipError_t e = collect_times(h);
  if (e != hipSuccess) return hip_fail(e, "sfista_kernel_times");
  for (int k = 0; k < 8; ++k) {
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

int sfista_release_cached(void) {
  clear_error();
  const hipError_t e = release_cached_pools();
  return e == hipSuccess ? SFISTA_OK : hip_fail(e, "sfista_release_cached");
}

const char* sfista_last_error(void) { return last_error_slot().c_str(); }

}  // extern "C"

// ======================================================================
// Batched form
// ======================================================================
#include <stdlib.h>

#include <algorithm>
#include <fstream>
#include <sstream>
#include <type_traits>

struct sfista_batch {
  int count = 0, mode = 0, kind = 0, max_iters = 0, flags = 0;
  long iter = 0;
  hipStream_t s = nullptr;          // internal stream (default priority)
  std::vector<sfista_plan*> plans;
  DeviceArena arena;
  GemmArgs* dargs[4] = {};          // per product: device array of GEMM arguments (one per problem)
  void* depi[4] = {};               // per product: device array of epilogues
  WorkItem* dwork[4][3] = {};       // per product and tile shape: work list
  int nwork[4][3] = {};
  int choice[4] = {0, 0, 0, 0};     // 0 = the mode's big tile, 1 = TileS, 2 = Tile128
  void* dpow[2] = {};               // power iteration: F2 without Bobs, G2 storing A_s^T A_s V (per problem)
  std::vector<char> need_L;         // problems whose L the batch estimates
  int power_steps = 30;             // steps of the estimate of L
  int lanczos = 0;                  // 1: Lanczos estimate, 0: power iteration
  double* beta = nullptr;           // beta[k] = (t_k - 1) / t_{k+1}, beta[0] = 0
  int* counter = nullptr;           // iterations completed (device)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  ~sfista_batch() {
    if (s) (void)hipStreamSynchronize(s);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (sfista_plan* p : plans) delete p;
    arena.release();                // its frees are ordered on s
    if (s) (void)hipStreamDestroy(s);
  }
};

namespace {

constexpr int GRAPH_ITERS = 10;

template <int MODE, class T>
int tile_shape_index() {
  if (std::is_same<T, TileS>::value) return 1;
  return std::is_same<T, typename BigTile<MODE>::T>::value ? 0 : 2;
}

// Tile shape c exists in this mode (FP64's big tile is already 128 x 128).
template <int MODE>
bool shape_offered(int c) { return c != 2 || !std::is_same<typename BigTile<MODE>::T, Tile128>::value; }

template <int MODE, class T, class Epi>
hipError_t launch_grouped(sfista_batch* b, int prod, const void* epis) {
  const int c = tile_shape_index<MODE, T>();
  if (b->nwork[prod][c] == 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_grouped_kernel<MODE, T, Epi>), dim3(b->nwork[prod][c]), dim3(T::THREADS), 0, b->s,
                     b->dargs[prod], static_cast<const Epi*>(epis), b->dwork[prod][c]);
  return hipGetLastError();
}

// Product `prod` of every problem with the epilogue table `epis` (default:
// the iteration's).
template <int MODE, class Epi>
hipError_t launch_product(sfista_batch* b, int prod, const void* epis = nullptr) {
  if (!epis) epis = b->depi[prod];
  if (b->choice[prod] == 2) return launch_grouped<MODE, Tile128, Epi>(b, prod, epis);
  return b->choice[prod] ? launch_grouped<MODE, TileS, Epi>(b, prod, epis)
                         : launch_grouped<MODE, typename BigTile<MODE>::T, Epi>(b, prod, epis);
}

template <int MODE, int KIND>
hipError_t batch_iteration_k(sfista_batch* b) {
  hipError_t e;
  if ((e = launch_product<MODE, EpiStack<MODE>>(b, 0)) != hipSuccess) return e;
  if ((e = launch_product<MODE, EpiResid<MODE>>(b, 1)) != hipSuccess) return e;
  if ((e = launch_product<MODE, EpiStack<MODE>>(b, 2)) != hipSuccess) return e;
  if ((e = launch_product<MODE, EpiUpdateSeq<MODE, KIND>>(b, 3)) != hipSuccess) return e;
  hipLaunchKernelGGL(advance_counter_kernel, dim3(1), dim3(64), 0, b->s, b->counter);
  return hipGetLastError();
}

template <int MODE>
hipError_t batch_iteration(sfista_batch* b) {
  if (b->kind == ST_F64) return batch_iteration_k<MODE, ST_F64>(b);
  if (b->kind == ST_PAIR) return batch_iteration_k<MODE, ST_PAIR>(b);
  return batch_iteration_k<MODE, ST_F32>(b);
}

// The G2 epilogues of the iteration: they hold 1 / (L + lambda^2) per problem.
template <int MODE>
void fill_update_tables(const sfista_batch* b, std::vector<EpiUpdateSeq<MODE, ST_F64>>& u64,
                        std::vector<EpiUpdateSeq<MODE, ST_PAIR>>& upr, std::vector<EpiUpdateSeq<MODE, ST_F32>>& u32) {
  const int cnt = b->count;
  u64.resize(cnt); upr.resize(cnt); u32.resize(cnt);
  for (int i = 0; i < cnt; ++i) {
    const sfista_plan* h = b->plans[i];
    const double inv = 1.0 / (h->L + h->lam * h->lam);
    auto fill = [&](auto& u) {
      u.y[0] = h->Y[0]; u.y[1] = h->Y[1]; u.ldy = h->ldY;
      u.st[0] = h->st[0]; u.st[1] = h->st[1]; u.n = h->n;
      u.c1 = h->L * inv; u.c2 = inv; u.nonneg = h->nonneg; u.beta = b->beta; u.counter = b->counter;
    };
    fill(u64[i]); fill(upr[i]); fill(u32[i]);
  }
}

// Builds the per-product GEMM arguments, epilogues and work lists.
template <int MODE>
int batch_build(sfista_batch* b) {
  const int cnt = b->count;
  std::vector<GemmArgs> args[4];
  std::vector<EpiStack<MODE>> e0(cnt), e2(cnt);
  std::vector<EpiResid<MODE>> e1(cnt);
  std::vector<EpiUpdateSeq<MODE, ST_F64>> u64;
  std::vector<EpiUpdateSeq<MODE, ST_PAIR>> upr;
  std::vector<EpiUpdateSeq<MODE, ST_F32>> u32;
  using Acc = typename ModeTraits<MODE>::Acc;
  for (int i = 0; i < cnt; ++i) {
    sfista_plan* h = b->plans[i];
    const int m = h->m, n = h->n, r = h->r;
    GemmArgs g;
    g = gargs<MODE>(h->W, h->ldW, h->Y, h->ldY, r * n, m, n); args[0].push_back(g);
    g = gargs<MODE>(h->T, h->ldT, h->Bc, h->ldBc, n, m, r * m); args[1].push_back(g);
    g = gargs<MODE>(h->Bt, h->ldBt, h->R, h->ldR, r * m, n, m); args[2].push_back(g);
    g = gargs<MODE>(h->S, h->ldS, h->At, h->ldAt, m, n, r * n); args[3].push_back(g);
    for (int q = 0; q < 4; ++q) args[q].back().kchunk = gemm_kstages<MODE>(args[q].back().K);
    e0[i].out[0] = h->T[0]; e0[i].out[1] = h->T[1]; e0[i].ldo = h->ldT; e0[i].D = n; e0[i].colblk = m;
    e1[i].out[0] = h->R[0]; e1[i].out[1] = h->R[1]; e1[i].ldo = h->ldR;
    e1[i].bobs_t = static_cast<const Acc*>(h->bobs_t); e1[i].m = m; e1[i].copy = nullptr; e1[i].n = n;
    e2[i].out[0] = h->S[0]; e2[i].out[1] = h->S[1]; e2[i].ldo = h->ldS; e2[i].D = m; e2[i].colblk = n;
  }
  fill_update_tables<MODE>(b, u64, upr, u32);
  auto upload = [&](const void* src, size_t bytes) -> void* {
    void* d = b->arena.alloc_zero(bytes, b->s);
    if (d && hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, b->s) != hipSuccess) return nullptr;
    return d;
  };
  for (int q = 0; q < 4; ++q) {
    b->dargs[q] = static_cast<GemmArgs*>(upload(args[q].data(), sizeof(GemmArgs) * cnt));
    if (!b->dargs[q]) return set_error(SFISTA_ERR_NOMEM, "batch allocation failed");
  }
  b->depi[0] = upload(e0.data(), sizeof(e0[0]) * cnt);
  b->depi[1] = upload(e1.data(), sizeof(e1[0]) * cnt);
  b->depi[2] = upload(e2.data(), sizeof(e2[0]) * cnt);
  {   // the power iteration's tables: F2 without Bobs, G2 storing the product
    std::vector<EpiResid<MODE>> p1(e1);
    std::vector<EpiStore<MODE>> p3(cnt);
    for (int i = 0; i < cnt; ++i) {
      p1[i].bobs_t = nullptr;
      p3[i].out = b->plans[i]->aux;
      p3[i].n = b->plans[i]->n;
    }
    b->dpow[0] = upload(p1.data(), sizeof(p1[0]) * cnt);
    b->dpow[1] = upload(p3.data(), sizeof(p3[0]) * cnt);
    if (!b->dpow[0] || !b->dpow[1]) return set_error(SFISTA_ERR_NOMEM, "batch allocation failed");
  }
  if (b->kind == ST_F64) b->depi[3] = upload(u64.data(), sizeof(u64[0]) * cnt);
  else if (b->kind == ST_PAIR) b->depi[3] = upload(upr.data(), sizeof(upr[0]) * cnt);
  else b->depi[3] = upload(u32.data(), sizeof(u32[0]) * cnt);
  if (!b->depi[0] || !b->depi[1] || !b->depi[2] || !b->depi[3]) return set_error(SFISTA_ERR_NOMEM, "batch allocation failed");
  // work lists: problems with the longest K first, tiles of one problem together
  for (int q = 0; q < 4; ++q) {
    std::vector<int> order(cnt);
    for (int i = 0; i < cnt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return args[q][x].K > args[q][y].K; });
    for (int c = 0; c < 3; ++c) {
      using TB = typename BigTile<MODE>::T;
      if (!shape_offered<MODE>(c)) continue;
      const int BM = c == 0 ? TB::BM : c == 1 ? TileS::BM : Tile128::BM;
      const int BN = c == 0 ? TB::BN : c == 1 ? TileS::BN : Tile128::BN;
      std::vector<WorkItem> w;
      for (int i : order) {
        const int tm_n = (args[q][i].M + BM - 1) / BM, tn_n = (args[q][i].N + BN - 1) / BN;
        for (int tm = 0; tm < tm_n; ++tm)
          for (int tn = 0; tn < tn_n; ++tn) w.push_back(WorkItem{i, tm, tn, 0});
      }
      b->nwork[q][c] = (int)w.size();
      b->dwork[q][c] = static_cast<WorkItem*>(upload(w.data(), sizeof(WorkItem) * w.size()));
      if (!b->dwork[q][c]) return set_error(SFISTA_ERR_NOMEM, "batch allocation failed");
    }
  }
  return SFISTA_OK;
}

// ---- batched power iteration: the iteration of run_power for every problem
// at once, the four products as grouped launches, the per-problem norms as
// one launch over all problems (same partial/sum structure as sumsq, so each
// problem's estimate is computed as a lone plan would compute it).
struct PowerImg {
  const double* v0;   // start vector
  double* aux;        // W = A_s^T A_s V, the next V
  double* red;        // the plan's reduction partials [RED_BLOCKS] + scalars
  void* Y[2];         // F1 operand planes
  long ldY;
  int m, n;
};

template <int MODE>
__global__ void pw_planes_kernel(const PowerImg* im, int first) {
  const PowerImg& d = im[blockIdx.y];
  const double* x = first ? d.v0 : d.aux;
  const double scale = 1.0 / sqrt(d.red[RED_BLOCKS]);
  void* p[2] = {d.Y[0], d.Y[1]};
  const int n = d.n;
  const long total = (long)d.m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n, j = e - i * n;
    store_planes<MODE>(p, op_index<MODE>(i, j, d.ldY), x[e] * scale);
  }
}

static __global__ __launch_bounds__(RED_THREADS) void pw_sumsq_partial_kernel(const PowerImg* im, int first) {
  __shared__ double sh[RED_THREADS / 64];
  const PowerImg& d = im[blockIdx.y];
  const double* x = first ? d.v0 : d.aux;
  const long total = (long)d.m * d.n;
  double acc = 0.0;
  for (long e = blockIdx.x * (long)RED_THREADS + threadIdx.x; e < total; e += (long)RED_BLOCKS * RED_THREADS) {
    const double v = x[e];
    acc += v * v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) d.red[blockIdx.x] = t;
}

static __global__ __launch_bounds__(RED_THREADS) void pw_sumsq_finish_kernel(const PowerImg* im, double* ss) {
  __shared__ double sh[RED_THREADS / 64];
  const PowerImg& d = im[blockIdx.y];
  double acc = 0.0;
  for (int e = threadIdx.x; e < RED_BLOCKS; e += RED_THREADS) acc += d.red[e];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    d.red[RED_BLOCKS] = t;
    ss[blockIdx.y] = t;
  }
}

// Estimates L for every problem (steps power steps from each plan's start
// vector) into Lout (host, count entries).
template <int MODE>
hipError_t batch_power(sfista_batch* b, const std::vector<const double*>& v0, int steps, std::vector<double>& Lout) {
  const int cnt = b->count;
  std::vector<PowerImg> im(cnt);
  for (int i = 0; i < cnt; ++i) {
    const sfista_plan* h = b->plans[i];
    im[i] = PowerImg{v0[i], h->aux, h->red, {h->Y[0], h->Y[1]}, h->ldY, h->m, h->n};
  }
  PowerImg* dim = static_cast<PowerImg*>(b->arena.alloc_zero(sizeof(PowerImg) * cnt, b->s));
  double* ss = static_cast<double*>(b->arena.alloc_zero(sizeof(double) * cnt, b->s));
  if (!dim || !ss) return hipErrorOutOfMemory;
  hipError_t e = hipMemcpyAsync(dim, im.data(), sizeof(PowerImg) * cnt, hipMemcpyHostToDevice, b->s);
  if (e != hipSuccess) return e;
  auto norms = [&](int first) {
    hipLaunchKernelGGL(pw_sumsq_partial_kernel, dim3(RED_BLOCKS, cnt), dim3(RED_THREADS), 0, b->s, dim, first);
    hipLaunchKernelGGL(pw_sumsq_finish_kernel, dim3(1, cnt), dim3(RED_THREADS), 0, b->s, dim, ss);
  };
  const dim3 pg(std::max(1, EW_BLOCKS / cnt), cnt);
  norms(1);
  hipLaunchKernelGGL(pw_planes_kernel<MODE>, pg, dim3(EW_THREADS), 0, b->s, dim, 1);
  for (int it = 0; it < steps; ++it) {
    if ((e = launch_product<MODE, EpiStack<MODE>>(b, 0)) != hipSuccess) return e;
    if ((e = launch_product<MODE, EpiResid<MODE>>(b, 1, b->dpow[0])) != hipSuccess) return e;
    if ((e = launch_product<MODE, EpiStack<MODE>>(b, 2)) != hipSuccess) return e;
    if ((e = launch_product<MODE, EpiStore<MODE>>(b, 3, b->dpow[1])) != hipSuccess) return e;
    norms(0);
    if (it + 1 < steps) hipLaunchKernelGGL(pw_planes_kernel<MODE>, pg, dim3(EW_THREADS), 0, b->s, dim, 0);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<double> h(cnt);
  if ((e = hipMemcpyAsync(h.data(), ss, sizeof(double) * cnt, hipMemcpyDeviceToHost, b->s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(b->s)) != hipSuccess) return e;
  Lout.resize(cnt);
  for (int i = 0; i < cnt; ++i) Lout[i] = sqrt(h[i]);
  return hipSuccess;
}

// ---- batched Lanczos: the recurrence of run_lanczos for every problem at
// once (same partial/sum structure per problem as a lone plan).
struct LanczosImg {
  const double* v0;   // start vector
  double* w;          // the plan's aux: A_s^T A_s q_j, then the orthogonalised residual
  double* q[2];       // q_j and q_{j-1} (ping-pong by step parity)
  double* red;        // the plan's reduction partials [RED_BLOCKS] + scalars
  double* coef;       // 2 x steps: alpha_j, beta_j^2
  void* Y[2];         // F1 operand planes
  long ldY;
  int m, n;
};

// which: 0 = ||v0||^2, 1 = <q_cur, w>, 2 = the three-term update of w and ||w||^2
static __global__ __launch_bounds__(RED_THREADS) void lz_partial_kernel(const LanczosImg* im, int which, int cur,
                                                                        int j) {
  __shared__ double sh[RED_THREADS / 64];
  const LanczosImg& d = im[blockIdx.y];
  const long total = (long)d.m * d.n;
  const double* q = d.q[cur];
  const double* qo = d.q[cur ^ 1];
  double a = 0.0, b = 0.0;
  if (which == 2) {
    a = d.coef[2 * j];
    b = j > 0 ? sqrt(d.coef[2 * j - 1]) : 0.0;
  }
  double acc = 0.0;
  for (long e = blockIdx.x * (long)RED_THREADS + threadIdx.x; e < total; e += (long)RED_BLOCKS * RED_THREADS) {
    if (which == 0) {
      const double v = d.v0[e];
      acc += v * v;
    } else if (which == 1) {
      acc += q[e] * d.w[e];
    } else {
      double v = d.w[e] - a * q[e];
      if (j > 0) v -= b * qo[e];
      d.w[e] = v;
      acc += v * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) d.red[blockIdx.x] = t;
}

// Adds the partials in index order into the scalar slot (slot < 0) or coef[slot].
static __global__ __launch_bounds__(RED_THREADS) void lz_finish_kernel(const LanczosImg* im, int slot) {
  __shared__ double sh[RED_THREADS / 64];
  const LanczosImg& d = im[blockIdx.y];
  double acc = 0.0;
  for (int e = threadIdx.x; e < RED_BLOCKS; e += RED_THREADS) acc += d.red[e];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (slot < 0) d.red[RED_BLOCKS] = t;
    else d.coef[slot] = t;
  }
}

// q_dst = src / sqrt(ss) (0 when ss is 0) and the F1 planes of it; src is
// v0 with ss = ||v0||^2 for the start (j < 0), else w with ss = beta_j^2.
template <int MODE>
__global__ void lz_next_kernel(const LanczosImg* im, int dst, int j) {
  const LanczosImg& d = im[blockIdx.y];
  const double* src = j < 0 ? d.v0 : d.w;
  const double ss = j < 0 ? d.red[RED_BLOCKS] : d.coef[2 * j + 1];
  const double scale = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  double* q = d.q[dst];
  void* p[2] = {d.Y[0], d.Y[1]};
  const int n = d.n;
  const long total = (long)d.m * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const double v = src[e] * scale;
    q[e] = v;
    const long i = e / n, c = e - i * n;
    store_planes<MODE>(p, op_index<MODE>(i, c, d.ldY), v);
  }
}

// Estimates L for every problem by `steps` Lanczos steps from each plan's
// start vector into Lout (host, count entries).
template <int MODE>
hipError_t batch_lanczos(sfista_batch* b, const std::vector<const double*>& v0, int steps,
                         std::vector<double>& Lout) {
  const int cnt = b->count;
  std::vector<LanczosImg> im(cnt);
  double* coef = static_cast<double*>(b->arena.alloc_zero(sizeof(double) * 2 * steps * cnt, b->s));
  if (!coef) return hipErrorOutOfMemory;
  for (int i = 0; i < cnt; ++i) {
    sfista_plan* h = b->plans[i];
    const size_t bytes = (size_t)h->m * h->n * 8;
    for (int k = 0; k < 2; ++k)
      if (!h->lzq[k] && !(h->lzq[k] = static_cast<double*>(h->mem->alloc_zero(bytes, b->s))))
        return hipErrorOutOfMemory;
    im[i] = LanczosImg{v0[i], h->aux, {h->lzq[0], h->lzq[1]}, h->red, coef + (size_t)2 * steps * i,
                       {h->Y[0], h->Y[1]}, h->ldY, h->m, h->n};
  }
  LanczosImg* dim = static_cast<LanczosImg*>(b->arena.alloc_zero(sizeof(LanczosImg) * cnt, b->s));
  if (!dim) return hipErrorOutOfMemory;
  hipError_t e = hipMemcpyAsync(dim, im.data(), sizeof(LanczosImg) * cnt, hipMemcpyHostToDevice, b->s);
  if (e != hipSuccess) return e;
  const dim3 rg(RED_BLOCKS, cnt), fg(1, cnt), pg(std::max(1, EW_BLOCKS / cnt), cnt);
  hipLaunchKernelGGL(lz_partial_kernel, rg, dim3(RED_THREADS), 0, b->s, dim, 0, 0, 0);
  hipLaunchKernelGGL(lz_finish_kernel, fg, dim3(RED_THREADS), 0, b->s, dim, -1);
  hipLaunchKernelGGL(lz_next_kernel<MODE>, pg, dim3(EW_THREADS), 0, b->s, dim, 0, -1);
  int cur = 0;
  for (int j = 0; j < steps; ++j) {
    if ((e = launch_product<MODE, EpiStack<MODE>>(b, 0)) != hipSuccess) return e;
    if ((e = launch_product<MODE, EpiResid<MODE>>(b, 1, b->dpow[0])) != hipSuccess) return e;
    if ((e = launch_product<MODE, EpiStack<MODE>>(b, 2)) != hipSuccess) return e;
    if ((e = launch_product<MODE, EpiStore<MODE>>(b, 3, b->dpow[1])) != hipSuccess) return e;
    hipLaunchKernelGGL(lz_partial_kernel, rg, dim3(RED_THREADS), 0, b->s, dim, 1, cur, j);
    hipLaunchKernelGGL(lz_finish_kernel, fg, dim3(RED_THREADS), 0, b->s, dim, 2 * j);
    hipLaunchKernelGGL(lz_partial_kernel, rg, dim3(RED_THREADS), 0, b->s, dim, 2, cur, j);
    hipLaunchKernelGGL(lz_finish_kernel, fg, dim3(RED_THREADS), 0, b->s, dim, 2 * j + 1);
    if (j + 1 < steps) {
      hipLaunchKernelGGL(lz_next_kernel<MODE>, pg, dim3(EW_THREADS), 0, b->s, dim, cur ^ 1, j);
      cur ^= 1;
    }
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<double> hc((size_t)2 * steps * cnt);
  if ((e = hipMemcpyAsync(hc.data(), coef, hc.size() * 8, hipMemcpyDeviceToHost, b->s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(b->s)) != hipSuccess) return e;
  Lout.resize(cnt);
  for (int i = 0; i < cnt; ++i) Lout[i] = lanczos_ritz_max(hc.data() + (size_t)2 * steps * i, steps);
  return hipSuccess;
}

// Times the tile shapes of every product on the batch itself and keeps the
// fastest; the state is reset afterwards.
template <int MODE>
hipError_t batch_autotune(sfista_batch* b) {
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
  for (int q = 0; q < 4; ++q) {
    float best = 1e30f;
    int pick = 0;
    for (int c = 0; c < 3; ++c) {
      if (!shape_offered<MODE>(c)) continue;
      b->choice[q] = c;
      for (int rep = 0; rep < 4; ++rep) {
        if (rep == 1) (void)hipEventRecord(e0, b->s);
        if (q == 0 || q == 2) e = launch_product<MODE, EpiStack<MODE>>(b, q);
        else if (q == 1) e = launch_product<MODE, EpiResid<MODE>>(b, q);
        else if (b->kind == ST_F64) e = launch_product<MODE, EpiUpdateSeq<MODE, ST_F64>>(b, q);
        else if (b->kind == ST_PAIR) e = launch_product<MODE, EpiUpdateSeq<MODE, ST_PAIR>>(b, q);
        else e = launch_product<MODE, EpiUpdateSeq<MODE, ST_F32>>(b, q);
        if (e != hipSuccess) return e;
      }
      (void)hipEventRecord(e1, b->s);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; pick = c; }
    }
    b->choice[q] = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (sfista_plan* h : b->plans)
    hipLaunchKernelGGL(init_state_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, b->s, nullptr, h->st[0],
                       h->st[1], h->kind, h->Y[0], h->Y[1], h->ldY, h->m, h->n);
  return hipGetLastError();
}

std::string batch_key(const sfista_batch* b) {
  std::ostringstream k;
  k << "m" << b->mode << "k" << b->kind;
  for (const sfista_plan* h : b->plans) k << "_" << h->m << "x" << h->n << "r" << h->r;
  std::hash<std::string> hs;
  std::ostringstream o;
  o << std::hex << hs(k.str());
  return o.str();
}

bool tune_cache_lookup(const std::string& key, int* choice) {
  const char* path = getenv("SFISTA_TUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k;
    int c[4];
    if ((ls >> k >> c[0] >> c[1] >> c[2] >> c[3]) && k == key) {
      for (int q = 0; q < 4; ++q) choice[q] = (c[q] >= 0 && c[q] <= 2) ? c[q] : 1;
      return true;
    }
  }
  return false;
}

void tune_cache_store(const std::string& key, const int* choice) {
  const char* path = getenv("SFISTA_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << choice[0] << " " << choice[1] << " " << choice[2] << " " << choice[3] << "\n";
}

// Estimates L for the problems that need it (one batched power iteration),
// then rebuilds the iteration's G2 epilogues and resets every state.
template <int MODE>
int batch_estimate_L(sfista_batch* b) {
  const int cnt = b->count;
  bool any = false;
  for (char c : b->need_L) any = any || c;
  if (!any) return SFISTA_OK;
  std::vector<const double*> v0(cnt);
  for (int i = 0; i < cnt; ++i) {
    sfista_plan* h = b->plans[i];
    // the fixed internal start of a lone plan (same hash, same seed)
    if (!h->v0buf && !(h->v0buf = static_cast<double*>(h->mem->alloc_zero((size_t)h->m * h->n * 8, b->s))))
      return set_error(SFISTA_ERR_NOMEM, "batch allocation failed");
    hipLaunchKernelGGL(hash_fill_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, b->s, h->v0buf, (long)h->m * h->n,
                       0x5f15a7ull);
    v0[i] = h->v0buf;
  }
  std::vector<double> L;
  hipError_t e = b->lanczos ? batch_lanczos<MODE>(b, v0, b->power_steps, L)
                             : batch_power<MODE>(b, v0, b->power_steps, L);
  if (e != hipSuccess) return hip_fail(e, b->lanczos ? "batch Lanczos estimate of L" : "batch power iteration");
  for (int i = 0; i < cnt; ++i) {
    if (!b->need_L[i]) continue;
    if (!isfinite(L[i]) || !(L[i] > 0.0)) return set_error(SFISTA_ERR_NONFINITE, "problem %d: Lipschitz estimate is %g", i, L[i]);
    b->plans[i]->L = L[i];
  }
  std::vector<EpiUpdateSeq<MODE, ST_F64>> u64;
  std::vector<EpiUpdateSeq<MODE, ST_PAIR>> upr;
  std::vector<EpiUpdateSeq<MODE, ST_F32>> u32;
  fill_update_tables<MODE>(b, u64, upr, u32);
  if (b->kind == ST_F64) e = hipMemcpyAsync(b->depi[3], u64.data(), sizeof(u64[0]) * cnt, hipMemcpyHostToDevice, b->s);
  else if (b->kind == ST_PAIR) e = hipMemcpyAsync(b->depi[3], upr.data(), sizeof(upr[0]) * cnt, hipMemcpyHostToDevice, b->s);
  else e = hipMemcpyAsync(b->depi[3], u32.data(), sizeof(u32[0]) * cnt, hipMemcpyHostToDevice, b->s);
  for (sfista_plan* h : b->plans)
    hipLaunchKernelGGL(init_state_kernel<MODE>, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, b->s, nullptr, h->st[0],
                       h->st[1], h->kind, h->Y[0], h->Y[1], h->ldY, h->m, h->n);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(b->s);   // the host tables die here
  if (e != hipSuccess) return hip_fail(e, "batch setup");
  return SFISTA_OK;
}

template <int MODE>
int batch_setup_mode(sfista_batch* b) {
  int rc = batch_build<MODE>(b);
  if (rc != SFISTA_OK) return rc;
  // default shape: the largest tile whose tiles fill the GPU twice over
  int cus = 256, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  const int slots = cus * resident_per_cu<MODE>();
  for (int q = 0; q < 4; ++q)
    b->choice[q] = b->nwork[q][0] >= 2 * slots ? 0 : (shape_offered<MODE>(2) && b->nwork[q][2] >= 2 * cus) ? 2 : 1;
  for (int q = 0; q < 4; ++q)
    if (!shape_offered<MODE>(b->choice[q])) b->choice[q] = 1;
  // a cached choice applies at once, so that the estimate of L already runs
  // on the tuned shapes (shapes do not change results); otherwise the timing
  // waits for L, which the update epilogue of G2 needs
  const bool tune = (b->flags & SFISTA_BATCH_AUTOTUNE) != 0;
  const std::string key = tune ? batch_key(b) : std::string();
  const bool cached = tune && tune_cache_lookup(key, b->choice);
  for (int q = 0; q < 4; ++q)
    if (!shape_offered<MODE>(b->choice[q])) b->choice[q] = 1;   // a cache line from elsewhere
  if ((rc = batch_estimate_L<MODE>(b)) != SFISTA_OK) return rc;
  if (tune && !cached) {
    hipError_t e = batch_autotune<MODE>(b);
    if (e != hipSuccess) return hip_fail(e, "batch autotune");
    tune_cache_store(key, b->choice);
  }
  hipError_t e = hipStreamSynchronize(b->s);
  if (e != hipSuccess) return hip_fail(e, "batch setup");
  return SFISTA_OK;
}

template <int MODE>
hipError_t batch_run(sfista_batch* b, int iters) {
  hipError_t e = hipSuccess;
  int left = iters;
  if ((b->flags & SFISTA_BATCH_GRAPH) && left >= GRAPH_ITERS) {
    if (!b->gexec) {
      if ((e = hipStreamBeginCapture(b->s, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
      for (int i = 0; i < GRAPH_ITERS && e == hipSuccess; ++i) e = batch_iteration<MODE>(b);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->s, &g);
      if (e != hipSuccess) return e;
      if (ec != hipSuccess) return ec;
      b->graph = g;
      if ((e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0)) != hipSuccess) return e;
    }
    while (left >= GRAPH_ITERS) {
      if ((e = hipGraphLaunch(b->gexec, b->s)) != hipSuccess) return e;
      left -= GRAPH_ITERS;
    }
  }
  for (int i = 0; i < left && e == hipSuccess; ++i) e = batch_iteration<MODE>(b);
  return e;
}

}  // namespace

extern "C" {

int sfista_batch_setup(const sfista_batch_item* items, int count, const sfista_params* common, int max_iters,
                       int flags, hipStream_t stream, sfista_batch_handle* out) {
  clear_error();
  if (!out) return set_error(SFISTA_ERR_ARG, "out handle pointer is NULL");
  *out = nullptr;
  if (!items || !common || count < 1) return set_error(SFISTA_ERR_ARG, "items, common and count >= 1 required");
  if (max_iters < 1 || max_iters > (1 << 24)) return set_error(SFISTA_ERR_ARG, "max_iters must lie in [1, 2^24]");
  if (common->precision < SFISTA_FP64 || common->precision > SFISTA_BF16X3)
    return set_error(SFISTA_ERR_UNSUPPORTED, "unknown precision %d", common->precision);
  if (common->x0 || common->v0)
    return set_error(SFISTA_ERR_UNSUPPORTED, "batch problems start from X_0 = 0 and an internal power start");
  for (int i = 0; i < count; ++i) {
    sfista_params p = *common;
    p.lambda = items[i].lambda;
    p.L = items[i].L;
    const int rc = validate_problem(items[i].Bobs, items[i].m, items[i].n, items[i].A, items[i].B, items[i].r, &p);
    if (rc != SFISTA_OK) {
      std::string msg = last_error_slot();
      return set_error(rc, "batch problem %d: %s", i, msg.c_str());
    }
  }
  sfista_batch* b = new (std::nothrow) sfista_batch();
  if (!b) return set_error(SFISTA_ERR_NOMEM, "host allocation failed");
  b->count = count; b->mode = common->precision; b->kind = state_kind(b->mode, common->pair_state);
  b->max_iters = max_iters; b->flags = flags;
  hipError_t e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess || (e = hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking)) != hipSuccess) {
    delete b;
    return hip_fail(e, "batch stream");
  }
  b->lanczos = common->l_estimate == SFISTA_L_LANCZOS ? 1 : 0;
  b->power_steps = common->power_iters > 0 ? common->power_iters : (b->lanczos ? 12 : 30);
  for (int i = 0; i < count; ++i) {
    sfista_params p = *common;
    p.lambda = items[i].lambda;
    // L <= 0: estimated below for all such problems at once; the plan holds
    // a placeholder until then
    b->need_L.push_back(items[i].L > 0.0 ? 0 : 1);
    p.L = items[i].L > 0.0 ? items[i].L : 1.0;
    sfista_handle h = nullptr;
    const int rc =
        plan_create(items[i].Bobs, items[i].m, items[i].n, items[i].A, items[i].B, items[i].r, &p, b->s, &b->arena, &h);
    if (rc != SFISTA_OK) {
      std::string msg = last_error_slot();
      delete b;
      return set_error(rc, "batch problem %d: %s", i, msg.c_str());
    }
    b->plans.push_back(h);
  }
  // momentum table and iteration counter
  std::vector<double> beta(max_iters + 2, 0.0);
  double t = 1.0;
  for (int k = 1; k <= max_iters + 1; ++k) {
    const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
    beta[k] = (t - 1.0) / tn;
    t = tn;
  }
  b->beta = static_cast<double*>(b->arena.alloc_zero(beta.size() * sizeof(double), b->s));
  b->counter = static_cast<int*>(b->arena.alloc_zero(256, b->s));
  if (!b->beta || !b->counter) {
    delete b;
    return set_error(SFISTA_ERR_NOMEM, "batch allocation failed");
  }
  if ((e = hipMemcpyAsync(b->beta, beta.data(), beta.size() * sizeof(double), hipMemcpyHostToDevice, b->s)) != hipSuccess) {
    delete b;
    return hip_fail(e, "batch upload");
  }
  int rc = SFISTA_OK;
  SF_DISPATCH(b->mode, rc = batch_setup_mode<MD>(b));
  if (rc != SFISTA_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return SFISTA_OK;
}

int sfista_batch_solve(sfista_batch_handle b, int iters, double* const* X_out, sfista_report* reps) {
  clear_error();
  if (!b) return set_error(SFISTA_ERR_ARG, "NULL handle");
  if (iters < 0 || b->iter + iters > b->max_iters)
    return set_error(SFISTA_ERR_ARG, "iterations beyond the batch's max_iters (%d)", b->max_iters);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) return hip_fail(e, "event");
  (void)hipEventRecord(e0, b->s);
  SF_DISPATCH(b->mode, e = batch_run<MD>(b, iters));
  (void)hipEventRecord(e1, b->s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "sfista_batch_solve iterations");
  b->iter += iters;
  int status = SFISTA_OK;
  for (int i = 0; i < b->count; ++i) {
    sfista_plan* h = b->plans[i];
    h->iter = b->iter;
    double rr = 0.0, xx = 0.0;
    SF_DISPATCH(h->mode, e = report_mode<MD>(h, &rr, &xx));
    if (e != hipSuccess) return hip_fail(e, "sfista_batch_solve report");
    const long mn = (long)h->m * h->n;
    if (X_out && X_out[i]) {
      hipLaunchKernelGGL(state_to_double_kernel, dim3(EW_BLOCKS), dim3(EW_THREADS), 0, h->s, h->st[h->iter & 1],
                         h->kind, X_out[i], mn);
      if ((e = hipStreamSynchronize(h->s)) != hipSuccess) return hip_fail(e, "copy X");
    }
    const double phi = 0.5 * rr + 0.5 * h->lam * h->lam * xx;
    int st = SFISTA_OK;
    if (!isfinite(phi)) st = status = set_error(SFISTA_ERR_NONFINITE, "problem %d: objective is not finite", i);
    if (reps) {
      reps[i].iters = (int)b->iter;
      reps[i].seconds = ms * 1e-3;
      reps[i].L = h->L;
      reps[i].phi_s = phi;
      reps[i].resid_norm = sqrt(rr);
      reps[i].bobs_norm = h->bobs_norm;
      reps[i].x_norm = sqrt(xx);
      reps[i].resid_rel = h->bobs_norm > 0 ? sqrt(rr) / h->bobs_norm : 0.0;
      reps[i].status = st;
    }
  }
  return status;
}

int sfista_batch_tiles(sfista_batch_handle b, int* choice) {
  clear_error();
  if (!b || !choice) return set_error(SFISTA_ERR_ARG, "NULL argument");
  for (int q = 0; q < 4; ++q) choice[q] = b->choice[q];
  return SFISTA_OK;
}

int sfista_batch_set_tiles(sfista_batch_handle b, const int* choice) {
  clear_error();
  if (!b || !choice) return set_error(SFISTA_ERR_ARG, "NULL argument");
  for (int q = 0; q < 4; ++q) {
    const bool ok = choice[q] >= 0 && choice[q] <= 2 &&
                    (b->mode != M_F64 || choice[q] != 2);   // FP64's big tile is the 128 x 128 one
    if (!ok) return set_error(SFISTA_ERR_ARG, "tile shape %d of product %d is not offered", choice[q], q);
  }
  hipError_t e = hipStreamSynchronize(b->s);
  if (e != hipSuccess) return hip_fail(e, "sfista_batch_set_tiles");
  for (int q = 0; q < 4; ++q) b->choice[q] = choice[q];
  // a captured graph holds the old launch shapes
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return SFISTA_OK;
}

void sfista_batch_destroy(sfista_batch_handle b) { delete b; }

}  // extern "C"
