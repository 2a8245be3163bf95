// Differentiable form: a batch of images, each restored by `iters`
// unrolled iterations of Algorithm 2 (L fixed), and the reverse-mode
// adjoint of that map with respect to every factor entry and lambda.
//
// Every product of an iteration is one grouped launch over the tiles of all
// images (no K splits).  The forward pass and the recomputation of a
// checkpoint segment run the same launches with the same epilogue
// parameters, so the recomputed trajectory is bitwise the forward one.
// C ABI declared in include/sfista.h.
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sfista.h"
#include "gemm.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "util.hpp"

using namespace sf;

namespace {

// Per-image view for the batched element-wise kernels (device copy).
struct DiffImg {
  int m, n;
  double c2;              // 1 / (L + lambda^2)
  double* ck;             // checkpoints: s -> (X_{sC-1}, X_{sC}), 2 m n each
  double* xs;             // segment iterates: slot t = X_{c0-1+t}
  double* ys;             // segment Y_k: slot t = Y_{c0+1+t}
  double* xbar;
  double* yb[3];          // Ybar_j lives in yb[j % 3]
  double* dots;           // <Xbar_k, X_k> at k - 1
  double* red;            // reduction partials
  void* Y[2];             // F1 operand planes of Y
  void* Xop[2];           // F1 operand planes of Gbar
  long ldY;
  void* AB[2];            // gradient operand [Gbar^T | Y^T], n x 2Cm
  long ldAB;
  void *BA[2], *GB[2], *AA[2];
  long ldBA, ldGB, ldAA;
  const double* dX;       // this backward call's d(loss)/d(X_iters)
  double* dA;             // this backward call's outputs
  double* dB;
  double* xout;           // this forward call's X_iters destination (nullable)
};

constexpr int DB = 512;   // blocks per image of the element-wise kernels

// X_{c0-1}, X_{c0} from checkpoint s into xs slots 0 and 1, and
// Y_{c0+1} = X_{c0} + beta (X_{c0} - X_{c0-1}) into ys slot 0 and the Y planes.
template <int MODE>
__global__ void diff_start_kernel(const DiffImg* im, int s, double beta) {
  const DiffImg d = im[blockIdx.y];
  const long mn = (long)d.m * d.n;
  const double* src = d.ck + (long)s * 2 * mn;
  void* p[2] = {d.Y[0], d.Y[1]};
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < mn; e += (long)gridDim.x * blockDim.x) {
    const double xp = src[e], xc = src[mn + e];
    d.xs[e] = xp;
    d.xs[mn + e] = xc;
    const double v = __builtin_fma(beta, xc - xp, xc);   // as in EpiUpd64
    d.ys[e] = v;
    const long i = e / d.n, j = e - i * d.n;
    store_planes<MODE>(p, op_index<MODE>(i, j, d.ldY), v);
  }
}

// xs slots t, t + 1 -> checkpoint s.
static __global__ void diff_save_kernel(const DiffImg* im, int t, int s) {
  const DiffImg d = im[blockIdx.y];
  const long mn = (long)d.m * d.n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < 2 * mn; e += (long)gridDim.x * blockDim.x)
    d.ck[(long)s * 2 * mn + e] = d.xs[(long)t * mn + e];
}

// xs slot t -> X_out.
static __global__ void diff_out_kernel(const DiffImg* im, int t) {
  const DiffImg d = im[blockIdx.y];
  if (!d.xout) return;
  const long mn = (long)d.m * d.n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < mn; e += (long)gridDim.x * blockDim.x)
    d.xout[e] = d.xs[(long)t * mn + e];
}

// The transposing kernels give each thread one column j and a strip of CE
// consecutive rows i (CE = 16 / element size): its reads are coalesced
// across threads along j, and its CE values make one whole 16-byte chunk of
// the transposed operand row j.
template <int MODE>
__device__ __forceinline__ void store_chunk_t(void* const* g, long ld, long row, long k0, const double* v, int cnt) {
  constexpr int CE = 16 / ModeTraits<MODE>::esize;
  if (cnt == CE && k0 % CE == 0) {
    const long idx = op_index<MODE>(row, k0, ld);
    if constexpr (MODE == M_F64) {
      *reinterpret_cast<double2*>(static_cast<double*>(g[0]) + idx) = make_double2(v[0], v[1]);
    } else {
      static_assert(MODE == M_F32, "the differentiable form runs in FP32 or FP64");
      *reinterpret_cast<float4*>(static_cast<float*>(g[0]) + idx) =
          make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    }
  } else {
    for (int q = 0; q < cnt; ++q) store_planes<MODE>(g, op_index<MODE>(row, k0 + q, ld), v[q]);
  }
}

// Y_k^T (ys slot t - 1) into the gradient operand AB at iteration slot
// `slot` (K offset slot * m).
template <int MODE>
__global__ void diff_pack_y_kernel(const DiffImg* im, int t, int slot) {
  constexpr int CE = 16 / ModeTraits<MODE>::esize;
  const DiffImg d = im[blockIdx.y];
  const long koff = (long)slot * d.m;
  const long mn = (long)d.m * d.n;
  const double* y = d.ys + (long)(t - 1) * mn;
  void* g[2] = {d.AB[0], d.AB[1]};
  const long strips = (d.m + CE - 1) / CE;
  for (long u = blockIdx.x * (long)blockDim.x + threadIdx.x; u < strips * d.n; u += (long)gridDim.x * blockDim.x) {
    const long sidx = u / d.n, j = u - sidx * d.n, i0 = sidx * CE;
    const int cnt = (int)(d.m - i0 < CE ? d.m - i0 : CE);
    double v[CE];
    for (int q = 0; q < CE; ++q) v[q] = q < cnt ? y[(i0 + q) * d.n + j] : 0.0;
    store_chunk_t<MODE>(g, d.ldAB, j, koff + i0, v, cnt);
  }
}

// Adjoint of Step 3 and the start of the adjoint of Step 1 at iteration k
// (reverse-mode recursion of the unrolled map):
//   Xbar_k = [k = K] dX + a1 Ybar_{k+1} - a2 Ybar_{k+2},  Gbar = -c2 Xbar_k,
// Gbar into the F1 planes (Xop) and, transposed, into AB at iteration slot
// `slot` (K offset slot * m).
template <int MODE>
__global__ void diff_adjoint_kernel(const DiffImg* im, int k, int last, double a1, double a2, int slot) {
  constexpr int CE = 16 / ModeTraits<MODE>::esize;
  const DiffImg d = im[blockIdx.y];
  const long koff = (long)slot * d.m;
  // the rotating buffers are picked in global memory: a run-time index into
  // the private copy would move that copy to scratch
  const double* yb1 = im[blockIdx.y].yb[(k + 1) % 3];
  const double* yb2 = im[blockIdx.y].yb[(k + 2) % 3];
  void* p[2] = {d.Xop[0], d.Xop[1]};
  void* g[2] = {d.AB[0], d.AB[1]};
  const long strips = (d.m + CE - 1) / CE;
  for (long u = blockIdx.x * (long)blockDim.x + threadIdx.x; u < strips * d.n; u += (long)gridDim.x * blockDim.x) {
    const long sidx = u / d.n, j = u - sidx * d.n, i0 = sidx * CE;
    const int cnt = (int)(d.m - i0 < CE ? d.m - i0 : CE);
    double v[CE];
    for (int q = 0; q < CE; ++q) {
      v[q] = 0.0;
      if (q < cnt) {
        const long e = (i0 + q) * d.n + j;
        double xb = a1 * yb1[e] - a2 * yb2[e];
        if (last) xb += d.dX[e];
        d.xbar[e] = xb;
        const double gb = -d.c2 * xb;
        store_planes<MODE>(p, op_index<MODE>(i0 + q, j, d.ldY), gb);
        v[q] = gb;
      }
    }
    store_chunk_t<MODE>(g, d.ldAB, j, koff + i0, v, cnt);
  }
}

// Deterministic <Xbar_k, X_k> (X_k in xs slot t): fixed partials per image,
// then their sum in index order.
static __global__ __launch_bounds__(RED_THREADS) void diff_dot_partial_kernel(const DiffImg* im, int t) {
  __shared__ double sh[RED_THREADS / 64];
  const DiffImg d = im[blockIdx.y];
  const long mn = (long)d.m * d.n;
  const double* x = d.xs + (long)t * mn;
  double acc = 0.0;
  for (long e = blockIdx.x * (long)RED_THREADS + threadIdx.x; e < mn; e += (long)RED_BLOCKS * RED_THREADS)
    acc += d.xbar[e] * x[e];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) d.red[blockIdx.x] = s;
}

static __global__ __launch_bounds__(RED_THREADS) void diff_dot_sum_kernel(const DiffImg* im, int k) {
  __shared__ double sh[RED_THREADS / 64];
  const DiffImg d = im[blockIdx.y];
  double acc = 0.0;
  for (int e = threadIdx.x; e < RED_BLOCKS; e += RED_THREADS) acc += d.red[e];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) d.dots[k - 1] = s;
}

// Zeroes the Ybar buffers of iterations K + 1 and K + 2 and the gradients.
static __global__ void diff_clear_kernel(const DiffImg* im, int K, int r) {
  const DiffImg d = im[blockIdx.y];
  const long mn = (long)d.m * d.n;
  const long na = (long)r * d.n * d.n, nb = (long)r * d.m * d.m;
  double* y1 = im[blockIdx.y].yb[(K + 1) % 3];
  double* y2 = im[blockIdx.y].yb[(K + 2) % 3];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < std::max(mn, std::max(na, nb));
       e += (long)gridDim.x * blockDim.x) {
    if (e < mn) { y1[e] = 0.0; y2[e] = 0.0; }
    if (e < na) d.dA[e] = 0.0;
    if (e < nb) d.dB[e] = 0.0;
  }
}

// Zeroes K indices [k0, k1) (times the image size factor) of the four
// gradient operands: iteration slots a short segment does not fill.
template <int MODE>
__global__ void diff_zero_slots_kernel(const DiffImg* im, int r, int s0, int s1) {
  const DiffImg d = im[blockIdx.y];
  const long n = d.n, m = d.m;
  struct Op { void* p0; void* p1; long ld, rows, w; };
  const Op ops[4] = {{d.BA[0], d.BA[1], d.ldBA, m, n}, {d.GB[0], d.GB[1], d.ldGB, (long)r * m, n},
                     {d.AA[0], d.AA[1], d.ldAA, (long)r * n, m}, {d.AB[0], d.AB[1], d.ldAB, n, m}};
  for (int q = 0; q < 4; ++q) {
    void* g[2] = {ops[q].p0, ops[q].p1};
    const long k0 = (long)s0 * ops[q].w, k1 = (long)s1 * ops[q].w, w = k1 - k0;
    const long total = ops[q].rows * w;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
      const long row = e / w, kk = k0 + (e - row * w);
      store_planes<MODE>(g, op_index<MODE>(row, kk, ops[q].ld), 0.0);
    }
  }
}

}  // namespace

struct sfista_diff {
  int count = 0, mode = 0, r = 0, iters = 0, ckpt = 0, nseg = 0;
  hipStream_t s = nullptr;
  std::vector<sfista_plan*> plans;
  std::vector<double> lam, L;
  std::vector<double> beta;                 // beta[k], k = 0..iters+1
  std::vector<DiffImg> img;                 // host copy of the per-image views
  DiffImg* dimg = nullptr;
  // grouped products: 0 F1 (Y), 1 F1 (Gbar), 2 F2, 3 G1, 4 G2, 5 dB, 6 dA
  GemmArgs* dargs[7] = {};
  WorkItem* dwork[7] = {};
  int nwork[7] = {};
  int choice[7] = {};                       // 0 = the mode's big tile, 1 = TileS, 2 = Tile128
  void* ep[7] = {};                         // epilogue tables (see diff_build)
  bool forward_done = false;
  DeviceArena arena;
  ~sfista_diff() {
    if (s) (void)hipStreamSynchronize(s);
    for (sfista_plan* p : plans) delete p;
  }
};

namespace {

// Epilogue tables: F1 and F1-adjoint stack the T/U operand, F2 the residual,
// G1 the S/W operand, G2 the update (forward and recomputation, per k) or
// Ybar (adjoint, per k), dB and dA the gradient accumulation.  Entry
// (index, image) sits at index * count + image.
//   ep[0]: EpiStack  index 0 = forward, 1 + t = recomputation slot t
//   ep[1]: EpiStack  index t = adjoint slot t
//   ep[2]: EpiResid  index 0 = forward, 1 + t = recomputation, 1 + C + t = adjoint
//   ep[3]: EpiStack  index 0 = forward, 1 + t = recomputation, 1 + C + t = adjoint
//   ep[4]: EpiUpd64  index k - 1, then EpiYbar after them (see ybar_base)
// The per-iteration update (EpiUpd64) and Ybar (EpiYbar) epilogues: the only
// tables that depend on lambda and L.
template <int MODE>
void fill_step_tables(const sfista_diff* d, std::vector<EpiUpd64<MODE>>& eu, std::vector<EpiYbar<MODE>>& ey) {
  const int cnt = d->count, C = d->ckpt, K = d->iters;
  eu.assign((size_t)K * cnt, EpiUpd64<MODE>{});
  ey.assign((size_t)K * cnt, EpiYbar<MODE>{});
  for (int b = 0; b < cnt; ++b) {
    const sfista_plan* h = d->plans[b];
    const DiffImg& im = d->img[b];
    const int n = h->n;
    const long mn = (long)h->m * n;
    for (int k = 1; k <= K; ++k) {
      const int t = (k - 1) % C + 1;   // position of k in its segment
      EpiUpd64<MODE>& e = eu[(size_t)(k - 1) * cnt + b];
      e.y[0] = h->Y[0]; e.y[1] = h->Y[1]; e.ldy = h->ldY;
      e.yin = im.ys + (long)(t - 1) * mn;
      e.xprev = im.xs + (long)t * mn;
      e.xout = im.xs + (long)(t + 1) * mn;
      e.ynext = im.ys + (long)t * mn;
      e.n = n; e.c1 = d->L[b] / (d->L[b] + d->lam[b] * d->lam[b]); e.c2 = im.c2; e.beta = d->beta[k];
      EpiYbar<MODE>& y = ey[(size_t)(k - 1) * cnt + b];
      y.ybar = im.yb[k % 3]; y.xbar = im.xbar; y.n = n; y.c1 = e.c1;
    }
  }
}

template <int MODE>
int diff_build(sfista_diff* d) {
  using TB = typename BigTile<MODE>::T;
  const int cnt = d->count, C = d->ckpt, K = d->iters, r = d->r;
  hipStream_t s = d->s;
  auto upload = [&](const void* src, size_t bytes) -> void* {
    void* p = d->arena.alloc_zero(bytes, s);
    if (p && hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return nullptr;
    return p;
  };
  std::vector<GemmArgs> args[7];
  for (int b = 0; b < cnt; ++b) {
    sfista_plan* h = d->plans[b];
    const DiffImg& im = d->img[b];
    const int m = h->m, n = h->n;
    void* const ba[2] = {im.BA[0], im.BA[1]};
    void* const gb[2] = {im.GB[0], im.GB[1]};
    void* const aa[2] = {im.AA[0], im.AA[1]};
    void* const ab[2] = {im.AB[0], im.AB[1]};
    args[0].push_back(gargs<MODE>(h->W, h->ldW, h->Y, h->ldY, r * n, m, n));
    args[1].push_back(gargs<MODE>(h->W, h->ldW, h->Xop, h->ldY, r * n, m, n));
    args[2].push_back(gargs<MODE>(h->T, h->ldT, h->Bc, h->ldBc, n, m, r * m));
    args[3].push_back(gargs<MODE>(h->Bt, h->ldBt, h->R, h->ldR, r * m, n, m));
    args[4].push_back(gargs<MODE>(h->S, h->ldS, h->At, h->ldAt, m, n, r * n));
    args[5].push_back(gargs<MODE>(ba, im.ldBA, gb, im.ldGB, m, r * m, 2 * C * n));
    args[6].push_back(gargs<MODE>(aa, im.ldAA, ab, im.ldAB, r * n, n, 2 * C * m));
  }
  int cus = 256, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  const int slots = cus * resident_per_cu<MODE>();
  for (int q = 0; q < 7; ++q) {
    if (!(d->dargs[q] = static_cast<GemmArgs*>(upload(args[q].data(), sizeof(GemmArgs) * cnt))))
      return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
    // the largest tile whose tiles alone fill the GPU twice over: the mode's
    // big tile, then 128 x 128, then 64 x 64
    auto count = [&](int bm, int bn) {
      long t = 0;
      for (const GemmArgs& g : args[q]) t += (long)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
      return t;
    };
    d->choice[q] = count(TB::BM, TB::BN) >= 2L * slots ? 0 : count(Tile128::BM, Tile128::BN) >= 2L * cus ? 2 : 1;
    const int BM = d->choice[q] == 0 ? TB::BM : d->choice[q] == 2 ? Tile128::BM : TileS::BM;
    const int BN = d->choice[q] == 0 ? TB::BN : d->choice[q] == 2 ? Tile128::BN : TileS::BN;
    std::vector<int> order(cnt);
    for (int i = 0; i < cnt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return args[q][x].K > args[q][y].K; });
    std::vector<WorkItem> w;
    for (int i : order)
      for (int tm = 0; tm < (args[q][i].M + BM - 1) / BM; ++tm)
        for (int tn = 0; tn < (args[q][i].N + BN - 1) / BN; ++tn) w.push_back(WorkItem{i, tm, tn, 0});
    d->nwork[q] = (int)w.size();
    if (!(d->dwork[q] = static_cast<WorkItem*>(upload(w.data(), sizeof(WorkItem) * w.size()))))
      return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
  }
  // epilogue tables
  std::vector<EpiStack<MODE>> e0((1 + C) * cnt), e1(C * cnt), e3((1 + 2 * C) * cnt);
  std::vector<EpiResid<MODE>> e2((1 + 2 * C) * cnt);
  std::vector<EpiUpd64<MODE>> eu;
  std::vector<EpiYbar<MODE>> ey;
  for (int b = 0; b < cnt; ++b) {
    sfista_plan* h = d->plans[b];
    const DiffImg& im = d->img[b];
    const int m = h->m, n = h->n;
    const long mn = (long)m * n;
    auto stack = [&](EpiStack<MODE>& e, bool f1) {
      e.out[0] = f1 ? h->T[0] : h->S[0]; e.out[1] = f1 ? h->T[1] : h->S[1];
      e.ldo = f1 ? h->ldT : h->ldS; e.D = f1 ? n : m; e.colblk = f1 ? m : n;
    };
    auto resid = [&](EpiResid<MODE>& e, bool bobs) {
      e.out[0] = h->R[0]; e.out[1] = h->R[1]; e.ldo = h->ldR;
      e.bobs_t = bobs ? static_cast<const typename ModeTraits<MODE>::Acc*>(h->bobs_t) : nullptr;
      e.m = m; e.copy = nullptr; e.n = n;
    };
    stack(e0[b], true);
    stack(e3[b], false);
    resid(e2[b], true);
    for (int t = 0; t < C; ++t) {
      EpiStack<MODE>& f = e0[(1 + t) * cnt + b];        // T_k -> GB slot (2t + 1)
      stack(f, true); f.g[0] = im.GB[0]; f.g[1] = im.GB[1]; f.ldg = im.ldGB; f.koff = (2L * t + 1) * n;
      EpiStack<MODE>& u = e1[t * cnt + b];              // U_k -> GB slot 2t
      stack(u, true); u.g[0] = im.GB[0]; u.g[1] = im.GB[1]; u.ldg = im.ldGB; u.koff = 2L * t * n;
      EpiResid<MODE>& rr = e2[(1 + t) * cnt + b];       // R_k -> BA slot 2t
      resid(rr, true); rr.g[0] = im.BA[0]; rr.g[1] = im.BA[1]; rr.ldg = im.ldBA; rr.koff = 2L * t * n;
      EpiResid<MODE>& ra = e2[(1 + C + t) * cnt + b];   // Rbar_k -> BA slot (2t + 1)
      resid(ra, false); ra.g[0] = im.BA[0]; ra.g[1] = im.BA[1]; ra.ldg = im.ldBA; ra.koff = (2L * t + 1) * n;
      EpiStack<MODE>& sr = e3[(1 + t) * cnt + b];       // S_k -> AA slot 2t
      stack(sr, false); sr.g[0] = im.AA[0]; sr.g[1] = im.AA[1]; sr.ldg = im.ldAA; sr.koff = 2L * t * m;
      EpiStack<MODE>& sa = e3[(1 + C + t) * cnt + b];   // W_k -> AA slot (2t + 1)
      stack(sa, false); sa.g[0] = im.AA[0]; sa.g[1] = im.AA[1]; sa.ldg = im.ldAA; sa.koff = (2L * t + 1) * m;
    }
  }
  fill_step_tables<MODE>(d, eu, ey);
  d->ep[0] = upload(e0.data(), sizeof(e0[0]) * e0.size());
  d->ep[1] = upload(e1.data(), sizeof(e1[0]) * e1.size());
  d->ep[2] = upload(e2.data(), sizeof(e2[0]) * e2.size());
  d->ep[3] = upload(e3.data(), sizeof(e3[0]) * e3.size());
  d->ep[4] = upload(eu.data(), sizeof(eu[0]) * eu.size());
  d->ep[5] = upload(ey.data(), sizeof(ey[0]) * ey.size());
  d->ep[6] = d->arena.alloc_zero(2 * sizeof(EpiAcc64<MODE>) * cnt, s);   // dB then dA, per backward call
  for (int q = 0; q < 7; ++q)
    if (!d->ep[q]) return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "diff setup");
  return SFISTA_OK;
}

template <int MODE, class T, class Epi>
hipError_t grouped(sfista_diff* d, int q, const void* epis) {
  if (d->nwork[q] == 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_grouped_kernel<MODE, T, Epi>), dim3(d->nwork[q]), dim3(T::THREADS), 0, d->s, d->dargs[q],
                     static_cast<const Epi*>(epis), d->dwork[q]);
  return hipGetLastError();
}

template <int MODE, class Epi>
hipError_t product(sfista_diff* d, int q, int table, long index) {
  const void* epis = static_cast<const Epi*>(d->ep[table]) + index * d->count;
  if (d->choice[q] == 2) return grouped<MODE, Tile128, Epi>(d, q, epis);
  return d->choice[q] ? grouped<MODE, TileS, Epi>(d, q, epis)
                      : grouped<MODE, typename BigTile<MODE>::T, Epi>(d, q, epis);
}

// Iteration k of the unrolled map from the segment's Y_k; recomputation
// slot t >= 1 also fills the forward halves of the gradient operands.
template <int MODE>
hipError_t diff_iteration(sfista_diff* d, int k, int t, bool grad) {
  hipError_t e;
  if (grad)
    hipLaunchKernelGGL(diff_pack_y_kernel<MODE>, dim3(DB, d->count), dim3(256), 0, d->s, d->dimg, t, 2 * (t - 1) + 1);
  if ((e = product<MODE, EpiStack<MODE>>(d, 0, 0, grad ? t : 0)) != hipSuccess) return e;
  if ((e = product<MODE, EpiResid<MODE>>(d, 2, 2, grad ? t : 0)) != hipSuccess) return e;
  if ((e = product<MODE, EpiStack<MODE>>(d, 3, 3, grad ? t : 0)) != hipSuccess) return e;
  return product<MODE, EpiUpd64<MODE>>(d, 4, 4, k - 1);
}

// New lambda and L: per-image constants and the tables that hold them.
template <int MODE>
hipError_t diff_refresh_tables(sfista_diff* d) {
  std::vector<EpiUpd64<MODE>> eu;
  std::vector<EpiYbar<MODE>> ey;
  fill_step_tables<MODE>(d, eu, ey);
  hipError_t e = hipMemcpyAsync(d->ep[4], eu.data(), sizeof(eu[0]) * eu.size(), hipMemcpyHostToDevice, d->s);
  if (e == hipSuccess) e = hipMemcpyAsync(d->ep[5], ey.data(), sizeof(ey[0]) * ey.size(), hipMemcpyHostToDevice, d->s);
  if (e == hipSuccess) e = hipStreamSynchronize(d->s);   // the host tables die here
  return e;
}

template <int MODE>
hipError_t diff_forward_mode(sfista_diff* d) {
  hipError_t e;
  const int C = d->ckpt, K = d->iters;
  for (int sg = 0; sg < d->nseg; ++sg) {
    const int c0 = sg * C, c1 = std::min(c0 + C, K);
    hipLaunchKernelGGL(diff_start_kernel<MODE>, dim3(DB, d->count), dim3(256), 0, d->s, d->dimg, sg, d->beta[c0]);
    for (int k = c0 + 1; k <= c1; ++k)
      if ((e = diff_iteration<MODE>(d, k, k - c0, false)) != hipSuccess) return e;
    if (sg + 1 < d->nseg)
      hipLaunchKernelGGL(diff_save_kernel, dim3(DB, d->count), dim3(256), 0, d->s, d->dimg, c1 - c0, sg + 1);
    else
      hipLaunchKernelGGL(diff_out_kernel, dim3(DB, d->count), dim3(256), 0, d->s, d->dimg, c1 - c0 + 1);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(d->s);
}

template <int MODE>
hipError_t diff_backward_mode(sfista_diff* d, double* dlam) {
  hipError_t e;
  const int C = d->ckpt, K = d->iters, cnt = d->count;
  hipLaunchKernelGGL(diff_clear_kernel, dim3(DB, cnt), dim3(256), 0, d->s, d->dimg, K, d->r);
  for (int sg = d->nseg - 1; sg >= 0; --sg) {
    const int c0 = sg * C, c1 = std::min(c0 + C, K), len = c1 - c0;
    hipLaunchKernelGGL(diff_start_kernel<MODE>, dim3(DB, cnt), dim3(256), 0, d->s, d->dimg, sg, d->beta[c0]);
    if (len < C)
      hipLaunchKernelGGL(diff_zero_slots_kernel<MODE>, dim3(DB, cnt), dim3(256), 0, d->s, d->dimg, d->r, 2 * len,
                         2 * C);
    for (int k = c0 + 1; k <= c1; ++k)
      if ((e = diff_iteration<MODE>(d, k, k - c0, true)) != hipSuccess) return e;
    for (int k = c1; k > c0; --k) {
      const int t = k - c0;
      hipLaunchKernelGGL(diff_adjoint_kernel<MODE>, dim3(DB, cnt), dim3(256), 0, d->s, d->dimg, k, k == K ? 1 : 0,
                         1.0 + d->beta[k], d->beta[k + 1], 2 * (t - 1));
      hipLaunchKernelGGL(diff_dot_partial_kernel, dim3(RED_BLOCKS, cnt), dim3(RED_THREADS), 0, d->s, d->dimg, t + 1);
      hipLaunchKernelGGL(diff_dot_sum_kernel, dim3(1, cnt), dim3(RED_THREADS), 0, d->s, d->dimg, k);
      if ((e = product<MODE, EpiStack<MODE>>(d, 1, 1, t - 1)) != hipSuccess) return e;        // U = Gbar A^T
      if ((e = product<MODE, EpiResid<MODE>>(d, 2, 2, 1 + C + (t - 1))) != hipSuccess) return e;   // Rbar
      if ((e = product<MODE, EpiStack<MODE>>(d, 3, 3, 1 + C + (t - 1))) != hipSuccess) return e;   // W = B^T Rbar
      if ((e = product<MODE, EpiYbar<MODE>>(d, 4, 5, k - 1)) != hipSuccess) return e;          // Ybar_k
    }
    if ((e = product<MODE, EpiAcc64<MODE>>(d, 5, 6, 0)) != hipSuccess) return e;   // dB of the segment
    if ((e = product<MODE, EpiAcc64<MODE>>(d, 6, 6, 1)) != hipSuccess) return e;   // dA of the segment
  }
  std::vector<double> dots((size_t)K);
  for (int b = 0; b < cnt; ++b) {
    if ((e = hipMemcpyAsync(dots.data(), d->img[b].dots, sizeof(double) * K, hipMemcpyDeviceToHost, d->s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(d->s)) != hipSuccess) return e;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += dots[k];
    dlam[b] = acc * (-2.0 * d->lam[b] / (d->L[b] + d->lam[b] * d->lam[b]));
  }
  return hipSuccess;
}

template <int MODE>
int diff_setup_mode(sfista_diff* d) {
  constexpr int P = ModeTraits<MODE>::planes;
  constexpr int es = ModeTraits<MODE>::esize;
  const int C = d->ckpt, cnt = d->count, r = d->r;
  hipStream_t s = d->s;
  d->img.resize(cnt);
  for (int b = 0; b < cnt; ++b) {
    sfista_plan* h = d->plans[b];
    DiffImg& im = d->img[b];
    const int m = h->m, n = h->n;
    const long mn = (long)m * n;
    auto dbl = [&](size_t c) { return static_cast<double*>(d->arena.alloc_zero(c * sizeof(double), s)); };
    im.m = m; im.n = n;
    im.c2 = 1.0 / (d->L[b] + d->lam[b] * d->lam[b]);
    im.ck = dbl((size_t)d->nseg * 2 * mn);
    im.xs = dbl((size_t)(C + 2) * mn);
    im.ys = dbl((size_t)(C + 1) * mn);
    im.xbar = dbl(mn);
    for (int q = 0; q < 3; ++q) im.yb[q] = dbl(mn);
    im.dots = dbl((size_t)d->iters + 1);
    im.red = h->red;
    im.Y[0] = h->Y[0]; im.Y[1] = h->Y[1]; im.ldY = h->ldY;
    im.Xop[0] = h->Xop[0]; im.Xop[1] = h->Xop[1];
    im.ldBA = ld_of(2L * C * n); im.ldGB = ld_of(2L * C * n); im.ldAA = ld_of(2L * C * m); im.ldAB = ld_of(2L * C * m);
    auto planes = [&](void** dst, long rows, long ld) -> bool {
      for (int q = 0; q < P; ++q)
        if (!(dst[q] = d->arena.alloc_zero((size_t)rows_of(rows) * ld * es, s))) return false;
      if (P == 1) dst[1] = nullptr;
      return true;
    };
    if (!im.ck || !im.xs || !im.ys || !im.xbar || !im.yb[0] || !im.yb[1] || !im.yb[2] || !im.dots ||
        !planes(im.BA, m, im.ldBA) || !planes(im.GB, (long)r * m, im.ldGB) || !planes(im.AA, (long)r * n, im.ldAA) ||
        !planes(im.AB, n, im.ldAB))
      return set_error(SFISTA_ERR_NOMEM, "device allocation failed (%s)", d->arena.last_error());
    im.dX = nullptr; im.dA = nullptr; im.dB = nullptr; im.xout = nullptr;
  }
  d->dimg = static_cast<DiffImg*>(d->arena.alloc_zero(sizeof(DiffImg) * cnt, s));
  if (!d->dimg) return set_error(SFISTA_ERR_NOMEM, "device allocation failed");
  if (hipMemcpyAsync(d->dimg, d->img.data(), sizeof(DiffImg) * cnt, hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(SFISTA_ERR_HIP, "upload failed");
  return diff_build<MODE>(d);
}

hipError_t upload_views(sfista_diff* d) {
  return hipMemcpyAsync(d->dimg, d->img.data(), sizeof(DiffImg) * d->count, hipMemcpyHostToDevice, d->s);
}

}  // namespace

extern "C" {

int sfista_diff_setup(const sfista_batch_item* items, int count, int precision, int iters, int ckpt_every,
                      hipStream_t stream, sfista_diff_handle* out) {
  clear_error();
  if (!out) return set_error(SFISTA_ERR_ARG, "out handle pointer is NULL");
  *out = nullptr;
  if (!items || count < 1) return set_error(SFISTA_ERR_ARG, "items and count >= 1 required");
  if (precision != SFISTA_FP32 && precision != SFISTA_FP64)
    return set_error(SFISTA_ERR_UNSUPPORTED, "the differentiable form runs in FP32 or FP64 (got %d)", precision);
  if (iters < 1 || iters > (1 << 20) || ckpt_every < 1)
    return set_error(SFISTA_ERR_ARG, "iters must lie in [1, 2^20] and ckpt_every be >= 1");
  if (ckpt_every > iters) ckpt_every = iters;
  for (int i = 0; i < count; ++i) {
    sfista_params p{};
    p.lambda = items[i].lambda; p.L = items[i].L; p.precision = precision; p.power_iters = 30;
    const int rc = validate_problem(items[i].Bobs, items[i].m, items[i].n, items[i].A, items[i].B, items[i].r, &p);
    if (rc != SFISTA_OK) {
      std::string msg = last_error_slot();
      return set_error(rc, "problem %d: %s", i, msg.c_str());
    }
    if (items[i].r != items[0].r)
      return set_error(SFISTA_ERR_UNSUPPORTED, "all problems of one differentiable batch share the rank r");
  }
  sfista_diff* d = new (std::nothrow) sfista_diff();
  if (!d) return set_error(SFISTA_ERR_NOMEM, "host allocation failed");
  d->count = count; d->mode = precision; d->r = items[0].r; d->iters = iters; d->ckpt = ckpt_every;
  d->nseg = (iters + ckpt_every - 1) / ckpt_every;
  d->s = stream;
  for (int i = 0; i < count; ++i) {
    sfista_params p{};
    p.lambda = items[i].lambda; p.L = items[i].L; p.precision = precision; p.power_iters = 30; p.pair_state = 0;
    sfista_handle h = nullptr;
    const int rc =
        plan_create(items[i].Bobs, items[i].m, items[i].n, items[i].A, items[i].B, items[i].r, &p, stream, &d->arena, &h);
    if (rc != SFISTA_OK) {
      std::string msg = last_error_slot();
      delete d;
      return set_error(rc, "problem %d: %s", i, msg.c_str());
    }
    d->plans.push_back(h);
    d->lam.push_back(items[i].lambda);
    d->L.push_back(h->L);
  }
  d->beta.assign(iters + 2, 0.0);
  double t = 1.0;
  for (int k = 1; k <= iters + 1; ++k) {
    const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
    d->beta[k] = (t - 1.0) / tn;
    t = tn;
  }
  const int rc = precision == SFISTA_FP64 ? diff_setup_mode<M_F64>(d) : diff_setup_mode<M_F32>(d);
  if (rc != SFISTA_OK) {
    delete d;
    return rc;
  }
  *out = d;
  return SFISTA_OK;
}

int sfista_diff_update(sfista_diff_handle d, const sfista_batch_item* items, int count) {
  clear_error();
  if (!d || !items) return set_error(SFISTA_ERR_ARG, "NULL argument");
  if (count != d->count) return set_error(SFISTA_ERR_ARG, "count %d differs from the handle's %d", count, d->count);
  for (int i = 0; i < count; ++i) {
    const sfista_plan* h = d->plans[i];
    if (items[i].m != h->m || items[i].n != h->n || items[i].r != h->r)
      return set_error(SFISTA_ERR_ARG, "problem %d: size %d x %d, rank %d differ from the handle's %d x %d, %d", i,
                       items[i].m, items[i].n, items[i].r, h->m, h->n, h->r);
    sfista_params p{};
    p.lambda = items[i].lambda; p.L = items[i].L; p.precision = d->mode; p.power_iters = 30;
    const int rc = validate_problem(items[i].Bobs, items[i].m, items[i].n, items[i].A, items[i].B, items[i].r, &p);
    if (rc != SFISTA_OK) {
      std::string msg = last_error_slot();
      return set_error(rc, "problem %d: %s", i, msg.c_str());
    }
  }
  d->forward_done = false;
  for (int i = 0; i < count; ++i) {
    sfista_plan* h = d->plans[i];
    const int rc = plan_refresh(h, items[i].Bobs, items[i].A, items[i].B, items[i].lambda, items[i].L);
    if (rc != SFISTA_OK) {
      std::string msg = last_error_slot();
      return set_error(rc, "problem %d: %s", i, msg.c_str());
    }
    d->lam[i] = items[i].lambda;
    d->L[i] = h->L;
    d->img[i].c2 = 1.0 / (h->L + items[i].lambda * items[i].lambda);
  }
  const hipError_t e = d->mode == M_F64 ? diff_refresh_tables<M_F64>(d) : diff_refresh_tables<M_F32>(d);
  if (e != hipSuccess) return hip_fail(e, "sfista_diff_update");
  return SFISTA_OK;
}

int sfista_diff_forward(sfista_diff_handle d, double* const* X_out) {
  clear_error();
  if (!d) return set_error(SFISTA_ERR_ARG, "NULL handle");
  for (int b = 0; b < d->count; ++b) d->img[b].xout = X_out ? X_out[b] : nullptr;
  hipError_t e = upload_views(d);
  if (e == hipSuccess) e = d->mode == M_F64 ? diff_forward_mode<M_F64>(d) : diff_forward_mode<M_F32>(d);
  if (e != hipSuccess) return hip_fail(e, "sfista_diff_forward");
  d->forward_done = true;
  return SFISTA_OK;
}

int sfista_diff_backward(sfista_diff_handle d, const double* const* dX, double* const* dA, double* const* dB,
                         double* dlambda) {
  clear_error();
  if (!d || !dX || !dA || !dB || !dlambda) return set_error(SFISTA_ERR_ARG, "NULL argument");
  if (!d->forward_done) return set_error(SFISTA_ERR_ARG, "sfista_diff_backward needs a forward pass first");
  for (int b = 0; b < d->count; ++b) {
    if (!dX[b] || !dA[b] || !dB[b]) return set_error(SFISTA_ERR_ARG, "NULL gradient buffer for problem %d", b);
    d->img[b].dX = dX[b]; d->img[b].dA = dA[b]; d->img[b].dB = dB[b];
  }
  hipError_t e = upload_views(d);
  if (e == hipSuccess) {
    // gradient epilogues of this call: dB (table index 0) and dA (index 1)
    const int cnt = d->count;
    if (d->mode == M_F64) {
      std::vector<EpiAcc64<M_F64>> g(2 * cnt);
      for (int b = 0; b < cnt; ++b) {
        const int m = d->img[b].m, n = d->img[b].n;
        g[b] = EpiAcc64<M_F64>{dB[b], m, (long)m * m, m};
        g[cnt + b] = EpiAcc64<M_F64>{dA[b], n, n, n};
      }
      e = hipMemcpyAsync(d->ep[6], g.data(), sizeof(g[0]) * g.size(), hipMemcpyHostToDevice, d->s);
      if (e == hipSuccess) e = diff_backward_mode<M_F64>(d, dlambda);
    } else {
      std::vector<EpiAcc64<M_F32>> g(2 * cnt);
      for (int b = 0; b < cnt; ++b) {
        const int m = d->img[b].m, n = d->img[b].n;
        g[b] = EpiAcc64<M_F32>{dB[b], m, (long)m * m, m};
        g[cnt + b] = EpiAcc64<M_F32>{dA[b], n, n, n};
      }
      e = hipMemcpyAsync(d->ep[6], g.data(), sizeof(g[0]) * g.size(), hipMemcpyHostToDevice, d->s);
      if (e == hipSuccess) e = diff_backward_mode<M_F32>(d, dlambda);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "sfista_diff_backward");
  for (int b = 0; b < d->count; ++b)
    if (!isfinite(dlambda[b])) return set_error(SFISTA_ERR_NONFINITE, "lambda gradient of problem %d is not finite", b);
  return SFISTA_OK;
}

int sfista_diff_get_L(sfista_diff_handle d, double* L) {
  clear_error();
  if (!d || !L) return set_error(SFISTA_ERR_ARG, "NULL argument");
  for (int b = 0; b < d->count; ++b) L[b] = d->L[b];
  return SFISTA_OK;
}

void sfista_diff_destroy(sfista_diff_handle d) { delete d; }

}  // extern "C"
