/*
 * sfista.h -- C ABI of the MI355X (gfx950) structured-FISTA library.
 *
 * The library solves the Tikhonov-regularised image-restoration problem of
 * Chen, Nagy, Xi and Yu, "Structured FISTA for Image Restoration", in its
 * matrix form (Section 1, "matrix minimization model"):
 *
 *     min_X  1/2 || sum_k B_k X A_k^T - Bobs ||_F^2  +  lambda^2/2 ||X||_F^2
 *
 * where the blur matrix is approximated by a sum of r Kronecker products,
 * A ~ A_s = sum_k A_k (x) B_k (Section 2; the paper writes K_i for the right
 * factor A_k and H_i for the left factor B_k, and s for r).
 *
 * Conventions for every call:
 *   - images, PSFs and factors are row-major: X[i*n + j], i the row (0..m-1);
 *     the PSF has the same orientation as the image;
 *   - A holds r right factors A_k (n x n) back to back, B holds r left factors
 *     B_k (m x m) back to back, each row-major;
 *   - pointers marked (device) are HIP device memory, (host) host memory;
 *     the caller owns every buffer it passes; the library never frees them;
 *   - calls return SFISTA_OK (0) or a negative sfista_status; no exception or
 *     abort crosses the ABI; sfista_last_error() gives a message for the
 *     calling thread's last failure;
 *   - arguments are validated on the host before any device work starts;
 *   - the library's own device buffers come from a memory pool of its own,
 *     one per device; freed buffers stay cached there (at most 8 GiB per
 *     device) for the next handle until sfista_release_cached() is called.
 */
#ifndef SFISTA_H
#define SFISTA_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFISTA_OK = 0,
    SFISTA_ERR_ARG = -1,          /* invalid argument (null pointer, size, range) */
    SFISTA_ERR_UNSUPPORTED = -2,  /* valid but not supported (unknown mode, size too large) */
    SFISTA_ERR_NOMEM = -3,        /* device allocation failed */
    SFISTA_ERR_HIP = -4,          /* a HIP runtime call failed */
    SFISTA_ERR_NONFINITE = -5     /* a final norm or the Lipschitz estimate is not finite */
} sfista_status;

/* Boundary condition of the blur (Section 2).  The periodic boundary is
 * excluded by the paper and not offered. */
typedef enum { SFISTA_BC_ZERO = 0, SFISTA_BC_REFLEXIVE = 1 } sfista_bc;

/* Arithmetic of the four GEMMs of one iteration.
 *   FP64   : FP64 MFMA, FP64 iterate state.
 *   FP32   : FP32 MFMA, FP32 accumulation.
 *   BF16   : BF16 MFMA, FP32 accumulation (operands rounded to bf16).
 *   FP16   : FP16 MFMA, FP32 accumulation (operands rounded to fp16).
 *   BF16X3 : every operand split as hi + lo in bf16; the product is
 *            a_hi b_hi + a_hi b_lo + a_lo b_hi on BF16 MFMA, FP32 accumulation.
 * Non-FP64 modes keep the iterate state in FP32 or float-float (pair_state). */
typedef enum {
    SFISTA_FP64 = 0, SFISTA_FP32 = 1, SFISTA_BF16 = 2, SFISTA_FP16 = 3, SFISTA_BF16X3 = 4
} sfista_precision;

/* Estimate of L = lambda_max(A_s^T A_s) when the caller gives none.
 *   SFISTA_L_POWER    power iteration: V <- A_s^T A_s V / ||V||, L = ||A_s^T A_s V||
 *                     for the last unit V (converges from below).
 *   SFISTA_L_LANCZOS  symmetric Lanczos on A_s^T A_s without reorthogonalisation
 *                     (Section 4 takes L from a Lanczos estimate of the norm): L is
 *                     the largest eigenvalue of the tridiagonal matrix of the
 *                     recurrence (bisection on the host), cut at the first
 *                     vanishing off-diagonal; also from below, and on blur
 *                     operators far closer than the same number of power steps
 *                     (a Krylov space's best Rayleigh quotient).
 * Both start from v0 (or the internal start) and run in the plan's precision,
 * with FP64 vectors, inner products and norms. */
typedef enum {
    SFISTA_L_POWER = 0,
    SFISTA_L_LANCZOS = 1
} sfista_l_estimate;

typedef struct {
    double lambda;       /* Tikhonov parameter, finite and >= 0 (Section 1) */
    double L;            /* Lipschitz constant of the data term, lambda_max(A_s^T A_s)
                            (Algorithm 2's input); <= 0 asks the library to estimate it
                            (see l_estimate) */
    int precision;       /* sfista_precision */
    int nonneg;          /* 1: project every iterate on X >= 0 (the constraint of
                            Section 1); 0: Algorithm 2 as printed */
    int power_iters;     /* steps of the estimate of L when L <= 0; 0 selects 30 power
                            steps or 12 Lanczos steps */
    int pair_state;      /* non-FP64 modes: 1 keeps X in float-float (hi + lo fp32),
                            0 in plain fp32; ignored in FP64 mode */
    const double* x0;    /* (device) m x n initial point X_0, or NULL for X_0 = 0 */
    const double* v0;    /* (device) m x n start of the estimate of L, or NULL for a
                            fixed internal start */
    int l_estimate;      /* sfista_l_estimate: how L is estimated when L <= 0 (the
                            single-image GEMM and FFT forms and the batched form;
                            the differentiable form takes no params and uses
                            the power iteration) */
} sfista_params;

typedef struct {
    int iters;           /* iterations completed by the plan so far */
    double seconds;      /* device time of the iterations run by this solve call */
    double L;            /* Lipschitz constant in use */
    double phi_s;        /* 1/2||A_s x - b||^2 + lambda^2/2||x||^2 at the returned X (FP64 sums) */
    double resid_norm;   /* ||sum_k B_k X A_k^T - Bobs||_F */
    double bobs_norm;    /* ||Bobs||_F */
    double x_norm;       /* ||X||_F */
    double resid_rel;    /* resid_norm / bobs_norm (gamma of Section 4, for A_s) */
    int status;          /* sfista_status of the solve */
} sfista_report;

typedef struct sfista_plan* sfista_handle;

/* Kronecker approximation of the blur (Section 2, Theorem 1).
 *   P      (device) m x n FP64 PSF, peak at the 0-based centre (l, q).
 *   bc     sfista_bc.
 *   r      number of Kronecker terms, 1 <= r <= min(m, n).
 *   A      (device, out) r x n x n FP64 right factors (Toeplitz for the zero
 *          boundary, Toeplitz + Hankel for the reflexive one).
 *   B      (device, out) r x m x m FP64 left factors.
 *   sigma  (host, out, nullable) the r largest singular values of the weighted
 *          PSF P_bar of Theorem 1.
 *   eps_s  (host, out, nullable) ||P_bar - sum_{k<=r} sigma_k u_k v_k^T||_F, which
 *          equals ||A - A_s||_F by Theorem 1.
 * The left factor B_k is built from the left singular vector u_k and the row
 * centre l, the right factor A_k from v_k and the column centre q.  Signs are
 * fixed so that the largest-magnitude entry of u_k is positive.  All device
 * work is FP64 on `stream`; the call synchronises the stream before returning. */
int kron_approx(const double* P, int m, int n, int l, int q, int bc, int r,
                double* A, double* B, double* sigma, double* eps_s, hipStream_t stream);

/* Kronecker approximations of `count` PSFs in one call (Section 2, Theorem 1
 * for each; the setup of a batch of images).  Every argument of kron_approx
 * becomes a host array of `count` entries: P[i] (device) m[i] x n[i], centre
 * (l[i], q[i]), bc[i], r[i], and the outputs A[i] (device) r[i] x n[i] x n[i]
 * and B[i] (device) r[i] x m[i] x m[i].
 *   sigma  (host, out, nullable) the singular values, packed: image i's r[i]
 *          values start at entry r[0] + ... + r[i-1].
 *   eps_s  (host, out, nullable) count entries.
 * Every image is checked as kron_approx checks it before any work is queued
 * (the message names the image).  Each image's kernels are those of
 * kron_approx, queued on one of up to sixteen internal streams of default
 * priority so that several images run at once; they start after the work
 * already queued on `stream`, and the call synchronises `stream` before
 * returning.  Results equal kron_approx's bit for bit. */
int kron_approx_batch(int count, const double* const* P, const int* m, const int* n, const int* l, const int* q,
                      const int* bc, const int* r, double* const* A, double* const* B, double* sigma,
                      double* eps_s, hipStream_t stream);

/* The same approximation, returned as its generator vectors instead of dense
 * factors (Section 2): h (device, out) r x m and k (device, out) r x n, FP64,
 * with B_k = toep(h_k, l + 1) [+ hank(h_k, l + 1)] and A_k = toep(k_k, q + 1)
 * [+ hank(k_k, q + 1)] in the paper's 1-based notation (Hankel part for the
 * reflexive boundary), so that kron_approx's factors are their expansions.  Arguments, checks, sigma and
 * eps_s as in kron_approx. */
int kron_generators(const double* P, int m, int n, int l, int q, int bc, int r,
                    double* h, double* k, double* sigma, double* eps_s, hipStream_t stream);

/* Build a solver plan for Algorithm 2 (sFISTA).
 *   Bobs   (device) m x n FP64 observed image.
 *   A, B   (device) dense factors as produced by kron_approx (any real factors
 *          are accepted).
 *   p      (host) parameters; p->L <= 0 runs the power iteration.
 *   out    (host, out) the new handle.
 * The plan allocates and owns its device buffers, packs the factors into the
 * operand layouts of its GEMMs, sets X_0 and synchronises `stream`, so the
 * caller may free its inputs afterwards.  All later work of the plan runs on
 * `stream`. */
int sfista_setup(const double* Bobs, int m, int n, const double* A, const double* B, int r,
                 const sfista_params* p, hipStream_t stream, sfista_handle* out);

/* Run `iters` more iterations of Algorithm 2 (Steps 1-3 each), asynchronously
 * on the plan's stream, with no host synchronisation.  The iteration count
 * and the momentum sequence t_k continue from the previous call, so
 * step(a) followed by step(b) equals step(a + b). */
int sfista_step(sfista_handle h, int iters);

/* Run up to `max_iters` more iterations, then evaluate the final report.
 * tol > 0 stops early once ||X_k - X_{k-1}||_F <= tol ||X_k||_F (checked every
 * 10 iterations; the paper stops after a fixed count, tol = 0).
 *   X_out (device, out, nullable) m x n FP64 copy of the current iterate.
 *   rep   (host, out, nullable) report.
 * Synchronous: returns after the stream has drained. */
int sfista_solve(sfista_handle h, int max_iters, double tol, double* X_out, sfista_report* rep);

/* Apply the approximate blur and its normal operator with the plan's GEMMs
 * and precision (Section 1, "matrix equation"; Theorem 3's proof):
 *   AX  (device, out, nullable) m x n FP64: sum_k B_k X A_k^T
 *   AtAX(device, out, nullable) m x n FP64: sum_j B_j^T (sum_k B_k X A_k^T) A_j
 * X (device) m x n FP64.  Does not touch the iterate state.  Synchronous. */
int sfista_apply(sfista_handle h, const double* X, double* AX, double* AtAX);

/* Per-kernel timing of the iteration's four GEMMs (F1: T_k = Y A_k^T,
 * F2: R = sum_k B_k T_k - Bobs, G1: S_k = B_k^T R, G2: sum_k S_k A_k with the
 * fused update).  With every = k >= 1 the GEMM launches of every k-th
 * iteration of sfista_step / sfista_solve (those begun after a multiple of k
 * completed iterations) are bracketed by HIP events on the plan's stream;
 * every = 1 times them all, 0 turns timing off, a negative value is an
 * argument error.  Each event leaves a gap of a few microseconds before the
 * next kernel, so a sample (k = 10, say) disturbs the run less.
 * sfista_kernel_times synchronises the stream and returns, per GEMM, the
 * mean device time in milliseconds (avg_ms, host, 8 entries) and the number
 * of timed launches (launches, host, 8 entries): index 0..3 = the GEMM kernel
 * of F1, F2, G1, G2; index 4..7 = the reduction of their K-split tiles
 * (0 when a product has none).  The samples are then cleared. */
int sfista_set_timing(sfista_handle h, int every);
int sfista_kernel_times(sfista_handle h, double* avg_ms, long* launches);

/* ------------------------------------------------------------------------
 * Batched form: many independent problems of Algorithm 2 (each with its own
 * image size, factors, rank, lambda and L) advanced together.  Each of the
 * four products of an iteration is one grouped launch over the tiles of all
 * problems; the momentum weights come from a device table indexed by a device
 * iteration counter, so a chunk of iterations can be captured once as a HIP
 * graph and replayed.  The batch runs on an internal stream of its own.
 * ------------------------------------------------------------------------ */
typedef struct {
    const double* Bobs;  /* (device) m x n observed image */
    int m, n;            /* image size */
    const double* A;     /* (device) r x n x n right factors */
    const double* B;     /* (device) r x m x m left factors */
    int r;               /* Kronecker terms */
    double lambda;       /* Tikhonov parameter, finite and >= 0 */
    double L;            /* Lipschitz constant; <= 0 runs the power iteration */
} sfista_batch_item;

typedef struct sfista_batch* sfista_batch_handle;

#define SFISTA_BATCH_AUTOTUNE 1  /* time the candidate tile shapes of each product at setup */
#define SFISTA_BATCH_GRAPH 2     /* replay chunks of 10 iterations from a captured HIP graph */

/* Build a batch of `count` problems.  `common` (host) supplies precision,
 * nonneg, power_iters, l_estimate and pair_state for all of them (its lambda
 * and L are ignored; x0 and v0 must be NULL: every problem starts from
 * X_0 = 0 and estimates L, when its item's L <= 0, from a lone plan's
 * internal start, all such problems together).  `max_iters` bounds the
 * iterations the batch may run (the size of its momentum table).  `flags`
 * is a mask of SFISTA_BATCH_*.  With SFISTA_BATCH_AUTOTUNE the choice of tile
 * shape per product is cached in the file named by the environment variable
 * SFISTA_TUNE_CACHE when it is set.  Inputs may be freed after the call. */
int sfista_batch_setup(const sfista_batch_item* items, int count, const sfista_params* common, int max_iters,
                       int flags, hipStream_t stream, sfista_batch_handle* out);

/* Run `iters` more iterations of every problem, then write the reports.
 *   X_out (host array of `count` device pointers, nullable; entries nullable)
 *         receives each problem's m x n FP64 iterate.
 *   reps  (host, `count` entries, nullable).
 * Synchronous. */
int sfista_batch_solve(sfista_batch_handle h, int iters, double* const* X_out, sfista_report* reps);

/* Tile shape chosen per product (host, 4 entries: F1, F2, G1, G2): 0 = the
 * mode's large tile (256 x 256, 8 waves; 128 x 128 in FP64), 1 = 64 x 64
 * tiles of 4 waves, 2 = 128 x 128 tiles of 8 waves (not in FP64). */
int sfista_batch_tiles(sfista_batch_handle h, int* choice);

/* Pin the tile shape of each product (host, 4 entries, codes as above; 2 is
 * refused in FP64).  The iterates do not depend on the shapes (every tile
 * takes the whole K in the same order).  Drops a captured graph, which is
 * captured again at the next solve.  Synchronises the batch's stream. */
int sfista_batch_set_tiles(sfista_batch_handle h, const int* choice);

void sfista_batch_destroy(sfista_batch_handle h);

/* ---------------------------------------------------------------------
 * Differentiable form: the unrolled iteration as a function of the factors
 * and lambda, and its reverse-mode adjoint.
 *
 * The forward pass runs `iters` unconstrained iterations of Algorithm 2 from
 * X_0 = 0 with L held fixed (a constant of the map, not differentiated) and
 * keeps (X_{c-1}, X_c) every `ckpt_every` iterations.  The backward pass
 * takes dX = d(loss)/d(X_iters) and returns the gradient with respect to
 * every entry of the dense factors A (r x n x n) and B (r x m x m) and to
 * lambda: it recomputes one checkpoint segment at a time and runs the adjoint
 * of Step 3 (momentum), of Step 1 (the normal-operator products, reusing the
 * GEMMs of the forward shapes) and the factor-gradient products
 *   dB_j += sum_k R_k (G~_k A_j^T)^T + Rbar_k (Y_k A_j^T)^T,
 *   dA_j += sum_k (B_j^T R_k)^T G~_k + (B_j^T Rbar_k)^T Y_k,
 * with G~_k = -Xbar_k / (L + lambda^2) and Rbar_k = A_s(G~_k), as two GEMMs
 * per segment whose K dimension runs over the segment's iterations.
 *
 * precision: SFISTA_FP32 (FP32 MFMA, FP32 accumulation) or SFISTA_FP64;
 * iterates and adjoints are FP64 in both.  Buffers are device memory,
 * row-major, caller-owned; setup copies what it needs (inputs may be freed
 * afterwards).  L <= 0 asks for the power estimate (30 steps).  nonneg is
 * not supported in this form.  The handle runs on the caller's stream and
 * the calls return after their work has finished.
 * --------------------------------------------------------------------- */
typedef struct sfista_diff* sfista_diff_handle;

/* One handle holds `count` problems (sfista_batch_item: Bobs, sizes, dense
 * factors, lambda, L), all of the same rank r.  Each product of an
 * iteration is one grouped launch over the tiles of all problems. */
int sfista_diff_setup(const sfista_batch_item* items, int count, int precision, int iters, int ckpt_every,
                      hipStream_t stream, sfista_diff_handle* out);

/* Load new problems into the handle: `count` items of the same sizes and
 * rank as at setup, in the same order (new Bobs, factors, lambda; L <= 0
 * estimates L again).  No device memory is allocated, except once for the
 * start vector of the first estimate of L; a training loop sets up once and
 * updates before each forward pass.  Items are validated before anything
 * changes; a failure later (a HIP error, a non-finite estimate) leaves the
 * handle to be updated again or destroyed.  A forward pass must follow
 * before the next backward pass. */
int sfista_diff_update(sfista_diff_handle h, const sfista_batch_item* items, int count);

/* Forward pass: X_out[b] (m x n, FP64, entries nullable, or X_out NULL)
 * receives X_iters of problem b.  May be called again (it restarts from 0). */
int sfista_diff_forward(sfista_diff_handle h, double* const* X_out);

/* Backward pass after a forward pass: dX[b] (m x n) in; dA[b] (r x n x n) and
 * dB[b] (r x m x m) are overwritten with the gradients; dlambda (host,
 * `count` entries) too. */
int sfista_diff_backward(sfista_diff_handle h, const double* const* dX, double* const* dA, double* const* dB,
                         double* dlambda);

/* The L in use per problem (host, `count` entries; given or estimated). */
int sfista_diff_get_L(sfista_diff_handle h, double* L);

void sfista_diff_destroy(sfista_diff_handle h);

/* ---------------------------------------------------------------------
 * Structured-FFT form (Section 3.3): the iteration of Algorithm 2 with each
 * Kronecker factor applied through its generator by 1-D FFTs instead of as
 * a dense matrix.  A factor toep(c, j) [+ hank(c, j)] times a line is a
 * convolution of the boundary-extended line with c; its transpose is the
 * matching correlation with the extension folded back.  Two real lines share
 * one complex transform.  Transforms are FP32 (radix-16 Stockham in LDS),
 * iterates FP64; a transform covers 2M - 1 points, so m, n <= 4096.
 *
 *   Bobs   (device) m x n FP64 observed image.
 *   h, k   (device) r x m and r x n FP64 generators as made by
 *          kron_generators (any real generators are accepted).
 *   l, q   0-based centre (the PSF's), bc the boundary.
 *   p      (host) lambda, L (<= 0: power estimate), nonneg, power_iters, x0,
 *          v0 as for sfista_setup; precision and pair_state are ignored.
 * Setup copies what it needs and synchronises `stream`; later calls run on
 * it.  sfista_fft_step is asynchronous; sfista_fft_solve and sfista_fft_apply
 * (A_s X and A_s^T A_s X, each output nullable) return after their work.
 * The report's residual uses Bobs rounded to FP32, as the iteration does.
 * --------------------------------------------------------------------- */
typedef struct sfista_fft* sfista_fft_handle;

int sfista_fft_setup(const double* Bobs, int m, int n, const double* h, const double* k, int r, int l, int q,
                     int bc, const sfista_params* p, hipStream_t stream, sfista_fft_handle* out);
int sfista_fft_step(sfista_fft_handle h, int iters);
int sfista_fft_solve(sfista_fft_handle h, int max_iters, double tol, double* X_out, sfista_report* rep);
int sfista_fft_apply(sfista_fft_handle h, const double* X, double* AX, double* AtAX);
int sfista_fft_get_L(sfista_fft_handle h, double* L);
void sfista_fft_destroy(sfista_fft_handle h);

/* Lipschitz constant in use by the plan (estimated or given). */
int sfista_get_L(sfista_handle h, double* L);

/* Release the plan and its device buffers (synchronises its stream). */
void sfista_destroy(sfista_handle h);

/* Hand the device memory cached by the library's pools (freed buffers of
 * destroyed handles) back to the system.  Buffers of live handles are not
 * affected; call it when no library work is in flight. */
int sfista_release_cached(void);

/* Message describing the calling thread's last failure ("" if none). */
const char* sfista_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SFISTA_H */
