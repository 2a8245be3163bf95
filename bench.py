#!/usr/bin/env python3
"""sFISTA benchmark on one MI355X.

Workload: the 2048 x 2048 precision configuration (reflexive boundary,
rotated Gaussian PSF sigma = (4, 12), theta = 30 deg, r = 5 Kronecker terms,
1% noise, lambda = 0.02, 300 iterations, split-BF16x3 GEMMs with
float-float iterate state).  One timed step is the whole path on one
synthetic image already resident in HBM: the Kronecker approximation
(kron_approx), the plan setup with the estimate of L (12 Lanczos steps, as
Section 4 estimates it; --l-estimate power for 30 power steps), 300
iterations of Algorithm 2 and the FP64 report.  `value` is iterations per
second of whole steps.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sFISTA iters/sec + MFMA TFLOP/s at 2048², r=5; rel err vs FP64 oracle"
PEAK_TFLOPS = {"bf16x3": 2516.6, "bf16": 2516.6, "fp16": 2516.6, "fp32": 157.3, "fp64": 78.6}
MFMA_PER_PRODUCT = {"bf16x3": 3, "bf16": 1, "fp16": 1, "fp32": 1, "fp64": 1}
GEMM_NAMES = ["F1 T=Y*A^T", "F2 R=B*T-Bobs", "G1 S=B^T*R", "G2 sum S*A + update"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel, precision, m, n, r):
    """HBM bytes per launch of a GEMM kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the counters'
    reading of a plain copy), or None when it does not apply (other workload)
    or the GEMM source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gemm_planned_bf16x3_2048_r5_traffic.txt")
    if not (precision == "bf16x3" and m == n == 2048 and r == 5 and os.path.exists(path)):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        key, val = line.split(":", 1)
        fields[key.strip()] = val.split()
    src = os.path.join(ROOT, "paper_1901_00913_amd", "csrc", "gemm.hpp")
    if fields.get("gemm_source_sha256", [""])[0] != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    tag = kernel.split("<")[1].split(">")[0] if "<" in kernel else kernel
    row = fields.get(tag)
    if not row:
        return None
    vals = dict(zip(row[0::2], row[1::2]))
    return float(vals["traffic_bytes"])


BATCH_COUNT = 64
BATCH_ITERS = 100


def run_batch(args, dev, steps, warmup):
    """64 uneven problems (square n in 128..1024, own PSF, rank 1..8, own
    lambda) in plain FP32: per step, the Kronecker approximation of every
    PSF (one kron_approx_batch call), the batch setup (12 Lanczos steps for
    every L, tile autotuning with a cache file) and 100 iterations replayed
    from a HIP graph."""
    import tempfile

    import numpy as np
    import torch

    import synth as S
    from paper_1901_00913_amd import sfista

    if not os.environ.get("SFISTA_TUNE_CACHE"):
        os.environ["SFISTA_TUNE_CACHE"] = os.path.join(tempfile.gettempdir(), f"sfista_tune_{os.getpid()}.txt")
    log(f"[batch] generating {BATCH_COUNT} problems")
    probs = S.batch_problems(count=BATCH_COUNT, iters=BATCH_ITERS)
    psf = [torch.as_tensor(p.psf).to(dev) for p in probs]
    bobs = [torch.as_tensor(p.bobs).to(dev) for p in probs]
    flops_iter = sum(4.0 * p.r * p.shape[0] * p.shape[1] * (p.shape[0] + p.shape[1]) for p in probs)
    torch.cuda.synchronize()

    def step():
        kron = sfista.kron_approx_many(psf, [p.center for p in probs], [p.bc for p in probs], [p.r for p in probs])
        items = [(Bo, A, B, p.lam, None) for p, Bo, (A, B, _, _) in zip(probs, bobs, kron)]
        b = sfista.Batch(items, precision="fp32", pair_state=False, max_iters=BATCH_ITERS, l_estimate="lanczos",
                         autotune=True, graph=True)
        _, reps = b.solve(BATCH_ITERS, want_x=False)
        tiles = b.tiles()
        b.close()
        return reps, tiles

    for w in range(warmup):
        log(f"[batch] warmup step {w + 1}/{warmup}")
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iter_s = float(np.mean([o[0][0]["seconds"] for o in out]))
    value = BATCH_COUNT * BATCH_ITERS * steps / elapsed
    achieved = flops_iter * BATCH_ITERS / iter_s / 1e12
    peak = PEAK_TFLOPS["fp32"]
    log(f"[batch] {steps} steps in {elapsed:.3f} s -> {value:.0f} image-iters/s; iterations {achieved:.1f} TFLOP/s")
    summary = {"image_iters_per_s": value, "iteration_only_image_iters_per_s": BATCH_COUNT * BATCH_ITERS / iter_s,
               "iteration_alg_tflops": achieved, "fp32_mfma_frac": achieved / peak, "tiles": out[-1][1],
               "ms_per_step": elapsed / steps * 1e3, "max_resid_rel": max(r["resid_rel"] for r in out[-1][0])}
    line = {
        "metric": "sFISTA image-iterations/s, 64 uneven images in one batch", "value": value,
        "unit": "image-iters/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"sfista-batch{BATCH_COUNT}-n128..1024-r1..8-{BATCH_ITERS}it",
                   "images": BATCH_COUNT, "iters": BATCH_ITERS, "precision": "fp32", "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "kernel": "gemm_grouped (all four phases, whole iterations)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None},
        "cpu_baseline": None,
        "extra": summary,
    }
    return {"line": line, "summary": summary}


DIFF_COUNT, DIFF_N, DIFF_R, DIFF_ITERS, DIFF_CKPT = 8, 512, 4, 50, 10


def run_diff(args, dev, steps, warmup):
    """Differentiable form: 8 images at 512^2 with one shared reflexive
    Gaussian blur (r = 4 factors from the GPU Kronecker approximation), 50
    unrolled FP32 iterations with checkpoints every 10, loss = mean squared
    error to the true images; a step loads the current factors and lambda
    into the handle (set up once, before the timed region), runs the forward
    pass and the backward pass to every factor entry and lambda (L estimated
    once by 12 Lanczos steps, held fixed)."""
    import numpy as np
    import torch

    import synth as S
    from paper_1901_00913_amd import sfista

    log(f"[diff] generating {DIFF_COUNT} problems at {DIFF_N}^2")
    probs = S.diff_problems(count=DIFF_COUNT, n=DIFF_N, r=DIFF_R, iters=DIFF_ITERS)
    p0 = probs[0]
    l, q = p0.center
    A1, B1, _, _ = sfista.kron_approx(torch.as_tensor(p0.psf).to(dev), l, q, p0.bc, DIFF_R)
    est = sfista.Solver(torch.as_tensor(p0.bobs).to(dev), A1, B1, lam=p0.lam, precision="fp32",
                        l_estimate="lanczos")
    L = est.L
    est.close()
    A = A1.unsqueeze(0).repeat(DIFF_COUNT, 1, 1, 1).contiguous().requires_grad_(True)
    B = B1.unsqueeze(0).repeat(DIFF_COUNT, 1, 1, 1).contiguous().requires_grad_(True)
    lam = torch.tensor(p0.lam, dtype=torch.float64, device=dev, requires_grad=True)
    Bobs = torch.tensor(np.stack([p.bobs for p in probs]), device=dev)
    xt = torch.tensor(np.stack([p.x_true for p in probs]), device=dev)
    n = DIFF_N
    # per iteration: 12 products of 2 r n^3 (forward, recompute, adjoint: F1, F2, G1, G2 each) and the
    # two factor-gradient products of 2 (r n) n (2 n) each
    flops_img = DIFF_ITERS * (12 * 2.0 * DIFF_R * n ** 3 + 2 * 4.0 * DIFF_R * n ** 3)

    plan = sfista.Unrolled([(Bobs[k], A1, B1, p0.lam, L) for k in range(DIFF_COUNT)], iters=DIFF_ITERS,
                           ckpt=DIFF_CKPT, precision="fp32")

    def step():
        A.grad = B.grad = lam.grad = None
        X = sfista.unrolled(A, B, lam, Bobs, L=L, plan=plan)
        loss = ((X - xt) ** 2).mean(dim=(1, 2)).sum()
        loss.backward()
        return loss.detach().item()

    for w in range(warmup):
        log(f"[diff] warmup step {w + 1}/{warmup}")
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.close()
    value = DIFF_COUNT * steps / elapsed
    achieved = flops_img * DIFF_COUNT * steps / elapsed / 1e12
    peak = PEAK_TFLOPS["fp32"]
    log(f"[diff] {steps} steps in {elapsed:.3f} s -> {value:.2f} image-gradients/s, {achieved:.1f} TFLOP/s")
    summary = {"image_gradients_per_s": value, "ms_per_step": elapsed / steps * 1e3, "alg_tflops": achieved,
               "fp32_mfma_frac": achieved / peak, "loss": losses[-1], "L": L,
               "dlam": float(lam.grad), "grad_norm_A": float(A.grad.norm()), "grad_norm_B": float(B.grad.norm())}
    line = {
        "metric": "sFISTA unrolled-gradient throughput, 8 images 512^2, r=4, 50 iterations",
        "value": value, "unit": "image-gradients/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"sfista-diff{DIFF_COUNT}-{n}-r{DIFF_R}-{DIFF_ITERS}it-ckpt{DIFF_CKPT}",
                   "images": DIFF_COUNT, "iters": DIFF_ITERS, "precision": "fp32", "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "kernel": "gemm_grouped (forward, recompute, adjoint and gradient GEMMs)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None},
        "cpu_baseline": None,
        "extra": summary,
    }
    return {"line": line, "summary": summary}


def run_shard(args, dev, steps, warmup):
    """One GPU's share of the 2048^2, r = 5 image under row-block sharding
    over 8 GPUs: a 256 x 2048 block.  Its row-local products have the shard's
    exact shapes, F1 (T = Y A^T: M = r n = 10240, N = 256, K = 2048) and G2
    (sum S_k A_k: M = 256, N = 2048, K = r n = 10240); F2 and G1 of a
    256-row image are not the shard's (those mix rows across GPUs).  A step is
    300 BF16X3 iterations on a synthetic 256 x 2048 problem (its own PSF and
    factors), with the GEMMs of every tenth iteration timed."""
    import numpy as np
    import torch

    import synth as S
    from paper_1901_00913_amd import sfista

    m, n, r, iters, G = 256, 2048, 5, args.iters, 8
    psf = S.gaussian_psf(m, n, sigma=(4.0, 12.0), theta_deg=30.0)
    l, q = m // 2, n // 2
    x = S.make_image(m, n, 1400)
    bobs = S.add_noise(S.blur(x, psf, (l, q), 1), 0.01, 2400)
    P = torch.as_tensor(psf).to(dev)
    Bobs = torch.as_tensor(bobs).to(dev)
    A, B, _, _ = sfista.kron_approx(P, l, q, 1, r)
    s = sfista.Solver(Bobs, A, B, lam=0.02, precision="bf16x3", l_estimate="lanczos")
    for w in range(warmup):
        log(f"[shard] warmup step {w + 1}/{warmup}")
        s.solve(iters, want_x=False)
    s.set_timing(args.timing_every)
    s.kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.solve(iters, want_x=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, cnt = s.kernel_times()
    s.close()
    # the same two products on the whole 2048^2 image, same box, same sampling
    p3 = S.config(3)
    A3, B3, _, _ = sfista.kron_approx(torch.as_tensor(p3.psf).to(dev), p3.center[0], p3.center[1], p3.bc, r)
    s3 = sfista.Solver(torch.as_tensor(p3.bobs).to(dev), A3, B3, lam=p3.lam, L=1.0, precision="bf16x3")
    s3.solve(20, want_x=False)
    s3.set_timing(args.timing_every)
    s3.kernel_times()
    s3.solve(iters, want_x=False)
    ms3, _ = s3.kernel_times()
    s3.close()
    peak = PEAK_TFLOPS["bf16x3"]
    prods = {}
    for name, g, (M, N, K) in (("F1", 0, (r * n, m, n)), ("G2", 3, (m, n, r * n))):
        t, t3 = ms[g] + ms[4 + g], ms3[g] + ms3[4 + g]   # the GEMM and its split reduction
        executed = 3 * 2.0 * M * N * K / (ms[g] * 1e-3) / 1e12
        prods[name] = {"shape_MNK": [M, N, K], "gemm_ms": ms[g], "reduce_ms": ms[4 + g], "launches": cnt[g],
                       "executed_tflops": executed, "mfma_frac": executed / peak, "full_image_ms": t3,
                       "ms_over_one_eighth_of_full": t / (t3 / G)}
        log(f"[shard] {name} {M}x{N}x{K}: {ms[g] * 1e3:.1f} + {ms[4 + g] * 1e3:.1f} us, "
            f"{executed:.0f} TFLOP/s executed ({executed / peak:.3f} of peak); full image {t3 * 1e3:.1f} us, "
            f"shard / (full / {G}) = {t / (t3 / G):.2f}")
    value = iters * steps / elapsed
    line = {
        "metric": "sFISTA iters/sec of one GPU's row block (2048^2 image over 8 GPUs)", "value": value,
        "unit": "iters/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
        "config": {"workload": f"sfista-shard-{m}x{n}-r{r}-of-2048x2048-g{G}", "image": [m, n], "rank": r,
                   "iters": iters, "precision": "bf16x3", "parallelism": "single-gpu (one shard)"},
        "roofline": None, "cpu_baseline": None, "extra": {"row_local_products": prods}}
    return {"line": line, "summary": prods}


def run_paper(args, dev, steps, warmup):
    """The paper's experiment shape (Section 4) on synthetic stand-ins: 256^2
    images, reflexive boundary, 1% noise, a defocus and a motion PSF, s = 1..5
    Kronecker terms, L by 20 Lanczos steps (Section 4 takes L from a Lanczos
    estimate), 50 iterations in FP64 (as the paper's double precision),
    lambda = 0.02.  Per (PSF, s): eps_s = ||A - A_s||_F (Theorem 1), the
    restoration error eta = ||X - x_true|| / ||x_true|| and the approximate
    residual gamma_s, and the time of the setup and of the iterations.  A step
    is the whole sweep; `value` is sweeps per second."""
    import numpy as np
    import torch

    import synth as S
    from paper_1901_00913_amd import sfista

    probs = S.paper_problems(256, iters=50)
    dat = {k: (torch.as_tensor(p.psf).to(dev), torch.as_tensor(p.bobs).to(dev), p) for k, p in probs.items()}

    def sweep():
        rows = []
        for kind, (P, Bo, p) in dat.items():
            l, q = p.center
            for s_ in range(1, 6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                A, B, sig, eps = sfista.kron_approx(P, l, q, p.bc, s_)
                sol = sfista.Solver(Bo, A, B, lam=p.lam, precision="fp64", power_iters=20, l_estimate="lanczos")
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                X, rep = sol.solve(p.iters)
                sol.close()
                eta = float(np.linalg.norm(X.cpu().numpy() - p.x_true) / np.linalg.norm(p.x_true))
                rows.append({"psf": kind, "s": s_, "eps_s": eps, "eta": eta, "gamma_s": rep["resid_rel"],
                             "setup_ms": (t1 - t0) * 1e3, "iter_ms": rep["seconds"] * 1e3})
        return rows

    for w in range(warmup):
        log(f"[paper] warmup sweep {w + 1}/{warmup}")
        sweep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [sweep() for _ in range(steps)]
    elapsed = time.perf_counter() - t0
    rows = out[-1]
    for r_ in rows:
        log(f"[paper] {r_['psf']:8s} s={r_['s']} eps_s={r_['eps_s']:.4e} eta={r_['eta']:.4f} "
            f"gamma_s={r_['gamma_s']:.4e} setup {r_['setup_ms']:.1f} ms, 50 its {r_['iter_ms']:.2f} ms")
    line = {
        "metric": "paper-shaped sweep (256^2, s=1..5, defocus and motion, 50 iterations FP64)",
        "value": steps / elapsed, "unit": "sweeps/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp64", "data": "synthetic",
        "config": {"workload": "sfista-paper-256-s1..5-50it", "image": [256, 256], "iters": 50,
                   "precision": "fp64", "parallelism": "single-gpu"},
        "roofline": None, "cpu_baseline": None, "extra": {"rows": rows},
    }
    return {"line": line, "summary": rows}


def l_steps(args) -> int:
    """Steps of the estimate of L that the library runs for these options."""
    return args.l_steps or (12 if args.l_estimate == "lanczos" else 30)


def run_fft(args, dev, steps, warmup):
    """Structured-FFT form on the precision workload (2048^2, r = 5,
    reflexive, 300 iterations): a step runs kron_generators, the plan setup
    with the estimate of L and the iterations, as the default line does
    with dense factors.  Transforms are FP32, iterates FP64."""
    import torch

    import synth as S
    from paper_1901_00913_amd import sfista

    p = S.config(3, n=args.n, iters=args.iters)
    m, n = p.shape
    l, q = p.center
    r, iters = p.r, p.iters
    P = torch.as_tensor(p.psf).to(dev)
    Bobs = torch.as_tensor(p.bobs).to(dev)
    v0 = torch.as_tensor(p.v0).to(dev)

    def step():
        h, k, _, eps = sfista.kron_generators(P, l, q, p.bc, r)
        s = sfista.FftSolver(Bobs, h, k, l, q, p.bc, lam=p.lam, power_iters=args.l_steps, v0=v0,
                             l_estimate=args.l_estimate)
        _, rep = s.solve(iters, want_x=False)
        L = s.L
        s.close()
        return rep, L

    for w in range(warmup):
        log(f"[fft] warmup step {w + 1}/{warmup}")
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = iters * steps / elapsed
    iter_s = sum(rp["seconds"] for rp, _ in reps) / steps
    # transforms per iteration: four line passes, each r + 1 transforms per
    # pair of lines; 5 N log2 N flops per complex transform of N points
    def nfft(M):
        N = 64
        while N < 2 * M - 1:
            N *= 2
        return N
    Nm, Nn = nfft(m), nfft(n)
    fl = lambda N, lines: (r + 1) * ((lines + 1) // 2) * 5.0 * N * math.log2(N)
    flops_it = 2 * fl(Nn, m) + 2 * fl(Nm, n)
    # algorithmic HBM bytes per iteration: F1 reads Y (8) and writes r T_k (4 r); the column pass reads
    # r T_k (4 r) and Bobs^T (4) and writes r S_k (4 r); G2 reads r S_k (4 r), Y and X_{k-1} (16) and
    # writes X_k and Y_{k+1} (16), per pixel
    bytes_it = m * n * (44 + 16 * r)
    log(f"[fft] {steps} steps in {elapsed:.3f} s -> {value:.1f} it/s; iterations only {iters / iter_s:.1f} it/s")
    summary = {"its_per_s": value, "iteration_only_its": iters / iter_s, "ms_per_step": elapsed / steps * 1e3,
               "fft_tflops": flops_it / (iter_s / iters) / 1e12,
               "fft_frac_of_fp32_vector_peak": flops_it / (iter_s / iters) / 1e12 / PEAK_TFLOPS["fp32"],
               "hbm_tb_per_s": bytes_it / (iter_s / iters) / 1e12, "transform_sizes": [Nm, Nn],
               "L": reps[-1][1], "resid_rel": reps[-1][0]["resid_rel"], "phi_s": reps[-1][0]["phi_s"]}
    line = {
        "metric": "sFISTA iterations/s, structured-FFT form, 2048^2, r=5", "value": value, "unit": "iters/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"sfista-fft-{m}x{n}-r{r}-reflexive-{iters}it", "image": [m, n], "rank": r,
                   "iters": iters, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "kernel": "fan_in_kernel / fan_out_kernel (all four line passes)",
                     "achieved": summary["fft_tflops"], "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": summary["fft_frac_of_fp32_vector_peak"], "traffic": None},
        "cpu_baseline": None,
        "extra": summary,
    }
    return {"line": line, "summary": summary}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048, help="image size (the workload is 2048)")
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--precision", default="bf16x3", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--l-estimate", default="lanczos", choices=["lanczos", "power"],
                    help="estimate of L in each step (Section 4 uses Lanczos)")
    ap.add_argument("--l-steps", type=int, default=0, help="steps of that estimate (0: 12 Lanczos, 30 power)")
    ap.add_argument("--timing-every", type=int, default=10,
                    help="HIP-event timing of the GEMMs of every k-th iteration in the timed steps (each event "
                         "leaves a few-microsecond gap, so timing every iteration would slow the step it times)")
    ap.add_argument("--cpu-iters", type=int, default=3, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--workload", default="precision-2048",
                    choices=("precision-2048", "batch64", "diff8", "paper256", "fft2048", "shard2048g8"),
                    help="precision-2048: one 2048^2 image, r = 5 (default); batch64: 64 uneven images "
                         "in grouped launches replayed from a HIP graph; diff8: gradient of 50 unrolled "
                         "iterations for 8 images at 512^2, r = 4; paper256: the paper-shaped sweep "
                         "(256^2, reflexive, 1%% noise, defocus and motion blur, s = 1..5, 50 iterations); "
                         "fft2048: the default workload in the structured-FFT form; shard2048g8: one GPU's "
                         "256 x 2048 row block of the default image split over 8 GPUs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch64 summary in the default line")
    ap.add_argument("--no-diff", action="store_true", help="skip the diff8 summary in the default line")
    ap.add_argument("--no-fft", action="store_true", help="skip the fft2048 summary in the default line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, copy a BYTES-long device buffer once (a plain copy kernel "
                         "of known traffic, for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run it with --gpus 1 "
              "(the shard2048g8 workload times one GPU's share of a sharded image).", file=sys.stderr)
        sys.exit(2)

    # hardware queues of this process, read when HIP starts: the batched
    # Kronecker setup runs sixteen streams of latency-bound kernels, which
    # overlap only as far as there are queues (16 instead of HIP's default 4:
    # 4.6% more image-iterations/s on the batch64 workload)
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

    import numpy as np
    import torch

    import synth as S
    from paper_1901_00913_amd import sfista

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    sfista.lib()
    dev = torch.device("cuda:0")

    if args.workload in ("batch64", "diff8", "paper256", "fft2048", "shard2048g8"):
        res = {"batch64": run_batch, "diff8": run_diff, "paper256": run_paper, "fft2048": run_fft,
               "shard2048g8": run_shard}[args.workload](
            args, dev, args.steps, args.warmup)
        print(json.dumps(res["line"]), flush=True)
        return

    log(f"[bench] generating the {args.n}x{args.n} workload")
    p = S.config(3, n=args.n, iters=args.iters)
    m, n = p.shape
    l, q = p.center
    r, lam, bc, iters = p.r, p.lam, p.bc, p.iters
    P = torch.as_tensor(p.psf).to(dev)
    Bobs = torch.as_tensor(p.bobs).to(dev)
    v0 = torch.as_tensor(p.v0).to(dev)
    torch.cuda.synchronize()

    def step(timing):
        A, B, sigma, eps = sfista.kron_approx(P, l, q, bc, r)
        s = sfista.Solver(Bobs, A, B, lam=lam, precision=args.precision, power_iters=args.l_steps, v0=v0,
                          l_estimate=args.l_estimate)
        if timing:
            s.set_timing(args.timing_every)
        _, rep = s.solve(iters, want_x=False)
        kt = s.kernel_times() if timing else None
        L = s.L
        s.close()
        return rep, kt, L, eps

    for w in range(args.warmup):
        log(f"[bench] warmup step {w + 1}/{args.warmup}")
        step(False)
    torch.cuda.synchronize()
    reps, kts = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        rep, kt, L, eps = step(True)
        reps.append(rep)
        kts.append(kt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = iters * args.steps / elapsed
    log(f"[bench] {args.steps} steps in {elapsed:.3f} s -> {value:.1f} it/s")

    # mean device times over the timed steps: GEMM kernels (0..3) and the
    # reductions of their K-split tiles (4..7)
    tot = [0.0] * 8
    cnt = [0] * 8
    for ms, c in kts:
        for g in range(8):
            tot[g] += ms[g] * c[g]
            cnt[g] += c[g]
    avg = [t / c if c else 0.0 for t, c in zip(tot, cnt)]
    flops = [2.0 * r * m * n * n, 2.0 * r * m * m * n, 2.0 * r * m * m * n, 2.0 * r * m * n * n]
    # kernels as rocprofv3 names them: F1 and G1 share one instantiation
    groups = {"gemm_planned_kernel<EpiStack> (F1, G1)": [0, 2], "gemm_planned_kernel<EpiResid> (F2)": [1],
              "gemm_planned_kernel<EpiUpdate> (G2)": [3]}
    gstat = {}
    for name, idx in groups.items():
        t = sum(tot[i] for i in idx)
        c = sum(cnt[i] for i in idx)
        f = sum(flops[i] * cnt[i] for i in idx) / max(c, 1)
        gstat[name] = {"total_ms": t, "launches": c, "avg_ms": t / max(c, 1), "alg_flops_per_launch": f}
    dom = max(gstat, key=lambda k: gstat[k]["total_ms"])
    mult = MFMA_PER_PRODUCT[args.precision]
    achieved_alg = gstat[dom]["alg_flops_per_launch"] / (gstat[dom]["avg_ms"] * 1e-3) / 1e12
    achieved = achieved_alg * mult   # executed MFMA flops (three bf16 products per product for bf16x3)
    peak = PEAK_TFLOPS[args.precision]
    iter_s = float(np.mean([rp["seconds"] for rp in reps]))
    iter_rate = iters / iter_s
    alg_tflops_iter = 8.0 * r * n ** 3 / (iter_s / iters) / 1e12 if m == n else None

    extra = {
        "iteration_only_its": iter_rate,
        "iteration_alg_tflops": alg_tflops_iter,
        "setup_ms_per_step": elapsed / args.steps * 1e3 - iter_s * 1e3,
        "gemm_avg_ms": dict(zip(GEMM_NAMES, avg[:4])),
        "split_reduce_avg_ms": dict(zip(GEMM_NAMES, avg[4:])),
        "gemm_alg_tflops": {GEMM_NAMES[g]: flops[g] / (avg[g] * 1e-3) / 1e12 for g in range(4) if avg[g] > 0},
        "iteration_mfma_util": (alg_tflops_iter or 0.0) * mult / peak,
        "L": L, "eps_s": eps, "resid_rel": reps[-1]["resid_rel"], "phi_s": reps[-1]["phi_s"],
    }

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if not args.no_fp32_compare and args.precision != "fp32":
        log("[bench] plain FP32 comparison solve")
        A, B, _, _ = sfista.kron_approx(P, l, q, bc, r)
        s = sfista.Solver(Bobs, A, B, lam=lam, L=L, precision="fp32", pair_state=False)
        _, rep32 = s.solve(iters, want_x=False)
        s.close()
        extra["fp32_iteration_only_its"] = iters / rep32["seconds"]
        extra["speedup_vs_fp32"] = rep32["seconds"] / iter_s

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        log("[bench] cpu_baseline: oracle Kronecker setup (untimed)")
        K, H, _, _, _, _ = O.kron_approx64(p.psf, l, q, bc, r)
        Lfix = 1.02   # a fixed step constant shared by both sides of the rel-err check
        log(f"[bench] cpu_baseline: timing {args.cpu_iters} oracle iterations")
        c0 = time.perf_counter()
        Xo = O.sfista64(K, H, p.bobs, lam, Lfix, args.cpu_iters)
        c1 = time.perf_counter()
        A, B, _, _ = sfista.kron_approx(P, l, q, bc, r)
        s = sfista.Solver(Bobs, A, B, lam=lam, L=Lfix, precision=args.precision)
        Xg, _ = s.solve(args.cpu_iters)
        s.close()
        rel_err = float(np.linalg.norm(Xg.cpu().numpy() - Xo) / np.linalg.norm(Xo))
        cpu = {"value": args.cpu_iters / (c1 - c0), "unit": "iters/s", "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_iters} FP64 numpy sFISTA iterations at {m}x{n}, r={r} "
                         f"(Kronecker setup excluded)",
               "rel_err_gpu_vs_oracle": rel_err, "rel_err_iters": args.cpu_iters}
        log(f"[bench] cpu_baseline {cpu['value']:.3f} it/s on {threads} threads; rel err {rel_err:.3e}")

    if not args.no_batch:
        extra["batch64"] = run_batch(args, dev, 1, 1)["summary"]
    if not args.no_diff:
        extra["diff8"] = run_diff(args, dev, 1, 1)["summary"]
    if not args.no_fft:
        fsum = run_fft(args, dev, 1, 1)["summary"]
        fsum["iteration_speedup_vs_gemm_form"] = fsum["iteration_only_its"] / iter_rate
        extra["fft2048"] = fsum

    out = {
        "metric": METRIC, "value": value, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"sfista-{m}x{n}-r{r}-reflexive-{iters}it", "image": [m, n], "rank": r,
                   "iters": iters, "precision": args.precision, "lambda": lam,
                   "l_estimate": args.l_estimate, "l_steps": l_steps(args), "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(dom, args.precision, m, n, r),
                     "flops_basis": "executed MFMA flops per launch (bf16x3: 3 bf16 products of 2*M*N*K)",
                     "achieved_algorithmic": achieved_alg, "avg_launch_ms": gstat[dom]["avg_ms"],
                     "launches": gstat[dom]["launches"], "timed_every": args.timing_every},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
