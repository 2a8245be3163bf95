"""Batched form: many uneven problems advanced together by grouped GEMM
launches (one launch per phase for the whole batch), optionally replayed
from a captured HIP graph, with tile shapes from the autotuner.

Every problem of a batch must follow Algorithm 2 exactly as a lone plan
does, so the checks are: each problem against the FP64 oracle, the batch
against per-image plans, graph replays against eager launches (bitwise),
and tile-shape choices against each other (bitwise: the shape changes which
workgroup computes an output, never the order of its K sum).
"""

import math
import os

import numpy as np
import pytest

import oracle as O
import synth as S
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

# uneven square sizes, one ragged (not a multiple of 64 or 16)
SIZES = [64, 100, 128, 192]
COUNT = 6
ITERS = 40


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available()
    from paper_1901_00913_amd import sfista
    sfista.lib()
    return sfista


@pytest.fixture(scope="module")
def case():
    """Batch recipe (per-image Gaussian or motion PSF, either boundary, rank
    1..8, log-uniform lambda) at small sizes, with the oracle's factors, L
    and FP64 iterates."""
    probs = S.batch_problems(count=COUNT, sizes=SIZES, iters=ITERS)
    out = []
    for p in probs:
        l, q = p.center
        K, H, _, _, _, _ = O.kron_approx64(p.psf, l, q, p.bc, p.r)
        L = O.lipschitz_power(K, H, p.v0, 200)
        ref = O.sfista64(K, H, p.bobs, p.lam, L, ITERS)
        out.append((p, K, H, L, ref))
        say(f"[batch] {p.name}: {p.shape} r={p.r} bc={p.bc} lam={p.lam:.4g} L={L:.6g}")
    return out


def _problems(case):
    return [(dev(p.bobs), dev(K), dev(H), p.lam, L) for p, K, H, L, _ in case]


# Relative error to the FP64 oracle after 40 iterations: FP64 to rounding,
# the float-float-state modes to what they are built for, plain FP32 state
# to single precision times the iteration's amplification.
BATCH_TOL = {("fp64", 1): 1e-12, ("fp32", 1): 2e-6, ("fp32", 0): 1e-4, ("bf16x3", 1): 1e-5}


@pytest.mark.parametrize("mode,pair", list(BATCH_TOL))
def test_batch_matches_oracle(sf, case, mode, pair):
    say(f"[batch] mode={mode} pair_state={pair}")
    b = sf.Batch(_problems(case), precision=mode, max_iters=ITERS, pair_state=bool(pair))
    xs, reps = b.solve(ITERS)
    for (p, K, H, L, ref), X, rep in zip(case, xs, reps):
        e = rel(host(X), ref)
        say(f"   {p.name} {p.shape} r={p.r}: rel err {e:.3e}")
        assert e < BATCH_TOL[(mode, pair)]
        assert rep["iters"] == ITERS and rep["status"] == 0
        assert math.isclose(rep["L"], L, rel_tol=1e-15)
        if mode == "fp64":
            assert math.isclose(rep["phi_s"], O.phi_s(K, H, p.bobs, ref, p.lam), rel_tol=1e-10)
    b.close()


def test_batch_matches_single_plans(sf, case):
    """The grouped launches compute what lone plans compute.  A lone plan
    splits K sums to fill the GPU (a small image has few tiles), which
    changes the FP32 summation order, so both sides are held to the oracle
    (1e-5 each, hence 2e-5 apart); bit-for-bit agreement is reported."""
    b = sf.Batch(_problems(case), precision="bf16x3", max_iters=ITERS)
    xs, _ = b.solve(ITERS)
    same = 0
    for (p, K, H, L, _), X in zip(case, xs):
        s = sf.Solver(dev(p.bobs), dev(K), dev(H), lam=p.lam, L=L, precision="bf16x3")
        Xs, _ = s.solve(ITERS)
        e = rel(host(X), host(Xs))
        same += int(e == 0.0)
        say(f"   {p.name}: batch vs plan {e:.3e}")
        assert e < 2e-5
        s.close()
    b.close()
    say(f"   {same} of {len(case)} bitwise equal")


def test_batch_power_iteration_L(sf, case):
    """An item without L gets the internal power estimate of
    lambda_max(A_s^T A_s) from the library's own start vector.  Any such
    estimate ||A_s^T A_s v|| with ||v|| = 1 is a lower bound of lambda_max,
    itself at most (sum_k ||A_k|| ||B_k||)^2; blur spectra cluster near the
    top, so two starts agree only loosely after 200 steps (1%)."""
    probs = [(Bo, A, B, lam, None) for Bo, A, B, lam, _ in _problems(case)]
    b = sf.Batch(probs, precision="fp64", max_iters=1, power_iters=200)
    _, reps = b.solve(0)
    for (p, K, H, L, _), rep in zip(case, reps):
        upper = sum(np.linalg.norm(K[k], 2) * np.linalg.norm(H[k], 2) for k in range(K.shape[0])) ** 2
        say(f"   {p.name}: L gpu={rep['L']:.12g} oracle={L:.12g} bound={upper:.12g}")
        assert rep["L"] <= upper * (1 + 1e-12)
        assert abs(rep["L"] - L) <= 1e-2 * L
    b.close()


def test_graph_replays_match_eager_bitwise(sf, case):
    """Graph mode (10-iteration replays plus eager remainders) against
    eager launches, checked after every call, with unrelated eager GPU work
    and synchronisations between the replays."""
    import torch
    splits = (10, 25, 10, 7, 20)
    total = sum(splits)
    probs = _problems(case)
    runs = {}
    for graph in (False, True):
        b = sf.Batch(probs, precision="fp32", max_iters=total, pair_state=False, graph=graph)
        seen = []
        for k in splits:
            xs, reps = b.solve(k)
            seen.append(([host(x) for x in xs], [r["phi_s"] for r in reps]))
            # eager work on the caller's stream between replays
            a = torch.randn(512, 512, device="cuda:0")
            (a @ a).sum().item()
            torch.cuda.synchronize()
        runs[graph] = seen
        b.close()
    for c, (eager, graphed) in enumerate(zip(runs[False], runs[True])):
        for i in range(len(probs)):
            assert np.array_equal(eager[0][i], graphed[0][i]), (c, i)
        assert eager[1] == graphed[1]
    say(f"   {len(splits)} calls, {total} iterations: graph == eager bitwise")


def test_autotune_cache_and_tile_invariance(sf, case, tmp_path, monkeypatch):
    """The autotuner writes its choice to the cache file and a second setup
    reads it back; whatever shapes it picks, the iterates equal those of the
    fixed shapes bit for bit, and the tuning runs leave no trace."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SFISTA_TUNE_CACHE", str(cache))
    probs = _problems(case)
    b1 = sf.Batch(probs, precision="bf16x3", max_iters=ITERS, autotune=True)
    t1 = b1.tiles()
    assert all(c in (0, 1, 2) for c in t1)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    X1, _ = b1.solve(ITERS)
    b1.close()
    b2 = sf.Batch(probs, precision="bf16x3", max_iters=ITERS, autotune=True)
    assert b2.tiles() == t1
    assert cache.read_text().splitlines() == lines
    b2.close()
    monkeypatch.delenv("SFISTA_TUNE_CACHE")
    b3 = sf.Batch(probs, precision="bf16x3", max_iters=ITERS)
    X3, _ = b3.solve(ITERS)
    say(f"   autotuned tiles {t1}, heuristic tiles {b3.tiles()}")
    b3.close()
    for a, c in zip(X1, X3):
        assert np.array_equal(host(a), host(c))


def test_pinned_tile_shapes_are_bitwise_equal(sf, case):
    """Every tile shape (the large tile, 64 x 64, 128 x 128) pinned for all
    four products gives the same iterates bit for bit, in eager launches and
    through a graph captured after the change; FP64 refuses the shape that
    is its own large tile."""
    probs = _problems(case)
    outs = []
    for shape in (0, 1, 2):
        for graph in (False, True):
            b = sf.Batch(probs, precision="fp32", max_iters=ITERS, graph=graph)
            b.solve(2)                      # a graph is captured with the default shapes first
            b.set_tiles([shape] * 4)
            assert b.tiles() == [shape] * 4
            X, _ = b.solve(ITERS - 2)
            outs.append([host(x) for x in X])
            b.close()
    for o in outs[1:]:
        for a, c in zip(outs[0], o):
            assert np.array_equal(a, c)
    b = sf.Batch(probs[:2], precision="fp64", max_iters=2)
    with pytest.raises(sf.SfistaError):
        b.set_tiles([2, 2, 2, 2])
    b.set_tiles([1, 0, 1, 0])
    b.close()


def test_batch_iteration_limit(sf, case):
    b = sf.Batch(_problems(case)[:2], precision="fp32", max_iters=5)
    b.solve(3)
    with pytest.raises(sf.SfistaError):
        b.solve(3)
    b.close()


def test_single_problem_batch(sf, case):
    p, K, H, L, ref = case[0]
    b = sf.Batch([(dev(p.bobs), dev(K), dev(H), p.lam, L)], precision="fp64", max_iters=ITERS)
    xs, _ = b.solve(ITERS)
    assert rel(host(xs[0]), ref) < 1e-12
    b.close()


@pytest.mark.parametrize("est,steps", [("power", 25), ("lanczos", 12)])
@pytest.mark.parametrize("mode,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_batched_estimate_of_L_matches_lone_plans(sf, case, mode, tol, est, steps):
    """Problems given without L: the batch estimates every L at once (power
    iteration or Lanczos; grouped products, per-problem reductions), from
    the same internal start vector and with the same reduction structure as
    a lone plan.  Each estimate equals the lone plan's up to the rounding of
    the products' different K order; the lone plan's estimates are held to
    the oracle's in test_gpu_parity.  The iterates that follow match the
    lone plans' to the mode's tolerance."""
    probs = [(dev(p.bobs), dev(K), dev(H), p.lam, None) for p, K, H, L, _ in case]
    b = sf.Batch(probs, precision=mode, max_iters=ITERS, power_iters=steps, l_estimate=est)
    Xb, reps = b.solve(ITERS)
    b.close()
    for (p, K, H, L, _), rp, xb in zip(case, reps, Xb):
        s = sf.Solver(dev(p.bobs), dev(K), dev(H), lam=p.lam, precision=mode, power_iters=steps, l_estimate=est)
        Ls = s.L
        X, _ = s.solve(ITERS)
        s.close()
        say(f"[batch {est} {mode}] {p.name}: batch L {rp['L']:.15g} lone {Ls:.15g}")
        assert math.isclose(rp["L"], Ls, rel_tol=tol)
        assert rel(host(xb), host(X)) < (1e-10 if mode == "fp64" else 1e-4)


def test_kron_approx_many_equals_single_calls(sf):
    """The batched Kronecker setup of twenty PSFs (more images than the
    sixteen internal streams, so streams are reused; both boundaries, ragged
    sizes, ranks 1..6) equals kron_approx called image by image, bit for
    bit: factors, sigma and eps_s."""
    import torch
    shapes = [(33, 47, 2, O.BC_ZERO), (64, 48, 3, O.BC_REFLEXIVE), (128, 128, 5, O.BC_REFLEXIVE),
              (200, 136, 1, O.BC_ZERO), (257, 130, 4, O.BC_REFLEXIVE), (40, 40, 6, O.BC_ZERO),
              (96, 160, 2, O.BC_REFLEXIVE), (17, 9, 3, O.BC_ZERO), (300, 300, 5, O.BC_REFLEXIVE)]
    shapes += [(24 + 7 * t, 30 + 5 * t, 1 + t % 4, t % 2) for t in range(11)]
    Ps, centers, bcs, rs = [], [], [], []
    for t, (m, n, r, bc) in enumerate(shapes):
        c = (m // 2 - t % 3, n // 2 + t % 2)
        Ps.append(dev(S.gaussian_psf(m, n, (1.0 + 0.3 * t, 2.5), 15.0 * t, c)))
        centers.append(c)
        bcs.append(bc)
        rs.append(r)
    many = sf.kron_approx_many(Ps, centers, bcs, rs)
    torch.cuda.synchronize()
    for i, (P, c, bc, r) in enumerate(zip(Ps, centers, bcs, rs)):
        A, B, sig, eps = sf.kron_approx(P, c[0], c[1], bc, r)
        Am, Bm, sigm, epsm = many[i]
        say(f"[kron many {i}] {tuple(P.shape)} r={r} eps {eps:.6e}")
        assert torch.equal(A, Am) and torch.equal(B, Bm)
        assert np.array_equal(sig, sigm) and eps == epsm
