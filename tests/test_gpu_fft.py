"""Structured-FFT form against the FP64 oracle: generators, the operator
pair (A_s X, A_s^T A_s X) on random generators over ragged sizes, centres
and both boundaries, the power estimate of L, and full solves.

Tolerances.  The transforms run in FP32 (unit roundoff u = 2^-24).  A
transform of N points perturbs its output by about u log2 N relative to the
norm of its input (each of the log2 N butterfly levels rounds once); A_s X
takes two forward and two inverse transforms along each path, A_s^T A_s X
four of each, and the inputs are rounded to FP32 once per pass.  With
log2 N <= 13 that is below 4 * 14 u = 3.3e-6 for A_s X and 6.7e-6 for
A_s^T A_s X, relative in the Frobenius norm; the tests allow 3x that.  Full
solves are held to the 1e-5 relative target of the reduced-precision modes.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth as S
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available()
    from paper_1901_00913_amd import sfista
    sfista.lib()
    return sfista


def _expand(h, k, l, q, bc):
    """The oracle's factors from generators (Section 2's toep/hank)."""
    H = np.stack([O.factor(h[i], l, bc) for i in range(h.shape[0])])
    K = np.stack([O.factor(k[i], q, bc) for i in range(k.shape[0])])
    return K, H


def _bound(m, n, transforms):
    lg = max(math.log2(max(64, 2 * m)), math.log2(max(64, 2 * n)))
    return 3.0 * transforms * (lg + 1) * U32


@pytest.mark.parametrize("m,n,l,q,bc,sig,theta", [
    (33, 47, 16, 23, O.BC_ZERO, (2.0, 3.0), 20.0),
    (64, 48, 32, 24, O.BC_REFLEXIVE, (3.0, 6.0), 45.0),
])
def test_generators_match_oracle(sf, m, n, l, q, bc, sig, theta):
    """kron_generators against the oracle's generators: each term h_k k_k^T
    (invariant under the joint sign of the pair), sigma and eps_s."""
    r = 4
    psf = S.gaussian_psf(m, n, sigma=sig, theta_deg=theta, center=(l, q))
    h, k, sigma, eps = sf.kron_generators(dev(psf), l, q, bc, r)
    _, _, osig, oeps, oh, ok = O.kron_approx64(psf, l, q, bc, r)
    h, k = host(h), host(k)
    for t in range(r):
        assert rel(np.outer(h[t], k[t]), np.outer(oh[t], ok[t])) < 1e-9
    assert np.allclose(sigma, osig[:r], rtol=1e-11)
    assert math.isclose(eps, oeps, rel_tol=1e-7, abs_tol=1e-14)


@pytest.mark.parametrize("m,n,r,l,q,bc", [
    (1, 1, 1, 0, 0, O.BC_ZERO),
    (5, 7, 2, 2, 3, O.BC_REFLEXIVE),
    (37, 53, 3, 0, 52, O.BC_REFLEXIVE),
    (37, 53, 3, 36, 0, O.BC_ZERO),
    (64, 48, 1, 31, 24, O.BC_REFLEXIVE),
    (200, 136, 3, 100, 68, O.BC_ZERO),
    (257, 130, 2, 128, 65, O.BC_REFLEXIVE),
    (33, 1030, 2, 16, 515, O.BC_REFLEXIVE),
    (600, 40, 2, 599, 20, O.BC_REFLEXIVE),     # 2048-point column transforms
    (9, 2100, 1, 4, 0, O.BC_ZERO),             # 8192-point row transforms (512 threads)
    (2049, 6, 1, 1024, 5, O.BC_REFLEXIVE),     # 8192-point column transforms
])
def test_operator_matches_oracle(sf, m, n, r, l, q, bc):
    """A_s X and A_s^T A_s X with random generators (full Toeplitz and
    Hankel parts, any centre) against the oracle's dense factors."""
    rng = np.random.default_rng(1000 * m + n)
    h = rng.standard_normal((r, m)) / math.sqrt(m)
    k = rng.standard_normal((r, n)) / math.sqrt(n)
    X = rng.standard_normal((m, n))
    K, H = _expand(h, k, l, q, bc)
    Bobs = np.zeros((m, n))
    s = sf.FftSolver(dev(Bobs), dev(h), dev(k), l, q, bc, lam=0.1, L=1.0)
    ax, atax = s.apply(dev(X))
    ref_ax = O.apply_As(K, H, X)
    ref_atax = O.apply_AsT(K, H, ref_ax)
    e1, e2 = rel(host(ax), ref_ax), rel(host(atax), ref_atax)
    b1, b2 = _bound(m, n, 4), _bound(m, n, 8)
    say(f"[fft op {m}x{n} r={r} c=({l},{q}) bc={bc}] AX {e1:.2e} (<{b1:.1e})  AtAX {e2:.2e} (<{b2:.1e})")
    assert e1 < b1
    assert e2 < b2
    s.close()


def test_operator_fullsize_sampled(sf):
    """2048 x 2048, r = 5, reflexive (the benchmark's shape): 64 sampled
    entries of A_s X, each computed by the oracle's factors one at a time,
    and the norm identity <A_s X, A_s X> = <X, A_s^T A_s X>."""
    p = S.config(3)
    l, q = p.center
    h, k, sigma, eps = sf.kron_generators(dev(p.psf), l, q, p.bc, p.r)
    hh, kk = host(h), host(k)
    X = p.x_true
    s = sf.FftSolver(dev(p.bobs), h, k, l, q, p.bc, lam=p.lam, L=1.0)
    ax, atax = s.apply(dev(X))
    ax, atax = host(ax), host(atax)
    rng = np.random.default_rng(77)
    m, n = X.shape
    rows = rng.integers(0, m, 64)
    cols = rng.integers(0, n, 64)
    got, ref = [], []
    for i, j in zip(rows, cols):
        v = 0.0
        for t in range(p.r):
            brow = O.factor(hh[t], l, p.bc)[i]          # row i of B_t
            arow = O.factor(kk[t], q, p.bc)[j]          # row j of A_t
            v += brow @ X @ arow
        got.append(ax[i, j])
        ref.append(v)
    e = rel(np.array(got), np.array(ref))
    lhs, rhs = float(np.sum(ax * ax)), float(np.sum(X * atax))
    say(f"[fft 2048] sampled AX rel {e:.2e}; <AX,AX> vs <X,AtAX> rel {abs(lhs - rhs) / lhs:.2e}")
    assert e < _bound(m, n, 4)
    assert abs(lhs - rhs) <= _bound(m, n, 12) * lhs
    s.close()


def test_power_iteration_matches_oracle(sf):
    p = S.config(2, n=192)
    l, q = p.center
    K, H, _, _, oh, ok = O.kron_approx64(p.psf, l, q, p.bc, p.r)
    s = sf.FftSolver(dev(p.bobs), dev(oh), dev(ok), l, q, p.bc, lam=p.lam, power_iters=40, v0=dev(p.v0))
    Lo = O.lipschitz_power(K, H, p.v0, 40)
    say(f"[fft power] gpu={s.L:.12e} oracle={Lo:.12e} rel={abs(s.L - Lo) / Lo:.2e}")
    assert math.isclose(s.L, Lo, rel_tol=1e-5)
    s.close()


@pytest.mark.parametrize("steps", [0, 12, 30])
def test_lanczos_estimate_matches_oracle(sf, steps):
    """Section 4's Lanczos estimate of L with the transform passes against
    the oracle's Lanczos from the same start (steps = 0: the default 12)."""
    p = S.config(2, n=192)
    l, q = p.center
    K, H, _, _, oh, ok = O.kron_approx64(p.psf, l, q, p.bc, p.r)
    s = sf.FftSolver(dev(p.bobs), dev(oh), dev(ok), l, q, p.bc, lam=p.lam, power_iters=steps, v0=dev(p.v0),
                     l_estimate="lanczos")
    Lo = O.lipschitz_lanczos(K, H, p.v0, steps or 12)
    say(f"[fft lanczos {steps}] gpu={s.L:.12e} oracle={Lo:.12e} rel={abs(s.L - Lo) / Lo:.2e}")
    assert math.isclose(s.L, Lo, rel_tol=1e-5)
    s.close()


@pytest.mark.parametrize("c,nonneg", [(1, False), (1, True), (2, False)])
def test_solve_matches_oracle(sf, c, nonneg):
    """Configurations 1 (64^2, zero boundary, r = 3, 100 iterations) and 2
    (512^2, reflexive, r = 5, 200 iterations) with the oracle's generators
    and L: X within 1e-5 of the oracle's FP64 Algorithm 2."""
    p = S.config(c)
    l, q = p.center
    K, H, _, _, oh, ok = O.kron_approx64(p.psf, l, q, p.bc, p.r)
    L = O.lipschitz_power(K, H, p.v0, 300)
    s = sf.FftSolver(dev(p.bobs), dev(oh), dev(ok), l, q, p.bc, lam=p.lam, L=L, nonneg=nonneg)
    X, rep = s.solve(p.iters)
    X = host(X)
    ref = O.sfista64(K, H, p.bobs, p.lam, L, p.iters, nonneg=nonneg)
    e = rel(X, ref)
    say(f"[fft cfg{c} nonneg={nonneg}] rel err {e:.2e}  phi_s {rep['phi_s']:.6e}")
    assert e < 1e-5
    if nonneg:
        assert (X >= 0).all()
    assert math.isclose(rep["phi_s"], O.phi_s(K, H, p.bobs, ref, p.lam), rel_tol=1e-5)
    assert rep["iters"] == p.iters
    s.close()


def test_step_split_is_bitwise_invariant(sf):
    p = S.config(1)
    l, q = p.center
    _, _, _, _, oh, ok = O.kron_approx64(p.psf, l, q, p.bc, p.r)
    a = sf.FftSolver(dev(p.bobs), dev(oh), dev(ok), l, q, p.bc, lam=p.lam, L=1.5)
    b = sf.FftSolver(dev(p.bobs), dev(oh), dev(ok), l, q, p.bc, lam=p.lam, L=1.5)
    a.step(3)
    a.step(4)
    b.step(7)
    xa, _ = a.solve(0)
    xb, _ = b.solve(0)
    assert np.array_equal(host(xa), host(xb))
    a.close()
    b.close()


def test_config3_fullsize_first_iterations(sf):
    """2048 x 2048, r = 5: GPU generators and the first 5 iterations against
    the oracle's factors and FP64 iterations."""
    p = S.config(3)
    l, q = p.center
    say("[fft cfg3] oracle kron_approx64")
    K, H, _, _, oh, ok = O.kron_approx64(p.psf, l, q, p.bc, p.r)
    L = 1.0 + 1e-3
    h, k, _, _ = sf.kron_generators(dev(p.psf), l, q, p.bc, p.r)
    s = sf.FftSolver(dev(p.bobs), h, k, l, q, p.bc, lam=p.lam, L=L)
    X, rep = s.solve(5)
    say("[fft cfg3] oracle 5 iterations")
    ref = O.sfista64(K, H, p.bobs, p.lam, L, 5)
    e = rel(host(X), ref)
    say(f"[fft cfg3] 5 iterations rel err {e:.3e}")
    assert e < 1e-5
    s.close()


def test_tolerance_stop(sf):
    """solve(tol): the FFT form stops at the first multiple of 10 iterations
    where ||X_k - X_{k-1}|| <= tol ||X_k||.  The iterates carry FP32 transform
    rounding (about 3e-7 of ||X||), so tol = 1e-4 keeps the step norms far
    above it, and the oracle's trajectory is checked with a 5% margin: the
    criterion holds at the stopping iteration and failed 10 iterations
    earlier."""
    p = S.config(1, n=40)
    l, q = p.center
    K, H, _, _, oh, ok = O.kron_approx64(p.psf, l, q, p.bc, p.r)
    L = O.lipschitz_power(K, H, p.v0, 200)
    tol = 1e-4
    s = sf.FftSolver(dev(p.bobs), dev(oh), dev(ok), l, q, p.bc, lam=0.1, L=L)
    X, rep = s.solve(5000, tol=tol)
    k = rep["iters"]
    s.close()
    assert 10 <= k < 5000 and k % 10 == 0
    hist = []
    O.sfista64(K, H, p.bobs, 0.1, L, k, history=hist)
    step = lambda j: np.linalg.norm(hist[j] - hist[j - 1]) / np.linalg.norm(hist[j])
    say(f"[fft tol] stopped at {k}: oracle step {step(-1):.3e}, 10 earlier {step(-11):.3e}")
    assert step(-1) <= tol * 1.05
    if k > 10:
        assert step(-11) > tol * 0.95
    assert rel(host(X), hist[-1]) < 1e-5
