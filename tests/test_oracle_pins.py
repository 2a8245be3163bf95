"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them re-types an oracle formula:
each compares the oracle with a printed example, a theorem, a closed form, a
special case or an independent construction.
"""

import math
import os

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle as O
import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden_5x5():
    mats = {}
    with open(os.path.join(GOLDEN, "toep_hank_5x5.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        name, j = lines[i][0], int(lines[i][1])
        rows = np.array([[int(v) for v in lines[i + 1 + t]] for t in range(5)])
        mats[name] = (j, rows)
        i += 6
    return mats


@pytest.mark.parametrize("which", ["toep", "hank"])
def test_toep_hank_match_printed_examples(which):
    """Section 2 prints toep(c,4) and hank(c,3) for a 5-vector c."""
    j, idx = _read_golden_5x5()[which]
    c = np.array([2.0, 3.0, 5.0, 7.0, 11.0])           # distinct values expose any index slip
    expect = np.where(idx > 0, c[np.maximum(idx - 1, 0)], 0.0)
    got = O.toep(c, j) if which == "toep" else O.hank(c, j)
    assert np.array_equal(got, expect)


def test_kronecker_identities():
    """The two identities used in the proof of Theorem 3, with the
    column-stacking vec of Section 1."""
    rng = np.random.default_rng(0)
    m, n = 5, 4
    H = rng.standard_normal((m, m))
    K = rng.standard_normal((n, n))
    Z = rng.standard_normal((m, n))
    lhs = np.kron(K, H) @ O.vec(Z)
    assert np.allclose(lhs, O.vec(H @ Z @ K.T), rtol=0, atol=1e-14)
    assert np.array_equal(np.kron(K, H).T, np.kron(K.T, H.T))


CASES = [(6, 6, 3, 3), (6, 6, 2, 4), (7, 5, 3, 1), (8, 8, 4, 4), (9, 7, 0, 6)]


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("m,n,l,q", CASES)
def test_blur_constructions_agree(bc, m, n, l, q):
    """Three independent constructions of the blur: point-source columns
    (Section 2), scattered PSF weights, and the FFT convolution of the extended
    image used by the input generator."""
    psf = S.gaussian_psf(m, n, (1.0, 2.0), 30.0, (l, q))
    a_ps = O.dense_A_pointsource(psf, l, q, bc)
    a_sc = O.dense_A(psf, l, q, bc)
    assert np.array_equal(a_ps, a_sc) or np.abs(a_ps - a_sc).max() < 1e-15
    x = np.random.default_rng(1).standard_normal((m, n))
    b_fft = S.blur(x, psf, (l, q), bc)
    assert np.abs(a_sc @ O.vec(x) - O.vec(b_fft)).max() < 1e-13


def test_reflexive_extension_is_half_sample():
    """Reflexive boundary: the pixel just outside the border mirrors the border
    pixel itself (x[-1] = x[0]); a 1-pixel shift PSF exposes it."""
    m, n = 5, 4
    x = np.arange(m * n, dtype=float).reshape(m, n)
    psf = np.zeros((m, n))
    psf[3, 2] = 1.0                 # centre (2, 2): output reads x[i-1, j]
    out = O.blur_direct(x, psf, 2, 2, O.BC_REFLEXIVE)
    assert np.array_equal(out[0], x[0])
    assert np.array_equal(out[1:], x[:-1])


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("m,n,l,q", CASES)
def test_separable_psf_gives_single_kronecker_term(bc, m, n, l, q):
    """A rank-one PSF c d^T blurs separably: A = F(d, q) (x) F(c, l), the
    structure claimed for K_i and H_i in Section 2 (toep for the zero
    boundary, toep + hank for the reflexive one)."""
    rng = np.random.default_rng(2)
    c, d = rng.random(m), rng.random(n)
    A = O.dense_A(np.outer(c, d), l, q, bc)
    assert np.abs(A - np.kron(O.factor(d, q, bc), O.factor(c, l, bc))).max() < 1e-15


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("size,center", [(6, 0), (6, 3), (7, 2), (7, 6), (10, 5)])
def test_factor_gram_equals_theorem1_weights(bc, size, center):
    """||F(c, l)||_F^2 = c^T R^T R c: the weights of Theorem 1 are the Gram
    matrix of the factor map (diag(n - |j - l|), resp. Toeplitz [n,1,0,1,...])."""
    rng = np.random.default_rng(3)
    R = O.weight_matrix(size, center, bc)
    for _ in range(5):
        c = rng.standard_normal(size)
        assert math.isclose(np.sum(O.factor(c, center, bc) ** 2), c @ (R.T @ R) @ c,
                            rel_tol=1e-13)


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("m,n,l,q", CASES)
def test_theorem1_error_identity(bc, m, n, l, q):
    """Theorem 1: ||A - A_s||_F equals the discarded tail of the SVD of P_bar,
    for every s; at s = min(m, n) the sum is exact (the Kronecker
    decomposition of Section 2)."""
    psf = S.gaussian_psf(m, n, (1.0, 2.0), 30.0, (l, q))
    A = O.dense_A(psf, l, q, bc)
    scale = np.linalg.norm(A)
    for s in range(1, min(m, n) + 1):
        K, H, sig, eps, _, _ = O.kron_approx64(psf, l, q, bc, s)
        err = np.linalg.norm(A - O.kron_sum_dense(K, H))
        assert abs(err - eps) <= 1e-12 * scale
    assert np.abs(A - O.kron_sum_dense(K, H)).max() < 1e-13


def test_paper_printed_pairing_is_not_the_blur():
    """Reading check: building the right factor from u (the pairing printed in
    Section 2) does not reproduce the blur of a non-symmetric PSF whose image
    shares the PSF's orientation; the pairing used by the oracle does."""
    m = n = 6
    l, q = 3, 2
    rng = np.random.default_rng(4)
    c, d = rng.random(m), rng.random(n)
    A = O.dense_A(np.outer(c, d), l, q, 0)
    ours = np.kron(O.factor(d, q, 0), O.factor(c, l, 0))
    printed = np.kron(O.factor(c, l, 0), O.factor(d, q, 0))
    assert np.abs(A - ours).max() < 1e-15
    assert np.abs(A - printed).max() > 1e-2


@pytest.mark.parametrize("bc", [0, 1])
def test_axis_aligned_gaussian_is_exact_at_rank_one(bc):
    """theta = 0 makes the Gaussian separable: sigma_2(P_bar) = 0 and A_1 = A."""
    m, n = 9, 8
    psf = S.gaussian_psf(m, n, (1.5, 2.5), 0.0)
    A = O.dense_A(psf, m // 2, n // 2, bc)
    K, H, sig, eps, _, _ = O.kron_approx64(psf, m // 2, n // 2, bc, 1)
    assert sig[1] < 1e-14 * sig[0]
    assert np.abs(A - O.kron_sum_dense(K, H)).max() < 1e-15


def _small_problem(m=12, n=10, bc=1, s=3, lam=0.05, nl=0.01, seed=7):
    x = S.make_image(m, n, seed)
    psf = S.gaussian_psf(m, n, (1.2, 2.0), 30.0)
    l, q = m // 2, n // 2
    b = S.blur(x, psf, (l, q), bc)
    bobs = S.add_noise(b, nl, seed + 1)
    K, H, sig, eps, _, _ = O.kron_approx64(psf, l, q, bc, s)
    As = O.kron_sum_dense(K, H)
    return x, psf, K, H, As, bobs, lam


def test_theorem3_sfista_equals_fista_on_As():
    """Theorem 3: sFISTA on the matrix model and FISTA on the vector model
    with A_s produce the same iterates (x_k = vec(X_k))."""
    x, psf, K, H, As, bobs, lam = _small_problem()
    m, n = bobs.shape
    L = O.lipschitz_dense(As)
    hx, hX = [], []
    O.fista_dense(As, O.vec(bobs), lam, L, 200, history=hx)
    O.sfista64(K, H, bobs, lam, L, 200, history=hX)
    gap = max(np.abs(a - O.vec(b)).max() for a, b in zip(hx, hX))
    assert gap < 1e-12


def test_theorem2_rate_bound():
    """Theorem 2 (Beck-Teboulle): Phi_s(X_k) - Phi_s* <= 2 L ||X_0 - x*||^2/(k+1)^2
    for every k, with the exact L and the exact minimiser."""
    x, psf, K, H, As, bobs, lam = _small_problem(lam=0.02)
    b = O.vec(bobs)
    L = O.lipschitz_dense(As)
    xs = O.closed_form(As, b, lam)
    fstar = O.phi_dense(As, b, xs, lam)
    hist = []
    O.sfista64(K, H, bobs, lam, L, 600, history=hist)
    for k, X in enumerate(hist, start=1):
        gap = O.phi_dense(As, b, O.vec(X), lam) - fstar
        assert gap <= 2 * L * (xs @ xs) / (k + 1) ** 2 + 1e-13


@pytest.mark.parametrize("bc", [0, 1])
def test_iterates_converge_to_closed_form(bc):
    """The unconstrained iterates converge to (A_s^T A_s + lam^2 I)^{-1} A_s^T b."""
    x, psf, K, H, As, bobs, lam = _small_problem(m=16, n=16, bc=bc, lam=0.1)
    L = O.lipschitz_dense(As)
    X = O.sfista64(K, H, bobs, lam, L, 3000)
    xs = O.closed_form(As, O.vec(bobs), lam)
    assert np.linalg.norm(O.vec(X) - xs) / np.linalg.norm(xs) < 1e-12


def test_step1_minimises_the_quadratic_model():
    """Step 1 returns the minimiser of Q_L(X, Y): the gradient of Q_L in X,
    A_s^T(A_s Y - b) + L (X - Y) + lam^2 X, vanishes there (Section 3.2)."""
    x, psf, K, H, As, bobs, lam = _small_problem()
    rng = np.random.default_rng(5)
    Y = rng.standard_normal(bobs.shape)
    L = 1.7
    X1 = O.sfista64(K, H, bobs, lam, L, 1, X0=Y)
    g = As.T @ (As @ O.vec(Y) - O.vec(bobs)) + L * (O.vec(X1) - O.vec(Y)) + lam ** 2 * O.vec(X1)
    assert np.abs(g).max() < 1e-13


def test_power_iteration_matches_eigensolver():
    x, psf, K, H, As, bobs, lam = _small_problem()
    v0 = S.power_start(*bobs.shape, seed=11)
    assert math.isclose(O.lipschitz_power(K, H, v0, 400), O.lipschitz_dense(As), rel_tol=1e-10)


def _krylov_ritz_max(M, v0, k):
    """Rayleigh-Ritz on the Krylov space span{v0, M v0, ..., M^(k-1) v0}
    from its definition: an orthonormal basis by QR of the (column-scaled)
    Krylov matrix, then the largest eigenvalue of Q^T M Q."""
    cols, v = [], v0 / np.linalg.norm(v0)
    for _ in range(k):
        cols.append(v)
        v = M @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    return float(np.linalg.eigvalsh(Q.T @ M @ Q)[-1])


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_lanczos_equals_rayleigh_ritz_on_krylov_space(k):
    """k Lanczos steps give the largest Ritz value of the k-dimensional
    Krylov space (the definition of the Lanczos estimate), built here with
    an explicit basis and a dense A_s^T A_s.  k = 1 is the Rayleigh
    quotient of v0."""
    x, psf, K, H, As, bobs, lam = _small_problem()
    M = As.T @ As
    v0 = S.power_start(*bobs.shape, seed=11)
    ref = _krylov_ritz_max(M, O.vec(v0), k)
    if k == 1:
        u = O.vec(v0)
        assert math.isclose(ref, u @ M @ u / (u @ u), rel_tol=1e-13)
    assert math.isclose(O.lipschitz_lanczos(K, H, v0, k), ref, rel_tol=1e-11)


def test_lanczos_converges_to_the_eigenvalue_and_rises_monotonically():
    """Interlacing: the largest Ritz value never falls as the Krylov space
    grows and never exceeds lambda_max(A_s^T A_s) (a dense eigensolver);
    with as many steps as unknowns it reaches it."""
    x, psf, K, H, As, bobs, lam = _small_problem(m=6, n=5, s=2)
    v0 = S.power_start(*bobs.shape, seed=3)
    lmax = O.lipschitz_dense(As)
    prev = -np.inf
    for k in range(1, 13):
        est = O.lipschitz_lanczos(K, H, v0, k)
        assert est >= prev - 1e-13 * lmax and est <= lmax * (1 + 1e-12)
        prev = est
    assert math.isclose(O.lipschitz_lanczos(K, H, v0, 30), lmax, rel_tol=1e-10)


def test_lanczos_rank1_closed_form():
    """r = 1: A_s^T A_s = (K^T K) (x) (H^T H), whose largest eigenvalue is
    ||K||_2^2 ||H||_2^2 (two library SVDs)."""
    rng = np.random.default_rng(5)
    m, n = 20, 30
    K = rng.standard_normal((1, n, n)) / math.sqrt(n)
    H = rng.standard_normal((1, m, m)) / math.sqrt(m)
    ref = (np.linalg.norm(K[0], 2) * np.linalg.norm(H[0], 2)) ** 2
    assert math.isclose(O.lipschitz_lanczos(K, H, rng.standard_normal((m, n)), 120), ref, rel_tol=1e-9)


def test_lanczos_stops_on_an_invariant_space():
    """Scaled identities: every start vector is an eigenvector of
    A_s^T A_s = (a b)^2 I, so the first step's residual vanishes and the
    estimate is (a b)^2, however many steps are asked for (a step past the
    vanishing residual would divide by zero).  The constant start and these
    scales keep every operation exact in binary floating point."""
    m, n, a, b = 4, 4, 1.5, 0.5
    K = (a * np.eye(n))[None]
    H = (b * np.eye(m))[None]
    v0 = np.ones((m, n))
    assert O.lipschitz_lanczos(K, H, v0, 10) == (a * b) ** 2


def test_lanczos_beats_power_on_a_blur():
    """On a reflexive Gaussian blur (slowly separating top eigenvalues) 10
    Lanczos steps land closer to lambda_max than 30 power steps."""
    x, psf, K, H, As, bobs, lam = _small_problem(m=24, n=20, s=3)
    v0 = S.power_start(*bobs.shape, seed=11)
    lmax = O.lipschitz_dense(As)
    lz = O.lipschitz_lanczos(K, H, v0, 10)
    pw = O.lipschitz_power(K, H, v0, 30)
    assert pw <= lmax * (1 + 1e-12) and lz <= lmax * (1 + 1e-12)
    assert lmax - lz < lmax - pw


def test_theorem4_error_falls_with_rank():
    """Theorem 4: the gap |Phi(x_k) - Phi(x*)| is bounded by a decaying FISTA
    term plus c0 eps_s; eps_s and the plateau of the gap fall as s grows."""
    m = n = 12
    bc = 1
    x = S.make_image(m, n, 3)
    psf = S.gaussian_psf(m, n, (1.5, 3.0), 30.0)
    l, q = m // 2, n // 2
    A = O.dense_A(psf, l, q, bc)
    b = A @ O.vec(x)
    bobs = b + 0.01 * np.linalg.norm(b) * np.random.default_rng(9).standard_normal(b.shape) / math.sqrt(b.size)
    lam = 0.05
    xstar = O.closed_form(A, bobs, lam)
    fstar = O.phi_dense(A, bobs, xstar, lam)
    eps_prev, gap_prev = np.inf, np.inf
    for s in (1, 2, 3, 4):
        K, H, sig, eps, _, _ = O.kron_approx64(psf, l, q, bc, s)
        As = O.kron_sum_dense(K, H)
        X = O.sfista64(K, H, O.unvec(bobs, m, n), lam, O.lipschitz_dense(As), 2000)
        gap = abs(O.phi_dense(A, bobs, O.vec(X), lam) - fstar)
        assert eps < eps_prev and gap < gap_prev
        eps_prev, gap_prev = eps, gap


def test_nonneg_variant_reaches_bounded_least_squares():
    """With the x >= 0 constraint the projected step converges to the
    minimiser of 1/2||A_s x - b||^2 + lam^2/2||x||^2 over x >= 0, computed
    independently as a bounded least-squares problem on [A_s; lam I]."""
    x, psf, K, H, As, bobs, lam = _small_problem(m=10, n=10, lam=0.1, nl=0.2, seed=3)
    N = As.shape[0]
    L = O.lipschitz_dense(As)
    X = O.sfista64(K, H, bobs, lam, L, 4000, nonneg=True)
    aug = np.vstack([As, lam * np.eye(N)])
    rhs = np.concatenate([O.vec(bobs), np.zeros(N)])
    ref = lsq_linear(aug, rhs, bounds=(0.0, np.inf), tol=1e-14, method="bvls").x
    assert (X >= 0).all()
    assert np.linalg.norm(O.vec(X) - ref) / np.linalg.norm(ref) < 1e-8


def test_generators():
    """Input generator contracts: exact noise level, normalised PSF peaked at
    the centre, image in [0, 1], reproducible seeds."""
    p = S.config(1, n=32)
    e = p.bobs - p.b
    assert math.isclose(np.linalg.norm(e) / np.linalg.norm(p.b), p.noise_level, rel_tol=1e-12)
    assert math.isclose(p.psf.sum(), 1.0, rel_tol=1e-12)
    assert np.unravel_index(np.argmax(p.psf), p.psf.shape) == p.center
    assert p.x_true.min() >= 0 and p.x_true.max() <= 1
    q = S.config(1, n=32)
    assert np.array_equal(p.bobs, q.bobs)
    mp = S.motion_psf(33, 33, 11.0, 30.0)
    assert math.isclose(mp.sum(), 1.0, rel_tol=1e-12) and mp[16, 16] > 0
