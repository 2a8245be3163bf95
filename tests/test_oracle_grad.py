"""Pins of the oracle's gradient of the unrolled iteration (the
differentiable form): central finite differences of the forward oracle and a
one-iteration closed form.  CPU only."""

import numpy as np
import pytest

import oracle as O


def _case(m=7, n=6, r=2, seed=5):
    rng = np.random.default_rng(seed)
    K = rng.standard_normal((r, n, n)) / np.sqrt(n)
    H = rng.standard_normal((r, m, m)) / np.sqrt(m)
    B = rng.standard_normal((m, n))
    x_true = rng.standard_normal((m, n))
    L = 1.05 * O.lipschitz_power(K, H, rng.standard_normal((m, n)), 400)
    return K, H, B, x_true, L


@pytest.mark.parametrize("iters", [1, 2, 3, 12])
def test_gradient_matches_central_differences(iters):
    """Directional derivatives along 16 seeded random directions of the
    factors and lambda jointly, against central differences of the forward
    oracle at h = 1e-4, and the lambda derivative alone.  The central
    difference errs by O(h^2) (about 2e-6 here after 12 iterations, and it
    shrinks 100-fold per 10-fold smaller h), so it is Richardson-extrapolated
    with h / 2, which leaves O(h^4)."""
    K, H, B, x_true, L = _case()
    lam = 0.3
    loss, dK, dH, dlam = O.sfista64_grad(K, H, B, lam, L, iters, x_true)
    assert np.isclose(loss, O.sfista64_loss(K, H, B, lam, L, iters, x_true), rtol=1e-14)
    h = 1e-4

    def central(vK, vH, vl, step):
        fp = O.sfista64_loss(K + step * vK, H + step * vH, B, lam + step * vl, L, iters, x_true)
        fm = O.sfista64_loss(K - step * vK, H - step * vH, B, lam - step * vl, L, iters, x_true)
        return (fp - fm) / (2 * step)

    rng = np.random.default_rng(77)
    for _ in range(16):
        vK = rng.standard_normal(K.shape)
        vH = rng.standard_normal(H.shape)
        vl = rng.standard_normal()
        fd = (4 * central(vK, vH, vl, h / 2) - central(vK, vH, vl, h)) / 3
        an = np.sum(dK * vK) + np.sum(dH * vH) + dlam * vl
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an)), (fd, an)
    zK, zH = np.zeros_like(K), np.zeros_like(H)
    fd = (4 * central(zK, zH, 1.0, h / 2) - central(zK, zH, 1.0, h)) / 3
    assert abs(fd - dlam) <= 1e-8 * max(1.0, abs(dlam))


def test_one_iteration_closed_form():
    """From X_0 = 0 one iteration gives X_1 = A_s^T B / (L + lam^2); with
    E = 2 (X_1 - x_true) / (m n) the gradients are dH_j = B K_j E^T / s,
    dK_j = B^T H_j E / s and dlam = -2 lam <E, X_1> / s."""
    K, H, B, x_true, L = _case(m=5, n=8, r=3, seed=9)
    lam = 0.7
    s = L + lam * lam
    X1 = sum(H[j].T @ B @ K[j] for j in range(3)) / s
    E = 2 * (X1 - x_true) / X1.size
    loss, dK, dH, dlam = O.sfista64_grad(K, H, B, lam, L, 1, x_true)
    assert np.isclose(loss, np.mean((X1 - x_true) ** 2), rtol=1e-14)
    for j in range(3):
        np.testing.assert_allclose(dH[j], B @ K[j] @ E.T / s, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(dK[j], B.T @ H[j] @ E / s, rtol=1e-12, atol=1e-15)
    assert np.isclose(dlam, -2 * lam * np.sum(E * X1) / s, rtol=1e-12)


def test_gradient_is_linear_in_the_loss_direction():
    """The backward pass is linear in dloss/dX: scaling x_true's offset
    scales nothing else, so the gradient of loss(x_true = X + c D) for two
    values of c interpolates linearly (a check of the seeding of Xbar)."""
    K, H, B, x_true, L = _case(seed=11)
    lam = 0.2
    X = O.sfista64(K, H, B, lam, L, 5)
    D = np.random.default_rng(3).standard_normal(X.shape)
    g = [O.sfista64_grad(K, H, B, lam, L, 5, X + c * D)[1:] for c in (1.0, 2.0, 3.0)]
    for a, b, c in zip(*g):
        np.testing.assert_allclose(np.asarray(c) - np.asarray(b), np.asarray(b) - np.asarray(a), rtol=1e-9, atol=1e-12)
