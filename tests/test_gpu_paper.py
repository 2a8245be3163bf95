"""The paper-shaped sweep (Section 4's experiment shape on synthetic
stand-ins): Theorem 1's error falls with the number of terms, and the
restoration reached with s terms is what the oracle reaches with the same
factors."""

import numpy as np
import pytest

import oracle as O
import synth as S
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    import torch
    assert torch.cuda.is_available()
    from paper_1901_00913_amd import sfista
    sfista.lib()
    return sfista


@pytest.mark.parametrize("kind", ["defocus", "motion"])
def test_sweep_over_terms(sf, kind):
    p = S.paper_problems(128, iters=30)[kind]
    l, q = p.center
    eps_prev = np.inf
    for s in range(1, 6):
        A, B, sig, eps = sf.kron_approx(dev(p.psf), l, q, p.bc, s)
        K, H, osig, oeps, _, _ = O.kron_approx64(p.psf, l, q, p.bc, s)
        L = O.lipschitz_power(K, H, p.v0, 200)
        sol = sf.Solver(dev(p.bobs), A, B, lam=p.lam, L=L, precision="fp64")
        X, rep = sol.solve(p.iters)
        sol.close()
        ref = O.sfista64(K, H, p.bobs, p.lam, L, p.iters)
        eta = rel(host(X), p.x_true)
        say(f"[paper {kind}] s={s} eps_s={eps:.4e} eta={eta:.4f} vs oracle {rel(host(X), ref):.2e}")
        # Theorem 1's error to FP64 rounding of the SVD (relative to sigma_1)
        assert abs(eps - oeps) <= 1e-9 * oeps + 1e-12 * osig[0]
        assert eps <= eps_prev * (1 + 1e-12) + 1e-12 * osig[0]
        assert rel(host(X), ref) < 1e-10
        eps_prev = eps
