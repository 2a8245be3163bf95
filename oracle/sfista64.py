"""FP64 CPU oracle for structured FISTA (sFISTA) image restoration.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  This module is a plain, slow,
obviously-correct float64 restatement of what the method computes.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may use
it; the GPU library never imports, links or calls it, and it imports nothing
from the GPU library.

Notation follows the paper (Chen, Nagy, Xi, Yu, "Structured FISTA for Image
Restoration"):

* ``A`` is the exact ``N x N`` blurring matrix (``N = m n``), ``b = vec(B)``
  with ``vec`` stacking columns (Section 1, "matrix equation");
* the Kronecker approximation is ``A_s = sum_i K_i (x) H_i`` with right
  factors ``K_i`` (``n x n``) and left factors ``H_i`` (``m x m``), so that
  ``A_s vec(X) = vec(sum_i H_i X K_i^T)`` (Section 1; Theorem 3's identities);
* ``s`` is the number of Kronecker terms, ``lam`` the Tikhonov parameter
  ``lambda`` of the objective ``1/2 ||A x - b||^2 + lambda^2/2 ||x||^2``.

Readings taken where the paper is ambiguous (each is pinned by a test):

* the left factor ``H_i`` (``m x m``, acting on the row index) is built from
  the left singular vector ``u_i`` and the row centre ``l``; the right factor
  ``K_i`` from ``v_i`` and the column centre ``q`` (Section 2 prints the
  opposite pairing, which does not reproduce the blur when the PSF and the
  image share one orientation);
* the SVD is taken of the weighted PSF ``P_bar`` of Theorem 1, not of ``P``;
* for the reflexive boundary, ``R`` is the upper Cholesky factor with
  ``R^T R = M`` (``M`` the symmetric Toeplitz matrix with first row
  ``[n, 1, 0, 1, 0, ...]``), ``P_bar = R_m P R_n^T``; for non-square PSFs the
  row side uses ``m`` and the row centre, the column side ``n`` and ``q``;
* ``L = lambda_max(A_s^T A_s)``, the Lipschitz constant of the data term of
  the approximate problem (Theorem 2 needs that one);
* indices are 0-based in code; ``toep`` and ``hank`` take the paper's 1-based
  column index ``j`` so that the printed examples of Section 2 apply directly.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular

BC_ZERO = 0
BC_REFLEXIVE = 1


# --------------------------------------------------------------------------
# Section 2: structured factors
# --------------------------------------------------------------------------

def toep(c, j: int) -> np.ndarray:
    """Banded Toeplitz matrix whose ``j``-th column (1-based) equals ``c``
    (Section 2, definition of ``toep(c, j)`` and its 5x5 example): column
    ``col`` is ``c`` moved down by ``col - (j - 1)`` rows, zero-filled."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    i = np.arange(n)[:, None]
    col = np.arange(n)[None, :]
    src = i - (col - (j - 1))
    ok = (src >= 0) & (src < n)
    return np.where(ok, c[np.clip(src, 0, n - 1)], 0.0)


def hank(c, j: int) -> np.ndarray:
    """Banded Hankel matrix whose first row is ``[c_{j+1}, ..., c_n, 0, ..., 0]``
    and whose last column is ``[0, ..., 0, c_1, ..., c_{j-1}]^T`` (1-based
    ``j``; Section 2, definition of ``hank(c, j)`` and its 5x5 example).  A
    Hankel matrix is constant along anti-diagonals ``d = i + k``: the first
    row gives ``d < n`` and the last column ``d >= n - 1``."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    first_row = np.zeros(n)
    tail = c[j:]                       # c_{j+1} .. c_n
    first_row[:tail.shape[0]] = tail
    last_col = np.zeros(n)
    head = c[:max(0, j - 1)]           # c_1 .. c_{j-1}
    if head.shape[0]:
        last_col[n - head.shape[0]:] = head
    antidiag = np.concatenate([first_row, last_col[1:]])   # value on anti-diagonal d
    d = np.arange(n)[:, None] + np.arange(n)[None, :]
    return antidiag[d]


def factor(c, center0: int, bc: int) -> np.ndarray:
    """``toep(c, j)`` (zero boundary) or ``toep(c, j) + hank(c, j)``
    (reflexive boundary) with ``j = center0 + 1`` (Section 2)."""
    j = center0 + 1
    if bc == BC_ZERO:
        return toep(c, j)
    if bc == BC_REFLEXIVE:
        return toep(c, j) + hank(c, j)
    raise ValueError("unknown boundary condition")


# --------------------------------------------------------------------------
# Section 2: the exact blur (definition of A through point sources)
# --------------------------------------------------------------------------

def _extend(idx: np.ndarray, size: int, bc: int) -> np.ndarray:
    """Source index of extended position ``idx``; -1 where the zero boundary
    puts a zero.  Reflexive = half-sample symmetric: x[-1-t] = x[t]."""
    if bc == BC_ZERO:
        return np.where((idx >= 0) & (idx < size), idx, -1)
    t = np.mod(idx, 2 * size)
    return np.where(t < size, t, 2 * size - 1 - t)


def blur_direct(x: np.ndarray, psf: np.ndarray, l: int, q: int, bc: int) -> np.ndarray:
    """Spatially invariant blur by its definition:
    ``B[i, j] = sum_{a, b} P[a, b] * X_ext[i - (a - l), j - (b - q)]``."""
    m, n = x.shape
    ii = np.arange(m)
    jj = np.arange(n)
    out = np.zeros((m, n))
    for a in range(m):
        rows = _extend(ii - (a - l), m, bc)
        for b in range(n):
            w = psf[a, b]
            if w == 0.0:
                continue
            cols = _extend(jj - (b - q), n, bc)
            src = x[np.maximum(rows, 0)][:, np.maximum(cols, 0)]
            mask = (rows[:, None] >= 0) & (cols[None, :] >= 0)
            out += w * np.where(mask, src, 0.0)
    return out


def vec(x: np.ndarray) -> np.ndarray:
    """Column-stacking ``vec`` (Section 1)."""
    return np.asarray(x).reshape(-1, order="F")


def unvec(v: np.ndarray, m: int, n: int) -> np.ndarray:
    return np.asarray(v).reshape((m, n), order="F")


def dense_A_pointsource(psf: np.ndarray, l: int, q: int, bc: int) -> np.ndarray:
    """Blurring matrix built column by column: column ``t`` is the blurred
    image of the point source at ``vec`` position ``t`` (Section 2).  Tiny
    sizes only."""
    m, n = psf.shape
    a = np.zeros((m * n, m * n))
    for t in range(m * n):
        e = np.zeros(m * n)
        e[t] = 1.0
        a[:, t] = vec(blur_direct(unvec(e, m, n), psf, l, q, bc))
    return a


def dense_A(psf: np.ndarray, l: int, q: int, bc: int) -> np.ndarray:
    """Same matrix as :func:`dense_A_pointsource`, assembled by scattering each
    PSF weight onto the source pixel it reads (the definition of
    :func:`blur_direct` read as a sum over matrix entries)."""
    m, n = psf.shape
    a = np.zeros((m * n, m * n))
    ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    out_idx = (ii + m * jj).ravel()
    for pa in range(m):
        rows = _extend(ii - (pa - l), m, bc)
        for pb in range(n):
            w = psf[pa, pb]
            if w == 0.0:
                continue
            cols = _extend(jj - (pb - q), n, bc)
            ok = ((rows >= 0) & (cols >= 0)).ravel()
            src_idx = (rows + m * cols).ravel()
            np.add.at(a, (out_idx[ok], src_idx[ok]), w)
    return a


# --------------------------------------------------------------------------
# Theorem 1: weighted PSF and the Kronecker approximation
# --------------------------------------------------------------------------

def gram_reflexive(n: int) -> np.ndarray:
    """Symmetric Toeplitz matrix with first row ``[n, 1, 0, 1, 0, 1, ...]``."""
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    return np.where(d == 0, float(n), np.where(d % 2 == 1, 1.0, 0.0))


def weight_matrix(size: int, center0: int, bc: int) -> np.ndarray:
    """``R`` of Theorem 1 (upper triangular, ``R^T R`` = Gram of the factor map):
    ``diag(sqrt(size - |i - center|))`` for the zero boundary, the upper
    Cholesky factor of :func:`gram_reflexive` for the reflexive boundary."""
    if bc == BC_ZERO:
        return np.diag(np.sqrt(size - np.abs(np.arange(size) - center0)).astype(np.float64))
    if bc == BC_REFLEXIVE:
        return np.linalg.cholesky(gram_reflexive(size)).T
    raise ValueError("unknown boundary condition")


def kron_approx64(psf: np.ndarray, l: int, q: int, bc: int, s: int):
    """Kronecker approximation ``A_s = sum_{i<=s} K_i (x) H_i`` (Section 2).

    Steps: ``P_bar = R_m P R_n^T`` (Theorem 1); SVD ``P_bar = U Sigma V^T``;
    signs fixed so that the largest-magnitude entry of each ``u_i`` is
    positive (lowest index on ties); generators
    ``h_i = sqrt(sigma_i) R_m^{-1} u_i`` and ``k_i = sqrt(sigma_i) R_n^{-1} v_i``;
    ``H_i = F(h_i, l)``, ``K_i = F(k_i, q)``; ``eps_s`` is the Frobenius norm of
    the discarded SVD tail, which equals ``||A - A_s||_F`` by Theorem 1.

    Returns ``(K, H, sigma, eps_s, h, k)`` with ``K`` of shape ``(s, n, n)``,
    ``H`` of shape ``(s, m, m)`` and ``sigma`` all singular values of ``P_bar``.
    """
    psf = np.asarray(psf, dtype=np.float64)
    m, n = psf.shape
    if not (1 <= s <= min(m, n)):
        raise ValueError("s must lie in [1, min(m, n)]")
    rm = weight_matrix(m, l, bc)
    rn = weight_matrix(n, q, bc)
    pbar = rm @ psf @ rn.T
    u, sig, vt = np.linalg.svd(pbar)
    v = vt.T.copy()
    u = u.copy()
    for i in range(sig.shape[0]):
        idx = int(np.argmax(np.abs(u[:, i])))
        if u[idx, i] < 0.0:
            u[:, i] = -u[:, i]
            v[:, i] = -v[:, i]
    hs = np.empty((s, m))
    ks = np.empty((s, n))
    H = np.empty((s, m, m))
    K = np.empty((s, n, n))
    for i in range(s):
        hs[i] = math.sqrt(sig[i]) * solve_triangular(rm, u[:, i], lower=False)
        ks[i] = math.sqrt(sig[i]) * solve_triangular(rn, v[:, i], lower=False)
        H[i] = factor(hs[i], l, bc)
        K[i] = factor(ks[i], q, bc)
    eps_s = float(np.sqrt(np.sum(sig[s:] ** 2)))
    return K, H, sig, eps_s, hs, ks


def kron_sum_dense(K: np.ndarray, H: np.ndarray) -> np.ndarray:
    """``A_s = sum_i K_i (x) H_i`` as a dense ``N x N`` matrix."""
    return sum(np.kron(K[i], H[i]) for i in range(K.shape[0]))


# --------------------------------------------------------------------------
# Matrix model of Section 1 ("matrix equation", "matrix minimization model")
# --------------------------------------------------------------------------

def apply_As(K, H, X):
    """``sum_i H_i X K_i^T`` (= ``A_s vec(X)`` reshaped)."""
    return sum(H[i] @ X @ K[i].T for i in range(K.shape[0]))


def apply_AsT(K, H, R):
    """``sum_j H_j^T R K_j`` (= ``A_s^T vec(R)`` reshaped)."""
    return sum(H[j].T @ R @ K[j] for j in range(K.shape[0]))


def phi_s(K, H, B, X, lam):
    """Objective of the matrix minimization model."""
    r = apply_As(K, H, X) - B
    return 0.5 * float(np.sum(r * r)) + 0.5 * lam * lam * float(np.sum(X * X))


def phi_dense(A, b, x, lam):
    """Objective of the vector minimization model."""
    r = A @ x - b
    return 0.5 * float(r @ r) + 0.5 * lam * lam * float(x @ x)


# --------------------------------------------------------------------------
# Algorithm 1 (FISTA on the vector model) and Algorithm 2 (sFISTA)
# --------------------------------------------------------------------------

def momentum(t_k: float) -> float:
    """Step 2 of Algorithms 1 and 2: ``t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2``."""
    return (1.0 + math.sqrt(1.0 + 4.0 * t_k * t_k)) / 2.0


def fista_dense(A, b, lam, L, iters, x0=None, nonneg=False, history=None):
    """Algorithm 1 on ``min 1/2||A x - b||^2 + lam^2/2 ||x||^2``.

    Step 1: ``x_k = (L y_k - A^T(A y_k - b)) / (L + lam^2)`` (projected on
    ``x >= 0`` when ``nonneg``); Step 2: ``t_{k+1}``; Step 3:
    ``y_{k+1} = x_k + (t_k - 1)/t_{k+1} (x_k - x_{k-1})``.  ``history``, if a
    list, receives every ``x_k``.
    """
    N = A.shape[1]
    x_prev = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    y = x_prev.copy()
    t = 1.0
    x = x_prev
    for _ in range(iters):
        x = (L * y - A.T @ (A @ y - b)) / (L + lam * lam)
        if nonneg:
            x = np.maximum(x, 0.0)
        t_next = momentum(t)
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        if history is not None:
            history.append(x.copy())
        x_prev = x
        t = t_next
    return x


def sfista64(K, H, B, lam, L, iters, X0=None, nonneg=False, history=None):
    """Algorithm 2 (sFISTA) on the matrix minimization model.

    Step 1: ``X_k = (L Y_k - sum_j H_j^T (sum_i H_i Y_k K_i^T - B) K_j) / (L + lam^2)``
    (projected on ``X >= 0`` when ``nonneg``); Step 2: ``t_{k+1}``; Step 3:
    ``Y_{k+1} = X_k + (t_k - 1)/t_{k+1} (X_k - X_{k-1})``; the loop runs a
    fixed number of iterations and returns ``X_iters``.
    """
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    x_prev = np.zeros((m, n)) if X0 is None else np.array(X0, dtype=np.float64)
    y = x_prev.copy()
    t = 1.0
    x = x_prev
    for _ in range(iters):
        resid = apply_As(K, H, y) - B
        x = (L * y - apply_AsT(K, H, resid)) / (L + lam * lam)
        if nonneg:
            x = np.maximum(x, 0.0)
        t_next = momentum(t)
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        if history is not None:
            history.append(x.copy())
        x_prev = x
        t = t_next
    return x


def sfista64_grad(K, H, B, lam, L, iters, x_true, X0=None):
    """Unrolled Algorithm 2 as a differentiable map (the differentiable form).

    Runs ``iters`` unconstrained iterations from ``X0`` (zero by default)
    with ``L`` held fixed, takes the loss ``mean((X_iters - x_true)^2)`` and
    differentiates it in reverse mode through every step of the iteration:

    * Step 1 written as ``R_k = sum_i H_i Y_k K_i^T - B``,
      ``G_k = sum_j H_j^T R_k K_j``, ``X_k = (L Y_k - G_k) / (L + lam^2)``;
    * Step 3 as ``Y_{k+1} = (1 + beta_k) X_k - beta_k X_{k-1}`` with
      ``beta_k = (t_k - 1) / t_{k+1}`` from Step 2 (data-independent).

    With ``s = L + lam^2`` and adjoints written with a bar, for k = iters..1:
    ``Xbar_k = [k = iters] dloss/dX + (1 + beta_k) Ybar_{k+1} - beta_{k+1} Ybar_{k+2}``,
    ``Gbar = -Xbar_k / s``, ``Rbar = sum_j H_j Gbar K_j^T``,
    ``Ybar_k = (L / s) Xbar_k + sum_i H_i^T Rbar K_i``,
    ``dH_j += R_k K_j Gbar^T + Rbar K_j Y_k^T``,
    ``dK_j += R_k^T H_j Gbar + Rbar^T H_j Y_k``,
    ``dlam += <Xbar_k, -2 lam X_k / s>``.

    Returns ``(loss, dK, dH, dlam)``.  Every iterate is kept (no
    checkpointing): this is the plain reference.
    """
    B = np.asarray(B, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    m, n = B.shape
    r = K.shape[0]
    s = L + lam * lam
    xs = [np.zeros((m, n)) if X0 is None else np.array(X0, dtype=np.float64)]
    ys, rs, betas = [None], [None], [0.0]
    y = xs[0].copy()
    t = 1.0
    for _ in range(iters):
        resid = apply_As(K, H, y) - B
        x = (L * y - apply_AsT(K, H, resid)) / s
        t_next = momentum(t)
        beta = (t - 1.0) / t_next
        ys.append(y)
        rs.append(resid)
        betas.append(beta)
        y = x + beta * (x - xs[-1])
        xs.append(x)
        t = t_next
    X = xs[iters]
    loss = float(np.mean((X - x_true) ** 2))
    dK = np.zeros_like(K)
    dH = np.zeros_like(H)
    dlam = 0.0
    ybar1 = np.zeros((m, n))   # Ybar_{k+1}
    ybar2 = np.zeros((m, n))   # Ybar_{k+2}
    for k in range(iters, 0, -1):
        xbar = (1.0 + betas[k]) * ybar1
        if k + 1 <= iters:
            xbar = xbar - betas[k + 1] * ybar2
        if k == iters:
            xbar = xbar + 2.0 * (X - x_true) / (m * n)
        gbar = -xbar / s
        dlam += float(np.sum(xbar * (-2.0 * lam / s) * xs[k]))
        rbar = apply_As(K, H, gbar)
        ybar = (L / s) * xbar + apply_AsT(K, H, rbar)
        for j in range(r):
            dH[j] += rs[k] @ K[j] @ gbar.T + rbar @ K[j] @ ys[k].T
            dK[j] += rs[k].T @ H[j] @ gbar + rbar.T @ H[j] @ ys[k]
        ybar2 = ybar1
        ybar1 = ybar
    return loss, dK, dH, dlam


def sfista64_loss(K, H, B, lam, L, iters, x_true, X0=None):
    """The loss of :func:`sfista64_grad` alone (forward only)."""
    X = sfista64(K, H, B, lam, L, iters, X0=X0)
    return float(np.mean((X - x_true) ** 2))


# --------------------------------------------------------------------------
# Lipschitz constant and closed forms
# --------------------------------------------------------------------------

def lipschitz_dense(A) -> float:
    """``L = lambda_max(A^T A)`` by a symmetric eigensolver."""
    return float(np.linalg.eigvalsh(A.T @ A)[-1])


def lipschitz_power(K, H, V0, steps: int) -> float:
    """Power iteration for ``lambda_max(A_s^T A_s)`` on the matrix form:
    ``V <- V / ||V||``; ``W = sum_j H_j^T (sum_i H_i V K_i^T) K_j``;
    the estimate is ``||W||_F``; repeat with ``V = W``."""
    v = np.asarray(V0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    est = 0.0
    for _ in range(steps):
        w = apply_AsT(K, H, apply_As(K, H, v))
        est = float(np.linalg.norm(w))
        v = w / est
    return est


def lipschitz_lanczos(K, H, V0, steps: int) -> float:
    """Lanczos estimate of ``lambda_max(A_s^T A_s)`` (Section 4 takes L from
    a Lanczos estimate of the operator norm; on ``A_s^T A_s`` the symmetric
    Lanczos process is, in exact arithmetic, the Golub-Kahan
    bidiagonalisation of ``A_s``).  From ``q_1 = V0 / ||V0||`` and
    ``q_0 = 0``, ``beta_0 = 0``, step ``j`` forms ``w = A_s^T A_s q_j``,
    ``alpha_j = <q_j, w>``, ``w -= alpha_j q_j + beta_{j-1} q_{j-1}``,
    ``beta_j = ||w||`` and ``q_{j+1} = w / beta_j``.  The estimate is the
    largest eigenvalue of the symmetric tridiagonal matrix with diagonal
    ``alpha_1..alpha_k`` and off-diagonal ``beta_1..beta_{k-1}``.  No
    reorthogonalisation.  The process stops early when ``beta_j`` vanishes
    (the Krylov space is invariant, and its Ritz values are exact)."""
    q = np.asarray(V0, dtype=np.float64)
    q = q / np.linalg.norm(q)
    q_prev = np.zeros_like(q)
    beta_prev = 0.0
    alpha, beta = [], []
    for _ in range(steps):
        w = apply_AsT(K, H, apply_As(K, H, q))
        a = float(np.sum(q * w))
        w = w - a * q - beta_prev * q_prev
        b = float(np.linalg.norm(w))
        alpha.append(a)
        if b == 0.0:
            break
        beta.append(b)
        q_prev, q, beta_prev = q, w / b, b
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def closed_form(A, b, lam):
    """Minimiser of the (unconstrained) vector model: the solution of the
    optimality condition ``A^T(A x - b) + lam^2 x = 0`` (Theorem 4's proof)."""
    N = A.shape[1]
    c = cho_factor(A.T @ A + lam * lam * np.eye(N))
    return cho_solve(c, A.T @ b)


def eta(x, x_true):
    """Relative error ``||x - x*|| / ||x*||`` (Section 4)."""
    return float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true))


def gamma(Ax, b):
    """Relative residual ``||A x - b|| / ||b||`` (Section 4), given ``A x``."""
    return float(np.linalg.norm(Ax - b) / np.linalg.norm(b))
