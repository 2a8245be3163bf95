"""Python binding of libsfista.so (argument marshalling only).

Every call forwards device pointers of torch tensors and the current HIP
stream to the C ABI declared in ``include/sfista.h``; all arithmetic runs in
the library's HIP kernels.  PyTorch only allocates device memory and provides
the stream.  There is no fallback: if the shared library is missing or fails
to load, every entry point raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfista.so")

SFISTA_OK = 0
SFISTA_ERR_ARG = -1
SFISTA_ERR_UNSUPPORTED = -2
SFISTA_ERR_NOMEM = -3
SFISTA_ERR_HIP = -4
SFISTA_ERR_NONFINITE = -5

BC_ZERO = 0
BC_REFLEXIVE = 1

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "bf16x3": 4}

EXPORTS = ("kron_approx", "sfista_setup", "sfista_step", "sfista_solve", "sfista_apply",
           "sfista_set_timing", "sfista_kernel_times", "sfista_get_L", "sfista_destroy",
           "sfista_last_error", "sfista_batch_setup", "sfista_batch_solve", "sfista_batch_tiles",
           "sfista_batch_destroy", "sfista_batch_set_tiles", "sfista_diff_setup", "sfista_diff_forward", "sfista_diff_backward",
           "sfista_diff_get_L", "sfista_diff_destroy", "sfista_diff_update", "sfista_release_cached",
           "kron_generators", "sfista_fft_setup", "sfista_fft_step", "sfista_fft_solve", "sfista_fft_apply",
           "sfista_fft_get_L", "sfista_fft_destroy", "kron_approx_batch")

BATCH_AUTOTUNE = 1
BATCH_GRAPH = 2


L_ESTIMATES = {"power": 0, "lanczos": 1}


def _l_estimate(name: str) -> int:
    """``"power"`` (power iteration) or ``"lanczos"`` (Section 4's Lanczos
    estimate); used when ``L`` is not given, with ``power_iters`` steps."""
    if name not in L_ESTIMATES:
        raise ValueError(f"l_estimate must be one of {sorted(L_ESTIMATES)}, not {name!r}")
    return L_ESTIMATES[name]


class SfistaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sfista error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("L", ctypes.c_double), ("precision", ctypes.c_int),
                ("nonneg", ctypes.c_int), ("power_iters", ctypes.c_int), ("pair_state", ctypes.c_int),
                ("x0", ctypes.c_void_p), ("v0", ctypes.c_void_p), ("l_estimate", ctypes.c_int)]


class BatchItem(ctypes.Structure):
    _fields_ = [("Bobs", ctypes.c_void_p), ("m", ctypes.c_int), ("n", ctypes.c_int), ("A", ctypes.c_void_p),
                ("B", ctypes.c_void_p), ("r", ctypes.c_int), ("lambda_", ctypes.c_double), ("L", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("seconds", ctypes.c_double), ("L", ctypes.c_double),
                ("phi_s", ctypes.c_double), ("resid_norm", ctypes.c_double),
                ("bobs_norm", ctypes.c_double), ("x_norm", ctypes.c_double),
                ("resid_rel", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsfista.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1901_00913_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.kron_approx.argtypes = [vp, i, i, i, i, i, i, vp, vp, vp, vp, vp]
    L.sfista_setup.argtypes = [vp, i, i, vp, vp, i, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.sfista_step.argtypes = [vp, i]
    L.sfista_solve.argtypes = [vp, i, d, vp, ctypes.POINTER(Report)]
    L.sfista_apply.argtypes = [vp, vp, vp, vp]
    L.sfista_get_L.argtypes = [vp, ctypes.POINTER(d)]
    L.sfista_set_timing.argtypes = [vp, i]
    L.sfista_kernel_times.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_long)]
    L.sfista_destroy.argtypes = [vp]
    L.sfista_destroy.restype = None
    L.sfista_batch_setup.argtypes = [ctypes.POINTER(BatchItem), i, ctypes.POINTER(Params), i, i, vp,
                                     ctypes.POINTER(vp)]
    L.sfista_batch_solve.argtypes = [vp, i, ctypes.POINTER(vp), ctypes.POINTER(Report)]
    L.sfista_batch_tiles.argtypes = [vp, ctypes.POINTER(i)]
    L.sfista_batch_set_tiles.argtypes = [vp, ctypes.POINTER(i)]
    L.sfista_batch_destroy.argtypes = [vp]
    L.sfista_batch_destroy.restype = None
    L.sfista_diff_setup.argtypes = [ctypes.POINTER(BatchItem), i, i, i, i, vp, ctypes.POINTER(vp)]
    L.sfista_diff_update.argtypes = [vp, ctypes.POINTER(BatchItem), i]
    L.sfista_diff_forward.argtypes = [vp, ctypes.POINTER(vp)]
    L.sfista_diff_backward.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(d)]
    L.sfista_diff_get_L.argtypes = [vp, ctypes.POINTER(d)]
    L.sfista_diff_destroy.argtypes = [vp]
    L.sfista_diff_destroy.restype = None
    L.sfista_release_cached.argtypes = []
    L.kron_generators.argtypes = [vp, i, i, i, i, i, i, vp, vp, vp, vp, vp]
    ip = ctypes.POINTER(i)
    L.kron_approx_batch.argtypes = [i, ctypes.POINTER(vp), ip, ip, ip, ip, ip, ip, ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), vp, vp, vp]
    L.sfista_fft_setup.argtypes = [vp, i, i, vp, vp, i, i, i, i, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.sfista_fft_step.argtypes = [vp, i]
    L.sfista_fft_solve.argtypes = [vp, i, d, vp, ctypes.POINTER(Report)]
    L.sfista_fft_apply.argtypes = [vp, vp, vp, vp]
    L.sfista_fft_get_L.argtypes = [vp, ctypes.POINTER(d)]
    L.sfista_fft_destroy.argtypes = [vp]
    L.sfista_fft_destroy.restype = None
    L.sfista_last_error.argtypes = []
    L.sfista_last_error.restype = ctypes.c_char_p
    for name in ("kron_approx", "sfista_setup", "sfista_step", "sfista_solve", "sfista_apply", "sfista_get_L",
                 "sfista_set_timing", "sfista_kernel_times", "sfista_batch_setup", "sfista_batch_solve",
                 "sfista_batch_tiles", "sfista_batch_set_tiles", "sfista_diff_setup", "sfista_diff_forward", "sfista_diff_backward",
                 "sfista_diff_get_L", "sfista_diff_update", "sfista_release_cached", "kron_generators",
                 "sfista_fft_setup", "sfista_fft_step", "sfista_fft_solve", "sfista_fft_apply", "sfista_fft_get_L"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def release_cached():
    """Return the device memory cached by the library's pools to the system."""
    _check(lib().sfista_release_cached())


def _check(rc: int):
    if rc != SFISTA_OK:
        raise SfistaError(rc, lib().sfista_last_error().decode())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t.data_ptr()


def kron_approx(P, l: int, q: int, bc: int, r: int, stream=None):
    """Kronecker approximation of the blur with PSF ``P`` (m x n, float64, on
    the GPU): returns ``(A, B, sigma, eps_s)`` with ``A`` (r, n, n) right
    factors, ``B`` (r, m, m) left factors (device tensors), ``sigma`` the r
    leading singular values of the weighted PSF and ``eps_s = ||A - A_s||_F``."""
    import torch
    m, n = P.shape
    A = torch.empty((r, n, n), dtype=torch.float64, device=P.device)
    B = torch.empty((r, m, m), dtype=torch.float64, device=P.device)
    sig = (ctypes.c_double * max(r, 1))()
    eps = ctypes.c_double(0.0)
    _check(lib().kron_approx(_dev_f64(P, "P"), m, n, l, q, bc, r, A.data_ptr(), B.data_ptr(),
                             ctypes.cast(sig, ctypes.c_void_p), ctypes.cast(ctypes.byref(eps), ctypes.c_void_p),
                             _stream(stream)))
    return A, B, np.array(sig[:r]), eps.value


def kron_approx_many(Ps, centers, bcs, rs, stream=None):
    """:func:`kron_approx` for several PSFs in one call (several images in
    flight on the device): ``Ps`` device float64 tensors, ``centers`` their
    ``(l, q)``, ``bcs`` and ``rs`` one value or one per PSF.  Returns a list
    of ``(A, B, sigma, eps_s)``, bit for bit those of :func:`kron_approx`."""
    import torch
    cnt = len(Ps)
    if cnt == 0:
        return []
    bcs = list(bcs) if isinstance(bcs, (list, tuple)) else [bcs] * cnt
    rs = list(rs) if isinstance(rs, (list, tuple)) else [rs] * cnt
    if len(centers) != cnt or len(bcs) != cnt or len(rs) != cnt:
        raise ValueError("centers, bcs and rs need one entry per PSF")
    ints = lambda v: (ctypes.c_int * cnt)(*[int(x) for x in v])
    ptrs = lambda v: (ctypes.c_void_p * cnt)(*v)
    As, Bs, pP = [], [], []
    for P, r in zip(Ps, rs):
        m, n = P.shape
        pP.append(_dev_f64(P, "P"))
        As.append(torch.empty((r, n, n), dtype=torch.float64, device=P.device))
        Bs.append(torch.empty((r, m, m), dtype=torch.float64, device=P.device))
    sig = (ctypes.c_double * max(sum(rs), 1))()
    eps = (ctypes.c_double * cnt)()
    _check(lib().kron_approx_batch(cnt, ptrs(pP), ints(P.shape[0] for P in Ps), ints(P.shape[1] for P in Ps),
                                   ints(c[0] for c in centers), ints(c[1] for c in centers), ints(bcs), ints(rs),
                                   ptrs(A.data_ptr() for A in As), ptrs(B.data_ptr() for B in Bs),
                                   ctypes.cast(sig, ctypes.c_void_p), ctypes.cast(eps, ctypes.c_void_p),
                                   _stream(stream)))
    out, o = [], 0
    for i in range(cnt):
        out.append((As[i], Bs[i], np.array(sig[o:o + rs[i]]), eps[i]))
        o += rs[i]
    return out


def kron_generators(P, l: int, q: int, bc: int, r: int, stream=None):
    """The approximation of :func:`kron_approx` as generator vectors:
    ``(h, k, sigma, eps_s)`` with ``h`` (r, m) and ``k`` (r, n) device tensors;
    ``B_k`` and ``A_k`` are their Toeplitz (+ Hankel) expansions."""
    import torch
    m, n = P.shape
    h = torch.empty((r, m), dtype=torch.float64, device=P.device)
    k = torch.empty((r, n), dtype=torch.float64, device=P.device)
    sig = (ctypes.c_double * max(r, 1))()
    eps = ctypes.c_double(0.0)
    _check(lib().kron_generators(_dev_f64(P, "P"), m, n, l, q, bc, r, h.data_ptr(), k.data_ptr(),
                                 ctypes.cast(sig, ctypes.c_void_p), ctypes.cast(ctypes.byref(eps), ctypes.c_void_p),
                                 _stream(stream)))
    return h, k, np.array(sig[:r]), eps.value


class FftSolver:
    """Structured-FFT sFISTA plan for one image: the factors enter through
    their generators ``h`` (r, m) and ``k`` (r, n), centre ``(l, q)`` and
    boundary ``bc``, and are applied by 1-D FFTs (FP32 transforms, FP64
    iterates)."""

    def __init__(self, Bobs, h, k, l: int, q: int, bc: int, lam: float, L: Optional[float] = None,
                 nonneg: bool = False, power_iters: int = 0, x0=None, v0=None, stream=None,
                 l_estimate: str = "power"):
        m, n = Bobs.shape
        r = h.shape[0]
        if h.shape != (r, m) or k.shape != (r, n):
            raise ValueError("h must be (r, m) and k (r, n) for Bobs of shape (m, n)")
        p = Params(float(lam), float(L) if L is not None else 0.0, PRECISIONS["fp32"], int(bool(nonneg)),
                   int(power_iters), 0, _dev_f64(x0, "x0") if x0 is not None else None,
                   _dev_f64(v0, "v0") if v0 is not None else None, _l_estimate(l_estimate))
        hd = ctypes.c_void_p()
        self._h = None
        self.shape = (m, n)
        self.device = Bobs.device
        _check(lib().sfista_fft_setup(_dev_f64(Bobs, "Bobs"), m, n, _dev_f64(h, "h"), _dev_f64(k, "k"), r, int(l),
                                      int(q), int(bc), ctypes.byref(p), _stream(stream), ctypes.byref(hd)))
        self._h = hd

    @property
    def L(self) -> float:
        v = ctypes.c_double()
        _check(lib().sfista_fft_get_L(self._h, ctypes.byref(v)))
        return v.value

    def step(self, iters: int):
        _check(lib().sfista_fft_step(self._h, int(iters)))

    def solve(self, max_iters: int, tol: float = 0.0, want_x: bool = True):
        import torch
        X = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_x else None
        rep = Report()
        _check(lib().sfista_fft_solve(self._h, int(max_iters), float(tol), X.data_ptr() if want_x else None,
                                      ctypes.byref(rep)))
        return X, rep.as_dict()

    def apply(self, X, want_ax: bool = True, want_atax: bool = True):
        """``(sum_k B_k X A_k^T, A_s^T A_s X)`` by the plan's transforms."""
        import torch
        ax = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_ax else None
        atax = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_atax else None
        _check(lib().sfista_fft_apply(self._h, _dev_f64(X, "X"), ax.data_ptr() if want_ax else None,
                                      atax.data_ptr() if want_atax else None))
        return ax, atax

    def close(self):
        if self._h is not None:
            lib().sfista_fft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """sFISTA plan (Algorithm 2) for one image."""

    def __init__(self, Bobs, A, B, lam: float, L: Optional[float] = None, precision: str = "bf16x3",
                 nonneg: bool = False, power_iters: int = 0, pair_state: bool = True, x0=None, v0=None,
                 stream=None, l_estimate: str = "power"):
        m, n = Bobs.shape
        r = A.shape[0]
        if A.shape != (r, n, n) or B.shape != (r, m, m):
            raise ValueError("A must be (r, n, n) and B (r, m, m) for Bobs of shape (m, n)")
        p = Params(float(lam), float(L) if L is not None else 0.0, PRECISIONS[precision], int(bool(nonneg)),
                   int(power_iters), int(bool(pair_state)),
                   _dev_f64(x0, "x0") if x0 is not None else None,
                   _dev_f64(v0, "v0") if v0 is not None else None, _l_estimate(l_estimate))
        h = ctypes.c_void_p()
        self._h = None
        self.shape = (m, n)
        self.device = Bobs.device
        self._stream = stream
        _check(lib().sfista_setup(_dev_f64(Bobs, "Bobs"), m, n, _dev_f64(A, "A"), _dev_f64(B, "B"), r,
                                  ctypes.byref(p), _stream(stream), ctypes.byref(h)))
        self._h = h

    @property
    def L(self) -> float:
        v = ctypes.c_double()
        _check(lib().sfista_get_L(self._h, ctypes.byref(v)))
        return v.value

    def step(self, iters: int):
        _check(lib().sfista_step(self._h, int(iters)))

    def solve(self, max_iters: int, tol: float = 0.0, want_x: bool = True):
        import torch
        X = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_x else None
        rep = Report()
        _check(lib().sfista_solve(self._h, int(max_iters), float(tol), X.data_ptr() if want_x else None,
                                  ctypes.byref(rep)))
        return X, rep.as_dict()

    def apply(self, X, want_ax: bool = True, want_atax: bool = True):
        """``(sum_k B_k X A_k^T, A_s^T A_s X)`` with the plan's GEMMs."""
        import torch
        ax = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_ax else None
        atax = torch.empty(self.shape, dtype=torch.float64, device=self.device) if want_atax else None
        _check(lib().sfista_apply(self._h, _dev_f64(X, "X"), ax.data_ptr() if want_ax else None,
                                  atax.data_ptr() if want_atax else None))
        return ax, atax

    def set_timing(self, every: int = 1):
        """Time the GEMMs of every ``every``-th iteration (``True`` = 1: all of
        them; 0 or ``False``: off)."""
        _check(lib().sfista_set_timing(self._h, int(every)))

    def kernel_times(self):
        """Mean device milliseconds and launch counts since the last call:
        entries 0..3 the GEMM kernels of F1, F2, G1, G2, entries 4..7 the
        reductions of their K-split tiles."""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_long * 8)()
        _check(lib().sfista_kernel_times(self._h, ms, cnt))
        return list(ms), list(cnt)

    def close(self):
        if self._h is not None:
            lib().sfista_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent sFISTA problems advanced together (Algorithm 2 on
    each): every GEMM phase of one iteration is a single grouped launch over
    all problems.  ``problems`` is a sequence of ``(Bobs, A, B, lam, L)`` with
    device float64 tensors; ``L = None`` estimates it (``l_estimate``, with
    ``power_iters`` steps) for all such problems at once.  ``autotune`` times
    the tile shapes of each phase on the batch itself; ``graph`` replays the
    iterations from a captured HIP graph."""

    def __init__(self, problems, precision: str = "bf16x3", max_iters: int = 1000, nonneg: bool = False,
                 power_iters: int = 0, pair_state: bool = True, autotune: bool = False, graph: bool = False,
                 stream=None, l_estimate: str = "power"):
        items = (BatchItem * max(len(problems), 1))()
        self.shapes = []
        self.device = None
        for k, (Bobs, A, B, lam, L) in enumerate(problems):
            m, n = Bobs.shape
            r = A.shape[0]
            if A.shape != (r, n, n) or B.shape != (r, m, m):
                raise ValueError(f"problem {k}: A must be (r, n, n) and B (r, m, m) for Bobs of shape (m, n)")
            items[k] = BatchItem(_dev_f64(Bobs, "Bobs"), m, n, _dev_f64(A, "A"), _dev_f64(B, "B"), r,
                                 float(lam), float(L) if L is not None else 0.0)
            self.shapes.append((m, n))
            self.device = Bobs.device
        common = Params(0.0, 0.0, PRECISIONS[precision], int(bool(nonneg)), int(power_iters),
                        int(bool(pair_state)), None, None, _l_estimate(l_estimate))
        flags = (BATCH_AUTOTUNE if autotune else 0) | (BATCH_GRAPH if graph else 0)
        h = ctypes.c_void_p()
        self._h = None
        _check(lib().sfista_batch_setup(items, len(problems), ctypes.byref(common), int(max_iters), flags,
                                        _stream(stream), ctypes.byref(h)))
        self._h = h

    def solve(self, iters: int, want_x: bool = True):
        """Run ``iters`` more iterations; returns (list of X or None, list of report dicts)."""
        import torch
        cnt = len(self.shapes)
        xs = [torch.empty(s, dtype=torch.float64, device=self.device) for s in self.shapes] if want_x else None
        ptrs = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs]) if want_x else None
        reps = (Report * cnt)()
        _check(lib().sfista_batch_solve(self._h, int(iters), ptrs, reps))
        return xs, [r.as_dict() for r in reps]

    def tiles(self):
        """Tile shape chosen per phase (F1, F2, G1, G2): 0 = the mode's large
        tile (256 x 256; 128 x 128 in FP64), 1 = 64 x 64, 2 = 128 x 128."""
        c = (ctypes.c_int * 4)()
        _check(lib().sfista_batch_tiles(self._h, c))
        return list(c)

    def set_tiles(self, choice):
        """Pin the tile shape of each phase (codes as in ``tiles``)."""
        c = (ctypes.c_int * 4)(*[int(v) for v in choice])
        _check(lib().sfista_batch_set_tiles(self._h, c))

    def close(self):
        if self._h is not None:
            lib().sfista_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Unrolled:
    """Differentiable unrolled sFISTA for a batch of problems of one rank r:
    ``forward()`` runs ``iters`` iterations of Algorithm 2 from zero on every
    problem (each ``L`` fixed, checkpoints every ``ckpt`` iterations) and
    returns the list of X; ``backward(dXs)`` returns ``(dAs, dBs, dlams)``,
    the gradients of a loss whose derivative in each X is the matching dX.
    ``problems`` is a sequence of ``(Bobs, A, B, lam, L)`` with float64 device
    tensors (``L`` None: power estimate).  ``precision`` is "fp32" or "fp64"."""

    def __init__(self, problems, iters: int = 50, ckpt: int = 10, precision: str = "fp32", stream=None):
        items, self.shapes, self.ranks, self.device = self._items(problems)
        self.iters, self.ckpt, self.precision = int(iters), int(ckpt), precision
        self._h = None
        h = ctypes.c_void_p()
        _check(lib().sfista_diff_setup(items, len(problems), PRECISIONS[precision], self.iters, self.ckpt,
                                       _stream(stream), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def _items(problems):
        cnt = len(problems)
        items = (BatchItem * max(cnt, 1))()
        shapes, ranks, device = [], [], None
        for k, (Bobs, A, B, lam, L) in enumerate(problems):
            m, n = Bobs.shape
            r = A.shape[0]
            if A.shape != (r, n, n) or B.shape != (r, m, m):
                raise ValueError(f"problem {k}: A must be (r, n, n) and B (r, m, m) for Bobs of shape (m, n)")
            items[k] = BatchItem(_dev_f64(Bobs, "Bobs"), m, n, _dev_f64(A, "A"), _dev_f64(B, "B"), r,
                                 float(lam), float(L) if L is not None else 0.0)
            shapes.append((m, n))
            ranks.append(r)
            device = Bobs.device
        return items, shapes, ranks, device

    def update(self, problems):
        """Load new problems of the same sizes and ranks (same order) into the
        handle without allocating: new factors, observations, lambda, L."""
        items, shapes, ranks, _ = self._items(problems)
        if shapes != self.shapes or ranks != self.ranks:
            raise ValueError("update needs the sizes and ranks the handle was set up with")
        _check(lib().sfista_diff_update(self._h, items, len(problems)))

    @property
    def L(self):
        v = (ctypes.c_double * len(self.shapes))()
        _check(lib().sfista_diff_get_L(self._h, v))
        return list(v)

    def forward(self):
        import torch
        xs = [torch.empty(s, dtype=torch.float64, device=self.device) for s in self.shapes]
        ptrs = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        _check(lib().sfista_diff_forward(self._h, ptrs))
        return xs

    def backward(self, dXs):
        import torch
        cnt = len(self.shapes)
        dXs = [_contig_f64(x, "dX") for x in dXs]
        dA = [torch.empty((r, n, n), dtype=torch.float64, device=self.device) for (m, n), r in zip(self.shapes, self.ranks)]
        dB = [torch.empty((r, m, m), dtype=torch.float64, device=self.device) for (m, n), r in zip(self.shapes, self.ranks)]
        P = ctypes.c_void_p * cnt
        dl = (ctypes.c_double * cnt)()
        _check(lib().sfista_diff_backward(self._h, P(*[x.data_ptr() for x in dXs]), P(*[a.data_ptr() for a in dA]),
                                          P(*[b.data_ptr() for b in dB]), dl))
        return dA, dB, list(dl)

    def close(self):
        if self._h is not None:
            lib().sfista_diff_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _contig_f64(t, name):
    import torch
    t = t.to(torch.float64).contiguous()
    _dev_f64(t, name)
    return t


def _unrolled_function():
    import torch

    class SfistaUnrolledFn(torch.autograd.Function):
        """Batch of images, each restored by ``iters`` unrolled iterations;
        gradients flow to the factors and lambda through the library's
        adjoint (L and Bobs are constants)."""

        @staticmethod
        def forward(ctx, A, B, lam, Bobs, L, iters, ckpt, precision, plan):
            N = Bobs.shape[0]
            lams = lam.detach().reshape(-1).expand(N).tolist()
            if L is None:
                Ls = [None] * N
            else:
                Lv = [float(v) for v in np.asarray(L.detach().cpu() if isinstance(L, torch.Tensor) else L,
                                                   dtype=np.float64).reshape(-1)]
                Ls = Lv * N if len(Lv) == 1 else Lv
            Ad, Bd, Od = A.detach(), B.detach(), Bobs.detach()
            probs = [(Od[k].contiguous(), Ad[k].contiguous(), Bd[k].contiguous(), lams[k], Ls[k]) for k in range(N)]
            if plan is None:
                u = Unrolled(probs, iters, ckpt, precision)
            else:
                u = plan
                u.update(probs)
            X = torch.stack(u.forward())
            ctx.plan = u
            ctx.owned = plan is None
            ctx.lam_shape = lam.shape
            return X

        @staticmethod
        def backward(ctx, dX):
            N = dX.shape[0]
            dA, dB, dl = ctx.plan.backward([dX[k] for k in range(N)])
            if ctx.owned:
                ctx.plan.close()
            dlam = torch.tensor(dl, dtype=torch.float64, device=dX.device)
            dlam = dlam.sum().reshape(ctx.lam_shape) if ctx.lam_shape.numel() == 1 else dlam.reshape(ctx.lam_shape)
            return torch.stack(dA), torch.stack(dB), dlam, None, None, None, None, None, None

    return SfistaUnrolledFn


def unrolled(A, B, lam, Bobs, L=None, iters: int = 50, ckpt: int = 10, precision: str = "fp32", plan=None):
    """X = unrolled sFISTA of a batch: A (N, r, n, n), B (N, r, m, m), lam a
    scalar or (N,) tensor, Bobs (N, m, n), all float64 on the GPU; L None
    (power estimate per image), a float, or (N,) values.  Differentiable in
    A, B and lam with torch.autograd.  ``plan``: an ``Unrolled`` handle of
    these sizes to reuse (its iters, ckpt and precision apply; the call
    updates it, so one backward must run before the next forward); without
    one, each call sets up and releases a handle of its own."""
    if plan is not None:
        iters, ckpt, precision = plan.iters, plan.ckpt, plan.precision
    return _unrolled_function().apply(A, B, lam, Bobs, L, iters, ckpt, precision, plan)
