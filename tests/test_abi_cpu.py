"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/sfista.h, and rejects invalid arguments before any
device work."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "sfista.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("kron_approx", "sfista_setup", "sfista_step", "sfista_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1901_00913_amd import sfista
    lib = sfista.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(sfista.EXPORTS)


@pytest.fixture(scope="module")
def L():
    from paper_1901_00913_amd import sfista
    return sfista.lib()


def _params(**kw):
    from paper_1901_00913_amd.sfista import Params
    p = Params(0.1, 1.0, 4, 0, 0, 1, None, None)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


@pytest.mark.parametrize("case,expect", [
    (dict(m=0), -1), (dict(n=-3), -1), (dict(r=0), -1), (dict(r=5, m=4, n=4), -1),
    (dict(lambda_=-1.0), -1), (dict(lambda_=float("nan")), -1), (dict(L=float("inf")), -1),
    (dict(precision=7), -2), (dict(power_iters=-1), -1), (dict(l_estimate=2), -1), (dict(l_estimate=-1), -1),
])
def test_setup_rejects_invalid_arguments(L, case, expect):
    m, n, r = case.pop("m", 4), case.pop("n", 4), case.pop("r", 1)
    p = _params(**case)
    h = ctypes.c_void_p()
    rc = L.sfista_setup(FAKE, m, n, FAKE, FAKE, r, ctypes.byref(p), None, ctypes.byref(h))
    assert rc == expect
    assert h.value is None
    assert L.sfista_last_error()


def test_setup_rejects_null_pointers(L):
    h = ctypes.c_void_p()
    p = _params()
    assert L.sfista_setup(None, 4, 4, FAKE, FAKE, 1, ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert L.sfista_setup(FAKE, 4, 4, FAKE, FAKE, 1, None, None, ctypes.byref(h)) == -1
    assert L.sfista_setup(FAKE, 4, 4, FAKE, FAKE, 1, ctypes.byref(p), None, None) == -1


@pytest.mark.parametrize("args,expect", [
    ((4, 4, 4, 1, 0, 1), -1),    # l out of range
    ((4, 4, 1, -1, 0, 1), -1),   # q out of range
    ((4, 4, 1, 1, 2, 1), -1),    # unknown boundary
    ((4, 4, 1, 1, 0, 5), -1),    # r > min(m, n)
    ((64, 64, 1, 1, 0, 40), -2), # r beyond the supported subspace width
])
def test_kron_approx_rejects_invalid_arguments(L, args, expect):
    m, n, l, q, bc, r = args
    assert L.kron_approx(FAKE, m, n, l, q, bc, r, FAKE, FAKE, None, None, None) == expect


def _kron_batch_call(L, imgs, P=FAKE, A=FAKE, B=FAKE, count=None):
    cnt = len(imgs) if count is None else count
    k = max(len(imgs), 1)
    col = lambda j: (ctypes.c_int * k)(*[im[j] for im in imgs] or [0])
    ptr = lambda v: (ctypes.c_void_p * k)(*[v] * k)
    return L.kron_approx_batch(cnt, ptr(P), col(0), col(1), col(2), col(3), col(4), col(5), ptr(A), ptr(B),
                               None, None, None)


@pytest.mark.parametrize("bad,expect", [
    ((4, 4, 4, 1, 0, 1), -1), ((4, 4, 1, 1, 2, 1), -1), ((4, 4, 1, 1, 0, 5), -1), ((64, 64, 1, 1, 0, 40), -2),
])
def test_kron_batch_checks_every_image_before_queuing(L, bad, expect):
    """One bad image among good ones: the call fails with kron_approx's code
    and names the image, and queues nothing (no device is touched here)."""
    good = (8, 8, 4, 4, 1, 2)
    assert _kron_batch_call(L, [good, good, bad]) == expect
    assert b"image 2" in L.sfista_last_error()


def test_kron_batch_rejects_null_and_empty(L):
    good = (8, 8, 4, 4, 1, 2)
    assert _kron_batch_call(L, [good], count=0) == -1
    assert _kron_batch_call(L, [good, good], P=None) == -1
    assert _kron_batch_call(L, [good], B=None) == -1
    assert L.kron_approx_batch(1, None, None, None, None, None, None, None, None, None, None, None, None) == -1


def test_handle_calls_reject_null(L):
    assert L.sfista_step(None, 1) == -1
    assert L.sfista_solve(None, 1, 0.0, None, None) == -1
    assert L.sfista_apply(None, FAKE, None, None) == -1
    L.sfista_destroy(None)


def _items(count=2, **kw):
    from paper_1901_00913_amd.sfista import BatchItem
    arr = (BatchItem * count)()
    for i in range(count):
        arr[i] = BatchItem(FAKE, 8, 8, FAKE, FAKE, 2, 0.01, 1.0)
    for k, v in kw.items():
        setattr(arr[count - 1], k, v)
    return arr


@pytest.mark.parametrize("count,max_iters,item,common,expect", [
    (0, 10, {}, {}, -1),                          # empty batch
    (2, 0, {}, {}, -1),                           # no iterations allowed
    (2, 10, dict(m=0), {}, -1),                   # bad size in the last problem
    (2, 10, dict(r=9), {}, -1),                   # r > min(m, n)
    (2, 10, dict(lambda_=-0.5), {}, -1),
    (2, 10, dict(L=float("nan")), {}, -1),
    (2, 10, dict(Bobs=None), {}, -1),
    (2, 10, {}, dict(precision=9), -2),
    (2, 10, {}, dict(x0=0x2000), -2),             # batch problems start from zero
    (2, 10, {}, dict(power_iters=-2), -1),
    (2, 10, {}, dict(l_estimate=3), -1),
])
def test_batch_setup_rejects_invalid_arguments(L, count, max_iters, item, common, expect):
    items = _items(max(count, 1), **item)
    p = _params(**common)
    h = ctypes.c_void_p()
    rc = L.sfista_batch_setup(items, count, ctypes.byref(p), max_iters, 0, None, ctypes.byref(h))
    assert rc == expect
    assert h.value is None
    assert L.sfista_last_error()


def test_batch_calls_reject_null(L):
    p = _params()
    assert L.sfista_batch_setup(None, 2, ctypes.byref(p), 10, 0, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert L.sfista_batch_setup(_items(), 2, None, 10, 0, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert L.sfista_batch_setup(_items(), 2, ctypes.byref(p), 10, 0, None, None) == -1
    assert L.sfista_batch_solve(None, 1, None, None) == -1
    assert L.sfista_batch_tiles(None, (ctypes.c_int * 4)()) == -1
    assert L.sfista_batch_set_tiles(None, (ctypes.c_int * 4)()) == -1
    L.sfista_batch_destroy(None)


@pytest.mark.parametrize("args,expect", [
    (dict(precision=4), -2),          # BF16X3 is not offered in the differentiable form
    (dict(iters=0), -1),
    (dict(ckpt=0), -1),
    (dict(count=0), -1),
    (dict(m=0), -1),
    (dict(r=9), -1),                  # r > min(m, n) in the last problem
    (dict(lambda_=-1.0), -1),
    (dict(r2=2), -2),                 # ranks differ between problems
])
def test_diff_setup_rejects_invalid_arguments(L, args, expect):
    a = dict(precision=1, iters=5, ckpt=2, count=2)
    a.update({k: v for k, v in args.items() if k in a})
    item = {k: v for k, v in args.items() if k in ("m", "r", "lambda_")}
    items = _items(2, **item)
    if "r2" in args:
        items[0].r = 1
        items[1].r = args["r2"]
    h = ctypes.c_void_p()
    rc = L.sfista_diff_setup(items, a["count"], a["precision"], a["iters"], a["ckpt"], None, ctypes.byref(h))
    assert rc == expect
    assert h.value is None


def test_diff_calls_reject_null(L):
    d = (ctypes.c_double * 2)()
    P = ctypes.c_void_p * 2
    assert L.sfista_diff_setup(_items(), 2, 1, 5, 2, None, None) == -1
    assert L.sfista_diff_setup(None, 2, 1, 5, 2, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert L.sfista_diff_forward(None, None) == -1
    assert L.sfista_diff_backward(None, P(), P(), P(), d) == -1
    assert L.sfista_diff_get_L(None, d) == -1
    assert L.sfista_diff_update(None, _items(), 2) == -1
    L.sfista_diff_destroy(None)


@pytest.mark.parametrize("args,expect", [
    (dict(m=0), -1), (dict(n=5000), -2), (dict(r=0), -1), (dict(r=5, m=4, n=4), -1),
    (dict(r=65, m=100, n=100), -2), (dict(l=4), -1), (dict(q=-1), -1), (dict(bc=2), -1),
    (dict(lambda_=-1.0), -1), (dict(L=float("nan")), -1), (dict(power_iters=-1), -1), (dict(l_estimate=5), -1),
])
def test_fft_setup_rejects_invalid_arguments(L, args, expect):
    m, n, r = args.pop("m", 4), args.pop("n", 4), args.pop("r", 1)
    l, q, bc = args.pop("l", 1), args.pop("q", 1), args.pop("bc", 1)
    p = _params(**args)
    h = ctypes.c_void_p()
    rc = L.sfista_fft_setup(FAKE, m, n, FAKE, FAKE, r, l, q, bc, ctypes.byref(p), None, ctypes.byref(h))
    assert rc == expect
    assert h.value is None
    assert L.sfista_last_error()


def test_fft_calls_reject_null(L):
    h = ctypes.c_void_p()
    p = _params()
    assert L.sfista_fft_setup(None, 4, 4, FAKE, FAKE, 1, 1, 1, 0, ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert L.sfista_fft_setup(FAKE, 4, 4, None, FAKE, 1, 1, 1, 0, ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert L.sfista_fft_setup(FAKE, 4, 4, FAKE, FAKE, 1, 1, 1, 0, None, None, ctypes.byref(h)) == -1
    assert L.sfista_fft_setup(FAKE, 4, 4, FAKE, FAKE, 1, 1, 1, 0, ctypes.byref(p), None, None) == -1
    assert L.sfista_fft_step(None, 1) == -1
    assert L.sfista_fft_solve(None, 1, 0.0, None, None) == -1
    assert L.sfista_fft_apply(None, FAKE, None, None) == -1
    assert L.sfista_fft_get_L(None, ctypes.byref(ctypes.c_double())) == -1
    L.sfista_fft_destroy(None)
    assert L.kron_generators(FAKE, 4, 4, 1, 1, 0, 1, None, FAKE, None, None, None) == -1
    assert L.kron_generators(FAKE, 4, 4, 4, 1, 0, 1, FAKE, FAKE, None, None, None) == -1


def test_kron_approx_many_checks_lengths_before_the_library():
    """The Python entry of the batched setup: an empty list needs no work, and
    per-PSF arguments of the wrong length are refused before any call."""
    from paper_1901_00913_amd import sfista
    assert sfista.kron_approx_many([], [], 1, 1) == []
    with pytest.raises(ValueError):
        sfista.kron_approx_many([object(), object()], [(1, 1)], 1, 2)
    with pytest.raises(ValueError):
        sfista.kron_approx_many([object()], [(1, 1)], [0, 1], 2)
