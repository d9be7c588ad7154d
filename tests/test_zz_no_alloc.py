"""The no-allocation entry point (etest_run_async_noalloc) against the allocating one
(ed_test_async / mmd_test_async), through the C ABI: same kernels, same inputs, so every
output must be identical bit for bit; each result is also checked against the oracle.
Two calls in a row on the same GPU share the scratch array, the second on a smaller test;
a test larger than the scratch is rejected before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2406_06488_amd import _lib, api, inputs
from tests.gpu_helpers import compare_run, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
KIND = {"ed": oracle.ED, "mmd": oracle.MMD}


def _noalloc():
    L = _lib.load()
    f = L.etest_run_async_noalloc
    f.argtypes = [ctypes.POINTER(_lib.Request), ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int32
    return f


def _both(nx, ny, p, B, seed, kind, prec, data_seed):
    dt = np.float64 if prec == "f64" else np.float32
    X, Y = inputs.gaussian_pair(nx, ny, p, data_seed, mean_shift=0.1, dtype=dt)
    tdt = torch.float64 if prec == "f64" else torch.float32
    Xd, Yd = torch.from_numpy(X).to(DEV, tdt), torch.from_numpy(Y).to(DEV, tdt)
    gamma = 1.0 / p
    ps_a = torch.full((B,), -1.0, dtype=torch.float64, device=DEV)
    buf_a = api.run_async(Xd, Yd, B, seed, kind, prec, gamma, ps_a)
    ps_n = torch.full((B,), -2.0, dtype=torch.float64, device=DEV)
    buf_n = torch.zeros(6, dtype=torch.float64, device=DEV)
    req = api.make_request(Xd, Yd, B, seed, kind, prec, gamma, ps_n)
    st = _noalloc()(ctypes.byref(req), ctypes.c_void_p(buf_n.data_ptr()), api._stream())
    assert st == 0, api.last_error()
    torch.cuda.synchronize()
    a, n = api.result_from_device(buf_a), api.result_from_device(buf_n)
    say("noalloc", nx, ny, p, B, kind, prec, n)
    for k in ("statistic", "threshold", "p_value", "count_ge", "B", "n_refined"):
        assert a[k] == n[k], (k, a[k], n[k])
    assert torch.equal(ps_a, ps_n)
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, seed, KIND[kind], gamma)
    n["perm_stats"] = ps_n.cpu().numpy()
    compare_run(n, o, prec, "noalloc %s %s" % (kind, prec))


def test_noalloc_equals_allocating_entry_point_two_calls():
    # first call: a larger test; second: a smaller one on the scratch the first left behind
    _both(900, 800, 100, 3000, 5, "ed", "f32", 31)
    _both(300, 200, 37, 1000, 6, "mmd", "bf16r", 32)


def test_noalloc_other_forms():
    _both(420, 390, 70, 1200, 7, "mmd", "bf16r", 33)
    _both(150, 130, 12, 800, 8, "ed", "f64", 34)
    _both(260, 240, 30, 700, 9, "mmd", "f32", 35)


def test_noalloc_rejects_a_test_beyond_the_scratch():
    """3000 + 3000 rows at p = 1000 need ~180 MB of workspace, past the 128 MiB scratch:
    ENOMEM before any device work, outputs untouched."""
    X = torch.zeros((3000, 1000), dtype=torch.float32, device=DEV)
    Y = torch.zeros((3000, 1000), dtype=torch.float32, device=DEV)
    ps = torch.full((100,), 7.0, dtype=torch.float64, device=DEV)
    buf = torch.full((6,), 3.0, dtype=torch.float64, device=DEV)
    req = api.make_request(X, Y, 100, 1, "ed", "f32", 0.0, ps)
    st = _noalloc()(ctypes.byref(req), ctypes.c_void_p(buf.data_ptr()), api._stream())
    torch.cuda.synchronize()
    assert st == _lib.ENOMEM, st
    assert "scratch" in api.last_error()
    assert torch.all(ps == 7.0) and torch.all(buf == 3.0)
    # the scratch still serves the next call
    _both(200, 180, 20, 500, 10, "ed", "f32", 36)
