"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2406_06488_amd import _lib, api
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "etest.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:etest_status|const char\s*\*)\s*(\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2406_06488_amd import build
        build.build(force=False)
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(names) == bound


def test_struct_layouts_match_header():
    assert ctypes.sizeof(_lib.Result) == 48
    assert ctypes.sizeof(_lib.Request) == 8 + 5 * 8 + 8 + 3 * 8
    assert ctypes.sizeof(_lib.ServerConfig) == 24
    assert ctypes.sizeof(_lib.CrossResult) == 40
    assert ctypes.sizeof(_lib.HsicRequest) == 8 + 5 * 8 + 2 * 8 + 3 * 8


def test_next_row_calls_reject_before_device():
    """The baseline, cross and HSIC entry points check their arguments on the host first."""
    L = _lib.load()
    r = _lib.Result()
    bad = _lib.Request(0, _lib.PREC_F32, 0, 5, 3, 10, 1, 0.0, 8, 8, None)  # nx = 0
    for fn in (L.etest_standard, L.etest_precomputed, L.etest_precomputed_dense):
        assert fn(ctypes.byref(bad), None, ctypes.byref(r)) == _lib.EINVAL
        assert fn(None, None, ctypes.byref(r)) == _lib.EINVAL
    cr = _lib.CrossResult()
    one = _lib.Request(0, _lib.PREC_F32, 1, 5, 3, 0, 1, 0.0, 8, 8, None)  # nx = 1: no halves
    assert L.etest_cross(ctypes.byref(one), None, ctypes.byref(cr)) == _lib.EINVAL

    def hreq(**kw):
        f = dict(prec=_lib.PREC_F32, reserved=0, n=10, p=3, q=2, B=10, seed=1, gamma_x=0.5,
                 gamma_y=0.5, X=8, Y=8, perm_stats=None)
        f.update(kw)
        return _lib.HsicRequest(*[f[k] for k, _ in _lib.HsicRequest._fields_])

    for kw in (dict(n=3), dict(n=4097), dict(q=0), dict(prec=_lib.PREC_BF16_REFINED),
               dict(gamma_x=0.0), dict(gamma_y=float("nan")), dict(B=-1), dict(reserved=1),
               dict(X=None), dict(B=2 ** 30)):
        assert L.etest_hsic(ctypes.byref(hreq(**kw)), None, ctypes.byref(r)) == _lib.EINVAL, kw
    assert L.etest_permutations(0, 1, 0, 1, 8, None) == _lib.EINVAL
    assert L.etest_permutations(5000, 1, 0, 1, 8, None) == _lib.EINVAL
    assert L.etest_permutations(5, 1, -1, 1, 8, None) == _lib.EINVAL


@pytest.mark.parametrize("args", [
    dict(nx=0, ny=5, p=3, B=10),
    dict(nx=5, ny=0, p=3, B=10),
    dict(nx=5, ny=5, p=0, B=10),
    dict(nx=5, ny=5, p=3, B=-1),
    dict(nx=5, ny=5, p=3, B=2**31),
    dict(nx=5, ny=5, p=3, B=10, X=None),
    dict(nx=5, ny=5, p=3, B=10, Y=None),
    dict(nx=5, ny=5, p=3, B=10, kind="mmd", gamma=0.0),
    dict(nx=5, ny=5, p=3, B=10, kind="mmd", gamma=-1.0),
    dict(nx=5, ny=5, p=3, B=10, kind="mmd", gamma=float("nan")),
    dict(nx=5, ny=5, p=3, B=10, kind="mmd", gamma=float("inf")),
    dict(nx=2 ** 30, ny=2 ** 30, p=3, B=10),
    dict(nx=5, ny=5, p=3, B=10, prec=7),
    dict(nx=5, ny=5, p=3, B=10, kind=3),
])
def test_validation_rejects(args):
    assert api.validate(**args) == _lib.EINVAL
    assert api.last_error() != ""


def test_validation_accepts():
    assert api.validate(5, 5, 3, 0) == _lib.OK
    assert api.validate(1, 1, 1, 10, kind="mmd", gamma=0.5) == _lib.OK
    assert api.validate(100, 100, 10, 1000, prec="f64") == _lib.OK


def test_footprint_grows_with_size():
    a = api.footprint(100, 100, 10, 1000, prec="f64")
    b = api.footprint(2000, 2000, 1000, 10000, prec="f32")
    c = api.footprint(5000, 4000, 4096, 10000, prec="bf16r")
    assert 0 < a < b < c
    # 2000 x 1000 x 2: staged operand + tiles + planes + split bits stay well under 1 GB
    assert b < 1 << 30


def test_host_calls_reject_before_device():
    import numpy as np
    L = _lib.load()
    r = _lib.Result()
    X = np.zeros((3, 2), np.float32)
    st = L.ed_test(X.ctypes.data, 0, X.ctypes.data, 3, 2, 10, 1, _lib.PREC_F32, None, ctypes.byref(r))
    assert st == _lib.EINVAL
    st = L.ed_test(X.ctypes.data, 3, X.ctypes.data, 3, 2, 10, 1, _lib.PREC_F64, None, ctypes.byref(r))
    assert st == _lib.EINVAL  # the float entry point does not take the FP64 form
    st = L.ed_test(X.ctypes.data, 3, X.ctypes.data, 3, 2, 10, 1, _lib.PREC_F32, None, None)
    assert st == _lib.EINVAL
