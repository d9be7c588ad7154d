"""FP64 CPU oracle for the efficient permutation ED / MMD two-sample test.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the HIP path.  The numerical work lives in ``oracle.c``
(plain C, FP64, exact block sums); this module only marshals numpy arrays.

What each function follows (Chaibub Neto, arXiv 2406.06488):
  blocks()        Alg. 3 (direct differences) and the Gaussian-kernel remark
                  after it (Appendix A.1).
  observed()      eq. (1) energy distance / eq. (2) biased MMD^2.
  membership()    the split drawn for permutation b (Alg. 2's sampling step;
                  Philox4x32-10 + selection sampling replaces R's sample()).
  split_indices() Alg. 2's index vectors i1, i2, j1, j2 from a split.
  perm_stat()     the Alg. 1 loop body: permuted blocks filled from the four
                  sub-blocks, then eq. (1)/(2).
  run_test()      Alg. 1 end to end, p-value as in Section 3.1.
  permutation(), hsic(), hsic_test()
                  the HSIC independence permutation test of the paper's
                  discussion (unbiased HSIC of Song et al. 2012; permutations
                  of the y sample from Philox keys).
"""
import ctypes
import os

import numpy as np

from . import build as _build

ED, MMD = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_xsum.argtypes = [dp, i64]
        L.orc_xsum.restype = ctypes.c_double
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_membership.argtypes = [i64, i64, ctypes.c_uint64, i64, u8p]
        L.orc_split_indices.argtypes = [i64, i64, u8p, i64p, i64p, i64p, i64p, i64p]
        L.orc_block.argtypes = [dp, i64, dp, i64, i64, ctypes.c_int, ctypes.c_double, dp,
                                ctypes.c_int]
        L.orc_observed.argtypes = [ctypes.c_int, dp, dp, dp, i64, i64, dp, dp]
        L.orc_perm_stat.argtypes = [ctypes.c_int, dp, dp, dp, i64, i64, u8p, dp]
        L.orc_perm_sums.argtypes = [dp, dp, dp, i64, i64, u8p, dp]
        L.orc_perm_stats_listed.argtypes = [ctypes.c_int, dp, dp, dp, i64, i64, ctypes.c_uint64,
                                            i64p, i64, dp, ctypes.c_int]
        L.orc_threshold.argtypes = [ctypes.c_int, dp, dp, dp, i64, i64, dp]
        L.orc_test.argtypes = [ctypes.c_int, dp, i64, dp, i64, i64, ctypes.c_double, i64,
                               ctypes.c_uint64, dp, dp, dp, i64p, dp, ctypes.c_int]
        L.orc_cross.argtypes = [ctypes.c_int, dp, i64, dp, i64, i64, ctypes.c_double, dp,
                                ctypes.c_int]
        L.orc_permutation.argtypes = [i64, ctypes.c_uint64, i64, i64p]
        L.orc_hsic.argtypes = [dp, dp, i64, i64p, dp]
        L.orc_hsic_test.argtypes = [dp, dp, i64, i64, i64, ctypes.c_double, ctypes.c_double, i64,
                                    ctypes.c_uint64, dp, dp, i64p, ctypes.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def xsum(v):
    """Exactly rounded sum of a float64 vector."""
    v = _f64(v).ravel()
    return lib().orc_xsum(_d(v), v.size)


def philox4x32_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    P = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def membership(nx, ny, seed, b):
    """Split b as a 0/1 vector over the pooled items (X rows, then Y rows)."""
    z = np.zeros(nx + ny, dtype=np.uint8)
    r = lib().orc_membership(nx, ny, seed, b, z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if r:
        raise ValueError("membership: invalid arguments")
    return z


def split_indices(nx, ny, z):
    """Alg. 2's (i1, i2, j1, j2), 0-based, from a 0/1 split vector."""
    z = np.ascontiguousarray(z, dtype=np.uint8)
    bufs = [np.zeros(max(nx, ny), dtype=np.int64) for _ in range(4)]
    counts = np.zeros(4, dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    lib().orc_split_indices(nx, ny, z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            *[b.ctypes.data_as(P) for b in bufs], counts.ctypes.data_as(P))
    return tuple(bufs[i][: counts[i]].copy() for i in range(4))


def block(A, B, kind=ED, gamma=1.0, nthreads=0):
    """Distance (kind=ED) or Gaussian-kernel (kind=MMD) matrix between the rows of A and B."""
    A = _f64(A)
    B = _f64(B)
    out = np.empty((A.shape[0], B.shape[0]), dtype=np.float64)
    r = lib().orc_block(_d(A), A.shape[0], _d(B), B.shape[0], A.shape[1], kind, gamma, _d(out),
                        nthreads)
    if r:
        raise ValueError("block: invalid arguments")
    return out


def blocks(X, Y, kind=ED, gamma=1.0, nthreads=0):
    """(D_XX, D_YY, D_XY): Alg. 1's three blocks."""
    return (block(X, X, kind, gamma, nthreads), block(Y, Y, kind, gamma, nthreads),
            block(X, Y, kind, gamma, nthreads))


def observed(XX, YY, XY, kind=ED):
    """eq. (1) or eq. (2) from the blocks; also returns the exact block sums."""
    XX, YY, XY = _f64(XX), _f64(YY), _f64(XY)
    st = ctypes.c_double()
    sums = np.zeros(3)
    lib().orc_observed(kind, _d(XX), _d(YY), _d(XY), XX.shape[0], YY.shape[0], ctypes.byref(st),
                       _d(sums))
    return st.value, sums


def perm_stat(XX, YY, XY, z, kind=ED):
    XX, YY, XY = _f64(XX), _f64(YY), _f64(XY)
    z = np.ascontiguousarray(z, dtype=np.uint8)
    st = ctypes.c_double()
    r = lib().orc_perm_stat(kind, _d(XX), _d(YY), _d(XY), XX.shape[0], YY.shape[0],
                            z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(st))
    if r:
        raise ValueError("perm_stat: split must hold exactly nx members")
    return st.value


def perm_sums(XX, YY, XY, z):
    """Element sums of the permuted blocks (D_{X*X*}, D_{Y*Y*}, D_{X*Y*}) for split z."""
    XX, YY, XY = _f64(XX), _f64(YY), _f64(XY)
    z = np.ascontiguousarray(z, dtype=np.uint8)
    out = np.zeros(3)
    r = lib().orc_perm_sums(_d(XX), _d(YY), _d(XY), XX.shape[0], YY.shape[0],
                            z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _d(out))
    if r:
        raise ValueError("perm_sums: split must hold exactly nx members")
    return out


def threshold(XX, YY, XY, kind=ED):
    XX, YY, XY = _f64(XX), _f64(YY), _f64(XY)
    st = ctypes.c_double()
    lib().orc_threshold(kind, _d(XX), _d(YY), _d(XY), XX.shape[0], YY.shape[0], ctypes.byref(st))
    return st.value


def perm_stats_listed(XX, YY, XY, seed, b_list, kind=ED, nthreads=0):
    XX, YY, XY = _f64(XX), _f64(YY), _f64(XY)
    bl = np.ascontiguousarray(b_list, dtype=np.int64)
    out = np.zeros(bl.size, dtype=np.float64)
    r = lib().orc_perm_stats_listed(kind, _d(XX), _d(YY), _d(XY), XX.shape[0], YY.shape[0], seed,
                                    bl.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), bl.size,
                                    _d(out), nthreads)
    if r:
        raise MemoryError("perm_stats_listed failed")
    return out


def run_test(X, Y, B, seed, kind=ED, gamma=1.0, nthreads=0):
    """Alg. 1 end to end. Returns dict(statistic, threshold, count_ge, p_value, perm_stats)."""
    X, Y = _f64(X), _f64(Y)
    ps = np.zeros(max(B, 1), dtype=np.float64)
    so, thr, pv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    cnt = ctypes.c_int64()
    r = lib().orc_test(kind, _d(X), X.shape[0], _d(Y), Y.shape[0], X.shape[1], gamma, B, seed,
                       _d(ps), ctypes.byref(so), ctypes.byref(thr), ctypes.byref(cnt),
                       ctypes.byref(pv), nthreads)
    if r:
        raise ValueError("oracle test failed with code %d" % r)
    return dict(statistic=so.value, threshold=thr.value, count_ge=cnt.value, p_value=pv.value,
                perm_stats=ps[:B].copy())


def cross(X, Y, kind=ED, gamma=1.0, nthreads=0):
    """Cross-MMD (Alg. 6) or cross-ED (Alg. 7) test: dict(statistic=U, sigma, z, p_value)."""
    X, Y = _f64(X), _f64(Y)
    if X.shape[1] != Y.shape[1]:
        raise ValueError("cross: X and Y need the same number of columns")
    out = np.empty(4, dtype=np.float64)
    r = lib().orc_cross(kind, _d(X), X.shape[0], _d(Y), Y.shape[0], X.shape[1], gamma, _d(out),
                        nthreads)
    if r:
        raise ValueError("cross: invalid arguments (nx, ny >= 2, p >= 1, gamma > 0 for MMD)")
    return {"statistic": float(out[0]), "sigma": float(out[1]), "z": float(out[2]),
            "p_value": float(out[3])}


def permutation(n, seed, b):
    """Permutation b of 0..n-1 (items ordered by their Philox key, ties by index)."""
    out = np.empty(n, dtype=np.int64)
    if lib().orc_permutation(n, seed, b, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))):
        raise ValueError("permutation: n >= 1, b >= 0")
    return out


def hsic(K, L, perm=None):
    """Unbiased HSIC of kernel matrices K and L, L read through perm (None: identity)."""
    K, L = _f64(K), _f64(L)
    n = K.shape[0]
    out = ctypes.c_double()
    pp = None
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int64)
        pp = perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if lib().orc_hsic(_d(K), _d(L), n, pp, ctypes.byref(out)):
        raise ValueError("hsic: n >= 4")
    return out.value


def hsic_test(X, Y, B, seed, gamma_x, gamma_y, nthreads=0):
    """HSIC independence permutation test on paired rows of X (n x p) and Y (n x q)."""
    X, Y = _f64(X), _f64(Y)
    n = X.shape[0]
    if Y.shape[0] != n:
        raise ValueError("hsic_test: X and Y need the same number of rows")
    ps = np.empty(max(B, 1), dtype=np.float64)
    out = np.empty(3, dtype=np.float64)
    cnt = ctypes.c_int64()
    r = lib().orc_hsic_test(_d(X), _d(Y), n, X.shape[1], Y.shape[1], gamma_x, gamma_y, B, seed,
                            _d(ps), _d(out), ctypes.byref(cnt), nthreads)
    if r:
        raise ValueError("hsic_test failed with code %d" % r)
    return dict(statistic=float(out[0]), threshold=float(out[1]), p_value=float(out[2]),
                count_ge=cnt.value, perm_stats=ps[:B].copy())

