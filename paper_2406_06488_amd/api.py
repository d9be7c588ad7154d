"""Python front end of the C ABI.

Host arrays (numpy) go through the host-buffer calls; torch tensors on the GPU
go through the device-buffer calls on torch's current stream.  Every numerical
step runs in the HIP library; this module only marshals arguments.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import ED, MMD, PREC_BF16_REFINED, PREC_F32, PREC_F64, Request, Result, check

PRECS = {"f64": PREC_F64, "f32": PREC_F32, "bf16r": PREC_BF16_REFINED}
KINDS = {"ed": ED, "mmd": MMD}


def _prec(p):
    return PRECS[p] if isinstance(p, str) else int(p)


def _kind(k):
    return KINDS[k] if isinstance(k, str) else int(k)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def ed_test(X, Y, B, seed, prec="f32", with_perm_stats=True):
    """Energy-distance permutation test on host arrays (float32, or float64 for prec='f64')."""
    L = _lib.load()
    pr = _prec(prec)
    dt = np.float64 if pr == PREC_F64 else np.float32
    X = np.ascontiguousarray(X, dtype=dt)
    Y = np.ascontiguousarray(Y, dtype=dt)
    ps = np.zeros(max(B, 1)) if with_perm_stats else None
    r = Result()
    pp = _ptr(ps) if ps is not None else None
    if pr == PREC_F64:
        check(L.ed_test_f64(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], X.shape[1], B, seed, pp,
                            ctypes.byref(r)))
    else:
        check(L.ed_test(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], X.shape[1], B, seed, pr, pp,
                        ctypes.byref(r)))
    out = r.as_dict()
    out["perm_stats"] = ps[:B].copy() if ps is not None else None
    return out


def mmd_test(X, Y, gamma, B, seed, prec="f32", with_perm_stats=True):
    """Gaussian-kernel MMD^2 permutation test on host arrays."""
    L = _lib.load()
    pr = _prec(prec)
    dt = np.float64 if pr == PREC_F64 else np.float32
    X = np.ascontiguousarray(X, dtype=dt)
    Y = np.ascontiguousarray(Y, dtype=dt)
    ps = np.zeros(max(B, 1)) if with_perm_stats else None
    r = Result()
    pp = _ptr(ps) if ps is not None else None
    if pr == PREC_F64:
        check(L.mmd_test_f64(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], X.shape[1], gamma, B, seed,
                             pp, ctypes.byref(r)))
    else:
        check(L.mmd_test(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], X.shape[1], gamma, B, seed, pr,
                         pp, ctypes.byref(r)))
    out = r.as_dict()
    out["perm_stats"] = ps[:B].copy() if ps is not None else None
    return out


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_request(X, Y, B, seed, kind="ed", prec="f32", gamma=0.0, perm_stats=None):
    """Request over device tensors X (nx x p), Y (ny x p); perm_stats a float64 device tensor or None."""
    r = Request()
    r.kind = _kind(kind)
    r.prec = _prec(prec)
    r.nx, r.p = X.shape
    r.ny = Y.shape[0]
    r.B = B
    r.seed = seed
    r.gamma = gamma
    r.X = X.data_ptr()
    r.Y = Y.data_ptr()
    r.perm_stats = perm_stats.data_ptr() if perm_stats is not None else None
    return r


def _check_dev(X, Y, prec):
    import torch
    want = torch.float64 if _prec(prec) == PREC_F64 else torch.float32
    for T in (X, Y):
        if not T.is_cuda or T.dtype != want or not T.is_contiguous() or T.dim() != 2:
            raise ValueError("device inputs must be contiguous 2-D %s CUDA tensors" % want)


def run(X, Y, B, seed, kind="ed", prec="f32", gamma=0.0, with_perm_stats=True):
    """One test on device tensors (torch), synchronous.  Returns a dict; perm_stats stays on device."""
    import torch
    _check_dev(X, Y, prec)
    ps = torch.empty(max(B, 1), dtype=torch.float64, device=X.device) if with_perm_stats else None
    req = make_request(X, Y, B, seed, kind, prec, gamma, ps)
    r = Result()
    check(_lib.load().etest_run(ctypes.byref(req), _stream(), ctypes.byref(r)))
    out = r.as_dict()
    out["perm_stats"] = ps[:B] if ps is not None else None
    return out


def _baseline(fn, X, Y, B, seed, kind, prec, gamma, with_perm_stats):
    import torch
    _check_dev(X, Y, prec)
    ps = torch.empty(max(B, 1), dtype=torch.float64, device=X.device) if with_perm_stats else None
    req = make_request(X, Y, B, seed, kind, prec, gamma, ps)
    r = Result()
    check(getattr(_lib.load(), fn)(ctypes.byref(req), _stream(), ctypes.byref(r)))
    out = r.as_dict()
    out["perm_stats"] = ps[:B] if ps is not None else None
    return out


def standard(X, Y, B, seed, kind="ed", prec="f32", gamma=0.0, with_perm_stats=True):
    """Standard permutation test (Alg. 4) on device tensors, synchronous: every split's
    statistic recomputed from blocks of its own X*, Y*.  Same splits and result fields as
    run(); statistic and threshold are both the identity split's recomputed statistic."""
    return _baseline("etest_standard", X, Y, B, seed, kind, prec, gamma, with_perm_stats)


def precomputed(X, Y, B, seed, kind="ed", prec="f32", gamma=0.0, with_perm_stats=True,
                dense=False):
    """Pre-computation permutation test (Alg. 5) on device tensors, synchronous: the pooled
    distance (kernel) matrix once, then per split the sums of the entries its index sets
    select.  dense: the pooled matrix as Alg. 5 prints it, (nx + ny)^2 entries with both
    orders of every pair (otherwise symmetric upper tiles).  Same splits and result fields
    as run()."""
    return _baseline("etest_precomputed_dense" if dense else "etest_precomputed", X, Y, B, seed,
                     kind, prec, gamma, with_perm_stats)


def hsic_request(X, Y, B, seed, gamma_x, gamma_y, prec="f32", perm_stats=None):
    return _lib.HsicRequest(_prec(prec), 0, X.shape[0], X.shape[1], Y.shape[1], B, seed,
                            gamma_x, gamma_y, X.data_ptr(), Y.data_ptr(),
                            perm_stats.data_ptr() if perm_stats is not None else None)


def hsic(X, Y, B, seed, gamma_x, gamma_y, prec="f32", with_perm_stats=True):
    """HSIC independence permutation test on paired device rows X (n x p), Y (n x q),
    synchronous.  Returns run()'s result fields; perm_stats (HSIC of each permutation of
    the y sample) stays on the device."""
    import torch
    _check_dev(X, Y, prec)
    if X.shape[0] != Y.shape[0]:
        raise ValueError("hsic: X and Y need the same number of rows")
    ps = torch.empty(max(B, 1), dtype=torch.float64, device=X.device) if with_perm_stats else None
    req = hsic_request(X, Y, B, seed, gamma_x, gamma_y, prec, ps)
    r = Result()
    check(_lib.load().etest_hsic(ctypes.byref(req), _stream(), ctypes.byref(r)))
    out = r.as_dict()
    out["perm_stats"] = ps[:B] if ps is not None else None
    return out


def permutations(n, seed, b0, count, device="cuda"):
    """Permutations b0 .. b0+count-1 of the HSIC test's stream, as a (count, n) int32 tensor."""
    import torch
    out = torch.empty((max(count, 1), n), dtype=torch.int32, device=device)
    check(_lib.load().etest_permutations(n, seed, b0, count, ctypes.c_void_p(out.data_ptr()),
                                         _stream()))
    return out[:count]


def cross(X, Y, kind="ed", prec="f32", gamma=0.0):
    """Cross-ED / cross-MMD test (permutation-free) on device tensors, synchronous.
    Returns dict(statistic, sigma, z, p_value, n_refined)."""
    _check_dev(X, Y, prec)
    req = make_request(X, Y, 0, 0, kind, prec, gamma, None)
    r = _lib.CrossResult()
    check(_lib.load().etest_cross(ctypes.byref(req), _stream(), ctypes.byref(r)))
    return r.as_dict()


def run_async(X, Y, B, seed, kind="ed", prec="f32", gamma=0.0, perm_stats=None):
    """Enqueue one test on torch's current stream; returns a device buffer holding the
    etest_result (6 x 8 bytes).  Use result_from_device() after synchronising."""
    import torch
    _check_dev(X, Y, prec)
    out = torch.empty(6, dtype=torch.float64, device=X.device)  # written by the library
    req = make_request(X, Y, B, seed, kind, prec, gamma, perm_stats)
    fn = _lib.load().ed_test_async if _kind(kind) == ED else _lib.load().mmd_test_async
    check(fn(ctypes.byref(req), ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def run_async_noalloc(X, Y, B, seed, kind="ed", prec="f32", gamma=0.0, perm_stats=None,
                      out=None):
    """run_async() through the entry point that allocates nothing on the library side (its
    workspace is a fixed device array).  out: a float64 device tensor of 6 for the result
    (allocated here when None, by torch)."""
    import torch
    _check_dev(X, Y, prec)
    if out is None:
        out = torch.empty(6, dtype=torch.float64, device=X.device)  # written by the library
    req = make_request(X, Y, B, seed, kind, prec, gamma, perm_stats)
    check(_lib.load().etest_run_async_noalloc(ctypes.byref(req), ctypes.c_void_p(out.data_ptr()),
                                              _stream()))
    return out


def result_from_device(buf):
    raw = buf.cpu().numpy().tobytes()
    r = Result.from_buffer_copy(raw)
    return r.as_dict()


_RESULT_KEYS = [k for k, _ in Result._fields_]


def batch(requests, keep=None):
    """Many tests in one batched, graph-captured pass.  requests: a list of Request, or a
    ctypes array of them (reused as it is)."""
    n = len(requests)
    arr = requests if isinstance(requests, ctypes.Array) else (Request * n)(*requests)
    outs = (Result * n)()
    check(_lib.load().etest_batch(arr, n, _stream(), outs))
    # one pass over the results as a structured array (a per-field getattr per test costs
    # more than the rest of the call's host work for a few hundred tests)
    dt = np.dtype([(k, "<f8" if i < 3 else "<i8") for i, k in enumerate(_RESULT_KEYS)])
    return [dict(zip(_RESULT_KEYS, r)) for r in np.frombuffer(outs, dtype=dt).tolist()]


def batch_async(requests, device="cuda"):
    """Enqueue many tests in one batched pass on torch's current stream and return a
    (n x 6) float64 device tensor of their etest_result records; read them with
    results_from_device() after synchronising.  requests: a list of Request, or a ctypes
    array of them."""
    import torch
    n = len(requests)
    arr = requests if isinstance(requests, ctypes.Array) else (Request * n)(*requests)
    out = torch.empty((n, 6), dtype=torch.float64, device=device)  # written by the library
    check(_lib.load().etest_batch_async(arr, n, _stream(), ctypes.c_void_p(out.data_ptr())))
    return out


def results_from_device(buf):
    """List of result dicts from the (n x 6) device tensor batch_async() returns."""
    dt = np.dtype([(k, "<f8" if i < 3 else "<i8") for i, k in enumerate(_RESULT_KEYS)])
    raw = buf.cpu().numpy().tobytes()
    return [dict(zip(_RESULT_KEYS, r)) for r in np.frombuffer(raw, dtype=dt).tolist()]


def membership(nx, ny, seed, b0, count, device="cuda"):
    """Splits b0..b0+count-1 as packed bits (count x ceil(n/32) int32 device tensor)."""
    import torch
    W = (nx + ny + 31) // 32
    words = torch.zeros((count, W), dtype=torch.int32, device=device)
    check(_lib.load().etest_membership(nx, ny, seed, b0, count, ctypes.c_void_p(words.data_ptr()),
                                       _stream()))
    return words


def unpack_words(words, n):
    """Packed membership words -> 0/1 uint8 array (count x n) on the host."""
    w = words.cpu().numpy().astype(np.uint32)
    bits = (w[:, :, None] >> np.arange(32, dtype=np.uint32)[None, None, :]) & 1
    return bits.reshape(w.shape[0], -1)[:, :n].astype(np.uint8)


def pack_splits(Z):
    """0/1 array (count x n) -> packed words (count x ceil(n/32)) as int32 numpy."""
    Z = np.asarray(Z, dtype=np.uint64)
    c, n = Z.shape
    W = (n + 31) // 32
    pad = np.zeros((c, W * 32), dtype=np.uint64)
    pad[:, :n] = Z
    pad = pad.reshape(c, W, 32)
    words = (pad << np.arange(32, dtype=np.uint64)[None, None, :]).sum(axis=2)
    return words.astype(np.uint32).view(np.int32)


def blocks(X, Y, kind="ed", prec="f32", gamma=0.0):
    """The three blocks (D_XX, D_YY, D_XY) as device tensors."""
    import torch
    _check_dev(X, Y, prec)
    dt = torch.float64 if _prec(prec) == PREC_F64 else torch.float32
    nx, ny = X.shape[0], Y.shape[0]
    dxx = torch.empty((nx, nx), dtype=dt, device=X.device)
    dyy = torch.empty((ny, ny), dtype=dt, device=X.device)
    dxy = torch.empty((nx, ny), dtype=dt, device=X.device)
    req = make_request(X, Y, 0, 0, kind, prec, gamma)
    check(_lib.load().etest_blocks(ctypes.byref(req), ctypes.c_void_p(dxx.data_ptr()),
                                   ctypes.c_void_p(dyy.data_ptr()),
                                   ctypes.c_void_p(dxy.data_ptr()), _stream()))
    return dxx, dyy, dxy


def perm_stats_from_membership(X, Y, words, kind="ed", prec="f32", gamma=0.0):
    """Statistics for caller-supplied splits (packed words, count x ceil(n/32), device int32)."""
    import torch
    _check_dev(X, Y, prec)
    count = words.shape[0]
    stats = torch.empty(count, dtype=torch.float64, device=X.device)
    req = make_request(X, Y, count, 0, kind, prec, gamma)
    r = Result()
    check(_lib.load().etest_perm_stats_from_membership(
        ctypes.byref(req), ctypes.c_void_p(words.data_ptr()), count,
        ctypes.c_void_p(stats.data_ptr()), _stream(), ctypes.byref(r)))
    out = r.as_dict()
    out["perm_stats"] = stats
    return out


def validate(nx, ny, p, B, kind="ed", prec="f32", gamma=1.0, X=1, Y=1):
    """Argument check without a device (returns the status code)."""
    r = Request()
    r.kind, r.prec, r.nx, r.ny, r.p, r.B, r.seed, r.gamma = (_kind(kind), _prec(prec), nx, ny, p,
                                                             B, 0, gamma)
    r.X, r.Y, r.perm_stats = X, Y, None
    return _lib.load().etest_validate(ctypes.byref(r))


def footprint(nx, ny, p, B, kind="ed", prec="f32"):
    r = Request()
    r.kind, r.prec, r.nx, r.ny, r.p, r.B, r.gamma = _kind(kind), _prec(prec), nx, ny, p, B, 1.0
    out = ctypes.c_int64()
    check(_lib.load().etest_footprint(ctypes.byref(r), ctypes.byref(out)))
    return out.value


def last_error():
    return _lib.load().etest_last_error().decode()


class Server:
    """Continuous-batching server over the C ABI.  Requests reference device tensors that
    must stay alive until the request completes (this wrapper keeps them)."""

    def __init__(self, memory_budget_bytes=32 << 30, max_resident=64, max_queue=1 << 20,
                 chunk_updates=0):
        cfg = _lib.ServerConfig(memory_budget_bytes, max_resident, max_queue, chunk_updates)
        self._h = ctypes.c_void_p()
        check(_lib.load().etest_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, X, Y, B, seed, kind="ed", prec="bf16r", gamma=0.0, perm_stats=None):
        """Queue one test; returns its id.  perm_stats: float64 device tensor of B or None."""
        _check_dev(X, Y, prec)
        req = make_request(X, Y, B, seed, kind, prec, gamma, perm_stats)
        rid = ctypes.c_uint64()
        check(_lib.load().etest_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._keep[rid.value] = (X, Y, perm_stats)
        return rid.value

    def poll(self, rid):
        """Result dict when finished, None while running."""
        r = Result()
        st = _lib.load().etest_server_poll(self._h, rid, ctypes.byref(r))
        if st == _lib.EBUSY:
            return None
        self._keep.pop(rid, None)
        check(st)
        return r.as_dict()

    def wait(self, rid):
        r = Result()
        st = _lib.load().etest_server_wait(self._h, rid, ctypes.byref(r))
        self._keep.pop(rid, None)
        check(st)
        return r.as_dict()

    def stats(self):
        q, res, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(_lib.load().etest_server_stats(self._h, ctypes.byref(q), ctypes.byref(res),
                                             ctypes.byref(b), ctypes.byref(c)))
        return {"queued": q.value, "resident": res.value, "bytes_held": b.value,
                "completed": c.value}

    def close(self):
        if self._h:
            check(_lib.load().etest_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def profile_enable(on=True, stages=None):
    """Stage timing on / off; `stages`: names from _lib.STAGES to time (default: all)."""
    if not on:
        mode = 0
    elif stages is None:
        mode = 1
    else:
        mode = sum(1 << (_lib.STAGES.index(s) + 1) for s in stages)
    check(_lib.load().etest_profile_enable(mode))


def profile_read():
    """{stage name: (total ms, launches)} for this thread's synchronous calls since enable."""
    n = len(_lib.STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    check(_lib.load().etest_profile_read(ms, cnt, n))
    return {name: (ms[k], cnt[k]) for k, name in enumerate(_lib.STAGES)}
