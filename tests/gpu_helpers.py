"""Shared helpers of the GPU parity tests (comparison rules and tolerances).

Statistic tolerances, relative to the oracle: FP64 1e-12, FP32 1e-5,
BF16-refined 1e-3.  A resampled statistic near zero has no useful relative
error, so each one is compared on the scale max(|oracle value|, mean |oracle
null values|): the null mean is the positive floor of the statistic under
random splits (for ED it equals the mean off-diagonal distance times
(1/nx + 1/ny) in expectation), the size its block-entry errors are measured
against.  Exceedance decisions must agree split by split except for splits
whose oracle statistic lies within that tolerance of the oracle threshold
(near-ties); those are returned so a test can report them.

The BF16 form rounds every coordinate to 8 significant bits, which moves a
distance by about 0.6 * 2^-9 / sqrt(p) of itself on Gaussian data; its 1e-3
target therefore applies to high-dimensional data (p >= 64 here), and below
that the form is checked against the oracle run on the bf16-rounded data.
"""
import sys

import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16r": 1e-3}
BF16_MIN_P = 64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_run(g, o, prec, label="", tol=None):
    """g: result dict from the HIP path (perm_stats on host or device); o: oracle dict."""
    tol = TOL[prec] if tol is None else tol
    ps = g["perm_stats"]
    if ps is not None and not isinstance(ps, np.ndarray):
        ps = ps.cpu().numpy()
    ops = o["perm_stats"]
    so, to = o["statistic"], o["threshold"]
    B = len(ops)
    floor = float(np.mean(np.abs(ops))) if B else 0.0
    assert abs(g["statistic"] - so) <= tol * max(abs(so), floor) + 1e-300, (label, g["statistic"], so)
    assert abs(g["threshold"] - to) <= tol * max(abs(to), floor) + 1e-300, (label, g["threshold"], to)
    assert g["B"] == B
    near = np.zeros(B, dtype=bool)
    if B:
        err = np.abs(ps - ops)
        scale = np.maximum(np.abs(ops), floor)
        bad = err > tol * scale
        assert not np.any(bad), (label, int(np.argmax(err / scale)), float((err / scale).max()))
        near = np.abs(ops - to) <= tol * max(abs(to), floor)
        differ = (ps >= g["threshold"]) != (ops >= to)
        assert not np.any(differ & ~near), (label, np.flatnonzero(differ & ~near)[:10])
        assert g["count_ge"] == int(np.sum(ps >= g["threshold"]))
        if not np.any(differ):
            assert g["count_ge"] == o["count_ge"]
            assert g["p_value"] == o["p_value"]
    else:
        assert g["count_ge"] == 0 and g["p_value"] == 1.0
    return np.flatnonzero(near)


def bf16_round(a):
    """float32 array -> float32 values rounded to bfloat16 (round to nearest, ties to even)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_operands(X, Y):
    """The operands the BF16 form multiplies: pooled-column-mean centred, then bf16-rounded."""
    mean = (X.astype(np.float64).sum(0) + Y.astype(np.float64).sum(0)) / (len(X) + len(Y))
    Xc = bf16_round((X.astype(np.float64) - mean).astype(np.float32))
    Yc = bf16_round((Y.astype(np.float64) - mean).astype(np.float32))
    return Xc.astype(np.float64), Yc.astype(np.float64)
