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

The BF16-refined form's 1e-3 bound holds on Gaussian data at every p: from 64
coordinates on its Gram reads BF16 operands, below that (where 8-bit coordinates
alone would move a distance by ~2^-9 / sqrt(p) of itself) the same fp16-pair
operands as the FP32 form.
"""
import sys

import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16r": 1e-3}


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
