"""Shared helpers of the GPU parity tests (comparison rules and tolerances).

Tolerances on statistics, relative to the oracle's value: FP64 1e-12, FP32
1e-5, BF16-refined 1e-3.  Exceedance decisions must agree split by split,
except for splits whose oracle statistic lies within that tolerance of the
oracle threshold (near-ties); those are returned so a test can report them.
"""
import sys

import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16r": 1e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_run(g, o, prec, label=""):
    """g: result dict from the HIP path (perm_stats on host or device); o: oracle dict."""
    tol = TOL[prec]
    ps = g["perm_stats"]
    if ps is not None and not isinstance(ps, np.ndarray):
        ps = ps.cpu().numpy()
    ops = o["perm_stats"]
    so, to = o["statistic"], o["threshold"]
    assert abs(g["statistic"] - so) <= tol * abs(so) + 1e-300, (label, g["statistic"], so)
    assert abs(g["threshold"] - to) <= tol * abs(to) + 1e-300, (label, g["threshold"], to)
    B = len(ops)
    assert g["B"] == B
    near = np.zeros(B, dtype=bool)
    if B:
        err = np.abs(ps - ops)
        bad = err > tol * np.abs(ops)
        assert not np.any(bad), (label, int(np.argmax(err)), float(err.max()),
                                 ops[np.argmax(err)])
        near = np.abs(ops - to) <= tol * abs(to)
        differ = (ps >= g["threshold"]) != (ops >= to)
        assert not np.any(differ & ~near), (label, np.flatnonzero(differ & ~near)[:10])
        assert g["count_ge"] == int(np.sum(ps >= g["threshold"]))
        if not np.any(differ):
            assert g["count_ge"] == o["count_ge"]
            assert g["p_value"] == o["p_value"]
    else:
        assert g["count_ge"] == 0 and g["p_value"] == 1.0
    return np.flatnonzero(near)
