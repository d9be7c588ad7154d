"""Parity at the benchmark workloads' full sizes, in the configuration the benchmark runs.

The oracle computes the three blocks by direct differences, the observed statistic, the
threshold and a sample of resampled splits one by one (the first and last splits plus a
seeded random sample); the GPU's count is checked against its own statistics, and its
exceedance decisions against the oracle's on the sampled splits.
"""
import numpy as np
import pytest

import oracle
from paper_2406_06488_amd import api, inputs
from tests.gpu_helpers import TOL, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KIND = {"ed": oracle.ED, "mmd": oracle.MMD}


def _sample(B, k=24, seed=0):
    g = np.random.Generator(np.random.PCG64(seed))
    idx = set(range(8)) | set(range(B - 8, B)) | set(int(x) for x in g.integers(0, B, size=k))
    return np.array(sorted(idx), dtype=np.int64)


def _check(wl, kind):
    X, Y = wl.data()
    dt = torch.float64 if wl.prec == "f64" else torch.float32
    Xd, Yd = torch.from_numpy(X).to("cuda:0", dt), torch.from_numpy(Y).to("cuda:0", dt)
    say("full-size", wl.name, kind)
    g = api.run(Xd, Yd, wl.B, wl.perm_seed, kind, wl.prec, wl.gamma())
    torch.cuda.synchronize()
    ps = g["perm_stats"].cpu().numpy()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    XX, YY, XY = oracle.blocks(X64, Y64, KIND[kind], wl.gamma())
    so, _ = oracle.observed(XX, YY, XY, KIND[kind])
    to = oracle.threshold(XX, YY, XY, KIND[kind])
    bl = _sample(wl.B)
    ops = oracle.perm_stats_listed(XX, YY, XY, wl.perm_seed, bl, KIND[kind])
    tol = TOL[wl.prec]
    floor = float(np.mean(np.abs(ops)))
    rel_stat = abs(g["statistic"] - so) / abs(so)
    rel_thr = abs(g["threshold"] - to) / abs(to)
    rel_perm = float(np.max(np.abs(ps[bl] - ops) / np.maximum(np.abs(ops), floor)))
    say("  statistic %.3e  threshold %.3e  sampled splits %.3e  (tolerance %.0e)  refined %d"
        % (rel_stat, rel_thr, rel_perm, tol, g["n_refined"]))
    assert rel_stat <= tol and rel_thr <= tol and rel_perm <= tol
    assert g["count_ge"] == int(np.sum(ps >= g["threshold"]))
    assert g["p_value"] == (1 + g["count_ge"]) / (1 + wl.B)
    near = np.abs(ops - to) <= tol * max(abs(to), floor)
    differ = (ps[bl] >= g["threshold"]) != (ops >= to)
    assert not np.any(differ & ~near)


def test_plain_f32_2000x1000_B10000():
    _check(inputs.plain_f32(), "ed")


@pytest.mark.parametrize("kind", ["ed", "mmd"])
def test_precision_bf16_5000x4000x4096_B10000(kind):
    _check(inputs.precision_bf16(), kind)


def test_small_f64_100x10_B1000_full():
    wl = inputs.small_null_f64()
    X, Y = wl.data()
    g = api.run(torch.from_numpy(X).to("cuda:0"), torch.from_numpy(Y).to("cuda:0"), wl.B,
                wl.perm_seed, "ed", "f64")
    o = oracle.run_test(X, Y, wl.B, wl.perm_seed)
    from tests.gpu_helpers import compare_run
    near = compare_run(g, o, "f64", wl.name)
    say("  f64 p =", g["p_value"], "oracle p =", o["p_value"], "near ties", near.tolist())
