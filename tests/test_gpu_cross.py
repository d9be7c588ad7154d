"""Cross-MMD / cross-ED tests (the paper's appendix, Alg. 6 and Alg. 7) through the C ABI
against the FP64 oracle, on the same seeded inputs.

U and sigma are compared on the scale of the block values they are built from (the mean
|value| of the four cross blocks: U can be near 0 under the null, so a relative error of U
itself means nothing there); z and p follow from them.  Tolerances as for the permutation
tests: 1e-12 (FP64), 1e-5 (FP32), 1e-3 (BF16-refined)."""
import math

import numpy as np
import pytest

import oracle
from paper_2406_06488_amd import api, inputs
from paper_2406_06488_amd._lib import EtestError
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
KIND = {"ed": oracle.ED, "mmd": oracle.MMD}
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16r": 1e-3}


def _dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dt)


def _scale(X, Y, kind, gamma):
    nx1, ny1 = X.shape[0] // 2, Y.shape[0] // 2
    parts = [(X[:nx1], X[nx1:]), (Y[:ny1], Y[ny1:]), (X[:nx1], Y[ny1:]), (Y[:ny1], X[nx1:])]
    return max(np.abs(oracle.block(a, b, KIND[kind], gamma)).mean() for a, b in parts)


CASES = [
    # nx, ny, p, data seed, shift
    (301, 170, 37, 1, 0.15),    # x2 / y2 boundary inside a tile, ragged tails
    (129, 127, 64, 2, 0.0),     # null case
    (2, 3, 5, 3, 0.5),          # smallest halves
    (700, 650, 130, 4, 0.05),
    (260, 190, 1030, 5, 0.1),   # many 32-column slices
]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
@pytest.mark.parametrize("kind", ["ed", "mmd"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_cross_matches_oracle(case, kind, prec):
    nx, ny, p, ds, shift = CASES[case]
    say("cross", case, kind, prec, nx, ny, p)
    dt = np.float64 if prec == "f64" else np.float32
    X, Y = inputs.gaussian_pair(nx, ny, p, ds, mean_shift=shift, dtype=dt)
    gamma = 1.0 / p
    g = api.cross(_dev(X, prec), _dev(Y, prec), kind, prec, gamma)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    o = oracle.cross(X64, Y64, KIND[kind], gamma)
    S = _scale(X64, Y64, kind, gamma)
    tol = TOL[prec] * S
    assert abs(g["statistic"] - o["statistic"]) <= tol, (g, o, S)
    assert abs(g["sigma"] - o["sigma"]) <= tol, (g, o, S)
    if o["sigma"] > 0:
        dz = (tol + abs(o["z"]) * tol) / o["sigma"]
        assert abs(g["z"] - o["z"]) <= dz * 1.01 + 1e-12, (g, o)
        phi = math.exp(-0.5 * min(o["z"] ** 2, 700.0)) / math.sqrt(2 * math.pi)
        assert abs(g["p_value"] - o["p_value"]) <= 1.01 * phi * dz * (1 + abs(o["z"])) + 1e-13, (g, o)
    if prec != "bf16r":
        assert g["n_refined"] == 0 or prec == "f32"


def test_cross_identical_samples():
    """y = x: every row's two means are the same numbers, summed over differently aligned
    tiles, so U and sigma vanish up to FP64 summation order (the oracle, with exact sums,
    gives exactly 0)."""
    X, _ = inputs.gaussian_pair(200, 200, 16, 9, dtype=np.float64)
    g = api.cross(_dev(X, "f64"), _dev(X.copy(), "f64"), "ed", "f64")
    S = _scale(X, X, "ed", 1.0)
    assert abs(g["statistic"]) <= 1e-13 * S and g["sigma"] <= 1e-13 * S, g


def test_cross_swap_symmetry():
    X, Y = inputs.gaussian_pair(333, 210, 40, 11, mean_shift=0.2, dtype=np.float32)
    a = api.cross(_dev(X, "f32"), _dev(Y, "f32"), "mmd", "f32", 1.0 / 40)
    b = api.cross(_dev(Y, "f32"), _dev(X, "f32"), "mmd", "f32", 1.0 / 40)
    for k in ("statistic", "sigma", "p_value"):
        assert abs(a[k] - b[k]) <= 1e-5 * max(abs(a[k]), 1e-3), (k, a, b)


def test_cross_rejects_bad_input():
    X, Y = inputs.gaussian_pair(10, 9, 4, 12, dtype=np.float32)
    with pytest.raises(EtestError):
        api.cross(_dev(X[:1], "f32"), _dev(Y, "f32"), "ed", "f32")
    bad = X.copy()
    bad[3, 2] = np.nan
    with pytest.raises(EtestError):
        api.cross(_dev(bad, "f32"), _dev(Y, "f32"), "ed", "f32")
