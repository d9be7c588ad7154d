"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage or fact it relies on.  None re-types the
oracle's own formula: they compare it with independent code (Alg. 4 / Alg. 5
brute force, math.fsum, scipy), printed worked examples, closed forms and
invariants.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from oracle import brute
from tests.conftest import GOLDEN

ED, MMD = oracle.ED, oracle.MMD


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------- sums

def test_exact_sum_matches_fsum():
    g = _rng(11)
    for trial in range(40):
        n = int(g.integers(1, 3000))
        v = g.standard_normal(n) * 10.0 ** g.uniform(-20, 20, size=n)
        if trial % 3 == 0:  # heavy cancellation
            v = np.concatenate([v, -v[: n // 2] * (1 + 1e-15)])
        assert oracle.xsum(v) == math.fsum(v)
    # half-way rounding cases
    for v in ([1.0, 2.0 ** -53], [1.0, 2.0 ** -53, 2.0 ** -106], [1.0, -(2.0 ** -54), -(2.0 ** -108)],
              [1e308, 1e308 * 0.5, -1e308]):
        assert oracle.xsum(np.array(v)) == math.fsum(v)


# --------------------------------------------------------------------------- split stream

def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split("->")
            w = [int(x, 16) for x in lhs.split()]
            rows.append((w[:4], w[4:6], [int(x, 16) for x in rhs.split()]))
    return rows


def test_philox_known_answers():
    for ctr, key, want in _kat():
        assert list(oracle.philox4x32_10(ctr, key)) == want
        assert brute.philox4x32_10(ctr, key) == want


def test_philox_two_implementations_agree():
    g = _rng(5)
    for _ in range(200):
        ctr = [int(x) for x in g.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        key = [int(x) for x in g.integers(0, 2 ** 32, size=2, dtype=np.uint64)]
        assert list(oracle.philox4x32_10(ctr, key)) == brute.philox4x32_10(ctr, key)


@pytest.mark.parametrize("nx,ny,seed", [(5, 4, 0), (1, 1, 7), (7, 31, 2 ** 40 + 3),
                                        (33, 64, 123456789), (100, 100, 1)])
def test_membership_two_implementations_agree(nx, ny, seed):
    for b in [0, 1, 2, 17, 999, 2 ** 32 + 5]:
        z = oracle.membership(nx, ny, seed, b)
        assert z.sum() == nx
        assert np.array_equal(z, brute.membership(nx, ny, seed, b))


def test_membership_splits_uniform():
    """Every one of the C(6,3) = 20 splits is equally likely (chi-square)."""
    nx, ny, draws = 3, 3, 20000
    counts = {}
    for b in range(draws):
        key = tuple(oracle.membership(nx, ny, 9, b))
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 20
    exp = draws / 20
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    # 19 degrees of freedom: P(chi2 > 43.8) = 0.001
    assert chi2 < 43.8


def test_membership_inclusion_rates():
    """Each item joins x* with rate nx/n; each pair with nx(nx-1)/(n(n-1))."""
    nx, ny, draws = 7, 5, 12000
    n = nx + ny
    Z = np.array([oracle.membership(nx, ny, 3, b) for b in range(draws)], dtype=np.float64)
    rate = Z.mean(axis=0)
    sd = math.sqrt((nx / n) * (1 - nx / n) / draws)
    assert np.all(np.abs(rate - nx / n) < 5 * sd)
    pair = (Z.T @ Z) / draws
    q = nx * (nx - 1) / (n * (n - 1))
    sdq = math.sqrt(q * (1 - q) / draws)
    off = pair[~np.eye(n, dtype=bool)]
    assert np.all(np.abs(off - q) < 5 * sdq)


def test_resumed_ranges_equal_one_shot():
    """Split b depends on (seed, b) only, so b-ranges concatenate to the one-shot run."""
    g = _rng(3)
    X = g.standard_normal((6, 2))
    Y = g.standard_normal((5, 2))
    XX, YY, XY = oracle.blocks(X, Y)
    one = oracle.perm_stats_listed(XX, YY, XY, 77, np.arange(40))
    parts = np.concatenate([oracle.perm_stats_listed(XX, YY, XY, 77, np.arange(0, 13)),
                            oracle.perm_stats_listed(XX, YY, XY, 77, np.arange(13, 40))])
    assert np.array_equal(one, parts)
    full = oracle.run_test(X, Y, 40, 77)
    assert np.array_equal(full["perm_stats"], one)


# --------------------------------------------------------------------------- worked example

def _read_toy():
    d = {}
    with open(os.path.join(GOLDEN, "toy_split.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            d[k] = [int(x) for x in v]
    return d


def test_toy_split_indices():
    """Alg. 2 on the paper's worked permutation (Appendix A.4)."""
    t = _read_toy()
    nx, ny = t["nx"][0], t["ny"][0]
    z = np.zeros(nx + ny, dtype=np.uint8)
    z[np.array(t["idx_p1"]) - 1] = 1
    assert sorted(np.flatnonzero(z == 0) + 1) == sorted(t["idx_p2"])
    i1, i2, j1, j2 = oracle.split_indices(nx, ny, z)
    assert sorted(i1 + 1) == sorted(t["i1"])
    assert sorted(i2 + 1) == sorted(t["i2"])
    assert sorted(j1 + 1) == sorted(t["j1"])
    assert sorted(j2 + 1) == sorted(t["j2"])
    # the starred positions are 1..len(i1) then the rest (Alg. 2)
    assert t["i1star"] == list(range(1, len(i1) + 1))
    assert t["i2star"] == list(range(len(i1) + 1, nx + 1))
    assert t["j1star"] == list(range(1, len(j1) + 1))
    assert t["j2star"] == list(range(len(j1) + 1, ny + 1))


def _read_toy_blocks():
    mats, cur = {}, None
    with open(os.path.join(GOLDEN, "toy_permuted_blocks.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                mats[cur] = []
            else:
                mats[cur].append([tuple(e.split(",")) for e in line.split()])
    return mats


@pytest.mark.parametrize("kind", [ED, MMD])
def test_toy_permuted_block_sums(kind):
    """The three permuted blocks printed in Appendix A.4, evaluated on random data, sum to
    what the oracle's Alg. 1 assembly sums to (catches a swapped or transposed sub-block)."""
    t = _read_toy()
    nx, ny = t["nx"][0], t["ny"][0]
    g = _rng(21)
    X = g.standard_normal((nx, 3))
    Y = g.standard_normal((ny, 3))
    gamma = 0.7
    pts = {"x%d" % (i + 1): X[i] for i in range(nx)}
    pts.update({"y%d" % (i + 1): Y[i] for i in range(ny)})

    def k(a, b):
        d2 = math.fsum((pts[a] - pts[b]) ** 2)
        return math.sqrt(d2) if kind == ED else math.exp(-gamma * d2)

    mats = _read_toy_blocks()
    want = [math.fsum(k(a, b) for row in mats[m] for (a, b) in row)
            for m in ("XsXs", "YsYs", "XsYs")]
    z = np.zeros(nx + ny, dtype=np.uint8)
    z[np.array(t["idx_p1"]) - 1] = 1
    XX, YY, XY = oracle.blocks(X, Y, kind, gamma)
    got = oracle.perm_sums(XX, YY, XY, z)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=0)


# --------------------------------------------------------------------------- Alg 1 = Alg 4 = Alg 5

@pytest.mark.parametrize("nx,ny,p", [(1, 1, 1), (1, 3, 2), (4, 2, 3), (5, 4, 3), (6, 9, 2),
                                     (9, 6, 4)])
@pytest.mark.parametrize("kind", [ED, MMD])
def test_efficient_equals_standard_and_precomputed(nx, ny, p, kind):
    """The efficient test gives the same statistic as the standard (Alg. 4) and the
    pre-computation (Alg. 5) tests on the same permutations (Section 1 / Section 2 claim)."""
    g = _rng(100 + nx * 10 + ny)
    X = g.standard_normal((nx, p))
    Y = g.standard_normal((ny, p)) + 0.3
    gamma = 1.0 / p
    XX, YY, XY = oracle.blocks(X, Y, kind, gamma)
    splits = [oracle.membership(nx, ny, 5, b) for b in range(12)]
    splits.append(np.r_[np.ones(nx), np.zeros(ny)].astype(np.uint8))
    eff = [oracle.perm_stat(XX, YY, XY, z, kind) for z in splits]
    std = brute.standard_test_stats(X, Y, splits, kind, gamma)
    pre = brute.precomputed_test_stats(X, Y, splits, kind, gamma)
    scale = max(abs(v) for v in std) + 1e-300
    for e, s, q in zip(eff, std, pre):
        assert abs(e - s) <= 1e-13 * scale
        assert abs(e - q) <= 1e-13 * scale
    # observed statistic (eq. 1/2) against the direct computation
    obs, _ = oracle.observed(XX, YY, XY, kind)
    assert abs(obs - brute.statistic(X, Y, kind, gamma)) <= 1e-13 * scale


def test_identity_split_equals_observed():
    """With exact sums, the identity split reproduces the observed statistic bit for bit."""
    g = _rng(8)
    for kind in (ED, MMD):
        X = g.standard_normal((17, 5))
        Y = g.standard_normal((11, 5))
        XX, YY, XY = oracle.blocks(X, Y, kind, 0.2)
        obs, _ = oracle.observed(XX, YY, XY, kind)
        assert oracle.threshold(XX, YY, XY, kind) == obs


# --------------------------------------------------------------------------- invariants

def test_energy_distance_properties():
    g = _rng(12)
    X = g.standard_normal((9, 4))
    Y = g.standard_normal((7, 4)) + 0.5
    XX, YY, XY = oracle.blocks(X, Y)
    ed, _ = oracle.observed(XX, YY, XY)
    assert ed > 0
    # ED(X, X) = 0 exactly
    A, B, C = oracle.blocks(X, X)
    assert oracle.observed(A, B, C)[0] == 0.0
    # symmetric under swapping the samples
    A, B, C = oracle.blocks(Y, X)
    assert oracle.observed(A, B, C)[0] == ed
    # invariant to row order within each sample
    A, B, C = oracle.blocks(X[::-1], Y[g.permutation(7)])
    assert oracle.observed(A, B, C)[0] == ed
    # translation and rotation of both samples together
    Q, _ = np.linalg.qr(g.standard_normal((4, 4)))
    A, B, C = oracle.blocks(X @ Q + 3.0, Y @ Q + 3.0)
    assert abs(oracle.observed(A, B, C)[0] - ed) < 1e-12 * ed
    # every split gives ED* >= 0 and MMD* >= 0 (negative-type metric / PD kernel)
    Xs, Ys = X[:5], Y[:4]
    XX, YY, XY = oracle.blocks(Xs, Ys)
    KX, KY, KXY = oracle.blocks(Xs, Ys, MMD, 0.3)
    for z in brute.all_splits(5, 4):
        assert oracle.perm_stat(XX, YY, XY, z) >= 0.0
        assert oracle.perm_stat(KX, KY, KXY, z, MMD) >= -1e-15


def test_row_offset_invariance():
    """Adding f(a) + f(b) to every pooled pair (a, b) leaves every resampled statistic
    unchanged: each pooled row of ED weights sums to zero (-nx/nx^2 + ny/(nx ny) = 0)."""
    g = _rng(14)
    nx, ny = 6, 8
    X = g.standard_normal((nx, 3))
    Y = g.standard_normal((ny, 3))
    f = g.standard_normal(nx + ny) * 5.0
    fx, fy = f[:nx], f[nx:]
    for kind in (ED, MMD):
        XX, YY, XY = oracle.blocks(X, Y, kind, 0.5)
        XX2 = XX + fx[:, None] + fx[None, :]
        YY2 = YY + fy[:, None] + fy[None, :]
        XY2 = XY + fx[:, None] + fy[None, :]
        for b in range(20):
            z = oracle.membership(nx, ny, 4, b)
            a = oracle.perm_stat(XX, YY, XY, z, kind)
            c = oracle.perm_stat(XX2, YY2, XY2, z, kind)
            assert abs(a - c) < 1e-12 * (abs(a) + 1.0)


def test_mmd_of_distance_induced_kernel_is_half_ed():
    """With k(a,b) = (|a| + |b| - |a-b|)/2, MMD_b^2 = ED/2 for every split."""
    g = _rng(15)
    nx, ny = 5, 7
    X = g.standard_normal((nx, 3))
    Y = g.standard_normal((ny, 3)) + 0.4
    XX, YY, XY = oracle.blocks(X, Y)
    nX = np.linalg.norm(X, axis=1)
    nY = np.linalg.norm(Y, axis=1)
    KX = 0.5 * (nX[:, None] + nX[None, :] - XX)
    KY = 0.5 * (nY[:, None] + nY[None, :] - YY)
    KXY = 0.5 * (nX[:, None] + nY[None, :] - XY)
    for b in range(25):
        z = oracle.membership(nx, ny, 6, b)
        e = oracle.perm_stat(XX, YY, XY, z, ED)
        m = oracle.perm_stat(KX, KY, KXY, z, MMD)
        assert abs(m - e / 2) < 1e-13 * abs(e)


# --------------------------------------------------------------------------- exact enumeration

@pytest.mark.parametrize("kind", [ED, MMD])
def test_exact_enumeration_nx5_ny5(kind):
    """nx = ny = 5: all C(10,5) = 252 splits.  (a) The exact permutation p-value; (b) each
    drawn split's statistic is the table entry of that split, so the count of a run is
    reproduced by lookup; (c) the average over all splits has a closed form."""
    nx = ny = 5
    n = nx + ny
    g = _rng(31)
    X = g.standard_normal((nx, 4))
    Y = g.standard_normal((ny, 4)) + 0.6
    gamma = 0.25
    XX, YY, XY = oracle.blocks(X, Y, kind, gamma)
    table = {}
    for z in brute.all_splits(nx, ny):
        table[tuple(z)] = oracle.perm_stat(XX, YY, XY, z, kind)
    assert len(table) == math.comb(n, nx) == 252
    thr = oracle.threshold(XX, YY, XY, kind)
    # the complement of the identity ties with it exactly (nx = ny, exact sums)
    comp = tuple([0] * nx + [1] * ny)
    assert table[comp] == thr
    exact_p = sum(v >= thr for v in table.values()) / 252
    assert 2 / 252 <= exact_p <= 1
    # Alg. 2 sampling: lookup reproduces the oracle's own count
    B = 3000
    run = oracle.run_test(X, Y, B, 17, kind, gamma)
    looked = [table[tuple(oracle.membership(nx, ny, 17, b))] for b in range(B)]
    assert np.array_equal(np.array(looked), run["perm_stats"])
    assert run["count_ge"] == sum(v >= thr for v in looked)
    # the Monte Carlo p-value estimates the exact one
    assert abs(run["p_value"] - exact_p) < 5 * math.sqrt(exact_p * (1 - exact_p) / B) + 1e-3
    # (c) mean over splits
    W = np.concatenate([X, Y])
    Dww = oracle.block(W, W, kind, gamma)
    T_off = math.fsum(Dww[~np.eye(n, dtype=bool)])
    mean = math.fsum(table.values()) / 252
    if kind == ED:
        want = T_off * (1 / nx + 1 / ny) / (n * (n - 1))
    else:
        want = (1 / nx + 1 / ny) * (1 - T_off / (n * (n - 1)))
    assert abs(mean - want) < 1e-13 * abs(want)


# --------------------------------------------------------------------------- hand cases

def _hand_cases():
    out = []
    with open(os.path.join(GOLDEN, "hand_cases.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, xs, ys, stat, pv = [s.strip() for s in line.split("|")]
            kind, gamma = head.split()
            out.append((ED if kind == "ed" else MMD, float(gamma),
                        np.array([[float(v)] for v in xs.split()]),
                        np.array([[float(v)] for v in ys.split()]),
                        eval(stat, {"exp": math.exp}), eval(pv)))
    return out


@pytest.mark.parametrize("case", range(4))
def test_hand_cases(case):
    kind, gamma, X, Y, stat, pv = _hand_cases()[case]
    XX, YY, XY = oracle.blocks(X, Y, kind, gamma)
    assert abs(oracle.observed(XX, YY, XY, kind)[0] - stat) <= 1e-15 * abs(stat)
    thr = oracle.threshold(XX, YY, XY, kind)
    vals = [oracle.perm_stat(XX, YY, XY, z, kind) for z in brute.all_splits(len(X), len(Y))]
    assert abs(sum(v >= thr for v in vals) / len(vals) - pv) < 1e-15


def test_single_points_closed_form():
    """nx = ny = 1: ED = 2|x - y|, and both splits tie, so p = 1 for any B."""
    g = _rng(41)
    x = g.standard_normal((1, 6))
    y = g.standard_normal((1, 6))
    r = oracle.run_test(x, y, 50, 3)
    d = oracle.block(x, y)[0, 0]
    assert r["statistic"] == 2 * d
    assert r["count_ge"] == 50 and r["p_value"] == 1.0


def test_zero_permutations():
    g = _rng(42)
    r = oracle.run_test(g.standard_normal((4, 2)), g.standard_normal((3, 2)), 0, 1)
    assert r["p_value"] == 1.0 and r["count_ge"] == 0


def test_pvalue_bounds():
    g = _rng(43)
    X = g.standard_normal((20, 3))
    Y = g.standard_normal((15, 3)) + 2.0   # strong shift: p at its floor
    r = oracle.run_test(X, Y, 99, 8)
    assert r["p_value"] == pytest.approx(1 / 100)
    r = oracle.run_test(X, X[:15] * 1.0, 99, 8)
    assert 1 / 100 <= r["p_value"] <= 1.0


# --------------------------------------------------------------------------- distances

def test_distance_blocks_against_scipy():
    g = _rng(51)
    A = g.standard_normal((13, 7))
    B = g.standard_normal((9, 7))
    np.testing.assert_allclose(oracle.block(A, B), cdist(A, B), rtol=1e-14, atol=1e-15)
    K = oracle.block(A, B, MMD, 0.3)
    np.testing.assert_allclose(K, np.exp(-0.3 * cdist(A, B, "sqeuclidean")), rtol=1e-14)
    # Pythagorean points: exact
    P = np.array([[0.0, 0.0], [3.0, 4.0], [5.0, 12.0], [8.0, 15.0]])
    D = oracle.block(P, P)
    assert D[0, 1] == 5.0 and D[0, 2] == 13.0 and D[0, 3] == 17.0 and D[1, 1] == 0.0
    assert np.array_equal(D, D.T)


# --------------------------------------------------------------------------- cross tests

def _h_quadruple_mean(X, Y, kind, gamma):
    """The cross statistic by its definition: the mean over all index quadruples
    (i in x1, i' in x2, j in y1, j' in y2) of h_K (cross-MMD) or h_D (cross-ED), written as
    plain loops over pairwise distances from scipy (no block means)."""
    nx1, ny1 = X.shape[0] // 2, Y.shape[0] // 2
    x1, x2, y1, y2 = X[:nx1], X[nx1:], Y[:ny1], Y[ny1:]
    d = lambda A, B: cdist(A, B)  # noqa: E731
    k = (lambda A, B: d(A, B)) if kind == ED else (lambda A, B: np.exp(-gamma * d(A, B) ** 2))
    kx1x2, kx1y2, ky1x2, ky1y2 = k(x1, x2), k(x1, y2), k(y1, x2), k(y1, y2)
    total, count = [], 0
    for i in range(len(x1)):
        for ip in range(len(x2)):
            for j in range(len(y1)):
                for jp in range(len(y2)):
                    if kind == ED:  # D(x_i, y_j') - D(x_i, x_i') - D(y_j, y_j') + D(y_j, x_i')
                        h = kx1y2[i, jp] - kx1x2[i, ip] - ky1y2[j, jp] + ky1x2[j, ip]
                    else:  # K(x_i, x_i') - K(x_i, y_j') - K(y_j, x_i') + K(y_j, y_j')
                        h = kx1x2[i, ip] - kx1y2[i, jp] - ky1x2[j, ip] + ky1y2[j, jp]
                    total.append(h)
                    count += 1
    return math.fsum(total) / count


@pytest.mark.parametrize("kind", [ED, MMD])
@pytest.mark.parametrize("nx,ny", [(4, 5), (7, 6), (2, 9)])
def test_cross_statistic_is_the_quadruple_mean(kind, nx, ny):
    """Appendix, cross-ED test: the statistic U of Alg. 6 / Alg. 7 (differences of block
    means) equals the V-statistic of h over all quadruples (brute force on tiny inputs)."""
    g = _rng(300 + nx * 10 + ny)
    X, Y = g.standard_normal((nx, 3)), g.standard_normal((ny, 3)) + 0.4
    gamma = 0.3
    got = oracle.cross(X, Y, kind, gamma)["statistic"]
    want = _h_quadruple_mean(X, Y, kind, gamma)
    assert abs(got - want) <= 1e-13 * max(1.0, abs(want))


@pytest.mark.parametrize("kind", [ED, MMD])
def test_cross_swap_symmetry_and_identical_samples(kind):
    """Swapping x and y leaves U, sigma and p unchanged (U_x and U_y trade places with
    their signs flipped); with y = x every block pair cancels row by row: U = 0, sigma = 0,
    and by the reading for sigma = 0, z = 0 and p = 1/2."""
    g = _rng(41)
    X, Y = g.standard_normal((31, 4)), g.standard_normal((26, 4)) * 1.3
    a, b = oracle.cross(X, Y, kind, 0.2), oracle.cross(Y, X, kind, 0.2)
    for k in ("statistic", "sigma", "p_value"):
        assert abs(a[k] - b[k]) <= 1e-13 * max(1.0, abs(a[k])), k
    same = oracle.cross(X, X.copy(), kind, 0.2)
    assert same["statistic"] == 0.0 and same["sigma"] == 0.0 and same["p_value"] == 0.5


def test_cross_ed_equals_cross_mmd_form_on_distances():
    """The paper's remark closing the cross-ED appendix: the cross-ED test is Alg. 6 with
    the four distance blocks in place of the kernel blocks and p = 1 - Phi(-U/sigma).
    That form is computed here from the oracle's distance blocks; its U is the negative
    of Alg. 7's, its sigma the same, and its p-value equal."""
    from scipy.stats import norm
    g = _rng(52)
    X, Y = g.standard_normal((45, 6)), g.standard_normal((38, 6)) + 0.25
    nx1, ny1 = 22, 19
    x1, x2, y1, y2 = X[:nx1], X[nx1:], Y[:ny1], Y[ny1:]
    b = lambda A, B: oracle.block(A, B, ED)  # noqa: E731
    kx1x2, ky1y2, kx1y2, ky1x2 = b(x1, x2), b(y1, y2), b(x1, y2), b(y1, x2)
    ux = kx1x2.mean() - kx1y2.mean()
    uy = ky1x2.mean() - ky1y2.mean()
    u = ux - uy
    sx = np.mean((kx1x2.mean(1) - kx1y2.mean(1) - ux) ** 2)
    sy = np.mean((ky1x2.mean(1) - ky1y2.mean(1) - uy) ** 2)
    sigma = math.sqrt(sx / nx1 + sy / ny1)
    p = norm.sf(-u / sigma)
    o = oracle.cross(X, Y, ED)
    assert abs(o["statistic"] + u) <= 1e-12 * abs(u)
    assert abs(o["sigma"] - sigma) <= 1e-12 * sigma
    assert abs(o["p_value"] - p) <= 1e-12 * max(p, 1e-300)


def test_cross_p_value_is_the_normal_upper_tail():
    """p = 1 - Phi(z) (Alg. 6 / Alg. 7 last line) against scipy's normal survival function,
    including far tails, where 1 - Phi would lose every digit."""
    from scipy.stats import norm
    g = _rng(63)
    for shift in (0.0, 0.05, 0.2, 0.6, 1.5, -0.3):
        X, Y = g.standard_normal((80, 5)), g.standard_normal((70, 5)) + shift
        for kind in (ED, MMD):
            o = oracle.cross(X, Y, kind, 0.2)
            assert abs(o["z"] - o["statistic"] / o["sigma"]) <= 1e-15 * abs(o["z"]) + 1e-300
            want = norm.sf(o["z"])
            assert abs(o["p_value"] - want) <= 1e-12 * want, (shift, kind, o, want)


def test_cross_null_p_values_are_roughly_uniform():
    """Under the null the studentised statistic is asymptotically N(0, 1) (the reason the
    cross tests need no permutations), so p-values over many null replications are close
    to uniform (a loose Kolmogorov-Smirnov check)."""
    from scipy.stats import kstest
    g = _rng(74)
    ps = []
    for rep in range(300):
        X, Y = g.standard_normal((60, 3)), g.standard_normal((60, 3))
        ps.append(oracle.cross(X, Y, ED)["p_value"])
    assert kstest(ps, "uniform").pvalue > 1e-3


def test_cross_rejects_too_few_rows():
    with pytest.raises(ValueError):
        oracle.cross(np.zeros((1, 3)), np.zeros((4, 3)), ED)
    with pytest.raises(ValueError):
        oracle.cross(np.zeros((4, 3)), np.zeros((4, 3)), MMD, 0.0)


# --------------------------------------------------------------------------- HSIC

def _gauss_kernel(A, gamma):
    return np.exp(-gamma * cdist(A, A, "sqeuclidean"))


def _hsic_u_statistic(K, L):
    """Unbiased HSIC as the U-statistic of Song et al. (2012, Theorem 2): the mean over
    ordered 4-tuples of distinct indices of h = (1/24) sum over the 24 orderings (s,t,u,v)
    of k_st l_st + k_st l_uv - 2 k_st l_su.  Independent of the oracle's closed form."""
    n = K.shape[0]
    total = []
    for quad in itertools.permutations(range(n), 4):
        h = []
        for s, t, u, v in itertools.permutations(quad):
            h.append(K[s, t] * L[s, t] + K[s, t] * L[u, v] - 2.0 * K[s, t] * L[s, u])
        total.append(math.fsum(h) / 24.0)
    return math.fsum(total) / len(total)


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_hsic_is_the_u_statistic(n):
    """The discussion's HSIC (Song et al.'s unbiased estimator) equals its U-statistic over
    distinct 4-tuples: pins all three terms, their coefficients and the 1/(n(n-3)) scale."""
    g = _rng(400 + n)
    X, Y = g.standard_normal((n, 3)), g.standard_normal((n, 2))
    Y[:, 0] += X[:, 0]  # dependent, so the terms do not nearly cancel
    K, L = _gauss_kernel(X, 0.4), _gauss_kernel(Y, 0.7)
    ref = _hsic_u_statistic(K, L)
    assert abs(oracle.hsic(K, L) - ref) <= 1e-13 * max(1.0, abs(ref)), (oracle.hsic(K, L), ref)
    # the same through a permutation of y: the U-statistic of the reordered kernel matrix
    pi = oracle.permutation(n, 3, 1)
    ref_p = _hsic_u_statistic(K, L[np.ix_(pi, pi)])
    assert abs(oracle.hsic(K, L, pi) - ref_p) <= 1e-13 * max(1.0, abs(ref_p))


def test_hsic_permuted_read_equals_reordered_data():
    """Reading L through pi is HSIC of (x_i, y_pi(i)): the kernel matrix of the reordered y."""
    g = _rng(41)
    n = 40
    X, Y = g.standard_normal((n, 5)), g.standard_normal((n, 3))
    K = _gauss_kernel(X, 0.2)
    for b in range(5):
        pi = oracle.permutation(n, 9, b)
        a = oracle.hsic(K, _gauss_kernel(Y, 0.3), pi)
        c = oracle.hsic(K, _gauss_kernel(Y[pi], 0.3))
        assert abs(a - c) <= 1e-14 * max(abs(c), 1e-3)


def test_hsic_joint_permutation_invariance_and_symmetry():
    """Relabelling the pairs leaves HSIC unchanged; HSIC(K, L) = HSIC(L, K)."""
    g = _rng(42)
    n = 33
    X, Y = g.standard_normal((n, 4)), g.standard_normal((n, 4))
    Y += 0.5 * X
    K, L = _gauss_kernel(X, 0.25), _gauss_kernel(Y, 0.25)
    s = g.permutation(n)
    h = oracle.hsic(K, L)
    assert abs(oracle.hsic(K[np.ix_(s, s)], L[np.ix_(s, s)]) - h) <= 1e-14 * abs(h)
    assert abs(oracle.hsic(L, K) - h) <= 1e-14 * abs(h)


def test_hsic_unbiased_under_independence():
    """Unbiased estimator: under independence its mean over datasets is 0 (population HSIC)."""
    g = _rng(43)
    vals = []
    for _ in range(1500):
        X, Y = g.standard_normal((12, 2)), g.standard_normal((12, 2))
        vals.append(oracle.hsic(_gauss_kernel(X, 0.5), _gauss_kernel(Y, 0.5)))
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean()) < 4.0 * se, (vals.mean(), se)
    # and positive in expectation under dependence
    dep = [oracle.hsic(_gauss_kernel(X, 0.5), _gauss_kernel(X + 0.3 * g.standard_normal(X.shape), 0.5))
           for X in (g.standard_normal((12, 2)) for _ in range(200))]
    assert np.mean(dep) > 10 * se


def test_permutations_are_uniform_permutations():
    """Each draw is a permutation; for n = 4 all 24 orders appear equally often (chi-square),
    and every item is equally likely at every position (n = 7)."""
    seen = {}
    for b in range(24000):
        pi = oracle.permutation(4, 77, b)
        seen[tuple(pi)] = seen.get(tuple(pi), 0) + 1
    assert len(seen) == 24
    from scipy.stats import chisquare
    assert chisquare(list(seen.values())).pvalue > 1e-3
    pos = np.zeros((7, 7))
    for b in range(7000):
        pi = oracle.permutation(7, 5, b)
        assert sorted(pi.tolist()) == list(range(7))
        pos[np.arange(7), pi] += 1
    assert chisquare(pos.ravel()).pvalue > 1e-3
    # the stream depends on the seed and on b
    assert not np.array_equal(oracle.permutation(50, 1, 0), oracle.permutation(50, 2, 0))
    assert not np.array_equal(oracle.permutation(50, 1, 0), oracle.permutation(50, 1, 1))


def test_hsic_test_null_uniform_and_detects_dependence():
    """Permutation test: p-values roughly uniform under independence, small under a clear
    dependence; p in [1/(B+1), 1] with the identity as threshold."""
    from scipy.stats import kstest
    g = _rng(44)
    ps = []
    for r in range(150):
        X, Y = g.standard_normal((20, 2)), g.standard_normal((20, 3))
        res = oracle.hsic_test(X, Y, 99, r, 0.5, 0.3)
        assert 1.0 / 100 <= res["p_value"] <= 1.0
        assert res["count_ge"] == int(np.sum(res["perm_stats"] >= res["threshold"]))
        ps.append(res["p_value"])
    assert kstest(ps, "uniform").pvalue > 1e-3
    X = g.standard_normal((40, 2))
    Y = np.column_stack([X[:, 0] ** 2, X[:, 1]]) + 0.2 * g.standard_normal((40, 2))
    assert oracle.hsic_test(X, Y, 199, 1, 0.5, 0.5)["p_value"] <= 0.01


def test_hsic_rejects_bad_input():
    X = np.zeros((3, 2))
    with pytest.raises(ValueError):
        oracle.hsic_test(X, X, 10, 1, 1.0, 1.0)
    with pytest.raises(ValueError):
        oracle.hsic_test(np.zeros((5, 2)), np.zeros((6, 2)), 10, 1, 1.0, 1.0)
    with pytest.raises(ValueError):
        oracle.hsic_test(np.zeros((5, 2)), np.zeros((5, 2)), 10, 1, 0.0, 1.0)
