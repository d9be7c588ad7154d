"""HIP path vs the FP64 oracle, through the C ABI, on the same seeded inputs."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2406_06488_amd import api, inputs
from paper_2406_06488_amd._lib import EtestError
from tests.gpu_helpers import TOL, compare_run, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
KIND = {"ed": oracle.ED, "mmd": oracle.MMD}


def _dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dt)


def _data(nx, ny, p, seed, prec, shift=0.1):
    dt = np.float64 if prec == "f64" else np.float32
    return inputs.gaussian_pair(nx, ny, p, seed, mean_shift=shift, dtype=dt)


# --------------------------------------------------------------------------- split stream

@pytest.mark.parametrize("nx,ny,seed,b0,count", [(5, 4, 0, 0, 300), (100, 100, 1, 0, 1000),
                                                 (33, 64, 123456789, 2 ** 32 - 5, 40),
                                                 (1, 1, 3, 0, 10), (300, 170, 9, 50, 257),
                                                 (127, 129, 2 ** 63 + 7, 1000, 33)])
def test_membership_bit_exact(nx, ny, seed, b0, count):
    say("membership", nx, ny, seed, b0, count)
    words = api.membership(nx, ny, seed, b0, count)
    torch.cuda.synchronize()
    Z = api.unpack_words(words, nx + ny)
    for q in range(count):
        assert np.array_equal(Z[q], oracle.membership(nx, ny, seed, b0 + q)), q


# --------------------------------------------------------------------------- blocks

@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
@pytest.mark.parametrize("kind", ["ed", "mmd"])
def test_blocks_against_direct_differences(prec, kind):
    nx, ny, p = 300, 170, 37
    say("blocks", prec, kind, nx, ny, p)
    X, Y = _data(nx, ny, p, 5, prec)
    gamma = 1.0 / p
    dxx, dyy, dxy = api.blocks(_dev(X, prec), _dev(Y, prec), kind, prec, gamma)
    torch.cuda.synchronize()
    oxx, oyy, oxy = oracle.blocks(X, Y, KIND[kind], gamma)
    tol = {"f64": 1e-13, "f32": 3e-6, "bf16r": 2e-2}[prec]
    for g, o in ((dxx, oxx), (dyy, oyy), (dxy, oxy)):
        g = g.double().cpu().numpy()
        scale = np.abs(o).max()
        assert np.abs(g - o).max() <= tol * scale, (prec, kind, np.abs(g - o).max(), scale)
    diag = 0.0 if kind == "ed" else 1.0
    assert np.all(np.diag(dxx.double().cpu().numpy()) == diag)
    assert np.all(np.diag(dyy.double().cpu().numpy()) == diag)


@pytest.mark.parametrize("kind", ["ed", "mmd"])
def test_fp32_form_wide_dynamic_range(kind):
    """The FP32 form stages each centred value as an fp16 pair scaled by a power of two set by
    the test's largest |x|: columns spanning six decades and a large common offset must still
    give FP32-accurate blocks and statistics."""
    nx, ny, p = 170, 150, 40
    g = np.random.Generator(np.random.PCG64(77))
    scales = np.logspace(-3, 3, p)
    X = g.standard_normal((nx, p)) * scales + 50.0
    Y = g.standard_normal((ny, p)) * scales * 1.05 + 50.0
    X, Y = X.astype(np.float32), Y.astype(np.float32)
    gamma = 1.0 / float(np.sum(scales ** 2))
    say("wide range", kind, nx, ny, p)
    dxx, dyy, dxy = api.blocks(_dev(X, "f32"), _dev(Y, "f32"), kind, "f32", gamma)
    torch.cuda.synchronize()
    oxx, oyy, oxy = oracle.blocks(X.astype(np.float64), Y.astype(np.float64), KIND[kind], gamma)
    for gm, o in ((dxx, oxx), (dyy, oyy), (dxy, oxy)):
        gm = gm.double().cpu().numpy()
        assert np.abs(gm - o).max() <= 3e-6 * np.abs(o).max(), (kind, np.abs(gm - o).max())
    r = api.run(_dev(X, "f32"), _dev(Y, "f32"), 300, 4, kind, "f32", gamma)
    torch.cuda.synchronize()
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), 300, 4, KIND[kind], gamma)
    compare_run(r, o, "f32", "wide range " + kind)


# --------------------------------------------------------------------------- whole test

CASES = [
    # nx, ny, p, B, data seed, perm seed, shift
    (100, 100, 10, 1000, 0, 1, 0.0),     # the small FP64 null workload
    (300, 170, 37, 700, 3, 5, 0.15),     # several tiles, ragged tails, B_pad > one chunk
    (129, 127, 64, 255, 4, 6, 0.3),      # one row past a tile / one short
    (1, 5, 3, 40, 5, 7, 0.5),
    (7, 1, 2, 40, 6, 8, 0.5),
    (1, 1, 4, 20, 7, 9, 1.0),
    (40, 33, 1, 300, 8, 10, 0.2),        # p = 1
    (300, 170, 1030, 400, 9, 11, 0.1),   # p above 1024: 33 K slices of 32 in the FP32 Gram
    (260, 300, 20, 1000, 12, 13, 0.05),  # BF16 form below 64 coordinates: fp16-pair operands
    (400, 380, 63, 600, 14, 15, 0.05),   # ... the last p before BF16 operands
    (400, 380, 64, 600, 14, 15, 0.05),   # ... the first p with BF16 operands
]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
@pytest.mark.parametrize("kind", ["ed", "mmd"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_full_test_matches_oracle(case, kind, prec):
    nx, ny, p, B, ds, ps_, shift = CASES[case]
    say("full", case, kind, prec, nx, ny, p, B)
    X, Y = _data(nx, ny, p, ds, prec, shift)
    gamma = 1.0 / p
    g = api.run(_dev(X, prec), _dev(Y, prec), B, ps_, kind, prec, gamma)
    torch.cuda.synchronize()
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, ps_, KIND[kind], gamma)
    near = compare_run(g, o, prec, "case %d %s %s" % (case, kind, prec))
    if len(near):
        say("near-ties within tolerance:", near.tolist())


# --------------------------------------------------------------------------- degenerate data

def _edge_data(name, prec):
    """Data on which the method's degenerate cases arise (seeded, Gaussian rows)."""
    g = np.random.Generator(np.random.PCG64(500 + EDGE.index(name)))
    if name == "same_sample":
        # X = Y: the observed ED and MMD are exactly 0, every split's statistic is >= 0, so
        # every split counts (p = 1 in exact arithmetic); splits that pair each row with its
        # copy tie with the threshold
        X = g.standard_normal((150, 40))
        Y = X.copy()
    elif name == "duplicated_rows":
        # rows repeated within and across the samples: zero distances off the diagonal
        base = g.standard_normal((90, 40))
        X = base[g.integers(0, 90, size=170)]
        Y = base[g.integers(0, 90, size=130)] + 0.1
    else:
        # near-duplicate pairs (y_j = x_j + 1e-4 noise, 80 coordinates, so the BF16 form's
        # Gram reads BF16 operands) on a common offset of 1000: the Gram-based d^2 of those
        # pairs cancels to noise, and only the direct difference of the input rows recovers it
        X = g.standard_normal((160, 80))
        Y = X[:140] + 1e-4 * g.standard_normal((140, 80))
        X, Y = X + 1000.0, Y + 1000.0
    dt = np.float64 if prec == "f64" else np.float32
    return X.astype(dt), Y.astype(dt)


EDGE = ["same_sample", "duplicated_rows", "near_duplicates_offset"]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
@pytest.mark.parametrize("kind", ["ed", "mmd"])
@pytest.mark.parametrize("name", EDGE)
def test_degenerate_data_matches_oracle(name, kind, prec):
    X, Y = _edge_data(name, prec)
    p = X.shape[1]
    gamma = 1.0 / p
    B, seed = 800, 61
    say("edge", name, kind, prec, X.shape, Y.shape)
    g = api.run(_dev(X, prec), _dev(Y, prec), B, seed, kind, prec, gamma)
    torch.cuda.synchronize()
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, seed, KIND[kind], gamma)
    near = compare_run(g, o, prec, "edge %s %s %s" % (name, kind, prec))
    if prec != "f64":
        # pairs at (near) zero distance: the form recomputes them as direct FP32 differences
        assert g["n_refined"] > 0, (name, kind, prec)
    if name == "same_sample":
        assert o["statistic"] == 0.0
        assert np.all(o["perm_stats"] >= o["threshold"])
    say("  refined %d, near-ties %d: %s" % (g["n_refined"], len(near), near[:20].tolist()))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
def test_many_split_chunks(prec):
    """B spans several groups of 256-split chunks per workgroup; results do not depend on
    how chunks are grouped."""
    import os
    nx, ny, p, B = 500, 450, 80, 2000
    say("chunks", prec, nx, ny, p, B)
    X, Y = _data(nx, ny, p, 21, prec, 0.05)
    Xd, Yd = _dev(X, prec), _dev(Y, prec)
    outs = []
    for cc in ("1", "3", "8"):
        os.environ["ETEST_CC"] = cc
        try:
            outs.append(api.run(Xd, Yd, B, 22, "ed", prec))
        finally:
            del os.environ["ETEST_CC"]
    torch.cuda.synchronize()
    for r in outs[1:]:
        assert torch.equal(r["perm_stats"], outs[0]["perm_stats"])
        assert r["count_ge"] == outs[0]["count_ge"]
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, 22)
    compare_run(outs[0], o, prec, "chunks " + prec)


def test_zero_and_one_permutations():
    X, Y = _data(20, 30, 5, 1, "f32")
    g = api.run(_dev(X, "f32"), _dev(Y, "f32"), 0, 1, "ed", "f32")
    assert g["p_value"] == 1.0 and g["count_ge"] == 0 and g["B"] == 0
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), 1, 1)
    g = api.run(_dev(X, "f32"), _dev(Y, "f32"), 1, 1, "ed", "f32")
    compare_run(g, o, "f32")


def test_nonfinite_input_rejected_and_outputs_untouched():
    X, Y = _data(50, 40, 6, 2, "f32")
    X[3, 2] = np.nan
    Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
    ps = torch.full((100,), 7.0, dtype=torch.float64, device=DEV)
    req = api.make_request(Xd, Yd, 100, 1, "ed", "f32", 0.0, ps)
    import ctypes
    from paper_2406_06488_amd import _lib
    r = _lib.Result()
    st = _lib.load().etest_run(ctypes.byref(req), None, ctypes.byref(r))
    assert st == _lib.ENONFINITE
    assert torch.all(ps == 7.0)
    Y[0, 0] = np.inf
    with pytest.raises(EtestError):
        api.ed_test(X, Y, 10, 1, "f32")


def test_without_per_split_output():
    """perm_stats = NULL: nothing is written for the splits, and the summary is unchanged."""
    X, Y = _data(260, 240, 30, 15, "f32")
    Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
    with_out = api.run(Xd, Yd, 3000, 5, "ed", "bf16r")
    without = api.run(Xd, Yd, 3000, 5, "ed", "bf16r", with_perm_stats=False)
    for k in ("statistic", "threshold", "count_ge", "p_value"):
        assert with_out[k] == without[k]
    h = api.ed_test(X, Y, 3000, 5, "bf16r", with_perm_stats=False)
    assert h["count_ge"] == with_out["count_ge"] and h["perm_stats"] is None


def test_repeat_runs_bit_identical():
    X, Y = _data(300, 200, 50, 9, "f32")
    Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
    a = api.run(Xd, Yd, 1000, 3, "ed", "bf16r")
    b = api.run(Xd, Yd, 1000, 3, "ed", "bf16r")
    assert torch.equal(a["perm_stats"], b["perm_stats"])
    assert a["statistic"] == b["statistic"] and a["threshold"] == b["threshold"]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
def test_graph_replay_with_new_inputs(prec):
    """A batch of the same shape replays its captured graph with this call's pointers, seed
    and gamma: new data, seeds and kinds on the same shape must still match the oracle, and
    a replay of the first call's inputs must reproduce it bit for bit."""
    nx, ny, p, B = 210, 150, 33, 600
    say("graph replay", prec)
    runs = []
    for rep, (ds, seed, kind) in enumerate([(31, 5, "ed"), (32, 6, "mmd"), (33, 7, "ed"),
                                            (31, 5, "ed")]):
        X, Y = _data(nx, ny, p, ds, prec, 0.2)
        Xd, Yd = _dev(X, prec), _dev(Y, prec)
        ps = torch.empty(B, dtype=torch.float64, device=DEV)
        req = api.make_request(Xd, Yd, B, seed, kind, prec, 1.0 / p, ps)
        g = api.batch([req])[0]
        torch.cuda.synchronize()
        g["perm_stats"] = ps
        runs.append(g)
        if rep in (1, 2):
            o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, seed, KIND[kind],
                                1.0 / p)
            compare_run(g, o, prec, "replay %d %s" % (rep, prec))
    assert torch.equal(runs[0]["perm_stats"], runs[3]["perm_stats"])
    assert runs[0]["statistic"] == runs[3]["statistic"]
    assert runs[0]["count_ge"] == runs[3]["count_ge"]


def test_batch_equals_alone():
    specs = [(120, 90, 20, 300, "ed", "f32"), (60, 200, 100, 500, "mmd", "bf16r"),
             (300, 170, 37, 257, "ed", "f64"), (5, 4, 3, 100, "mmd", "f32"),
             (700, 650, 64, 1000, "ed", "bf16r"), (300, 170, 1030, 300, "ed", "f32")]
    reqs, keep, alone = [], [], []
    for t, (nx, ny, p, B, kind, prec) in enumerate(specs):
        X, Y = _data(nx, ny, p, 100 + t, prec)
        Xd, Yd = _dev(X, prec), _dev(Y, prec)
        ps = torch.zeros(B, dtype=torch.float64, device=DEV)
        keep += [Xd, Yd, ps]
        reqs.append(api.make_request(Xd, Yd, B, 200 + t, kind, prec, 1.0 / p, ps))
        alone.append(api.run(Xd, Yd, B, 200 + t, kind, prec, 1.0 / p))
    for rep in range(2):  # second call replays the captured graph
        outs = api.batch(reqs)
        torch.cuda.synchronize()
        for t in range(len(specs)):
            for k in ("statistic", "threshold", "count_ge", "p_value"):
                assert outs[t][k] == alone[t][k], (rep, t, k)
            assert torch.equal(keep[3 * t + 2], alone[t]["perm_stats"]), (rep, t)


def test_wide_split_stream_equals_narrow():
    """A batch whose split stream outgrows the chip runs it 32 splits per workgroup instead of
    16: the split words, and so every result, are those of the same test run alone (narrow),
    and the large test that tips the batch over matches the oracle."""
    big = (60, 50, 8, 40000, 301)   # nx, ny, p, B, seed: 40 000 splits, 2 501 workgroups at 16
    small = (100, 80, 12, 999, 302)
    runs = []
    for nx, ny, p, B, seed in (big, small):
        X, Y = _data(nx, ny, p, seed, "f32")
        Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
        runs.append((X, Y, Xd, Yd, B, seed, torch.zeros(B, dtype=torch.float64, device=DEV)))
    reqs = [api.make_request(Xd, Yd, B, seed + 100, "ed", "f32", 0.0, ps)
            for _, _, Xd, Yd, B, seed, ps in runs]
    say("wide split stream: batch of B = %d and B = %d" % (big[3], small[3]))
    outs = api.batch(reqs)
    torch.cuda.synchronize()
    X, Y, Xd, Yd, B, seed, ps = runs[1]
    alone = api.run(Xd, Yd, B, seed + 100, "ed", "f32", 0.0)
    for k in ("statistic", "threshold", "count_ge", "p_value"):
        assert outs[1][k] == alone[k], k
    assert torch.equal(ps, alone["perm_stats"])
    X, Y, Xd, Yd, B, seed, ps = runs[0]
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, seed + 100)
    g = dict(outs[0])
    g["perm_stats"] = ps
    compare_run(g, o, "f32", "wide split stream")


@pytest.mark.parametrize("prec,p", [("f32", 70), ("bf16r", 70), ("f32", 1030)])
def test_shared_block_stage_equals_alone(prec, p):
    """An ED and an MMD test on the same X, Y in one batch share staging and Gram (the ED
    test's epilogue writes the kernel blocks too), and with the same seed and B also the
    split stream; each result must equal its run alone, bit for bit, also when the MMD
    test comes first."""
    X, Y = _data(260, 190, p, 41, prec, 0.2)
    X2, Y2 = _data(260, 190, p, 42, prec, 0.2)
    Xd, Yd, X2d, Y2d = _dev(X, prec), _dev(Y, prec), _dev(X2, prec), _dev(Y2, prec)
    specs = [("mmd", Xd, Yd, 11), ("ed", Xd, Yd, 12), ("mmd", X2d, Y2d, 13), ("ed", X2d, Y2d, 13)]
    B, gamma = 700, 1.0 / p
    reqs, outs_ps, alone = [], [], []
    for kind, A, Bm, seed in specs:
        ps = torch.zeros(B, dtype=torch.float64, device=DEV)
        outs_ps.append(ps)
        reqs.append(api.make_request(A, Bm, B, seed, kind, prec, gamma, ps))
        alone.append(api.run(A, Bm, B, seed, kind, prec, gamma))
    for rep in range(2):
        outs = api.batch(reqs)
        torch.cuda.synchronize()
        for t in range(len(specs)):
            for k in ("statistic", "threshold", "count_ge", "p_value", "n_refined"):
                assert outs[t][k] == alone[t][k], (rep, t, k)
            assert torch.equal(outs_ps[t], alone[t]["perm_stats"]), (rep, t)


def test_enumeration_through_supplied_splits():
    """nx = ny = 5: all 252 splits evaluated on the GPU equal the oracle's table; the
    identity equals the threshold and its complement ties with it."""
    nx = ny = 5
    X, Y = _data(nx, ny, 4, 31, "f64", 0.6)
    splits = np.array(list(brute.all_splits(nx, ny)), dtype=np.uint8)
    words = torch.from_numpy(api.pack_splits(splits)).to(DEV)
    for kind in ("ed", "mmd"):
        g = api.perm_stats_from_membership(_dev(X, "f64"), _dev(Y, "f64"), words, kind, "f64", 0.25)
        torch.cuda.synchronize()
        gs = g["perm_stats"].cpu().numpy()
        XX, YY, XY = oracle.blocks(X, Y, KIND[kind], 0.25)
        want = np.array([oracle.perm_stat(XX, YY, XY, z, KIND[kind]) for z in splits])
        assert np.all(np.abs(gs - want) <= 1e-12 * np.abs(want))
        ident = np.flatnonzero((splits[:, :nx] == 1).all(axis=1))[0]
        assert abs(gs[ident] - g["threshold"]) <= 1e-12 * abs(g["threshold"])


def test_supplied_split_with_wrong_size_rejected():
    X, Y = _data(6, 5, 3, 1, "f32")
    Z = np.zeros((1, 11), dtype=np.uint8)
    Z[0, :5] = 1  # five members instead of six
    words = torch.from_numpy(api.pack_splits(Z)).to(DEV)
    with pytest.raises(EtestError):
        api.perm_stats_from_membership(_dev(X, "f32"), _dev(Y, "f32"), words, "ed", "f32")


def test_host_buffer_calls_match_device_calls():
    X, Y = _data(210, 190, 30, 12, "f32")
    h = api.ed_test(X, Y, 500, 4, "f32")
    d = api.run(_dev(X, "f32"), _dev(Y, "f32"), 500, 4, "ed", "f32")
    assert h["statistic"] == d["statistic"] and h["count_ge"] == d["count_ge"]
    assert np.array_equal(h["perm_stats"], d["perm_stats"].cpu().numpy())
    h = api.mmd_test(X, Y, 0.05, 500, 4, "bf16r")
    d = api.run(_dev(X, "f32"), _dev(Y, "f32"), 500, 4, "mmd", "bf16r", 0.05)
    assert h["statistic"] == d["statistic"] and h["count_ge"] == d["count_ge"]
    X64, Y64 = _data(50, 60, 5, 13, "f64")
    h = api.ed_test(X64, Y64, 300, 4, "f64")
    o = oracle.run_test(X64, Y64, 300, 4)
    compare_run(h, o, "f64")


def test_async_call_matches_sync():
    X, Y = _data(150, 140, 20, 14, "f32")
    Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
    ps = torch.zeros(400, dtype=torch.float64, device=DEV)
    buf = api.run_async(Xd, Yd, 400, 9, "mmd", "f32", 0.05, ps)
    torch.cuda.synchronize()
    a = api.result_from_device(buf)
    s = api.run(Xd, Yd, 400, 9, "mmd", "f32", 0.05)
    assert a["statistic"] == s["statistic"] and a["count_ge"] == s["count_ge"]
    assert torch.equal(ps, s["perm_stats"])


def test_async_calls_back_to_back_reuse_the_stream_workspace():
    """Asynchronous calls keep one workspace per (device, stream) and reuse it in stream
    order.  Back-to-back calls with no synchronisation between them -- growing (the
    workspace is replaced while earlier work is still queued), shrinking, on a second
    stream, both statistics and all three forms -- must each equal the synchronous call
    bit for bit."""
    cases = [(150, 140, 20, "f32", "ed"), (700, 650, 90, "f32", "ed"),
             (130, 170, 37, "bf16r", "mmd"), (900, 820, 64, "bf16r", "ed"),
             (60, 75, 12, "f64", "ed"), (150, 140, 20, "f32", "ed")]
    B = 600
    data, outs = [], []
    side = torch.cuda.Stream()
    for k, (nx, ny, p, prec, kind) in enumerate(cases):
        X, Y = _data(nx, ny, p, 80 + k, prec)
        Xd, Yd = _dev(X, prec), _dev(Y, prec)
        ps = torch.zeros(B, dtype=torch.float64, device=DEV)
        gamma = 1.0 / p if kind == "mmd" else 0.0
        data.append((Xd, Yd, prec, kind, gamma, ps))
    say("async back to back", len(cases), "tests")
    torch.cuda.synchronize()
    for k, (Xd, Yd, prec, kind, gamma, ps) in enumerate(data):
        if k == 3:  # one on a second stream, between the others
            with torch.cuda.stream(side):
                outs.append(api.run_async(Xd, Yd, B, 30 + k, kind, prec, gamma, ps))
        else:
            outs.append(api.run_async(Xd, Yd, B, 30 + k, kind, prec, gamma, ps))
    torch.cuda.synchronize()
    for k, (Xd, Yd, prec, kind, gamma, ps) in enumerate(data):
        a = api.result_from_device(outs[k])
        s = api.run(Xd, Yd, B, 30 + k, kind, prec, gamma)
        assert a["statistic"] == s["statistic"] and a["count_ge"] == s["count_ge"], k
        assert a["p_value"] == s["p_value"] and a["threshold"] == s["threshold"], k
        assert torch.equal(ps, s["perm_stats"]), k


def test_async_calls_from_two_threads_on_one_stream():
    """Two host threads enqueue asynchronous tests on the same (default) stream at once:
    each pass holds the stream's workspace until all its launches are queued, so the
    passes cannot interleave over it; every result must equal the synchronous call's."""
    import threading
    B = 400
    X, Y = _data(400, 380, 40, 95, "f32")
    Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
    torch.cuda.synchronize()
    outs = {}

    def worker(tag):
        for k in range(4):
            seed = 100 * tag + k
            outs[seed] = api.run_async(Xd, Yd, B, seed, "ed", "f32")

    say("two threads, one stream")
    th = [threading.Thread(target=worker, args=(t,)) for t in (1, 2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    for seed, buf in sorted(outs.items()):
        a = api.result_from_device(buf)
        s = api.run(Xd, Yd, B, seed, "ed", "f32", with_perm_stats=False)
        assert a["statistic"] == s["statistic"] and a["count_ge"] == s["count_ge"], seed
        assert a["threshold"] == s["threshold"], seed


def test_batch_async_equals_batch():
    """etest_batch_async runs the batched pass eagerly on the stream's workspace and writes
    each result from the test's last kernel; called twice back to back (no synchronisation
    between) it must equal etest_batch bit for bit, an ED / MMD pair sharing its Gram and a
    lone test included."""
    B = 500
    specs = [(300, 170, 37, "f32", "ed", 91), (300, 170, 37, "f32", "mmd", 91),
             (520, 480, 70, "bf16r", "ed", 92), (90, 110, 12, "f32", "ed", 93)]
    data = {}
    reqs, stats = [], []
    for nx, ny, p, prec, kind, seed in specs:
        if seed not in data:
            X, Y = _data(nx, ny, p, seed, prec)
            data[seed] = (_dev(X, prec), _dev(Y, prec))
        Xd, Yd = data[seed]
        ps = torch.zeros(B, dtype=torch.float64, device=DEV)
        stats.append(ps)
        reqs.append(api.make_request(Xd, Yd, B, seed + 7, kind, prec,
                                     1.0 / p if kind == "mmd" else 0.0, ps))
    say("batch_async", len(reqs), "tests")
    first = api.batch_async(reqs)
    second = api.batch_async(reqs)
    torch.cuda.synchronize()
    a1, a2 = api.results_from_device(first), api.results_from_device(second)
    got = [t.clone() for t in stats]
    ref = api.batch(reqs)
    torch.cuda.synchronize()
    assert a1 == ref and a2 == ref
    for g, t in zip(got, stats):
        assert torch.equal(g, t)


# --------------------------------------------------------------------------- tuned shapes

@pytest.mark.parametrize("prec,kc,cc", [("f32", 1, 1), ("f32", 5, 2), ("f32", 64, 2),
                                        ("bf16r", 1, 2), ("bf16r", 3, 1), ("bf16r", 64, 2),
                                        ("f64", 1, 8), ("f64", 7, 3)])
def test_tuned_work_shapes_match_oracle(prec, kc, cc):
    """Resampling work shapes installed through the tuning rules (row units of kc column
    tiles, cc chunks of 256 splits per workgroup) regroup the FP32 partial sums; every
    shape must still meet the form's tolerance against the oracle."""
    from paper_2406_06488_amd import autotune
    nx, ny, p, B = 700, 650, 72, 1500
    X, Y = _data(nx, ny, p, 71, prec, 0.05)
    say("tuned shape", prec, kc, cc)
    autotune.install([{"prec": prec, "n_lo": nx + ny, "n_hi": nx + ny + 1, "kc": kc, "cc": cc}])
    try:
        g = api.run(_dev(X, prec), _dev(Y, prec), B, 72, "ed", prec)
        torch.cuda.synchronize()
    finally:
        autotune.clear()
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, 72)
    compare_run(g, o, prec, "tuned %s kc=%d cc=%d" % (prec, kc, cc))


def test_autotuner_picks_a_shape_and_results_hold():
    """The tuner times every candidate shape on one bucket and installs the fastest; a test
    run under the installed rule matches the oracle."""
    from paper_2406_06488_amd import autotune
    nx, ny, p, B = 600, 500, 40, 1024
    X, Y = _data(nx, ny, p, 81, "f32", 0.05)
    Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
    try:
        rules = autotune.tune([{"prec": "f32", "n_lo": nx + ny, "n_hi": nx + ny + 1, "X": Xd,
                                "Y": Yd, "B": B}], reps=1, log=say)
        assert len(rules) == 1 and (rules[0]["kc"], rules[0]["cc"]) in autotune.MFMA_CANDIDATES
        g = api.run(Xd, Yd, B, 82, "ed", "f32")
        torch.cuda.synchronize()
    finally:
        autotune.clear()
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, 82)
    compare_run(g, o, "f32", "autotuned")


def test_batch_tuner_picks_shapes_and_results_hold():
    """The batch tuner times candidate shapes on the whole batch, per size bucket, and
    installs the fastest; under those rules the batch equals its tests run alone, and a test
    of it matches the oracle."""
    from paper_2406_06488_amd import autotune
    specs = [(300, 250, 20, 600), (90, 60, 100, 600), (700, 650, 40, 1000), (40, 50, 7, 300)]
    data, reqs, keep = [], [], []
    for t, (nx, ny, p, B) in enumerate(specs):
        X, Y = _data(nx, ny, p, 140 + t, "f32")
        Xd, Yd = _dev(X, "f32"), _dev(Y, "f32")
        data.append((X, Y))
        keep += [Xd, Yd]
        reqs.append(api.make_request(Xd, Yd, B, 160 + t, "ed", "f32"))
    reqs = (api.Request * len(reqs))(*reqs)
    ranges = [(0, 1024), (1024, 1 << 31)]
    try:
        rules = autotune.tune_batch(lambda: api.batch(reqs), ranges, "f32", reps=1, log=say)
        assert [(r["n_lo"], r["n_hi"]) for r in rules] == ranges
        assert all((r["kc"], r["cc"]) in autotune.MFMA_CANDIDATES for r in rules)
        outs = api.batch(reqs)
        alone = [api.run(keep[2 * t], keep[2 * t + 1], B, 160 + t, "ed", "f32")
                 for t, (_, _, _, B) in enumerate(specs)]
        torch.cuda.synchronize()
    finally:
        autotune.clear()
    for t in range(len(specs)):
        for k in ("statistic", "threshold", "count_ge", "p_value"):
            assert outs[t][k] == alone[t][k], (t, k)
    X, Y = data[2]
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), specs[2][3], 162)
    compare_run(alone[2], o, "f32", "batch-tuned")


# --------------------------------------------------------------------------- Gram shapes

def _with_gram_shape(shape, prec, n, fn):
    from paper_2406_06488_amd import autotune
    autotune.install([{"prec": prec, "n_lo": n, "n_hi": n + 1, "gram_shape": shape}])
    try:
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        autotune.clear()


@pytest.mark.parametrize("prec", ["f32", "bf16r"])
@pytest.mark.parametrize("kind", ["ed", "mmd"])
@pytest.mark.parametrize("nx,ny,p", [(300, 170, 37), (640, 700, 72), (1000, 900, 130),
                                     (129, 1, 80), (1, 1, 3), (260, 300, 1030)])
def test_gram_super_tiles_equal_block_tiles(nx, ny, p, kind, prec):
    """The 256 x 256 super-tile Gram adds each entry's products in the same order as the
    128-tile Gram and shares its epilogue: blocks, block sums and every statistic must be
    identical bit for bit (odd tile grids leave super tiles past the edge; the diagonal
    super tiles hold a lower tile that is not stored), and both meet the oracle."""
    X, Y = _data(nx, ny, p, 90 + p, prec, 0.1)
    Xd, Yd = _dev(X, prec), _dev(Y, prec)
    gamma = 1.0 / p
    say("gram shapes", nx, ny, p, kind, prec)
    blocks = [_with_gram_shape(s_, prec, nx + ny,
                               lambda: api.blocks(Xd, Yd, kind, prec, gamma)) for s_ in (0, 1)]
    for a, b in zip(*blocks):
        assert torch.equal(a, b)
    runs = [_with_gram_shape(s_, prec, nx + ny,
                             lambda: api.run(Xd, Yd, 600, 91, kind, prec, gamma)) for s_ in (0, 1)]
    for k in ("statistic", "threshold", "count_ge", "p_value", "n_refined"):
        assert runs[0][k] == runs[1][k], k
    assert torch.equal(runs[0]["perm_stats"], runs[1]["perm_stats"])
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), 600, 91, KIND[kind], gamma)
    compare_run(runs[1], o, prec, "super tiles %s %s" % (kind, prec))


@pytest.mark.parametrize("prec", ["f32", "bf16r"])
def test_gram_super_tiles_shared_block_stage(prec):
    """ED and MMD on the same data in one batch (the ED test's Gram writes both tests'
    blocks) with super tiles: each result equal to the block-tile run, bit for bit."""
    nx, ny, p, B = 700, 650, 96, 800
    X, Y = _data(nx, ny, p, 93, prec, 0.1)
    Xd, Yd = _dev(X, prec), _dev(Y, prec)

    def pair():
        outs = [torch.zeros(B, dtype=torch.float64, device=DEV) for _ in range(2)]
        reqs = [api.make_request(Xd, Yd, B, 94, k, prec, 1.0 / p, o)
                for k, o in zip(("ed", "mmd"), outs)]
        res = api.batch(reqs)
        return res, outs
    (r0, o0), (r1, o1) = [_with_gram_shape(s_, prec, nx + ny, pair) for s_ in (0, 1)]
    for t in range(2):
        for k in ("statistic", "threshold", "count_ge", "p_value", "n_refined"):
            assert r0[t][k] == r1[t][k], (t, k)
        assert torch.equal(o0[t], o1[t])


def test_gram_shape_autotuner():
    """The tuner times both Gram shapes on one bucket and installs the faster; a run under
    the installed rule matches the oracle."""
    from paper_2406_06488_amd import autotune
    nx, ny, p = 1500, 1400, 256
    X, Y = _data(nx, ny, p, 95, "bf16r", 0.05)
    Xd, Yd = _dev(X, "bf16r"), _dev(Y, "bf16r")
    try:
        rules = autotune.tune_gram([{"prec": "bf16r", "n_lo": nx + ny, "n_hi": nx + ny + 1,
                                     "X": Xd, "Y": Yd}], reps=2, log=say)
        assert len(rules) == 1 and rules[0]["gram_shape"] in (0, 1)
        g = api.run(Xd, Yd, 500, 96, "ed", "bf16r")
        torch.cuda.synchronize()
    finally:
        autotune.clear()
    o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), 500, 96)
    compare_run(g, o, "bf16r", "gram-shape tuned")
