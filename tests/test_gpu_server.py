"""Continuous-batching server: every served result against the FP64 oracle and equal to the
stand-alone call, a request mix shaped like the serving stream, admission and errors."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2406_06488_amd import _lib, api, inputs
from paper_2406_06488_amd._lib import EtestError
from tests.gpu_helpers import compare_run, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _pair(nx, ny, p, seed, prec="f32", shift=0.05):
    X, Y = inputs.gaussian_pair(nx, ny, p, seed, mean_shift=shift,
                                dtype=np.float64 if prec == "f64" else np.float32)
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd, Yd = torch.from_numpy(X).to(DEV, dt), torch.from_numpy(Y).to(DEV, dt)
    torch.cuda.synchronize()  # the server reads them on its own stream
    return Xd, Yd


SPECS = [(300, 200, 40, 1000, "ed", "bf16r"), (120, 150, 300, 2000, "mmd", "bf16r"),
         (50, 60, 20, 1000, "ed", "f32"), (700, 500, 64, 3000, "mmd", "f32"),
         (100, 100, 10, 500, "ed", "f64"), (1200, 900, 128, 1000, "ed", "bf16r"),
         (64, 65, 7, 300, "mmd", "f64"), (400, 410, 96, 10000, "ed", "bf16r"),
         # 40 000 splits: a serving step that admits it runs its split streams 32 per workgroup
         (80, 70, 12, 40000, "ed", "f32")]


def _alone(specs):
    out = []
    for t, (nx, ny, p, B, kind, prec) in enumerate(specs):
        X, Y = _pair(nx, ny, p, 300 + t, prec)
        r = api.run(X, Y, B, 400 + t, kind, prec, 1.0 / p)
        out.append((X, Y, r))
    return out


_ORACLE = {}


def _oracle_of(t, X, Y, B, kind, p):
    """The oracle's result for spec t (cached: both server configurations serve the same
    requests)."""
    if t not in _ORACLE:
        _ORACLE[t] = oracle.run_test(X.double().cpu().numpy(), Y.double().cpu().numpy(), B,
                                     400 + t, oracle.ED if kind == "ed" else oracle.MMD, 1.0 / p)
    return _ORACLE[t]


@pytest.mark.parametrize("resident,chunk", [(3, int(2e9)), (16, 0)])
def test_server_results_equal_standalone(resident, chunk):
    say("server", resident, chunk)
    ref = _alone(SPECS)
    with api.Server(memory_budget_bytes=4 << 30, max_resident=resident,
                    chunk_updates=chunk) as srv:
        ids, bufs = [], []
        for t, (nx, ny, p, B, kind, prec) in enumerate(SPECS):
            X, Y, _ = ref[t]
            ps = torch.zeros(B, dtype=torch.float64, device=DEV)
            torch.cuda.synchronize()
            bufs.append(ps)
            ids.append(srv.submit(X, Y, B, 400 + t, kind, prec, 1.0 / p, ps))
        for t, rid in enumerate(ids):
            r = srv.wait(rid)
            a = ref[t][2]
            for k in ("statistic", "threshold", "count_ge", "p_value", "n_refined"):
                assert r[k] == a[k], (t, k, r[k], a[k])
            assert torch.equal(bufs[t], a["perm_stats"]), t
            nx, ny, p, B, kind, prec = SPECS[t]
            o = _oracle_of(t, ref[t][0], ref[t][1], B, kind, p)
            r["perm_stats"] = bufs[t]
            compare_run(r, o, prec, "served %d" % t)
        st = srv.stats()
        assert st["resident"] == 0 and st["queued"] == 0 and st["bytes_held"] == 0
        assert st["completed"] == len(SPECS)


def test_server_admission_and_errors():
    X, Y = _pair(200, 200, 30, 1)
    fp = api.footprint(200, 200, 30, 1000, "ed", "bf16r")
    # budget below one request's footprint: rejected at submission
    with api.Server(memory_budget_bytes=fp // 2, max_resident=2) as srv:
        with pytest.raises(EtestError) as e:
            srv.submit(X, Y, 1000, 1)
        assert e.value.status == _lib.ENOMEM
    # budget for exactly one request at a time: all still complete, in order
    with api.Server(memory_budget_bytes=fp + fp // 2, max_resident=8) as srv:
        ids = [srv.submit(X, Y, 1000, s) for s in range(5)]
        res = [srv.wait(i) for i in ids]
        for s, r in enumerate(res):
            a = api.run(X, Y, 1000, s, "ed", "bf16r")
            assert r["count_ge"] == a["count_ge"] and r["statistic"] == a["statistic"]
        with pytest.raises(EtestError) as e:
            srv.poll(ids[0])  # already collected
        assert e.value.status == _lib.ENOTFOUND
    # bad input surfaces as the request's own status
    Xb = X.clone()
    Xb[0, 0] = float("nan")
    torch.cuda.synchronize()
    with api.Server(memory_budget_bytes=1 << 30, max_resident=2) as srv:
        good = srv.submit(X, Y, 500, 2)
        bad = srv.submit(Xb, Y, 500, 2)
        assert srv.wait(good)["B"] == 500
        with pytest.raises(EtestError) as e:
            srv.wait(bad)
        assert e.value.status == _lib.ENONFINITE


def test_server_queue_limit_and_poll():
    X, Y = _pair(1500, 1500, 200, 3)
    with api.Server(memory_budget_bytes=1 << 34, max_resident=1, max_queue=2,
                    chunk_updates=int(1e9)) as srv:
        ids = []
        busy = False
        for s in range(40):
            try:
                ids.append(srv.submit(X, Y, 10000, s))
            except EtestError as e:
                assert e.status == _lib.EBUSY
                busy = True
                break
        assert busy
        # poll until done
        deadline = time.time() + 60
        pending = set(ids)
        while pending and time.time() < deadline:
            for i in list(pending):
                if srv.poll(i) is not None:
                    pending.discard(i)
            time.sleep(0.001)
        assert not pending


def test_server_concurrent_submitters():
    specs = SPECS[:4]
    ref = _alone(specs)
    errors = []
    with api.Server(memory_budget_bytes=4 << 30, max_resident=4) as srv:
        def worker(t):
            try:
                nx, ny, p, B, kind, prec = specs[t]
                X, Y, a = ref[t]
                r = srv.wait(srv.submit(X, Y, B, 400 + t, kind, prec, 1.0 / p))
                if r["count_ge"] != a["count_ge"] or r["statistic"] != a["statistic"]:
                    errors.append(t)
            except Exception as e:  # noqa: BLE001
                errors.append(repr(e))
        th = [threading.Thread(target=worker, args=(t,)) for t in range(len(specs))]
        for x in th:
            x.start()
        for x in th:
            x.join()
    assert not errors, errors


def _serving_mix():
    """Requests shaped like the serving stream (BF16-refined, ED or Gaussian MMD with
    sigma^2 = p, mean shift on every coordinate, data seed 100000 + r, split seed
    200000 + r), at sizes the oracle finishes in seconds: p across the stream's range
    (10 .. 2000, both sides of the BF16 operand switch at 64), uneven nx, ny up to 3000,
    B in {1000, 10000}."""
    g = np.random.Generator(np.random.PCG64(7))
    shapes = [(2000, 1000, 10, 1000), (300, 250, 10, 10000), (1500, 900, 30, 1000),
              (400, 520, 30, 10000), (700, 800, 500, 1000), (128, 129, 500, 10000),
              (600, 300, 2000, 1000), (260, 340, 2000, 10000), (3000, 100, 64, 1000),
              (100, 2900, 63, 1000), (450, 460, 200, 10000), (1200, 1300, 1000, 1000)]
    out = []
    for r, (nx, ny, p, B) in enumerate(shapes):
        kind = "ed" if r % 2 == 0 else "mmd"
        delta = float(g.uniform(0.0, 0.1))
        out.append((r, nx, ny, p, B, kind, delta))
    return out


def test_serving_mix_against_oracle():
    """Every request of a serving-shaped mix, submitted at once so that their blocks are
    resident together and their resampling chunks interleave, against the FP64 oracle."""
    mix = _serving_mix()
    with api.Server(memory_budget_bytes=8 << 30, max_resident=16,
                    chunk_updates=int(3e10)) as srv:
        sub = []
        for r, nx, ny, p, B, kind, delta in mix:
            X, Y = _pair(nx, ny, p, 100000 + r, "bf16r", delta)
            ps = torch.zeros(B, dtype=torch.float64, device=DEV)
            gamma = 1.0 / p if kind == "mmd" else 0.0
            sub.append((srv.submit(X, Y, B, 200000 + r, kind, "bf16r", gamma, ps), X, Y, ps))
        for (rid, X, Y, ps), (r, nx, ny, p, B, kind, delta) in zip(sub, mix):
            g = srv.wait(rid)
            g["perm_stats"] = ps
            say("served", r, nx, ny, p, B, kind, "p =", g["p_value"], "refined", g["n_refined"])
            o = oracle.run_test(X.double().cpu().numpy(), Y.double().cpu().numpy(), B,
                                200000 + r, oracle.ED if kind == "ed" else oracle.MMD,
                                1.0 / p if kind == "mmd" else 1.0)
            near = compare_run(g, o, "bf16r", "serving mix %d" % r)
            if len(near):
                say("  near-ties", near[:20].tolist())
