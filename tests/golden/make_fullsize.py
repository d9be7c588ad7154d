"""Write the oracle's expected results for the benchmark workloads at their full sizes.

Calls only ``oracle/`` (the FP64 CPU oracle) and ``paper_2406_06488_amd.inputs`` (the
seeded data generator, which holds none of the method's arithmetic).  Nothing here
comes from the HIP path.  For every workload and statistic it runs the whole test the
way Alg. 1 states it -- the three blocks by direct differences (Alg. 3), the observed
statistic (eq. 1 / eq. 2), every one of the B resampled statistics, the identity-split
threshold, the exceedance count and the Section 3.1 p-value -- and stores:

  fullsize_<workload>_<kind>.json   scalars, input hashes, near-tie lists, oracle time
  fullsize_<workload>_<kind>.npy    the B resampled statistics (float64), when stored

Near-ties (the splits whose exceedance decision a correct implementation at a given
relative tolerance may take either way) are listed per tolerance: those are the only
splits whose decision may differ between the GPU and the oracle.  The per-split scale is
max(|statistic|, mean |null statistic|), as in the parity tests.

The batched workload (256 tests) stores, per test, the decision bits of all B splits,
every near-tie's statistic and a sample of statistics, in one .npz.

Usage:  python tests/golden/make_fullsize.py [plain_f32] [precision_bf16] [batched]
        (no argument: all three; each file is rewritten only for the workloads named)
"""
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_06488_amd import inputs  # noqa: E402

KIND = {"ed": oracle.ED, "mmd": oracle.MMD}
# relative statistic tolerances of the three forms (FP64, FP32, BF16-refined)
TOLS = (1e-12, 1e-5, 1e-3)


def sha256(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def near_ties(ps, thr, tol):
    floor = float(np.mean(np.abs(ps))) if len(ps) else 0.0
    return np.flatnonzero(np.abs(ps - thr) <= tol * max(abs(thr), floor))


def summary(wl, kind, o, X, Y, secs):
    ps = o["perm_stats"]
    return {
        "workload": wl.name, "kind": kind, "nx": wl.nx, "ny": wl.ny, "p": wl.p, "B": wl.B,
        "data_seed": wl.data_seed, "perm_seed": wl.perm_seed, "input_dtype": str(X.dtype),
        "gamma": wl.gamma() if kind == "mmd" else 0.0,
        "sha256_x": sha256(X), "sha256_y": sha256(Y),
        "statistic": o["statistic"], "threshold": o["threshold"], "count_ge": o["count_ge"],
        "p_value": o["p_value"], "null_mean_abs": float(np.mean(np.abs(ps))) if len(ps) else 0.0,
        "near_ties": {"%g" % t: near_ties(ps, o["threshold"], t).tolist() for t in TOLS},
        "oracle_seconds": secs, "oracle_threads": os.cpu_count(), "oracle_host": cpu_model(),
    }


def single(wl, kinds):
    X, Y = wl.data()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    for kind in kinds:
        t0 = time.time()
        o = oracle.run_test(X64, Y64, wl.B, wl.perm_seed, KIND[kind], wl.gamma())
        secs = time.time() - t0
        base = os.path.join(HERE, "fullsize_%s_%s" % (wl.name, kind))
        np.save(base + ".npy", o["perm_stats"])
        with open(base + ".json", "w") as f:
            json.dump(summary(wl, kind, o, X, Y, secs), f, indent=1)
        print("%s %s: statistic %.17g threshold %.17g count %d p %.17g  (%.0f s)"
              % (wl.name, kind, o["statistic"], o["threshold"], o["count_ge"], o["p_value"], secs),
              flush=True)


def batched():
    tests = inputs.batched_tests()
    keys = ["statistic", "threshold", "count_ge", "p_value", "null_mean_abs"]
    cols = {k: [] for k in keys}
    decisions, sample_idx, sample_val, near_idx, near_val, near_off = [], [], [], [], [], [0]
    shas = []
    t0 = time.time()
    for t, wl in enumerate(tests):
        X, Y = wl.data()
        o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), wl.B, wl.perm_seed)
        ps = o["perm_stats"]
        for k in keys[:4]:
            cols[k].append(o[k])
        cols["null_mean_abs"].append(float(np.mean(np.abs(ps))))
        decisions.append(np.packbits(ps >= o["threshold"]))
        g = np.random.Generator(np.random.PCG64(1000 + t))
        idx = np.unique(np.concatenate([np.arange(8), np.arange(wl.B - 8, wl.B),
                                        g.integers(0, wl.B, size=16)]))
        sample_idx.append(np.pad(idx, (0, 32 - len(idx)), constant_values=-1))
        sample_val.append(np.pad(ps[idx], (0, 32 - len(idx))))
        nt = near_ties(ps, o["threshold"], 1e-5)
        near_idx.append(nt)
        near_val.append(ps[nt])
        near_off.append(near_off[-1] + len(nt))
        shas.append(sha256(X) + sha256(Y))
        if t % 32 == 31:
            print("batched: %d tests, %.0f s" % (t + 1, time.time() - t0), flush=True)
    secs = time.time() - t0
    np.savez(os.path.join(HERE, "fullsize_batched_256x_B2000.npz"),
             **{k: np.array(v) for k, v in cols.items()},
             decisions=np.stack(decisions), sample_idx=np.stack(sample_idx),
             sample_val=np.stack(sample_val), near_idx=np.concatenate(near_idx).astype(np.int64),
             near_val=np.concatenate(near_val), near_off=np.array(near_off, dtype=np.int64),
             sha256=np.array(shas))
    with open(os.path.join(HERE, "fullsize_batched_256x_B2000.json"), "w") as f:
        json.dump({"workload": "batched 256 ED tests, FP32 inputs, B = 2000",
                   "near_tie_tolerance": 1e-5, "oracle_seconds": secs,
                   "oracle_threads": os.cpu_count(), "oracle_host": cpu_model(),
                   "near_ties_total": int(near_off[-1])}, f, indent=1)
    print("batched: done in %.0f s, %d near-ties at 1e-5" % (secs, near_off[-1]), flush=True)


def main(argv):
    which = argv or ["plain_f32", "precision_bf16", "batched"]
    if "plain_f32" in which:
        single(inputs.plain_f32(), ["ed"])
    if "precision_bf16" in which:
        single(inputs.precision_bf16(), ["ed", "mmd"])
    if "batched" in which:
        batched()


if __name__ == "__main__":
    main(sys.argv[1:])
