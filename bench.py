#!/usr/bin/env python3
"""Benchmark of the MI355X permutation two-sample test.

One step = one whole test on device-resident synthetic inputs: staging, the
three blocks (Gram on MFMA + epilogue), block sums and observed statistic,
centring, the B-split stream, all B resampled statistics, threshold, count and
p-value (every stage of the hot path).  Default workload: energy distance,
FP32 form, X 2000 x 1000 ~ N(0, I), Y 2000 x 1000 with mean 0.05 on the first 50
coordinates, B = 10^4 (metric: resampled statistics per second).

Prints ONE JSON line on stdout.  Per-stage device times come from HIP events
recorded by the library on the launch stream during the timed steps.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "permuted statistics/sec and Gram TFLOP/s vs plain FP32; serving p50/p99 latency"
PEAK = {"hbm_GBs": 8000.0, "bf16_TF": 2500.0, "fp32_TF": 157.3, "fp64_TF": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gram_flops(nx, ny, p):
    """Distinct Gram products: upper-triangular XX / YY (with diagonal) plus XY, 2p flops each."""
    return 2.0 * p * (nx * (nx + 1) / 2 + ny * (ny + 1) / 2 + nx * ny)


def packed_pairs(nx, ny):
    """Distinct off-diagonal block entries that determine every statistic."""
    return nx * (nx - 1) / 2 + ny * (ny - 1) / 2 + nx * ny


def run_single(args, wl, kinds):
    import numpy as np
    import torch

    from paper_2406_06488_amd import api

    X, Y = wl.data()
    dt = torch.float64 if wl.prec == "f64" else torch.float32
    Xd = torch.from_numpy(X).to("cuda:0", dt)
    Yd = torch.from_numpy(Y).to("cuda:0", dt)
    torch.cuda.synchronize()

    def step():
        out = []
        for k in kinds:
            out.append(api.run(Xd, Yd, wl.B, wl.perm_seed, k, wl.prec, wl.gamma()))
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    api.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = api.profile_read()
    api.profile_enable(False)
    return (t1 - t0), prof, res, X, Y


def cpu_baseline(wl, kinds, budget_s):
    """The FP64 oracle on the host: blocks once, then resampled splits for ~budget_s seconds;
    the full-test rate is projected from the measured block and per-split times."""
    import numpy as np

    import oracle

    X, Y = wl.data()
    X = X.astype(np.float64)
    Y = Y.astype(np.float64)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    total_blocks = 0.0
    total_split = 0.0
    m_done = 0
    for k in kinds:
        kind = oracle.ED if k == "ed" else oracle.MMD
        t0 = time.perf_counter()
        XX, YY, XY = oracle.blocks(X, Y, kind, wl.gamma(), threads)
        tb = time.perf_counter() - t0
        m = max(threads, 8)
        t0 = time.perf_counter()
        oracle.perm_stats_listed(XX, YY, XY, wl.perm_seed, list(range(m)), kind, threads)
        tp = (time.perf_counter() - t0) / m
        # spend what is left of the budget on more splits for a steadier per-split time
        more = int(max(0.0, budget_s / len(kinds) - tb - tp * m) / max(tp, 1e-9))
        more = min(more, wl.B)
        if more > m:
            t0 = time.perf_counter()
            oracle.perm_stats_listed(XX, YY, XY, wl.perm_seed, list(range(more)), kind, threads)
            tp = (time.perf_counter() - t0) / more
            m = more
        total_blocks += tb
        total_split += tp
        m_done += m
        del XX, YY, XY
    full = total_blocks + total_split * wl.B
    return {"value": len(kinds) * wl.B / full, "unit": "permuted statistics/s", "cores": threads,
            "kind": "oracle",
            "sample": "%s: blocks once + %d of %d splits per statistic (%s), projected to the "
                      "full test; blocks %.2f s, %.4f s per split" %
                      (wl.name, m_done // len(kinds), wl.B, "+".join(kinds), total_blocks,
                       total_split)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_f32",
                    choices=["plain_f32", "small_f64", "precision_bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    from paper_2406_06488_amd import inputs

    if args.workload == "plain_f32":
        wl, kinds = inputs.plain_f32(), ["ed"]
    elif args.workload == "small_f64":
        wl, kinds = inputs.small_null_f64(), ["ed"]
    else:
        wl = inputs.precision_bf16()
        kinds = wl.kinds
    log("workload", wl.name, "kinds", kinds, "steps", args.steps, "warmup", args.warmup)
    elapsed, prof, res, X, Y = run_single(args, wl, kinds)
    ms_step = 1e3 * elapsed / args.steps
    value = len(kinds) * wl.B * args.steps / elapsed
    stage_ms = {k: (v[0] / max(v[1], 1)) for k, v in prof.items()}  # per launch of the stage
    log("stage ms per test:", json.dumps({k: round(v, 4) for k, v in stage_ms.items()}))

    nx, ny, p, B = wl.nx, wl.ny, wl.p, wl.B
    gflops = gram_flops(nx, ny, p)
    gram_peak = {"f64": PEAK["fp64_TF"], "f32": PEAK["fp32_TF"], "bf16r": PEAK["bf16_TF"]}[wl.prec]
    gram_tf = gflops / (stage_ms["blocks"] * 1e-3) / 1e12
    upd = packed_pairs(nx, ny) * B
    res_tf = 2.0 * upd / (stage_ms["resampling"] * 1e-3) / 1e12
    if stage_ms["resampling"] >= stage_ms["blocks"]:
        if wl.prec == "f64":
            roof = {"bound": "alu", "achieved": res_tf, "peak": PEAK["fp64_TF"], "unit": "TFLOP/s"}
        else:
            roof = {"bound": "mfma", "achieved": res_tf, "peak": PEAK["bf16_TF"], "unit": "TFLOP/s"}
        roof["kernel"] = "resampling (k_perm)"
        roof["algorithmic"] = "2 flops per (distinct off-diagonal block entry, split): %.4g" % (2 * upd)
    else:
        roof = {"bound": "mfma", "achieved": gram_tf, "peak": gram_peak, "unit": "TFLOP/s",
                "kernel": "blocks (k_gram)",
                "algorithmic": "2p flops per distinct Gram entry: %.4g" % gflops}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None

    line = {
        "metric": METRIC, "value": value, "unit": "permuted statistics/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16r": "bf16"}[wl.prec], "data": "synthetic",
        "config": {"workload": wl.name, "nx": nx, "ny": ny, "p": p, "B": B,
                   "statistics": kinds, "precision": wl.prec},
        "gram_tflops": gram_tf,
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "p_values": [r["p_value"] for r in res],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(wl, kinds, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
