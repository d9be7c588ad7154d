#!/usr/bin/env python3
"""Benchmark of the MI355X permutation two-sample test.

One step = one whole test (or batch of tests) on device-resident synthetic inputs:
staging, the three blocks (Gram on MFMA + epilogue), block sums and observed
statistic, centring, the split stream, all resampled statistics, threshold, count
and p-value -- every stage of the hot path.

Workloads (--workload):
  plain_f32       energy distance, FP32 form, X 2000 x 1000 ~ N(0, I), Y 2000 x 1000 with
                  mean 0.05 on the first 50 coordinates, B = 10^4        (default)
  small_f64       100 x 10 vs 100 x 10 null case, FP64 form, B = 1000
  precision_bf16  5000 x 4096 vs 4000 x 4096 (Y variance 1.1 on 200 coordinates), ED and
                  Gaussian MMD (sigma^2 = p), BF16-refined form, B = 10^4; the FP32 form of
                  the same tests is timed beside it
  batched         256 independent ED tests (nx, ny in [50, 1500], p in {20, 100, 500},
                  B = 2000) in one graph-captured batch; work shapes tuned on the batch
                  itself; the same tests run one by one (the library's shapes for a lone
                  test) are timed beside it
  serving         Poisson stream of tests (200/s by default) through the continuous-batching
                  server; latency p50 / p99 and served tests per second
  cross_f32/_bf16 cross-ED test (permutation-free) on the plain_f32 / precision_bf16 data
  studies         Section 5.2 null and power studies (efficient test vs cross-ED)
  timing          Section 5.1 computing-time experiments: standard, pre-computation,
                  efficient and cross-ED tests, B = 200, FP64 and FP32 forms
  hsic            HSIC independence permutation test (the discussion's extension), FP32,
                  n = 2000 and 4096 pairs, p = q = 500, B = 200

Prints ONE JSON line on stdout.  Per-stage device times come from HIP events recorded by
the library on the launch stream.
"""
import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "permuted statistics/sec and Gram TFLOP/s vs plain FP32; serving p50/p99 latency"
# The FP32 form's Gram forms each FP32-accurate product from three fp16 MFMA products
# (hi hi + hi lo + lo hi): its peak in algorithmic flops is the fp16 peak over three.
PEAK = {"hbm_GBs": 8000.0, "bf16_TF": 2500.0, "fp16_TF": 2500.0, "fp32_TF": 157.3,
        "f16x3_TF": 2500.0 / 3,
        "fp64_TF": 78.6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gram_flops(nx, ny, p):
    """Distinct Gram products: upper-triangular XX / YY (with diagonal) plus XY, 2p flops each."""
    return 2.0 * p * (nx * (nx + 1) / 2 + ny * (ny + 1) / 2 + nx * ny)


def packed_pairs(nx, ny):
    """Distinct off-diagonal block entries that determine every statistic."""
    return nx * (nx - 1) / 2 + ny * (ny - 1) / 2 + nx * ny


def to_dev(X, Y, prec):
    import torch
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = torch.from_numpy(X).to("cuda:0", dt)
    Yd = torch.from_numpy(Y).to("cuda:0", dt)
    torch.cuda.synchronize()
    return Xd, Yd


LIVE_STAGES = ["blocks", "resampling"]


def timed(fn, steps, warmup, profile=True):
    """Run fn warmup + steps times.  Returns (seconds for the timed steps, live profile,
    breakdown profile, last output).  During the timed steps the library brackets only the
    two candidate dominant stages (Gram, resampling) with HIP events on their launch stream
    ("live" times, every step); the full per-stage breakdown comes from a separate pass of
    min(steps, 5) calls, so its extra events stay out of the timed region."""
    import torch

    from paper_2406_06488_amd import api
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if profile:
        api.profile_enable(True, LIVE_STAGES)
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    live = breakdown = None
    if profile:
        live = api.profile_read()
        api.profile_enable(True)
        for _ in range(min(steps, 5)):
            fn()
        torch.cuda.synchronize()
        breakdown = api.profile_read()
        api.profile_enable(False)
    return t1 - t0, live, breakdown, out


def per_launch(prof):
    """{stage: ms per launch} for the stages that were timed."""
    return {k: v[0] / v[1] for k, v in prof.items() if v[1] > 0}


def roofline(stage_ms, tests, prec, workload=None, gram_tests=None):
    """Dominant kernel's algorithmic rate against its peak.  tests: list of (nx, ny, p, B)
    whose resampled statistics one launch of the resampling stage computes; gram_tests: the
    Gram products one launch of the block stage computes (default: the same tests; an ED
    and an MMD test on the same data share one Gram)."""
    gram_tests = tests if gram_tests is None else gram_tests
    # the Gram variant that also writes a partner test's blocks runs when tests share one
    dual = "true" if len(tests) > len(gram_tests) else "false"
    gflops = sum(gram_flops(nx, ny, p) for nx, ny, p, B in gram_tests)
    upd = sum(packed_pairs(nx, ny) * B for nx, ny, p, B in tests)
    if not stage_ms.get("blocks") or not stage_ms.get("resampling"):
        return None, None, None
    gram_tf = gflops / (stage_ms["blocks"] * 1e-3) / 1e12
    res_tf = 2.0 * upd / (stage_ms["resampling"] * 1e-3) / 1e12
    if stage_ms["resampling"] >= stage_ms["blocks"]:
        if prec == "f64":
            r = {"bound": "alu", "achieved": res_tf, "peak": PEAK["fp64_TF"], "unit": "TFLOP/s"}
        else:
            r = {"bound": "mfma", "achieved": res_tf, "peak": PEAK["fp16_TF"], "unit": "TFLOP/s"}
        r["kernel"] = {"f64": "k_perm_f64", "f32": "k_perm_mfma<2>", "bf16r": "k_perm_mfma<3>"}[prec]
        r["algorithmic"] = ("2 flops per (distinct off-diagonal block entry, split) = %.4g per "
                            "launch" % (2 * upd))
    else:
        peak = {"f64": PEAK["fp64_TF"], "f32": PEAK["f16x3_TF"], "bf16r": PEAK["bf16_TF"]}[prec]
        r = {"bound": "alu" if prec == "f64" else "mfma", "achieved": gram_tf, "peak": peak,
             "unit": "TFLOP/s",
             "kernel": {"f64": "k_dist_f64", "f32": "k_gram_f16x3<%s>" % dual,
                        "bf16r": "k_gram_bf16<%s>" % dual}[prec],
             "algorithmic": "2p flops per distinct Gram entry = %.4g per launch" % gflops}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = measured_traffic(r["kernel"], workload) if workload else None
    return r, gram_tf, res_tf


# a kernel's traffic depends on its source and on the launch shape the runtime picks
KERNEL_SOURCES = {"k_gram_f16x3": ["k_gram.hip", "k_prep.hip", "common.h", "runtime.cpp"],
                  "k_gram_bf16": ["k_gram.hip", "k_prep.hip", "common.h", "runtime.cpp"],
                  "k_gram_super": ["k_gram.hip", "k_prep.hip", "common.h", "runtime.cpp"],
                  "k_gram_finish": ["k_gram.hip", "common.h", "runtime.cpp"],
                  "k_dist_f64": ["k_gram.hip", "common.h", "runtime.cpp"],
                  "k_perm_mfma": ["k_perm.hip", "common.h", "runtime.cpp"],
                  "k_perm_f64": ["k_perm.hip", "common.h", "runtime.cpp"],
                  "k_precomp": ["k_baseline.hip", "common.h", "runtime.cpp"],
                  "k_hsic_terms": ["k_hsic.hip", "common.h", "runtime.cpp"]}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.md")


def source_hash(kernel):
    """Hash of the code (comments and whitespace dropped) of the files behind a kernel and its
    launch shape: a stored counter entry stays valid across comment-only edits."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2406_06488_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, or None when there is none
    for this kernel and workload or the kernel's source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
        blob = text[text.index("```json") + 7:]
        table = json.loads(blob[:blob.index("```")])
    except (OSError, ValueError):
        return None
    e = table.get("%s|%s" % (kernel, workload))
    if not e or e.get("source_sha256") != source_hash(kernel.split("<")[0]):
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def base_line(args, wl_name, value, elapsed, steps, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "permuted statistics/s", "n_gpus": 1,
            "steps": steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": dict(workload=wl_name, **config)}


# ---------------------------------------------------------------------------- CPU oracle

def cpu_baseline(tests, budget_s, label):
    """The FP64 oracle on the host: for each sampled test, blocks once and as many resampled
    splits as the time budget allows; the full-test rate is projected from the measured
    block and per-split times.  tests: list of (X, Y, B, seed, kind, gamma)."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    tot_time = 0.0
    tot_stats = 0
    done = 0
    detail = []
    per = budget_s / max(len(tests), 1)
    t_start = time.perf_counter()
    for X, Y, B, seed, kind, gamma in tests:
        if time.perf_counter() - t_start > budget_s:
            break
        X = X.astype(np.float64)
        Y = Y.astype(np.float64)
        k = oracle.ED if kind == "ed" else oracle.MMD
        t0 = time.perf_counter()
        XX, YY, XY = oracle.blocks(X, Y, k, gamma, threads)
        tb = time.perf_counter() - t0
        m = min(B, max(threads, 8))
        t0 = time.perf_counter()
        oracle.perm_stats_listed(XX, YY, XY, seed, list(range(m)), k, threads)
        tp = (time.perf_counter() - t0) / m
        more = int(min(B, max(0.0, per - tb - tp * m) / max(tp, 1e-9)))
        if more > m:
            t0 = time.perf_counter()
            oracle.perm_stats_listed(XX, YY, XY, seed, list(range(more)), k, threads)
            tp = (time.perf_counter() - t0) / more
        tot_time += tb + tp * B
        tot_stats += B
        done += 1
        detail.append("blocks %.2f s + %.3g s/split x %d measured" % (tb, tp, max(m, more)))
    return {"value": tot_stats / tot_time, "unit": "permuted statistics/s", "cores": threads,
            "kind": "oracle",
            "sample": "%s: %d test(s); per test the blocks once plus a bounded number of "
                      "splits, projected to all B splits (%s)" % (label, done,
                                                                  "; ".join(detail[:4]))}


def golden_parity(wl_name, kind, prec, res, ps):
    """The served result against the oracle's stored result for the same workload
    (tests/golden/fullsize_*, written by a script that runs the oracle alone): statistic and
    threshold error, the largest split error, count and p-value match, near-ties at the
    form's tolerance and the near-ties whose decision flipped.  None when no stored result
    exists for this workload."""
    import numpy as np
    base = os.path.join(ROOT, "tests", "golden", "fullsize_%s_%s" % (wl_name, kind))
    try:
        with open(base + ".json") as f:
            meta = json.load(f)
        ops = np.load(base + ".npy", allow_pickle=False)
    except OSError:
        return None
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16r": 1e-3}[prec]
    floor = float(np.mean(np.abs(ops)))
    err = np.abs(ps - ops) / np.maximum(np.abs(ops), floor)
    near = np.array(meta["near_ties"]["%g" % tol], dtype=np.int64)
    flipped = np.flatnonzero((ps >= res["threshold"]) != (ops >= meta["threshold"]))
    return {"kind": kind, "tolerance": tol,
            "rel_err_statistic": abs(res["statistic"] - meta["statistic"]) /
                                 max(abs(meta["statistic"]), floor),
            "rel_err_threshold": abs(res["threshold"] - meta["threshold"]) /
                                 max(abs(meta["threshold"]), floor),
            "max_rel_err_splits": float(err.max()), "count_ge": int(res["count_ge"]),
            "oracle_count_ge": meta["count_ge"], "p_value": res["p_value"],
            "oracle_p_value": meta["p_value"], "p_value_match": res["p_value"] == meta["p_value"],
            "near_ties": int(len(near)), "flipped": flipped.tolist()[:32],
            "flipped_outside_near_ties": int(np.sum(~np.isin(flipped, near))),
            "oracle_seconds": meta["oracle_seconds"], "oracle_threads": meta["oracle_threads"]}


def cpu_full(X, Y, B, seed, kind, gamma, label):
    """The oracle's whole test (blocks, observed statistic, all B splits, count, p-value) on
    the host's cores, timed; returns the baseline record and the oracle's result."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    o = oracle.run_test(X.astype("float64"), Y.astype("float64"), B, seed,
                        oracle.ED if kind == "ed" else oracle.MMD, gamma, threads)
    secs = time.perf_counter() - t0
    return {"value": B / secs, "unit": "permuted statistics/s", "cores": threads,
            "kind": "oracle", "sample": "%s: the whole test, all %d splits (%.1f s)"
                                        % (label, B, secs)}, o


# ---------------------------------------------------------------------------- workloads

def run_single(args):
    from paper_2406_06488_amd import api, inputs
    if args.workload == "plain_f32":
        wl, kinds = inputs.plain_f32(), ["ed"]
    elif args.workload == "small_f64":
        wl, kinds = inputs.small_null_f64(), ["ed"]
    else:
        wl = inputs.precision_bf16()
        kinds = wl.kinds
    log("workload", wl.name, "kinds", kinds, "steps", args.steps, "warmup", args.warmup)
    X, Y = wl.data()
    Xd, Yd = to_dev(X, Y, wl.prec)

    if len(kinds) == 1:
        # tests enqueued back to back (results land in device memory; the host reads them
        # after the closing synchronisation); single-test latency is reported beside it
        import torch
        ps = torch.empty(wl.B, dtype=torch.float64, device="cuda:0")

        def step(prec=wl.prec):
            return [api.run_async(Xd, Yd, wl.B, wl.perm_seed, kinds[0], prec, wl.gamma(), ps)]
    else:
        # ED and MMD on the same data in one batch: they share staging and the Gram
        import torch
        outs = [torch.empty(wl.B, dtype=torch.float64, device="cuda:0") for _ in kinds]

        def step(prec=wl.prec):
            reqs = [api.make_request(Xd, Yd, wl.B, wl.perm_seed, k, prec, wl.gamma(), o)
                    for k, o in zip(kinds, outs)]
            return api.batch(reqs)

    elapsed, live, prof, res = timed(step, args.steps, args.warmup)
    if len(kinds) == 1:
        res = [api.result_from_device(r) for r in res]

    stage = per_launch(prof)
    live_ms = {k: v for k, v in per_launch(live).items() if k in LIVE_STAGES}
    stage.update(live_ms)
    log("stage ms per test:", json.dumps({k: round(v, 4) for k, v in stage.items()}))
    gshape = [(wl.nx, wl.ny, wl.p, wl.B)]
    shape = gshape * len(kinds)
    roof, gram_tf, res_tf = roofline(stage, shape, wl.prec, wl.name, gshape)
    value = len(kinds) * wl.B * args.steps / elapsed
    # what the arithmetic is: the FP32 form multiplies fp16 pairs (22 significant bits)
    # with FP32 accumulation; the BF16-refined form BF16 operands with FP32 accumulation
    # (fp16 + e4m3 planes in the resampling stage); both reduce in FP64
    dtype = {"f64": "f64", "f32": "f16x2->f32", "bf16r": "bf16->f32"}[wl.prec]
    arith = {"f64": "FP64 end to end",
             "f32": "Gram and resampling on fp16 MFMA from fp16 (hi, lo) pairs of each value "
                    "(22 significant bits), FP32 accumulation, FP64 reductions",
             "bf16r": "Gram on BF16 MFMA (fp16 pairs below p = 64) with FP32 accumulation and "
                      "FP32 recomputation of near pairs; resampling on fp16 + e4m3 planes; "
                      "FP64 reductions"}[wl.prec]
    line = base_line(args, wl.name, value, elapsed, args.steps, dtype,
                     {"nx": wl.nx, "ny": wl.ny, "p": wl.p, "B": wl.B, "statistics": kinds,
                      "precision": wl.prec, "arithmetic": arith})
    line.update({"gram_tflops": gram_tf, "resampling_tflops": res_tf,
                 "stage_ms": {k: round(v, 5) for k, v in stage.items()},
                 "stage_ms_live": sorted(live_ms),
                 "p_values": [r["p_value"] for r in res], "roofline": roof})
    if len(kinds) == 1:
        lat = []
        for _ in range(5):
            t0 = time.perf_counter()
            api.run(Xd, Yd, wl.B, wl.perm_seed, kinds[0], wl.prec, wl.gamma())
            lat.append(time.perf_counter() - t0)
        line["config"]["submission"] = "asynchronous, back to back"
        line["latency_ms_single_test"] = 1e3 * sorted(lat)[len(lat) // 2]
    else:
        line["config"]["submission"] = "one synchronous etest_batch call per step (graph replay)"
    # this run's per-split statistics, read before the FP32 form below reuses the outputs
    host_ps = [ps.cpu().numpy()] if len(kinds) == 1 else [o.cpu().numpy() for o in outs]
    if wl.prec == "bf16r":
        # the plain FP32 form on the same tests
        e32, l32, p32, _ = timed(lambda: step("f32"), max(2, args.steps // 2), 1)
        s32 = per_launch(p32)
        s32.update({k: v for k, v in per_launch(l32).items() if k in LIVE_STAGES})
        _, g32, r32 = roofline(s32, shape, "f32", None, gshape)
        line["f32_form"] = {"ms_per_step": 1e3 * e32 / max(2, args.steps // 2),
                            "gram_tflops": g32, "resampling_tflops": r32,
                            "stage_ms": {k: round(v, 5) for k, v in s32.items()}}
        line["speedup_vs_f32_form"] = line["f32_form"]["ms_per_step"] / line["ms_per_step"]
    # parity of this run's results with the oracle's stored results for the workload
    par = [golden_parity(wl.name, k, wl.prec, r, h) for k, r, h in zip(kinds, res, host_ps)]
    line["oracle_parity"] = par if any(x is not None for x in par) else None
    if args.no_cpu_baseline:
        line["cpu_baseline"] = None
    elif wl.name == "ed_f32_2000x1000_B10000" or wl.prec == "f64":
        # small enough for the oracle's whole test (about 40 s on 16 host cores)
        log("cpu baseline (oracle, whole test) ...")
        line["cpu_baseline"], o = cpu_full(X, Y, wl.B, wl.perm_seed, kinds[0], wl.gamma(),
                                           wl.name)
        line["oracle_same_run"] = {"count_ge": o["count_ge"], "p_value": o["p_value"],
                                   "p_value_match": o["p_value"] == res[0]["p_value"],
                                   "rel_err_statistic": abs(res[0]["statistic"] - o["statistic"])
                                   / abs(o["statistic"])}
    else:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(
            [(X, Y, wl.B, wl.perm_seed, k, wl.gamma()) for k in kinds], args.cpu_seconds,
            wl.name)
    return line


def run_batched(args):
    import numpy as np
    import torch

    from paper_2406_06488_amd import api, autotune, inputs
    tests = inputs.batched_tests()
    log("batched: %d tests, generating inputs" % len(tests))
    data, reqs, keep = [], [], []
    for w in tests:
        X, Y = w.data()
        Xd, Yd = to_dev(X, Y, w.prec)
        data.append((X, Y))
        keep += [Xd, Yd]
        reqs.append(api.make_request(Xd, Yd, w.B, w.perm_seed, "ed", w.prec))
    reqs = (api.Request * len(reqs))(*reqs)  # built once, passed as it is every step
    # the same tests one by one (plain path), timed first, under the library's own shapes
    # for a lone test (row units short enough that each test spreads over the chip)
    seq_steps = max(1, args.steps // 4)

    def seq():
        return [api.run(keep[2 * i], keep[2 * i + 1], w.B, w.perm_seed, "ed", w.prec,
                        with_perm_stats=False) for i, w in enumerate(tests)]
    autotune.clear()
    e_seq, _, _, _ = timed(seq, seq_steps, 1, profile=False)
    # tune the resampling work shape per size bucket on the batch itself
    ranges = [(lo, hi) for lo, hi in ((0, 1024), (1024, 2048), (2048, 1 << 31))
              if any(lo <= w.nx + w.ny < hi for w in tests)]
    rules = autotune.tune_batch(lambda: api.batch(reqs), ranges, "f32", reps=5, log=log)
    log("tuned:", [(r["n_lo"], r["n_hi"], r["kc"], r["cc"]) for r in rules])
    elapsed, _, _, outs = timed(lambda: api.batch(reqs), args.steps, args.warmup, profile=False)
    total_B = sum(w.B for w in tests)
    value = total_B * args.steps / elapsed
    # stage times of the same batch through the non-graph path (one launch per stage)
    _, live, prof, _ = timed(lambda: api.batch(reqs), 2, 0, profile=True)
    stage = per_launch(prof)
    live_ms = {k: v for k, v in per_launch(live).items() if k in LIVE_STAGES}
    stage.update(live_ms)
    shape = [(w.nx, w.ny, w.p, w.B) for w in tests]
    roof, gram_tf, res_tf = roofline(stage, shape, "f32", "ed_f32_batch256_B2000")
    # ... and the same tests one by one again, under the batch's rules: the results must be
    # the batch's
    t_id = time.perf_counter()
    seq_out = seq()
    import torch
    torch.cuda.synchronize()
    log("one by one under the batch's rules: %.1f ms" % (1e3 * (time.perf_counter() - t_id)))
    same = all(a["count_ge"] == b["count_ge"] and a["statistic"] == b["statistic"]
               for a, b in zip(outs, seq_out))
    autotune.clear()
    line = base_line(args, "ed_f32_batch256_B2000", value, elapsed, args.steps, "f32",
                     {"tests": len(tests), "B": 2000, "nx_ny_range": [50, 1500],
                      "p": [20, 100, 500], "precision": "f32",
                      "submission": "one synchronous etest_batch call per step (graph replay)"})
    line.update({"gram_tflops": gram_tf, "resampling_tflops": res_tf,
                 "stage_ms": {k: round(v, 5) for k, v in stage.items()}, "roofline": roof,
                 "sequential_ms_per_step": 1e3 * e_seq / seq_steps,
                 "speedup_vs_sequential": (e_seq / seq_steps) / (elapsed / args.steps),
                 "batch_equals_sequential": same,
                 "tuning": [{k: r[k] for k in ("n_lo", "n_hi", "kc", "cc")} for r in rules]})
    if not args.no_cpu_baseline:
        sample = [(data[i][0], data[i][1], w.B, w.perm_seed, "ed", 0.0)
                  for i, w in enumerate(tests[:16])]
        line["cpu_baseline"] = cpu_baseline(sample, args.cpu_seconds, "batch256 (first tests)")
    else:
        line["cpu_baseline"] = None
    return line


def run_cross(args):
    """Cross-ED test (permutation-free, the paper's Alg. 7) on the plain_f32 data (FP32) or
    the precision_bf16 data (BF16-refined): tests/s, and the cross blocks' Gram rate."""
    import numpy as np

    from paper_2406_06488_amd import api, inputs
    wl = inputs.plain_f32() if args.workload == "cross_f32" else inputs.precision_bf16()
    prec = "f32" if args.workload == "cross_f32" else "bf16r"
    X, Y = wl.data()
    Xd, Yd = to_dev(X, Y, prec)
    nx1, ny1 = wl.nx // 2, wl.ny // 2
    rows, cols = nx1 + ny1, wl.nx + wl.ny - nx1 - ny1
    name = "cross_ed_%s_%dx%dx%d" % (prec, wl.nx, wl.ny, wl.p)
    log("workload", name, "steps", args.steps, "warmup", args.warmup)

    def step():
        return api.cross(Xd, Yd, "ed", prec)

    elapsed, live, prof, res = timed(step, args.steps, args.warmup)
    stage = per_launch(prof)
    stage.update({k: v for k, v in per_launch(live).items() if k in LIVE_STAGES})
    flops = 2.0 * wl.p * rows * cols  # every cross pair once: no symmetry to use
    gram_tf = flops / (stage["blocks"] * 1e-3) / 1e12
    peak = PEAK["f16x3_TF"] if prec == "f32" else PEAK["bf16_TF"]
    kernel = "k_gram_f16x3<false>" if prec == "f32" else "k_gram_bf16<false>"
    line = base_line(args, name, args.steps / elapsed, elapsed, args.steps,
                     "f32" if prec == "f32" else "bf16",
                     {"nx": wl.nx, "ny": wl.ny, "p": wl.p, "statistic": "cross-ed",
                      "precision": prec})
    line.update({"metric": "cross-ED tests/s", "unit": "tests/s", "gram_tflops": gram_tf,
                 "stage_ms": {k: round(v, 5) for k, v in stage.items()},
                 "stage_ms_live": [k for k in LIVE_STAGES if k in stage],
                 "result": res,
                 "roofline": {"bound": "mfma", "achieved": gram_tf, "peak": peak,
                              "unit": "TFLOP/s", "kernel": kernel,
                              "algorithmic": "2p flops per cross pair = %.4g per launch" % flops,
                              "frac": gram_tf / peak, "traffic": measured_traffic(kernel, name)}})
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle) ...")
        t0 = time.perf_counter()
        oracle.cross(X.astype(np.float64), Y.astype(np.float64), oracle.ED)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "tests/s",
                                "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                "kind": "oracle", "sample": "%s: one whole test" % name}
    else:
        line["cpu_baseline"] = None
    return line


def run_studies(args):
    """Section 5.2 studies through the batched path: null p-values and power of the
    efficient permutation ED test vs the cross-ED test (200 permutations), with the
    paper's replication counts unless --reps scales them."""
    from paper_2406_06488_amd import studies
    scale = args.reps_scale
    t0 = time.perf_counter()
    null = studies.null_study(reps=max(1, int(2000 * scale)))
    power = {name: studies.power_study(st, reps=max(1, int(500 * scale)))
             for name, st in (("setting_1", studies.SETTING_1), ("setting_2", studies.SETTING_2),
                              ("setting_3", studies.SETTING_3))}
    elapsed = time.perf_counter() - t0
    tests = sum(2 * r["reps"] for r in null) + sum(2 * pt["reps"] for pts in power.values() for pt in pts)
    line = base_line(args, "studies_section5_2", tests / elapsed, elapsed, 1, "f32",
                     {"B": 200, "tests": tests})
    line.update({"metric": "tests/s over the Section 5.2 studies (both tests counted)",
                 "unit": "tests/s", "null": null, "power": power, "roofline": None,
                 "cpu_baseline": None})
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["oracle_parity"] = studies_oracle_leg()
    return line


def studies_oracle_leg(reps=4, B=200):
    """The CPU leg of the studies: the FP64 oracle's efficient permutation test and cross-ED
    test on the first replications of the null study (n = 200, p = 100 and 1000; the same
    data and split seeds as the GPU run), timed; returns the baseline and the comparison."""
    import numpy as np

    import oracle
    from paper_2406_06488_amd import studies
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    recs, secs = [], 0.0
    for p in (100, 1000):
        res, cross, kept = studies.pvalues(200, 200, p, reps, B=B, seed=1 + p, keep=reps,
                                           detail=True)
        for r, c, (X, Y, sd) in zip(res, cross, kept):
            t0 = time.perf_counter()
            o = oracle.run_test(X.astype(np.float64), Y.astype(np.float64), B, sd, oracle.ED,
                                1.0, threads)
            oc = oracle.cross(X.astype(np.float64), Y.astype(np.float64), oracle.ED, 1.0,
                              threads)
            secs += time.perf_counter() - t0
            floor = float(np.mean(np.abs(o["perm_stats"])))
            near = int(np.sum(np.abs(o["perm_stats"] - o["threshold"]) <=
                              1e-5 * max(abs(o["threshold"]), floor)))
            recs.append({"p": p, "split_seed": sd,
                         "rel_err_statistic": abs(r["statistic"] - o["statistic"]) /
                                              max(abs(o["statistic"]), floor),
                         "count_ge": r["count_ge"], "oracle_count_ge": o["count_ge"],
                         "p_value_match": r["p_value"] == o["p_value"], "near_ties": near,
                         "cross_p_value": c, "oracle_cross_p_value": oc["p_value"]})
    base = {"value": len(recs) / secs, "unit": "tests/s", "cores": threads, "kind": "oracle",
            "sample": "%d null replications (n = 200, p = 100 and 1000, B = %d): efficient "
                      "permutation test and cross-ED test, %.1f s" % (len(recs), B, secs)}
    return base, {"replications": recs,
                  "p_value_matches": sum(1 for x in recs if x["p_value_match"]),
                  "max_abs_cross_p_diff": max(abs(x["cross_p_value"] - x["oracle_cross_p_value"])
                                              for x in recs)}


# VALU issue rate of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions/s
# (FP64 FMA issues at the full rate: 78.6 TFLOP/s = this rate x 2 flops)
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
PRECOMP_OPS_PER_ENTRY = 1   # one FP64 FMA (entry x split bit) per entry and split


def run_timing(args):
    """Section 5.1 computing-time experiments on one GPU: seconds per test of the standard
    (Alg. 4), pre-computation (Alg. 5: on symmetric upper tiles, and on the dense pooled
    matrix as printed), efficient (Alg. 1) and cross-ED (Alg. 7) energy
    distance tests with B = 200, data N_p(0, I); experiment 1: p = 500, nx = ny = 100..1000;
    experiment 2: nx = ny = 200, p = 200..2000.  Wall time of each synchronous call (inputs
    already on the device), averaged over --timing-reps replications (half as many for the
    standard test, as in the paper's ratio of 10 to 100), each on freshly drawn data."""
    import numpy as np
    import torch

    from paper_2406_06488_amd import api
    B = 200
    exps = {"exp1_p500_n": [(n, 500) for n in range(100, 1001, 100)],
            "exp2_n200_p": [(200, p) for p in range(200, 2001, 200)]}
    precs = [q for q in args.timing_precs.split(",") if q]
    fns = {
        "standard": lambda X, Y, q: api.standard(X, Y, B, 1, "ed", q, with_perm_stats=False),
        "precomputed": lambda X, Y, q: api.precomputed(X, Y, B, 1, "ed", q,
                                                       with_perm_stats=False),
        # Alg. 5 as printed: the dense (nx + ny)^2 pooled matrix, D_YX included
        "precomputed_dense": lambda X, Y, q: api.precomputed(X, Y, B, 1, "ed", q,
                                                             with_perm_stats=False, dense=True),
        "efficient": lambda X, Y, q: api.run(X, Y, B, 1, "ed", q, with_perm_stats=False),
        "cross": lambda X, Y, q: api.cross(X, Y, "ed", q),
    }
    gen = torch.Generator(device="cuda")
    gen.manual_seed(20240610)
    tables = {}
    t_all = time.perf_counter()
    for q in precs:
        dt = torch.float64 if q == "f64" else torch.float32
        for ename, shapes in exps.items():
            tab = {}
            for n, p in shapes:
                key = str(n if ename.startswith("exp1") else p)
                row = {}
                for mname, fn in fns.items():
                    reps = args.timing_reps if mname != "standard" else max(1, args.timing_reps // 2)
                    X = torch.randn(n, p, generator=gen, device="cuda", dtype=dt)
                    Y = torch.randn(n, p, generator=gen, device="cuda", dtype=dt)
                    fn(X, Y, q)  # first call of the shape: pools and modules warm
                    ts = []
                    for _ in range(reps):
                        X = torch.randn(n, p, generator=gen, device="cuda", dtype=dt)
                        Y = torch.randn(n, p, generator=gen, device="cuda", dtype=dt)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        fn(X, Y, q)
                        ts.append(time.perf_counter() - t0)
                    row[mname] = {"mean_ms": 1e3 * float(np.mean(ts)),
                                  "min_ms": 1e3 * float(np.min(ts)), "reps": reps}
                row["speedup_vs_standard"] = row["standard"]["mean_ms"] / row["efficient"]["mean_ms"]
                row["speedup_vs_precomputed"] = (row["precomputed"]["mean_ms"] /
                                                 row["efficient"]["mean_ms"])
                row["speedup_vs_precomputed_dense"] = (row["precomputed_dense"]["mean_ms"] /
                                                       row["efficient"]["mean_ms"])
                tab[key] = row
                log(q, ename, key, {m: round(row[m]["mean_ms"], 3) for m in fns})
            tables["%s_%s" % (q, ename)] = tab
    elapsed = time.perf_counter() - t_all
    # the per-split sums of the pre-computation test at the largest experiment-1 shape:
    # kernel time from HIP events on its launch stream, against the VALU issue bound
    n, p = 1000, 500
    X = torch.randn(n, p, generator=gen, device="cuda", dtype=torch.float32)
    Y = torch.randn(n, p, generator=gen, device="cuda", dtype=torch.float32)
    fns["precomputed"](X, Y, "f32")
    torch.cuda.synchronize()
    api.profile_enable(True, ["resampling"])
    for _ in range(5):
        fns["precomputed"](X, Y, "f32")
    prof = per_launch(api.profile_read())
    api.profile_enable(False)
    pc_ms = prof["resampling"]
    entries = (B + 1) * (2 * n) * (2 * n + 1) / 2.0   # every unordered pooled pair, every split
    achieved = entries / (pc_ms * 1e-3)
    peak = VALU_LANE_OPS / PRECOMP_OPS_PER_ENTRY
    big = tables.get("f32_exp1_p500_n", tables[next(iter(tables))])["1000"]
    line = base_line(args, "timing_section5_1", 1e3 / big["efficient"]["mean_ms"], elapsed, 1,
                     "f32", {"B": B, "experiments": list(exps), "precisions": precs,
                             "reps": args.timing_reps})
    line.update({"metric": "efficient ED tests/s at nx = ny = 1000, p = 500, B = 200 "
                           "(Section 5.1 timing experiments, all four tests timed)",
                 "unit": "tests/s", "tables": tables,
                 "roofline": {"bound": "alu", "kernel": "k_precomp<float>",
                              "achieved": achieved, "peak": peak,
                              "unit": "entry selections/s",
                              "algorithmic": "(B+1) n(n+1)/2 = %.4g per launch" % entries,
                              "frac": achieved / peak, "traffic": None, "ms": pc_ms}})
    if not args.no_cpu_baseline:
        import oracle
        Xh, Yh = X.double().cpu().numpy(), Y.double().cpu().numpy()
        log("cpu baseline (oracle) ...")
        t0 = time.perf_counter()
        oracle.run_test(Xh, Yh, B, 1)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "tests/s",
                                "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                "kind": "oracle",
                                "sample": "one whole test, nx = ny = 1000, p = 500, B = 200"}
    else:
        line["cpu_baseline"] = None
    return line


def run_hsic(args):
    """HSIC independence permutation test (the extension in the paper's discussion), FP32
    form: n pairs, x and y of dimension p = q = 500, Gaussian kernels with gamma = 1/p,
    B = 200 permutations (the paper's count), dependence through tanh of the first
    coordinates.  n = 2000 (headline) and n = 4096 (the largest supported).  Steps are whole
    tests; the per-stage times come from HIP events on the launch stream."""
    import numpy as np
    import torch

    from paper_2406_06488_amd import api
    B, p = 200, 500
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    rows = {}
    head = None
    for n in [int(v) for v in args.hsic_n.split(",") if v]:
        X = torch.randn(n, p, generator=gen, device="cuda")
        Y = torch.randn(n, p, generator=gen, device="cuda")
        Y[:, :10] += 0.2 * torch.tanh(X[:, :10])

        def step():
            return api.hsic(X, Y, B, 1, 1.0 / p, 1.0 / p, "f32", with_perm_stats=False)

        elapsed, live, prof, res = timed(step, args.steps, args.warmup)
        stage = per_launch(prof)
        terms_ms = per_launch(live)["resampling"]
        entries = (B + 1) * n * n
        rows[str(n)] = {"ms_per_test": 1e3 * elapsed / args.steps, "p_value": res["p_value"],
                        "statistic": res["statistic"],
                        "stage_ms": {k: round(v, 5) for k, v in stage.items()},
                        "terms_ms_live": terms_ms,
                        "terms_gather_GBs": entries * 8 / (terms_ms * 1e-3) / 1e9}
        log("hsic n", n, rows[str(n)])
        if head is None:
            head = (n, elapsed, terms_ms, entries, X, Y)
    n, elapsed, terms_ms, entries, X, Y = head
    achieved = entries * 8 / (terms_ms * 1e-3) / 1e9
    line = base_line(args, "hsic_f32_n2000_p500_B200", args.steps / elapsed, elapsed, args.steps,
                     "f32", {"n": n, "p": p, "q": p, "B": B, "kernel": "gaussian, gamma = 1/p"})
    line.update({"metric": "HSIC permutation tests/s (n = 2000, p = q = 500, B = 200)",
                 "unit": "tests/s", "sizes": rows,
                 "roofline": {"bound": "hbm", "kernel": "k_hsic_terms<float>",
                              "achieved": achieved, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                              "algorithmic": "8 bytes (one Kt and one gathered Lt entry) per "
                                             "entry and permutation: (B+1) n^2 x 8 = %.4g per "
                                             "launch" % (entries * 8),
                              "frac": achieved / PEAK["hbm_GBs"],
                              "traffic": measured_traffic("k_hsic_terms<float>",
                                                          "hsic_f32_n2000_p500_B200")}})
    if not args.no_cpu_baseline:
        import oracle
        Xh, Yh = X.double().cpu().numpy(), Y.double().cpu().numpy()
        bs = 4
        log("cpu baseline (oracle) ...")
        t0 = time.perf_counter()
        oracle.hsic_test(Xh, Yh, bs, 1, 1.0 / p, 1.0 / p)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.hsic_test(Xh, Yh, 0, 1, 1.0 / p, 1.0 / p)
        d0 = time.perf_counter() - t0
        per_perm = max(dt - d0, 1e-9) / bs
        line["cpu_baseline"] = {"value": 1.0 / (d0 + per_perm * B), "unit": "tests/s",
                                "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                                "kind": "oracle",
                                "sample": "kernel matrices and identity, then %d permutations "
                                          "at n = %d (projected to B = %d)" % (bs, n, B)}
    else:
        line["cpu_baseline"] = None
    return line


def serving_oracle_check(checked, budget_s, tol=1e-3):
    """The oracle on the served results kept for checking: per request the blocks, the
    observed statistic, the threshold and the splits whose served statistic lies within
    twice the tolerance of the served threshold (the only ones whose decision a result
    within the tolerance could flip), plus 16 seeded random splits.  The oracle's count is
    the served count corrected by the oracle's decisions on those splits.  Stops when the
    time budget is spent; returns the per-request records."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = []
    t_start = time.perf_counter()
    for rec in checked:
        if time.perf_counter() - t_start > budget_s:
            break
        X, Y, ps, r, w = rec["X"], rec["Y"], rec["ps"], rec["res"], rec["w"]
        kind = w.kinds[0]
        k = oracle.ED if kind == "ed" else oracle.MMD
        gamma = w.gamma() if kind == "mmd" else 1.0
        XX, YY, XY = oracle.blocks(X, Y, k, gamma, threads)
        so, _ = oracle.observed(XX, YY, XY, k)
        to = oracle.threshold(XX, YY, XY, k)
        g = np.random.Generator(np.random.PCG64(1000 + int(w.name[3:])))
        rnd = g.integers(0, w.B, size=16)
        floor_g = float(np.mean(np.abs(ps)))
        band = np.flatnonzero(np.abs(ps - r["threshold"]) <= 2 * tol * max(abs(r["threshold"]), floor_g))
        whole_band = len(band) <= 256  # else the p-value is not reconstructed
        idx = np.unique(np.concatenate([rnd, band if whole_band else band[:0]]))
        ops = oracle.perm_stats_listed(XX, YY, XY, w.perm_seed, idx, k, threads)
        floor = float(np.mean(np.abs(ops)))
        err = np.abs(ps[idx] - ops) / np.maximum(np.abs(ops), floor)
        o_count, near, flips, flips_out = None, 0, 0, 0
        if whole_band:
            ob = ops[np.searchsorted(idx, band)]
            o_count = int(r["count_ge"] - np.sum(ps[band] >= r["threshold"]) + np.sum(ob >= to))
            is_near = np.abs(ob - to) <= tol * max(abs(to), floor)
            near = int(np.sum(is_near))
            flipped = (ps[band] >= r["threshold"]) != (ob >= to)
            flips = int(np.sum(flipped))
            flips_out = int(np.sum(flipped & ~is_near))
        out.append({"request": w.name, "nx": w.nx, "ny": w.ny, "p": w.p, "B": w.B, "kind": kind,
                    "rel_err_statistic": abs(r["statistic"] - so) / max(abs(so), floor),
                    "rel_err_threshold": abs(r["threshold"] - to) / max(abs(to), floor),
                    "max_rel_err_splits": float(err.max()), "splits_checked": int(len(idx)),
                    "count_ge": int(r["count_ge"]), "oracle_count_ge": o_count,
                    "p_value_match": None if o_count is None else o_count == r["count_ge"],
                    "near_ties": near, "flipped": flips, "flipped_outside_near_ties": flips_out})
    return out


def run_serving(args):
    """Open-loop Poisson stream through the continuous-batching server (latency, served
    rate), the oracle on every 50th request with nx, ny <= 5000, then capacity: the first
    requests submitted all at once, against the same requests run one by one through the
    synchronous entry point in the plain FP32 form and in the BF16-refined form."""
    import queue

    import numpy as np
    import torch

    from paper_2406_06488_amd import api, inputs
    stream = inputs.serving_stream(rate=args.rate, duration=args.duration)
    log("serving: %d requests over %.0f s at %.0f/s" % (len(stream), args.duration, args.rate))
    dev = "cuda:0"

    def data_of(w):
        # per-request data from the request's own seed (data seed 100000 + r)
        return inputs.device_pair(w.nx, w.ny, w.p, w.data_seed, w.mean_shift, dev)

    def gamma_of(w):
        return w.gamma() if w.kinds[0] == "mmd" else 0.0

    # producer: each request's data is drawn on a stream of its own before its arrival time
    # (the data arrive with the request); at most `ahead` requests wait
    ready = queue.Queue(maxsize=48)

    def producer():
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            for t_arr, w in stream:
                X, Y = data_of(w)
                gs.synchronize()
                ready.put((X, Y))
        ready.put(None)

    check_every = 50
    srv = api.Server(memory_budget_bytes=int(args.budget_gb * (1 << 30)), max_resident=64,
                     max_queue=1 << 20)
    lat, submitted, done_t, checked = {}, {}, {}, {}
    lock = threading.Lock()
    stop = threading.Event()

    def collector():
        while not (stop.is_set() and not submitted):
            with lock:
                ids = list(submitted.keys())
            for rid in ids:
                r = srv.poll(rid)
                if r is not None:
                    now = time.perf_counter()
                    with lock:
                        t_arr = submitted.pop(rid)
                        lat[rid] = now - t_arr
                        done_t[rid] = (now, r)
            time.sleep(0.0005)

    pth = threading.Thread(target=producer, daemon=True)
    pth.start()
    th = threading.Thread(target=collector, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for idx, (t_arr, w) in enumerate(stream):
        X, Y = ready.get()
        now = time.perf_counter() - t0
        if now < t_arr:
            time.sleep(t_arr - now)
        ps = None
        if idx % check_every == 0 and w.nx <= 5000 and w.ny <= 5000:
            ps = torch.empty(w.B, dtype=torch.float64, device=dev)
        rid = srv.submit(X, Y, w.B, w.perm_seed, w.kinds[0], "bf16r", gamma_of(w), ps)
        if ps is not None:
            checked[rid] = {"X": X, "Y": Y, "ps": ps, "w": w}
        with lock:
            submitted[rid] = t0 + t_arr
    t_last = time.perf_counter()
    stop.set()
    th.join()
    t_end = max(v[0] for v in done_t.values())
    srv.close()
    L = np.array(sorted(lat.values())) * 1e3
    served = len(lat) / (t_end - t0)
    total_B = sum(w.B for _, w in stream)
    line = base_line(args, "serving_poisson%d_%ds" % (args.rate, args.duration),
                     total_B / (t_end - t0), t_end - t0, 1, "bf16",
                     {"rate_per_s": args.rate, "duration_s": args.duration,
                      "requests": len(stream), "nx_ny_range": [100, 20000],
                      "p_range": [10, 2000], "B": [1000, 10000], "statistics": ["ed", "mmd"],
                      "precision": "bf16r",
                      "data": "per request N(0, I) / N(delta 1, I) from torch's device "
                              "generator seeded 100000 + r"})
    line.update({"p50_ms": float(np.percentile(L, 50)), "p99_ms": float(np.percentile(L, 99)),
                 "mean_ms": float(L.mean()), "max_ms": float(L.max()),
                 "tests_per_s": served, "offered_per_s": len(stream) / args.duration,
                 "submit_lag_s": t_last - t0 - stream[-1][0], "roofline": None})

    # oracle subset
    recs = []
    for rid, c in sorted(checked.items(), key=lambda kv: kv[1]["w"].name):
        recs.append({"X": c["X"].double().cpu().numpy(), "Y": c["Y"].double().cpu().numpy(),
                     "ps": c["ps"].cpu().numpy(), "res": done_t[rid][1], "w": c["w"]})
    checked.clear()
    log("serving: oracle on %d requests (budget %.0f s)" % (len(recs), args.cpu_seconds * 4))
    # the CPU leg: the oracle on the checked requests, timed; its results give the parity
    if args.no_cpu_baseline:
        recs.clear()
        par = None
    else:
        t_or = time.perf_counter()
        par = serving_oracle_check(recs, args.cpu_seconds * 4)
        t_or = time.perf_counter() - t_or
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        line["cpu_baseline"] = {
            "value": len(par) / t_or if par else None, "unit": "checked requests/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d requests (every %dth with nx, ny <= 5000): FP64 blocks, observed "
                      "statistic, threshold and the splits near the threshold, %.1f s"
                      % (len(par), check_every, t_or)}
    line["oracle_parity"] = None if par is None else {
        "rule": "every %dth request with nx, ny <= 5000; statistic, threshold and the splits "
                "within twice the 1e-3 tolerance of the threshold plus 16 random splits by the "
                "FP64 oracle; oracle count = served count corrected by the oracle's decisions "
                "on those splits" % check_every,
        "eligible": len(recs), "checked": len(par),
        "max_rel_err_statistic": max((x["rel_err_statistic"] for x in par), default=None),
        "max_rel_err_threshold": max((x["rel_err_threshold"] for x in par), default=None),
        "max_rel_err_splits": max((x["max_rel_err_splits"] for x in par), default=None),
        "p_value_matches": sum(1 for x in par if x["p_value_match"]),
        "p_value_unreconstructed": sum(1 for x in par if x["p_value_match"] is None),
        "near_ties": sum(x["near_ties"] for x in par),
        "flipped": sum(x["flipped"] for x in par),
        "flipped_outside_near_ties": sum(x["flipped_outside_near_ties"] for x in par),
        # every request whose p-value differs, then the first few others
        "requests": ([x for x in par if x["p_value_match"] is False] +
                     [x for x in par if x["p_value_match"] is not False])[:12]}
    recs.clear()

    # capacity: the first requests all at once, and one by one in the FP32 and BF16 forms
    ncap = min(len(stream), args.capacity_requests)
    cap = []
    for _, w in stream[:ncap]:
        X, Y = data_of(w)
        cap.append((X, Y, w))
    torch.cuda.synchronize()
    with api.Server(memory_budget_bytes=int(args.budget_gb * (1 << 30)), max_resident=64,
                    max_queue=1 << 20) as srv2:
        t1 = time.perf_counter()
        ids = [srv2.submit(X, Y, w.B, w.perm_seed, w.kinds[0], "bf16r", gamma_of(w))
               for X, Y, w in cap]
        for rid in ids:
            srv2.wait(rid)
        t_srv = time.perf_counter() - t1
    one = {}
    for prec in ("f32", "bf16r"):
        t1 = time.perf_counter()
        for X, Y, w in cap:
            api.run(X, Y, w.B, w.perm_seed, w.kinds[0], prec, gamma_of(w), with_perm_stats=False)
        one[prec] = time.perf_counter() - t1
    line["capacity"] = {
        "requests": ncap, "served_all_at_once_tests_per_s": ncap / t_srv,
        "one_by_one_f32_tests_per_s": ncap / one["f32"],
        "one_by_one_bf16r_tests_per_s": ncap / one["bf16r"],
        "served_vs_one_by_one_f32": one["f32"] / t_srv,
        "served_vs_one_by_one_bf16r": one["bf16r"] / t_srv}
    log("serving capacity:", json.dumps(line["capacity"]))
    line.setdefault("cpu_baseline", None)
    return line


def copy_calibration():
    """A plain device-to-device copy of known size, run under the same HBM counters as the
    kernels: FETCH_SIZE / WRITE_SIZE per copy dispatch divided by 256 MiB gives each
    counter's scale."""
    import torch
    n = 64 << 20  # float32 elements: 256 MiB each way
    src = torch.randn(n, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps-scale", type=float, default=1.0,
                    help="studies: fraction of the paper's replication counts")
    ap.add_argument("--workload", default="plain_f32",
                    choices=["plain_f32", "small_f64", "precision_bf16", "batched", "serving",
                             "cross_f32", "cross_bf16", "studies", "timing", "hsic"])
    ap.add_argument("--timing-reps", type=int, default=20,
                    help="timing: replications per shape and test (standard test: half)")
    ap.add_argument("--timing-precs", default="f64,f32",
                    help="timing: comma-separated forms to time")
    ap.add_argument("--hsic-n", default="2000,4096",
                    help="hsic: comma-separated pair counts (the first one is the headline)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=20.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--capacity-requests", type=int, default=600,
                    help="serving: requests of the capacity comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to scale the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload in ("plain_f32", "small_f64", "precision_bf16"):
        line = run_single(args)
    elif args.workload == "batched":
        line = run_batched(args)
    elif args.workload.startswith("cross"):
        line = run_cross(args)
    elif args.workload == "studies":
        line = run_studies(args)
    elif args.workload == "timing":
        line = run_timing(args)
    elif args.workload == "hsic":
        line = run_hsic(args)
    else:
        line = run_serving(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
