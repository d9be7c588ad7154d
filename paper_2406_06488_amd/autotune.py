"""Autotuner for the work shapes of the Gram and resampling stages.

For each bucket of pooled sample sizes n = nx + ny the tuner times, with HIP events inside
the library, a representative test under every candidate shape and keeps the fastest
(tune), or times the whole batch the rules will serve (tune_batch: in a batch the tests
fill the chip together, so shapes that spread one small test over many workgroups lose to
longer row units):
  resampling: kc column tiles of 128 items and cc chunks of 256 splits per workgroup
              (etest_tune_set);
  Gram:       one 128 x 128 block tile or one 256 x 256 super tile per workgroup
              (etest_tune_set_gram).
The winning rules can be saved to / loaded from a JSON file (install() takes both kinds).
"""
import json

from . import _lib, api
from ._lib import check

PRECS = {"f64": 0, "f32": 1, "bf16r": 2}
MFMA_CANDIDATES = [(kc, cc) for kc in (2, 4, 8, 16, 32) for cc in (1, 2)]
F64_CANDIDATES = [(kc, cc) for kc in (2, 4, 8) for cc in (1, 4, 8)]


def clear():
    check(_lib.load().etest_tune_clear())


def install(rules):
    """rules: list of dicts(prec, n_lo, n_hi, kc, cc) (resampling) or dicts(prec, n_lo,
    n_hi, gram_shape) (Gram: 0 = block tiles, 1 = super tiles)."""
    L = _lib.load()
    check(L.etest_tune_clear())
    for r in rules:
        if "gram_shape" in r:
            check(L.etest_tune_set_gram(PRECS[r["prec"]], r["n_lo"], r["n_hi"], r["gram_shape"]))
        else:
            check(L.etest_tune_set(PRECS[r["prec"]], r["n_lo"], r["n_hi"], r["kc"], r["cc"]))


def save(rules, path):
    with open(path, "w") as f:
        json.dump(rules, f, indent=1)


def load(path):
    with open(path) as f:
        rules = json.load(f)
    install(rules)
    return rules


def _time_resampling(X, Y, B, kind, prec, gamma, reps):
    api.run(X, Y, B, 1, kind, prec, gamma, with_perm_stats=False)  # warm-up
    api.profile_enable(True)
    for _ in range(reps):
        api.run(X, Y, B, 1, kind, prec, gamma, with_perm_stats=False)
    ms, cnt = api.profile_read()["resampling"]
    api.profile_enable(False)
    return ms / max(cnt, 1)


def tune(buckets, reps=3, log=None):
    """buckets: list of dicts(prec, n_lo, n_hi, X, Y, B, kind, gamma) where X, Y are device
    tensors of a representative test.  Returns the chosen rules (and installs them)."""
    L = _lib.load()
    rules = []
    for b in buckets:
        cands = F64_CANDIDATES if b["prec"] == "f64" else MFMA_CANDIDATES
        best = None
        for kc, cc in cands:
            check(L.etest_tune_clear())
            check(L.etest_tune_set(PRECS[b["prec"]], b["n_lo"], b["n_hi"], kc, cc))
            t = _time_resampling(b["X"], b["Y"], b["B"], b.get("kind", "ed"), b["prec"],
                                 b.get("gamma", 0.0), reps)
            if log:
                log("tune %s n[%d,%d) kc=%d cc=%d: %.4f ms" % (b["prec"], b["n_lo"], b["n_hi"],
                                                               kc, cc, t))
            if best is None or t < best[0]:
                best = (t, kc, cc)
        rules.append({"prec": b["prec"], "n_lo": b["n_lo"], "n_hi": b["n_hi"], "kc": best[1],
                      "cc": best[2], "ms": best[0]})
    install(rules)
    return rules


def _time_blocks(X, Y, kind, prec, gamma, reps):
    api.run(X, Y, 0, 1, kind, prec, gamma, with_perm_stats=False)  # warm-up
    api.profile_enable(True, ["blocks"])
    for _ in range(reps):
        api.run(X, Y, 0, 1, kind, prec, gamma, with_perm_stats=False)
    ms, cnt = api.profile_read()["blocks"]
    api.profile_enable(False)
    return ms / max(cnt, 1)


def tune_gram(buckets, reps=3, log=None, keep=()):
    """buckets: list of dicts(prec, n_lo, n_hi, X, Y, kind, gamma) of representative tests
    (FP32 or BF16-refined).  Times the block stage under both Gram workgroup shapes and
    installs the faster per bucket, together with the rules in `keep`.  Returns the rules."""
    L = _lib.load()
    rules = []
    for b in buckets:
        best = None
        for shape in (0, 1):
            install(list(keep) + [{"prec": b["prec"], "n_lo": b["n_lo"], "n_hi": b["n_hi"],
                                   "gram_shape": shape}])
            t = _time_blocks(b["X"], b["Y"], b.get("kind", "ed"), b["prec"], b.get("gamma", 0.0),
                             reps)
            if log:
                log("tune gram %s n[%d,%d) shape=%d: %.4f ms" % (b["prec"], b["n_lo"], b["n_hi"],
                                                               shape, t))
            if best is None or t < best[0]:
                best = (t, shape)
        rules.append({"prec": b["prec"], "n_lo": b["n_lo"], "n_hi": b["n_hi"],
                      "gram_shape": best[1], "ms": best[0]})
    check(L.etest_tune_clear())
    install(list(keep) + rules)
    return rules


def tune_batch(run_batch, ranges, prec="f32", reps=5, log=None):
    """Resampling shapes tuned on the batch they serve.  run_batch(): one synchronous pass of
    the batch (e.g. lambda: api.batch(reqs)); ranges: the buckets [(n_lo, n_hi), ...].
    First one shape for every bucket, then each bucket in turn with the others fixed
    (coordinate descent), every candidate timed on the whole batch.  Returns the chosen
    rules (and installs them)."""
    import time

    import torch
    cands = F64_CANDIDATES if prec == "f64" else MFMA_CANDIDATES

    def rules_of(shapes):
        return [{"prec": prec, "n_lo": lo, "n_hi": hi, "kc": kc, "cc": cc}
                for (lo, hi), (kc, cc) in zip(ranges, shapes)]

    def timed(shapes):
        install(rules_of(shapes))
        run_batch()  # warm-up (captures the batch's graph under these rules)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            run_batch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / reps
        if log:
            log("tune batch %s: %.4f ms" % (shapes, ms))
        return ms

    best_ms, best = min((timed([c] * len(ranges)), [c] * len(ranges)) for c in cands)
    for i in range(len(ranges)):
        for c in cands:
            if c == best[i]:
                continue
            trial = best[:i] + [c] + best[i + 1:]
            ms = timed(trial)
            if ms < best_ms:
                best_ms, best = ms, trial
    rules = rules_of(best)
    install(rules)
    for r in rules:
        r["ms"] = best_ms
    return rules
