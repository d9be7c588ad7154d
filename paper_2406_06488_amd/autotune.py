"""Autotuner for the resampling stage's work shape.

For each bucket of pooled sample sizes n = nx + ny the tuner times the resampling stage
(HIP events inside the library) of a representative test under every candidate shape --
kc column tiles of 128 items and cc chunks of 256 splits per workgroup -- and keeps the
fastest.  The winning rules are installed with etest_tune_set and can be saved to /
loaded from a JSON file.
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
    """rules: list of dicts(prec, n_lo, n_hi, kc, cc)."""
    L = _lib.load()
    check(L.etest_tune_clear())
    for r in rules:
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
