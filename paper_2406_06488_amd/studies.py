"""Statistical studies of the paper's Section 5.2 on the GPU path.

Null study: under X, Y ~ N(0, I_p) the p-values of a valid test are uniform; the paper
shows this for the efficient permutation ED test and the cross-ED test at n = 200 with
p = 100 and p = 1000 (read as nx = ny = 200, the notation of its power settings).  Power study: X ~ N(0, I_p), Y ~ N(mu, I_p) with the first j
coordinates of mu equal to eps, empirical power at level 0.05 of both tests over three
settings (n growing at p = 50, j = 5, eps = 0.25; p growing at n = 200 with j = 50 or
j = p/10, eps = 0.1), 200 permutations.

The efficient test runs through the batched entry point (many replications per launch),
the cross test through etest_cross.  Data are drawn on the device from a seeded torch
generator (plain synthetic inputs, no part of the method); split seeds are the
replication numbers.  Each power estimate carries the spread the paper draws around its
power curves: one bootstrap standard deviation of the estimate from 200 resamples of the
replications.
"""
import numpy as np

from . import api

SETTING_1 = {"ns": list(range(60, 361, 20)), "p": 50, "j": 5, "eps": 0.25}
SETTING_2 = {"n": 200, "ps": list(range(200, 2001, 100)), "j": 50, "eps": 0.1}
SETTING_3 = {"n": 200, "ps": list(range(200, 2001, 100)), "j_frac": 0.1, "eps": 0.1}


def _draw(g, nx, ny, p, j, eps, device):
    import torch
    X = torch.randn(nx, p, generator=g, device=device)
    Y = torch.randn(ny, p, generator=g, device=device)
    if j > 0 and eps != 0.0:
        Y[:, :j] += eps
    return X.contiguous(), Y.contiguous()


def split_seed(seed, r):
    """Split-stream seed of replication r of a study seeded with `seed`."""
    return seed * 1000003 + r


def pvalues(nx, ny, p, reps, j=0, eps=0.0, B=200, seed=0, prec="f32", chunk=256,
            device="cuda:0", keep=0, detail=False):
    """p-values of the efficient permutation ED test and of the cross-ED test on `reps`
    replications (same data for both).  keep: also return the first `keep` replications'
    data as host arrays (X, Y, split seed) for an independent check.  detail: return the
    efficient test's full results (count, threshold, ...) instead of its p-values."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    eff, cross, kept = [], [], []
    for start in range(0, reps, chunk):
        pairs = [_draw(g, nx, ny, p, j, eps, device) for _ in range(min(chunk, reps - start))]
        reqs = [api.make_request(X, Y, B, split_seed(seed, start + r), "ed", prec)
                for r, (X, Y) in enumerate(pairs)]
        res = api.batch(reqs)
        eff += res if detail else [o["p_value"] for o in res]
        cross += [api.cross(X, Y, "ed", prec)["p_value"] for X, Y in pairs]
        for r, (X, Y) in enumerate(pairs):
            if start + r < keep:
                kept.append((X.cpu().numpy(), Y.cpu().numpy(), split_seed(seed, start + r)))
    out = (eff if detail else np.array(eff)), np.array(cross)
    return out + (kept,) if keep else out


def bootstrap_sd(hits, nboot=200, seed=0):
    """Standard deviation of the mean of `hits` (one 0/1 outcome per replication) over
    `nboot` bootstrap resamples of the replications (Efron and Tibshirani, 1993)."""
    hits = np.asarray(hits, dtype=np.float64)
    g = np.random.Generator(np.random.PCG64(seed))
    idx = g.integers(0, len(hits), size=(nboot, len(hits)))
    return float(np.std(hits[idx].mean(axis=1), ddof=1))


def null_study(reps=2000, n=200, ps=(100, 1000), B=200, seed=1):
    """Type-I error at 0.05 and the Kolmogorov-Smirnov distance to uniform, per p."""
    from scipy.stats import kstest
    out = []
    for p in ps:
        e, c = pvalues(n, n, p, reps, B=B, seed=seed + p)
        out.append({"n": n, "p": p, "reps": reps,
                    "efficient": {"reject_0.05": float(np.mean(e <= 0.05)),
                                  "ks_pvalue": float(kstest(e, "uniform").pvalue)},
                    "cross": {"reject_0.05": float(np.mean(c <= 0.05)),
                              "ks_pvalue": float(kstest(c, "uniform").pvalue)}})
    return out


def power_study(setting, reps=500, B=200, seed=2, alpha=0.05, nboot=200):
    """Empirical power of both tests along one of the paper's three settings, each with one
    bootstrap standard deviation (nboot resamples of the replications)."""
    pts = []
    if "ns" in setting:
        grid = [(n, setting["p"], setting["j"]) for n in setting["ns"]]
    else:
        grid = [(setting["n"], p, setting.get("j") or max(1, int(round(setting["j_frac"] * p))))
                for p in setting["ps"]]
    for k, (n, p, j) in enumerate(grid):
        e, c = pvalues(n, n, p, reps, j=j, eps=setting["eps"], B=B, seed=seed * 1000 + k)
        pts.append({"n": n, "p": p, "j": j, "reps": reps,
                    "efficient": float(np.mean(e <= alpha)), "cross": float(np.mean(c <= alpha)),
                    "efficient_sd": bootstrap_sd(e <= alpha, nboot, seed * 1000 + k),
                    "cross_sd": bootstrap_sd(c <= alpha, nboot, seed * 1000 + k + 1)})
    return pts
