"""Seeded synthetic inputs shaped like the paper's Gaussian workloads.

This module draws data only; it holds none of the test's arithmetic.  It is
the one piece shared by the HIP path's callers and the oracle's callers.

The paper simulates every dataset from multivariate normals (Section 5.1:
N_p(0, I); Section 5.2: Y ~ N_p(mu_{eps,j}, I) with the first j coordinates
of the mean set to eps).  The workloads below follow that recipe.  Data are
drawn in float64 from numpy's PCG64 with a fixed seed (X first, then Y) and
rounded once to float32 for the float32 / bf16 precision forms, so the oracle
receives exactly the values the GPU receives.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def gaussian_pair(nx, ny, p, seed, mean_shift=None, var_scale=None, dtype=np.float32):
    """X ~ N(0, I_p) (nx rows), Y ~ N(mu, diag(s)) (ny rows).

    ``mean_shift``: None, a scalar (added to every coordinate of Y) or a length-p vector.
    ``var_scale``: None or a length-p vector of variances s (Y columns scaled by sqrt(s)).
    """
    g = np.random.Generator(np.random.PCG64(seed))
    X = g.standard_normal((nx, p))
    Y = g.standard_normal((ny, p))
    if var_scale is not None:
        Y = Y * np.sqrt(np.asarray(var_scale, dtype=np.float64))[None, :]
    if mean_shift is not None:
        Y = Y + np.asarray(mean_shift, dtype=np.float64)
    return X.astype(dtype), Y.astype(dtype)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    p: int
    B: int
    data_seed: int
    perm_seed: int
    prec: str                      # "f64" | "f32" | "bf16r"
    kinds: List[str] = field(default_factory=lambda: ["ed"])
    mean_shift: Optional[object] = None
    var_scale: Optional[object] = None

    def data(self):
        dt = np.float64 if self.prec == "f64" else np.float32
        return gaussian_pair(self.nx, self.ny, self.p, self.data_seed, self.mean_shift,
                             self.var_scale, dt)

    def gamma(self):
        """Gaussian-kernel bandwidth sigma^2 = p, i.e. gamma = 1/p."""
        return 1.0 / self.p


def small_null_f64():
    """100 x 10 vs 100 x 10, N(0,1) null case, FP64 end to end, B = 1000."""
    return Workload("ed_f64_100x10_B1000", 100, 100, 10, 1000, 0, 1, "f64")


def plain_f32():
    """2000 x 1000 vs 2000 x 1000; Y mean 0.05 on the first 50 coordinates; B = 10^4."""
    mu = np.zeros(1000)
    mu[:50] = 0.05
    return Workload("ed_f32_2000x1000_B10000", 2000, 2000, 1000, 10000, 0, 1, "f32",
                    mean_shift=mu)


def precision_bf16():
    """5000 x 4096 vs 4000 x 4096; Y variance 1.1 on the first 200 coordinates; B = 10^4.

    Both ED and Gaussian-kernel MMD (sigma^2 = p) are run on the same data.
    """
    s = np.ones(4096)
    s[:200] = 1.1
    return Workload("ed_mmd_bf16r_5000x4000x4096_B10000", 5000, 4000, 4096, 10000, 0, 1,
                    "bf16r", kinds=["ed", "mmd"], var_scale=s)


def batched_tests(count=256, B=2000):
    """Independent ED tests: nx, ny ~ U{50..1500}, p in {20, 100, 500},
    Y ~ N(delta * 1, I) with delta ~ U[0, 0.1]; parameters from rng(4)."""
    g = np.random.Generator(np.random.PCG64(4))
    out = []
    for t in range(count):
        nx = int(g.integers(50, 1501))
        ny = int(g.integers(50, 1501))
        p = int(g.choice([20, 100, 500]))
        delta = float(g.uniform(0.0, 0.1))
        out.append(Workload("batch%03d" % t, nx, ny, p, B, 10000 + t, 20000 + t, "f32",
                            mean_shift=delta))
    return out


def device_pair(nx, ny, p, seed, mean_shift=0.0, device="cuda:0"):
    """X ~ N(0, I_p) (nx rows), Y ~ N(mean_shift * 1, I_p) (ny rows) as float32 device
    tensors, drawn by torch's device generator seeded with `seed` (X first, then Y).  Used
    where host generation would not keep up (a request stream); the values are copied back
    to the host when the oracle checks a result."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    X = torch.randn((nx, p), generator=g, device=device, dtype=torch.float32)
    Y = torch.randn((ny, p), generator=g, device=device, dtype=torch.float32)
    if mean_shift:
        Y += float(mean_shift)
    return X, Y


def serving_stream(rate=200.0, duration=60.0, seed=5):
    """Poisson arrivals; per request nx, ny, p log-uniform, B in {1000, 10000},
    ED or MMD 50/50, Y shifted by delta ~ U[0, 0.1] on every coordinate."""
    g = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    r = 0
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration:
            break
        nx = int(np.clip(round(float(np.exp(g.uniform(np.log(100), np.log(20000))))), 100, 20000))
        ny = int(np.clip(round(float(np.exp(g.uniform(np.log(100), np.log(20000))))), 100, 20000))
        p = int(np.clip(round(float(np.exp(g.uniform(np.log(10), np.log(2000))))), 10, 2000))
        B = int(g.choice([1000, 10000]))
        kind = "ed" if g.uniform() < 0.5 else "mmd"
        delta = float(g.uniform(0.0, 0.1))
        w = Workload("req%05d" % r, nx, ny, p, B, 100000 + r, 200000 + r, "bf16r", kinds=[kind],
                     mean_shift=delta)
        reqs.append((t, w))
        r += 1
    return reqs
