"""Brute-force checkers for tiny inputs (TEST INFRASTRUCTURE ONLY).

Written independently of ``oracle.c`` so that the two can pin each other:

* ``standard_test_stats``  -- Alg. 4 (standard permutation test): for every
  split, build x* and y* from the pooled rows and recompute all three
  distance matrices on them (Alg. 3), then eq. (1)/(2).
* ``precomputed_test_stats`` -- Alg. 5 (pre-computation strategy): one pooled
  matrix D_WW, sub-blocks extracted per split.  (Both are the paper's
  baselines, used here only as references.)
* ``all_splits`` -- every nx-subset of the pooled items, for exact
  enumeration of the permutation distribution.
* ``philox4x32_10`` / ``membership`` -- a second, pure-Python implementation of
  the split stream (Philox4x32-10 of Salmon et al., SC'11, driving selection
  sampling, Knuth TAOCP vol. 2, 3.4.2, Algorithm S).

All sums use ``math.fsum`` (exactly rounded).
"""
import itertools
import math

import numpy as np


def _dist(a, b, kind, gamma):
    s = math.fsum(float(u - v) ** 2 for u, v in zip(a, b))
    return math.sqrt(s) if kind == 0 else math.exp(-gamma * s)


def _matrix(A, B, kind, gamma):
    return [[_dist(a, b, kind, gamma) for b in B] for a in A]


def _stat_from_matrices(Mxx, Myy, Mxy, nx, ny, kind):
    sxx = math.fsum(v for row in Mxx for v in row)
    syy = math.fsum(v for row in Myy for v in row)
    sxy = math.fsum(v for row in Mxy for v in row)
    txy = 2.0 * sxy / (nx * ny)
    txx = sxx / (nx * nx)
    tyy = syy / (ny * ny)
    if kind == 0:
        return math.fsum([txy, -txx, -tyy])
    return math.fsum([txx, tyy, -txy])


def statistic(X, Y, kind=0, gamma=1.0):
    """eq. (1) / eq. (2) computed directly on the data."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    return _stat_from_matrices(_matrix(X, X, kind, gamma), _matrix(Y, Y, kind, gamma),
                               _matrix(X, Y, kind, gamma), len(X), len(Y), kind)


def standard_test_stats(X, Y, splits, kind=0, gamma=1.0):
    """Alg. 4: statistic recomputed from scratch on each split's (x*, y*).

    ``splits`` is a list of 0/1 vectors over the pooled items (1 = goes to x*).
    """
    W = np.concatenate([np.asarray(X, np.float64), np.asarray(Y, np.float64)], axis=0)
    out = []
    for z in splits:
        z = np.asarray(z).astype(bool)
        out.append(statistic(W[z], W[~z], kind, gamma))
    return out


def precomputed_test_stats(X, Y, splits, kind=0, gamma=1.0):
    """Alg. 5: the pooled matrix D_WW once, then sub-blocks per split."""
    W = np.concatenate([np.asarray(X, np.float64), np.asarray(Y, np.float64)], axis=0)
    Dww = _matrix(W, W, kind, gamma)
    nx = len(X)
    ny = len(Y)
    out = []
    for z in splits:
        ix = [i for i in range(len(W)) if z[i]]
        iy = [i for i in range(len(W)) if not z[i]]
        Mxx = [[Dww[a][b] for b in ix] for a in ix]
        Myy = [[Dww[a][b] for b in iy] for a in iy]
        Mxy = [[Dww[a][b] for b in iy] for a in ix]
        out.append(_stat_from_matrices(Mxx, Myy, Mxy, nx, ny, kind))
    return out


def all_splits(nx, ny):
    """Every split of the n = nx + ny pooled items into x* (size nx) and y*."""
    n = nx + ny
    for comb in itertools.combinations(range(n), nx):
        z = np.zeros(n, dtype=np.uint8)
        z[list(comb)] = 1
        yield z


# --- independent split stream ---------------------------------------------

_MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    c = [int(v) & _MASK for v in counter]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for _ in range(10):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c[3] ^ k1) & _MASK,
             p0 & _MASK]
        k0 = (k0 + 0x9E3779B9) & _MASK
        k1 = (k1 + 0xBB67AE85) & _MASK
    return c


def membership(nx, ny, seed, b):
    """Split b: item t kept with probability need/(n-t), decided exactly in integers."""
    n = nx + ny
    key = (seed & _MASK, (seed >> 32) & _MASK)
    need = nx
    z = np.zeros(n, dtype=np.uint8)
    words = None
    for t in range(n):
        if t % 2 == 0:
            words = philox4x32_10((t // 2, b & _MASK, (b >> 32) & _MASK, 0), key)
        u = (words[1] << 32 | words[0]) if t % 2 == 0 else (words[3] << 32 | words[2])
        take = 1 if (u * (n - t)) >> 64 < need else 0
        z[t] = take
        need -= take
    return z
