"""Seeded synthetic inputs for R-tree range select and spatial join.

This module only draws rectangles, query windows and arrival times.  It
contains none of the method's arithmetic (no overlap test, no tree build, no
traversal), so the CPU oracle and the GPU library can both be fed from it
without sharing any computation.

Conventions (the paper evaluates on synthetic uniform 2D data, section 5;
the larger workloads below add clustered data and log-uniform selectivity):

* Every generator takes an explicit integer seed and uses
  ``numpy.random.Generator(PCG64(seed))``.
* Draws are float64 and are cast once to float32 (round to nearest even).
  The high corner is ``f32(lo64 + side64)``; rounding is monotone, so
  ``lx <= hx`` and ``ly <= hy`` always hold.
* Rectangles are ``float32[n, 4]`` rows ``(low_x, low_y, high_x, high_y)``,
  the MBR order of an R-tree entry (section 2.3).  Object ID = row index.
* Selectivity of a square window is its area (side = sqrt(sel)).
* Nonzero magnitudes below 2**-126 are flushed to 0 and counted, so no
  subnormal coordinates appear unless a test builds them on purpose.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32_TINY = np.float32(2.0 ** -126)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _finish(lo_x, lo_y, w, h) -> np.ndarray:
    """Assemble float32 rectangles from float64 low corners and sides."""
    out = np.empty((lo_x.shape[0], 4), dtype=np.float32)
    out[:, 0] = lo_x.astype(np.float32)
    out[:, 1] = lo_y.astype(np.float32)
    out[:, 2] = (lo_x + w).astype(np.float32)
    out[:, 3] = (lo_y + h).astype(np.float32)
    flush_subnormals(out)
    return out


def flush_subnormals(a: np.ndarray) -> int:
    """Map nonzero |v| < 2**-126 to +0 in place; return how many were hit."""
    sub = (a != 0) & (np.abs(a) < F32_TINY)
    k = int(sub.sum())
    if k:
        a[sub] = np.float32(0.0)
    return k


def uniform_rects(n: int, side_max: float, seed: int) -> np.ndarray:
    """Low corner ~ U[0,1)^2, width and height ~ U[0, side_max] independently."""
    g = rng(seed)
    lo = g.random((2, n))
    wh = g.random((2, n)) * side_max
    return _finish(lo[0], lo[1], wh[0], wh[1])


def clustered_rects(n: int, k: int, sigma: float, side_max: float, seed: int) -> np.ndarray:
    """k Gaussian clusters: centers ~ U[0,1)^2 drawn first, then each rectangle
    picks a cluster uniformly and offsets its low corner by N(0, sigma^2) per
    axis (not clipped to the unit square)."""
    g = rng(seed)
    centers = g.random((k, 2))
    c = g.integers(0, k, size=n)
    off = g.normal(0.0, sigma, size=(2, n))
    wh = g.random((2, n)) * side_max
    return _finish(centers[c, 0] + off[0], centers[c, 1] + off[1], wh[0], wh[1])


def permute(rects: np.ndarray, seed: int) -> np.ndarray:
    """Seeded row permutation, so object IDs are spatially uncorrelated."""
    g = rng(seed)
    return rects[g.permutation(rects.shape[0])]


def windows_fixed(nq: int, side: float, seed: int) -> np.ndarray:
    """Square windows of a fixed side, centers ~ U[0,1)^2."""
    g = rng(seed)
    c = g.random((2, nq))
    half = side / 2.0
    s = np.full(nq, side)
    return _finish(c[0] - half, c[1] - half, s, s)


def windows_loguniform(nq: int, sel_lo: float, sel_hi: float, seed: int) -> np.ndarray:
    """Square windows, centers ~ U[0,1)^2, area ~ LogUniform[sel_lo, sel_hi]."""
    g = rng(seed)
    c = g.random((2, nq))
    sel = np.exp(g.uniform(math.log(sel_lo), math.log(sel_hi), size=nq))
    side = np.sqrt(sel)
    return _finish(c[0] - side / 2.0, c[1] - side / 2.0, side, side)


def loguniform_ints(m: int, lo: float, hi: float, seed: int) -> np.ndarray:
    g = rng(seed)
    return np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=m))).astype(np.int64)


# ---------------------------------------------------------------------------
# Adversarial small inputs: coordinates snapped to a coarse grid so that edges
# and corners touch exactly, plus degenerate (point and segment) rectangles,
# duplicates, coordinates outside [0,1] and infinite windows.
# ---------------------------------------------------------------------------

def adversarial_rects(n: int, seed: int, grid: int = 8) -> np.ndarray:
    g = rng(seed)
    lo = g.integers(-2, grid + 2, size=(n, 2)).astype(np.float64) / grid
    wh = g.integers(0, 3, size=(n, 2)).astype(np.float64) / grid
    kind = g.integers(0, 10, size=n)
    wh[kind == 0] = 0.0                       # points
    wh[kind == 1, 0] = 0.0                    # vertical segments
    wh[kind == 2, 1] = 0.0                    # horizontal segments
    out = _finish(lo[:, 0], lo[:, 1], wh[:, 0], wh[:, 1])
    if n >= 4:                                # exact duplicates
        d = g.integers(0, n, size=max(1, n // 10))
        out[d] = out[d[0]]
    return out


def adversarial_windows(nq: int, seed: int, grid: int = 8) -> np.ndarray:
    out = adversarial_rects(nq, seed, grid)
    g = rng(seed + 7)
    inf = np.float32(np.inf)
    for i in range(nq):
        r = g.integers(0, 12)
        if r == 0:
            out[i] = (-inf, -inf, inf, inf)        # select all
        elif r == 1:
            out[i, 0] = -inf                        # half-infinite
        elif r == 2:
            out[i, 3] = inf
    return out


# ---------------------------------------------------------------------------
# Named workloads (sizes from the evaluation configurations the benchmark and
# the parity tests use).  Seeds: data 1000*k + 1, queries 1000*k + 2.
# ---------------------------------------------------------------------------

@dataclass
class SelectWorkload:
    name: str
    rects: np.ndarray
    queries: np.ndarray
    fanout: int
    layout: str


def c1_plain(seed_base: int = 1000) -> SelectWorkload:
    """100k uniform rectangles (sides U[0,1e-3]), fanout 16 SoA, 1000 windows of
    side sqrt(1e-4)."""
    r = uniform_rects(100_000, 1e-3, seed_base + 1)
    q = windows_fixed(1000, math.sqrt(1e-4), seed_base + 2)
    return SelectWorkload("select_uniform_100k_q1k_f16_soa", r, q, 16, "soa")


def c2_rects(n: int = 10_000_000, seed_base: int = 2000) -> np.ndarray:
    """Half uniform, half in 64 Gaussian clusters (sigma 0.01), sides U[0,1e-4],
    concatenated then permuted."""
    h = n // 2
    a = uniform_rects(h, 1e-4, seed_base + 1)
    b = clustered_rects(n - h, 64, 0.01, 1e-4, seed_base + 3)
    return permute(np.concatenate([a, b]), seed_base + 5)


def c2_queries(nq: int = 1_000_000, seed_base: int = 2000) -> np.ndarray:
    return windows_loguniform(nq, 1e-6, 1e-3, seed_base + 2)


def c3_join(n: int = 2_000_000, seed_base: int = 3000):
    """A: uniform, B: 32 Gaussian clusters (sigma 0.02); sides U[0,5e-4]."""
    a = uniform_rects(n, 5e-4, seed_base + 1)
    b = clustered_rects(n, 32, 0.02, 5e-4, seed_base + 3)
    return a, b


@dataclass
class BatchInstance:
    rects: np.ndarray
    queries: np.ndarray
    clustered: bool


def c4_batch(ntrees: int = 256, n_lo: float = 1e3, n_hi: float = 1e6,
             q_lo: float = 100, q_hi: float = 1e5, seed_base: int = 4000,
             scale: float = 1.0) -> list:
    """Independent instances: sizes LogU[n_lo,n_hi], uniform or clustered
    (64 clusters, sigma 0.01) by a seeded coin, sides U[0,1e-4]; each with
    LogU[q_lo,q_hi] windows of selectivity LogU[1e-6,1e-2].  ``scale`` shrinks
    both sizes for small test runs."""
    sizes = loguniform_ints(ntrees, n_lo, n_hi, seed_base + 997)
    nqs = loguniform_ints(ntrees, q_lo, q_hi, seed_base + 998)
    coin = rng(seed_base + 999).integers(0, 2, size=ntrees)
    out = []
    for t in range(ntrees):
        n = max(1, int(sizes[t] * scale))
        nq = max(1, int(nqs[t] * scale))
        ds = seed_base + 2 * t
        if coin[t]:
            r = clustered_rects(n, 64, 0.01, 1e-4, ds)
        else:
            r = uniform_rects(n, 1e-4, ds)
        q = windows_loguniform(nq, 1e-6, 1e-2, ds + 1)
        out.append(BatchInstance(r, q, bool(coin[t])))
    return out


def c5_trees(n_big: int = 50_000_000, n_join: int = 5_000_000, seed_base: int = 5000):
    """Resident serving trees: 256 Gaussian clusters (sigma 0.005) with sides
    U[0,5e-5], plus a uniform tree with sides U[0,5e-5] for join requests."""
    big = clustered_rects(n_big, 256, 0.005, 5e-5, seed_base + 1)
    jt = uniform_rects(n_join, 5e-5, seed_base + 2)
    return big, jt


@dataclass
class Request:
    t_arrival: float          # seconds from stream start
    kind: str                 # "select" or "join"
    payload: np.ndarray       # window (1x4) or probe rectangles (m x 4)
    rid: int = 0
    meta: dict = field(default_factory=dict)


def c5_requests(nreq: int, rate: float, seed_base: int = 5000, join_frac: float = 0.01,
                probe_n: int = 10_000, sel_lo: float = 1e-7, sel_hi: float = 1e-2) -> list:
    """Open-loop Poisson arrivals at ``rate`` requests/s; a ``join_frac``
    share are joins of a uniform probe set (sides U[0,5e-5]) against the join
    tree, the rest single windows with selectivity LogU[sel_lo, sel_hi]."""
    g = rng(seed_base + 3)
    gaps = g.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps)
    is_join = g.random(nreq) < join_frac
    wins = windows_loguniform(nreq, sel_lo, sel_hi, seed_base + 6)
    reqs = []
    for i in range(nreq):
        if is_join[i]:
            p = uniform_rects(probe_n, 5e-5, seed_base + 4 + 10 * i)
            reqs.append(Request(float(t[i]), "join", p, i))
        else:
            reqs.append(Request(float(t[i]), "select", wins[i:i + 1], i))
    return reqs
