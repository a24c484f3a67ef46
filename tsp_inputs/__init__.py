"""Seeded synthetic TSP instances.

This module is the one thing the HIP library's callers and the oracle's
callers share: it makes inputs and holds none of the Ant System arithmetic.
It draws city coordinates with numpy's PCG64 generator and turns them into the
integer distance matrix both sides consume.

The paper measures on TSPLIB instances (att48 ... pr2392) that are not
available here; these synthetic layouts stand in for them at the same sizes
(n = 100, 1000, 2400) with m = n ants.

* ``uniform_cities``   -- distinct integer points uniform in [0, side]^2.
* ``clustered_cities`` -- 20 Gaussian clusters, sigma = 2% of the side,
  centres uniform, points rounded and clamped to the square, distinct.
* ``euc2d``            -- d_ij = nint(sqrt(dx^2 + dy^2)) as int32 (the usual
  EUC_2D rounding of TSPLIB), symmetric with a zero diagonal.
"""
from __future__ import annotations

import numpy as np

__all__ = ["uniform_cities", "clustered_cities", "euc2d", "instance", "log_uniform_sizes",
           "poisson_arrivals"]


def _dedupe_fill(pts: np.ndarray, draw_more, n: int) -> np.ndarray:
    """Keep the first occurrence of every point; redraw until n are distinct."""
    out = []
    seen = set()
    for p in map(tuple, pts):
        if p not in seen:
            seen.add(p)
            out.append(p)
    while len(out) < n:
        for p in map(tuple, draw_more(n - len(out))):
            if p not in seen:
                seen.add(p)
                out.append(p)
    return np.asarray(out[:n], dtype=np.int64)


def uniform_cities(n: int, side: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x5EED_0001])
    draw = lambda k: rng.integers(0, side + 1, size=(k, 2), dtype=np.int64)  # noqa: E731
    return _dedupe_fill(draw(n), draw, n)


def clustered_cities(n: int, side: int, seed: int, clusters: int = 20,
                     sigma_frac: float = 0.02) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x5EED_0002])
    centres = rng.uniform(0.0, float(side), size=(clusters, 2))
    sigma = sigma_frac * side

    def draw(k):
        which = rng.integers(0, clusters, size=k)
        pts = centres[which] + rng.normal(0.0, sigma, size=(k, 2))
        return np.clip(np.rint(pts), 0, side).astype(np.int64)

    return _dedupe_fill(draw(n), draw, n)


def euc2d(coords: np.ndarray) -> np.ndarray:
    c = np.asarray(coords, dtype=np.int64)
    dx = c[:, None, 0] - c[None, :, 0]
    dy = c[:, None, 1] - c[None, :, 1]
    sq = (dx * dx + dy * dy).astype(np.float64)  # exact: < 2^53
    d = np.floor(np.sqrt(sq) + 0.5).astype(np.int64)
    if d.max(initial=0) >= 2**31:
        raise ValueError("distance does not fit int32")
    return d.astype(np.int32)


def instance(n: int, layout: str = "uniform", side: int = 1_000_000, seed: int = 1):
    """(coords, dist) for one seeded instance."""
    if layout == "uniform":
        xy = uniform_cities(n, side, seed)
    elif layout in ("cluster", "clustered"):
        xy = clustered_cities(n, side, seed)
    else:
        raise ValueError(f"unknown layout {layout!r}")
    return xy, euc2d(xy)


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Instance sizes round(exp(U(ln lo, ln hi))) for batched/served workloads."""
    rng = np.random.default_rng([seed, 0x5EED_0003])
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng([seed, 0x5EED_0004])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
