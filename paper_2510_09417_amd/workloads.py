"""Seeded synthetic point sets.

This module only draws inputs; it holds none of the hull method's arithmetic, so
that the CPU oracle and the GPU library can be fed the same bits without
sharing code.

The four distributions stand in for the datasets of the paper's evaluation
(Section 5.2: Kuzmin, Circle and Disk, each of 10^8 points) plus the unit
square.  They are drawn here from their textbook definitions with NumPy's PCG64
generator; no file of the original benchmark suite is used or reproduced.

Recipe (every dataset gets a fresh ``numpy.random.default_rng(seed)``; two
uniform arrays ``U1 = g.random(n)`` then ``U2 = g.random(n)`` are drawn in that
order, float64 in [0, 1)):

  disk    r = sqrt(U1), theta = 2*pi*U2, (x, y) = (r cos theta, r sin theta)
  square  (x, y) = (U1, U2)
  circle  theta = 2*pi*U1, (x, y) = (cos theta, sin theta)   (U2 unused)
  kuzmin  r = sqrt(1/(1-U1)^2 - 1), theta = 2*pi*U2, polar as for disk

The served mix draws request sizes log-uniform in [16, 10^6], a distribution
per request and Poisson arrival gaps from ``default_rng(5)``, and the points of
request i from ``default_rng([5, i])``.
"""
from __future__ import annotations

import math

import numpy as np

DISTRIBUTIONS = ("disk", "square", "circle", "kuzmin")


def _polar(r: np.ndarray, u2: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    theta = u2
    theta *= 2.0 * math.pi
    x = np.cos(theta)
    y = np.sin(theta, out=theta)
    x *= r
    y *= r
    return x, y


def points(dist: str, n: int, seed) -> tuple[np.ndarray, np.ndarray]:
    """Return (x, y) float64 arrays of ``n`` points of distribution ``dist``."""
    g = np.random.default_rng(seed)
    u1 = g.random(n)
    u2 = g.random(n)
    if dist == "disk":
        r = np.sqrt(u1, out=u1)
        return _polar(r, u2)
    if dist == "square":
        return u1, u2
    if dist == "circle":
        theta = u1
        theta *= 2.0 * math.pi
        x = np.cos(theta)
        y = np.sin(theta, out=theta)
        return x, y
    if dist == "kuzmin":
        t = np.subtract(1.0, u1, out=u1)
        np.square(t, out=t)
        np.reciprocal(t, out=t)
        t -= 1.0
        r = np.sqrt(t, out=t)
        return _polar(r, u2)
    raise ValueError(f"unknown distribution {dist!r}")


# Named workloads at the sizes the evaluation uses.
WORKLOADS = {
    "disk_1e6": ("disk", 1_000_000, 1),
    "disk_1e8": ("disk", 100_000_000, 2),
    "square_1e8": ("square", 100_000_000, 2),
    "circle_5e7": ("circle", 50_000_000, 3),
    "kuzmin_1e8": ("kuzmin", 100_000_000, 4),
}


def workload(name: str, n: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Points of a named workload; ``n`` overrides the size (same seed)."""
    dist, n0, seed = WORKLOADS[name]
    return points(dist, n0 if n is None else n, seed)


def lattice(n: int, seed, lo: int = 0, hi: int = 7, dup_frac: float = 0.0,
            collinear_runs: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Integer-valued points in [lo, hi]^2 stored as float64.

    With |coordinates| < 2^25 every subtraction and product of the orientation
    formula is exact, so these inputs have an exactly defined hull.
    ``dup_frac`` of the points are copies of earlier ones and
    ``collinear_runs`` short runs of evenly spaced collinear points are mixed
    in (both at random positions).
    """
    g = np.random.default_rng(seed)
    x = g.integers(lo, hi + 1, size=n).astype(np.float64)
    y = g.integers(lo, hi + 1, size=n).astype(np.float64)
    for _ in range(collinear_runs):
        if n < 3:
            break
        k = int(g.integers(3, max(4, min(n, 12))))
        x0, y0 = g.integers(lo, hi + 1, size=2)
        dx, dy = g.integers(-2, 3, size=2)
        pos = g.choice(n, size=min(k, n), replace=False)
        steps = np.arange(len(pos))
        xs = np.clip(x0 + dx * steps, lo, hi)
        ys = np.clip(y0 + dy * steps, lo, hi)
        x[pos] = xs
        y[pos] = ys
    ndup = int(dup_frac * n)
    if ndup and n > 1:
        src = g.integers(0, n, size=ndup)
        dst = g.integers(0, n, size=ndup)
        x[dst] = x[src]
        y[dst] = y[src]
    return x, y


# ---------------------------------------------------------------- served mix
SERVED_SEED = 5
SERVED_REQUESTS = 65536
SERVED_MIN, SERVED_MAX = 16, 1_000_000


def served_plan(nreq: int = SERVED_REQUESTS, rate: float = 1.0, seed: int = SERVED_SEED):
    """Sizes, distributions and arrival times (seconds) of the served mix.

    Sizes are log-uniform in [16, 10^6]: floor(16 * 62500^U), clamped; the
    distribution index is floor(4U); arrival gaps are exponential with the
    given ``rate`` (requests per second).
    """
    g = np.random.default_rng(seed)
    us = g.random(nreq)
    ud = g.random(nreq)
    ua = g.random(nreq)
    sizes = np.clip(np.floor(SERVED_MIN * np.power(SERVED_MAX / SERVED_MIN, us)), SERVED_MIN, SERVED_MAX)
    dists = np.floor(4.0 * ud).astype(np.int64)
    gaps = -np.log1p(-ua) / rate
    return sizes.astype(np.int64), dists, np.cumsum(gaps)


def served_request(i: int, n: int, dist_index: int, seed: int = SERVED_SEED):
    """Points of request ``i`` of the served mix."""
    return points(DISTRIBUTIONS[dist_index], int(n), [seed, int(i)])


def device_points_into(dist: str, x, y, generator) -> None:
    """Fill the float64 GPU tensors x and y (same length) with points of
    ``dist`` drawn on the device from a seeded torch generator: the same
    formulas as ``points`` with the device's random numbers (used where host
    generation would take too long, e.g. the full served mix)."""
    import torch

    n = x.numel()
    if n == 0:
        return
    u1 = torch.rand(n, dtype=torch.float64, device=x.device, generator=generator)
    u2 = torch.rand(n, dtype=torch.float64, device=x.device, generator=generator)
    if dist == "square":
        x.copy_(u1)
        y.copy_(u2)
        return
    if dist == "circle":
        theta = u1.mul_(2.0 * math.pi)
        torch.cos(theta, out=x)
        torch.sin(theta, out=y)
        return
    if dist == "disk":
        r = u1.sqrt_()
    elif dist == "kuzmin":
        r = u1.neg_().add_(1.0).square_().reciprocal_().sub_(1.0).sqrt_()
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    theta = u2.mul_(2.0 * math.pi)
    torch.cos(theta, out=x)
    torch.sin(theta, out=y)
    x.mul_(r)
    y.mul_(r)
