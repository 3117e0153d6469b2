"""The seeded input generators (host only): the served mix's arrival replay is
deterministic and follows its stated laws, and every point distribution draws
what its recipe says (the same bits for the same seed, the stated support)."""
import math

import numpy as np
import pytest

from paper_2510_09417_amd import workloads


def test_served_replay_is_deterministic():
    a = workloads.served_plan(4096, rate=1000.0, seed=5)
    b = workloads.served_plan(4096, rate=1000.0, seed=5)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    c = workloads.served_plan(4096, rate=1000.0, seed=6)
    assert not np.array_equal(a[0], c[0])
    # a prefix of the plan does not depend on how many requests are drawn
    assert np.array_equal(workloads.served_plan(100, seed=5)[0], workloads.served_plan(4096, seed=5)[0][:100])


def test_served_plan_laws():
    sizes, dists, arrivals = workloads.served_plan(1 << 16, rate=2000.0, seed=5)
    assert sizes.min() >= workloads.SERVED_MIN and sizes.max() <= workloads.SERVED_MAX
    # log-uniform: log(size / 16) / log(62500) is uniform on [0, 1) (up to the floor)
    u = np.log(sizes / 16.0) / math.log(workloads.SERVED_MAX / workloads.SERVED_MIN)
    assert abs(u.mean() - 0.5) < 0.01 and abs(np.median(u) - 0.5) < 0.01
    assert set(np.unique(dists)) == {0, 1, 2, 3}
    assert np.all(np.abs(np.bincount(dists) / len(dists) - 0.25) < 0.01)
    gaps = np.diff(np.concatenate([[0.0], arrivals]))
    assert np.all(gaps >= 0) and abs(gaps.mean() * 2000.0 - 1.0) < 0.02  # exponential, mean 1/rate


def test_served_request_points_are_seeded_per_request():
    x1, y1 = workloads.served_request(7, 1000, 0)
    x2, y2 = workloads.served_request(7, 1000, 0)
    x3, _ = workloads.served_request(8, 1000, 0)
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2) and not np.array_equal(x1, x3)


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_points_support_and_determinism(dist):
    x, y = workloads.points(dist, 200_000, seed=9)
    x2, y2 = workloads.points(dist, 200_000, seed=9)
    assert np.array_equal(x, x2) and np.array_equal(y, y2)
    assert x.dtype == np.float64 and len(x) == len(y) == 200_000 and np.isfinite(x).all() and np.isfinite(y).all()
    r = np.hypot(x, y)
    if dist == "disk":
        assert r.max() <= 1.0 + 1e-15
        assert abs((r <= 0.5).mean() - 0.25) < 0.01  # uniform in area
    elif dist == "square":
        assert x.min() >= 0 and x.max() < 1 and y.min() >= 0 and y.max() < 1
    elif dist == "circle":
        assert np.all(np.abs(r - 1.0) < 1e-15)
    else:  # Kuzmin: P(radius <= s) = 1 - 1 / sqrt(1 + s^2)
        for s in (0.5, 1.0, 3.0):
            assert abs((r <= s).mean() - (1.0 - 1.0 / math.sqrt(1.0 + s * s))) < 0.01


def test_lattice_has_requested_structure():
    x, y = workloads.lattice(5000, seed=3, lo=-4, hi=4, dup_frac=0.3, collinear_runs=2)
    assert np.all(x == np.round(x)) and np.all(y == np.round(y))
    assert x.min() >= -4 and x.max() <= 4 and y.min() >= -4 and y.max() <= 4
    pts = set(zip(x.tolist(), y.tolist()))
    assert len(pts) < len(x)  # duplicates present
