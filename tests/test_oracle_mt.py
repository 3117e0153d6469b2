"""The multithreaded oracle (the all-core CPU baseline) against references.

Its lists must equal the exact references where those apply (brute force and
Andrew's monotone chain on lattices) and the single-threaded oracle's
everywhere (the same steps: chunked scans combined in chunk order, the two
recursive calls of each step as tasks joined in Algorithm 1's order), for any
thread count and chunk size.  Small chunk sizes put even tiny inputs through
every parallel code path (chunked extremes, chunked partitions, tasks).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "known_hulls.json")
SETTINGS = [(1, 1), (2, 2), (3, 7), (8, 64), (8, 0)]


def _known():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _known(), ids=lambda c: c["name"])
def test_known_hulls_any_threads(case, oracle_lib):
    x = np.array(case["x"], dtype=np.float64)
    y = np.array(case["y"], dtype=np.float64)
    for th, grain in SETTINGS:
        assert oracle.hull_mt(x, y, th, grain, lib=oracle_lib).tolist() == case["hull"], (th, grain)


def test_brute_force_lattices_any_threads(oracle_lib):
    for seed in range(300):
        n = 3 + seed % 90
        x, y = workloads.lattice(n, seed=[41, seed], hi=5 + seed % 9, dup_frac=0.2, collinear_runs=2)
        want = pins.brute_force_hull(x, y)
        th, grain = SETTINGS[seed % len(SETTINGS)]
        assert oracle.hull_mt(x, y, th, grain, lib=oracle_lib).tolist() == want, (seed, th, grain)


@pytest.mark.parametrize("n,hi", [(20_000, 300), (200_000, 3000)])
def test_andrew_lattices_any_threads(n, hi, oracle_lib):
    x, y = workloads.lattice(n, seed=[42, n], hi=hi, dup_frac=0.05, collinear_runs=20)
    want = pins.andrew_hull(x, y)
    for th, grain in SETTINGS[2:]:
        assert oracle.hull_mt(x, y, th, grain, lib=oracle_lib).tolist() == want, (th, grain)


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_float_inputs_equal_single_thread(dist, oracle_lib):
    x, y = workloads.points(dist, 300_000, seed=43)
    want = oracle.hull(x, y, lib=oracle_lib)
    for th, grain in SETTINGS[1:]:
        assert np.array_equal(oracle.hull_mt(x, y, th, grain, lib=oracle_lib), want), (th, grain)


def test_degenerate_and_nonfinite(oracle_lib):
    for th, grain in SETTINGS:
        assert oracle.hull_mt(np.zeros(0), np.zeros(0), th, grain, lib=oracle_lib).tolist() == []
        assert oracle.hull_mt(np.full(50, 2.0), np.full(50, -1.0), th, grain, lib=oracle_lib).tolist() == [0]
        t = np.arange(40, dtype=np.float64)[::-1].copy()
        assert oracle.hull_mt(t, 2 * t, th, grain, lib=oracle_lib).tolist() == [39, 0]
        x, y = workloads.points("disk", 1000, seed=44)
        y[517] = np.inf
        with pytest.raises(oracle.OracleError) as e:
            oracle.hull_mt(x, y, th, grain, lib=oracle_lib)
        assert e.value.status == oracle.ORACLE_ERR_NONFINITE
