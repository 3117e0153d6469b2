"""Pins of the CPU oracle against references that do not use it.

Exact inputs (integer coordinates below 2^25, every predicate exact) must give
the exact strictly convex hull: brute force from the definition on tiny inputs,
Andrew's monotone chain on large ones, hand-computed hulls in
``golden/known_hulls.json``.  Floating-point inputs are pinned by the exact
rational hull in general position, by metamorphic relations (permutation,
power-of-two scaling) and by the rounding of the fixed orientation formula.
"""
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "known_hulls.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_known_hulls(case, oracle_lib):
    x = np.array(case["x"], dtype=np.float64)
    y = np.array(case["y"], dtype=np.float64)
    got = oracle.hull(x, y, lib=oracle_lib).tolist()
    assert got == case["hull"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_known_hulls_agree_with_references(case):
    """The hand-computed fixtures themselves agree with both exact references."""
    x = np.array(case["x"], dtype=np.float64)
    y = np.array(case["y"], dtype=np.float64)
    assert pins.exact_hull_fraction(x, y) == case["hull"]
    if np.all(x == np.round(x)) and np.all(y == np.round(y)):
        assert pins.brute_force_hull(x, y) == case["hull"]
        assert pins.andrew_hull(x, y) == case["hull"]


def _splits():
    with open(GOLDEN) as f:
        return json.load(f)["splits"]


@pytest.mark.parametrize("case", _splits(), ids=lambda c: c["name"])
def test_known_splits(case, oracle_lib):
    x = np.array(case["x"], dtype=np.float64)
    y = np.array(case["y"], dtype=np.float64)
    s1, s2, r1, r2 = oracle.split(x, y, np.arange(len(x)), case["a"], case["r"], case["b"], lib=oracle_lib)
    assert sorted(s1.tolist()) == case["s1"] and sorted(s2.tolist()) == case["s2"]
    assert (r1, r2) == (case["r1"], case["r2"])


def _tiny_lattice_cases(count, seed0):
    rng = random.Random(seed0)
    for k in range(count):
        n = rng.choice([1, 2, 3, 4, 5, 8, 13, 21, 40, 64, 100, 150])
        hi = rng.choice([1, 2, 3, 7, 15, 2**20 - 1])
        lo = rng.choice([0, -hi])
        yield k, workloads.lattice(n, seed=seed0 * 100003 + k, lo=lo, hi=hi,
                                   dup_frac=rng.choice([0.0, 0.1, 0.5]), collinear_runs=rng.choice([0, 1, 3]))


def test_brute_force_tiny_lattices(oracle_lib):
    """Oracle equals the O(u^3) brute-force hull on 10^4 seeded lattice inputs."""
    for k, (x, y) in _tiny_lattice_cases(10_000, 7):
        want = pins.brute_force_hull(x, y)
        got = oracle.hull(x, y, lib=oracle_lib).tolist()
        assert got == want, f"case {k}: n={len(x)}"


@pytest.mark.parametrize("n,hi,seed", [(1000, 7, 1), (10_000, 100, 2), (100_000, 2**20 - 1, 3),
                                       (300_000, 1000, 4), (200_000, 2**24 - 1, 5),
                                       (1_000_000, 2**20 - 1, 6)])
def test_andrew_lattices(n, hi, seed, oracle_lib):
    x, y = workloads.lattice(n, seed=seed, lo=-hi, hi=hi, dup_frac=0.05, collinear_runs=4)
    assert oracle.hull(x, y, lib=oracle_lib).tolist() == pins.andrew_hull(x, y)


def test_andrew_lattice_circle_like(oracle_lib):
    """Many exactly collinear and cocircular lattice points (deep recursion, many ties)."""
    r = 300
    pts = set()
    for a in range(-r, r + 1):
        b = int(math.isqrt(r * r - a * a))
        pts.update({(a, b), (a, -b), (b, a), (-b, a)})
    pts = sorted(pts)
    rng = np.random.default_rng(11)
    order = rng.permutation(len(pts))
    x = np.array([pts[i][0] for i in order], dtype=np.float64)
    y = np.array([pts[i][1] for i in order], dtype=np.float64)
    assert oracle.hull(x, y, lib=oracle_lib).tolist() == pins.andrew_hull(x, y)


@pytest.mark.parametrize("dist", ["disk", "square", "kuzmin"])
def test_float_general_position_equals_exact_hull(dist, oracle_lib):
    """In general position every predicate has the exact sign, so the result is the exact hull."""
    for seed in range(20):
        x, y = workloads.points(dist, 300, seed=1000 + seed)
        assert oracle.hull(x, y, lib=oracle_lib).tolist() == pins.exact_hull_fraction(x, y)


@pytest.mark.parametrize("dist", list(workloads.DISTRIBUTIONS))
def test_metamorphic_permutation(dist, oracle_lib):
    """The coordinate sequence of the result does not depend on the input order."""
    x, y = workloads.points(dist, 20_000, seed=21)
    h = oracle.hull(x, y, lib=oracle_lib)
    perm = np.random.default_rng(5).permutation(len(x))
    h2 = oracle.hull(x[perm], y[perm], lib=oracle_lib)
    assert np.array_equal(x[h], x[perm][h2]) and np.array_equal(y[h], y[perm][h2])


@pytest.mark.parametrize("k", [-40, -3, 1, 7, 60])
def test_metamorphic_power_of_two_scaling(k, oracle_lib):
    """Scaling by 2^k scales every rounded operation exactly: identical index list."""
    for dist in workloads.DISTRIBUTIONS:
        x, y = workloads.points(dist, 20_000, seed=33)
        h = oracle.hull(x, y, lib=oracle_lib)
        s = math.ldexp(1.0, k)
        assert np.array_equal(h, oracle.hull(x * s, y * s, lib=oracle_lib))


def test_invariants_float_inputs(oracle_lib):
    for dist in workloads.DISTRIBUTIONS:
        x, y = workloads.points(dist, 50_000, seed=44)
        h = oracle.hull(x, y, lib=oracle_lib)
        assert len(set(h.tolist())) == len(h)
        assert h.min() >= 0 and h.max() < len(x)
        p, q = oracle.extremes(x, y, lib=oracle_lib)
        assert h[0] == p and q in h.tolist()
        assert p == int(np.lexsort((np.arange(len(x)), y, x))[0])


def test_extremes_ties(oracle_lib):
    x = np.array([1.0, 0.0, 0.0, 2.0, 2.0, 0.0, 2.0])
    y = np.array([0.0, 5.0, -1.0, 3.0, 3.0, -1.0, -9.0])
    assert oracle.extremes(x, y, lib=oracle_lib) == (2, 3)


def test_orient_sign_matches_exact_beyond_error_bound(oracle_lib):
    """Sign of the fixed formula equals the exact sign whenever |exact| exceeds the
    classical forward error bound (3 + 16 eps) eps (|t1 t2| + |t3 t4|)."""
    rng = np.random.default_rng(3)
    eps = 2.0 ** -53
    for _ in range(20_000):
        a, b, c = rng.standard_normal(2), rng.standard_normal(2), rng.standard_normal(2)
        if rng.random() < 0.5:  # near-collinear: c close to the line ab
            t = rng.random()
            c = a + t * (b - a) + rng.standard_normal(2) * 1e-12
        o = oracle.orient(*a, *b, *c, lib=oracle_lib)
        ex = pins.exact_orient(a, b, c)
        det_sum = abs((a[0] - c[0]) * (b[1] - c[1])) + abs((a[1] - c[1]) * (b[0] - c[0]))
        bound = (3.0 + 16.0 * eps) * eps * det_sum
        if abs(float(ex)) > bound:
            assert (o > 0) == (ex > 0) and (o < 0) == (ex < 0)


def test_orient_rounding_is_binary64_without_contraction(oracle_lib):
    """Each operation rounded on its own (no fused multiply-add): matches exact-rational emulation."""
    rng = np.random.default_rng(4)
    cases = []
    for _ in range(5000):
        a, b = rng.standard_normal(2), rng.standard_normal(2)
        t = rng.random()
        c = a + t * (b - a) + rng.standard_normal(2) * 1e-14
        cases.append((a, b, c))
    # subnormal and huge magnitudes, signed zeros
    cases += [((1e-160, 3e-160), (2e-160, -1e-160), (0.0, 1e-161)),
              ((1e150, -1e150), (-3e150, 2e150), (1e149, 1e149)),
              ((0.0, -0.0), (-0.0, 0.0), (0.0, 0.0)),
              ((1.0, 2.0), (3.0, 4.0), (5.0, 6.0 + 2.0 ** -50))]
    for a, b, c in cases:
        o = oracle.orient(*a, *b, *c, lib=oracle_lib)
        r = pins.rounded_orient(a, b, c)
        assert o == r or (math.isnan(o) and math.isnan(r)), (a, b, c, o, r)


def _find_both_left_case():
    """Search circle-like triples for a point that is (after rounding) left of both a->r and r->b."""
    rng = np.random.default_rng(99)
    for _ in range(200_000):
        th = rng.random() * 2 * math.pi
        d = 10.0 ** rng.uniform(-9, -7)
        a = (math.cos(th - d), math.sin(th - d))
        r = (math.cos(th), math.sin(th))
        b = (math.cos(th + d), math.sin(th + d))
        e = d * rng.uniform(-1, 1)
        u = (math.cos(th + e), math.sin(th + e))
        if pins.rounded_orient(a, r, u) > 0 and pins.rounded_orient(r, b, u) > 0:
            return a, r, b, u
    return None


def test_point_left_of_both_edges_goes_to_s1(oracle_lib):
    """Reading R5: under rounding a point may test left of both a->r and r->b; it goes to S1."""
    found = _find_both_left_case()
    assert found is not None
    a, r, b, u = found
    x = np.array([a[0], r[0], b[0], u[0]])
    y = np.array([a[1], r[1], b[1], u[1]])
    s1, s2, r1, r2 = oracle.split(x, y, [3], 0, 1, 2, lib=oracle_lib)
    assert s1.tolist() == [3] and s2.tolist() == [] and r1 == 3 and r2 == -1


def test_split_level0_sets(oracle_lib):
    """The top-level step (p, q, p): S1 is strictly above p->q, S2 strictly below, by exact signs."""
    x, y = workloads.lattice(2000, seed=8, lo=-50, hi=50, collinear_runs=5)
    p, q = oracle.extremes(x, y, lib=oracle_lib)
    s1, s2, r1, r2 = oracle.split(x, y, np.arange(len(x)), p, q, p, lib=oracle_lib)
    P, Q = (x[p], y[p]), (x[q], y[q])
    sign = np.array([int(np.sign(pins.exact_orient(P, Q, (x[i], y[i])))) for i in range(len(x))])
    assert sorted(s1.tolist()) == np.nonzero(sign > 0)[0].tolist()
    assert sorted(s2.tolist()) == np.nonzero(sign < 0)[0].tolist()
    k1 = [pins.exact_orient(P, Q, (x[i], y[i])) for i in s1]
    best = max(zip(k1, [-x[i] for i in s1], [-y[i] for i in s1], [-i for i in s1]))
    assert r1 == -best[3]


def test_nonfinite_inputs_rejected(oracle_lib):
    for bad in (math.nan, math.inf, -math.inf):
        x = np.array([0.0, 1.0, 2.0])
        y = np.array([0.0, bad, 1.0])
        with pytest.raises(oracle.OracleError) as e:
            oracle.hull(x, y, lib=oracle_lib)
        assert e.value.status == oracle.ORACLE_ERR_NONFINITE


def test_circle_sanity(oracle_lib):
    """Points on a circle: the recursion is balanced and most points are found when n is small."""
    x, y = workloads.points("circle", 20_000, seed=3)
    h = oracle.hull(x, y, lib=oracle_lib)
    assert 0.5 * len(x) < len(h) <= len(x)
