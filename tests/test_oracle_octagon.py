"""Pins of the oracle's octagon prefilter (the Akl-Toussaint heuristic of the
paper's Section 6, rules F1-F5 of the C source).

What pins it, independently of its own code:
* the eight vertices attain the extreme of their direction over all points,
  at the lowest index among equal values (checked by sorting, not by the
  oracle's scan);
* every dropped point is strictly inside the exact convex hull (exact
  rational arithmetic), so no hull vertex and no point on a hull edge is ever
  dropped;
* on a uniform disk the kept fraction is the area outside the inscribed
  regular octagon, 1 - 2*sqrt(2)/pi (closed form);
* points on, or closer than the margin to, an octagon edge are kept; points
  well inside are dropped; repeated vertices do not disable the filter; all
  equal points keep everything;
* the prefiltered variant returns the same hull as the plain method on the
  synthetic workloads;
* planted mistakes in a copy of the oracle each fail one of these pins.
"""
import math
import os
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads
from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "vqhull_oracle.c")


def _direction_values(x, y):
    """Per direction d (F1), the value whose minimum v_d attains (None: p or q)."""
    return [y, -(x - y), None, -(x + y), -y, x - y, None, x + y]


def check_vertices(x, y, vert, p, q):
    vals = _direction_values(x, y)
    for d in range(8):
        if vals[d] is None:
            assert vert[d] == (q if d == 2 else p), d
            continue
        v = vals[d]
        order = sorted(range(len(v)), key=lambda i: (v[i], i))
        assert vert[d] == order[0], (d, vert[d], order[0])


def check_dropped_strictly_inside(x, y, keep):
    """Every dropped point is strictly right of every clockwise hull edge (exact)."""
    hull = pins.exact_hull_fraction(x, y)
    if len(hull) < 3:
        assert keep.all()
        return
    H = [(Fraction(x[i]), Fraction(y[i])) for i in hull]
    for u in np.flatnonzero(~keep):
        U = (Fraction(x[u]), Fraction(y[u]))
        for k in range(len(H)):
            a, b = H[k], H[(k + 1) % len(H)]
            cross = (b[0] - a[0]) * (U[1] - a[1]) - (b[1] - a[1]) * (U[0] - a[0])
            assert cross < 0, (u, k)  # clockwise hull: the interior is on the right


def _small_cases():
    for seed in range(6):
        for dist in workloads.DISTRIBUTIONS:
            yield f"{dist}-{seed}", workloads.points(dist, 300, seed=seed)
    for k in range(12):
        yield f"lattice-{k}", workloads.lattice(200, seed=900 + k, lo=-(2 + k), hi=3 + k, dup_frac=0.3,
                                                collinear_runs=k % 3)
    rng = np.random.default_rng(7)
    for k in range(4):  # coordinates far from the origin relative to their spread
        x = 1e6 + rng.random(300) * 10.0 ** -(k + 1)
        y = -3e5 + rng.random(300) * 10.0 ** -(k + 1)
        yield f"offset-{k}", (x, y)


@pytest.mark.parametrize("name,pts", list(_small_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_vertices_extreme_and_dropped_points_strictly_inside(name, pts):
    x, y = pts
    vert, keep = oracle.octagon(x, y)
    p, q = oracle.extremes(x, y)
    check_vertices(x, y, vert, p, q)
    check_dropped_strictly_inside(x, y, keep)
    assert keep[vert].all()


def test_kept_fraction_on_a_disk_is_outside_the_inscribed_octagon():
    x, y = workloads.points("disk", 400_000, seed=11)
    _, keep = oracle.octagon(x, y)
    expect = 1.0 - 2.0 * math.sqrt(2.0) / math.pi  # regular octagon inscribed in the unit circle
    assert abs(keep.mean() - expect) < 0.004, keep.mean()


def test_square_keeps_almost_nothing():
    # Heavy-tailed inputs (kuzmin) carry no such bound: their octagon may miss
    # a hull vertex on the side where the dense core lies, and then keeps it.
    x, y = workloads.points("square", 200_000, seed=3)
    _, keep = oracle.octagon(x, y)
    assert keep.mean() < 0.01, keep.mean()


def _integer_octagon():
    # one vertex per direction, each the unique extreme of its direction
    return [(0, -4), (3, -3), (4, 0), (3, 3), (0, 4), (-3, 3), (-4, 0), (-3, -3)]


def test_margin_edges_and_interior():
    V = _integer_octagon()
    on_edge = [((a[0] + b[0]) / 2, (a[1] + b[1]) / 2) for a, b in zip(V, V[1:] + V[:1])]
    # just inside the edge v0->v1 (y = (x - 12) / 3), by about 1e-15 of the size
    t = 1.5
    just_inside = [(t, (t - 12.0) / 3.0 + 4e-15)]
    just_outside = [(t, np.nextafter((t - 12.0) / 3.0, -np.inf))]
    well_inside = [(0.0, 0.0), (1.0, 1.0), (-2.0, 0.5), (2.5, -2.0)]
    pts = V + on_edge + just_inside + just_outside + well_inside
    x = np.array([p[0] for p in pts], dtype=np.float64)
    y = np.array([p[1] for p in pts], dtype=np.float64)
    vert, keep = oracle.octagon(x, y)
    assert vert.tolist() == list(range(8))
    n_keep = len(V) + len(on_edge) + len(just_inside) + len(just_outside)
    assert keep[:n_keep].all()
    assert not keep[n_keep:].any()
    # exact check of the "just inside" point: it is strictly inside, yet kept
    a, b = V[0], V[1]
    u = just_inside[0]
    cross = (Fraction(b[0] - a[0]) * (Fraction(u[1]) - a[1]) - Fraction(b[1] - a[1]) * (Fraction(u[0]) - a[0]))
    assert cross > 0


def test_repeated_vertices_still_filter():
    rng = np.random.default_rng(5)
    tri = [(0.0, 0.0), (10.0, 0.0), (0.0, 10.0)]  # several directions share a corner
    inner = rng.random((500, 2)) * 3.0 + 1.0  # strictly inside, far from the edges
    x = np.array([p[0] for p in tri] + inner[:, 0].tolist())
    y = np.array([p[1] for p in tri] + inner[:, 1].tolist())
    vert, keep = oracle.octagon(x, y)
    assert set(vert.tolist()) == {0, 1, 2}
    assert keep[:3].all() and not keep[3:].any()
    assert oracle.hull_prefiltered(x, y, 10).tolist() == oracle.hull(x, y).tolist()


def test_degenerate_inputs_keep_everything():
    x = np.full(50, 2.5)
    y = np.full(50, -1.0)
    _, keep = oracle.octagon(x, y)
    assert keep.all()
    assert oracle.hull_prefiltered(x, y, 10).tolist() == [0]
    xs = np.arange(100, dtype=np.float64)
    _, keep = oracle.octagon(xs, 2.0 * xs + 1.0)  # collinear
    assert keep.all()
    _, keep = oracle.octagon(np.array([0.0, 1.0]), np.array([0.0, 1.0]))
    assert keep.all()


def test_threshold_and_nonfinite():
    x, y = workloads.points("disk", 1000, seed=2)
    assert oracle.hull_prefiltered(x, y, 1000).tolist() == oracle.hull(x, y).tolist()
    x[7] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.hull_prefiltered(x, y, 10)


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_prefiltered_hull_equals_plain_hull(dist):
    for seed in range(3):
        x, y = workloads.points(dist, 100_000, seed=40 + seed)
        assert np.array_equal(oracle.hull_prefiltered(x, y, 2048), oracle.hull(x, y))
    for k in range(20):
        x, y = workloads.lattice(3000, seed=70 + k, lo=-k - 1, hi=k + 2, dup_frac=0.2, collinear_runs=k % 3)
        assert np.array_equal(oracle.hull_prefiltered(x, y, 100), oracle.hull(x, y))


# ------------------------------------------------------------- planted mistakes

MUTANTS = {
    "margin_dropped": ("T[i] = c + M;", "T[i] = c;"),
    "vertex_not_translated": ("double ay = y[a] - oy;", "double ay = y[a];"),
    "point_not_translated": ("double ux = x[u] - ox;", "double ux = x[u];"),
    "edge_reversed": ("ex[i] = x[b] - x[a];\n    ey[i] = y[b] - y[a];", "ex[i] = x[a] - x[b];\n    ey[i] = y[a] - y[b];"),
    "cross_sign": ("double L = l1 - l2;", "double L = l2 - l1;"),
    "cross_dropped_term": ("double L = l1 - l2;", "double L = l1;"),
    "tie_highest_index": ("if (i == 0 || v < bv) {", "if (i == 0 || v <= bv) {"),
    "sum_for_difference": ("case 1: v = -(x[i] - y[i]); break;", "case 1: v = -(x[i] + y[i]); break;"),
    "zero_edges_not_skipped": ("      T[i] = -INFINITY;\n", ""),
    "all_equal_guard_removed": ("    if (edges == 0) {\n      keep[u] = 1;\n      continue;\n    }\n", ""),
    "vertex_order_mirrored": ("vert[d] = d == 2 ? q : d == 6 ? p : oct_extreme(x, y, n, d);",
                              "vert[d] = d == 2 ? p : d == 6 ? q : oct_extreme(x, y, n, d);"),
}


def _octagon_battery(lib) -> list[str]:
    failed = []

    def run(name, f):
        try:
            f()
        except (AssertionError, oracle.OracleError):
            failed.append(name)

    cases = list(_small_cases())[::5]

    def extremes_and_inside():
        for _, (x, y) in cases:
            vert, keep = oracle.octagon(x, y, lib=lib)
            check_vertices(x, y, vert, *oracle.extremes(x, y))
            check_dropped_strictly_inside(x, y, keep)

    def ties():
        for k in range(6):
            x, y = workloads.lattice(200, seed=900 + k, lo=-(2 + k), hi=3 + k, dup_frac=0.3, collinear_runs=k % 3)
            vert, _ = oracle.octagon(x, y, lib=lib)
            check_vertices(x, y, vert, *oracle.extremes(x, y))

    def fraction():
        x, y = workloads.points("disk", 100_000, seed=11)
        _, keep = oracle.octagon(x, y, lib=lib)
        assert abs(keep.mean() - (1.0 - 2.0 * math.sqrt(2.0) / math.pi)) < 0.006

    def margin():
        V = _integer_octagon()
        t = 1.5
        pts = V + [(t, (t - 12.0) / 3.0 + 4e-15), (0.0, 0.0)]
        x = np.array([p[0] for p in pts], dtype=np.float64)
        y = np.array([p[1] for p in pts], dtype=np.float64)
        _, keep = oracle.octagon(x, y, lib=lib)
        assert keep[:9].all() and not keep[9]

    def repeated():
        rng = np.random.default_rng(5)
        inner = rng.random((100, 2)) * 3.0 + 1.0
        x = np.array([0.0, 10.0, 0.0] + inner[:, 0].tolist())
        y = np.array([0.0, 0.0, 10.0] + inner[:, 1].tolist())
        _, keep = oracle.octagon(x, y, lib=lib)
        assert keep[:3].all() and not keep[3:].any()

    def all_equal():
        _, keep = oracle.octagon(np.full(20, 1.0), np.full(20, 1.0), lib=lib)
        assert keep.all()

    for name, f in (("inside", extremes_and_inside), ("ties", ties), ("fraction", fraction), ("margin", margin),
                    ("repeated", repeated), ("all_equal", all_equal)):
        run(name, f)
    return failed


def test_unmodified_oracle_passes_the_battery():
    assert _octagon_battery(oracle.load()) == []


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_is_caught(mutant):
    old, new = MUTANTS[mutant]
    src = open(SRC).read()
    assert src.count(old) == 1, mutant
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = oracle.load(oracle.build(src=path, out=os.path.join(d, "libmutant.so")))
        assert _octagon_battery(lib), f"mutant {mutant} passes every octagon pin"
