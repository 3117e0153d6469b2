"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle (a flipped sign, a transposed operand, a dropped term, a wrong tie rule,
a wrong output order) makes at least one pin fail.

The mutants are built on the CPU from a textual edit of the oracle source into
a temporary directory; the oracle itself is never modified.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads
from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "vqhull_oracle.c")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "known_hulls.json")

MUTANTS = {
    "orient_sign": ("return m1 - m2;", "return m2 - m1;"),
    "orient_dropped_term": ("return m1 - m2;", "return m1;"),
    "orient_transposed_operand": ("double t2 = by - cy;", "double t2 = cy - by;"),
    "orient_wrong_index": ("double t4 = bx - cx;", "double t4 = bx - ax;"),
    "non_strict_left": ("if (o1 > 0.0) {", "if (o1 >= 0.0) {"),
    "non_strict_left_s2": ("if (o2 > 0.0) {", "if (o2 >= 0.0) {"),
    "tie_x_descending": ("if (x[i] < x[bi]) return 1;\n  if (x[i] > x[bi]) return 0;",
                         "if (x[i] > x[bi]) return 1;\n  if (x[i] < x[bi]) return 0;"),
    "tie_index_only": ("if (x[i] < x[bi]) return 1;\n  if (x[i] > x[bi]) return 0;\n  if (y[i] < y[bi]) return 1;\n"
                       "  if (y[i] > y[bi]) return 0;", ""),
    "argmax_is_argmin": ("if (k > bk) return 1;\n  if (k < bk) return 0;", "if (k < bk) return 1;\n  if (k > bk) return 0;"),
    "tie_highest_index": ("return i < bi;", "return i > bi;"),
    "lexmin_y_tie_flipped": ("(x[i] == x[p] && y[i] < y[p])", "(x[i] == x[p] && y[i] > y[p])"),
    "lexmax_highest_index": ("if (x[i] > x[q] || (x[i] == x[q] && y[i] > y[q])) q = i;",
                             "if (x[i] > x[q] || (x[i] == x[q] && y[i] >= y[q])) q = i;"),
    "vertex_before_s1": ("  int st = hull_rec(x, y, s, n1, a, r1, r, out);\n  if (st == ORACLE_OK) {\n"
                         "    out->idx[out->len++] = r;\n",
                         "  out->idx[out->len++] = r;\n  int st = hull_rec(x, y, s, n1, a, r1, r, out);\n"
                         "  if (st == ORACLE_OK) {\n"),
    "s2_wrong_far_end": ("st = hull_rec(x, y, s + (m - n2), n2, r, r2, b, out);",
                         "st = hull_rec(x, y, s + (m - n2), n2, r, r2, a, out);"),
    "s1_wrong_edge": ("int st = hull_rec(x, y, s, n1, a, r1, r, out);", "int st = hull_rec(x, y, s, n1, a, r1, b, out);"),
    "top_level_swapped": ("split(x, y, all, n, p, q, p, s, &n1, &n2, &r1, &r2);",
                          "split(x, y, all, n, q, p, q, s, &n1, &n2, &r1, &r2);"),
    "base_case_too_big": ("if (m <= 1) { /* base case: return P itself */\n    if (m == 1) out->idx[out->len++] = P[0];",
                          "if (m <= 2) { /* base case: return P itself */\n    for (int64_t j = 0; j < m; ++j) "
                          "out->idx[out->len++] = P[j];"),
    "s2_priority": ("    double o1 = vqhull_oracle_orient(x[a], y[a], x[r], y[r], x[u], y[u]);\n    if (o1 > 0.0) {",
                    "    double o1 = vqhull_oracle_orient(x[a], y[a], x[r], y[r], x[u], y[u]);\n"
                    "    if (o1 > 0.0 && !(vqhull_oracle_orient(x[r], y[r], x[b], y[b], x[u], y[u]) > 0.0)) {"),
    "q_not_emitted": ("    out.idx[out.len++] = q;\n", ""),
}


def _pin_battery(lib) -> list[str]:
    """Run a fast subset of the pins against a library; return the names that failed."""
    failed = []
    with open(GOLDEN) as f:
        for case in json.load(f)["cases"]:
            x = np.array(case["x"], dtype=np.float64)
            y = np.array(case["y"], dtype=np.float64)
            try:
                if oracle.hull(x, y, lib=lib).tolist() != case["hull"]:
                    failed.append("known:" + case["name"])
            except oracle.OracleError:
                failed.append("known:" + case["name"])
        for case in json.load(open(GOLDEN))["splits"]:
            x = np.array(case["x"], dtype=np.float64)
            y = np.array(case["y"], dtype=np.float64)
            s1, s2, r1, r2 = oracle.split(x, y, np.arange(len(x)), case["a"], case["r"], case["b"], lib=lib)
            if (sorted(s1.tolist()), sorted(s2.tolist()), r1, r2) != (case["s1"], case["s2"], case["r1"], case["r2"]):
                failed.append("split:" + case["name"])
    for k in range(200):
        x, y = workloads.lattice(1 + k % 60, seed=5000 + k, lo=0, hi=1 + k % 9, dup_frac=0.2, collinear_runs=k % 3)
        try:
            if oracle.hull(x, y, lib=lib).tolist() != pins.brute_force_hull(x, y):
                failed.append(f"brute:{k}")
        except oracle.OracleError:
            failed.append(f"brute:{k}")
    for seed in range(5):
        x, y = workloads.points("disk", 200, seed=900 + seed)
        if oracle.hull(x, y, lib=lib).tolist() != pins.exact_hull_fraction(x, y):
            failed.append(f"exact_float:{seed}")
    # R5: a point left of both edges after rounding goes to S1
    from tests.test_oracle import _find_both_left_case

    a, r, b, u = _find_both_left_case()
    s1, s2, _, _ = oracle.split(np.array([a[0], r[0], b[0], u[0]]), np.array([a[1], r[1], b[1], u[1]]), [3], 0, 1, 2,
                                lib=lib)
    if s1.tolist() != [3]:
        failed.append("both_left_goes_to_s1")
    return failed


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_unmutated_passes_battery(oracle_lib):
    assert _pin_battery(oracle_lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    so = oracle.build(str(src), str(tmp_path / "libmutant.so"))
    # A mutant may crash (runaway recursion, writes past the output): run it in
    # a child process; a crash or any failed pin counts as caught.
    code = ("import sys, oracle; from tests.test_oracle_mutants import _pin_battery; "
            f"sys.exit(1 if _pin_battery(oracle.load({so!r})) else 0)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    proc = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, timeout=600)
    assert proc.returncode != 0, f"mutant {name} survived every pin"
