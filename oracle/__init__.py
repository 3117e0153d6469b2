"""CPU oracle for planar Quickhull (ctypes binding of ``vqhull_oracle.c``).

Test infrastructure only: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only users.  The GPU library never imports
or calls anything here, and nothing here imports the GPU library.

The C source follows Algorithm 1 (Section 2.1) of the VQhull paper with every
floating-point and tie decision fixed; its header lists the rules.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vqhull_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# The predicate must be evaluated exactly as written: no contraction into FMA,
# no fast-math reassociation, binary64 SSE arithmetic.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-fPIC", "-shared", "-fopenmp"]

ORACLE_OK = 0
ORACLE_ERR_INVALID_ARGUMENT = 1
ORACLE_ERR_OUT_OF_MEMORY = 2
ORACLE_ERR_NONFINITE = 3

_lock = threading.Lock()
_lib = None


def build(src: str = _SRC, out: str = _LIB, extra_flags: list[str] | None = None) -> str:
    """Compile the oracle with gcc into a shared library and return its path."""
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    d, i64, pd, pi64 = ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    lib.vqhull_oracle_orient.restype = d
    lib.vqhull_oracle_orient.argtypes = [d, d, d, d, d, d]
    lib.vqhull_oracle_extremes.restype = ctypes.c_int
    lib.vqhull_oracle_extremes.argtypes = [pd, pd, i64, pi64, pi64]
    lib.vqhull_oracle_split.restype = ctypes.c_int
    lib.vqhull_oracle_split.argtypes = [pd, pd, pi64, i64, i64, i64, i64, pi64, pi64, pi64, pi64, pi64]
    lib.vqhull_oracle_hull.restype = ctypes.c_int
    lib.vqhull_oracle_hull.argtypes = [pd, pd, i64, pi64, pi64]
    lib.vqhull_oracle_orient_batch.restype = ctypes.c_int
    lib.vqhull_oracle_orient_batch.argtypes = [pd, i64, pd]
    lib.vqhull_oracle_hull_mt.restype = ctypes.c_int
    lib.vqhull_oracle_hull_mt.argtypes = [pd, pd, i64, pi64, pi64, ctypes.c_int, i64]
    lib.vqhull_oracle_octagon.restype = ctypes.c_int
    lib.vqhull_oracle_octagon.argtypes = [pd, pd, i64, pi64, ctypes.POINTER(ctypes.c_uint8)]
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the oracle library (building it first if it is not built yet).

    With ``path`` given, load that library instead (used by tests that build
    deliberately broken variants of the oracle to check the pins).
    """
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _pd(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


def orient(ax, ay, bx, by, cx, cy, lib=None) -> float:
    """orient(a, b, c) > 0 iff c is strictly left of a->b (Section 2.1)."""
    return (lib or load()).vqhull_oracle_orient(ax, ay, bx, by, cx, cy)


def orient_batch(abc, lib=None) -> np.ndarray:
    """R1 on the rows of an (n, 6) array (a.x, a.y, b.x, b.y, c.x, c.y)."""
    abc = np.ascontiguousarray(abc, dtype=np.float64)
    if abc.ndim != 2 or abc.shape[1] != 6:
        raise ValueError("abc must be an (n, 6) array")
    out = np.empty(len(abc), dtype=np.float64)
    st = (lib or load()).vqhull_oracle_orient_batch(_pd(abc), len(abc), _pd(out))
    if st:
        raise OracleError(st)
    return out


def extremes(x, y, lib=None) -> tuple[int, int]:
    """(p, q): lexicographic minimum and maximum points of the input."""
    x, y = _f64(x), _f64(y)
    p, q = ctypes.c_int64(), ctypes.c_int64()
    st = (lib or load()).vqhull_oracle_extremes(_pd(x), _pd(y), len(x), ctypes.byref(p), ctypes.byref(q))
    if st:
        raise OracleError(st)
    return p.value, q.value


def split(x, y, P, a: int, r: int, b: int, lib=None):
    """One partition step of Algorithm 1 on the subset ``P`` for triangle (a, r, b).

    Returns (S1, S2, r1, r2) with S1, S2 int64 index arrays and r1 / r2 the
    farthest points (-1 when the subset is empty).
    """
    x, y = _f64(x), _f64(y)
    P = np.ascontiguousarray(P, dtype=np.int64)
    m = len(P)
    s = np.empty(max(m, 1), dtype=np.int64)
    n1, n2, r1, r2 = (ctypes.c_int64() for _ in range(4))
    st = (lib or load()).vqhull_oracle_split(_pd(x), _pd(y), _pi(P), m, a, r, b, _pi(s), ctypes.byref(n1),
                                             ctypes.byref(n2), ctypes.byref(r1), ctypes.byref(r2))
    if st:
        raise OracleError(st)
    return s[: n1.value].copy(), s[m - n2.value: m].copy(), r1.value, r2.value


def hull(x, y, lib=None) -> np.ndarray:
    """Hull vertex indices, clockwise from the lexicographically smallest point."""
    x, y = _f64(x), _f64(y)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of equal length")
    n = len(x)
    out = np.empty(max(n, 1), dtype=np.int64)
    cnt = ctypes.c_int64()
    st = (lib or load()).vqhull_oracle_hull(_pd(x), _pd(y), n, _pi(out), ctypes.byref(cnt))
    if st:
        raise OracleError(st)
    return out[: cnt.value].copy()


def hull_mt(x, y, threads: int = 0, grain: int = 0, lib=None) -> np.ndarray:
    """The multithreaded form of ``hull`` (OpenMP, ``threads`` threads, 0 = all
    the runtime offers; ``grain`` points per parallel chunk and smallest task,
    0 = default): the same index list, computed on every core."""
    x, y = _f64(x), _f64(y)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of equal length")
    n = len(x)
    out = np.empty(max(n, 1), dtype=np.int64)
    cnt = ctypes.c_int64()
    st = (lib or load()).vqhull_oracle_hull_mt(_pd(x), _pd(y), n, _pi(out), ctypes.byref(cnt), int(threads),
                                               int(grain))
    if st:
        raise OracleError(st)
    return out[: cnt.value].copy()


def octagon(x, y, lib=None) -> tuple[np.ndarray, np.ndarray]:
    """Octagon prefilter (rules F1-F4 of the C source): the eight vertices
    (v0 = min y, then counter-clockwise) and a keep mask (False = dropped as
    strictly inside the octagon)."""
    x, y = _f64(x), _f64(y)
    if x.shape != y.shape or x.ndim != 1 or len(x) == 0:
        raise ValueError("x and y must be non-empty 1-D arrays of equal length")
    vert = np.empty(8, dtype=np.int64)
    keep = np.empty(len(x), dtype=np.uint8)
    st = (lib or load()).vqhull_oracle_octagon(_pd(x), _pd(y), len(x), _pi(vert),
                                               keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if st:
        raise OracleError(st)
    return vert, keep.astype(bool)


def hull_prefiltered(x, y, min_points: int, lib=None) -> np.ndarray:
    """The prefiltered variant of the method (rule F5): with more than
    ``min_points`` points, the octagon filter first, then Algorithm 1 on the
    kept points in their index order (so index tie-breaks are unchanged), the
    result mapped back to input indices; otherwise Algorithm 1 on all points."""
    x, y = _f64(x), _f64(y)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of equal length")
    if len(x) <= min_points:
        return hull(x, y, lib=lib)
    if not (np.isfinite(x).all() and np.isfinite(y).all()):
        raise OracleError(ORACLE_ERR_NONFINITE)
    _, keep = octagon(x, y, lib=lib)
    kept = np.flatnonzero(keep)
    return kept[hull(x[kept], y[kept], lib=lib)]
