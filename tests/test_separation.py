"""Structural checks that the product path and the oracle stay apart: the
package (Python, HIP and C++ sources) never imports, loads or includes
anything from oracle/; the oracle never imports the package (the seeded
generators in workloads.py are the only shared module, and the oracle does not
even use those); bench.py imports the oracle only in its CPU-baseline leg; and
the binding raises when the library is missing instead of computing anything
itself."""
import glob
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2510_09417_amd")


def _sources(pattern_dirs, exts):
    out = []
    for d in pattern_dirs:
        for e in exts:
            out += glob.glob(os.path.join(d, "**", "*" + e), recursive=True)
    return [f for f in out if "/_build/" not in f and "__pycache__" not in f]


def test_package_never_uses_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b)|liboracle|vqhull_oracle|#include\s+\"[^\"]*oracle", re.M)
    files = _sources([PKG, os.path.join(ROOT, "include")], (".py", ".hip", ".cpp", ".h"))
    assert len(files) >= 8
    for f in files:
        assert not pat.search(open(f).read()), f


def test_oracle_never_uses_the_package():
    for f in _sources([os.path.join(ROOT, "oracle")], (".py", ".c", ".h")):
        text = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+paper_2510_09417_amd", text, re.M), f
        assert "libvqhull" not in text and "vqhull.h" not in text, f


def test_bench_imports_the_oracle_only_for_the_cpu_baseline():
    text = open(os.path.join(ROOT, "bench.py")).read()
    imports = [m.start() for m in re.finditer(r"^\s*import oracle\b", text, re.M)]
    assert len(imports) == 1
    guard = text.rfind("if not args.no_cpu_baseline", 0, imports[0])
    assert guard != -1 and imports[0] - guard < 200  # inside the CPU-baseline leg


def test_missing_library_raises():
    code = ("import paper_2510_09417_amd as vq\n"
            "try:\n    vq.load_library('/nonexistent/libvqhull.so')\n"
            "except FileNotFoundError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.startswith("raised"), r.stdout + r.stderr
