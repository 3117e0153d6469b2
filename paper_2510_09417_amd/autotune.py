"""Autotuning cache for the hull kernels.

``vqhull_autotune`` (the library) times every supported configuration --
sweep workgroup shape, LDS-finisher threshold, persistent or one workgroup per
tile -- on given points and returns the fastest one whose result equals the
others'.  This module keeps the winners in a JSON file keyed by
(GPU architecture, compute-unit count, size bucket) and applies them:

    python -m paper_2510_09417_amd.autotune --dist disk --n 100000000   # tune, store
    paper_2510_09417_amd.autotune.apply(n)                               # set config for a size

The size bucket of n is n.bit_length() (points within a factor of 2 share it);
``apply`` uses the nearest tuned bucket of the same GPU.  The cache file is
``$VQHULL_TUNE_CACHE`` or ``~/.cache/vqhull/tune.json``.
"""
from __future__ import annotations

import argparse
import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "vqhull", "tune.json")


def cache_path(path: str | None = None) -> str:
    return path or os.environ.get("VQHULL_TUNE_CACHE") or DEFAULT_CACHE


def bucket(n: int) -> int:
    return int(n).bit_length()


def device_key() -> str:
    import torch

    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}/{p.multi_processor_count}cu"


def load(path: str | None = None) -> dict:
    try:
        with open(cache_path(path)) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store(entries: dict, path: str | None = None) -> None:
    p = cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(cache: dict, dev: str, n: int):
    """The entry of the tuned bucket of ``dev`` nearest to n's, or None."""
    b = bucket(n)
    best = None
    for key, e in cache.items():
        d, _, kb = key.rpartition("/b")
        if d != dev or not kb.isdigit():
            continue
        if best is None or abs(int(kb) - b) < abs(best[0] - b):
            best = (int(kb), e)
    return None if best is None else best[1]


def tune(x, y, repeats: int = 3, path: str | None = None) -> dict:
    """Tune on (x, y) (float64 GPU tensors), store and return the cache entry."""
    import paper_2510_09417_amd as vq

    t0 = time.perf_counter()
    best, table = vq.autotune_table(x, y, repeats=repeats)
    dev = device_key()
    entry = {"config": best, "n": int(x.numel()), "table": table, "tuning_seconds": time.perf_counter() - t0}
    cache = load(path)
    cache[f"{dev}/b{bucket(x.numel())}"] = entry
    store(cache, path)
    return entry


# The configuration space of the tuner (the same as the library's single-hull
# tuner): sweep shapes, LDS-finisher thresholds, persistent grid or not.
SHAPES = ((256, 16), (256, 32), (512, 8), (512, 16), (1024, 8))
LDS_LIMITS = (512, 1024, 2048)


def tune_batched(x, y, offsets, repeats: int = 3, stream=None, persistent=(1, 0)) -> tuple[dict, list[dict]]:
    """Tune the batched path on one representative batch: times
    ``hull_batched(x, y, offsets)`` (median of ``repeats`` runs after a warm-up)
    under every configuration (grid modes limited to ``persistent``: the
    server's graph-captured batches need persistent sweeps; the octagon
    prefilter and level pairs off, as the server's lanes run the plain method
    level by level) and checks that
    each gives the same index lists and counts as the first.  Returns (fastest
    equal configuration, table); the library configuration is restored
    afterwards."""
    import numpy as np
    import torch

    import paper_2510_09417_amd as vq

    offsets = np.asarray(offsets, dtype=np.int64)
    saved = vq.get_config()
    table, ref, best = [], None, None
    vq.set_level_pairs(0)
    try:
        for blk, ppt in SHAPES:
            for lds in LDS_LIMITS:
                for pers in persistent:
                    cfg = vq.set_config(sweep_block=blk, sweep_ppt=ppt, lds_limit=lds, sweep_persistent=pers,
                                        level_block=256, prefilter=0)
                    out, cnt = vq.hull_batched(x, y, offsets, stream=stream)
                    torch.cuda.synchronize()
                    times = []
                    for _ in range(max(1, repeats)):
                        t0 = time.perf_counter()
                        out, cnt = vq.hull_batched(x, y, offsets, stream=stream)
                        torch.cuda.synchronize()
                        times.append(time.perf_counter() - t0)
                    # the index lists only: out_idx past each request's count is unspecified
                    o, c = out.cpu().numpy(), cnt.cpu().numpy()
                    res = (c, [o[offsets[i]:offsets[i] + max(int(c[i]), 0)] for i in range(len(c))])
                    if ref is None:
                        ref = res
                    same = bool(np.array_equal(res[0], ref[0])
                                and all(np.array_equal(a, b) for a, b in zip(res[1], ref[1])))
                    ms = 1e3 * sorted(times)[len(times) // 2]
                    table.append({"config": cfg, "ms": ms, "same_result": same})
                    if same and (best is None or ms < best["ms"]):
                        best = table[-1]
    finally:
        vq.set_config(**saved)
        vq.set_level_pairs(1)
    return best["config"], table


def apply(n: int, path: str | None = None) -> dict | None:
    """Set the library configuration tuned for size n on this GPU; returns it,
    or None (configuration unchanged) when nothing is cached for this GPU."""
    import paper_2510_09417_amd as vq

    e = lookup(load(path), device_key(), n)
    if e is None:
        return None
    return vq.set_config(**e["config"])


def main() -> int:
    import torch

    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--dist", default="disk", choices=workloads.DISTRIBUTIONS)
    ap.add_argument("--n", type=float, default=1e8)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--cache", default=None)
    a = ap.parse_args()
    vq.load_library()
    x, y = workloads.points(a.dist, int(a.n), a.seed)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    e = tune(tx, ty, repeats=a.repeats, path=a.cache)
    for row in sorted(e["table"], key=lambda r: r["ms"]):
        c = row["config"]
        print(f"{c['sweep_block']:5d}x{c['sweep_ppt']:<3d} lds {c['lds_limit']:5d} persistent {c['sweep_persistent']}"
              f"  {row['ms']:8.3f} ms  {'same' if row['same_result'] else 'DIFFERENT'}")
    print("best:", e["config"], "->", cache_path(a.cache))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
