#!/usr/bin/env python3
"""Benchmark of the gfx950 Quickhull on one GPU.

One step = the hull of 10^8 uniform unit-disk points plus the hull of 10^8
uniform unit-square points (seed 2 each; recipe in paper_2510_09417_amd/
workloads.py), i.e. every kernel of the path (extremes, every sweep level,
planners, LDS finisher, assembly) over 2e8 points already resident in HBM.
Prints one JSON line:

  value       whole-step throughput, Gpoints/s (points hulled / wall time);
  roofline    the fused top-level sweep (the dominant kernel: it classifies every
              input point against p->q and against its child's triangle and
              writes the grandchild subsets): algorithmic bytes per launch
              (16 B read per input point + 20 B written per kept point) over its
              average duration, from HIP events recorded on the launch stream
              around that kernel alone during the timed steps (no other launch
              is timed there), against 8 TB/s; the argmax pass and all-sweep
              rates beside it come from two untimed breakdown steps;
  per_hull    each dataset's hull alone: HIP events on the launch stream
              around the call (first kernel to the count written), 10 runs
              after a warm-up, median and standard deviation.
  configs     the other single-hull workloads (disk 10^6, circle 5*10^7,
              Kuzmin 10^8) each alone: median and spread of 10 runs,
              Gpoints/s, algorithmic bytes per point and per second against
              8 TB/s, and equality of the GPU's list with the CPU oracle's.
  cpu_baseline  the CPU oracle on the host: one whole step on every core (its
              multithreaded form) and single-threaded, median of 3 runs each;
              every configuration above on every core; a seeded sample of the
              served requests, one request per thread.
  prefilter   the same step with the octagon prefilter on (Section 6's
              Akl-Toussaint heuristic, a variant of the method; outside the
              timed region): throughput, a check that every hull equals the
              plain path's, the points kept, and the bandwidth of its passes.
  aos         the same step from interleaved (x, y) input (the array-of-
              structures layout of the paper's inputs), without and with the
              prefilter: throughput and equality with the plain path.
  served      the served mix (65,536 requests, sizes log-uniform in [16, 10^6],
              disk / square / circle / Kuzmin in equal shares, drawn on the GPU):
              hulls/s with every request submitted at once; p50 / p99 latency
              (submit to results written) under Poisson arrivals at half that
              rate; the plain path (one vqhull_hull call per request) on a
              time-boxed prefix of the same mix; both paths under the same
              Poisson stream at 0.9 x the plain path's capacity (latency from
              the scheduled arrival on both); the algorithmic bytes of the whole
              mix per second against 8 TB/s; checks that served results equal
              the plain path's on a prefix and the CPU oracle's on a seeded
              sample (random requests plus the largest of each distribution).

Usage: python bench.py [--gpus 1] [--steps 50] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_fused_traffic.json")
METRIC = "Gpoints/s + % HBM peak (1e8 FP64 pts); batched hulls/s + p50/p99 latency"


def load_traffic():
    """Measured HBM bytes per fused-sweep launch (from rocprofv3 counters), or
    None when absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2510_09417_amd.profiling import kernel_source_hash

    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def percentile(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(q * len(v)))]


SERVED_SAMPLE = 64  # random served requests checked against the CPU oracle (plus the largest of each distribution)
CONFIG_LEGS = ("disk_1e6", "circle_5e7", "kuzmin_1e8")
CONFIG_RUNS = 10


def configs_leg(vq, torch, workloads, stream) -> tuple[dict, list]:
    """The other single-hull workloads (disk 10^6, circle 5*10^7, Kuzmin
    10^8), each alone: HIP events on the launch stream around the call, 10
    runs after a warm-up (median and spread), Gpoints/s, and the algorithmic
    bytes of the call (from its level statistics) per point and per second
    against 8 TB/s.  Returns the results and, per workload, the points and the
    GPU's index list for the CPU-baseline leg."""
    import numpy as np

    from paper_2510_09417_amd import profiling

    res, kept = {}, []
    dev = torch.device("cuda:0")
    for name in CONFIG_LEGS:
        x, y = workloads.workload(name)
        tx, ty = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        oi = torch.empty(len(x), dtype=torch.int64, device=dev)
        oc = torch.empty(1, dtype=torch.int64, device=dev)
        vq.hull_into(tx, ty, oi, oc, stream)
        torch.cuda.synchronize()
        levels = vq.level_stats()
        ms = []
        for _ in range(CONFIG_RUNS):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            vq.hull_into(tx, ty, oi, oc, stream)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        h = int(oc.item())
        med = float(np.median(ms))
        alg = profiling.alg_bytes(len(x), levels)["total"]
        gbs = alg / (med * 1e-3) / 1e9
        res[name] = {"n": len(x), "hull_vertices": h, "levels": len(levels), "median_ms": round(med, 4),
                     "std_ms": round(float(np.std(ms)), 4), "runs": CONFIG_RUNS,
                     "gpoints_per_s": round(len(x) / (med * 1e-3) / 1e9, 3),
                     "alg_bytes_per_point": round(alg / len(x), 2), "alg_gbs": round(gbs, 1),
                     "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        kept.append((name, x, y, oi[:max(h, 0)].cpu().numpy()))
        log(f"{name}: {res[name]}")
        del tx, ty, oi, oc
    torch.cuda.empty_cache()
    return res, kept


def cpu_baseline_leg(oracle, data, npts, configs_kept, served_sample) -> dict:
    """The CPU oracle on the host: the step (disk 10^8 + square 10^8) single-
    threaded and on every core (its multithreaded form, the same lists),
    median of three runs each; every other single-hull workload on every core;
    the sample of served requests one request per thread on every core.  The
    oracle's lists are compared with the GPU's (configurations and served
    sample)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    oracle.load()
    threads = len(os.sched_getaffinity(0))

    def med3(f):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[1], ts

    t1, t1s = med3(lambda: [oracle.hull(x, y) for _, x, y in data])
    tn, tns = med3(lambda: [oracle.hull_mt(x, y, threads) for _, x, y in data])
    log(f"cpu oracle, one step: {t1:.2f} s on 1 core, {tn:.2f} s on {threads} threads")
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    names = " + ".join(n for n, _, _ in data)
    out = {"value": round(npts / tn / 1e9, 5), "unit": "Gpoints/s", "cores": threads, "kind": "oracle",
           "sample": f"one whole step: {names} ({npts} points), the oracle's multithreaded form (OpenMP) on "
                     f"{threads} threads, median of 3 runs ({', '.join(f'{t:.2f}' for t in tns)} s)",
           "single_core": {"value": round(npts / t1 / 1e9, 5), "unit": "Gpoints/s", "cores": 1,
                           "sample": f"the same step single-threaded, median of 3 runs "
                                     f"({', '.join(f'{t:.2f}' for t in t1s)} s)"},
           "host": {"cpu_model": model, "logical_cpus": os.cpu_count(), "threads_used": threads}}
    cfg = {}
    for name, x, y, gpu in configs_kept:
        t0 = time.perf_counter()
        want = oracle.hull_mt(x, y, threads)
        dt = time.perf_counter() - t0
        cfg[name] = {"seconds": round(dt, 3), "gpoints_per_s": round(len(x) / dt / 1e9, 5),
                     "gpu_equals_oracle": bool(np.array_equal(gpu, want))}
        log(f"cpu oracle, {name}: {dt:.2f} s on {threads} threads, GPU list equal: {cfg[name]['gpu_equals_oracle']}")
    out["configs"] = cfg
    if served_sample:
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            wants = list(ex.map(lambda r: oracle.hull(r["x"], r["y"]), served_sample))
        dt = time.perf_counter() - t0
        same = sum(int(r["gpu"] is not None and np.array_equal(r["gpu"], w)) for r, w in zip(served_sample, wants))
        pts = sum(len(r["x"]) for r in served_sample)
        out["served_sample"] = {"requests": len(served_sample), "points": pts, "seconds": round(dt, 3),
                                "hulls_per_s": round(len(served_sample) / dt, 1),
                                "largest_request": max(len(r["x"]) for r in served_sample),
                                "served_equals_oracle": f"{same}/{len(served_sample)}"}
        log(f"cpu oracle, served sample: {len(served_sample)} requests in {dt:.2f} s; served == oracle on "
            f"{same}/{len(served_sample)}")
    return out


def served_benchmark(vq, workloads, torch, nreq: int, lanes: int, lane_points: int = 1 << 25,
                     graph_levels: int = 16) -> tuple[dict, list]:
    """The served mix through vqhull_server_*, against the plain per-request
    path.  Returns the results and a seeded sample of served requests (points
    and index lists, on the host) for the CPU-baseline leg."""
    import numpy as np

    from paper_2510_09417_amd import profiling

    sizes, dists, _ = workloads.served_plan(nreq)
    total = int(sizes.sum())
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    X = torch.empty(total, dtype=torch.float64, device=dev)
    Y = torch.empty(total, dtype=torch.float64, device=dev)
    OUT = torch.empty(total, dtype=torch.int64, device=dev)
    CNT = torch.empty(nreq, dtype=torch.int64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(workloads.SERVED_SEED)
    for d, name in enumerate(workloads.DISTRIBUTIONS):  # one draw per distribution, split into requests
        idx = np.nonzero(dists == d)[0]
        for lo in range(0, len(idx), 4096):
            part = idx[lo:lo + 4096]
            m = int(sizes[part].sum())
            bx = torch.empty(m, dtype=torch.float64, device=dev)
            by = torch.empty(m, dtype=torch.float64, device=dev)
            workloads.device_points_into(name, bx, by, gen)
            k = 0
            for i in part:
                n = int(sizes[i])
                X[off[i]:off[i] + n].copy_(bx[k:k + n])
                Y[off[i]:off[i] + n].copy_(by[k:k + n])
                k += n
    torch.cuda.synchronize()
    log(f"served mix: {nreq} requests, {total} points, generated in {time.perf_counter() - t0:.1f}s")
    # device addresses of every request's arrays (float64 / int64: 8 bytes per entry)
    px = X.data_ptr() + 8 * off[:-1]
    py = Y.data_ptr() + 8 * off[:-1]
    po = OUT.data_ptr() + 8 * off[:-1]
    pc = CNT.data_ptr() + 8 * np.arange(nreq, dtype=np.int64)

    # Autotune the batched kernels on one lane-sized batch of the mix (the
    # first requests up to lane_points points) and serve with the winner;
    # only persistent-grid shapes, which the lanes' captured graphs replay.
    from paper_2510_09417_amd import autotune

    nb = int(np.searchsorted(off, lane_points, side="right")) - 1
    t0 = time.perf_counter()
    tuned, table = autotune.tune_batched(X[: off[nb]], Y[: off[nb]], off[: nb + 1], repeats=5, persistent=(1,))
    saved_cfg = vq.get_config()
    vq.set_config(**tuned)
    tune_s = time.perf_counter() - t0
    log(f"served autotune: {len(table)} configurations on {nb} requests ({int(off[nb])} points) "
        f"in {tune_s:.1f}s -> {tuned}")

    def run(arrivals):
        """Submit request i at arrivals[i] seconds (all that are due in one call)."""
        srv = vq.Server(lanes=lanes, lane_points=lane_points, lane_requests=8192, graph_levels=graph_levels)
        try:
            m = len(arrivals)
            first = None
            i = 0
            t_start = time.perf_counter()
            delay = np.zeros(m)  # scheduled arrival -> submit call, seconds
            while i < m:
                now = time.perf_counter() - t_start
                j = int(np.searchsorted(arrivals, now, side="right"))
                if j <= i:
                    continue
                delay[i:j] = now - arrivals[i:j]
                t = srv.submit_pointers(px[i:j], py[i:j], sizes[i:j], po[i:j], pc[i:j])
                first = t if first is None else first
                i = j
            srv.drain()
            infos = [srv.info(first + k) for k in range(m)]
            st = srv.stats()
        finally:
            srv.close()
        # latency from the scheduled arrival: the wait to be submitted plus
        # submit -> results written on the server's clock
        lat_ms = [1e3 * (delay[k] + infos[k]["t_done"] - infos[k]["t_submit"]) for k in range(m)]
        # the part of it spent waiting for a lane (admission is per batch)
        wait_ms = [1e3 * (delay[k] + infos[k]["t_start"] - infos[k]["t_submit"]) for k in range(m)]
        return infos, st, lat_ms, wait_ms

    # warm-up (lane allocation, first launches)
    run(np.zeros(min(nreq, 256)))
    infos, st, _, _ = run(np.zeros(nreq))
    t_first = min(i["t_submit"] for i in infos)
    t_last = max(i["t_done"] for i in infos)
    thr = nreq / (t_last - t_first)
    bad = sum(1 for i in infos if i["status"] != 0)
    log(f"served throughput: {thr:.0f} hulls/s over {st['batches']} batches")
    counts_served = CNT.cpu().numpy().copy()

    # A seeded sample of the served results, with the requests' points, kept on
    # the host for the CPU-baseline leg (which runs the CPU oracle on them and
    # compares): random requests from the whole mix plus the largest request
    # of every distribution.
    gs = np.random.default_rng(workloads.SERVED_SEED + 3)
    pick = sorted(set(gs.choice(nreq, size=min(nreq, SERVED_SAMPLE), replace=False).tolist())
                  | {int(np.nonzero(dists == d)[0][np.argmax(sizes[dists == d])])
                     for d in range(len(workloads.DISTRIBUTIONS)) if np.any(dists == d)})
    sample = []
    for i in pick:
        a, b = int(off[i]), int(off[i + 1])
        h = int(counts_served[i])
        sample.append({"request": i, "dist": workloads.DISTRIBUTIONS[int(dists[i])],
                       "x": X[a:b].cpu().numpy(), "y": Y[a:b].cpu().numpy(),
                       "gpu": OUT[a:a + max(h, 0)].cpu().numpy() if h >= 0 else None})

    # Algorithmic bytes of the whole mix: the batched path over lane-sized
    # batches of the same requests (the same kernels as the lanes, which sweep
    # level by level: no level pairs here either), with its level statistics
    # (outputs discarded)
    alg_total, lo = 0, 0
    vq.set_level_pairs(0)
    try:
        while lo < nreq:
            hi = max(lo + 1, int(np.searchsorted(off, off[lo] + lane_points, side="right")) - 1)
            hi = min(hi, nreq)
            vq.hull_batched(X[off[lo]:off[hi]], Y[off[lo]:off[hi]], off[lo:hi + 1] - off[lo], check=False)
            alg_total += profiling.alg_bytes_batched(int(off[hi] - off[lo]), vq.level_stats())["total"]
            lo = hi
    finally:
        vq.set_level_pairs(1)
    torch.cuda.synchronize()
    served_gbs = alg_total / (t_last - t_first) / 1e9
    log(f"served: {alg_total / total:.1f} algorithmic B/pt, {served_gbs:.0f} GB/s ({served_gbs / HBM_PEAK_GBS:.3f} "
        f"of {HBM_PEAK_GBS:.0f} GB/s)")

    # latency under Poisson arrivals at half the measured throughput
    nlat = min(nreq, 16384)
    g = np.random.default_rng(workloads.SERVED_SEED + 1)
    arr = np.cumsum(-np.log1p(-g.random(nlat)) / (0.5 * thr))
    linfos, lst, lat, lwait = run(arr)
    log(f"at {0.5 * thr:.0f} hulls/s: served p50 {percentile(lat, 0.50):.3f} p99 {percentile(lat, 0.99):.3f} ms, "
        f"of which waiting for a lane p50 {percentile(lwait, 0.50):.3f} p99 {percentile(lwait, 0.99):.3f} ms")

    # plain path: one synchronous vqhull_hull per request, time-boxed
    stream = torch.cuda.current_stream()
    oi = torch.empty(1 << 20, dtype=torch.int64, device=dev)
    oc = torch.empty(1, dtype=torch.int64, device=dev)
    plain_lat, same = [], 0
    tp0 = time.perf_counter()
    i = 0
    while i < nreq and time.perf_counter() - tp0 < 15.0:
        a = time.perf_counter()
        vq.hull_into(X[off[i]:off[i + 1]], Y[off[i]:off[i + 1]], oi, oc, stream)
        h = int(oc.item())
        plain_lat.append(1e3 * (time.perf_counter() - a))
        if i < 512:
            same += int(h == counts_served[i] and torch.equal(oi[:max(h, 0)], OUT[off[i]:off[i] + max(h, 0)]))
        i += 1
    plain_thr = len(plain_lat) / (time.perf_counter() - tp0)
    checked = min(i, 512)
    log(f"plain path: {plain_thr:.0f} hulls/s over {len(plain_lat)} requests; served == plain on {same}/{checked}")

    # both paths under the same Poisson stream at 0.9 x the plain path's
    # capacity, where both are stable; latency from the scheduled arrival on
    # both (queueing behind earlier requests included)
    nm = min(nreq, 4096)
    lam = 0.9 * plain_thr
    gm = np.random.default_rng(workloads.SERVED_SEED + 2)
    arr_m = np.cumsum(-np.log1p(-gm.random(nm)) / lam)
    _, _, m_served, _ = run(arr_m)
    m_plain = []
    t_start = time.perf_counter()
    for k in range(nm):
        while time.perf_counter() - t_start < arr_m[k]:
            pass
        vq.hull_into(X[off[k]:off[k + 1]], Y[off[k]:off[k + 1]], oi, oc, stream)
        int(oc.item())
        m_plain.append(1e3 * (time.perf_counter() - t_start - arr_m[k]))
    matched = {"rate_hulls_per_s": round(lam, 1), "requests": nm,
               "served_p50_ms": round(percentile(m_served, 0.50), 3),
               "served_p99_ms": round(percentile(m_served, 0.99), 3),
               "plain_p50_ms": round(percentile(m_plain, 0.50), 3),
               "plain_p99_ms": round(percentile(m_plain, 0.99), 3)}
    log(f"at {lam:.0f} hulls/s: served p50 {matched['served_p50_ms']} p99 {matched['served_p99_ms']} ms, "
        f"plain p50 {matched['plain_p50_ms']} p99 {matched['plain_p99_ms']} ms")
    vq.set_config(**saved_cfg)
    return {
        "workload": f"{nreq} requests, sizes log-uniform in [16, 1e6] (seed {workloads.SERVED_SEED}), "
                    f"disk/square/circle/kuzmin, {total} points, drawn on the GPU",
        "lanes": lanes, "lane_points": lane_points, "graph_levels": graph_levels,
        "autotuned_config": {k: tuned[k] for k in ("sweep_block", "sweep_ppt", "lds_limit", "sweep_persistent",
                                                    "level_block")},
        "autotune": f"{len(table)} configurations timed on the first {nb} requests ({int(off[nb])} points), "
                    f"{tune_s:.1f} s",
        "hulls_per_s": round(thr, 1),
        "gpoints_per_s": round(total / (t_last - t_first) / 1e9, 3),
        "alg_bytes_per_point": round(alg_total / total, 2),
        "alg_gbs": round(served_gbs, 1),
        "frac_of_hbm_peak": round(served_gbs / HBM_PEAK_GBS, 4),
        "batches": st["batches"], "graph_batches": st["graph_batches"], "plain_batches": st["plain_batches"],
        "failed": bad,
        "latency_load_hulls_per_s": round(0.5 * thr, 1), "latency_requests": nlat,
        "p50_ms": round(percentile(lat, 0.50), 3), "p99_ms": round(percentile(lat, 0.99), 3),
        "lane_wait_p50_ms": round(percentile(lwait, 0.50), 3), "lane_wait_p99_ms": round(percentile(lwait, 0.99), 3),
        "plain_hulls_per_s": round(plain_thr, 1), "plain_requests": len(plain_lat),
        "plain_p50_ms": round(percentile(plain_lat, 0.50), 3), "plain_p99_ms": round(percentile(plain_lat, 0.99), 3),
        "served_equals_plain": f"{same}/{checked}",
        "matched_rate": matched,
        "latency_from": "scheduled arrival (both paths)",
    }, sample


LEG_BLOCKS = 3


def timed_blocks(torch, step, steps: int) -> list:
    """Wall-clock seconds of LEG_BLOCKS blocks of ``steps`` steps each
    (synchronized before and after every block)."""
    walls = []
    for _ in range(LEG_BLOCKS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    return walls


def prefilter_leg(vq, torch, dx, outs, names, npts, step, args, plain) -> dict:
    """The step again with the octagon prefilter on: wall-clock throughput
    over the same number of steps (the median of three such blocks), equality of every hull with the plain
    path's, the points kept, and the bandwidth of the eight-direction extremes
    pass (16 B per point) and of the filter (16 B read per point, 20 B written
    per kept point) from HIP events on the launch stream."""
    vq.set_config(prefilter=1)
    try:
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        kept = {}
        for name, (tx, ty), (oi, oc) in zip(names, dx, outs):
            vq.hull_into(tx, ty, oi, oc)
            torch.cuda.synchronize()
            kept[name] = vq.level_stats()[0]["swept"]
        same = all(int(oc.item()) == len(p) and torch.equal(oi[: len(p)], p) for (oi, oc), p in zip(outs, plain))
        walls = timed_blocks(torch, step, args.steps)
        wall = sorted(walls)[len(walls) // 2]
        vq.set_timing(True)
        per_kind, ext, filt = {}, [], []
        for _ in range(2):
            for name, (tx, ty), (oi, oc) in zip(names, dx, outs):
                vq.hull_into(tx, ty, oi, oc)
                for r in vq.kernel_times():
                    per_kind[r["kind"]] = per_kind.get(r["kind"], 0.0) + r["ms"]
                    if r["kind"] == "extremes":
                        ext.append((r["ms"], 16 * tx.numel()))
                    elif r["kind"] == "filter":
                        filt.append((r["ms"], 16 * tx.numel() + 20 * kept[name]))
        torch.cuda.synchronize()
        vq.set_timing(False)
    finally:
        vq.set_config(prefilter=0)

    def gbs(recs):
        return round(sum(b for _, b in recs) / (sum(m for m, _ in recs) * 1e-3) / 1e9, 1)

    res = {
        "value": round(npts * args.steps / wall / 1e9, 4),
        "unit": "Gpoints/s",
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "ms_per_step_blocks": [round(1e3 * w / args.steps, 4) for w in walls],
        "same_result_as_plain": bool(same),
        "kept_points": kept,
        "octagon_extremes_gbs": gbs(ext),
        "filter_gbs": gbs(filt),
        "kernel_ms_per_step": {k: round(v / 2, 4) for k, v in per_kind.items()},
    }
    log(f"prefilter: {res['value']} Gpoints/s, same result: {same}, kept {kept}")
    return res


def aos_leg(vq, torch, dx, outs, npts, args, plain, stream) -> dict:
    """The step from interleaved input (one (n, 2) tensor per dataset),
    without and with the prefilter: wall-clock throughput over the same
    number of steps (the median of three such blocks) and equality of every hull with the plain path's."""
    xys = [torch.stack([tx, ty], dim=1).contiguous() for tx, ty in dx]
    res = {}
    try:
        for pf in (0, 1):
            vq.set_config(prefilter=pf)

            def step_xy():
                for xy, (oi, oc) in zip(xys, outs):
                    vq.hull_xy_into(xy, oi, oc, stream)

            for _ in range(args.warmup):
                step_xy()
            torch.cuda.synchronize()
            same = all(int(oc.item()) == len(p) and torch.equal(oi[: len(p)], p) for (oi, oc), p in zip(outs, plain))
            walls = timed_blocks(torch, step_xy, args.steps)
            wall = sorted(walls)[len(walls) // 2]
            res["prefilter" if pf else "plain"] = {"value": round(npts * args.steps / wall / 1e9, 4), "unit": "Gpoints/s",
                                                   "ms_per_step": round(1e3 * wall / args.steps, 4),
                                                   "ms_per_step_blocks": [round(1e3 * w / args.steps, 4) for w in walls],
                                                   "same_result_as_plain": bool(same)}
    finally:
        vq.set_config(prefilter=0)
        del xys
    log(f"aos: {res}")
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--no-prefilter", action="store_true")
    ap.add_argument("--no-aos", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--served-requests", type=int, default=65536)
    ap.add_argument("--served-lanes", type=int, default=8)
    ap.add_argument("--served-lane-points", type=int, default=1 << 25)
    ap.add_argument("--served-graph-levels", type=int, default=16,
                    help="recursion levels each lane's captured batch step holds (deeper batches fall back to "
                         "plain launches)")
    ap.add_argument("--n", type=int, default=100_000_000, help="points per dataset (default 1e8)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is a design that is "
              "not built.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    vq.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    names = ("disk_1e8", "square_1e8")
    data = []
    for name in names:
        t0 = time.perf_counter()
        x, y = workloads.workload(name, n=args.n)
        data.append((name, x, y))
        log(f"generated {name} n={len(x)} in {time.perf_counter() - t0:.1f}s")
    dx = [(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)) for _, x, y in data]
    outs = [(torch.empty(len(x), dtype=torch.int64, device=dev), torch.empty(1, dtype=torch.int64, device=dev))
            for _, x, _ in data]
    npts = sum(len(x) for _, x, _ in data)
    stream = torch.cuda.current_stream()

    def step():
        for (tx, ty), (oi, oc) in zip(dx, outs):
            vq.hull_into(tx, ty, oi, oc, stream)

    # STREAM-Scale probe (context: achievable HBM bandwidth)
    a = torch.empty(args.n, dtype=torch.float64, device=dev).uniform_()
    b = torch.empty_like(a)
    probe = []
    for i in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        vq.stream_scale(a, b, 3.0, stream)
        e1.record(stream)
        e1.synchronize()
        if i:
            probe.append(e0.elapsed_time(e1))
    del a, b
    probe_gbs = 16.0 * args.n / (sorted(probe)[len(probe) // 2] * 1e-3) / 1e9
    log(f"stream-scale probe: {probe_gbs:.0f} GB/s")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hulls = [int(oc.item()) for _, oc in outs]
    log(f"hull sizes: {dict(zip(names, hulls))}")

    def sweep_rec(r):
        """(ms, algorithmic bytes) of a sweep launch: level 0, the argmax pass
        over the caller's arrays, reads 16 B per point; level 1, the fused
        pass, 16 B per point and 20 B per kept point; deeper levels read and
        write 20 B per point."""
        rd = 16 if r["level"] <= 1 else 20
        return (r["ms"], rd * r["points_in"] + 20 * r["points_out"])

    # timed region: timing events around the fused pass (the roofline's
    # kernel) are recorded on the launch stream; no other launch is timed
    # here, since each timed launch adds two timestamped events to the stream
    vq.set_timing(True, fused_only=True)
    lib = vq.load_library()
    recbuf = (vq.KernelTime * 16)()  # the last call's timing records (one: the fused pass), read in place
    fused = []  # (ms, algorithmic bytes) per launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for (tx, ty), (oi, oc) in zip(dx, outs):
            vq.hull_into(tx, ty, oi, oc, stream)
            for i in range(min(16, lib.vqhull_last_kernel_times(recbuf, 16))):
                r = recbuf[i]
                if vq.KERNEL_KINDS[r.kind] == "sweep" and r.level == 1:
                    fused.append(sweep_rec({"level": r.level, "ms": r.ms, "points_in": r.points_in,
                                            "points_out": r.points_out}))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel breakdown: two more steps with every launch timed (outside
    # the timed region: the extra events cost wall time); the argmax pass and
    # all-sweep rates come from these
    vq.set_timing(True)
    per_kind = {}
    argmax, sweeps = [], []
    breakdown_steps = 2
    for _ in range(breakdown_steps):
        for (tx, ty), (oi, oc) in zip(dx, outs):
            vq.hull_into(tx, ty, oi, oc, stream)
            for r in vq.kernel_times():
                per_kind[r["kind"]] = per_kind.get(r["kind"], 0.0) + r["ms"]
                if r["kind"] == "sweep":
                    sweeps.append(sweep_rec(r))
                    if r["level"] == 0:
                        argmax.append(sweep_rec(r))
    torch.cuda.synchronize()
    vq.set_timing(False)
    # per hull: events on the launch stream around each call (first kernel to
    # the count written), 10 runs after one warm-up, median and spread
    per_hull = {}
    for name, (tx, ty), (oi, oc) in zip(names, dx, outs):
        vq.hull_into(tx, ty, oi, oc, stream)
        ms = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            vq.hull_into(tx, ty, oi, oc, stream)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        per_hull[name] = {"median_ms": round(med, 4), "std_ms": round(float(np.std(ms)), 4),
                          "gpoints_per_s": round(tx.numel() / (med * 1e-3) / 1e9, 3)}
    log(f"per hull: {per_hull}")
    # energy per hull: the GPU's energy counter over ~2 s of steps, idle draw
    # subtracted (outside the timed region)
    from paper_2510_09417_amd import energy

    en = ({"available": False, "reason": "--no-energy"} if args.no_energy
          else energy.measure(step, len(names), torch.cuda.synchronize))
    if en.get("available"):
        en["unit"] = "hull (disk 1e8 or square 1e8)"
        en["gpoints_per_joule"] = round(npts / len(names) / 1e9 / en["joules_per_unit"], 3)
        log(f"energy: {en['joules_per_unit']:.4f} J per hull ({en['dynamic_joules_per_unit']:.4f} J above idle "
            f"{en['idle_w']} W)")
    else:
        log(f"energy: not measured ({en.get('reason')})")
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = npts * args.steps / wall / 1e9
    plain = [oi[: int(oc.item())].clone() for oi, oc in outs]
    pre = None if args.no_prefilter else prefilter_leg(vq, torch, dx, outs, names, npts, step, args, plain)
    aos = None if args.no_aos else aos_leg(vq, torch, dx, outs, npts, args, plain, stream)

    def rate(recs):
        ms = sum(m for m, _ in recs)
        by = sum(b for _, b in recs)
        return by / (ms * 1e-3) / 1e9, ms / len(recs), by / len(recs)

    achieved, avg_ms, avg_bytes = rate(fused)
    a_gbs, a_ms, _ = rate(argmax)
    s_gbs, _, _ = rate(sweeps)
    traffic = load_traffic()
    roofline = {
        "bound": "hbm",
        "kernel": "k_sweep fused pass (orient against p->q and the child triangle, farthest points, "
                  "extraction of the four grandchild subsets)",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "bytes_per_launch_alg": int(avg_bytes),
        "avg_launch_ms": round(avg_ms, 4),
        "launches": len(fused),
        "argmax_pass_gbs": round(a_gbs, 1),
        "argmax_pass_ms": round(a_ms, 4),
        "all_sweeps_gbs": round(s_gbs, 1),
        "stream_scale_gbs": round(probe_gbs, 1),
        "frac_of_stream_scale": round(achieved / probe_gbs, 4),
    }

    del dx, outs
    torch.cuda.empty_cache()
    configs, configs_kept = (None, []) if args.no_configs else configs_leg(vq, torch, workloads, stream)

    served, served_sample = None, []
    if not args.no_served:
        served, served_sample = served_benchmark(vq, workloads, torch, args.served_requests, args.served_lanes,
                                                 args.served_lane_points, args.served_graph_levels)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        cpu = cpu_baseline_leg(oracle, data, npts, configs_kept, served_sample)
        for name, r in cpu["configs"].items():
            configs[name]["gpu_equals_oracle"] = r["gpu_equals_oracle"]
        if served is not None and "served_sample" in cpu:
            served["served_equals_oracle"] = cpu["served_sample"]["served_equals_oracle"]

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{'+'.join(names)} (uniform disk and unit square, seed 2)",
                   "points_per_step": npts, "hull_sizes": hulls},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": {k: round(v / breakdown_steps, 4) for k, v in per_kind.items()},
        "per_hull": per_hull,
        "energy": en,
        "prefilter": pre,
        "aos": aos,
        "configs": configs,
        "served": served,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
