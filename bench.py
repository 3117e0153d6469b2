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
              during the timed steps, against 8 TB/s;
  per_hull    each dataset's hull alone: HIP events on the launch stream
              around the call (first kernel to the count written), 10 runs
              after a warm-up, median and standard deviation.
  cpu_baseline  the CPU oracle (single thread) on one whole step.
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
              time-boxed prefix of the same mix; and a check that served results
              equal the plain path's on a sample.

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


def served_benchmark(vq, workloads, torch, nreq: int, lanes: int, lane_points: int = 1 << 25) -> dict:
    """The served mix through vqhull_server_*, against the plain per-request path."""
    import numpy as np

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
    tuned, table = autotune.tune_batched(X[: off[nb]], Y[: off[nb]], off[: nb + 1], repeats=3, persistent=(1,))
    saved_cfg = vq.get_config()
    vq.set_config(**tuned)
    tune_s = time.perf_counter() - t0
    log(f"served autotune: {len(table)} configurations on {nb} requests ({int(off[nb])} points) "
        f"in {tune_s:.1f}s -> {tuned}")

    def run(arrivals):
        """Submit request i at arrivals[i] seconds (all that are due in one call)."""
        srv = vq.Server(lanes=lanes, lane_points=lane_points, lane_requests=8192)
        try:
            m = len(arrivals)
            first = None
            i = 0
            t_start = time.perf_counter()
            while i < m:
                now = time.perf_counter() - t_start
                j = int(np.searchsorted(arrivals, now, side="right"))
                if j <= i:
                    continue
                t = srv.submit_pointers(px[i:j], py[i:j], sizes[i:j], po[i:j], pc[i:j])
                first = t if first is None else first
                i = j
            srv.drain()
            infos = [srv.info(first + k) for k in range(m)]
            st = srv.stats()
        finally:
            srv.close()
        return infos, st

    # warm-up (lane allocation, first launches)
    run(np.zeros(min(nreq, 256)))
    infos, st = run(np.zeros(nreq))
    t_first = min(i["t_submit"] for i in infos)
    t_last = max(i["t_done"] for i in infos)
    thr = nreq / (t_last - t_first)
    bad = sum(1 for i in infos if i["status"] != 0)
    log(f"served throughput: {thr:.0f} hulls/s over {st['batches']} batches")
    counts_served = CNT.cpu().numpy().copy()

    # latency under Poisson arrivals at half the measured throughput
    nlat = min(nreq, 16384)
    g = np.random.default_rng(workloads.SERVED_SEED + 1)
    arr = np.cumsum(-np.log1p(-g.random(nlat)) / (0.5 * thr))
    linfos, lst = run(arr)
    lat = [1e3 * (i["t_done"] - i["t_submit"]) for i in linfos]

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
    # capacity, where both are stable; latency from the scheduled arrival
    # (plain: queueing behind earlier requests included)
    nm = min(nreq, 4096)
    lam = 0.9 * plain_thr
    gm = np.random.default_rng(workloads.SERVED_SEED + 2)
    arr_m = np.cumsum(-np.log1p(-gm.random(nm)) / lam)
    minfos, _ = run(arr_m)
    m_served = [1e3 * (i["t_done"] - i["t_submit"]) for i in minfos]
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
        "lanes": lanes, "lane_points": lane_points,
        "autotuned_config": {k: tuned[k] for k in ("sweep_block", "sweep_ppt", "lds_limit", "sweep_persistent",
                                                    "level_block")},
        "autotune": f"{len(table)} configurations timed on the first {nb} requests ({int(off[nb])} points), "
                    f"{tune_s:.1f} s",
        "hulls_per_s": round(thr, 1),
        "gpoints_per_s": round(total / (t_last - t_first) / 1e9, 3),
        "batches": st["batches"], "graph_batches": st["graph_batches"], "plain_batches": st["plain_batches"],
        "failed": bad,
        "latency_load_hulls_per_s": round(0.5 * thr, 1), "latency_requests": nlat,
        "p50_ms": round(percentile(lat, 0.50), 3), "p99_ms": round(percentile(lat, 0.99), 3),
        "plain_hulls_per_s": round(plain_thr, 1), "plain_requests": len(plain_lat),
        "plain_p50_ms": round(percentile(plain_lat, 0.50), 3), "plain_p99_ms": round(percentile(plain_lat, 0.99), 3),
        "served_equals_plain": f"{same}/{checked}",
        "matched_rate": matched,
    }


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
    ap.add_argument("--served-requests", type=int, default=65536)
    ap.add_argument("--served-lanes", type=int, default=4)
    ap.add_argument("--served-lane-points", type=int, default=1 << 25)
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

    # timed region: timing events around the partition sweeps are recorded on
    # the launch stream (the roofline's kernel durations)
    vq.set_timing(True, sweeps_only=True)
    fused, argmax, sweeps = [], [], []  # (ms, algorithmic bytes) per launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for (tx, ty), (oi, oc) in zip(dx, outs):
            vq.hull_into(tx, ty, oi, oc, stream)
            for r in vq.kernel_times():
                if r["kind"] != "sweep":
                    continue
                # level 0: argmax pass over the caller's arrays (16 B read per point);
                # level 1: fused pass (16 B read per point, 20 B per kept point);
                # deeper levels read and write 20 B per point.
                rd = 16 if r["level"] <= 1 else 20
                rec = (r["ms"], rd * r["points_in"] + 20 * r["points_out"])
                sweeps.append(rec)
                if r["level"] == 0:
                    argmax.append(rec)
                elif r["level"] == 1:
                    fused.append(rec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel breakdown: two more steps with every launch timed (outside
    # the timed region: the extra events cost wall time)
    vq.set_timing(True)
    per_kind = {}
    breakdown_steps = 2
    for _ in range(breakdown_steps):
        for (tx, ty), (oi, oc) in zip(dx, outs):
            vq.hull_into(tx, ty, oi, oc, stream)
            for r in vq.kernel_times():
                per_kind[r["kind"]] = per_kind.get(r["kind"], 0.0) + r["ms"]
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

    served = None
    if not args.no_served:
        del dx, outs
        torch.cuda.empty_cache()
        served = served_benchmark(vq, workloads, torch, args.served_requests, args.served_lanes,
                                  args.served_lane_points)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.load()
        t0 = time.perf_counter()
        for _, x, y in data:
            oracle.hull(x, y)
        tc = time.perf_counter() - t0
        model = "unknown"
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
        except OSError:
            pass
        cpu = {"value": round(npts / tc / 1e9, 5), "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
               "sample": f"one whole step: {' + '.join(names)} ({npts} points), single-threaded C oracle, "
                         f"{tc:.2f} s",
               "host": {"cpu_model": model, "logical_cpus": os.cpu_count()}}
        log(f"cpu oracle: {tc:.2f}s for one step")

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
        "served": served,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
