"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_2510_09417_amd.profiling stats  <kernel_stats.csv> <out.md> "<command>"
    python -m paper_2510_09417_amd.profiling traffic <fetch counter_collection.csv> <write counter_collection.csv>
            <out.json> <out.md> "<fetch command>" "<write command>" [elements of the probe, default 1e8]

    python -m paper_2510_09417_amd.profiling hull-run <workload>
    python -m paper_2510_09417_amd.profiling size-sweep <out.md>
    python -m paper_2510_09417_amd.profiling sq-counters <pass-1 counter_collection.csv>
            <pass-2 counter_collection.csv> <hull-run output> <out.md> "<pass-1 command>" "<pass-2 command>"
    python -m paper_2510_09417_amd.profiling hull-bytes <out.md> "<fetch command>" "<write command>"
            <workload> <fetch counter_collection.csv> <write counter_collection.csv> <hull-run output> [...]

``hull-run`` is the GPU program the whole-hull counters are taken on: the
STREAM-Scale probe, then two plain hull calls on the named workload, then one
JSON line with the level statistics.  ``hull-bytes`` sums the calibrated
counters of every library kernel of those calls and sets the measured bytes
per input point beside the algorithmic bytes computed from the level
statistics (``alg_bytes``).

``traffic`` calibrates the byte counters on the STREAM-Scale probe kernel, which
reads and writes exactly 8 bytes per element: factor = known bytes / counted
bytes, separately for FETCH_SIZE and WRITE_SIZE.  The fused sweep's counted
bytes per dispatch (template mode 2 of k_sweep), times those factors, give its
measured HBM traffic per launch.  The JSON records the hash of the fused pass's source (``fused_source``)
it was taken on; the benchmark ignores it once that source has changed.
"""
from __future__ import annotations

import csv
import hashlib
import re
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "vqhull_kernels.hip")
SWEEP = "k_sweep<"
FUSED_MODE = ", 2>"  # k_sweep<BLOCK, PPT, MODE>: mode 2 is the fused top-level pass
PROBE = "k_stream_scale"


HEADER_SRC = os.path.join(HERE, "csrc", "vqhull_internal.h")
SWEEP_END = "// --------------------------------------------------------- block utilities"
LAUNCH_BEGIN = "int sweep_one("
LAUNCH_END = "int launch_plan0("


def fused_source(kernels: str, header: str) -> str:
    """The source the fused pass is built from: the kernel file up to the end
    of the sweep kernel (every device function it calls sits above it), the
    sweep launchers and grid sizing, and the shared header.  The planners,
    finisher and assembly below the sweep do not enter its code."""
    head = kernels.split(SWEEP_END, 1)[0]
    launch = kernels[kernels.index(LAUNCH_BEGIN):kernels.index(LAUNCH_END)]
    return head + "\n" + launch + "\n" + header


def code_only(src: str) -> str:
    """Source without comments and blank lines: comments do not change the code.
    (Simple textual stripping; no string literal in these sources contains a
    comment marker.)"""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_source_hash() -> str:
    with open(KERNEL_SRC) as f, open(HEADER_SRC) as g:
        return hashlib.sha256(code_only(fused_source(f.read(), g.read())).encode()).hexdigest()[:16]


def short(name: str) -> str:
    name = name.replace("(vqh::SweepArgs)", "").replace("void ", "")
    if len(name) > 70:
        name = name[:67] + "..."
    return name


def stats(path: str, out: str, command: str) -> None:
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_kernel(path: str, counter: str) -> dict:
    agg = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return agg


def _pick(agg: dict, pred) -> list:
    vals = []
    for k, v in agg.items():
        if pred(k):
            vals += v
    return vals


def traffic(fetch_csv: str, write_csv: str, out_json: str, out_md: str, fetch_cmd: str, write_cmd: str,
            probe_elems: float = 1e8) -> dict:
    fa, wa = _per_kernel(fetch_csv, "FETCH_SIZE"), _per_kernel(write_csv, "WRITE_SIZE")
    is_l0 = lambda k: SWEEP in k and FUSED_MODE in k
    is_probe = lambda k: PROBE in k
    f_probe, w_probe = _pick(fa, is_probe), _pick(wa, is_probe)
    f_l0, w_l0 = _pick(fa, is_l0), _pick(wa, is_l0)
    if not (f_probe and w_probe and f_l0 and w_l0):
        raise SystemExit("missing probe or fused sweep dispatches in the counter files")
    mean = lambda v: sum(v) / len(v)
    known = 8.0 * probe_elems  # bytes read (and written) by the probe
    ff = known / (mean(f_probe) * 1024.0)
    fw = known / (mean(w_probe) * 1024.0)
    fetch_b = mean(f_l0) * 1024.0 * ff
    write_b = mean(w_l0) * 1024.0 * fw
    res = {
        "kernel": "k_sweep fused pass",
        "bytes_per_launch": int(fetch_b + write_b),
        "fetch_bytes_per_launch": int(fetch_b),
        "write_bytes_per_launch": int(write_b),
        "fetch_size_kib_per_dispatch": round(mean(f_l0), 1),
        "write_size_kib_per_dispatch": round(mean(w_l0), 1),
        "probe_fetch_kib": round(mean(f_probe), 1),
        "probe_write_kib": round(mean(w_probe), 1),
        "fetch_scale": round(ff, 4),
        "write_scale": round(fw, 4),
        "dispatches": len(f_l0),
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    lines = ["# HBM traffic of the fused top-level sweep (rocprofv3 counters)", "",
             f"FETCH_SIZE command: `{fetch_cmd}`", "", f"WRITE_SIZE command: `{write_cmd}`", "",
             "Calibration: the STREAM-Scale probe reads and writes exactly 8 bytes per element "
             f"({probe_elems:.0f} elements); scale = known bytes / counted bytes.", "",
             "| quantity | value |", "|---|---|",
             f"| probe FETCH_SIZE (KiB/dispatch) | {res['probe_fetch_kib']} |",
             f"| probe WRITE_SIZE (KiB/dispatch) | {res['probe_write_kib']} |",
             f"| fetch scale | {res['fetch_scale']} |",
             f"| write scale | {res['write_scale']} |",
             f"| fused sweep FETCH_SIZE (KiB/dispatch, {len(f_l0)} dispatches) | {res['fetch_size_kib_per_dispatch']} |",
             f"| fused sweep WRITE_SIZE (KiB/dispatch) | {res['write_size_kib_per_dispatch']} |",
             f"| fused sweep fetched bytes per launch (scaled) | {res['fetch_bytes_per_launch']} |",
             f"| fused sweep written bytes per launch (scaled) | {res['write_bytes_per_launch']} |",
             f"| fused sweep HBM traffic per launch | {res['bytes_per_launch']} |",
             f"| fused-pass code sha256[:16] (kernel file up to the sweep kernel, sweep launchers, shared header; comments stripped) | `{res['kernel_source_sha256_16']}` |"]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return res


HULL_RUN_CALLS = 2


def hull_run(name: str) -> None:
    """The program profiled for ``hull_bytes`` (see the module docstring)."""
    import torch

    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    vq.load_library()
    x, y = workloads.workload(name)
    n = len(x)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    del x, y
    a = torch.empty(100_000_000, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a)
    vq.stream_scale(a, b, 3.0)
    torch.cuda.synchronize()
    del a, b
    oi = torch.empty(n, dtype=torch.int64, device="cuda")
    oc = torch.empty(1, dtype=torch.int64, device="cuda")
    for _ in range(HULL_RUN_CALLS):
        vq.hull_into(tx, ty, oi, oc)
    torch.cuda.synchronize()
    print(json.dumps({"workload": name, "n": n, "calls": HULL_RUN_CALLS, "h": int(oc.item()),
                      "levels": vq.level_stats(), "config": vq.get_config()}), flush=True)


SIZE_SWEEP_SIZES = (10**5, 10**6, 10**7, 10**8, 10**9, 2**31 - 1)


def size_sweep(out_md: str, dists=("disk", "square"), sizes=SIZE_SWEEP_SIZES, calls: int = 5) -> list:
    """Per-hull time against n: for each distribution and size, points drawn
    on the GPU (seeded torch generator), two warm-up calls, then the median of
    ``calls`` plain hull calls timed with HIP events on the call's stream.
    Writes a markdown table (time, Gpoints/s, algorithmic bytes per point and
    their rate against 8 TB/s) and prints one JSON line per case."""
    import torch

    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    vq.load_library()
    rows = []
    for dist in dists:
        for n in sizes:
            g = torch.Generator(device="cuda")
            g.manual_seed(7)
            x = torch.empty(n, dtype=torch.float64, device="cuda")
            y = torch.empty(n, dtype=torch.float64, device="cuda")
            workloads.device_points_into(dist, x, y, g)
            oi = torch.empty(n, dtype=torch.int64, device="cuda")
            oc = torch.empty(1, dtype=torch.int64, device="cuda")
            for _ in range(2):
                vq.hull_into(x, y, oi, oc)
            ms = []
            st = torch.cuda.current_stream()
            for _ in range(calls):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                vq.hull_into(x, y, oi, oc)
                e1.record(st)
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            ms.sort()
            t = ms[len(ms) // 2]
            alg = alg_bytes(n, vq.level_stats())["total"]
            row = {"dist": dist, "n": n, "h": int(oc.item()), "median_ms": round(t, 4),
                   "gpoints_per_s": round(n / t / 1e6, 2), "alg_bytes_per_point": round(alg / n, 1),
                   "alg_gbs": round(alg / t / 1e6, 1)}
            rows.append(row)
            print(json.dumps(row), flush=True)
            del x, y, oi, oc
            vq.release_workspace()
            torch.cuda.empty_cache()
    lines = ["# Per-hull time against the number of points (plain hull call, one MI355X)", "",
             f"Command: `python3 -m paper_2510_09417_amd.profiling size-sweep {out_md}`", "",
             f"Points drawn on the GPU (uniform disk and unit square, torch generator seed 7); two warm-up calls, then the "
             f"median of {calls} calls timed with HIP events on the call's stream; benchmark configuration.  Algorithmic "
             "bytes per point from the call's level statistics (`alg_bytes`); their rate is set against 8 TB/s.", "",
             "| distribution | n | h | median ms | Gpoints/s | algorithmic B/pt | algorithmic GB/s | of 8 TB/s |",
             "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['dist']} | {r['n']:,} | {r['h']} | {r['median_ms']:.3f} | {r['gpoints_per_s']:.1f} | "
                     f"{r['alg_bytes_per_point']:.1f} | {r['alg_gbs']:.0f} | {r['alg_gbs'] / 8000:.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def _deep_terms(levels: list) -> tuple:
    """(writes, level reads) in bytes of the levels below the top, 20 B per
    point moved.  Level k's jobs are written once (by sweep k-1, or as
    pass-through copies by a fused sweep k); its segments are written by sweep
    k-1 unless that sweep was an argmax pass (then they are read in place).
    Sweep k reads its own segments' points, or a fused sweep those of level
    k-1 again."""
    sw = [lv["swept"] for lv in levels]
    jp = [lv["job_points"] for lv in levels]
    kind = [lv.get("sweep", "level") for lv in levels]
    writes = 20 * ((jp[1] if len(jp) > 1 else 0)
                   + sum(jp[k] + (sw[k] if kind[k - 1] != "argmax" else 0) for k in range(2, len(levels))))
    reads = 20 * sum(sw[k - 1] if kind[k] == "fused" else sw[k] for k in range(2, len(levels)))
    return writes, reads


def alg_bytes_batched(n_total: int, levels: list) -> dict:
    """Algorithmic bytes of one batched call (any mix of request sizes) from
    its level statistics: extremes 8 B per point (x) of every request; the
    requests above the LDS threshold (level 0's segments, ``swept[0]``
    points) are read twice at 16 B per point (argmax and fused passes); the
    requests at most the threshold (level 0's jobs) are read once by the LDS
    finisher at 16 B per point; deeper levels as in ``alg_bytes``."""
    sw = [lv["swept"] for lv in levels]
    jp = [lv["job_points"] for lv in levels]
    top = 8 * n_total + 32 * (sw[0] if sw else 0) + 16 * (jp[0] if jp else 0)
    writes, level_reads = _deep_terms(levels)
    finisher = 20 * sum(jp[k] for k in range(1, len(levels)))
    total = top + writes + level_reads + finisher
    return {"top": top, "writes": writes, "level_reads": level_reads, "finisher_reads": finisher, "total": total}


def alg_bytes(n: int, levels: list) -> dict:
    """Algorithmic bytes of one plain hull of a single request of more than
    the LDS threshold's points, from its level statistics (level k: segments
    swept and points of the jobs created):
      extremes 8 B per point (x); argmax pass 16 B per point; fused pass 16 B
      per point read, and 20 B written per point of the level-1 jobs (copies)
      and of the level-2 segments and jobs (grandchildren); level k >= 2:
      20 B read per swept point, 20 B written per point of level k+1's
      segments and jobs (a level pair: the second level re-reads the first's
      points and the first writes none); the LDS finisher reads 20 B per job
      point.
    Vertex lists and the output (O(h)) are left out."""
    sw = [lv["swept"] for lv in levels]
    jp = [lv["job_points"] for lv in levels]
    top = 8 * n + 16 * n + 16 * n
    writes, level_reads = _deep_terms(levels)
    finisher = 20 * sum(jp[k] for k in range(1, len(levels)))
    total = top + writes + level_reads + finisher
    return {"top": top, "writes": writes, "level_reads": level_reads, "finisher_reads": finisher, "total": total}


def hull_bytes(out_md: str, fetch_cmd: str, write_cmd: str, runs: list, probe_elems: float = 1e8) -> list:
    """runs: (workload, fetch csv, write csv, hull-run output file) per workload."""
    rows = []
    for name, fcsv, wcsv, run_out in runs:
        run = json.loads([ln for ln in open(run_out).read().splitlines() if ln.startswith("{")][-1])
        fa, wa = _per_kernel(fcsv, "FETCH_SIZE"), _per_kernel(wcsv, "WRITE_SIZE")
        is_probe = lambda k: PROBE in k
        is_lib = lambda k: "vqh::" in k and PROBE not in k
        mean = lambda v: sum(v) / len(v)
        known = 8.0 * probe_elems
        ff = known / (mean(_pick(fa, is_probe)) * 1024.0)
        fw = known / (mean(_pick(wa, is_probe)) * 1024.0)
        fetched = sum(_pick(fa, is_lib)) * 1024.0 * ff / run["calls"]
        written = sum(_pick(wa, is_lib)) * 1024.0 * fw / run["calls"]
        alg = alg_bytes(run["n"], run["levels"])
        rows.append((name, run, fetched, written, alg))
    lines = ["# Bytes per input point of one whole hull: rocprofv3 counters against the algorithmic bytes", "",
             f"FETCH_SIZE command (per workload W): `{fetch_cmd}`", "",
             f"WRITE_SIZE command (per workload W): `{write_cmd}`", "",
             "Every library kernel of the two plain hull calls is summed (the probe and torch's own kernels "
             "excluded) and divided by the two calls; the counters are calibrated on the STREAM-Scale probe "
             "(known bytes / counted bytes, per counter).  Algorithmic bytes: "
             "`paper_2510_09417_amd.profiling.alg_bytes` on the calls' level statistics.", "",
             "| workload | n | h | levels | algorithmic (GB) | alg. B/pt | fetched (GB) | written (GB) | measured (GB) "
             "| measured B/pt | measured / algorithmic |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, run, fetched, written, alg in rows:
        n = run["n"]
        meas = fetched + written
        lines.append(f"| {name} | {n} | {run['h']} | {len(run['levels'])} | {alg['total'] / 1e9:.3f} | "
                     f"{alg['total'] / n:.1f} | {fetched / 1e9:.3f} | {written / 1e9:.3f} | {meas / 1e9:.3f} | "
                     f"{meas / n:.1f} | {meas / alg['total']:.3f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


SQ_KINDS = (("fused pass", lambda k: SWEEP in k and FUSED_MODE in k),
            ("argmax pass", lambda k: SWEEP in k and ", 1>" in k),
            ("extremes", lambda k: "k_extremes" in k),
            ("level sweeps (all levels)", lambda k: SWEEP in k and ", 0>" in k))


def _sums(path: str) -> dict:
    agg = {}
    for r in csv.DictReader(open(path)):
        a = agg.setdefault(short(r["Kernel_Name"]), {})
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        a.setdefault("_dispatches", set()).add(r.get("Dispatch_Id"))
    return agg


def sq_counters(csv1: str, csv2: str, run_out: str, out_md: str, cmd1: str, cmd2: str) -> list:
    """Issue and wait counters of the partition sweeps from two rocprofv3
    --pmc passes over ``hull-run`` (pass 1: wave cycles and activity; pass 2:
    instruction counts).  Points per kernel from the run's level statistics:
    n per call for the extremes, argmax and fused passes, the swept points of
    levels >= 2 for the level sweeps.  Instructions per point are wave
    instructions x 64 / points."""
    run = json.loads([ln for ln in open(run_out).read().splitlines() if ln.startswith("{")][-1])
    n, calls = run["n"], run["calls"]
    lv = run["levels"]
    pts = {"fused pass": n * calls, "argmax pass": n * calls, "extremes": n * calls,
           "level sweeps (all levels)": sum(l["swept"] for l in lv[2:]) * calls}
    a1, a2 = _sums(csv1), _sums(csv2)
    rows = []
    for name, pred in SQ_KINDS:
        c = {}
        disp = 0
        for agg in (a1, a2):
            for k, v in agg.items():
                if pred(k):
                    disp = max(disp, len(v["_dispatches"]))
                    for key, val in v.items():
                        if key != "_dispatches":
                            c[key] = c.get(key, 0.0) + val
        if not c or not pts[name]:
            continue
        wc = c.get("SQ_WAVE_CYCLES", 0.0) or 1.0
        per = lambda key: 64.0 * c.get(key, 0.0) / pts[name]
        rows.append((name, disp, c.get("SQ_WAIT_ANY", 0.0) / wc, c.get("SQ_WAIT_INST_ANY", 0.0) / wc,
                     c.get("SQ_ACTIVE_INST_ANY", 0.0) / wc, c.get("SQ_ACTIVE_INST_VALU", 0.0) / wc,
                     per("SQ_INSTS_VALU"), per("SQ_INSTS_SALU"), per("SQ_INSTS_VMEM_RD"), per("SQ_INSTS_VMEM_WR"), c))
    lines = [f"# Issue and wait counters of the partition sweeps (rocprofv3 SQ counters, {run['workload']})", "",
             f"Pass 1: `{cmd1}`", "", f"Pass 2: `{cmd2}`", "",
             f"{calls} plain hull calls (n = {n:,}, h = {run['h']}) under the configuration "
             f"{run['config']}.  Counters are summed over each kernel's dispatches in both calls; ratios are taken "
             "against SQ_WAVE_CYCLES (the waves' resident cycles); instructions per point are wave instructions "
             "x 64 / (points that kernel swept).", "",
             "| kernel | dispatches | waiting (WAIT_ANY / WAVE_CYCLES) | waiting on a dependency (WAIT_INST_ANY) "
             "| issuing any (ACTIVE_INST_ANY) | issuing VALU (ACTIVE_INST_VALU) | VALU instr / pt | SALU instr / pt "
             "| vector loads / pt | vector stores / pt |", "|---|---|---|---|---|---|---|---|---|---|"]
    for name, disp, w, wi, ai, av, va, sa, vr, vw, _ in rows:
        lines.append(f"| {name} | {disp} | {w:.3f} | {wi:.3f} | {ai:.3f} | {av:.3f} | {va:.1f} | {sa:.1f} | "
                     f"{vr:.1f} | {vw:.1f} |")
    lines += ["", "Raw sums:", "", "| kernel | counter | sum |", "|---|---|---|"]
    for name, *_, c in rows:
        for key in sorted(c):
            lines.append(f"| {name} | {key} | {c[key]:.0f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


if __name__ == "__main__":
    if sys.argv[1] == "hull-run":
        hull_run(sys.argv[2])
    elif sys.argv[1] == "hull-bytes":
        rest = sys.argv[5:]
        hull_bytes(sys.argv[2], sys.argv[3], sys.argv[4], [tuple(rest[i:i + 4]) for i in range(0, len(rest), 4)])
    elif sys.argv[1] == "sq-counters":
        sq_counters(*sys.argv[2:8])
    elif sys.argv[1] == "size-sweep":
        size_sweep(sys.argv[2])
    elif sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], sys.argv[7],
                float(sys.argv[8]) if len(sys.argv) > 8 else 1e8)
    else:
        raise SystemExit(__doc__)
