"""The rocprofv3 summary helpers (CPU): the fused pass's source hash follows
the code the fused pass is built from and nothing else, and the traffic
calibration scales the counters on the probe kernel."""
import csv

from paper_2510_09417_amd import profiling as P


def _sources():
    with open(P.KERNEL_SRC) as f, open(P.HEADER_SRC) as g:
        return f.read(), g.read()


def test_fused_source_hash_scope():
    k, h = _sources()
    base = P.fused_source(k, h)
    assert P.SWEEP_END in k and P.LAUNCH_BEGIN in k and P.LAUNCH_END in k
    # below the sweep kernel (planners, finisher, assembly): not part of it
    i = k.index(P.SWEEP_END) + len(P.SWEEP_END)
    assert P.fused_source(k[:i] + "\n// planner note\n" + k[i:], h) == base
    # inside the sweep section, in its launchers or in the shared header: part of it
    j = k.index("__global__ __launch_bounds__(BLOCK) void k_sweep")
    assert P.fused_source(k[:j] + "// x\n" + k[j:], h) != base
    m = k.index(P.LAUNCH_BEGIN) + len(P.LAUNCH_BEGIN)
    assert P.fused_source(k[:m] + "\n// x\n" + k[m:], h) != base
    assert P.fused_source(k, h + "// x\n") != base


def test_hash_ignores_comments_only():
    k, h = _sources()
    base = P.kernel_source_hash()
    j = k.index("__global__ __launch_bounds__(BLOCK) void k_sweep")
    same = P.code_only(P.fused_source(k[:j] + "// a note\n/* more */\n" + k[j:], h))
    assert same == P.code_only(P.fused_source(k, h))
    assert P.code_only("a = 1; // c\n/* x\n y */ b = 2;\n\n") == "a = 1;\n  b = 2;"
    assert base == P.kernel_source_hash()


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_calibration(tmp_path):
    n = 1000
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    # probe: 8 B read and 8 B written per element; counters in KiB, FETCH_SIZE reads half
    _write_counters(fetch, [
        {"Dispatch_Id": 1, "Kernel_Name": "vqh::k_stream_scale(double const*, double*, unsigned long, double)",
         "Counter_Name": "FETCH_SIZE", "Counter_Value": 8 * n / 1024 / 2},
        {"Dispatch_Id": 2, "Kernel_Name": "void vqh::k_sweep<512, 8, 2>(vqh::SweepArgs)",
         "Counter_Name": "FETCH_SIZE", "Counter_Value": 100.0},
    ])
    _write_counters(write, [
        {"Dispatch_Id": 1, "Kernel_Name": "vqh::k_stream_scale(double const*, double*, unsigned long, double)",
         "Counter_Name": "WRITE_SIZE", "Counter_Value": 8 * n / 1024},
        {"Dispatch_Id": 2, "Kernel_Name": "void vqh::k_sweep<512, 8, 2>(vqh::SweepArgs)",
         "Counter_Name": "WRITE_SIZE", "Counter_Value": 50.0},
    ])
    out_json, out_md = tmp_path / "t.json", tmp_path / "t.md"
    P.traffic(str(fetch), str(write), str(out_json), str(out_md), "fetch cmd", "write cmd", n)
    import json

    t = json.loads(out_json.read_text())
    assert abs(t["fetch_scale"] - 2.0) < 1e-9 and abs(t["write_scale"] - 1.0) < 1e-9
    assert t["fetch_bytes_per_launch"] == 2 * 100 * 1024 and t["write_bytes_per_launch"] == 50 * 1024
    assert t["bytes_per_launch"] == 2 * 100 * 1024 + 50 * 1024
    assert t["kernel_source_sha256_16"] == P.kernel_source_hash()
    assert "fetch cmd" in out_md.read_text()


def test_alg_bytes_counts_every_move():
    from paper_2510_09417_amd import profiling

    levels = [dict(segments=1, swept=100, jobs=0, job_points=0),   # roots
              dict(segments=2, swept=90, jobs=1, job_points=5),    # children of the roots (not written)
              dict(segments=2, swept=30, jobs=2, job_points=10),   # grandchildren (written by the fused pass)
              dict(segments=0, swept=0, jobs=3, job_points=6)]     # written by the level-2 sweep
    b = profiling.alg_bytes(100, levels)
    assert b["top"] == (8 + 16 + 16) * 100
    assert b["writes"] == 20 * (5 + 30 + 10 + 0 + 6)
    assert b["level_reads"] == 20 * 30
    assert b["finisher_reads"] == 20 * (5 + 10 + 6)
    assert b["total"] == b["top"] + b["writes"] + b["level_reads"] + b["finisher_reads"]


def test_alg_bytes_level_pair():
    """A level pair at levels 2 and 3: level 3's segments are never written
    (read in place from level 2's range), its jobs are copied by the fused
    sweep, and sweep 3 reads level 2's points again."""
    from paper_2510_09417_amd import profiling

    levels = [dict(segments=1, swept=100, jobs=0, job_points=0, sweep="argmax"),
              dict(segments=2, swept=90, jobs=1, job_points=5, sweep="fused"),
              dict(segments=4, swept=80, jobs=0, job_points=0, sweep="argmax"),
              dict(segments=8, swept=70, jobs=4, job_points=20, sweep="fused"),
              dict(segments=0, swept=0, jobs=3, job_points=6, sweep="level")]
    b = profiling.alg_bytes(100, levels)
    assert b["writes"] == 20 * (5 + (0 + 80) + (20 + 0) + (6 + 0))
    assert b["level_reads"] == 20 * (80 + 80 + 0)
    assert b["finisher_reads"] == 20 * (5 + 0 + 20 + 6)
    plain = [dict(lv, sweep="level") for lv in levels]  # the same counts swept level by level
    assert profiling.alg_bytes(100, plain)["total"] - b["total"] == 20 * (70 + 70 - 80)


def test_alg_bytes_batched_reduces_to_single_and_counts_small_requests():
    from paper_2510_09417_amd import profiling

    levels = [dict(segments=1, swept=100, jobs=0, job_points=0),
              dict(segments=2, swept=90, jobs=1, job_points=5),
              dict(segments=2, swept=30, jobs=2, job_points=10),
              dict(segments=0, swept=0, jobs=3, job_points=6)]
    assert profiling.alg_bytes_batched(100, levels) == profiling.alg_bytes(100, levels)
    # a request of 100 points above the LDS threshold and two small ones of 7
    # and 9 points (root jobs: read once by the finisher)
    mixed = [dict(segments=1, swept=100, jobs=2, job_points=16)] + levels[1:]
    b = profiling.alg_bytes_batched(116, mixed)
    assert b["top"] == 8 * 116 + 32 * 100 + 16 * 16
    assert b["total"] - b["top"] == profiling.alg_bytes(100, levels)["total"] - profiling.alg_bytes(100, levels)["top"]
    only_small = [dict(segments=0, swept=0, jobs=3, job_points=40)]
    assert profiling.alg_bytes_batched(40, only_small)["total"] == 8 * 40 + 16 * 40


def test_sq_counters_summary(tmp_path):
    """Per-kernel sums of two counter passes, ratios against the waves'
    resident cycles, and instructions per point from the run's levels."""
    import csv

    from paper_2510_09417_amd import profiling as P

    fused = "void vqh::k_sweep<256, 16, 2>(vqh::SweepArgs)"
    level = "void vqh::k_sweep<256, 16, 0>(vqh::SweepArgs)"

    def write(path, rows):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for r in rows:
                w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))

    write(tmp_path / "p1.csv", [(1, fused, "SQ_WAVE_CYCLES", 1000), (1, fused, "SQ_WAIT_ANY", 400),
                                (2, fused, "SQ_WAVE_CYCLES", 1000), (2, fused, "SQ_WAIT_ANY", 200),
                                (3, level, "SQ_WAVE_CYCLES", 500)])
    write(tmp_path / "p2.csv", [(1, fused, "SQ_INSTS_VALU", 3000), (2, fused, "SQ_INSTS_VALU", 3000),
                                (3, level, "SQ_INSTS_VALU", 640)])
    run = tmp_path / "run.txt"
    run.write_text('noise\n{"workload": "disk_1e8", "n": 6400, "calls": 2, "h": 9, "config": {}, '
                   '"levels": [{"swept": 6400}, {"swept": 6400}, {"swept": 320}, {"swept": 0}]}\n')
    rows = P.sq_counters(str(tmp_path / "p1.csv"), str(tmp_path / "p2.csv"), str(run), str(tmp_path / "o.md"),
                         "c1", "c2")
    by = {r[0]: r for r in rows}
    assert by["fused pass"][1] == 2 and abs(by["fused pass"][2] - 0.3) < 1e-12
    assert abs(by["fused pass"][6] - 64 * 6000 / 12800) < 1e-9
    assert abs(by["level sweeps (all levels)"][6] - 64 * 640 / 640) < 1e-9
    assert "c1" in (tmp_path / "o.md").read_text()
