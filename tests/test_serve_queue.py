"""The batching server's host logic on the CPU, with a fake backend: the queue
the GPU lanes use (csrc/serve_queue.h: tickets, FIFO admission bounded by the
lane's points and requests, completion, wait, poll, drain, counters, stop) is
driven by host lane threads whose executor is the oracle's hull
(tests/fake_serve.cpp, built here with g++).  Checked for every run:
* every request completes once, with its own result (the oracle's hull of its
  own points) and status; a request with a NaN fails alone;
* a batch is a run of consecutive tickets on one lane, within the lane's
  request and point limits (a single request may fill it), and is maximal:
  the ticket after it was either over a limit or not yet submitted when the
  batch was taken;
* tickets start in submission order; submit <= start <= done;
* poll returns every ticket exactly once, in completion order;
* the counters agree with the tickets; busy time is bounded by the batches'
  spans;
* after stop, pending work still completes and new submissions are refused;
  unknown tickets are refused;
* the watchdog wait (bounded in time) reports a timeout while a request is
  still queued or running and its status once done."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2510_09417_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


@pytest.fixture(scope="module")
def fake_serve(tmp_path_factory):
    d = tmp_path_factory.mktemp("fake_serve")
    obj = str(d / "oracle.o")
    exe = str(d / "fake_serve")
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-c",
                    os.path.join(ROOT, "oracle", "vqhull_oracle.c"), "-o", obj], check=True)
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-Wall", "-Werror", f"-I{CSRC}",
                    os.path.join(HERE, "fake_serve.cpp"), obj, "-o", exe, "-fopenmp", "-lm"], check=True)
    return exe


def make_requests(count, max_n, seed, nan_every=0, zero_every=0):
    """Sizes log-uniform in [16, max_n] (the served mix's law, smaller cap),
    distributions in turn; every `zero_every`-th request is empty and every
    `nan_every`-th holds a NaN."""
    g = np.random.default_rng(seed)
    sizes = np.clip(np.floor(16 * np.power(max_n / 16, g.random(count))), 16, max_n).astype(np.int64)
    reqs = []
    for i, n in enumerate(sizes):
        if zero_every and i % zero_every == zero_every - 1:
            n = 0
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], int(n), [seed, i])
        if nan_every and i % nan_every == nan_every - 1 and n > 0:
            y = y.copy()
            y[int(n) // 2] = np.nan
        reqs.append((x, y))
    return reqs


def run(exe, tmp_path, reqs, lanes, lane_points, lane_requests, submitters=1, chunk=1, delay_us=0,
        stop_early=False):
    inp = tmp_path / "in.bin"
    outp = tmp_path / "out.bin"
    n = np.array([len(x) for x, _ in reqs], dtype=np.int64)
    with open(inp, "wb") as f:
        f.write(np.int64(len(reqs)).tobytes())
        f.write(n.tobytes())
        for x, _ in reqs:
            f.write(np.ascontiguousarray(x, dtype=np.float64).tobytes())
        for _, y in reqs:
            f.write(np.ascontiguousarray(y, dtype=np.float64).tobytes())
    subprocess.run([exe, str(inp), str(outp), str(lanes), str(lane_points), str(lane_requests), str(submitters),
                    str(chunk), str(delay_us), str(int(stop_early))], check=True, timeout=120)
    buf = np.fromfile(outp, dtype=np.int64)
    count, stop_rejected, unknown_rejected, npolled, wd_early, wd_late, wd_unknown = (int(v) for v in buf[:7])
    pos = 7
    polled = buf[pos: pos + npolled]
    pos += npolled
    counters = dict(zip(("submitted", "completed", "failed", "batches", "points", "pending"),
                        (int(v) for v in buf[pos: pos + 6])))
    pos += 6
    counters["busy"], counters["now"] = buf[pos: pos + 2].view(np.float64)
    pos += 2
    tickets = []
    for _ in range(count):
        v = [int(a) for a in buf[pos: pos + 9]]
        ts = buf[pos + 9: pos + 12].view(np.float64)
        pos += 12
        idx = buf[pos: pos + v[8]].copy()
        pos += v[8]
        tickets.append(dict(payload=v[0], req=v[1], n=v[2], batch=v[3], lane=v[4], status=v[5], done=v[6],
                            wait=v[7], idx=idx, t_submit=ts[0], t_start=ts[1], t_done=ts[2]))
    assert pos == len(buf)
    return dict(count=count, stop_rejected=stop_rejected, unknown_rejected=unknown_rejected, polled=polled,
                counters=counters, tickets=tickets, wd_early=wd_early, wd_late=wd_late, wd_unknown=wd_unknown)


def check(res, reqs, lanes, lane_points, lane_requests, delay_us=0):
    count = len(reqs)
    T = res["tickets"]
    assert res["count"] == count == len(T)
    assert res["stop_rejected"] == 1 and res["unknown_rejected"] == 1
    # watchdog: a bounded wait returns once done, refuses unknown tickets
    assert res["wd_unknown"] == -1
    assert res["wd_late"] == (1 if count else -2)
    # results: each ticket carries its own request, done once, with its own hull
    nonfinite = [not (np.isfinite(x).all() and np.isfinite(y).all()) for x, y in reqs]
    for t, k in enumerate(T):
        r = k["payload"]
        assert k["req"] == r, (t, k["req"], r)
        x, y = reqs[r]
        assert k["n"] == len(x) and k["done"] == 1 and k["wait"] == k["status"]
        if nonfinite[r]:
            assert k["status"] == oracle.ORACLE_ERR_NONFINITE and len(k["idx"]) == 0
        else:
            assert k["status"] == oracle.ORACLE_OK
            assert np.array_equal(k["idx"], oracle.hull(x, y)), f"ticket {t} (request {r})"
    assert sorted(k["payload"] for k in T) == list(range(count))
    # timing and FIFO start order
    for k in T:
        assert k["t_submit"] <= k["t_start"] <= k["t_done"]
    starts = [k["t_start"] for k in T]
    assert all(a <= b for a, b in zip(starts, starts[1:])), "tickets started out of submission order"
    # batches
    by_batch = {}
    for t, k in enumerate(T):
        by_batch.setdefault(k["batch"], []).append(t)
    assert sorted(by_batch) == list(range(len(by_batch)))
    span = 0.0
    for b, ids in by_batch.items():
        assert ids == list(range(ids[0], ids[-1] + 1)), f"batch {b} is not a run of tickets"
        ks = [T[t] for t in ids]
        assert len({k["lane"] for k in ks}) == 1 and 0 <= ks[0]["lane"] < lanes
        assert len({k["t_start"] for k in ks}) == 1 and len({k["t_done"] for k in ks}) == 1
        pts = sum(k["n"] for k in ks)
        assert len(ids) <= lane_requests
        assert len(ids) == 1 or pts <= lane_points, (b, len(ids), pts)
        e = ids[-1] + 1
        if e < count and len(ids) < lane_requests and pts + T[e]["n"] <= lane_points:
            # the next ticket fit: it cannot have been pending when this batch was taken
            assert T[e]["t_submit"] >= ks[0]["t_start"], f"batch {b} left a fitting pending ticket behind"
        span += ks[0]["t_done"] - ks[0]["t_start"]
    # poll: every ticket once, in completion (batch) order
    polled = [int(t) for t in res["polled"]]
    assert sorted(polled) == list(range(count))
    pb = [T[t]["batch"] for t in polled]
    assert all(a <= b for a, b in zip(pb, pb[1:])), "poll order is not completion order"
    # counters
    c = res["counters"]
    assert c["submitted"] == c["completed"] == count and c["pending"] == 0
    assert c["failed"] == sum(nonfinite) and c["batches"] == len(by_batch)
    assert c["points"] == sum(len(x) for x, _ in reqs)
    assert c["busy"] <= span + 1e-9
    assert c["busy"] >= len(by_batch) * delay_us * 1e-6
    assert c["now"] >= max((k["t_done"] for k in T), default=0.0)
    return by_batch


def test_one_lane_one_submitter(fake_serve, tmp_path):
    reqs = make_requests(120, 4000, seed=1, nan_every=17, zero_every=11)
    res = run(fake_serve, tmp_path, reqs, lanes=1, lane_points=10_000, lane_requests=8, delay_us=200)
    check(res, reqs, 1, 10_000, 8, delay_us=200)


def test_many_lanes_many_submitters(fake_serve, tmp_path):
    reqs = make_requests(400, 6000, seed=2, nan_every=31, zero_every=23)
    res = run(fake_serve, tmp_path, reqs, lanes=3, lane_points=25_000, lane_requests=16, submitters=3, chunk=5,
              delay_us=300)
    by_batch = check(res, reqs, 3, 25_000, 16, delay_us=300)
    # the lanes share the work: batches run on more than one lane at once
    lanes_used = {res["tickets"][ids[0]]["lane"] for ids in by_batch.values()}
    assert len(lanes_used) > 1


def test_one_request_per_batch(fake_serve, tmp_path):
    reqs = make_requests(60, 3000, seed=3)
    res = run(fake_serve, tmp_path, reqs, lanes=2, lane_points=1 << 20, lane_requests=1, chunk=60)
    by_batch = check(res, reqs, 2, 1 << 20, 1)
    assert len(by_batch) == 60


def test_point_budget_binds(fake_serve, tmp_path):
    """A small point budget: requests that exactly fill it go alone, empty
    requests ride along with anything."""
    lane_points = 64
    reqs = [workloads.points("disk", n, [4, i]) for i, n in
            enumerate([64, 0, 0, 30, 34, 1, 63, 0, 64, 0, 16, 16, 16, 16, 16, 0, 50, 14, 3] * 4)]
    res = run(fake_serve, tmp_path, reqs, lanes=1, lane_points=lane_points, lane_requests=100, chunk=len(reqs))
    by_batch = check(res, reqs, 1, lane_points, 100)
    for ids in by_batch.values():
        assert sum(res["tickets"][t]["n"] for t in ids) <= lane_points


def test_requests_at_the_lane_size(fake_serve, tmp_path):
    reqs = [workloads.points(workloads.DISTRIBUTIONS[i % 4], 5000, [6, i]) for i in range(20)]
    res = run(fake_serve, tmp_path, reqs, lanes=2, lane_points=5000, lane_requests=50, submitters=2, chunk=3)
    by_batch = check(res, reqs, 2, 5000, 50)
    assert all(len(ids) == 1 for ids in by_batch.values())


def test_stop_with_pending_work(fake_serve, tmp_path):
    reqs = make_requests(150, 3000, seed=7, nan_every=13)
    res = run(fake_serve, tmp_path, reqs, lanes=2, lane_points=8000, lane_requests=6, submitters=2, chunk=9,
              delay_us=500, stop_early=True)
    check(res, reqs, 2, 8000, 6, delay_us=500)


def test_watchdog_times_out_on_a_slow_lane(fake_serve, tmp_path):
    """A lane that takes 0.3 s per batch: the last of 12 requests cannot be
    done right after submission, so the zero-timeout look reports a timeout;
    the request is not cancelled and completes with its own hull."""
    reqs = make_requests(12, 1000, seed=11)
    res = run(fake_serve, tmp_path, reqs, lanes=1, lane_points=1 << 20, lane_requests=4, chunk=12,
              delay_us=300_000)
    assert res["wd_early"] == 0
    by_batch = check(res, reqs, 1, 1 << 20, 4, delay_us=300_000)
    assert len(by_batch) == 3


def test_no_requests(fake_serve, tmp_path):
    res = run(fake_serve, tmp_path, [], lanes=2, lane_points=100, lane_requests=4)
    check(res, [], 2, 100, 4)
    assert res["counters"]["batches"] == 0


# ---------------------------------------------------------------- the checks catch mistakes
def test_checks_reject_a_misrouted_result(fake_serve, tmp_path):
    reqs = make_requests(30, 2000, seed=8)
    res = run(fake_serve, tmp_path, reqs, lanes=1, lane_points=10_000, lane_requests=4)
    a, b = res["tickets"][3], res["tickets"][4]
    a["idx"], b["idx"] = b["idx"], a["idx"]
    with pytest.raises(AssertionError):
        check(res, reqs, 1, 10_000, 4)


def test_checks_reject_an_oversized_batch(fake_serve, tmp_path):
    reqs = make_requests(30, 2000, seed=9)
    res = run(fake_serve, tmp_path, reqs, lanes=1, lane_points=10_000, lane_requests=4, chunk=30)
    assert max(list(t["batch"] for t in res["tickets"]).count(b) for b in range(res["counters"]["batches"])) == 4
    with pytest.raises(AssertionError):
        check(res, reqs, 1, 10_000, 3)  # a tighter request limit than the run had


def test_checks_reject_a_lost_poll(fake_serve, tmp_path):
    reqs = make_requests(30, 2000, seed=10)
    res = run(fake_serve, tmp_path, reqs, lanes=2, lane_points=10_000, lane_requests=4)
    res["polled"] = res["polled"][:-1]
    with pytest.raises(AssertionError):
        check(res, reqs, 2, 10_000, 4)
