"""GPU tests of the continuous-batching server (vqhull_server_*, the served
form of the batched hull): every request's result is bit-exact against the
CPU oracle and identical to the same request computed alone by vqhull_hull,
whatever batch it lands in; requests submitted while batches run are admitted
by the next free lane; errors stay with their request."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vq():
    import torch

    import paper_2510_09417_amd as vq

    assert torch.cuda.is_available()
    vq.load_library()
    vq.set_config(sweep_block=512, sweep_ppt=8, lds_limit=2048, reverse_tiles=0, sweep_persistent=1, level_block=256, prefilter=0)
    return vq


def _requests(nreq, max_n, seed):
    sizes, dists, _ = workloads.served_plan(nreq, seed=seed)
    sizes = np.minimum(sizes, max_n)
    return [(i, int(sizes[i]), int(dists[i])) for i in range(nreq)]


def _device(x, y):
    import torch

    return torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()


def test_mix_matches_oracle_and_alone(vq):
    import torch

    reqs = _requests(240, 150_000, seed=11)
    reqs += [(240, 0, 0), (241, 1, 1), (242, 2, 2), (243, 3, 3), (244, 2049, 0)]
    data = []
    for i, n, d in reqs:
        x, y = workloads.served_request(i, n, d, seed=11)
        tx, ty = _device(x, y)
        data.append((x, y, tx, ty, torch.empty(max(n, 1), dtype=torch.int64, device="cuda"),
                     torch.empty(1, dtype=torch.int64, device="cuda")))
    torch.cuda.synchronize()
    with vq.Server(lanes=3, lane_points=1 << 19, lane_requests=48) as srv:
        tickets = []
        for k, (_, _, tx, ty, oi, oc) in enumerate(data):
            tickets.append(srv.submit(tx, ty, oi, oc))
            if k % 40 == 39:
                time.sleep(0.002)  # later requests arrive while batches run
        for t in tickets:
            assert srv.wait(t) == vq.VQHULL_OK
        st = srv.stats()
        infos = [srv.info(t) for t in tickets]
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["batches"] >= 4
    lanes = {inf["lane"] for inf in infos}
    assert len(lanes) >= 2, "only one lane was used"
    for inf in infos:
        assert inf["done"] == 1 and inf["t_submit"] <= inf["t_start"] <= inf["t_done"]
    for (x, y, tx, ty, oi, oc), (i, n, d) in zip(data, reqs):
        h = int(oc.item())
        got = oi[:h].cpu().numpy()
        want = oracle.hull(x, y)
        assert np.array_equal(got, want), f"request {i} n={n} {workloads.DISTRIBUTIONS[d]}"
        alone = vq.hull(tx, ty).cpu().numpy()
        assert np.array_equal(got, alone)


def test_submit_from_several_threads_and_poll(vq):
    import torch

    reqs = _requests(96, 60_000, seed=12)
    data = {}
    for i, n, d in reqs:
        x, y = workloads.served_request(i, n, d, seed=12)
        tx, ty = _device(x, y)
        data[i] = (x, y, tx, ty, torch.empty(max(n, 1), dtype=torch.int64, device="cuda"),
                   torch.empty(1, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    tickets = {}
    lock = threading.Lock()
    with vq.Server(lanes=2, lane_points=1 << 18, lane_requests=16) as srv:
        def worker(part):
            for i in part:
                _, _, tx, ty, oi, oc = data[i]
                t = srv.submit(tx, ty, oi, oc)
                with lock:
                    tickets[t] = i

        ths = [threading.Thread(target=worker, args=([i for i, _, _ in reqs][k::4],)) for k in range(4)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        srv.drain()
        seen = srv.poll(cap=1000)
        assert sorted(seen) == sorted(tickets) and srv.poll() == []
    for t, i in tickets.items():
        x, y, _, _, oi, oc = data[i]
        assert np.array_equal(oi[:int(oc.item())].cpu().numpy(), oracle.hull(x, y)), f"request {i}"


def test_nonfinite_request_is_isolated(vq):
    import torch

    outs = []
    with vq.Server(lanes=1, lane_points=1 << 16, lane_requests=8) as srv:
        tks = []
        for k in range(3):
            x, y = workloads.points("disk", 5000, seed=[13, k])
            if k == 1:
                y[77] = np.nan
            tx, ty = _device(x, y)
            oi = torch.empty(5000, dtype=torch.int64, device="cuda")
            oc = torch.empty(1, dtype=torch.int64, device="cuda")
            outs.append((x, y, tx, ty, oi, oc))
            tks.append(srv.submit(tx, ty, oi, oc))
        status = [srv.wait(t) for t in tks]
    assert status == [vq.VQHULL_OK, vq.VQHULL_ERR_NONFINITE, vq.VQHULL_OK]
    assert int(outs[1][5].item()) == -vq.VQHULL_ERR_NONFINITE
    for k in (0, 2):
        x, y, _, _, oi, oc = outs[k]
        assert np.array_equal(oi[:int(oc.item())].cpu().numpy(), oracle.hull(x, y))


def test_request_larger_than_a_lane_is_rejected(vq):
    import torch

    x, y = _device(*workloads.points("square", 5000, seed=14))
    oi = torch.empty(5000, dtype=torch.int64, device="cuda")
    oc = torch.empty(1, dtype=torch.int64, device="cuda")
    with vq.Server(lanes=1, lane_points=4096, lane_requests=4) as srv:
        with pytest.raises(vq.VqhullError) as e:
            srv.submit(x, y, oi, oc)
        assert e.value.status == vq.VQHULL_ERR_INVALID_ARGUMENT
        t = srv.submit(x[:4096], y[:4096], oi, oc)  # exactly a lane fits
        assert srv.wait(t) == vq.VQHULL_OK
        xs, ys = x[:4096].cpu().numpy(), y[:4096].cpu().numpy()
        assert np.array_equal(oi[:int(oc.item())].cpu().numpy(), oracle.hull(xs, ys))


def test_submit_pointers_batch_path(vq):
    """The one-call submission of many requests (device addresses in host
    arrays), as the benchmark uses it, on requests packed in one buffer."""
    import torch

    reqs = _requests(150, 40_000, seed=15)
    xs, ys = [], []
    for i, n, d in reqs:
        x, y = workloads.served_request(i, n, d, seed=15)
        xs.append(x)
        ys.append(y)
    sizes = np.array([n for _, n, _ in reqs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    OUT = torch.full((int(off[-1]),), -7, dtype=torch.int64, device="cuda")
    CNT = torch.full((len(reqs),), -7, dtype=torch.int64, device="cuda")
    with vq.Server(lanes=2, lane_points=1 << 18, lane_requests=32) as srv:
        first = srv.submit_pointers(X.data_ptr() + 8 * off[:-1], Y.data_ptr() + 8 * off[:-1], sizes,
                                    OUT.data_ptr() + 8 * off[:-1], CNT.data_ptr() + 8 * np.arange(len(reqs)))
        srv.drain()
        assert [srv.info(first + k)["status"] for k in range(len(reqs))] == [0] * len(reqs)
    cnt = CNT.cpu().numpy()
    out = OUT.cpu().numpy()
    for k in range(len(reqs)):
        assert np.array_equal(out[off[k]:off[k] + cnt[k]], oracle.hull(xs[k], ys[k])), f"request {k}"


def _run_server(vq, data, **kw):
    import torch

    outs = []
    with vq.Server(**kw) as srv:
        tks = []
        for x, y, tx, ty in data:
            oi = torch.full((max(len(x), 1),), -5, dtype=torch.int64, device="cuda")
            oc = torch.full((1,), -5, dtype=torch.int64, device="cuda")
            outs.append((oi, oc))
            tks.append(srv.submit(tx, ty, oi, oc))
        for t in tks:
            assert srv.wait(t) == vq.VQHULL_OK
        st = srv.stats()
    return [oi[:int(oc.item())].cpu().numpy() for oi, oc in outs], st


def test_graph_lanes_equal_plain_lanes(vq):
    """The captured batch step (one hipGraph replay per batch) and plain
    launches give the same lists; the graph is replayed for many batches."""
    data = []
    for i, n, d in _requests(120, 80_000, seed=16):
        x, y = workloads.served_request(i, n, d, seed=16)
        data.append((x, y) + _device(x, y))
    got_g, st_g = _run_server(vq, data, lanes=2, lane_points=1 << 18, lane_requests=24, graph_levels=20)
    got_p, st_p = _run_server(vq, data, lanes=2, lane_points=1 << 18, lane_requests=24, graph_levels=0)
    assert st_g["graph_batches"] >= 4 and st_p["graph_batches"] == 0 and st_p["plain_batches"] == st_p["batches"]
    for k, ((x, y, _, _), a, b) in enumerate(zip(data, got_g, got_p)):
        want = oracle.hull(x, y)
        assert np.array_equal(a, want) and np.array_equal(b, want), f"request {k}"


def test_graph_falls_back_when_recursion_is_deeper(vq):
    """A lane captured with 2 levels cannot finish a large circle inside the
    graph: the batch is computed again with plain launches, bit-exact."""
    data = []
    for k, (dist, n) in enumerate((("circle", 300_000), ("disk", 50_000), ("circle", 9_000))):
        x, y = workloads.points(dist, n, seed=[17, k])
        data.append((x, y) + _device(x, y))
    got, st = _run_server(vq, data, lanes=1, lane_points=1 << 19, lane_requests=2, graph_levels=2)
    assert st["plain_batches"] >= 1
    for (x, y, _, _), a in zip(data, got):
        assert np.array_equal(a, oracle.hull(x, y))


def test_prefilter_setting_does_not_reach_the_lanes(vq):
    """The lanes run the plain method whatever the library-wide prefilter
    setting: graph replays never use it and the plain fallback turns it off."""
    data = []
    for i, n, d in _requests(60, 80_000, seed=19):
        x, y = workloads.served_request(i, n, d, seed=19)
        data.append((x, y) + _device(x, y))
    vq.set_config(prefilter=1)
    try:
        got_p, st_p = _run_server(vq, data, lanes=1, lane_points=1 << 18, lane_requests=24, graph_levels=0)
        got_g, st_g = _run_server(vq, data, lanes=1, lane_points=1 << 18, lane_requests=24, graph_levels=20)
    finally:
        vq.set_config(prefilter=0)
    assert st_p["plain_batches"] == st_p["batches"] and st_g["graph_batches"] >= 1
    for k, ((x, y, _, _), a, b) in enumerate(zip(data, got_p, got_g)):
        want = oracle.hull(x, y)
        assert np.array_equal(a, want) and np.array_equal(b, want), f"request {k}"


def test_wait_timeout_watchdog(vq):
    """The bounded wait: a request queued behind several batches on one lane is
    not done right after submission (timeout reported, nothing cancelled); a
    long enough bound returns its status, and its hull is the oracle's."""
    import torch

    data = []
    for i in range(16):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], 400_000, seed=[15, i])
        tx, ty = _device(x, y)
        data.append((x, y, tx, ty, torch.empty(400_000, dtype=torch.int64, device="cuda"),
                     torch.empty(1, dtype=torch.int64, device="cuda")))
    torch.cuda.synchronize()
    with vq.Server(lanes=1, lane_points=400_000, lane_requests=4) as srv:
        tickets = [srv.submit(tx, ty, oi, oc) for (_, _, tx, ty, oi, oc) in data]
        # 16 batches of one request each are ahead of the last ticket
        assert srv.wait_timeout(tickets[-1], 0.0) == vq.VQHULL_ERR_TIMEOUT
        assert srv.wait_timeout(tickets[-1], 120.0) == vq.VQHULL_OK
        assert srv.wait_timeout(tickets[0], 0.0) == vq.VQHULL_OK  # done long before
        for bad in (-1.0, float("nan"), 2e6):
            assert srv.wait_timeout(tickets[0], bad) == vq.VQHULL_ERR_INVALID_ARGUMENT
        assert srv.wait_timeout(tickets[-1] + 1, 0.01) == vq.VQHULL_ERR_INVALID_ARGUMENT
        srv.drain()
        assert srv.stats()["completed"] == 16
    for x, y, _, _, oi, oc in data:
        assert np.array_equal(oi[:int(oc.item())].cpu().numpy(), oracle.hull(x, y))


def test_tiny_budget_completes_every_request(vq):
    """Lanes of 4096 points and 3 requests: admission is bound by the budget
    (many batches, a request that fills a lane goes alone) and every request
    still completes with the oracle's hull."""
    import torch

    rng = np.random.default_rng(16)
    sizes = list(rng.integers(0, 4097, 150)) + [4096, 4096, 0, 1, 2, 3]
    data = []
    for i, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], int(n), seed=[16, i])
        tx, ty = _device(x, y)
        data.append((x, y, tx, ty, torch.empty(max(int(n), 1), dtype=torch.int64, device="cuda"),
                     torch.empty(1, dtype=torch.int64, device="cuda")))
    torch.cuda.synchronize()
    with vq.Server(lanes=2, lane_points=4096, lane_requests=3) as srv:
        tickets = [srv.submit(tx, ty, oi, oc) for (_, _, tx, ty, oi, oc) in data]
        srv.drain()
        st = srv.stats()
        infos = [srv.info(t) for t in tickets]
    assert st["completed"] == len(sizes) and st["failed"] == 0 and st["points"] == sum(int(n) for n in sizes)
    batches = {}
    for inf in infos:
        batches.setdefault(inf["batch"], []).append(inf["n"])
    assert st["batches"] == len(batches) >= len(sizes) // 3
    for ns in batches.values():
        assert len(ns) <= 3 and (len(ns) == 1 or sum(ns) <= 4096)
    for x, y, _, _, oi, oc in data:
        assert np.array_equal(oi[:int(oc.item())].cpu().numpy(), oracle.hull(x, y))
