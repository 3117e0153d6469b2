"""GPU test of the server in the exact shape the benchmark times it: 8 lanes
of 2^25 points and 8192 requests, each lane replaying its batch step captured
with 16 recursion levels, under the persistent kernel configuration that the
batched autotuner picks on the request mix.  The requests are the served mix's
own: the first 400 of the 65,536-request plan (sizes log-uniform in
[16, 10^6], disk / square / circle / Kuzmin, ``default_rng(5)``) with the
points of request i from ``default_rng([5, i])``, plus the plan's largest
request of every distribution (each of more than 5 * 10^5 points).  Every
index list is compared element by element with the CPU oracle's."""
import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import autotune, workloads

pytestmark = pytest.mark.gpu

LANES, LANE_POINTS, LANE_REQUESTS, GRAPH_LEVELS = 8, 1 << 25, 8192, 16
FIRST = 400


def _plan_requests():
    sizes, dists, _ = workloads.served_plan(workloads.SERVED_REQUESTS)
    picked = list(range(FIRST))
    for d in range(len(workloads.DISTRIBUTIONS)):
        idx = np.nonzero(dists == d)[0]
        big = int(idx[np.argmax(sizes[idx])])
        assert sizes[big] > 500_000
        if big not in picked:
            picked.append(big)
    return [(i, int(sizes[i]), int(dists[i])) for i in picked]


@pytest.fixture(scope="module")
def mix():
    import torch

    reqs = _plan_requests()
    xs, ys = [], []
    for i, n, d in reqs:
        x, y = workloads.served_request(i, n, d)
        xs.append(x)
        ys.append(y)
    sizes = np.array([n for _, n, _ in reqs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    want = [oracle.hull(x, y) for x, y in zip(xs, ys)]
    return reqs, sizes, off, X, Y, want


def test_bench_shaped_server_matches_oracle(mix):
    import torch

    import paper_2510_09417_amd as vq

    vq.load_library()
    reqs, sizes, off, X, Y, want = mix
    saved = vq.get_config()
    # tuned the way the benchmark tunes: on one lane-sized batch of the mix,
    # persistent shapes only (the lanes replay captured graphs)
    nb = int(np.searchsorted(off, LANE_POINTS, side="right")) - 1
    tuned, table = autotune.tune_batched(X[:off[nb]], Y[:off[nb]], off[:nb + 1], repeats=1, persistent=(1,))
    assert tuned["sweep_persistent"] == 1 and all(e["same_result"] for e in table)
    vq.set_config(**tuned)
    try:
        for rnd in range(2):  # a fresh server, then a second one over the same lanes' shapes
            OUT = torch.full((int(off[-1]),), -9, dtype=torch.int64, device="cuda")
            CNT = torch.full((len(reqs),), -9, dtype=torch.int64, device="cuda")
            with vq.Server(lanes=LANES, lane_points=LANE_POINTS, lane_requests=LANE_REQUESTS,
                           graph_levels=GRAPH_LEVELS) as srv:
                # all at once (the throughput run's arrival pattern); the
                # second round submits in small groups while batches run
                step = len(reqs) if rnd == 0 else 37
                first = None
                for lo in range(0, len(reqs), step):
                    hi = min(len(reqs), lo + step)
                    t = srv.submit_pointers(X.data_ptr() + 8 * off[lo:hi], Y.data_ptr() + 8 * off[lo:hi],
                                            sizes[lo:hi], OUT.data_ptr() + 8 * off[lo:hi],
                                            CNT.data_ptr() + 8 * np.arange(lo, hi))
                    first = t if first is None else first
                srv.drain()
                infos = [srv.info(first + k) for k in range(len(reqs))]
                st = srv.stats()
            assert [inf["status"] for inf in infos] == [0] * len(reqs)
            assert st["completed"] == len(reqs) and st["failed"] == 0
            assert st["graph_batches"] >= 1
            cnt = CNT.cpu().numpy()
            out = OUT.cpu().numpy()
            for k, (i, n, d) in enumerate(reqs):
                got = out[off[k]:off[k] + cnt[k]]
                assert cnt[k] == len(want[k]) and np.array_equal(got, want[k]), \
                    f"round {rnd} request {i} n={n} {workloads.DISTRIBUTIONS[d]} config {tuned}"
    finally:
        vq.set_config(**saved)
