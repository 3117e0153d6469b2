"""The caller-owned-workspace calls on the GPU (vqhull_hull_ws,
vqhull_hull_batched_ws): index lists equal the CPU oracle's element by
element, the same workspace serves calls of different sizes in turn, two
host threads run calls on their own streams and workspaces at once, and a
call takes no device memory of its own (the device's free memory does not
move while the library-owned workspace is released)."""
import threading

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu

CASES = [("disk", 3), ("square", 2048), ("circle", 2049), ("kuzmin", 70_001), ("disk", 123_457),
         ("circle", 400_000), ("square", 1_000_000)]


@pytest.fixture(scope="module")
def vq():
    import paper_2510_09417_amd as m

    m.load_library()
    return m


@pytest.mark.parametrize("dist,n", CASES)
def test_hull_ws_matches_oracle(vq, dist, n):
    import torch

    x, y = workloads.points(dist, n, seed=[77, n])
    got = vq.hull(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()  # the _ws path
    assert np.array_equal(got, oracle.hull(x, y)), (dist, n)


def test_one_workspace_many_sizes(vq):
    """A workspace sized for the largest call serves smaller calls of every
    path (one launch for a tiny request, the level loop for large ones) in
    any order; stale contents never leak into a result."""
    import torch

    sizes = [1_000_000, 17, 0, 2048, 300_000, 1, 5000, 1_000_000]
    ws = vq.workspace(max(sizes), 1)
    out = torch.empty(max(sizes), dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    for k, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[k % 4], n, seed=[78, k])
        tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        vq.hull_ws_into(tx, ty, out, cnt, ws)
        h = int(cnt.item())
        assert np.array_equal(out[:h].cpu().numpy(), oracle.hull(x, y)), (k, n)


def test_batched_ws_matches_oracle_and_isolates_nan(vq):
    import torch

    g = np.random.default_rng(79)
    sizes = [int(v) for v in np.clip(np.floor(16 * np.power(40000 / 16, g.random(60))), 16, 40000)]
    sizes[7] = 0
    xs, ys = [], []
    for i, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], n, seed=[79, i])
        xs.append(x)
        ys.append(y)
    xs[11] = xs[11].copy()
    xs[11][len(xs[11]) // 2] = np.nan
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    out, cnt = vq.hull_batched_ws(X, Y, off)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    for i in range(len(sizes)):
        if i == 11:
            assert cnt[i] == -vq.VQHULL_ERR_NONFINITE
            continue
        assert np.array_equal(out[off[i]:off[i] + cnt[i]], oracle.hull(xs[i], ys[i])), i
    # the same batch through the library-owned path gives the same lists
    out2, cnt2 = vq.hull_batched(X, Y, off)
    assert np.array_equal(cnt2.cpu().numpy(), cnt)
    for i in range(len(sizes)):
        if cnt[i] > 0:
            assert np.array_equal(out2[off[i]:off[i] + cnt[i]].cpu().numpy(), out[off[i]:off[i] + cnt[i]])


def test_ws_call_takes_no_device_memory(vq):
    import torch

    n = 20_000_000
    x, y = workloads.points("disk", n, seed=80)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = vq.workspace(n, 1)
    vq.release_workspace()  # no library-owned workspace on this device
    vq.hull_ws_into(tx, ty, out, cnt, ws)  # first call: host-side staging and events are created
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        vq.hull_ws_into(tx, ty, out, cnt, ws)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    # the library-owned path would take about 40 bytes per point (800 MB) here
    assert abs(free0 - free1) < 32 << 20, (free0, free1)
    h = int(cnt.item())
    assert np.array_equal(out[:h].cpu().numpy(), oracle.hull(x, y))


def test_two_threads_two_streams(vq):
    """Calls with their own streams and workspaces from two host threads at
    once: every result equals the oracle's."""
    import torch

    inputs = [workloads.points(d, 600_000, seed=[81, k]) for k, d in enumerate(("circle", "disk"))]
    want = [oracle.hull(x, y) for x, y in inputs]
    errors = []

    def worker(k):
        try:
            x, y = inputs[k]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
                out = torch.empty(len(x), dtype=torch.int64, device="cuda")
                cnt = torch.empty(1, dtype=torch.int64, device="cuda")
                ws = vq.workspace(len(x), 1)
                s.synchronize()
                for _ in range(5):
                    vq.hull_ws_into(tx, ty, out, cnt, ws, s)
                    h = int(cnt.item())
                    if not np.array_equal(out[:h].cpu().numpy(), want[k]):
                        errors.append(k)
        except Exception as e:  # reported below
            errors.append(repr(e))

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert errors == []
