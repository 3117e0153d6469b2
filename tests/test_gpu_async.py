"""The stream-ordered batched call on the GPU (vqhull_hull_batched_async):
index lists equal the CPU oracle's element by element and those of the
synchronous batched call; a level budget that ends before the recursion
marks every request of the call incomplete and writes no list; several calls
queue on one stream, each with its own buffers, with no host wait between
them, and on a side stream."""
import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vq():
    import paper_2510_09417_amd as m

    m.load_library()
    return m


def _batch(tag, sizes):
    xs, ys = [], []
    for i, (dist, n) in enumerate(sizes):
        x, y = workloads.points(dist, n, seed=[tag, i])
        xs.append(x)
        ys.append(y)
    off = np.concatenate([[0], np.cumsum([n for _, n in sizes])]).astype(np.int64)
    return xs, ys, off


MIX = [("disk", 200_000), ("square", 100_000), ("circle", 30_000), ("kuzmin", 100_000), ("disk", 10),
       ("square", 2000), ("circle", 1500), ("disk", 0), ("kuzmin", 1), ("square", 3), ("circle", 2049)]


def test_async_matches_oracle_and_sync(vq):
    import torch

    xs, ys, off = _batch(91, MIX)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    out, cnt, ws = vq.hull_batched_async(X, Y, off, levels=64)
    torch.cuda.synchronize()
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    out2, cnt2 = vq.hull_batched(X, Y, off)
    out2, cnt2 = out2.cpu().numpy(), cnt2.cpu().numpy()
    for i in range(len(MIX)):
        want = oracle.hull(xs[i], ys[i])
        assert cnt[i] == len(want), (i, MIX[i], cnt[i])
        assert np.array_equal(out[off[i]:off[i] + cnt[i]], want), (i, MIX[i])
        assert cnt2[i] == cnt[i] and np.array_equal(out2[off[i]:off[i] + cnt2[i]], want), i


def test_short_budget_marks_every_request_incomplete(vq):
    """A circle of 30 000 points needs more than three levels: with a budget
    of three the whole call reports INCOMPLETE (small requests included) and
    the same call with a larger budget completes."""
    import torch

    xs, ys, off = _batch(92, [("circle", 30_000), ("disk", 500), ("square", 40_000)])
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    _, cnt, _ = vq.hull_batched_async(X, Y, off, levels=3)
    torch.cuda.synchronize()
    assert (cnt.cpu().numpy() == vq.INCOMPLETE).all()
    out, cnt, _ = vq.hull_batched_async(X, Y, off, levels=40)
    torch.cuda.synchronize()
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    for i in range(3):
        assert np.array_equal(out[off[i]:off[i] + cnt[i]], oracle.hull(xs[i], ys[i])), i


def test_calls_queue_without_host_waits(vq):
    """Four calls enqueued back to back on one stream, each with its own
    inputs, outputs and workspace, then one on a side stream; the host waits
    once at the end.  Every list equals the oracle's."""
    import torch

    batches = [_batch(93 + k, [(workloads.DISTRIBUTIONS[(k + j) % 4], 20_000 + 7919 * j) for j in range(5)])
               for k in range(5)]
    side = torch.cuda.Stream()
    inputs = [(torch.from_numpy(np.concatenate(xs)).cuda(), torch.from_numpy(np.concatenate(ys)).cuda())
              for xs, ys, _ in batches]
    torch.cuda.synchronize()  # the inputs are on the device before either stream reads them
    results = []
    for k, ((X, Y), (_, _, off)) in enumerate(zip(inputs, batches)):
        if k < 4:
            results.append(vq.hull_batched_async(X, Y, off, levels=48))
        else:
            with torch.cuda.stream(side):
                results.append(vq.hull_batched_async(X, Y, off, levels=48, stream=side))
    torch.cuda.synchronize()
    for k, (out, cnt, _) in enumerate(results):
        xs, ys, off = batches[k]
        out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
        for i in range(len(xs)):
            assert np.array_equal(out[off[i]:off[i] + cnt[i]], oracle.hull(xs[i], ys[i])), (k, i)


def test_nonfinite_request_alone(vq):
    import torch

    xs, ys, off = _batch(99, [("disk", 5000), ("square", 7000), ("kuzmin", 3000)])
    xs[1] = xs[1].copy()
    xs[1][123] = np.inf
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    out, cnt, _ = vq.hull_batched_async(X, Y, off, levels=32)
    torch.cuda.synchronize()
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    assert cnt[1] == -vq.VQHULL_ERR_NONFINITE
    for i in (0, 2):
        assert np.array_equal(out[off[i]:off[i] + cnt[i]], oracle.hull(xs[i], ys[i])), i
