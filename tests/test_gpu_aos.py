"""GPU parity of the interleaved (array-of-structures) input, x_i = xy[2i],
y_i = xy[2i+1], through vqhull_hull_xy / vqhull_hull_batched_xy: the same
index lists as the oracle (bit-exact) on every distribution, size class
(the one-workgroup range, the LDS threshold, several extremes tiles with
ragged tails), batches with empty requests, degenerate and non-finite inputs,
and with the octagon prefilter on against the oracle's prefiltered variant."""
import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu

BASE = dict(sweep_block=512, sweep_ppt=8, lds_limit=2048, reverse_tiles=0, sweep_persistent=1, level_block=256,
            prefilter=0)


@pytest.fixture(scope="module")
def vq():
    import torch

    import paper_2510_09417_amd as vq

    assert torch.cuda.is_available()
    vq.load_library()
    vq.set_config(**BASE)
    yield vq
    vq.set_config(**BASE)


def interleaved(x, y):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.stack([x, y], axis=1), dtype=np.float64)).cuda()


def check(vq, x, y, label, prefiltered=False):
    want = oracle.hull_prefiltered(x, y, 2048) if prefiltered else oracle.hull(x, y)
    got = vq.hull_xy(interleaved(x, y)).cpu().numpy()
    assert np.array_equal(got, want), f"{label}: gpu h={len(got)} oracle h={len(want)}"


@pytest.mark.parametrize("dist", list(workloads.DISTRIBUTIONS))
@pytest.mark.parametrize("n", [1, 2, 3, 100, 2047, 2048, 2049, 16_385, 123_457, 1_000_003])
def test_aos_distributions(vq, dist, n):
    x, y = workloads.points(dist, n, seed=n + 41)
    check(vq, x, y, f"{dist} n={n}")


@pytest.mark.parametrize("dist", list(workloads.DISTRIBUTIONS))
def test_aos_prefilter(vq, dist):
    vq.set_config(prefilter=1)
    try:
        for n in (1000, 2049, 40_000, 700_001):
            x, y = workloads.points(dist, n, seed=n + 43)
            check(vq, x, y, f"{dist} n={n} prefilter", prefiltered=True)
    finally:
        vq.set_config(prefilter=0)


def test_aos_empty(vq):
    import torch

    assert vq.hull_xy(torch.empty((0, 2), dtype=torch.float64, device="cuda")).numel() == 0


@pytest.mark.parametrize("prefilter", [0, 1])
def test_aos_batched(vq, prefilter):
    sizes = [0, 1, 2, 3, 17, 2048, 2049, 5000, 0, 100_000, 7, 40_000, 1, 16_384, 16_385, 0]
    xs, ys = [], []
    for i, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], n, seed=[23, i])
        xs.append(x)
        ys.append(y)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    vq.set_config(prefilter=prefilter)
    try:
        out, cnt = vq.hull_batched_xy(interleaved(np.concatenate(xs), np.concatenate(ys)), off)
    finally:
        vq.set_config(prefilter=0)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    for i, n in enumerate(sizes):
        want = oracle.hull_prefiltered(xs[i], ys[i], 2048) if prefilter else oracle.hull(xs[i], ys[i])
        assert cnt[i] == len(want) and np.array_equal(out[off[i]: off[i] + cnt[i]], want), f"request {i} (n={n})"


def test_aos_degenerate(vq):
    for k in range(6):
        x, y = workloads.lattice(20_000 + 1511 * k, seed=500 + k, lo=-k - 2, hi=k + 3, dup_frac=0.3,
                                 collinear_runs=k % 3)
        check(vq, x, y, f"lattice {k}")
    check(vq, np.full(3000, 2.5), np.full(3000, -1.0), "all equal")
    xs = np.arange(3000, dtype=np.float64)
    check(vq, xs, 2.0 * xs + 1.0, "collinear")
    check(vq, np.array([0.0, -0.0, 1.0]), np.array([0.0, 0.0, -0.0]), "signed zeros")


def test_aos_nonfinite(vq):
    import torch

    x, y = workloads.points("disk", 30_000, seed=6)
    for which, pos, val in (("y", 3, np.nan), ("x", 29_999, np.inf), ("y", 16_384, -np.inf)):
        xx, yy = x.copy(), y.copy()
        (xx if which == "x" else yy)[pos] = val
        out = torch.empty(30_000, dtype=torch.int64, device="cuda")
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        vq.hull_xy_into(interleaved(xx, yy), out, cnt)
        assert int(cnt.item()) == -vq.VQHULL_ERR_NONFINITE, (which, pos)
    sizes = [1000, 3000, 5000]
    xs, ys = [], []
    for i, n in enumerate(sizes):
        a, b = workloads.points("disk", n, seed=[9, i])
        xs.append(a)
        ys.append(b)
    ys[1][10] = np.nan
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out, cnt = vq.hull_batched_xy(interleaved(np.concatenate(xs), np.concatenate(ys)), off)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    assert cnt[1] == -vq.VQHULL_ERR_NONFINITE
    for i in (0, 2):
        assert np.array_equal(out[off[i]: off[i] + cnt[i]], oracle.hull(xs[i], ys[i]))


def test_aos_equals_soa_at_1e7(vq):
    import torch

    for dist in ("disk", "square"):
        x, y = workloads.points(dist, 10_000_000, seed=8)
        soa = vq.hull(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()
        aos = vq.hull_xy(interleaved(x, y)).cpu().numpy()
        assert np.array_equal(aos, soa), dist
        assert np.array_equal(soa, oracle.hull(x, y)), dist


def test_aos_ingest_is_timed(vq):
    x, y = workloads.points("square", 300_000, seed=2)
    xy = interleaved(x, y)
    vq.set_timing(True)
    try:
        vq.hull_xy(xy)
        kinds = [t["kind"] for t in vq.kernel_times()]
    finally:
        vq.set_timing(False)
    assert kinds.count("ingest") == 1 and "sweep" in kinds
