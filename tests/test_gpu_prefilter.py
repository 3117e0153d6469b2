"""GPU parity of the octagon prefilter (the variant of Section 6's
Akl-Toussaint heuristic): the HIP path with the prefilter on, through the C
ABI, against the oracle's prefiltered variant, index list for index list
(bit-exact), and the number of points the filter keeps against the oracle's
keep mask (exact count).  Sizes span several extremes tiles (16384 points)
with ragged tails; the LDS threshold is crossed from both sides (a request
at the threshold is not filtered; just above it, the filtered root may itself
fit in LDS and is finished from the compacted copy)."""
import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu

BASE = dict(sweep_block=512, sweep_ppt=8, lds_limit=2048, reverse_tiles=0, sweep_persistent=1, level_block=256)


@pytest.fixture(scope="module")
def vq():
    import torch

    import paper_2510_09417_amd as vq

    assert torch.cuda.is_available()
    vq.load_library()
    vq.set_config(**BASE, prefilter=1)
    yield vq
    vq.set_config(**BASE, prefilter=0)


def gpu_hull(x, y):
    import torch

    import paper_2510_09417_amd as vq

    tx = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    ty = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).cuda()
    return vq.hull(tx, ty).cpu().numpy()


def check(x, y, label, lds=2048):
    want = oracle.hull_prefiltered(x, y, lds)
    got = gpu_hull(x, y)
    if not np.array_equal(got, want):
        k = next((i for i in range(min(len(got), len(want))) if got[i] != want[i]), min(len(got), len(want)))
        raise AssertionError(f"{label}: gpu h={len(got)} oracle h={len(want)}; first difference at {k}")


def kept(x, y):
    return int(oracle.octagon(x, y)[1].sum())


@pytest.mark.parametrize("dist", list(workloads.DISTRIBUTIONS))
@pytest.mark.parametrize("n", [2049, 2050, 16_383, 16_385, 40_000, 123_457, 1_000_003])
def test_prefilter_distributions(vq, dist, n):
    x, y = workloads.points(dist, n, seed=n + 29)
    check(x, y, f"{dist} n={n}")
    k = kept(x, y)
    st = vq.level_stats()
    if k > 2048:  # the filtered root is a swept segment of exactly the kept points
        assert st[0]["segments"] == 1 and st[0]["swept"] == k, (st[0], k)
    else:  # the filtered root fits in LDS: one job of the kept points
        assert st[0]["segments"] == 0 and st[0]["jobs"] == 1 and st[0]["job_points"] == k, (st[0], k)


def test_prefilter_equals_plain_on_workloads(vq):
    """On the synthetic workloads the variant returns the plain method's hull."""
    for dist in workloads.DISTRIBUTIONS:
        x, y = workloads.points(dist, 500_000, seed=77)
        assert np.array_equal(gpu_hull(x, y), oracle.hull(x, y)), dist


@pytest.mark.parametrize("lds", [512, 1024, 2048])
def test_prefilter_thresholds(vq, lds):
    vq.set_config(lds_limit=lds)
    try:
        for n in (lds - 1, lds, lds + 1, lds + 2, 3 * lds + 5, 20_000):
            for dist in workloads.DISTRIBUTIONS:
                x, y = workloads.points(dist, n, seed=[lds, n])
                check(x, y, f"lds={lds} {dist} n={n}", lds=lds)
    finally:
        vq.set_config(lds_limit=2048)


def test_prefilter_degenerate(vq):
    for k in range(8):
        x, y = workloads.lattice(50_000 + 977 * k, seed=300 + k, lo=-k - 2, hi=k + 3, dup_frac=0.3,
                                 collinear_runs=k % 3)
        check(x, y, f"lattice {k}")
    check(np.full(5000, 2.5), np.full(5000, -1.0), "all equal")
    xs = np.arange(5000, dtype=np.float64)
    check(xs, 2.0 * xs + 1.0, "collinear")
    check(np.tile([0.0, 1.0], 3000), np.tile([0.0, 1.0], 3000), "two points")
    # a triangle: several octagon vertices coincide, the interior still drops
    rng = np.random.default_rng(9)
    inner = rng.random((30_000, 2)) * 3.0 + 1.0
    x = np.concatenate([[0.0, 10.0, 0.0], inner[:, 0]])
    y = np.concatenate([[0.0, 0.0, 10.0], inner[:, 1]])
    check(x, y, "triangle")
    assert kept(x, y) == 3


def test_prefilter_batched(vq):
    import torch

    sizes = [0, 1, 2, 3, 17, 2048, 2049, 5000, 0, 100_000, 7, 40_000, 1, 16_384, 16_385, 2100]
    xs, ys = [], []
    for i, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], n, seed=[17, i])
        xs.append(x)
        ys.append(y)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out, cnt = vq.hull_batched(torch.from_numpy(np.concatenate(xs)).cuda(),
                               torch.from_numpy(np.concatenate(ys)).cuda(), off)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    for i, n in enumerate(sizes):
        want = oracle.hull_prefiltered(xs[i], ys[i], 2048)
        got = out[off[i]: off[i] + cnt[i]]
        assert cnt[i] == len(want) and np.array_equal(got, want), f"request {i} (n={n})"


def test_prefilter_nonfinite(vq):
    import torch

    x, y = workloads.points("disk", 30_000, seed=4)
    for arr, pos, val in ((y, 10, np.nan), (x, 29_999, np.inf), (y, 16_384, -np.inf)):
        xx, yy = x.copy(), y.copy()
        (xx if arr is x else yy)[pos] = val
        out_idx = torch.empty(30_000, dtype=torch.int64, device="cuda")
        out_cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        vq.hull_into(torch.from_numpy(xx).cuda(), torch.from_numpy(yy).cuda(), out_idx, out_cnt)
        assert int(out_cnt.item()) == -vq.VQHULL_ERR_NONFINITE
    sizes = [10_000, 30_000, 5000]
    xs, ys = [], []
    for i, n in enumerate(sizes):
        a, b = workloads.points("square", n, seed=[8, i])
        xs.append(a)
        ys.append(b)
    xs[1][123] = np.nan
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out, cnt = vq.hull_batched(torch.from_numpy(np.concatenate(xs)).cuda(),
                               torch.from_numpy(np.concatenate(ys)).cuda(), off)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    assert cnt[1] == -vq.VQHULL_ERR_NONFINITE
    for i in (0, 2):
        assert np.array_equal(out[off[i]: off[i] + cnt[i]], oracle.hull_prefiltered(xs[i], ys[i], 2048))


@pytest.mark.parametrize("shape,persistent", [((256, 32), 1), ((1024, 8), 1), ((512, 8), 0), ((256, 16), 0)])
def test_prefilter_shapes(vq, shape, persistent):
    vq.set_config(sweep_block=shape[0], sweep_ppt=shape[1], sweep_persistent=persistent)
    try:
        for dist in ("disk", "circle"):
            x, y = workloads.points(dist, 300_000, seed=12)
            check(x, y, f"{dist} {shape} persistent={persistent}")
    finally:
        vq.set_config(**BASE, prefilter=1)


def test_prefilter_timing_records(vq):
    x, y = workloads.points("disk", 400_000, seed=3)
    vq.set_timing(True)
    try:
        gpu_hull(x, y)
        kinds = {t["kind"] for t in vq.kernel_times()}
    finally:
        vq.set_timing(False)
    assert {"extremes", "filter", "compact", "plan0", "sweep"} <= kinds


@pytest.mark.parametrize("scale", [1e300, 1e150, 1e-150, 1e-300, 2.0 ** -1060])
def test_prefilter_extreme_scales(vq, scale):
    """Products that overflow to infinity, thresholds that become NaN or
    infinite, keys in the subnormal range: the kernels take every decision
    the oracle takes."""
    for dist in ("disk", "square", "kuzmin"):
        x, y = workloads.points(dist, 60_000, seed=31)
        check(x * scale, y * scale, f"{dist} x{scale:g}")
