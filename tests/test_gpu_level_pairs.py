"""Level pairs below the top: a level swept without writing (sizes and
farthest points of its segments' children), then the next level read in
place from it, classified against the segment (a, r, b) and then against its
child (a, r1, r) or (r, r2, b), its grandchildren written.  Every index list
equals the CPU oracle's element by element, with pairs forced on every level
from the third (every distribution, single and batched, every entry point
that runs the level loop, several sweep shapes, per-tile grids) and chosen
adaptively (circles); the recorded level kinds show the pairs."""
import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vq():
    import paper_2510_09417_amd as m

    m.load_library()
    yield m
    m.set_level_pairs(1)


def _pairs_in(levels):
    """Levels >= 2 come as (argmax, fused) pairs or single level sweeps; the
    last level (no segment left) may be the first of a pair that never ran."""
    kinds = [lv["sweep"] for lv in levels]
    assert levels[-1]["segments"] == 0
    k, n = 2, 0
    while k < len(kinds):
        if kinds[k] == "argmax" and k + 1 < len(kinds):
            assert kinds[k + 1] == "fused", kinds
            k, n = k + 2, n + 1
        else:
            assert kinds[k] == "level" or k == len(kinds) - 1, kinds
            k += 1
    return n


def _dev(x, y):
    import torch

    return torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()


@pytest.mark.parametrize("dist,n", [("disk", 300_001), ("square", 1_000_003), ("kuzmin", 700_001), ("circle", 200_003),
                                    ("circle", 2_000_001), ("disk", 4_000_037)])
def test_forced_pairs_match_oracle(vq, dist, n):
    x, y = workloads.points(dist, n, seed=[71, n])
    tx, ty = _dev(x, y)
    want = oracle.hull(x, y)
    try:
        vq.set_level_pairs(2)
        got = vq.hull(tx, ty).cpu().numpy()
        levels = vq.level_stats()
    finally:
        vq.set_level_pairs(1)
    assert [lv["sweep"] for lv in levels[:2]] == ["argmax", "fused"]
    if len(levels) >= 5:
        assert _pairs_in(levels) >= 1
    assert np.array_equal(got, want), (dist, n, len(got), len(want))


def test_adaptive_pairs_on_a_circle(vq):
    x, y = workloads.points("circle", 3_000_017, seed=72)
    tx, ty = _dev(x, y)
    got = vq.hull(tx, ty).cpu().numpy()
    assert _pairs_in(vq.level_stats()) >= 2
    vq.set_level_pairs(0)
    try:
        plain = vq.hull(tx, ty).cpu().numpy()
        assert _pairs_in(vq.level_stats()) == 0
    finally:
        vq.set_level_pairs(1)
    assert np.array_equal(got, plain)
    assert np.array_equal(got, oracle.hull(x, y))


def test_adaptive_pairs_leave_a_disk_alone(vq):
    x, y = workloads.points("disk", 2_000_003, seed=73)
    got = vq.hull(*_dev(x, y)).cpu().numpy()
    assert _pairs_in(vq.level_stats()) == 0
    assert np.array_equal(got, oracle.hull(x, y))


MIX = [("circle", 400_001), ("disk", 150_000), ("square", 3000), ("kuzmin", 90_000), ("circle", 2049), ("disk", 5),
       ("square", 0), ("circle", 60_000), ("kuzmin", 1), ("disk", 1_000_000)]


def _batch(tag):
    xs, ys = [], []
    for i, (d, n) in enumerate(MIX):
        x, y = workloads.points(d, n, seed=[tag, i])
        xs.append(x)
        ys.append(y)
    off = np.concatenate([[0], np.cumsum([n for _, n in MIX])]).astype(np.int64)
    return xs, ys, off


@pytest.mark.parametrize("form", ["batched", "ws", "xy", "inplace"])
def test_forced_pairs_batched_forms(vq, form):
    import torch

    xs, ys, off = _batch(74)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    try:
        vq.set_level_pairs(2)
        if form == "batched":
            out, cnt = vq.hull_batched(X, Y, off)
        elif form == "ws":
            out, cnt = vq.hull_batched_ws(X, Y, off)
        elif form == "xy":
            out, cnt = vq.hull_batched_xy(torch.stack([X, Y], dim=1).contiguous(), off)
        else:
            out, cnt = vq.hull_inplace(X.clone(), Y.clone(), off)
        levels = vq.level_stats()
    finally:
        vq.set_level_pairs(1)
    assert _pairs_in(levels) >= 1
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    for i in range(len(MIX)):
        want = oracle.hull(xs[i], ys[i])
        assert cnt[i] == len(want) and np.array_equal(out[off[i]:off[i] + cnt[i]], want), (form, i, MIX[i])


@pytest.mark.parametrize("cfg", [dict(sweep_block=512, sweep_ppt=8, level_block=256), dict(sweep_block=256, sweep_ppt=32),
                                 dict(sweep_persistent=0), dict(lds_limit=512), dict(prefilter=1),
                                 dict(reverse_tiles=1)])
def test_forced_pairs_configurations(vq, cfg):
    x, y = workloads.points("circle", 500_009, seed=75)
    x2, y2 = workloads.points("disk", 800_011, seed=76)
    want = [oracle.hull(x, y), oracle.hull(x2, y2)]
    saved = vq.get_config()
    try:
        vq.set_config(**cfg)
        vq.set_level_pairs(2)
        got = [vq.hull(*_dev(x, y)).cpu().numpy(), vq.hull(*_dev(x2, y2)).cpu().numpy()]
    finally:
        vq.set_level_pairs(1)
        vq.set_config(**saved)
    for g, w in zip(got, want):
        assert np.array_equal(g, w), cfg

