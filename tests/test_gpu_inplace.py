"""In-place mode on the GPU (vqhull_hull_inplace, vqhull_hull_batched_inplace):
the caller's x and y double as one point buffer and are overwritten; the
index lists equal the CPU oracle's on the points they held on entry, element
by element: single requests of every distribution across the size paths
(one launch, the level loop, deep recursion), a batch of mixed sizes with an
empty and a non-finite request, the prefilter on, and lattices with
duplicates."""
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


@pytest.mark.parametrize("dist,n", [("disk", 7), ("square", 2048), ("kuzmin", 2049), ("circle", 70_001),
                                    ("disk", 1_000_000), ("circle", 3_000_000), ("square", 4_000_003)])
def test_inplace_single_matches_oracle(vq, dist, n):
    import torch

    x, y = workloads.points(dist, n, seed=[95, n])
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    got = vq.hull_inplace(tx, ty).cpu().numpy()
    assert np.array_equal(got, oracle.hull(x, y)), (dist, n)


def test_inplace_batched_matches_oracle(vq):
    import torch

    g = np.random.default_rng(96)
    sizes = [int(v) for v in np.clip(np.floor(16 * np.power(300_000 / 16, g.random(40))), 16, 300_000)]
    sizes[3] = 0
    xs, ys = [], []
    for i, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], n, seed=[96, i])
        xs.append(x)
        ys.append(y)
    xs[9] = xs[9].copy()
    xs[9][1] = np.inf
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    out, cnt = vq.hull_inplace(X, Y, off)
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    for i in range(len(sizes)):
        if i == 9:
            assert cnt[i] == -vq.VQHULL_ERR_NONFINITE
            continue
        assert np.array_equal(out[off[i]:off[i] + cnt[i]], oracle.hull(xs[i], ys[i])), i


def test_inplace_with_prefilter_and_lattices(vq):
    import torch

    old = vq.get_config()
    try:
        vq.set_config(prefilter=1)
        for k, (x, y) in enumerate([workloads.points("disk", 2_000_000, seed=97),
                                    workloads.lattice(500_000, seed=98, hi=300, dup_frac=0.3, collinear_runs=6)]):
            tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
            got = vq.hull_inplace(tx, ty).cpu().numpy()
            assert np.array_equal(got, oracle.hull_prefiltered(x, y, vq.get_config()["lds_limit"])), k
    finally:
        vq.set_config(**old)
