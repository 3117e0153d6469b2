"""Inputs whose levels keep nearly all of their points (a circle: every point
a hull vertex) switch from the 2048-point LDS threshold to 1024 part-way down
the recursion; the levels planned before and after the switch are finished
with their own finisher sizes.  The index lists equal the CPU oracle's and
those of a run under the 1024 threshold throughout, alone and in a batch
where a disk shares the levels with the circle."""
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


def _run(vq, X, Y, off, **cfg):
    saved = vq.get_config()
    try:
        vq.set_config(**cfg)
        out, cnt = vq.hull_batched(X, Y, off)
        return out.cpu().numpy(), cnt.cpu().numpy()
    finally:
        vq.set_config(**saved)


@pytest.mark.parametrize("parts", [[("circle", 3_000_001)], [("circle", 2_500_000), ("disk", 2_000_000)]])
def test_switch_matches_oracle(vq, parts):
    import torch

    xs, ys = [], []
    for i, (d, n) in enumerate(parts):
        x, y = workloads.points(d, n, seed=[61, i])
        xs.append(x)
        ys.append(y)
    off = np.concatenate([[0], np.cumsum([n for _, n in parts])]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    out, cnt = _run(vq, X, Y, off, lds_limit=2048)
    out1, cnt1 = _run(vq, X, Y, off, lds_limit=1024)
    assert np.array_equal(cnt, cnt1)
    for i in range(len(parts)):
        assert np.array_equal(out[off[i]:off[i] + cnt[i]], out1[off[i]:off[i] + cnt1[i]]), parts[i]
    lib = oracle.load()
    for i in range(len(parts)):
        want = oracle.hull(xs[i], ys[i], lib)
        assert cnt[i] == len(want) and np.array_equal(out[off[i]:off[i] + cnt[i]], want), parts[i]
