"""GPU test of the level planner's rounds: a level with far more segments than
one planner round holds is planned by several workgroups, each round's
output offsets found by a look-back over the rounds before it, 64 rounds a
step.  40 000 requests of 513-700 points under an LDS threshold of 512
(256-thread planner rounds) give the root level some 157 rounds, so the
look-back crosses more than two of its 64-round windows; every request's
index list is compared element by element with the CPU oracle's."""
import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu

NREQ = 40_000


def test_many_rounds_match_oracle():
    import torch

    import paper_2510_09417_amd as vq

    vq.load_library()
    g = np.random.default_rng(123)
    sizes = g.integers(513, 701, size=NREQ)
    xs, ys = [], []
    for i, n in enumerate(sizes):
        x, y = workloads.points(workloads.DISTRIBUTIONS[i % 4], int(n), seed=[123, i])
        xs.append(x)
        ys.append(y)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).cuda()
    Y = torch.from_numpy(np.concatenate(ys)).cuda()
    saved = vq.get_config()
    try:
        vq.set_config(lds_limit=512)
        out, cnt = vq.hull_batched(X, Y, off)
        levels = vq.level_stats()
    finally:
        vq.set_config(**saved)
    assert levels[0]["segments"] == NREQ  # every request a root segment: ~157 rounds of 256
    out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
    lib = oracle.load()
    for i in range(NREQ):
        want = oracle.hull(xs[i], ys[i], lib)
        assert cnt[i] == len(want) and np.array_equal(out[off[i]:off[i] + cnt[i]], want), i
