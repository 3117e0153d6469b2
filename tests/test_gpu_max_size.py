"""The largest request the library accepts, n = 2^31 - 1 points (positions and
offsets at the top of their 32-bit range), drawn on the GPU from a seeded
generator (uniform unit square).  The oracle does not run at this size, so
the result is checked by properties that hold at any size:
* every index is distinct and in range, and the first is the lexicographic
  minimum of (x, y, index) (computed on the GPU by torch);
* consecutive vertices turn strictly clockwise (exact rational arithmetic);
* 8*10^6 sampled input points are not outside any hull edge by more than the
  binary64 rounding bound of the orientation value;
* the same list with the octagon prefilter on (a second code path).
The calls use the library-owned workspace (vqhull_hull): about 150 GB of
device memory in all; everything is released at the end."""
import numpy as np
import pytest
from fractions import Fraction

pytestmark = pytest.mark.gpu

N = (1 << 31) - 1


@pytest.fixture(scope="module")
def vq():
    import torch

    import paper_2510_09417_amd as vq

    assert torch.cuda.is_available()
    vq.load_library()
    vq.set_config(sweep_block=512, sweep_ppt=8, lds_limit=2048, reverse_tiles=0, sweep_persistent=1,
                  level_block=256, prefilter=0)
    yield vq
    vq.set_config(prefilter=0)
    vq.release_workspace()
    torch.cuda.empty_cache()


def test_max_size_square(vq):
    import torch

    vq.release_workspace()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 200 * (1 << 30):
        pytest.skip(f"needs about 200 GiB of free device memory, {free >> 30} GiB free")
    g = torch.Generator(device="cuda")
    g.manual_seed(2031)
    x = torch.rand(N, dtype=torch.float64, device="cuda", generator=g)
    y = torch.rand(N, dtype=torch.float64, device="cuda", generator=g)
    def hull(x, y):  # the library-owned workspace (40 B per point): the _ws path needs 73 B per point
        oi = torch.empty(N, dtype=torch.int64, device="cuda")
        oc = torch.empty(1, dtype=torch.int64, device="cuda")
        vq.hull_into(x, y, oi, oc)
        return oi[: int(oc.item())]

    try:
        out = hull(x, y)
        h = out.numel()
        idx = out.cpu().numpy()
        assert 3 <= h < 1000
        assert len(np.unique(idx)) == h and idx.min() >= 0 and idx.max() < N
        # lexicographic minimum (x, then y, then index) by torch on the device
        xmin = x.min()
        cand = torch.nonzero(x == xmin).flatten()
        ymin = y[cand].min()
        p = int(cand[y[cand] == ymin].min().item())
        assert int(idx[0]) == p
        hx = x[out].cpu().numpy()
        hy = y[out].cpu().numpy()
        # strictly clockwise, exactly
        for k in range(h):
            a, b, c = k, (k + 1) % h, (k + 2) % h
            ax, ay, bx, by, cx, cy = (Fraction(float(v)) for v in (hx[a], hy[a], hx[b], hy[b], hx[c], hy[c]))
            assert (bx - ax) * (cy - ay) - (by - ay) * (cx - ax) < 0, k
        # sampled points are inside every clockwise edge up to the rounding bound
        s = torch.randint(0, N, (8_000_000,), device="cuda", generator=g)
        sx, sy = x[s], y[s]
        ex = torch.from_numpy(hx).cuda()
        ey = torch.from_numpy(hy).cuda()
        for k in range(h):
            a, b = k, (k + 1) % h
            dx, dy = ex[b] - ex[a], ey[b] - ey[a]
            o = dx * (sy - ey[a]) - dy * (sx - ex[a])  # > 0: left of a clockwise edge = outside
            bound = 8 * 2.0 ** -53 * (dx.abs() * (sy - ey[a]).abs() + dy.abs() * (sx - ex[a]).abs())
            assert not bool((o > bound).any()), f"a sampled point is outside edge {k}"
        # the prefiltered path gives the same list
        vq.set_config(prefilter=1)
        try:
            assert torch.equal(hull(x, y), out)
        finally:
            vq.set_config(prefilter=0)
        print(f"max size: n={N} h={h}, {torch.cuda.max_memory_allocated() >> 30} GiB allocated at most", flush=True)
    finally:
        del x, y
        vq.release_workspace()
        torch.cuda.empty_cache()
