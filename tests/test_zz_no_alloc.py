"""vqhull_hull_noalloc (every device table in the library's static per-GPU
array) through the C ABI against vqhull_hull, the existing entry point, and
the CPU oracle: bit-exact index lists on two calls in a row, the second
smaller than the first (the array keeps the first call's contents), plus the
sizes at the edges of its paths; more than VQHULL_NOALLOC_MAX_POINTS points
is refused on the host; and the calls take no device memory."""
import ctypes

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


def _both(vq, x, y):
    import torch

    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    n = len(x)
    o1 = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
    c1 = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    o2 = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
    c2 = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    vq.hull_noalloc_into(tx, ty, o1, c1)
    vq.hull_into(tx, ty, o2, c2)
    h1, h2 = int(c1.item()), int(c2.item())
    return o1[:max(h1, 0)].cpu().numpy(), h1, o2[:max(h2, 0)].cpu().numpy(), h2


def test_two_calls_second_smaller(vq):
    big = workloads.points("disk", vq.NOALLOC_MAX_POINTS, seed=[90, 1])
    small = workloads.points("circle", 300_000, seed=[90, 2])
    for x, y in (big, small):
        got, h, want_gpu, h2 = _both(vq, x, y)
        want = oracle.hull(x, y)
        assert h == h2 == len(want)
        assert np.array_equal(got, want_gpu) and np.array_equal(got, want)


@pytest.mark.parametrize("n", [0, 1, 2, 2048, 2049, 4097, 65_537, 1_000_000])
def test_edges_of_each_path(vq, n):
    for k, dist in enumerate(("square", "kuzmin")):
        x, y = workloads.points(dist, n, seed=[91, n, k])
        got, h, want_gpu, h2 = _both(vq, x, y)
        assert h == h2 and np.array_equal(got, want_gpu) and np.array_equal(got, oracle.hull(x, y)), (dist, n)


def test_lattice_with_duplicates_and_nan(vq):
    x, y = workloads.lattice(200_000, seed=92, hi=40, dup_frac=0.3, collinear_runs=5)
    got, h, want_gpu, _ = _both(vq, x, y)
    assert np.array_equal(got, want_gpu) and np.array_equal(got, oracle.hull(x, y))
    x = x.copy()
    x[12345] = np.nan
    _, h, _, h2 = _both(vq, x, y)
    assert h == h2 == -vq.VQHULL_ERR_NONFINITE


def test_too_many_points_refused(vq):
    lib = vq.load_library()
    dummy = ctypes.c_void_p(0x1000)
    assert lib.vqhull_hull_noalloc(dummy, dummy, vq.NOALLOC_MAX_POINTS + 1, dummy, dummy, None) == 1
    assert lib.vqhull_hull_noalloc(dummy, dummy, -1, dummy, dummy, None) == 1
    assert lib.vqhull_hull_noalloc(None, dummy, 5, dummy, dummy, None) == 1


def test_calls_take_no_device_memory(vq):
    import torch

    x, y = workloads.points("disk", vq.NOALLOC_MAX_POINTS, seed=[93, 1])
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    out = torch.empty(len(x), dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    vq.hull_noalloc_into(tx, ty, out, cnt)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        vq.hull_noalloc_into(tx, ty, out, cnt)
    torch.cuda.synchronize()
    assert abs(torch.cuda.mem_get_info()[0] - free0) < 8 << 20
    assert np.array_equal(out[:int(cnt.item())].cpu().numpy(), oracle.hull(x, y))
