"""GPU parity at the full workload sizes, in the kernel configuration the
benchmark times: the complete index list of every hull is compared with the
CPU oracle's (bit-exact).  Inputs: the unit disk and unit square at 10^8
points (seed 2), the unit circle at 5*10^7 (seed 3) and the Kuzmin disk at
10^8 (seed 4), drawn by paper_2510_09417_amd.workloads."""
import time

import numpy as np
import pytest

import oracle
from paper_2510_09417_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vq():
    import torch

    import paper_2510_09417_amd as vq

    assert torch.cuda.is_available()
    vq.load_library()
    vq.set_config(sweep_block=512, sweep_ppt=8, lds_limit=2048, reverse_tiles=0, sweep_persistent=1, level_block=256, prefilter=0)
    yield vq
    vq.release_workspace()


@pytest.mark.parametrize("name", ["disk_1e8", "square_1e8", "kuzmin_1e8", "circle_5e7"])
def test_full_size_bit_exact(vq, name):
    import torch

    t0 = time.perf_counter()
    x, y = workloads.workload(name)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    got = vq.hull(tx, ty).cpu().numpy()
    del tx, ty
    t1 = time.perf_counter()
    want = oracle.hull(x, y)
    t2 = time.perf_counter()
    print(f"{name}: h={len(want)} gpu+transfer {t1 - t0:.1f}s oracle {t2 - t1:.1f}s", flush=True)
    assert len(got) == len(want)
    assert np.array_equal(got, want)
    # the result is a set of distinct input indices starting at the lexicographic minimum
    assert got[0] == int(np.lexsort((np.arange(len(x)), y, x))[0])


@pytest.mark.parametrize("name", ["disk_1e8", "square_1e8"])
def test_full_size_prefilter_bit_exact(vq, name):
    """The octagon prefilter at full size: bit-exact against the oracle's
    prefiltered variant, and the same list as the plain path."""
    import torch

    x, y = workloads.workload(name)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    plain = vq.hull(tx, ty).cpu().numpy()
    vq.set_config(prefilter=1)
    try:
        got = vq.hull(tx, ty).cpu().numpy()
        swept = vq.level_stats()[0]["swept"]
    finally:
        vq.set_config(prefilter=0)
    del tx, ty
    t0 = time.perf_counter()
    want = oracle.hull_prefiltered(x, y, 2048)
    keep = int(oracle.octagon(x, y)[1].sum())
    print(f"{name}: kept {keep} of {len(x)}; oracle variant {time.perf_counter() - t0:.1f}s", flush=True)
    assert swept == keep
    assert np.array_equal(got, want)
    assert np.array_equal(got, plain)


def test_full_size_interleaved_input(vq):
    """Disk 1e8 from interleaved (x, y) input, plain and with the prefilter:
    the same lists as the structure-of-arrays call (itself bit-exact against
    the oracle in the tests above)."""
    import torch

    x, y = workloads.workload("disk_1e8")
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    xy = torch.stack([tx, ty], dim=1).contiguous()
    del x, y
    try:
        for pf in (0, 1):
            vq.set_config(prefilter=pf)
            soa = vq.hull(tx, ty).cpu().numpy()
            aos = vq.hull_xy(xy).cpu().numpy()
            assert len(soa) == 1555 and np.array_equal(aos, soa), pf
    finally:
        vq.set_config(prefilter=0)


def test_disk_1e6_repeated_and_reversed(vq):
    """The 10^6-point disk (seed 1) in the benchmark configuration, then with the
    tile order reversed: the same list both times."""
    import torch

    x, y = workloads.workload("disk_1e6")
    want = oracle.hull(x, y)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    assert np.array_equal(vq.hull(tx, ty).cpu().numpy(), want)
    vq.set_config(reverse_tiles=1)
    try:
        assert np.array_equal(vq.hull(tx, ty).cpu().numpy(), want)
    finally:
        vq.set_config(reverse_tiles=0)
