"""Kernel timing records: every launch (mode 1), the partition sweeps only
(mode 2) or the fused top-level pass only (mode 3, the benchmark's timed
region), and the result does not depend on the timing mode."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_timing_modes():
    import torch

    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    vq.load_library()
    x, y = workloads.points("disk", 300_001, seed=41)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    ref = vq.hull(tx, ty).cpu().numpy()
    try:
        vq.set_timing(True)
        h1 = vq.hull(tx, ty).cpu().numpy()
        all_kinds = {r["kind"] for r in vq.kernel_times()}
        vq.set_timing(True, sweeps_only=True)
        h2 = vq.hull(tx, ty).cpu().numpy()
        recs = vq.kernel_times()
        vq.set_timing(True, fused_only=True)
        h3 = vq.hull(tx, ty).cpu().numpy()
        fused = vq.kernel_times()
    finally:
        vq.set_timing(False)
    assert np.array_equal(h1, ref) and np.array_equal(h2, ref) and np.array_equal(h3, ref)
    # mode 3: one record, the level-1 sweep, with the same point counts as in mode 2
    assert [(r["kind"], r["level"]) for r in fused] == [("sweep", 1)]
    assert fused[0]["points_in"] == recs[1]["points_in"] == len(x)
    assert fused[0]["points_out"] == recs[1]["points_out"] > 0
    assert {"extremes", "plan0", "sweep", "finish_plan", "assemble"} <= all_kinds
    assert recs and {r["kind"] for r in recs} == {"sweep"}
    levels = [r["level"] for r in recs]
    assert levels == list(range(len(levels)))  # one sweep per level, in order
    assert recs[0]["points_in"] == len(x)  # the argmax pass reads every point
    assert all(r["ms"] >= 0.0 for r in recs)
