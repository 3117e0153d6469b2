"""Autotuner: the cache's keys and lookup (CPU), and on the GPU that every
configuration gives the same hull and the winner is one of them."""
import json

import numpy as np
import pytest

from paper_2510_09417_amd import autotune


def test_bucket_and_lookup(tmp_path):
    p = str(tmp_path / "t.json")
    assert autotune.bucket(1) == 1 and autotune.bucket(1 << 20) == 21 and autotune.bucket((1 << 20) - 1) == 20
    autotune.store({"gfx950/256cu/b21": {"config": {"lds_limit": 1024}}, "gfx950/256cu/b27": {"config": {"lds_limit": 2048}},
                    "gfx942/304cu/b21": {"config": {"lds_limit": 512}}}, p)
    c = autotune.load(p)
    assert autotune.lookup(c, "gfx950/256cu", 1 << 20)["config"]["lds_limit"] == 1024
    assert autotune.lookup(c, "gfx950/256cu", 1 << 26)["config"]["lds_limit"] == 2048  # nearest bucket
    assert autotune.lookup(c, "gfx942/304cu", 10)["config"]["lds_limit"] == 512
    assert autotune.lookup(c, "gfx90a/104cu", 10) is None
    with open(p) as f:
        assert json.load(f) == c


def test_missing_or_corrupt_cache(tmp_path):
    assert autotune.load(str(tmp_path / "none.json")) == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert autotune.load(str(bad)) == {}


@pytest.mark.gpu
def test_autotune_same_result_everywhere(tmp_path):
    import torch

    import oracle
    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    vq.load_library()
    before = vq.get_config()
    x, y = workloads.points("circle", 200_003, seed=21)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    e = autotune.tune(tx, ty, repeats=1, path=str(tmp_path / "c.json"))
    assert vq.get_config() == before  # tuning leaves the configuration alone
    assert len(e["table"]) == 30 and all(r["same_result"] for r in e["table"])
    assert e["config"] in [r["config"] for r in e["table"]]
    try:
        assert autotune.apply(200_003, path=str(tmp_path / "c.json")) == e["config"]
        assert np.array_equal(vq.hull(tx, ty).cpu().numpy(), oracle.hull(x, y))
    finally:
        vq.set_config(**before)


@pytest.mark.gpu
def test_tune_batched_same_result_everywhere():
    import torch

    import oracle
    import paper_2510_09417_amd as vq
    from paper_2510_09417_amd import workloads

    vq.load_library()
    before = vq.get_config()
    parts = [workloads.points(d, n, seed=30 + k) for k, (d, n) in
             enumerate([("disk", 40_000), ("circle", 5_001), ("square", 17), ("kuzmin", 120_000), ("circle", 3_000)])]
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])]).astype(np.int64)
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    best, table = autotune.tune_batched(tx, ty, off, repeats=1)
    assert vq.get_config() == before  # tuning leaves the configuration alone
    assert len(table) == 30 and all(r["same_result"] for r in table)
    assert best in [r["config"] for r in table]
    try:
        vq.set_config(**best)
        out, cnt = vq.hull_batched(tx, ty, off)
        out, cnt = out.cpu().numpy(), cnt.cpu().numpy()
        for i, (px, py) in enumerate(parts):
            assert np.array_equal(out[off[i]:off[i] + cnt[i]], oracle.hull(px, py))
    finally:
        vq.set_config(**before)
