"""The C ABI boundary on the CPU: the library loads, exports every function the
public header declares, and rejects bad arguments on the host (these calls
return before any HIP call, so no GPU is needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vqhull.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vqhull_[a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2510_09417_amd as vq

    return vq.load_library()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("vqhull_hull", "vqhull_hull_batched", "vqhull_status_string", "vqhull_stream_scale"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in include/vqhull.h but not exported"


def test_binding_lists_the_same_symbols():
    import paper_2510_09417_amd as vq

    assert sorted(vq.EXPORTED) == declared_functions()


def test_invalid_arguments_rejected_on_host(lib):
    vp = ctypes.c_void_p
    dummy = vp(0x1000)  # never dereferenced: the checks fail first
    one = (ctypes.c_int64 * 1)()
    assert lib.vqhull_hull(dummy, dummy, -1, dummy, dummy, None) == 1
    assert lib.vqhull_hull(dummy, dummy, 1 << 31, dummy, dummy, None) == 1
    assert lib.vqhull_hull(None, dummy, 5, dummy, dummy, None) == 1
    assert lib.vqhull_hull(dummy, dummy, 5, None, dummy, None) == 1
    assert lib.vqhull_hull(dummy, dummy, 5, dummy, None, None) == 1
    off = np.array([0, 5, 3], dtype=np.int64)  # decreasing
    p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    assert lib.vqhull_hull_batched(dummy, dummy, p, 2, dummy, dummy, None) == 1
    off2 = np.array([1, 5], dtype=np.int64)  # offsets[0] != 0
    assert lib.vqhull_hull_batched(dummy, dummy, off2.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, dummy,
                                   dummy, None) == 1
    assert lib.vqhull_hull_batched(dummy, dummy, None, 1, dummy, dummy, None) == 1
    assert lib.vqhull_hull_batched(dummy, dummy, p, -1, dummy, dummy, None) == 1
    # interleaved input: misaligned (not a whole double2), null, bad offsets
    assert lib.vqhull_hull_xy(vp(0x1008), 5, dummy, dummy, None) == 1
    assert lib.vqhull_hull_xy(None, 5, dummy, dummy, None) == 1
    assert lib.vqhull_hull_xy(dummy, -1, dummy, dummy, None) == 1
    assert lib.vqhull_hull_xy(dummy, 5, None, dummy, None) == 1
    assert lib.vqhull_hull_batched_xy(dummy, p, 2, dummy, dummy, None) == 1
    ok = np.array([0, 5], dtype=np.int64)
    q = ok.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    assert lib.vqhull_hull_batched_xy(vp(0x1008), q, 1, dummy, dummy, None) == 1
    assert lib.vqhull_hull_batched_xy(None, q, 1, dummy, dummy, None) == 1
    assert lib.vqhull_hull_batched_xy(dummy, q, 1, None, dummy, None) == 1
    assert lib.vqhull_orient(dummy, -1, dummy, None) == 1
    assert lib.vqhull_orient(None, 3, dummy, None) == 1
    assert lib.vqhull_orient(dummy, 3, None, None) == 1
    assert lib.vqhull_stream_scale(dummy, dummy, -1, 2.0, None) == 1
    assert lib.vqhull_stream_scale(None, dummy, 4, 2.0, None) == 1
    assert one[0] == 0


def test_timing_modes_on_host(lib):
    try:
        for mode in (0, 1, 2, 3):
            assert lib.vqhull_set_timing(mode) == 0
        for bad in (-1, 4, 100):
            assert lib.vqhull_set_timing(bad) == 1
    finally:
        assert lib.vqhull_set_timing(0) == 0


def test_level_pair_modes_on_host(lib):
    try:
        for mode in (0, 1, 2):
            assert lib.vqhull_set_level_pairs(mode) == 0
        for bad in (-1, 3, 100):
            assert lib.vqhull_set_level_pairs(bad) == 1
    finally:
        assert lib.vqhull_set_level_pairs(1) == 0  # the default


def test_status_strings(lib):
    for code in range(6):
        assert lib.vqhull_status_string(code)
    assert b"unknown" in lib.vqhull_status_string(99)


def test_config_roundtrip_and_sanitizing():
    import paper_2510_09417_amd as vq

    old = vq.get_config()
    try:
        c = vq.set_config(sweep_block=256, sweep_ppt=16, lds_limit=1000, reverse_tiles=5, sweep_persistent=0)
        assert (c["sweep_block"], c["sweep_ppt"], c["lds_limit"], c["reverse_tiles"], c["sweep_persistent"]) == \
            (256, 16, 1000, 1, 0)
        c = vq.set_config(sweep_block=300, sweep_ppt=7, lds_limit=10**6)
        assert (c["sweep_block"], c["sweep_ppt"], c["lds_limit"]) == (256, 16, 2048)  # the default shape
        # deeper levels: a workgroup size with the same tile, else the sweep shape (0)
        assert vq.set_config(sweep_block=512, sweep_ppt=8, level_block=256)["level_block"] == 256
        assert vq.set_config(level_block=512)["level_block"] == 0  # the sweep shape itself
        assert vq.set_config(level_block=1024)["level_block"] == 0  # 1024 x 4 is not a shape
        assert vq.set_config(sweep_block=256, sweep_ppt=32, level_block=1024)["level_block"] == 1024
        assert vq.set_config(level_block=-3)["level_block"] == 0
    finally:
        vq.set_config(**old)


def test_python_binding_checks():
    import torch

    import paper_2510_09417_amd as vq

    with pytest.raises(TypeError):
        vq.hull(torch.zeros(3, dtype=torch.float32), torch.zeros(3, dtype=torch.float32))
    with pytest.raises(ValueError):
        vq.hull(torch.zeros(3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64))  # not on a GPU


def test_server_arguments_rejected_on_host(lib):
    import paper_2510_09417_amd as vq

    vq.load_library()
    vp = ctypes.c_void_p
    h = vp()
    assert lib.vqhull_server_create(None, ctypes.byref(h)) == 1
    for lanes, pts, reqs, lv in ((0, 1000, 10, 0), (9, 1000, 10, 0), (1, 0, 10, 0), (1, 1 << 31, 10, 0),
                                 (1, 1000, 0, 0), (1, 1000, (1 << 24) + 1, 0), (1, 1000, 10, -1), (1, 1000, 10, 65)):
        cfg = vq.ServerConfig(lanes, lv, pts, reqs)
        assert lib.vqhull_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1
    t = ctypes.c_int64()
    dummy = vp(0x1000)
    assert lib.vqhull_server_submit(None, dummy, dummy, 5, dummy, dummy, ctypes.byref(t)) == 1
    assert lib.vqhull_server_submit_batch(None, 1, dummy, dummy, dummy, dummy, dummy, ctypes.byref(t)) == 1
    assert lib.vqhull_server_wait(None, 0) == 1
    lib.vqhull_server_wait_timeout.argtypes = [vp, ctypes.c_int64, ctypes.c_double]
    assert lib.vqhull_server_wait_timeout(None, 0, 1.0) == 1
    assert lib.vqhull_server_poll(None, None, 0) == -1
    assert lib.vqhull_server_drain(None) == 1
    assert lib.vqhull_server_ticket_info(None, 0, None) == 1
    assert lib.vqhull_server_stats(None, None) == 1
    assert lib.vqhull_server_destroy(None) == 1


def test_kernel_kind_names_follow_the_header():
    import paper_2510_09417_amd as vq

    text = open(HEADER).read()
    kinds = dict((int(v), k.lower()) for k, v in re.findall(r"VQHULL_K_([A-Z0-9_]+)\s*=\s*(\d+)", text))
    assert sorted(kinds) == list(range(len(vq.KERNEL_KINDS)))
    names = {"plan": "finish_plan"}  # the level planner shares its launch with the finisher
    assert [names.get(kinds[i], kinds[i]) for i in range(len(kinds))] == list(vq.KERNEL_KINDS)


def test_config_has_prefilter_flag():
    import paper_2510_09417_amd as vq

    old = vq.get_config()
    try:
        assert vq.set_config(prefilter=7)["prefilter"] == 1
        assert vq.set_config(prefilter=0)["prefilter"] == 0
    finally:
        vq.set_config(**old)


def test_status_constants_follow_the_header():
    """The binding's status constants equal the header's vqhull_status enum,
    and every status has its own text."""
    import re

    import paper_2510_09417_amd as vq

    text = open(HEADER).read()
    body = text[text.index("typedef enum {"): text.index("} vqhull_status;")]
    enum = {m.group(1): int(m.group(2)) for m in re.finditer(r"(VQHULL_(?:OK|ERR_[A-Z_]+))\s*=\s*(\d+)", body)}
    assert len(enum) >= 6
    for name, value in enum.items():
        assert getattr(vq, name) == value, name
    lib = vq.load_library()
    texts = {lib.vqhull_status_string(v) for v in enum.values()}
    assert len(texts) == len(enum) and not any(b"unknown" in t for t in texts)


def test_workspace_bytes_on_host():
    """vqhull_workspace_bytes: 0 outside [0, 2^31); about 72 bytes per point
    (two 20-byte ping-pong point buffers and one 32-byte node per point) plus
    tables, growing with the point count and the request count, and following
    the configuration's LDS threshold (segment tables)."""
    import paper_2510_09417_amd as vq

    lib = vq.load_library()
    assert lib.vqhull_workspace_bytes(-1, 1) == 0
    assert lib.vqhull_workspace_bytes(1 << 31, 1) == 0
    assert lib.vqhull_workspace_bytes(10, -1) == 0
    with pytest.raises(ValueError):
        vq.workspace_bytes(-5)
    small = vq.workspace_bytes(0, 0)
    assert 0 < small < 1 << 20
    prev = 0
    for n in (1, 1000, 10**6, 10**8):
        b = vq.workspace_bytes(n, 1)
        assert b > prev and b % 256 == 0
        prev = b
    b = vq.workspace_bytes(10**8, 1)
    assert 72 * 10**8 <= b <= 76 * 10**8
    assert vq.workspace_bytes(10**6, 1000) > vq.workspace_bytes(10**6, 1)
    old = vq.get_config()
    try:
        vq.set_config(lds_limit=256)
        b256 = vq.workspace_bytes(10**7, 1)
        vq.set_config(lds_limit=2048)
        assert b256 > vq.workspace_bytes(10**7, 1)
    finally:
        vq.set_config(**old)


def test_workspace_calls_reject_bad_arguments_on_host(lib):
    """The _ws calls check their arguments and the workspace (null, not
    256-byte aligned, smaller than vqhull_workspace_bytes) before any HIP
    call."""
    import paper_2510_09417_amd as vq

    vp = ctypes.c_void_p
    dummy = vp(0x1000)
    need = vq.workspace_bytes(5, 1)
    ws = vp(0x100000)
    assert lib.vqhull_hull_ws(dummy, dummy, -1, dummy, dummy, ws, need, None) == 1
    assert lib.vqhull_hull_ws(None, dummy, 5, dummy, dummy, ws, need, None) == 1
    assert lib.vqhull_hull_ws(dummy, dummy, 5, None, dummy, ws, need, None) == 1
    assert lib.vqhull_hull_ws(dummy, dummy, 5, dummy, dummy, None, need, None) == 1
    assert lib.vqhull_hull_ws(dummy, dummy, 5, dummy, dummy, vp(0x100080), need, None) == 1  # misaligned
    assert lib.vqhull_hull_ws(dummy, dummy, 5, dummy, dummy, ws, need - 1, None) == 1  # too small
    off = np.array([0, 3, 5], dtype=np.int64)
    p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    need2 = vq.workspace_bytes(5, 2)
    assert lib.vqhull_hull_batched_ws(dummy, dummy, p, 2, dummy, dummy, ws, need2 - 256, None) == 1
    assert lib.vqhull_hull_batched_ws(dummy, dummy, p, 2, dummy, dummy, None, need2, None) == 1
    bad = np.array([0, 5, 3], dtype=np.int64)
    assert lib.vqhull_hull_batched_ws(dummy, dummy, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2, dummy,
                                      dummy, ws, need2, None) == 1
    assert lib.vqhull_hull_batched_ws(dummy, dummy, None, 2, dummy, dummy, ws, need2, None) == 1
    assert lib.vqhull_hull_batched_ws(dummy, dummy, p, 0, dummy, dummy, None, 0, None) == 0  # nothing to do


def test_async_call_rejects_bad_arguments_on_host(lib):
    """The stream-ordered batched call checks its sizes, offsets, level budget
    (1 .. 4096) and workspace (the _ws one) before any HIP call, and returns
    at once with nothing to do for no requests."""
    import paper_2510_09417_amd as vq

    vp = ctypes.c_void_p
    dummy = vp(0x1000)
    off = np.array([0, 3, 5], dtype=np.int64)
    p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    need = vq.workspace_bytes(5, 2)
    ws = vp(0x100000)
    f = lib.vqhull_hull_batched_async
    for levels in (0, -3, 4097):
        assert f(dummy, dummy, p, 2, dummy, dummy, levels, ws, need, None) == 1
    assert f(dummy, dummy, p, -1, dummy, dummy, 8, ws, need, None) == 1
    assert f(dummy, dummy, None, 2, dummy, dummy, 8, ws, need, None) == 1
    bad = np.array([0, 5, 3], dtype=np.int64)
    assert f(dummy, dummy, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2, dummy, dummy, 8, ws, need,
             None) == 1
    assert f(None, dummy, p, 2, dummy, dummy, 8, ws, need, None) == 1
    assert f(dummy, dummy, p, 2, None, dummy, 8, ws, need, None) == 1
    assert f(dummy, dummy, p, 2, dummy, None, 8, ws, need, None) == 1
    assert f(dummy, dummy, p, 2, dummy, dummy, 8, None, need, None) == 1
    assert f(dummy, dummy, p, 2, dummy, dummy, 8, vp(0x100080), need, None) == 1  # misaligned
    assert f(dummy, dummy, p, 2, dummy, dummy, 8, ws, need - 256, None) == 1  # too small
    assert f(dummy, dummy, p, 0, dummy, dummy, 8, None, 0, None) == 0  # nothing to do
    assert lib.vqhull_status_string(6) == b"the level budget ended before the recursion"


def test_inplace_workspace_and_arguments_on_host(lib):
    """In-place mode: its workspace is the _ws one less buffer A's two
    coordinate arrays (16 bytes per point), and its calls check arguments and
    the workspace before any HIP call."""
    import paper_2510_09417_amd as vq

    for n, nreq in ((10**6, 1), (10**8, 1), (10**7, 500)):
        full, inpl = vq.workspace_bytes(n, nreq), lib.vqhull_workspace_bytes_inplace(n, nreq)
        assert full - inpl == 2 * ((8 * n + 255) // 256 * 256)
    assert lib.vqhull_workspace_bytes_inplace(-1, 1) == 0
    vp = ctypes.c_void_p
    dummy = vp(0x1000)
    ws = vp(0x100000)
    need = lib.vqhull_workspace_bytes_inplace(5, 1)
    assert lib.vqhull_hull_inplace(dummy, dummy, -1, dummy, dummy, ws, need, None) == 1
    assert lib.vqhull_hull_inplace(None, dummy, 5, dummy, dummy, ws, need, None) == 1
    assert lib.vqhull_hull_inplace(dummy, dummy, 5, dummy, dummy, ws, need - 1, None) == 1
    assert lib.vqhull_hull_inplace(dummy, dummy, 5, dummy, dummy, vp(0x100010), need, None) == 1
    off = np.array([0, 3, 5], dtype=np.int64)
    p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    need2 = lib.vqhull_workspace_bytes_inplace(5, 2)
    assert lib.vqhull_hull_batched_inplace(dummy, dummy, p, 2, dummy, dummy, ws, need2 - 256, None) == 1
    assert lib.vqhull_hull_batched_inplace(dummy, dummy, None, 2, dummy, dummy, ws, need2, None) == 1
