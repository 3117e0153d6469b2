"""MI355X-native planar Quickhull (the VQhull paper's Algorithm 1 on gfx950).

Thin ctypes binding of ``libvqhull.so``: argument checks and marshalling only;
every step of the hull runs in the library's HIP kernels.  PyTorch provides the
device tensors and the current stream.  If the library is not built this
module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvqhull.so")

VQHULL_OK = 0
VQHULL_ERR_INVALID_ARGUMENT = 1
VQHULL_ERR_OUT_OF_MEMORY = 2
VQHULL_ERR_NONFINITE = 3
VQHULL_ERR_HIP = 4
VQHULL_ERR_TIMEOUT = 5
VQHULL_ERR_INCOMPLETE = 6

# Symbols that include/vqhull.h declares.
EXPORTED = (
    "vqhull_hull", "vqhull_hull_batched", "vqhull_workspace_bytes", "vqhull_hull_ws", "vqhull_hull_batched_ws",
    "vqhull_hull_batched_async",
    "vqhull_workspace_bytes_inplace", "vqhull_hull_inplace", "vqhull_hull_batched_inplace",
    "vqhull_hull_noalloc", "vqhull_hull_xy", "vqhull_hull_batched_xy", "vqhull_get_config", "vqhull_set_config", "vqhull_autotune",
    "vqhull_last_level_stats", "vqhull_last_level_kinds", "vqhull_set_level_pairs", "vqhull_set_timing", "vqhull_last_kernel_times", "vqhull_orient", "vqhull_stream_scale",
    "vqhull_release_workspace", "vqhull_status_string", "vqhull_last_error",
    "vqhull_server_create", "vqhull_server_submit", "vqhull_server_submit_batch", "vqhull_server_wait", "vqhull_server_wait_timeout",
    "vqhull_server_poll",
    "vqhull_server_drain", "vqhull_server_ticket_info", "vqhull_server_stats", "vqhull_server_destroy",
)

SWEEP_KINDS = ("level", "argmax", "fused")  # VQHULL_SWEEP_*: how a level's sweep read and wrote its points
KERNEL_KINDS = ("extremes", "plan0", "sweep", "finish_plan", "finish", "assemble", "filter", "compact", "ingest")


class VqhullError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vqhull status {status}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("sweep_block", ctypes.c_int), ("sweep_ppt", ctypes.c_int), ("lds_limit", ctypes.c_int),
                ("reverse_tiles", ctypes.c_int), ("sweep_persistent", ctypes.c_int), ("level_block", ctypes.c_int),
                ("prefilter", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("cfg", Config), ("ms", ctypes.c_double), ("same_result", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("level", ctypes.c_int32), ("ms", ctypes.c_double),
                ("points_in", ctypes.c_int64), ("points_out", ctypes.c_int64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("graph_levels", ctypes.c_int32), ("lane_points", ctypes.c_int64),
                ("lane_requests", ctypes.c_int64)]


class TicketInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("batch", ctypes.c_int64), ("lane", ctypes.c_int32),
                ("status", ctypes.c_int32), ("done", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("points", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("busy_seconds", ctypes.c_double), ("now", ctypes.c_double), ("graph_batches", ctypes.c_int64),
                ("plain_batches", ctypes.c_int64)]


_lock = threading.Lock()
_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load ``libvqhull.so`` (raises FileNotFoundError if it has not been built).

    torch is imported first: its wheel carries its own HIP runtime, whose
    soname (libamdhip64.so.7) the library's dependency then resolves to, so the
    process holds one HIP runtime.  Loaded the other way round, the process
    would hold two, and the one initialized second sees no GPU."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} is not built; run `python -m paper_2510_09417_amd.build`")
        import torch  # noqa: F401  (see above)

        lib = ctypes.CDLL(path)
        vp, i64, pi64 = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)
        lib.vqhull_hull.restype = ctypes.c_int
        lib.vqhull_hull.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.vqhull_hull_batched.restype = ctypes.c_int
        lib.vqhull_hull_batched.argtypes = [vp, vp, pi64, i64, vp, vp, vp]
        lib.vqhull_workspace_bytes.restype = ctypes.c_size_t
        lib.vqhull_workspace_bytes.argtypes = [i64, i64]
        lib.vqhull_hull_ws.restype = ctypes.c_int
        lib.vqhull_hull_ws.argtypes = [vp, vp, i64, vp, vp, vp, ctypes.c_size_t, vp]
        lib.vqhull_hull_batched_ws.restype = ctypes.c_int
        lib.vqhull_hull_batched_ws.argtypes = [vp, vp, pi64, i64, vp, vp, vp, ctypes.c_size_t, vp]
        lib.vqhull_hull_batched_async.restype = ctypes.c_int
        lib.vqhull_hull_batched_async.argtypes = [vp, vp, pi64, i64, vp, vp, ctypes.c_int32, vp, ctypes.c_size_t, vp]
        lib.vqhull_workspace_bytes_inplace.restype = ctypes.c_size_t
        lib.vqhull_workspace_bytes_inplace.argtypes = [i64, i64]
        lib.vqhull_hull_inplace.restype = ctypes.c_int
        lib.vqhull_hull_inplace.argtypes = [vp, vp, i64, vp, vp, vp, ctypes.c_size_t, vp]
        lib.vqhull_hull_batched_inplace.restype = ctypes.c_int
        lib.vqhull_hull_batched_inplace.argtypes = [vp, vp, pi64, i64, vp, vp, vp, ctypes.c_size_t, vp]
        lib.vqhull_hull_noalloc.restype = ctypes.c_int
        lib.vqhull_hull_noalloc.argtypes = [vp, vp, i64, vp, vp, vp]
        lib.vqhull_hull_xy.restype = ctypes.c_int
        lib.vqhull_hull_xy.argtypes = [vp, i64, vp, vp, vp]
        lib.vqhull_hull_batched_xy.restype = ctypes.c_int
        lib.vqhull_hull_batched_xy.argtypes = [vp, pi64, i64, vp, vp, vp]
        lib.vqhull_get_config.restype = ctypes.c_int
        lib.vqhull_get_config.argtypes = [ctypes.POINTER(Config)]
        lib.vqhull_set_config.restype = ctypes.c_int
        lib.vqhull_set_config.argtypes = [ctypes.POINTER(Config)]
        lib.vqhull_autotune.restype = ctypes.c_int
        lib.vqhull_autotune.argtypes = [vp, vp, i64, ctypes.c_int32, ctypes.POINTER(TuneEntry), i64, pi64,
                                        ctypes.POINTER(Config), vp]
        lib.vqhull_last_level_stats.restype = i64
        lib.vqhull_last_level_stats.argtypes = [pi64, i64]
        lib.vqhull_last_level_kinds.restype = i64
        lib.vqhull_last_level_kinds.argtypes = [ctypes.POINTER(ctypes.c_int32), i64]
        lib.vqhull_set_level_pairs.restype = ctypes.c_int
        lib.vqhull_set_level_pairs.argtypes = [ctypes.c_int]
        lib.vqhull_set_timing.restype = ctypes.c_int
        lib.vqhull_set_timing.argtypes = [ctypes.c_int]
        lib.vqhull_last_kernel_times.restype = i64
        lib.vqhull_last_kernel_times.argtypes = [ctypes.POINTER(KernelTime), i64]
        lib.vqhull_orient.restype = ctypes.c_int
        lib.vqhull_orient.argtypes = [vp, i64, vp, vp]
        lib.vqhull_stream_scale.restype = ctypes.c_int
        lib.vqhull_stream_scale.argtypes = [vp, vp, i64, ctypes.c_double, vp]
        lib.vqhull_release_workspace.restype = ctypes.c_int
        lib.vqhull_release_workspace.argtypes = []
        lib.vqhull_status_string.restype = ctypes.c_char_p
        lib.vqhull_status_string.argtypes = [ctypes.c_int]
        lib.vqhull_last_error.restype = ctypes.c_char_p
        lib.vqhull_last_error.argtypes = []
        ci = ctypes.c_int
        lib.vqhull_server_create.restype = ci
        lib.vqhull_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        lib.vqhull_server_submit.restype = ci
        lib.vqhull_server_submit.argtypes = [vp, vp, vp, i64, vp, vp, pi64]
        lib.vqhull_server_submit_batch.restype = ci
        lib.vqhull_server_submit_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, pi64]
        lib.vqhull_server_wait.restype = ci
        lib.vqhull_server_wait.argtypes = [vp, i64]
        lib.vqhull_server_wait_timeout.restype = ci
        lib.vqhull_server_wait_timeout.argtypes = [vp, i64, ctypes.c_double]
        lib.vqhull_server_poll.restype = i64
        lib.vqhull_server_poll.argtypes = [vp, pi64, i64]
        lib.vqhull_server_drain.restype = ci
        lib.vqhull_server_drain.argtypes = [vp]
        lib.vqhull_server_ticket_info.restype = ci
        lib.vqhull_server_ticket_info.argtypes = [vp, i64, ctypes.POINTER(TicketInfo)]
        lib.vqhull_server_stats.restype = ci
        lib.vqhull_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
        lib.vqhull_server_destroy.restype = ci
        lib.vqhull_server_destroy.argtypes = [vp]
        _lib = lib
        return lib


def _check(lib, status: int):
    if status != VQHULL_OK:
        msg = lib.vqhull_status_string(status).decode()
        if status == VQHULL_ERR_HIP:
            msg += ": " + lib.vqhull_last_error().decode()
        raise VqhullError(status, msg)


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_points(x, y):
    import torch

    if not (isinstance(x, torch.Tensor) and isinstance(y, torch.Tensor)):
        raise TypeError("x and y must be torch tensors")
    if x.dtype != torch.float64 or y.dtype != torch.float64:
        raise TypeError("x and y must be float64")
    if not (x.is_cuda and y.is_cuda) or x.device != y.device:
        raise ValueError("x and y must be on the same GPU")
    if x.dim() != 1 or x.shape != y.shape:
        raise ValueError("x and y must be 1-D of equal length")
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("x and y must be contiguous")


def hull_into(x, y, out_idx, out_count, stream=None) -> None:
    """vqhull_hull on preallocated device outputs.  The call returns after the
    result is written (it waits on the stream), and the library's own
    workspace may be allocated or grown on the first call of a device or when
    n exceeds every earlier call's."""
    lib = load_library()
    n = x.numel()
    st = lib.vqhull_hull(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), n,
                         ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_count.data_ptr()),
                         _stream_handle(stream))
    _check(lib, st)


def workspace_bytes(n_total: int, nreq: int = 1) -> int:
    """Bytes of device workspace a _ws call needs (vqhull_workspace_bytes)."""
    b = load_library().vqhull_workspace_bytes(int(n_total), int(nreq))
    if b == 0:
        raise ValueError("n_total and nreq must lie in [0, 2^31)")
    return int(b)


def workspace(n_total: int, nreq: int = 1, device=None):
    """A device workspace tensor (uint8, from torch's allocator) for a _ws call
    on n_total points in nreq requests.  torch's allocator returns blocks
    aligned to at least 512 bytes, which covers the 256 bytes the calls ask."""
    import torch

    ws = torch.empty(workspace_bytes(n_total, nreq), dtype=torch.uint8, device=device or "cuda")
    if ws.data_ptr() % 256:
        raise RuntimeError("torch returned a workspace that is not 256-byte aligned")
    return ws


def hull_ws_into(x, y, out_idx, out_count, ws, stream=None) -> None:
    """vqhull_hull_ws: vqhull_hull with every device buffer in the caller's
    workspace tensor ws (see ``workspace``); the library allocates no device
    memory.  Returns after the result is written."""
    lib = load_library()
    st = lib.vqhull_hull_ws(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
                            ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_count.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), _stream_handle(stream))
    _check(lib, st)


def hull_inplace(x, y, offsets=None, stream=None):
    """In-place mode (vqhull_hull_inplace / vqhull_hull_batched_inplace): x and y
    are overwritten (their contents afterwards are unspecified) and serve as
    one of the two point buffers; the workspace (24 B per point for the point
    buffers instead of 40) comes from torch's allocator.  Without offsets:
    the hull index list of the single request; with offsets (host sequence of
    nreq + 1 ints): (out_idx, counts) as hull_batched returns them."""
    import numpy as np
    import torch

    _check_points(x, y)
    lib = load_library()
    n = x.numel()
    with torch.cuda.device(x.device):
        if offsets is None:
            out = torch.empty(max(n, 1), dtype=torch.int64, device=x.device)
            cnt = torch.empty(1, dtype=torch.int64, device=x.device)
            ws = torch.empty(lib.vqhull_workspace_bytes_inplace(n, 1), dtype=torch.uint8, device=x.device)
            st = lib.vqhull_hull_inplace(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), n,
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
            _check(lib, st)
            h = int(cnt.item())
            if h < 0:
                raise VqhullError(-h, "non-finite coordinate in the input")
            return out[:h]
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        nreq = len(off) - 1
        if nreq < 0 or off[-1] != n:
            raise ValueError("offsets must have nreq+1 entries ending at len(x)")
        out = torch.empty(max(n, 1), dtype=torch.int64, device=x.device)
        cnt = torch.empty(max(nreq, 1), dtype=torch.int64, device=x.device)
        ws = torch.empty(lib.vqhull_workspace_bytes_inplace(n, nreq), dtype=torch.uint8, device=x.device)
        st = lib.vqhull_hull_batched_inplace(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nreq,
                                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
        _check(lib, st)
        return out, cnt[:nreq]


NOALLOC_MAX_POINTS = 1 << 20  # VQHULL_NOALLOC_MAX_POINTS


def hull_noalloc_into(x, y, out_idx, out_count, stream=None) -> None:
    """vqhull_hull_noalloc: vqhull_hull with every device table in the
    library's static per-GPU array (at most NOALLOC_MAX_POINTS points); the
    library allocates nothing.  Returns after the result is written."""
    lib = load_library()
    st = lib.vqhull_hull_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
                                 ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_count.data_ptr()),
                                 _stream_handle(stream))
    _check(lib, st)


def hull(x, y, stream=None):
    """Hull vertex indices (int64 tensor on the same GPU), clockwise from the
    lexicographically smallest point.  Every device buffer (output and
    workspace) comes from torch's allocator (vqhull_hull_ws).  Raises
    VqhullError on a non-finite input."""
    import torch

    _check_points(x, y)
    n = x.numel()
    out = torch.empty(max(n, 1), dtype=torch.int64, device=x.device)
    cnt = torch.empty(1, dtype=torch.int64, device=x.device)
    with torch.cuda.device(x.device):
        ws = workspace(n, 1, x.device)
        hull_ws_into(x, y, out, cnt, ws, stream)
        h = int(cnt.item())
    del ws
    if h < 0:
        raise VqhullError(-h, "non-finite coordinate in the input")
    return out[:h]


def _check_xy(xy):
    import torch

    if not isinstance(xy, torch.Tensor) or xy.dtype != torch.float64 or not xy.is_cuda:
        raise TypeError("xy must be a float64 GPU tensor")
    if xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_contiguous():
        raise ValueError("xy must be a contiguous (n, 2) tensor of interleaved (x, y) pairs")
    if xy.data_ptr() % 16:
        raise ValueError("xy must be 16-byte aligned")


def hull_xy_into(xy, out_idx, out_count, stream=None) -> None:
    """vqhull_hull_xy on preallocated device outputs (returns after the result
    is written; the library's workspace may be allocated or grown)."""
    lib = load_library()
    st = lib.vqhull_hull_xy(ctypes.c_void_p(xy.data_ptr()), xy.shape[0], ctypes.c_void_p(out_idx.data_ptr()),
                            ctypes.c_void_p(out_count.data_ptr()), _stream_handle(stream))
    _check(lib, st)


def hull_xy(xy, stream=None):
    """Hull of interleaved points xy[i] = (x_i, y_i) (an (n, 2) float64 GPU tensor):
    the same index list as hull(xy[:, 0], xy[:, 1])."""
    import torch

    _check_xy(xy)
    n = xy.shape[0]
    out = torch.empty(max(n, 1), dtype=torch.int64, device=xy.device)
    cnt = torch.empty(1, dtype=torch.int64, device=xy.device)
    with torch.cuda.device(xy.device):
        hull_xy_into(xy, out, cnt, stream)
        h = int(cnt.item())
    if h < 0:
        raise VqhullError(-h, "non-finite coordinate in the input")
    return out[:h]


def hull_batched_xy(xy, offsets, stream=None):
    """hull_batched for interleaved points (an (N, 2) float64 GPU tensor)."""
    import numpy as np
    import torch

    _check_xy(xy)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    nreq = len(off) - 1
    if nreq < 0 or off[-1] != xy.shape[0]:
        raise ValueError("offsets must have nreq+1 entries ending at len(xy)")
    lib = load_library()
    out = torch.empty(max(xy.shape[0], 1), dtype=torch.int64, device=xy.device)
    cnt = torch.empty(max(nreq, 1), dtype=torch.int64, device=xy.device)
    with torch.cuda.device(xy.device):
        st = lib.vqhull_hull_batched_xy(ctypes.c_void_p(xy.data_ptr()),
                                        off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nreq,
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                        _stream_handle(stream))
    _check(lib, st)
    return out, cnt[:nreq]


def hull_batched_ws(x, y, offsets, ws=None, stream=None):
    """hull_batched through vqhull_hull_batched_ws: every device buffer comes
    from torch's allocator (ws: a tensor from ``workspace``, or None for a
    fresh one)."""
    import numpy as np
    import torch

    _check_points(x, y)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    nreq = len(off) - 1
    if nreq < 0 or off[-1] != x.numel():
        raise ValueError("offsets must have nreq+1 entries ending at len(x)")
    lib = load_library()
    out = torch.empty(max(x.numel(), 1), dtype=torch.int64, device=x.device)
    cnt = torch.empty(max(nreq, 1), dtype=torch.int64, device=x.device)
    with torch.cuda.device(x.device):
        if ws is None:
            ws = workspace(x.numel(), nreq, x.device)
        st = lib.vqhull_hull_batched_ws(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                        off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nreq,
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                        _stream_handle(stream))
    _check(lib, st)
    return out, cnt[:nreq]


INCOMPLETE = -VQHULL_ERR_INCOMPLETE  # a count of hull_batched_async: the level budget ended before the recursion


def hull_batched_async(x, y, offsets, levels: int = 64, ws=None, stream=None):
    """vqhull_hull_batched_async: the batched hulls enqueued on the stream with
    no host wait, in a budget of ``levels`` recursion levels.  Returns
    (out_idx, counts, ws) device tensors, valid once the stream has finished
    the call's work; a count of INCOMPLETE for every request means the budget
    was too small.  ws (a tensor from ``workspace``, or None for a fresh one)
    must stay alive until then; it is returned for that purpose."""
    import numpy as np
    import torch

    _check_points(x, y)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    nreq = len(off) - 1
    if nreq < 0 or off[-1] != x.numel():
        raise ValueError("offsets must have nreq+1 entries ending at len(x)")
    lib = load_library()
    out = torch.empty(max(x.numel(), 1), dtype=torch.int64, device=x.device)
    cnt = torch.empty(max(nreq, 1), dtype=torch.int64, device=x.device)
    with torch.cuda.device(x.device):
        if ws is None:
            ws = workspace(x.numel(), nreq, x.device)
        st = lib.vqhull_hull_batched_async(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                           off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nreq,
                                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                           int(levels), ctypes.c_void_p(ws.data_ptr()),
                                           ws.numel() * ws.element_size(), _stream_handle(stream))
    _check(lib, st)
    return out, cnt[:nreq], ws


def hull_batched(x, y, offsets, stream=None, check=True):
    """Hulls of the requests x[offsets[i]:offsets[i+1]] (offsets: host sequence of
    nreq+1 ints).  Returns (out_idx, counts) device tensors: request i's list is
    out_idx[offsets[i] : offsets[i] + counts[i]] (indices local to the request)."""
    import numpy as np
    import torch

    _check_points(x, y)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    nreq = len(off) - 1
    if nreq < 0 or (nreq >= 0 and len(off) and off[-1] != x.numel()):
        raise ValueError("offsets must have nreq+1 entries ending at len(x)")
    lib = load_library()
    out = torch.empty(max(x.numel(), 1), dtype=torch.int64, device=x.device)
    cnt = torch.empty(max(nreq, 1), dtype=torch.int64, device=x.device)
    with torch.cuda.device(x.device):
        st = lib.vqhull_hull_batched(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nreq,
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                     _stream_handle(stream))
    _check(lib, st)
    return out, cnt[:nreq]


def get_config() -> dict:
    lib = load_library()
    c = Config()
    _check(lib, lib.vqhull_get_config(ctypes.byref(c)))
    return c.as_dict()


def set_config(**kw) -> dict:
    """Update tuning knobs (sweep_block, sweep_ppt, lds_limit, reverse_tiles, sweep_persistent, level_block,
    prefilter)."""
    lib = load_library()
    c = Config()
    _check(lib, lib.vqhull_get_config(ctypes.byref(c)))
    for k, v in kw.items():
        if k not in c.as_dict():
            raise KeyError(k)
        setattr(c, k, int(v))
    _check(lib, lib.vqhull_set_config(ctypes.byref(c)))
    return get_config()


def level_stats() -> list[dict]:
    """Per-level statistics of the last call on the current device."""
    lib = load_library()
    n = lib.vqhull_last_level_stats(None, 0)
    buf = (ctypes.c_int64 * (4 * max(n, 1)))()
    n = lib.vqhull_last_level_stats(buf, n)
    kinds = (ctypes.c_int32 * max(n, 1))()
    nk = lib.vqhull_last_level_kinds(kinds, n)
    return [dict(segments=buf[4 * i], swept=buf[4 * i + 1], jobs=buf[4 * i + 2], job_points=buf[4 * i + 3],
                 sweep=SWEEP_KINDS[kinds[i]] if i < nk else "level")
            for i in range(n)]


def set_level_pairs(mode: int) -> None:
    """Level pairs below the top (0 never, 1 where levels keep most of their
    points, the default; 2 from the first level sweep on)."""
    _check(load_library(), load_library().vqhull_set_level_pairs(int(mode)))


def set_timing(enable, sweeps_only: bool = False, fused_only: bool = False) -> None:
    """Record HIP events around every kernel launch of later calls (with
    sweeps_only, around the partition sweeps alone; with fused_only, around
    the fused top-level pass alone)."""
    lib = load_library()
    mode = (3 if fused_only else 2 if sweeps_only else 1) if enable else 0
    _check(lib, lib.vqhull_set_timing(mode))


def kernel_times() -> list[dict]:
    """Per-launch timing records of the last call (needs set_timing(True))."""
    lib = load_library()
    n = lib.vqhull_last_kernel_times(None, 0)
    buf = (KernelTime * max(n, 1))()
    n = lib.vqhull_last_kernel_times(buf, n)
    return [dict(kind=KERNEL_KINDS[buf[i].kind], level=buf[i].level, ms=buf[i].ms, points_in=buf[i].points_in,
                 points_out=buf[i].points_out) for i in range(n)]


def orient_batch(abc, stream=None):
    """The kernels' orientation predicate on the triples abc (an (n, 6) float64
    GPU tensor: a.x, a.y, b.x, b.y, c.x, c.y): returns an (n, 2) tensor, the
    value as the finisher computes it and as the sweeps compute it."""
    import torch

    if not isinstance(abc, torch.Tensor) or abc.dtype != torch.float64 or not abc.is_cuda:
        raise TypeError("abc must be a float64 GPU tensor")
    if abc.dim() != 2 or abc.shape[1] != 6 or not abc.is_contiguous():
        raise ValueError("abc must be a contiguous (n, 6) tensor")
    lib = load_library()
    out = torch.empty((abc.shape[0], 2), dtype=torch.float64, device=abc.device)
    with torch.cuda.device(abc.device):
        _check(lib, lib.vqhull_orient(ctypes.c_void_p(abc.data_ptr()), abc.shape[0], ctypes.c_void_p(out.data_ptr()),
                                      _stream_handle(stream)))
    return out


def stream_scale(src, dst, s: float = 3.0, stream=None) -> None:
    """dst = s * src on the GPU (float64 tensors of equal length): the HBM probe."""
    import torch

    if src.dtype != torch.float64 or dst.dtype != torch.float64 or src.numel() != dst.numel():
        raise ValueError("src and dst must be float64 tensors of equal length")
    lib = load_library()
    _check(lib, lib.vqhull_stream_scale(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                        src.numel(), float(s), _stream_handle(stream)))


def release_workspace() -> None:
    lib = load_library()
    _check(lib, lib.vqhull_release_workspace())


def autotune_table(x, y, repeats: int = 3, stream=None):
    """Run vqhull_autotune on (x, y): returns (best config dict, list of
    {config, ms, same_result}).  The library's configuration is unchanged."""
    _check_points(x, y)
    lib = load_library()
    cap = 64
    entries = (TuneEntry * cap)()
    count = ctypes.c_int64()
    best = Config()
    _check(lib, lib.vqhull_autotune(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
                                    repeats, entries, cap, ctypes.byref(count), ctypes.byref(best),
                                    _stream_handle(stream)))
    table = [{"config": entries[i].cfg.as_dict(), "ms": entries[i].ms, "same_result": bool(entries[i].same_result)}
             for i in range(min(count.value, cap))]
    return best.as_dict(), table


class Server:
    """Continuous-batching hull server (vqhull_server_*): requests are queued
    as they are submitted and computed in batches by ``lanes`` concurrent batch
    lanes; see include/vqhull.h.  The caller keeps each request's tensors alive
    until the request is done (``wait``, ``drain`` or ``poll``)."""

    def __init__(self, lanes: int = 2, lane_points: int = 1 << 24, lane_requests: int = 4096, graph_levels: int = 20):
        self._lib = load_library()
        cfg = ServerConfig(lanes, graph_levels, lane_points, lane_requests)
        h = ctypes.c_void_p()
        _check(self._lib, self._lib.vqhull_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.lane_points = lane_points

    def submit(self, x, y, out_idx, out_count) -> int:
        """Queue the hull of (x, y) into out_idx (int64, >= len(x) entries) and
        out_count (int64 scalar tensor); returns the request's ticket."""
        import torch

        _check_points(x, y)
        if out_idx.dtype != torch.int64 or out_count.dtype != torch.int64 or not out_idx.is_cuda:
            raise TypeError("out_idx and out_count must be int64 GPU tensors")
        if out_idx.numel() < x.numel():
            raise ValueError("out_idx needs room for len(x) entries")
        t = ctypes.c_int64()
        _check(self._lib, self._lib.vqhull_server_submit(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
            ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(out_count.data_ptr()), ctypes.byref(t)))
        return t.value

    def submit_pointers(self, x_ptrs, y_ptrs, sizes, out_ptrs, count_ptrs) -> int:
        """Queue len(sizes) requests given as numpy int64 arrays of device
        addresses (x, y, out_idx, out_count per request) and sizes, with one
        library call; returns the first ticket (the others follow in order).
        The caller guarantees the addresses (float64 / int64 device buffers)."""
        import numpy as np

        arrs = [np.ascontiguousarray(a, dtype=np.int64) for a in (x_ptrs, y_ptrs, sizes, out_ptrs, count_ptrs)]
        k = len(arrs[2])
        if any(len(a) != k for a in arrs):
            raise ValueError("all arrays need one entry per request")
        t = ctypes.c_int64()
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
        _check(self._lib, self._lib.vqhull_server_submit_batch(self._h, k, *[ptr(a) for a in arrs],
                                                                ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int) -> int:
        """Block until the request is done; returns its status (0 = ok)."""
        return self._lib.vqhull_server_wait(self._h, ticket)

    def wait_timeout(self, ticket: int, seconds: float) -> int:
        """Wait at most ``seconds``; the request's status once done, else
        VQHULL_ERR_TIMEOUT (the request still completes later)."""
        return self._lib.vqhull_server_wait_timeout(self._h, ticket, float(seconds))

    def poll(self, cap: int = 4096) -> list:
        buf = (ctypes.c_int64 * cap)()
        k = self._lib.vqhull_server_poll(self._h, buf, cap)
        if k < 0:
            _check(self._lib, -k)
        return list(buf[:k])

    def drain(self) -> None:
        _check(self._lib, self._lib.vqhull_server_drain(self._h))

    def info(self, ticket: int) -> dict:
        ti = TicketInfo()
        _check(self._lib, self._lib.vqhull_server_ticket_info(self._h, ticket, ctypes.byref(ti)))
        return {k: getattr(ti, k) for k, _ in TicketInfo._fields_ if k != "reserved"}

    def stats(self) -> dict:
        c = ServerCounters()
        _check(self._lib, self._lib.vqhull_server_stats(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in ServerCounters._fields_}

    def close(self) -> None:
        if self._h:
            _check(self._lib, self._lib.vqhull_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
