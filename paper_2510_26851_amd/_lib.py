"""ctypes view of libfof.so (include/fof.h).  Argument marshalling only.

The library must have been built (``python paper_2510_26851_amd/build.py`` or
``__graft_entry__.build()``); importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfof.so")

FOF_OK = 0
FOF_EINVAL = -1
FOF_ENOMEM = -2
FOF_EOVERFLOW = -3
FOF_EDEVICE = -4
FOF_ENOTSUP = -5
FOF_STATUS_RANGE = 1
FOF_PROB_DISTANCE = 0
FOF_PROB_QUADRATIC = 1
FOF_TUNE_NO_TILES = 1
FOF_STATUS_DENSE_CAP = 2
FOF_STATUS_EDGE_CAP = 4
FOF_STATUS_OVERFLOW = 8
FOF_STATUS_SLAB_CAP = 16
FOF_FROZEN = 0
FOF_SCORE = 1
FOF_BASELINE_NONE = 0
FOF_BASELINE_MEAN = 1
FOF_BASELINE_LOO = 2


def sample_scratch_bytes(n: int, K: int, edge_cap: int) -> int:
    """FOF_SAMPLE_SCRATCH_BYTES of include/fof.h."""
    vcap = min(2 * edge_cap, n)
    return (8192 + 8 * (n + 1) + 4 * (n // 2048 + 2) + 8 * edge_cap + 8 * K + 8 * vcap +
            12 * K * vcap + 4 * (K * vcap // 2048 + 3) + 24 * vcap + 8 + 8 * edge_cap)

# Every symbol include/fof.h declares.
EXPORTS = ("fof_workspace_bytes", "fof_build_grid", "fof_link", "fof_groups", "fof_backward",
           "fof_group_dispersion", "fof_backward_dispersion", "fof_subhalo_scratch_bytes",
           "fof_subhalo", "fof_status", "fof_strerror", "fof_last_device_error", "fof_init",
           "fof_find_groups_static", "fof_stream_counts", "fof_stream_workspace_bytes",
           "fof_link_stream")
FOF_STATIC_SCRATCH_BYTES = 160 << 20


class fof_box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("b", ctypes.c_double)]


class fof_tune(ctypes.Structure):
    _fields_ = [("cell_side", ctypes.c_double), ("dense_threshold", ctypes.c_int32),
                ("block", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("link_edges", ctypes.c_int32), ("cell_factor", ctypes.c_double),
                ("dense_cells", ctypes.c_int64)]


class fof_sample(ctypes.Structure):
    _fields_ = [("b", ctypes.c_double), ("tau", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("K", ctypes.c_int32), ("edge_cap", ctypes.c_int32), ("ei", ctypes.c_void_p),
                ("ej", ctypes.c_void_p), ("d2", ctypes.c_void_p), ("n_edges", ctypes.c_void_p),
                ("scratch", ctypes.c_void_p), ("scratch_bytes", ctypes.c_size_t),
                ("form", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("s_first", ctypes.c_int32)]


class fof_grid(ctypes.Structure):
    _fields_ = [("nbox", ctypes.c_int32), ("block", ctypes.c_int32), ("n", ctypes.c_int64),
                ("ncell", ctypes.c_int64), ("dense_cap", ctypes.c_int64),
                ("ntiles", ctypes.c_int64), ("n_plain", ctypes.c_int64),
                ("dense_threshold", ctypes.c_int32), ("table_words", ctypes.c_int32),
                ("link_edges", ctypes.c_int64), ("ws_bytes", ctypes.c_size_t), ("desc_bytes", ctypes.c_size_t),
                ("off_desc", ctypes.c_size_t)] + [
                   (f, ctypes.c_size_t) for f in (
                       "off_status", "off_counters", "off_cell_count", "off_cell_start",
                       "off_rank", "off_sorted", "off_parent", "off_flags", "off_keep",
                       "off_scan", "off_dense", "off_units", "off_table", "off_aux")]


class FoFError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        msg = f"{fn} failed: {strerror(code)} ({code})"
        if code == FOF_EDEVICE:
            name = ctypes.c_char_p()
            hip = load().fof_last_device_error(ctypes.byref(name))
            msg += f": {name.value.decode() if name.value else '?'} ({hip})"
        super().__init__(msg)


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime, which its libraries request as "libamdhip64.so".
    # Loaded first, that copy also satisfies libfof.so's "libamdhip64.so.7", so the process
    # holds one runtime.  The other order maps two, and the second sees no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.fof_workspace_bytes.argtypes = [i32, P, P, P, P, P, sz]
    L.fof_build_grid.argtypes = [P, P, P, sz, P]
    L.fof_link.argtypes = [P, P, sz, P, P, P]
    L.fof_groups.argtypes = [P, P, sz, P, i32, P, i32, P, P, P, P, P, P, P]
    L.fof_backward.argtypes = [P, P, sz, i32, P, i32, P, P, P, P, P, P, P, P, P, i32, P, P, P]
    L.fof_group_dispersion.argtypes = [P, P, sz, i32, P, P, P, P, P]
    L.fof_backward_dispersion.argtypes = [P, P, sz, P, P, i32, P, P, P, P, P, P]
    L.fof_subhalo_scratch_bytes.argtypes = [i64, i32]
    L.fof_subhalo_scratch_bytes.restype = sz
    L.fof_subhalo.argtypes = [P, P, sz, P, P, P, i32, P, P, P, ctypes.c_double, P, sz, P, P]
    L.fof_status.argtypes = [P, P, sz, ctypes.POINTER(ctypes.c_void_p)]
    L.fof_strerror.argtypes = [ctypes.c_int]
    L.fof_strerror.restype = ctypes.c_char_p
    L.fof_last_device_error.argtypes = [ctypes.POINTER(ctypes.c_char_p)]
    L.fof_init.argtypes = []
    L.fof_find_groups_static.argtypes = [P, i64, P, P, i32, P, i32, P, P, P, P, P, P, P, P, P]
    L.fof_stream_counts.argtypes = [P, i64, P, i32, P, P]
    L.fof_stream_workspace_bytes.argtypes = [P, i64, i32, P, P, ctypes.POINTER(sz)]
    L.fof_link_stream.argtypes = [P, i64, P, i32, P, P, P, sz, P, P, P]
    for f in EXPORTS:
        if f != "fof_strerror":
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def init():
    """Creates the current device's helper stream (fof_init), once."""
    check("fof_init", load().fof_init())


def strerror(code: int) -> str:
    return load().fof_strerror(int(code)).decode()


def check(fn: str, code: int):
    if code != FOF_OK:
        raise FoFError(fn, code)
