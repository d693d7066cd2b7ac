"""ctypes loader and prototypes for libunimgs.so (the C ABI in include/unimgs.h).

The library is built in-tree by ``python -m paper_2601_19233_amd.build``.
Loading fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libunimgs.so")

UMGS_OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "CAPACITY", -3: "HIP", -4: "STATE", -5: "UNSUPPORTED"}

MODE_UNIMGS, MODE_DIRECT, MODE_ONE_ENTITY, MODE_LITERAL_T = 0, 1, 2, 3
SCHEDULE_TILE_GRID, SCHEDULE_PERSISTENT = 0, 1
STATE_KEYS, STATE_SORTED_KEYS, STATE_SORTED_VALS, STATE_RANGES, STATE_TRI_FIXED, STATE_GRAD2D = 0, 1, 2, 3, 4, 5


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("frag_batch", C.c_int32),
                ("sh_degree", C.c_int32), ("k_bind", C.c_int32), ("mode", C.c_int32),
                ("schedule", C.c_int32), ("bg", C.c_float * 3)]


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64

PROTOTYPES = {
    "umgs_default_options": (None, [C.POINTER(Options)]),
    "umgs_create": (C.c_int, [C.POINTER(P), C.POINTER(Options), P]),
    "umgs_destroy": (None, [P]),
    "umgs_last_error": (C.c_char_p, [P]),
    "umgs_set_options": (C.c_int, [P, C.POINTER(Options)]),
    "umgs_set_proxy": (C.c_int, [P, I32, P, I32, P]),
    "umgs_bind_transfer": (C.c_int, [P, P, I32, P, P, P, P, P, P, P, P, P, P]),
    "umgs_bind_transfer_noalloc": (C.c_int, [P, P, I32, P, P, P, P, P, P, P, P, P, P]),
    "umgs_bind_raycast": (C.c_int, [P, I32, P, P, P, I32, I32, C.POINTER(C.c_float), P, P, P]),
    "umgs_project": (C.c_int, [P, I32, C.POINTER(Camera), I32, P, P, P, P, P, P, I32, P, P, P]),
    "umgs_set_texture": (C.c_int, [P, I32, I32, P, I32, P]),
    "umgs_bin": (C.c_int, [P]),
    "umgs_sort": (C.c_int, [P]),
    "umgs_blend": (C.c_int, [P, P, P, P, P]),
    "umgs_render_batched": (C.c_int, [P, I32, C.POINTER(Camera), C.POINTER(I64), I32, P, P, P, P, P,
                                      P, I32, P, P, P, P, P, P, P]),
    "umgs_query": (C.c_int, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I32)]),
    "umgs_reserve": (C.c_int, [P, I64]),
    "umgs_query_bins": (C.c_int, [P, C.POINTER(I64), C.POINTER(I64)]),
    "umgs_blend_pairs": (C.c_int, [P, P, C.POINTER(I64)]),
    "umgs_graph_begin": (C.c_int, [P]),
    "umgs_graph_end": (C.c_int, [P]),
    "umgs_graph_launch": (C.c_int, [P]),
    "umgs_update_views": (C.c_int, [P, I32, C.POINTER(Camera), C.POINTER(Camera)]),
    "umgs_view_dups": (C.c_int, [P, C.POINTER(I64)]),
    "umgs_copy_state": (C.c_int, [P, I32, P, I64]),
    "umgs_backward": (C.c_int, [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, I32]),
    "umgs_backward_transfer": (C.c_int, [P, P, I32, P, P, P, P, P, I32]),
    "umgs_backward_triangles": (C.c_int, [P, P, P, P, P, P, P, I32]),
    "umgs_set_profiling": (C.c_int, [P, I32]),
    "umgs_profile_read": (C.c_int, [P, I32, C.POINTER(I64), C.POINTER(C.c_double)]),
}

KERNEL_NAMES = ["vertex_frames", "transfer", "project_gaussians", "setup_triangles", "count_scan",
                "emit_keys", "sort_upsweep", "sort_scan", "sort_downsweep", "tile_ranges", "blend",
                "blend_backward", "project_backward", "depth_sort", "tile_count", "tile_scatter",
                "st_mask", "blend_backward_tri", "transfer_backward"]

_lib = None


class UmgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"umgs error {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load() -> C.CDLL:
    """Load libunimgs.so and attach prototypes (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2601_19233_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
