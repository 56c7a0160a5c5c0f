"""ctypes loader for libpft.so (the HIP library built by ``paper_2104_08309_amd.build``).

Loading fails loudly when the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PFT_LIBRARY", os.path.join(HERE, "libpft.so"))

PFT_OK, PFT_EINVAL, PFT_EUNSUPPORTED, PFT_EHIP, PFT_ENOMEM = 0, -1, -2, -3, -4
PFT_FP64, PFT_FP32C = 0, 1
PFT_F32, PFT_F64 = 0, 1

# every symbol declared in include/pft.h
EXPORTS = [
    "pft_forward_2d", "pft_forward_3d", "pft_backward_3d", "pft_batch_forward", "pft_batch_backward",
    "pft_forward_3d_poly", "pft_orientation_average", "pft_forward_3d_regions", "pft_backward_3d_regions",
    "pft_intensity_loss_3d", "pft_strip_order", "pft_forward_3d_ordered", "pft_batch_forward_ordered",
    "pft_q_order", "pft_backward_3d_ordered", "pft_forward_3d_noalloc", "pft_check_mesh", "pft_tuning_info",
    "pft_fp32c_q_limit",
    "pft_validate_mesh", "pft_last_error", "pft_release_workspace", "pft_profile_enable",
    "pft_profile_reset", "pft_profile_read", "pft_version",
]


class PftMeshBatch(ctypes.Structure):
    """Mirror of ``pft_mesh_batch``."""

    _fields_ = [
        ("n_meshes", ctypes.c_int64),
        ("vert_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("tri_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("q_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("verts", ctypes.c_void_p),
        ("vdtype", ctypes.c_int),
        ("tris", ctypes.c_void_p),
        ("q", ctypes.c_void_p),
        ("qdtype", ctypes.c_int),
    ]


class PftMeshCheck(ctypes.Structure):
    """Mirror of ``pft_mesh_check``."""

    _fields_ = [(name, ctypes.c_int64) for name in
                ("bad_index", "repeated_vertex", "open_edges", "nonmanifold_edges", "misoriented_edges")]


class PftError(RuntimeError):
    """A libpft entry point returned a non-OK status."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"libpft status {status}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libpft.so once and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libpft.so not found at {LIB_PATH}; build it with `python -m paper_2104_08309_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, cint = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "pft_forward_2d": [vp, i64, P(i64), i64, vp, i64, vp, vp],
        "pft_forward_3d": [vp, cint, i64, vp, i64, vp, cint, i64, cint, vp, vp, vp],
        "pft_forward_3d_noalloc": [vp, cint, i64, vp, i64, vp, cint, i64, cint, vp, vp, vp],
        "pft_backward_3d": [vp, cint, i64, vp, i64, vp, cint, i64, cint, vp, vp, vp],
        "pft_batch_forward": [P(PftMeshBatch), cint, vp, vp, vp],
        "pft_batch_forward_ordered": [P(PftMeshBatch), vp, vp, cint, vp, vp, vp],
        "pft_batch_backward": [P(PftMeshBatch), cint, vp, vp, vp],
        "pft_orientation_average": [vp, cint, i64, vp, i64, vp, i64, vp, vp, i64, cint, vp, vp, vp, vp],
        "pft_forward_3d_poly": [vp, cint, i64, P(i64), vp, i64, vp, cint, i64, cint, vp, vp, vp],
        "pft_strip_order": [vp, i64, i64, vp, vp],
        "pft_forward_3d_ordered": [vp, cint, i64, vp, i64, vp, vp, vp, cint, i64, cint, vp, vp, vp, vp],
        "pft_q_order": [vp, cint, i64, vp, vp],
        "pft_backward_3d_ordered": [vp, cint, i64, vp, i64, vp, cint, i64, cint, vp, vp, vp, vp],
        "pft_intensity_loss_3d": [vp, cint, i64, vp, i64, vp, cint, i64, cint, vp, vp, vp, vp, vp, vp, vp, vp],
        "pft_forward_3d_regions": [vp, cint, i64, vp, i64, P(i64), i64, vp, vp, cint, i64, cint, vp, vp, vp, vp, vp,
                                   vp],
        "pft_backward_3d_regions": [vp, cint, i64, vp, i64, P(i64), i64, vp, vp, cint, i64, cint, vp, vp, vp, vp,
                                    vp],
        "pft_validate_mesh": [vp, i64, i64, P(i64), P(i64), vp],
        "pft_check_mesh": [vp, i64, i64, P(PftMeshCheck)],
        "pft_fp32c_q_limit": [vp, cint, i64, vp, i64, P(ctypes.c_double)],
        "pft_last_error": [],
        "pft_release_workspace": [],
        "pft_profile_enable": [cint],
        "pft_profile_reset": [],
        "pft_profile_read": [ctypes.c_char_p, P(i64), P(ctypes.c_double)],
        "pft_version": [],
        "pft_tuning_info": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("pft_last_error", "pft_version", "pft_tuning_info") else cint
    _lib = lib
    return lib


def check(status: int) -> None:
    """Raise PftError for a non-OK status, with the library's message."""
    if status != PFT_OK:
        msg = load().pft_last_error().decode(errors="replace")
        raise PftError(status, msg)
