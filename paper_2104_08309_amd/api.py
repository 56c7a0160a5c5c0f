"""PyTorch-facing wrappers over the libpft C ABI.

Argument marshalling only: tensors are checked (device, dtype, shape,
contiguity), outputs are allocated with torch, and raw device pointers plus
the current HIP stream are handed to the library. All arithmetic runs in the
library's HIP kernels; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import weakref
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import PFT_F32, PFT_F64, PFT_FP32C, PFT_FP64, PftMeshBatch, check

__all__ = [
    "forward_2d", "forward_3d", "forward_3d_noalloc", "forward_3d_poly", "backward_3d", "batch_forward", "batch_backward",
    "orientation_average", "forward_3d_regions", "backward_3d_regions", "intensity_loss_3d", "strip_order",
    "batch_strip_order", "q_order",
    "validate_mesh", "check_mesh", "fp32c_q_limit",
    "profile_enable", "profile_reset", "profile_read", "release_workspace", "version", "mode_id", "tuning_info",
]

_MODES = {"fp64": PFT_FP64, "fp32c": PFT_FP32C}


def mode_id(mode: str) -> int:
    try:
        return _MODES[mode.lower()]
    except (KeyError, AttributeError):
        raise ValueError(f"mode must be one of {sorted(_MODES)}, got {mode!r}") from None


def _real_dtype_id(t: torch.Tensor, name: str) -> int:
    if t.dtype == torch.float32:
        return PFT_F32
    if t.dtype == torch.float64:
        return PFT_F64
    raise TypeError(f"{name} must be float32 or float64, got {t.dtype}")


def _on_gpu(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU (HIP) tensor; libpft has no CPU path")
    return t.contiguous()


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None or t.numel() == 0 else t.data_ptr()


def _mesh(verts: torch.Tensor, tris: torch.Tensor):
    verts = _on_gpu(verts, "verts")
    tris = _on_gpu(tris, "tris")
    if verts.dim() != 2 or verts.shape[1] != 3:
        raise ValueError(f"verts must have shape [nv, 3], got {tuple(verts.shape)}")
    if tris.dim() != 2 or tris.shape[1] != 3:
        raise ValueError(f"tris must have shape [nf, 3], got {tuple(tris.shape)}")
    if tris.dtype != torch.int32:
        if tris.dtype not in (torch.int64, torch.int16, torch.uint8):
            raise TypeError(f"tris must be an integer tensor, got {tris.dtype}")
        tris = tris.to(torch.int32)
    if tris.device != verts.device:
        raise ValueError("verts and tris must be on the same device")
    return verts, tris


def _qlist(q: torch.Tensor, device, dim: int = 3) -> torch.Tensor:
    q = _on_gpu(q, "q")
    if q.dim() != 2 or q.shape[1] != dim:
        raise ValueError(f"q must have shape [nq, {dim}], got {tuple(q.shape)}")
    if q.device != device:
        raise ValueError("q must be on the same device as the mesh")
    return q


def forward_2d(verts: torch.Tensor, q: torch.Tensor, contour_offsets: Optional[Sequence[int]] = None) -> torch.Tensor:
    """F(Q) of a polygon (complex128 [nq]); ``contour_offsets`` splits verts into closed contours."""
    verts = _on_gpu(verts, "verts")
    if verts.dim() != 2 or verts.shape[1] != 2 or verts.dtype != torch.float64:
        raise ValueError("verts must be float64 with shape [nv, 2]")
    q = _qlist(q, verts.device, dim=2)
    if q.dtype != torch.float64:
        raise ValueError("q must be float64 for the 2D transform")
    out = torch.empty(q.shape[0], dtype=torch.complex128, device=verts.device)
    if contour_offsets is None:
        off_p, nc = None, 0
    else:
        off = np.ascontiguousarray(np.asarray(contour_offsets, dtype=np.int64))
        nc = off.size - 1
        off_p = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_forward_2d(_ptr(verts), verts.shape[0], off_p, nc, _ptr(q), q.shape[0], _ptr(out),
                                         _stream(verts.device)))
    return out


def strip_order(tris, nv: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Edge-sharing face order of a triangle mesh (pft_strip_order, host code): (order int32 [nf],
    meta uint8 [nf]) for forward_3d's ``order``. ``tris`` may be a tensor (copied to the host)."""
    t = tris.detach().cpu().numpy() if isinstance(tris, torch.Tensor) else np.asarray(tris)
    t = np.ascontiguousarray(t, dtype=np.int32).reshape(-1, 3)
    if nv is None:
        nv = int(t.max()) + 1 if t.size else 0
    order = np.empty(t.shape[0], dtype=np.int32)
    meta = np.empty(t.shape[0], dtype=np.uint8)
    check(_lib.load().pft_strip_order(t.ctypes.data, t.shape[0], nv, order.ctypes.data, meta.ctypes.data))
    return order, meta


# Edge-sharing orders of triangle tensors seen by forward_3d (order="auto"), keyed by the tensor
# object (its id, confirmed through a weak reference) and checked against its storage, shape and
# in-place version counter on every use.
_ORDER_CACHE: dict = {}
_AUTO_ORDER_MIN_FACES = 256


def _auto_order(tris_key: torch.Tensor, tris: torch.Tensor, nv: int):
    stamp = (tris_key.data_ptr(), tuple(tris_key.shape), tris_key._version, nv)
    hit = _ORDER_CACHE.get(id(tris_key))
    if hit is not None and hit[0]() is tris_key and hit[1] == stamp:
        return hit[2]
    order, meta = strip_order(tris, nv)
    dev_order = (torch.from_numpy(order).to(tris.device), torch.from_numpy(meta).to(tris.device))
    if len(_ORDER_CACHE) >= 64:  # drop the entries whose tensors are gone
        for k in [k for k, e in _ORDER_CACHE.items() if e[0]() is None]:
            del _ORDER_CACHE[k]
    _ORDER_CACHE[id(tris_key)] = (weakref.ref(tris_key), stamp, dev_order)
    return dev_order


def _order_arg(order, tris_key, tris: torch.Tensor, nv: int, m: int):
    """(order, meta) device tensors or (None, None) for an ``order`` argument ("auto", None or a pair)."""
    if isinstance(order, str):
        if order != "auto":
            raise ValueError(f"order must be 'auto', None or (order, meta), got {order!r}")
        use = m == PFT_FP32C and tris.shape[0] >= _AUTO_ORDER_MIN_FACES and isinstance(tris_key, torch.Tensor)
        return _auto_order(tris_key, tris, nv) if use else (None, None)
    if order is None:
        return None, None
    fo, fm = (_on_gpu(x, name) for x, name in zip(order, ("order", "meta")))
    if fo.dtype != torch.int32 or fm.dtype != torch.uint8 or fo.numel() != tris.shape[0] \
            or fm.numel() != tris.shape[0] or fo.device != tris.device or fm.device != tris.device:
        raise ValueError("order must be (int32 [nf], uint8 [nf]) tensors on the mesh's device")
    return fo, fm


def q_order(q: torch.Tensor) -> torch.Tensor:
    """The kernels' visiting order of a Q list (pft_q_order): uint32 [nq] on the device, computed there."""
    q = _on_gpu(q, "q")
    if q.dim() != 2 or q.shape[1] != 3:
        raise ValueError(f"q must have shape [nq, 3], got {tuple(q.shape)}")
    out = torch.empty(q.shape[0], dtype=torch.uint32, device=q.device)
    with torch.cuda.device(q.device):
        check(_lib.load().pft_q_order(_ptr(q), _real_dtype_id(q, "q"), q.shape[0], _ptr(out), _stream(q.device)))
    return out


# Visiting orders of Q tensors seen by forward_3d / backward_3d (q_order="auto"), keyed and checked
# like the face orders; below the sorting size the kernels keep the list order and nothing is cached.
_Q_ORDER_CACHE: dict = {}
_Q_ORDER_MIN = 8192


def _q_order_arg(q_order, q_key, q: torch.Tensor):
    if isinstance(q_order, str):
        if q_order != "auto":
            raise ValueError(f"q_order must be 'auto', None or a uint32 tensor, got {q_order!r}")
        if not isinstance(q_key, torch.Tensor) or q.shape[0] < _Q_ORDER_MIN:
            return None
        stamp = (q_key.data_ptr(), tuple(q_key.shape), q_key._version, q_key.dtype)
        hit = _Q_ORDER_CACHE.get(id(q_key))
        if hit is not None and hit[0]() is q_key and hit[1] == stamp:
            return hit[2]
        perm = q_order_fn(q)
        if len(_Q_ORDER_CACHE) >= 64:
            for k in [k for k, e in _Q_ORDER_CACHE.items() if e[0]() is None]:
                del _Q_ORDER_CACHE[k]
        _Q_ORDER_CACHE[id(q_key)] = (weakref.ref(q_key), stamp, perm)
        return perm
    if q_order is None:
        return None
    qo = _on_gpu(q_order, "q_order")
    if qo.dtype != torch.uint32 or qo.numel() != q.shape[0] or qo.device != q.device:
        raise ValueError("q_order must be a uint32 [nq] tensor on the device of q")
    return qo


q_order_fn = q_order


def forward_3d(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, mode: str = "fp32c",
               intensity: bool = False, order="auto", q_order="auto"):
    """F(Q) of the closed mesh; complex128 for mode 'fp64', complex64 for 'fp32c'.

    Returns F, or (F, |F|^2) when ``intensity`` is True. ``order``: "auto" (FP32C meshes of 256 faces
    or more are evaluated in an edge-sharing face order, computed on the host at the first call for
    a triangle tensor and reused while it is unchanged), None (the list order), or a pair of device
    tensors (order int32, meta uint8) from ``strip_order``. ``q_order``: "auto" (the visiting order of
    Q, computed on the device once per Q tensor and reused while it is unchanged), None (sorted in
    the call), or a uint32 tensor from ``q_order``. "Unchanged" is judged by the tensor's storage,
    shape and version counter, which torch advances on every in-place write through the tensor or
    its views; memory rewritten behind torch's back (another library writing the same device buffer)
    is not seen, and such callers pass None. A stale order gives wrong values, never a fault.
    """
    tris_key, q_key = tris, q
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    rdt = torch.float64 if m == PFT_FP64 else torch.float32
    out = torch.empty(q.shape[0], dtype=cdt, device=verts.device)
    inten = torch.empty(q.shape[0], dtype=rdt, device=verts.device) if intensity else None
    fo, fm = _order_arg(order, tris_key, tris, verts.shape[0], m)
    qo = _q_order_arg(q_order, q_key, q)
    with torch.cuda.device(verts.device):
        if fo is None and qo is None:
            check(_lib.load().pft_forward_3d(_ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0],
                                             _ptr(tris), tris.shape[0], _ptr(q), _real_dtype_id(q, "q"),
                                             q.shape[0], m, _ptr(out), _ptr(inten), _stream(verts.device)))
        else:
            check(_lib.load().pft_forward_3d_ordered(
                _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0], _ptr(tris), tris.shape[0], _ptr(fo),
                _ptr(fm), _ptr(q), _real_dtype_id(q, "q"), q.shape[0], m, _ptr(out), _ptr(inten), _ptr(qo),
                _stream(verts.device)))
    return (out, inten) if intensity else out


def forward_3d_noalloc(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, mode: str = "fp32c",
                       intensity: bool = False):
    """forward_3d through pft_forward_3d_noalloc: the library allocates nothing in the call (its
    temporaries are in a fixed 64 MiB device array per GPU); Q in the list order, faces in the list
    order. The outputs are allocated here by torch, as for every wrapper."""
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    rdt = torch.float64 if m == PFT_FP64 else torch.float32
    out = torch.empty(q.shape[0], dtype=cdt, device=verts.device)
    inten = torch.empty(q.shape[0], dtype=rdt, device=verts.device) if intensity else None
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_forward_3d_noalloc(_ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0],
                                                 _ptr(tris), tris.shape[0], _ptr(q), _real_dtype_id(q, "q"),
                                                 q.shape[0], m, _ptr(out), _ptr(inten), _stream(verts.device)))
    return (out, inten) if intensity else out


def forward_3d_poly(verts: torch.Tensor, faces: Sequence[Sequence[int]], q: torch.Tensor, mode: str = "fp32c",
                    intensity: bool = False):
    """F(Q) of a closed mesh of planar polygon faces (each a CCW list of vertex indices, 3 to 256).

    Returns F (complex128 for 'fp64', complex64 for 'fp32c'), or (F, |F|^2) when ``intensity``.
    """
    verts = _on_gpu(verts, "verts")
    if verts.dim() != 2 or verts.shape[1] != 3:
        raise ValueError(f"verts must have shape [nv, 3], got {tuple(verts.shape)}")
    off = np.zeros(len(faces) + 1, dtype=np.int64)
    for i, f in enumerate(faces):
        off[i + 1] = off[i] + len(f)
    flat = np.fromiter((int(x) for f in faces for x in f), dtype=np.int32, count=int(off[-1]))
    fv = torch.from_numpy(flat).to(verts.device)
    q = _qlist(q, verts.device)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    rdt = torch.float64 if m == PFT_FP64 else torch.float32
    out = torch.empty(q.shape[0], dtype=cdt, device=verts.device)
    inten = torch.empty(q.shape[0], dtype=rdt, device=verts.device) if intensity else None
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_forward_3d_poly(
            _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0],
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(fv), len(faces), _ptr(q),
            _real_dtype_id(q, "q"), q.shape[0], m, _ptr(out), _ptr(inten), _stream(verts.device)))
    return (out, inten) if intensity else out


def orientation_average(verts: torch.Tensor, tris: torch.Tensor, qabs: torch.Tensor, dirs: torch.Tensor,
                        weights: torch.Tensor, mode: str = "fp32c", order="auto") -> torch.Tensor:
    """I(|Q|) = sum_j w_j |F(|Q| s_j)|^2 for each magnitude in ``qabs`` (float64 result).

    ``dirs`` [ndir, 3] unit vectors and ``weights`` [ndir] form the direction
    quadrature (float64, on the mesh's device).
    """
    tris_key = tris
    verts, tris = _mesh(verts, tris)
    qabs = _on_gpu(qabs, "qabs")
    dirs = _on_gpu(dirs, "dirs")
    weights = _on_gpu(weights, "weights")
    for name, t in (("qabs", qabs), ("dirs", dirs), ("weights", weights)):
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64, got {t.dtype}")
        if t.device != verts.device:
            raise ValueError(f"{name} must be on the same device as the mesh")
    if qabs.dim() != 1:
        raise ValueError(f"qabs must have shape [nqa], got {tuple(qabs.shape)}")
    if dirs.dim() != 2 or dirs.shape[1] != 3:
        raise ValueError(f"dirs must have shape [ndir, 3], got {tuple(dirs.shape)}")
    if weights.dim() != 1 or weights.shape[0] != dirs.shape[0]:
        raise ValueError("weights must have shape [ndir] matching dirs")
    out = torch.empty(qabs.shape[0], dtype=torch.float64, device=verts.device)
    fo, fm = _order_arg(order, tris_key, tris, verts.shape[0], mode_id(mode))
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_orientation_average(
            _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0], _ptr(tris), tris.shape[0], _ptr(qabs),
            qabs.shape[0], _ptr(dirs), _ptr(weights), dirs.shape[0], mode_id(mode), _ptr(out), _ptr(fo), _ptr(fm),
            _stream(verts.device)))
    return out


def backward_3d(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, grad_out: torch.Tensor,
                mode: str = "fp32c", q_order="auto") -> torch.Tensor:
    """dL/dverts for grad_out = dL/dReF + i dL/dImF; same dtype and shape as verts. ``q_order`` as for
    forward_3d."""
    q_key = q
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    g = _on_gpu(grad_out, "grad_out").reshape(-1)
    if g.shape[0] != q.shape[0]:
        raise ValueError("grad_out must have one entry per Q")
    g = g.to(cdt).contiguous()
    grad = torch.empty_like(verts)
    qo = _q_order_arg(q_order, q_key, q)
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_backward_3d_ordered(
            _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0], _ptr(tris), tris.shape[0], _ptr(q),
            _real_dtype_id(q, "q"), q.shape[0], m, _ptr(g), _ptr(grad), _ptr(qo), _stream(verts.device)))
    return grad


def intensity_loss_3d(verts: torch.Tensor, tris: torch.Tensor, q: torch.Tensor, target: torch.Tensor,
                      weight: Optional[torch.Tensor] = None, mode: str = "fp32c", need_grad: bool = True,
                      return_F: bool = False, order="auto"):
    """L = sum_Q w (|F|^2 - I)^2 and dL/dverts in one library call (forward, cotangent and adjoint
    sharing the face records and the Q order). ``target`` and ``weight`` are float64 [nq] on the
    device (weight None: w = 1). Returns (L as a 0-dim float64 tensor, dL/dverts or None[, F]).
    ``order`` as for forward_3d (the FP32C forward part in an edge-sharing face order).
    """
    tris_key = tris
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    m = mode_id(mode)
    nq = q.shape[0]

    def f64vec(t, name):
        t = _on_gpu(t, name).reshape(-1)
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64, got {t.dtype}")
        if t.shape[0] != nq or t.device != verts.device:
            raise ValueError(f"{name} must have one entry per Q on the mesh's device")
        return t.contiguous()
    target = f64vec(target, "target")
    weight = None if weight is None else f64vec(weight, "weight")
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    loss = torch.empty((), dtype=torch.float64, device=verts.device)
    F = torch.empty(nq, dtype=cdt, device=verts.device) if return_F else None
    gv = torch.empty_like(verts) if need_grad else None
    fo, fm = _order_arg(order, tris_key, tris, verts.shape[0], m)
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_intensity_loss_3d(
            _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0], _ptr(tris), tris.shape[0], _ptr(q),
            _real_dtype_id(q, "q"), nq, m, _ptr(weight), _ptr(target), loss.data_ptr(), _ptr(F), _ptr(gv),
            _ptr(fo), _ptr(fm), _stream(verts.device)))
    return (loss, gv, F) if return_F else (loss, gv)


def _regions(region_offsets, nf: int, rho: torch.Tensor, device):
    off = np.ascontiguousarray(np.asarray(region_offsets, dtype=np.int64).reshape(-1))
    if off.size < 1 or off[0] != 0 or off[-1] != nf or np.any(np.diff(off) < 0):
        raise ValueError("region_offsets must rise from 0 to the number of triangles")
    rho = _on_gpu(rho, "rho").reshape(-1)
    if rho.dtype != torch.float64:
        raise TypeError(f"rho must be float64, got {rho.dtype}")
    if rho.device != device:
        raise ValueError("rho must be on the same device as the mesh")
    if rho.shape[0] != off.size - 1:
        raise ValueError("rho needs one density per region")
    return off, rho.contiguous()


def forward_3d_regions(verts: torch.Tensor, tris: torch.Tensor, region_offsets, rho: torch.Tensor, q: torch.Tensor,
                       mode: str = "fp32c", per_region: bool = False, intensity: bool = False, order="auto"):
    """F = sum_j rho_j F_j for a density rho_j constant on closed region j, whose outward boundary is
    triangles region_offsets[j] .. region_offsets[j+1] (host offsets; rho float64 on the device).

    Returns F, with F_j [nreg, nq] (= dF/drho) when ``per_region`` and |F|^2 when ``intensity``
    appended in that order. ``order``: "auto" (FP32C: each region's faces in an edge-sharing order,
    cached per triangle tensor and offsets), None, or (order, meta) device tensors that keep every face
    within its region.
    """
    tris_key = tris
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    off, rho = _regions(region_offsets, tris.shape[0], rho, verts.device)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    rdt = torch.float64 if m == PFT_FP64 else torch.float32
    out = torch.empty(q.shape[0], dtype=cdt, device=verts.device)
    regs = torch.empty((off.size - 1, q.shape[0]), dtype=cdt, device=verts.device) if per_region else None
    inten = torch.empty(q.shape[0], dtype=rdt, device=verts.device) if intensity else None
    if isinstance(order, str):
        if order != "auto":
            raise ValueError(f"order must be 'auto', None or (order, meta), got {order!r}")
        use = m == PFT_FP32C and isinstance(tris_key, torch.Tensor) and tris.shape[0] >= _AUTO_ORDER_MIN_FACES
        # regions are ranges of one triangle list over shared vertices: order each range on its own
        nvs = np.full(off.size, verts.shape[0], dtype=np.int64)
        nvs[0] = 0
        order = _batch_auto_order(tris_key, (np.cumsum(nvs), off), verts.device) if use else None
    fo, fm = _order_arg(order, None, tris, verts.shape[0], m) if order is not None else (None, None)
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_forward_3d_regions(
            _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0], _ptr(tris), tris.shape[0],
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), off.size - 1, _ptr(rho), _ptr(q),
            _real_dtype_id(q, "q"), q.shape[0], m, _ptr(out), _ptr(regs), _ptr(inten), _ptr(fo), _ptr(fm),
            _stream(verts.device)))
    res = (out,) + ((regs,) if per_region else ()) + ((inten,) if intensity else ())
    return res[0] if len(res) == 1 else res


def backward_3d_regions(verts: torch.Tensor, tris: torch.Tensor, region_offsets, rho: torch.Tensor, q: torch.Tensor,
                        grad_out: torch.Tensor, mode: str = "fp32c", need_verts: bool = True, need_rho: bool = True,
                        need_q: bool = True):
    """(dL/dverts, dL/drho, dL/dQ) for grad_out = dL/dReF + i dL/dImF, F = sum_j rho_j F_j.

    Entries not asked for are None. dL/dverts has the dtype of verts, dL/drho float64, dL/dQ the
    dtype of q.
    """
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    off, rho = _regions(region_offsets, tris.shape[0], rho, verts.device)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    g = _on_gpu(grad_out, "grad_out").reshape(-1)
    if g.shape[0] != q.shape[0]:
        raise ValueError("grad_out must have one entry per Q")
    g = g.to(cdt).contiguous()
    gv = torch.empty_like(verts) if need_verts else None
    gr = torch.empty(off.size - 1, dtype=torch.float64, device=verts.device) if need_rho else None
    gq = torch.empty_like(q) if need_q else None
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_backward_3d_regions(
            _ptr(verts), _real_dtype_id(verts, "verts"), verts.shape[0], _ptr(tris), tris.shape[0],
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), off.size - 1, _ptr(rho), _ptr(q),
            _real_dtype_id(q, "q"), q.shape[0], m, _ptr(g), _ptr(gv), _ptr(gr), _ptr(gq), _stream(verts.device)))
    return gv, gr, gq


def _batch_struct(verts, tris, q, vert_offsets, tri_offsets, q_offsets):
    verts, tris = _mesh(verts, tris)
    q = _qlist(q, verts.device)
    offs = [np.ascontiguousarray(np.asarray(o, dtype=np.int64)) for o in (vert_offsets, tri_offsets, q_offsets)]
    n = offs[0].size - 1
    if any(o.size != n + 1 for o in offs):
        raise ValueError("offset arrays must all have n_meshes + 1 entries")
    if offs[0][-1] != verts.shape[0] or offs[1][-1] != tris.shape[0] or offs[2][-1] != q.shape[0]:
        raise ValueError("offsets must end at the concatenated sizes")
    b = PftMeshBatch()
    b.n_meshes = n
    b.vert_offsets = offs[0].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    b.tri_offsets = offs[1].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    b.q_offsets = offs[2].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    b.verts = _ptr(verts)
    b.vdtype = _real_dtype_id(verts, "verts")
    b.tris = _ptr(tris)
    b.q = _ptr(q)
    b.qdtype = _real_dtype_id(q, "q")
    return b, offs, verts, tris, q


def batch_strip_order(tris, vert_offsets, tri_offsets) -> Tuple[np.ndarray, np.ndarray]:
    """Edge-sharing order of every mesh of a batch (indices local to each mesh): global (order, meta)
    for batch_forward's ``order``, each mesh's order offset by its first triangle."""
    t = tris.detach().cpu().numpy() if isinstance(tris, torch.Tensor) else np.asarray(tris)
    t = np.ascontiguousarray(t, dtype=np.int32).reshape(-1, 3)
    vo = np.asarray(vert_offsets, dtype=np.int64)
    to = np.asarray(tri_offsets, dtype=np.int64)
    order = np.empty(t.shape[0], dtype=np.int32)
    meta = np.empty(t.shape[0], dtype=np.uint8)
    for i in range(to.size - 1):
        a, b = int(to[i]), int(to[i + 1])
        if b > a:
            o, mt = strip_order(t[a:b], int(vo[i + 1] - vo[i]))
            order[a:b] = o + a
            meta[a:b] = mt
    return order, meta


_BATCH_ORDER_CACHE: dict = {}


def _batch_auto_order(tris_key: torch.Tensor, offs, device):
    stamp = (tris_key.data_ptr(), tuple(tris_key.shape), tris_key._version, offs[0].tobytes(), offs[1].tobytes())
    hit = _BATCH_ORDER_CACHE.get(id(tris_key))
    if hit is not None and hit[0]() is tris_key and hit[1] == stamp:
        return hit[2]
    order, meta = batch_strip_order(tris_key, offs[0], offs[1])
    dev_order = (torch.from_numpy(order).to(device), torch.from_numpy(meta).to(device))
    if len(_BATCH_ORDER_CACHE) >= 16:
        for k in [k for k, e in _BATCH_ORDER_CACHE.items() if e[0]() is None]:
            del _BATCH_ORDER_CACHE[k]
    _BATCH_ORDER_CACHE[id(tris_key)] = (weakref.ref(tris_key), stamp, dev_order)
    return dev_order


def batch_forward(verts, tris, q, vert_offsets, tri_offsets, q_offsets, mode: str = "fp32c",
                  intensity: bool = False, order="auto"):
    """Transform of every mesh of a concatenated batch (indices local to each mesh).

    ``order``: "auto" (FP32C: each mesh's faces in an edge-sharing order, computed on the host at the
    first call for a triangle tensor and reused while it is unchanged), None, or device tensors
    (order int32, meta uint8) from ``batch_strip_order``.
    """
    tris_key = tris
    b, offs, verts, tris, q = _batch_struct(verts, tris, q, vert_offsets, tri_offsets, q_offsets)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    rdt = torch.float64 if m == PFT_FP64 else torch.float32
    out = torch.empty(q.shape[0], dtype=cdt, device=verts.device)
    inten = torch.empty(q.shape[0], dtype=rdt, device=verts.device) if intensity else None
    if isinstance(order, str):
        if order != "auto":
            raise ValueError(f"order must be 'auto', None or (order, meta), got {order!r}")
        use = m == PFT_FP32C and isinstance(tris_key, torch.Tensor) and tris.shape[0] >= _AUTO_ORDER_MIN_FACES
        order = _batch_auto_order(tris_key, offs, verts.device) if use else None
    with torch.cuda.device(verts.device):
        if order is None:
            check(_lib.load().pft_batch_forward(ctypes.byref(b), m, _ptr(out), _ptr(inten), _stream(verts.device)))
        else:
            fo, fm = (_on_gpu(x, name) for x, name in zip(order, ("order", "meta")))
            if fo.dtype != torch.int32 or fm.dtype != torch.uint8 or fo.numel() != tris.shape[0] \
                    or fm.numel() != tris.shape[0]:
                raise ValueError("order must be (int32 [nf], uint8 [nf]) device tensors")
            check(_lib.load().pft_batch_forward_ordered(ctypes.byref(b), _ptr(fo), _ptr(fm), m, _ptr(out),
                                                        _ptr(inten), _stream(verts.device)))
    del offs  # host offsets are read synchronously by the call
    return (out, inten) if intensity else out


def batch_backward(verts, tris, q, vert_offsets, tri_offsets, q_offsets, grad_out, mode: str = "fp32c"):
    """dL/dverts of every mesh of a batch; [total_nv, 3] like verts."""
    b, offs, verts, tris, q = _batch_struct(verts, tris, q, vert_offsets, tri_offsets, q_offsets)
    m = mode_id(mode)
    cdt = torch.complex128 if m == PFT_FP64 else torch.complex64
    g = _on_gpu(grad_out, "grad_out").reshape(-1).to(cdt).contiguous()
    if g.shape[0] != q.shape[0]:
        raise ValueError("grad_out must have one entry per Q")
    grad = torch.empty_like(verts)
    with torch.cuda.device(verts.device):
        check(_lib.load().pft_batch_backward(ctypes.byref(b), m, _ptr(g), _ptr(grad), _stream(verts.device)))
    del offs
    return grad


def check_mesh(tris, nv: Optional[int] = None) -> dict:
    """pft_check_mesh on the host: counts of out-of-range indices, faces with a repeated vertex, open
    edges, edges of more than two faces and edges both faces run the same way (all zero for a closed,
    consistently oriented triangle mesh). ``tris`` may be a tensor (copied to the host)."""
    t = tris.detach().cpu().numpy() if isinstance(tris, torch.Tensor) else np.asarray(tris)
    t = np.ascontiguousarray(t, dtype=np.int32).reshape(-1, 3)
    if nv is None:
        nv = int(t.max()) + 1 if t.size else 0
    rep = _lib.PftMeshCheck()
    check(_lib.load().pft_check_mesh(t.ctypes.data, t.shape[0], nv, ctypes.byref(rep)))
    return {name: int(getattr(rep, name)) for name, _ in rep._fields_}


def fp32c_q_limit(verts, tris) -> float:
    """pft_fp32c_q_limit on the host: the largest |Q| at which PFT_FP32C evaluates this triangle mesh
    (PFT_FP32C_PHASE_MAX over the largest face centroid-to-vertex distance; inf for a mesh without
    extent). Beyond it the FP32C outputs at that Q are NaN. Tensors are copied to the host."""
    v = verts.detach().cpu().numpy() if isinstance(verts, torch.Tensor) else np.asarray(verts)
    t = tris.detach().cpu().numpy() if isinstance(tris, torch.Tensor) else np.asarray(tris)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(t, dtype=np.int32).reshape(-1, 3)
    lim = ctypes.c_double(0.0)
    check(_lib.load().pft_fp32c_q_limit(v.ctypes.data, _lib.PFT_F64, v.shape[0], t.ctypes.data, t.shape[0],
                                        ctypes.byref(lim)))
    return float(lim.value)


def validate_mesh(tris: torch.Tensor, nv: int) -> Tuple[int, int]:
    """(number of out-of-range indices, number of faces with a repeated vertex)."""
    tris = _on_gpu(tris, "tris").to(torch.int32)
    bad, rep = ctypes.c_int64(0), ctypes.c_int64(0)
    with torch.cuda.device(tris.device):
        check(_lib.load().pft_validate_mesh(_ptr(tris), tris.shape[0], int(nv), ctypes.byref(bad), ctypes.byref(rep),
                                            _stream(tris.device)))
    return int(bad.value), int(rep.value)


def profile_enable(on: bool = True) -> None:
    check(_lib.load().pft_profile_enable(1 if on else 0))


def profile_reset() -> None:
    check(_lib.load().pft_profile_reset())


def profile_read(name: str) -> Tuple[int, float]:
    """(launches, total milliseconds) of a kernel family since the last reset."""
    n, ms = ctypes.c_int64(0), ctypes.c_double(0.0)
    check(_lib.load().pft_profile_read(name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def release_workspace() -> None:
    check(_lib.load().pft_release_workspace())


def tuning_info() -> str:
    """The batched launches' tile sizes chosen at run time in this process (pft_tuning_info), one line
    per (GPU, form, size bucket): the choice and each candidate's time in ms."""
    return _lib.load().pft_tuning_info().decode()


def version() -> str:
    return _lib.load().pft_version().decode()
