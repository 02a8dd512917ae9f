"""Binding of the visual-hull initialisation and the multi-view consistency
filter (Sec. 3.1 initialisation; the appendix's consistency check): libdpr
entry points, argument marshalling only."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import torch

from . import _abi
from ._abi import check, load
from .renderer import SceneTensors, _stream_handle, camera_struct


def _tables(cams: Sequence, masks: Sequence[torch.Tensor]):
    if len(cams) != len(masks) or not cams:
        raise ValueError("one mask per camera, at least one camera")
    for m in masks:
        if m.dtype != torch.uint8 or not m.is_cuda or not m.is_contiguous() or m.dim() != 2:
            raise ValueError("masks must be contiguous uint8 [H, W] device tensors")
    c = (_abi.Camera * len(cams))(*[camera_struct(x) for x in cams])
    mk = (_abi.Mask * len(masks))(*[_abi.Mask(m.data_ptr(), int(m.shape[1]), int(m.shape[0])) for m in masks])
    return c, mk


def _ws(lib, n: int, c, dev) -> torch.Tensor:
    nbytes = lib.dpr_hull_ws_bytes(int(n), len(c), c)
    if nbytes == 0:
        check(_abi.DPR_ERR_INVALID_ARG)
    return torch.empty(int(nbytes), dtype=torch.uint8, device=dev)


def hull_sample(cams: Sequence, masks: Sequence[torch.Tensor], lo, hi, seed: int, n: int,
                capacity: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None
                ) -> Tuple[torch.Tensor, int]:
    """Rejection sampling of n candidates in the box [lo, hi]: the consistent
    ones in candidate order (at most `capacity`, default n) and their number."""
    lib = load()
    c, mk = _tables(cams, masks)
    dev = masks[0].device
    cap = int(n if capacity is None else capacity)
    out = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
    lo_c = (ctypes.c_float * 3)(*[float(v) for v in lo])
    hi_c = (ctypes.c_float * 3)(*[float(v) for v in hi])
    ws = _ws(lib, n, c, dev)
    cnt = ctypes.c_int64(0)
    check(lib.dpr_hull_sample(len(cams), c, mk, lo_c, hi_c, int(seed), int(n), out.data_ptr(), cap,
                              ctypes.byref(cnt), ws.data_ptr(), int(ws.numel()), _stream_handle(stream)))
    kept = int(cnt.value)
    return out[:min(kept, cap)], kept


def consistency(xyz: torch.Tensor, cams: Sequence, masks: Sequence[torch.Tensor],
                stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """CC of every point (uint8 [n], 1 = inside the foreground of every mask)."""
    if xyz.dtype != torch.float32 or not xyz.is_cuda or not xyz.is_contiguous() or xyz.dim() != 2 \
            or xyz.shape[1] != 3:
        raise ValueError("xyz must be a contiguous float32 [n, 3] device tensor")
    lib = load()
    c, mk = _tables(cams, masks)
    n = int(xyz.shape[0])
    keep = torch.empty(max(n, 1), dtype=torch.uint8, device=xyz.device)
    ws = _ws(lib, n, c, xyz.device)
    check(lib.dpr_consistency(n, xyz.data_ptr(), len(cams), c, mk, keep.data_ptr(), ws.data_ptr(), int(ws.numel()),
                              _stream_handle(stream)))
    return keep[:n]


def consistency_filter(scene: SceneTensors, cams: Sequence, masks: Sequence[torch.Tensor],
                       stream: Optional[torch.cuda.Stream] = None) -> SceneTensors:
    """The points of the cloud that pass the consistency check, every
    parameter, in input order."""
    scene.c_struct()                      # validates dtype / contiguity / device
    lib = load()
    c, mk = _tables(cams, masks)
    n = scene.n
    dev = scene.xyz.device
    out = SceneTensors(torch.empty((max(n, 1), 3), dtype=torch.float32, device=dev),
                       torch.empty((max(n, 1),) + tuple(scene.sh.shape[1:]), dtype=torch.float32, device=dev),
                       torch.empty((max(n, 1),), dtype=torch.float32, device=dev),
                       torch.empty((max(n, 1),), dtype=torch.float32, device=dev))
    ws = _ws(lib, n, c, dev)
    cnt = ctypes.c_int64(0)
    check(lib.dpr_consistency_filter(n, scene.sh_degree, scene.xyz.data_ptr(), scene.sh.data_ptr(),
                                     scene.opacity.data_ptr(), scene.radius.data_ptr(), len(cams), c, mk,
                                     out.xyz.data_ptr(), out.sh.data_ptr(), out.opacity.data_ptr(),
                                     out.radius.data_ptr(), ctypes.byref(cnt), ws.data_ptr(), int(ws.numel()),
                                     _stream_handle(stream)))
    k = int(cnt.value)
    return SceneTensors(out.xyz[:k], out.sh[:k], out.opacity[:k], out.radius[:k])
