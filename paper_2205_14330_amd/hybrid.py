"""Binding of the hybrid coarse-to-fine update of the point cloud (Sec. 3.3,
Alg. 1) and of its exact K-nearest-neighbour search (libdpr; argument
marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from . import _abi
from ._abi import check, load
from .renderer import SceneTensors, _stream_handle


def _check_scene(s: SceneTensors):
    s.c_struct()                      # validates dtype / contiguity / device


def _ws(nbytes: int, dev) -> torch.Tensor:
    if nbytes == 0:
        check(_abi.DPR_ERR_INVALID_ARG)
    return torch.empty(int(nbytes), dtype=torch.uint8, device=dev)


def knn(xyz: torch.Tensor, K: int, stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Exact K nearest other points of each point (K <= 32): (idx int32 [m, K]
    with -1 past min(K, m - 1), float32 squared distances [m, K])."""
    if xyz.dtype != torch.float32 or not xyz.is_contiguous() or xyz.dim() != 2 or xyz.shape[1] != 3 \
            or not xyz.is_cuda:
        raise ValueError("xyz must be a contiguous float32 [m, 3] device tensor")
    lib = load()
    m = int(xyz.shape[0])
    idx = torch.empty((m, K), dtype=torch.int32, device=xyz.device)
    d2 = torch.empty((m, K), dtype=torch.float32, device=xyz.device)
    ws = _ws(lib.dpr_knn_ws_bytes(m, K), xyz.device)
    check(lib.dpr_knn(m, xyz.data_ptr(), K, idx.data_ptr(), d2.data_ptr(), ws.data_ptr(), int(ws.numel()),
                      _stream_handle(stream)))
    return idx, d2


def _empty_like_scene(s: SceneTensors, n: int) -> SceneTensors:
    dev = s.xyz.device
    return SceneTensors(torch.empty((n, 3), dtype=torch.float32, device=dev),
                        torch.empty((n,) + tuple(s.sh.shape[1:]), dtype=torch.float32, device=dev),
                        torch.empty((n,), dtype=torch.float32, device=dev),
                        torch.empty((n,), dtype=torch.float32, device=dev))


def _trim(s: SceneTensors, n: int) -> SceneTensors:
    return SceneTensors(s.xyz[:n], s.sh[:n], s.opacity[:n], s.radius[:n])


def voxel_reduce(scene: SceneTensors, N: int, stream: Optional[torch.cuda.Stream] = None) -> SceneTensors:
    """Step 1 of Alg. 1: one point per non-empty voxel of an N^3 grid over the
    bounding box, the average of its points, in ascending voxel order."""
    _check_scene(scene)
    lib = load()
    n = scene.n
    out = _empty_like_scene(scene, n)
    ws = _ws(lib.dpr_hybrid_ws_bytes(n, scene.sh_degree, 1), scene.xyz.device)
    cnt = ctypes.c_int64(0)
    check(lib.dpr_voxel_reduce(n, scene.sh_degree, scene.xyz.data_ptr(), scene.sh.data_ptr(),
                               scene.opacity.data_ptr(), scene.radius.data_ptr(), int(N), out.xyz.data_ptr(),
                               out.sh.data_ptr(), out.opacity.data_ptr(), out.radius.data_ptr(), ctypes.byref(cnt),
                               ws.data_ptr(), int(ws.numel()), _stream_handle(stream)))
    return _trim(out, int(cnt.value))


def hybrid_update(scene: SceneTensors, N: int, K: int, eps: float,
                  stream: Optional[torch.cuda.Stream] = None) -> Tuple[SceneTensors, dict]:
    """Alg. 1: voxel reduction, outlier removal, point generation.  Returns the
    new cloud (kept points, then the generated ones) and the counts."""
    _check_scene(scene)
    lib = load()
    n = scene.n
    out = _empty_like_scene(scene, 2 * n)
    ws = _ws(lib.dpr_hybrid_ws_bytes(n, scene.sh_degree, K), scene.xyz.device)
    counts = (ctypes.c_int64 * 3)()
    check(lib.dpr_hybrid_update(n, scene.sh_degree, scene.xyz.data_ptr(), scene.sh.data_ptr(),
                                scene.opacity.data_ptr(), scene.radius.data_ptr(), int(N), int(K), float(eps),
                                out.xyz.data_ptr(), out.sh.data_ptr(), out.opacity.data_ptr(),
                                out.radius.data_ptr(), counts, ws.data_ptr(), int(ws.numel()),
                                _stream_handle(stream)))
    c = {"voxels": int(counts[0]), "kept": int(counts[1]), "points": int(counts[2])}
    return _trim(out, c["points"]), c
