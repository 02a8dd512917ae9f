"""Python binding of libdpr: argument marshalling only.

Every step of the renderer runs in the HIP kernels of libdpr.so; this module
turns torch tensors (device memory) and camera descriptions into the C-ABI
structs, allocates the workspaces the library asks for, and passes the
current torch stream.  ``RenderFn`` is the autograd form.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import (BWD_RECOMPUTE, BWD_STORED, FLAG_KERNEL_NORM, FLAG_PERSISTENT, FLAG_STATS, FLAG_TIMING, check,
                   load)


@dataclasses.dataclass
class RenderParams:
    """Thresholds and options of one render (see include/dpr.h)."""
    alpha_min: float = 1e-5
    t_min: float = 1e-5
    alpha_max: float = 0.99
    z_near: float = 0.01
    sh_frame: int = 0              # 0: camera-frame view direction, 1: world frame
    bwd_mode: str = "stored"       # "stored" or "recompute"
    timing: bool = False
    stats: bool = False
    persistent: bool = False
    max_splats: int = 0            # > 0: a pixel blends at most this many splats (the paper's n = 15)
    kernel_norm: bool = False      # keep Eq. (5)'s normalisation prefactor
    timing_stages: tuple = ()      # with timing: names of the stages to time (empty: all)

    @staticmethod
    def paper(**kw) -> "RenderParams":
        """The paper's literal renderer: n = 15 splats per pixel, Eq. (5) normalised."""
        return RenderParams(max_splats=15, kernel_norm=True, **kw)

    def to_c(self) -> _abi.Params:
        flags = (FLAG_TIMING if self.timing else 0) | (FLAG_STATS if self.stats else 0) | \
                (FLAG_PERSISTENT if self.persistent else 0) | (FLAG_KERNEL_NORM if self.kernel_norm else 0)
        mode = {"stored": BWD_STORED, "recompute": BWD_RECOMPUTE}[self.bwd_mode]
        mask = 0
        for name in self.timing_stages:
            mask |= 1 << _abi.STAGES.index(name)
        return _abi.Params(self.alpha_min, self.t_min, self.alpha_max, self.z_near, self.sh_frame, mode, flags,
                           int(self.max_splats), mask)


@dataclasses.dataclass
class SceneTensors:
    """Device tensors of one point cloud (float32, contiguous)."""
    xyz: torch.Tensor        # [N, 3]
    sh: torch.Tensor         # [N, K, 3]
    opacity: torch.Tensor    # [N]
    radius: torch.Tensor     # [N]

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def sh_degree(self) -> int:
        return {1: 0, 4: 1, 9: 2, 16: 3}[int(self.sh.shape[1])]

    @staticmethod
    def from_numpy(scene, device="cuda") -> "SceneTensors":
        def t(a):
            return torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        return SceneTensors(t(scene.xyz), t(scene.sh), t(scene.opacity), t(scene.radius))

    def c_struct(self) -> _abi.Scene:
        for name in ("xyz", "sh", "opacity", "radius"):
            v = getattr(self, name)
            if v.dtype != torch.float32 or not v.is_contiguous() or not v.is_cuda:
                raise ValueError(f"scene.{name} must be a contiguous float32 CUDA tensor")
        return _abi.Scene(self.n, self.sh_degree, 0, self.xyz.data_ptr(), self.sh.data_ptr(),
                          self.opacity.data_ptr(), self.radius.data_ptr())


def camera_struct(cam) -> _abi.Camera:
    """``cam``: any object with R (3x3), t (3), fx, fy, cx, cy, width, height."""
    c = _abi.Camera()
    R = np.asarray(cam.R, dtype=np.float32).reshape(9).tolist()
    t = np.asarray(cam.t, dtype=np.float32).reshape(3).tolist()
    c.R[:] = R
    c.t[:] = t
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Workspace:
    """Device buffers for the plan, forward and backward workspaces, reused by
    successive plans and grown geometrically (never shrunk), so a loop whose
    pair count varies from step to step stops allocating device memory after
    its first steps.

    A Workspace serves ONE plan at a time: making a new plan with it hands the
    buffers to that plan, and the earlier plan's forward/backward then raise.
    Work of successive plans on one stream is ordered by the stream, so a plan
    may be made while the previous one's kernels are still queued; plans on
    different streams, or two plans alive at once (e.g. one's statistics read
    while the next runs), need a Workspace each.
    """

    def __init__(self, device="cuda", headroom: float = 1.25):
        self.device = torch.device(device)
        self.headroom = float(headroom)
        self.bufs = {}
        self.owner = None

    def get(self, name: str, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 1)
        b = self.bufs.get(name)
        if b is None or b.numel() < nbytes:
            size = (int(nbytes * self.headroom) + (1 << 21) - 1) & ~((1 << 21) - 1)
            self.bufs.pop(name, None)
            b = torch.empty(size, dtype=torch.uint8, device=self.device)
            self.bufs[name] = b
        return b

    def reserved_bytes(self) -> int:
        return sum(b.numel() for b in self.bufs.values())


class Plan:
    """One batch of views over one or more resident scenes.

    The plan workspace, the forward workspace and the output images are
    allocated with torch on the scenes' device (or taken from `workspace`);
    the library does no device allocation of its own.
    """

    def __init__(self, scenes: Sequence[SceneTensors], views: Sequence[Tuple[int, object]],
                 params: RenderParams = RenderParams(), stream: Optional[torch.cuda.Stream] = None,
                 images: Optional[Sequence[torch.Tensor]] = None, trans: Optional[Sequence[torch.Tensor]] = None,
                 workspace: Optional[Workspace] = None, forward_now: bool = False):
        """forward_now: also render, in the same call (then forward() returns
        the images without further work the first time).  With a Workspace
        that already holds a forward buffer, the forward is queued behind the
        plan stage before the host waits for the pair count
        (dpr_plan_forward_render); if the buffer proves too small, it is grown
        and the forward runs after the wait."""
        self.lib = load()
        self.workspace = workspace
        self.scenes = list(scenes)
        self.views = list(views)
        self.params = params
        self.stream = stream
        dev = self.scenes[0].xyz.device
        self.device = dev
        self._c_scenes = (_abi.Scene * len(self.scenes))(*[s.c_struct() for s in self.scenes])
        self._cams = [camera_struct(c) for _, c in self.views]
        if images is None:
            images = [torch.empty((c.height, c.width, 3), device=dev, dtype=torch.float32) for c in self._cams]
        if trans is None:
            trans = [torch.empty((c.height, c.width), device=dev, dtype=torch.float32) for c in self._cams]
        self.images = list(images)
        self.trans = list(trans)
        cv = []
        for (si, _), cam, img, tr in zip(self.views, self._cams, self.images, self.trans):
            cv.append(_abi.View(int(si), 0, cam, img.data_ptr(), 0 if tr is None else tr.data_ptr()))
        self._c_views = (_abi.View * len(cv))(*cv)
        self._c_params = params.to_c()
        nbytes = self.lib.dpr_plan_ws_bytes(self._c_scenes, len(self.scenes), self._c_views, len(cv))
        if nbytes == 0:
            check(_abi.DPR_ERR_INVALID_ARG)
        if workspace is not None:
            workspace.owner = self
            self.plan_ws = workspace.get("plan", nbytes)
        else:
            self.plan_ws = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        self._plan = ctypes.c_void_p()
        self.ws = None
        self._rendered = False
        fwd = workspace.bufs.get("fwd") if (forward_now and workspace is not None) else None
        if fwd is not None:
            done = ctypes.c_int32(0)
            rc = self.lib.dpr_plan_forward_render(self._c_scenes, len(self.scenes), self._c_views, len(cv),
                                                  ctypes.byref(self._c_params), self.plan_ws.data_ptr(),
                                                  int(nbytes), fwd.data_ptr(), int(fwd.numel()),
                                                  _stream_handle(stream), ctypes.byref(self._plan),
                                                  ctypes.byref(done))
            check(rc)
            if done.value:
                self.ws = fwd
                self._rendered = True
        else:
            rc = self.lib.dpr_plan_forward(self._c_scenes, len(self.scenes), self._c_views, len(cv),
                                           ctypes.byref(self._c_params), self.plan_ws.data_ptr(), int(nbytes),
                                           _stream_handle(stream), ctypes.byref(self._plan))
            check(rc)
        if forward_now and not self._rendered:
            self.forward()
            self._rendered = True

    def _check_owner(self):
        if self.workspace is not None and self.workspace.owner is not self:
            raise RuntimeError("this plan's Workspace has been handed to a newer plan")

    # -- forward ------------------------------------------------------------------
    def forward(self):
        self._check_owner()
        if self._rendered:           # rendered together with the plan
            self._rendered = False
            return self.images, self.trans
        n = int(self.lib.dpr_workspace_bytes(self._plan))
        if self.ws is None or self.ws.numel() < n:
            if self.workspace is not None:
                self.ws = self.workspace.get("fwd", n)
            else:
                self.ws = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        check(self.lib.dpr_render_forward(self._plan, self.ws.data_ptr(), int(self.ws.numel()),
                                          _stream_handle(self.stream)))
        return self.images, self.trans

    # -- backward -----------------------------------------------------------------
    def backward(self, dL_dimage: Sequence[torch.Tensor], dL_dtrans: Optional[Sequence[Optional[torch.Tensor]]] = None,
                 want=("xyz", "sh", "opacity"), out=None):
        """Returns per-scene lists of (dxyz, dsh, dopacity) tensors (None where not wanted)."""
        if self.ws is None:
            raise RuntimeError("backward before forward")
        self._check_owner()
        gi = []
        for g, c in zip(dL_dimage, self._cams):
            if g.dtype != torch.float32 or not g.is_contiguous() or tuple(g.shape) != (c.height, c.width, 3):
                raise ValueError("dL_dimage entries must be contiguous float32 [H, W, 3]")
            gi.append(g)
        gt = None
        if dL_dtrans is not None:
            gt = []
            for g, c in zip(dL_dtrans, self._cams):
                if g is not None and (g.dtype != torch.float32 or not g.is_contiguous()
                                      or tuple(g.shape) != (c.height, c.width)):
                    raise ValueError("dL_dtrans entries must be contiguous float32 [H, W]")
                gt.append(g)
        if out is None:
            out = []
            for s in self.scenes:
                out.append((torch.empty_like(s.xyz) if "xyz" in want else None,
                            torch.empty_like(s.sh) if "sh" in want else None,
                            torch.empty_like(s.opacity) if "opacity" in want else None))
        nb = int(self.lib.dpr_backward_ws_bytes(self._plan))
        if self.workspace is not None:
            bws = self.workspace.get("bwd", nb)
        else:
            bws = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device)
        P = _abi.ptr_array
        di = P([g.data_ptr() for g in gi])
        dt = None if gt is None else P([0 if g is None else g.data_ptr() for g in gt])
        dx = P([0 if o[0] is None else o[0].data_ptr() for o in out])
        ds = P([0 if o[1] is None else o[1].data_ptr() for o in out])
        do = P([0 if o[2] is None else o[2].data_ptr() for o in out])
        check(self.lib.dpr_render_backward(self._plan, self.ws.data_ptr(), int(self.ws.numel()), di, dt, dx, ds, do,
                                           bws.data_ptr(), int(bws.numel()), _stream_handle(self.stream)))
        self._bws = bws   # keep alive until the stream has consumed it
        return out

    # -- diagnostics --------------------------------------------------------------
    def info(self) -> _abi.PlanInfo:
        inf = _abi.PlanInfo()
        check(self.lib.dpr_plan_get_info(self._plan, ctypes.byref(inf)))
        return inf

    def stage_times(self) -> dict:
        arr = (ctypes.c_float * len(_abi.STAGES))()
        check(self.lib.dpr_stage_times(self._plan, arr, len(_abi.STAGES)))
        return {name: float(arr[i]) for i, name in enumerate(_abi.STAGES)}

    def free(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            self.lib.dpr_plan_free(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class RenderFn(torch.autograd.Function):
    """Differentiable render of V same-sized views of one scene.

    forward(xyz, sh, opacity, radius, cameras, params) -> image [V,H,W,3], trans [V,H,W]
    backward returns gradients for xyz, sh and opacity (radius gets none).
    """

    @staticmethod
    def forward(ctx, xyz, sh, opacity, radius, cameras, params: RenderParams):
        V = len(cameras)
        H, W = int(cameras[0].height), int(cameras[0].width)
        if any(int(c.height) != H or int(c.width) != W for c in cameras):
            raise ValueError("RenderFn needs views of one size; use Plan for mixed sizes")
        scene = SceneTensors(xyz.detach().contiguous(), sh.detach().contiguous(),
                             opacity.detach().contiguous(), radius.detach().contiguous())
        img = torch.empty((V, H, W, 3), device=xyz.device, dtype=torch.float32)
        tr = torch.empty((V, H, W), device=xyz.device, dtype=torch.float32)
        plan = Plan([scene], [(0, c) for c in cameras], params, images=list(img.unbind(0)),
                    trans=list(tr.unbind(0)))
        plan.forward()
        ctx.plan = plan
        ctx.save_for_backward(tr)
        return img, tr

    @staticmethod
    def backward(ctx, g_img, g_tr):
        (tr,) = ctx.saved_tensors   # version check: trans must not have been modified in place
        plan: Plan = ctx.plan
        V = g_img.shape[0] if g_img is not None else tr.shape[0]
        if g_img is None:
            g_img = torch.zeros((V,) + tuple(plan.images[0].shape), device=tr.device)
        g_img = g_img.contiguous().float()
        gi = list(g_img.unbind(0))
        gt = None
        if g_tr is not None:
            g_tr = g_tr.contiguous().float()
            gt = list(g_tr.unbind(0))
        (dx, ds, do), = plan.backward(gi, gt)
        return dx, ds, do, None, None, None


def render(xyz, sh, opacity, radius, cameras, params: RenderParams = RenderParams()):
    """Autograd-aware render of one scene from a list of same-sized cameras."""
    return RenderFn.apply(xyz, sh, opacity, radius, list(cameras), params)


def render_views(scenes: Sequence[SceneTensors], views: Sequence[Tuple[int, object]],
                 params: RenderParams = RenderParams(), stream=None) -> Plan:
    """Forward render of many views of many resident scenes in one batch
    (mixed resolutions allowed).  Returns the executed Plan (images in
    plan.images, transmittance in plan.trans)."""
    p = Plan(scenes, views, params, stream=stream)
    p.forward()
    return p


def loss_l2_tv(renders: Sequence[torch.Tensor], targets: Sequence[torch.Tensor], lam: float = 0.01,
               grads: Optional[Sequence[torch.Tensor]] = None, stream: Optional[torch.cuda.Stream] = None,
               workspace: Optional[Workspace] = None):
    """Eq. (8) per image: squared L2 + lam * anisotropic TV, and its gradient,
    in one pass (libdpr).  renders/targets: contiguous float32 [H, W, 3] device
    tensors.  Returns (loss float64 tensor [n] on the device, list of dL/drender)."""
    lib = load()
    n = len(renders)
    if n == 0 or len(targets) != n:
        raise ValueError("need the same non-zero number of renders and targets")
    for r, t in zip(renders, targets):
        if (r.dtype != torch.float32 or t.dtype != torch.float32 or not r.is_contiguous() or not t.is_contiguous()
                or r.dim() != 3 or r.shape[2] != 3 or tuple(r.shape) != tuple(t.shape) or not r.is_cuda):
            raise ValueError("renders and targets must be matching contiguous float32 [H, W, 3] device tensors")
    dev = renders[0].device
    if grads is None:
        grads = [torch.empty_like(r) for r in renders]
    W = (ctypes.c_int32 * n)(*[int(r.shape[1]) for r in renders])
    H = (ctypes.c_int32 * n)(*[int(r.shape[0]) for r in renders])
    nb = int(lib.dpr_loss_ws_bytes(n, W, H))
    if nb == 0:
        check(_abi.DPR_ERR_INVALID_ARG)
    ws = workspace.get("loss", nb) if workspace is not None else torch.empty(nb, dtype=torch.uint8, device=dev)
    loss = torch.empty(n, dtype=torch.float64, device=dev)
    P = _abi.ptr_array
    check(lib.dpr_loss_l2_tv(n, P([r.data_ptr() for r in renders]), P([t.data_ptr() for t in targets]), W, H,
                             float(lam), P([g.data_ptr() for g in grads]), loss.data_ptr(), ws.data_ptr(),
                             int(ws.numel()), _stream_handle(stream)))
    return loss, grads
