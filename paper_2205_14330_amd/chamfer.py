"""Binding of the video warm start (Sec. 3.4 "Video Synthesis"): the Chamfer
distance of Eq. (9) and its gradient, the Adam step on the next frame's
positions, and the top-k SH transfer (libdpr entry points; argument
marshalling only)."""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import _abi
from ._abi import check, load
from .renderer import _stream_handle


def _xyz(t: torch.Tensor, name: str):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{name} must be a contiguous float32 [n, 3] device tensor")


def chamfer(s1: torch.Tensor, s2: torch.Tensor, grad: bool = True, nn: bool = False,
            stream: Optional[torch.cuda.Stream] = None) -> dict:
    """Eq. (9) between s1 [n1, 3] and s2 [n2, 3]: {"cd": float64 [1] device
    tensor, "grad2": dCD/ds2 [n2, 3] (if grad), "nn12", "nn21": nearest indices
    (if nn)}.  Asynchronous."""
    _xyz(s1, "s1"); _xyz(s2, "s2")
    lib = load()
    n1, n2 = int(s1.shape[0]), int(s2.shape[0])
    dev = s1.device
    out = {"cd": torch.empty(1, dtype=torch.float64, device=dev)}
    if grad:
        out["grad2"] = torch.empty((n2, 3), dtype=torch.float32, device=dev)
    if nn:
        out["nn12"] = torch.empty(n1, dtype=torch.int32, device=dev)
        out["nn21"] = torch.empty(n2, dtype=torch.int32, device=dev)
    nbytes = lib.dpr_chamfer_ws_bytes(n1, n2)
    if nbytes == 0:
        check(_abi.DPR_ERR_INVALID_ARG)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
    p = lambda k: out[k].data_ptr() if k in out else None
    check(lib.dpr_chamfer(n1, s1.data_ptr(), n2, s2.data_ptr(), p("cd"), p("grad2"), p("nn12"), p("nn21"),
                          ws.data_ptr(), int(nbytes), _stream_handle(stream)))
    return out


def topk_sh(s1: torch.Tensor, sh1: torch.Tensor, s2: torch.Tensor, K: int, with_index: bool = False,
            stream: Optional[torch.cuda.Stream] = None):
    """Mean SH [n2, C, 3] of each s2 point's K nearest s1 points (and their
    indices [n2, K], -1 past n1, if with_index).  Asynchronous."""
    _xyz(s1, "s1"); _xyz(s2, "s2")
    if sh1.dtype != torch.float32 or not sh1.is_contiguous() or sh1.dim() != 3 or sh1.shape[0] != s1.shape[0]:
        raise ValueError("sh1 must be a contiguous float32 [n1, C, 3] tensor")
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[int(sh1.shape[1])]
    lib = load()
    n1, n2 = int(s1.shape[0]), int(s2.shape[0])
    out = torch.empty((n2,) + tuple(sh1.shape[1:]), dtype=torch.float32, device=s1.device)
    idx = torch.empty((n2, K), dtype=torch.int32, device=s1.device) if with_index else None
    check(lib.dpr_topk_sh(n1, s1.data_ptr(), sh1.data_ptr(), n2, s2.data_ptr(), deg, int(K), out.data_ptr(),
                          idx.data_ptr() if idx is not None else None, _stream_handle(stream)))
    return (out, idx) if with_index else out


def adam_step(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
              stream: Optional[torch.cuda.Stream] = None) -> None:
    """One Adam step (bias-corrected, step t >= 1) in place on p, m, v (float32)."""
    for x in (p, g, m, v):
        if x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != p.numel():
            raise ValueError("p, g, m, v must be contiguous float32 tensors of one size")
    check(load().dpr_adam_step(p.numel(), p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), int(t), float(lr),
                               float(beta1), float(beta2), float(eps), _stream_handle(stream)))


def warm_start(s1: torch.Tensor, sh1: torch.Tensor, s2: torch.Tensor, steps: int, lr: float, K: int = 4
               ) -> Tuple[torch.Tensor, torch.Tensor]:
    """Initial cloud of the next frame: `steps` Adam steps on the positions of
    s2 against Eq. (9) to s1, then the mean SH of the K nearest s1 points.
    Returns (positions [n2, 3], SH [n2, C, 3])."""
    p = s2.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    for t in range(1, steps + 1):
        g = chamfer(s1, p)["grad2"]
        adam_step(p, g, m, v, t, lr)
    return p, topk_sh(s1, sh1, p, K)


class ChamferFn(torch.autograd.Function):
    """Eq. (9) as an autograd function of the positions of s2 (s1 is a
    constant: the learned cloud of the previous frame)."""

    @staticmethod
    def forward(ctx, s1, s2):
        out = chamfer(s1.detach().contiguous(), s2.detach().contiguous())
        ctx.save_for_backward(out["grad2"])
        return out["cd"][0]

    @staticmethod
    def backward(ctx, go):
        (g2,) = ctx.saved_tensors
        return None, (g2 * go.to(torch.float32))
