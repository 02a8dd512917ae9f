"""FP64 CPU oracle of the splat renderer (ctypes wrapper around oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  The product path never imports this package, and
this package imports nothing from the product path; the only thing both sides
share is the seeded input generator package ``workloads``.

Camera arguments are ``workloads.Camera`` objects (or anything with R, t, fx,
fy, cx, cy, width, height).  All arrays are widened exactly from float32 to
float64 before the call.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "hybrid.c"), os.path.join(_HERE, "hull.c"), os.path.join(_HERE, "chamfer.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ALPHA_MIN = 1e-5
T_MIN = 1e-5
ALPHA_MAX = 0.99
Z_NEAR = 0.01


@dataclass
class Params:
    """Renderer thresholds.  ``Params.untruncated()`` gives the literal
    Eq. (6)-(7) sum over every point (no cull, no early stop, no clamp)."""
    alpha_min: float = ALPHA_MIN
    t_min: float = T_MIN
    alpha_max: float = ALPHA_MAX
    z_near: float = Z_NEAR
    sh_frame: int = 0          # 0 = camera-frame direction (Eq. 3), 1 = world frame
    max_splats: int = 0        # > 0: a pixel blends at most this many splats (Sec. 3.3's n)
    kernel_norm: int = 0       # 1: keep Eq. (5)'s 1/sqrt(2 pi r^2) prefactor, per axis (2 pi sx sy)^-1/2

    @staticmethod
    def untruncated(z_near: float = Z_NEAR, sh_frame: int = 0) -> "Params":
        return Params(0.0, 0.0, 1.0, z_near, sh_frame)

    def array(self) -> np.ndarray:
        return np.array([self.alpha_min, self.t_min, self.alpha_max, self.z_near, float(self.max_splats),
                         float(self.kernel_norm)], np.float64)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C99, OpenMP, no FP contraction)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= max(os.path.getmtime(f) for f in _SRCS):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp] + _SRCS + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(f) for f in _SRCS):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.oracle_sh_basis.argtypes = [i32, P, i64, P, P]
        L.oracle_project.argtypes = [i64, P, P, i32, P, P, f64, i32, P, P]
        L.oracle_depth_order.argtypes = [i64, P, P, f64, P, P]
        L.oracle_render.argtypes = [i64, P, P, i32, P, P, P, i32, i32, P, i32, i32, i64, P,
                                    P, P, P, P, i32]
        L.oracle_backward.argtypes = [i64, P, P, i32, P, P, P, i32, i32, P, i32, i32, i64, P,
                                      P, P, P, P, P, i32]
        L.oracle_max_threads.argtypes = []
        L.hybrid_voxel_keys.argtypes = [i64, P, i32, P]
        L.hybrid_voxel_keys.restype = ctypes.c_int
        L.hybrid_voxel_reduce.argtypes = [i64, i32, P, P, P, P, i32, P, P, P, P]
        L.hybrid_voxel_reduce.restype = i64
        L.hybrid_knn.argtypes = [i64, P, i32, P, P]
        L.hybrid_knn.restype = ctypes.c_int
        L.hybrid_filter_generate.argtypes = [i64, i32, P, P, P, P, i32, ctypes.c_float, P, P, P, P, P]
        L.hybrid_filter_generate.restype = i64
        L.hull_philox.argtypes = [P, P, P]
        L.hull_philox.restype = None
        L.hull_candidates.argtypes = [ctypes.c_uint64, i64, P, P, P]
        L.hull_candidates.restype = None
        L.hull_consistent.argtypes = [i64, P, i32, P, P, P, P]
        L.hull_consistent.restype = ctypes.c_int
        L.hull_sample.argtypes = [i32, P, P, P, P, P, ctypes.c_uint64, i64, P, i64]
        L.hull_sample.restype = i64
        L.chamfer_nn.argtypes = [i64, P, i64, P, P, P]
        L.chamfer_nn.restype = ctypes.c_int
        L.chamfer_forward_backward.argtypes = [i64, P, i64, P, P, P]
        L.chamfer_forward_backward.restype = ctypes.c_int
        L.chamfer_topk_sh.argtypes = [i64, P, P, i64, P, i32, i32, P, P]
        L.chamfer_topk_sh.restype = ctypes.c_int
        L.adam_step.argtypes = [i64, P, P, P, P, i32, f64, f64, f64, f64]
        L.adam_step.restype = ctypes.c_int
        for f in (L.oracle_sh_basis, L.oracle_project, L.oracle_depth_order, L.oracle_render,
                  L.oracle_backward, L.oracle_max_threads):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32), dtype=np.float64)


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def cam_array(cam) -> np.ndarray:
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    v = np.concatenate([R, t, np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32)])
    return v.astype(np.float64)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def sh_basis(degree: int, dirs: np.ndarray, grad: bool = False):
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    K = (degree + 1) ** 2
    Y = np.zeros((dirs.shape[0], K))
    dY = np.zeros((dirs.shape[0], K, 3)) if grad else None
    rc = lib().oracle_sh_basis(degree, _p(dirs), dirs.shape[0], _p(Y), _p(dY))
    if rc:
        raise ValueError("bad SH degree")
    return (Y, dY) if grad else Y


def project(scene, cam, params: Params = Params()):
    """Per-point quantities of one view.  Returns a dict of float64 arrays
    (px, py, sx, sy, z, color[N,3], dir[N,3], valid[N] bool) and zkey float32."""
    xyz, sh, rad = _d(scene.xyz), _d(scene.sh), _d(scene.radius)
    n = xyz.shape[0]
    out = np.zeros((n, 12))
    zk = np.zeros(n, np.float32)
    rc = lib().oracle_project(n, _p(xyz), _p(sh), scene.sh_degree, _p(rad), _p(cam_array(cam)),
                              params.z_near, params.sh_frame, _p(out), _p(zk))
    if rc:
        raise ValueError("oracle_project failed")
    return dict(px=out[:, 0], py=out[:, 1], sx=out[:, 2], sy=out[:, 3], z=out[:, 4],
                color=out[:, 5:8], dir=out[:, 8:11], valid=out[:, 11] > 0.5, zkey=zk)


def depth_order(scene, cam, params: Params = Params()) -> np.ndarray:
    xyz = _d(scene.xyz)
    n = xyz.shape[0]
    order = np.zeros(max(n, 1), np.int64)
    m = np.zeros(1, np.int64)
    lib().oracle_depth_order(n, _p(xyz), _p(cam_array(cam)), params.z_near, _p(order), _p(m))
    return order[: int(m[0])]


@dataclass
class RenderResult:
    image: np.ndarray      # [npix, 3] (or [H, W, 3] for a full frame)
    trans: np.ndarray      # [npix]    (or [H, W])
    ncontrib: np.ndarray   # number of blended splats per pixel
    stopped: np.ndarray    # early stop fired
    # under a cap (max_splats > 0): the pixel's result rests on a predicate
    # decided within a relative 1e-4 of alpha_min, which an evaluation in
    # another precision may decide the other way (two valid results)
    near_tie: Optional[np.ndarray] = None


def render(scene, cam, params: Params = Params(), pixels: Optional[np.ndarray] = None,
           mode: str = "grid", threads: int = 0) -> RenderResult:
    """Forward render of one view.  ``pixels``: linear indices y*W+x, or None
    for the full frame (then the outputs are shaped [H, W, ...])."""
    xyz, sh, op, rad = _d(scene.xyz), _d(scene.sh), _d(scene.opacity), _d(scene.radius)
    n = xyz.shape[0]
    W, H = cam.width, cam.height
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = W * H if pix is None else pix.shape[0]
    img = np.zeros((npix, 3))
    tr = np.zeros(npix)
    nc = np.zeros(npix, np.int64)
    st = np.zeros(npix, np.int32)
    m = {"brute": 0, "grid": 1}[mode]
    rc = lib().oracle_render(n, _p(xyz), _p(sh), scene.sh_degree, _p(op), _p(rad), _p(cam_array(cam)),
                             W, H, _p(params.array()), params.sh_frame, m, npix, _p(pix),
                             _p(img), _p(tr), _p(nc), _p(st), threads)
    if rc:
        raise ValueError("oracle_render failed")
    tie = (st >> 1) & 1
    st = st & 1
    if pix is None:
        return RenderResult(img.reshape(H, W, 3), tr.reshape(H, W), nc.reshape(H, W), st.reshape(H, W),
                            tie.reshape(H, W).astype(bool))
    return RenderResult(img, tr, nc, st, tie.astype(bool))


@dataclass
class Grads:
    xyz: np.ndarray
    sh: np.ndarray
    opacity: np.ndarray


def backward(scene, cams: Sequence, dL_dimage: Sequence[np.ndarray],
             dL_dtrans: Optional[Sequence[Optional[np.ndarray]]] = None,
             params: Params = Params(), pixels: Optional[Sequence[Optional[np.ndarray]]] = None,
             mode: str = "grid", threads: int = 0) -> Grads:
    """Analytic gradients summed over views.  dL_dimage[v] is [H,W,3] (full
    frame) or [npix,3] matching pixels[v]."""
    xyz, sh, op, rad = _d(scene.xyz), _d(scene.sh), _d(scene.opacity), _d(scene.radius)
    n = xyz.shape[0]
    gx = np.zeros((n, 3))
    gs = np.zeros(sh.shape)
    go = np.zeros(n)
    m = {"brute": 0, "grid": 1}[mode]
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        pix = None if pixels is None or pixels[v] is None else np.ascontiguousarray(pixels[v], np.int64)
        npix = W * H if pix is None else pix.shape[0]
        gI = np.ascontiguousarray(dL_dimage[v], np.float64).reshape(npix, 3)
        gT = None
        if dL_dtrans is not None and dL_dtrans[v] is not None:
            gT = np.ascontiguousarray(dL_dtrans[v], np.float64).reshape(npix)
        rc = lib().oracle_backward(n, _p(xyz), _p(sh), scene.sh_degree, _p(op), _p(rad),
                                   _p(cam_array(cam)), W, H, _p(params.array()), params.sh_frame, m,
                                   npix, _p(pix), _p(gI), _p(gT), _p(gx), _p(gs), _p(go), threads)
        if rc:
            raise ValueError("oracle_backward failed")
    return Grads(gx, gs, go)


def render_double(xyz, sh, opacity, radius, cam, params: Params = Params(), pixels=None,
                  mode: str = "brute", threads: int = 0) -> RenderResult:
    """Forward render from float64 arrays as given (no float32 rounding of the
    inputs), used by the finite-difference checks of the gradients.  The depth
    key is still the float32 key of the (rounded) positions."""
    class _S:
        pass
    s = _S()
    s.xyz = np.ascontiguousarray(xyz, np.float64)
    s.sh = np.ascontiguousarray(sh, np.float64)
    s.opacity = np.ascontiguousarray(opacity, np.float64)
    s.radius = np.ascontiguousarray(radius, np.float64)
    s.sh_degree = {1: 0, 4: 1, 9: 2, 16: 3}[s.sh.shape[1]]
    W, H = cam.width, cam.height
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = W * H if pix is None else pix.shape[0]
    img = np.zeros((npix, 3))
    tr = np.zeros(npix)
    nc = np.zeros(npix, np.int64)
    st = np.zeros(npix, np.int32)
    m = {"brute": 0, "grid": 1}[mode]
    n = s.xyz.shape[0]
    rc = lib().oracle_render(n, _p(s.xyz), _p(s.sh), s.sh_degree, _p(s.opacity), _p(s.radius),
                             _p(cam_array(cam)), W, H, _p(params.array()), params.sh_frame, m, npix,
                             _p(pix), _p(img), _p(tr), _p(nc), _p(st), threads)
    if rc:
        raise ValueError("oracle_render failed")
    return RenderResult(img, tr, nc, st & 1, ((st >> 1) & 1).astype(bool))


def backward_double(xyz, sh, opacity, radius, cam, dL_dimage, dL_dtrans=None, params: Params = Params(),
                    pixels=None, mode: str = "brute", threads: int = 0) -> Grads:
    """Analytic gradients from float64 arrays as given (one view)."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    sh = np.ascontiguousarray(sh, np.float64)
    op = np.ascontiguousarray(opacity, np.float64)
    rad = np.ascontiguousarray(radius, np.float64)
    deg = {1: 0, 4: 1, 9: 2, 16: 3}[sh.shape[1]]
    n = xyz.shape[0]
    W, H = cam.width, cam.height
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = W * H if pix is None else pix.shape[0]
    gI = np.ascontiguousarray(dL_dimage, np.float64).reshape(npix, 3)
    gT = None if dL_dtrans is None else np.ascontiguousarray(dL_dtrans, np.float64).reshape(npix)
    gx = np.zeros((n, 3))
    gs = np.zeros(sh.shape)
    go = np.zeros(n)
    m = {"brute": 0, "grid": 1}[mode]
    rc = lib().oracle_backward(n, _p(xyz), _p(sh), deg, _p(op), _p(rad), _p(cam_array(cam)), W, H,
                               _p(params.array()), params.sh_frame, m, npix, _p(pix), _p(gI), _p(gT),
                               _p(gx), _p(gs), _p(go), threads)
    if rc:
        raise ValueError("oracle_backward failed")
    return Grads(gx, gs, go)


def loss_l2_tv(render, target, lam: float):
    """Eq. (8) for one image: the squared L2 difference plus lam times the
    anisotropic total variation |grad_x R|_1 + |grad_y R|_1 of the render, with
    forward differences between horizontally and vertically adjacent pixels,
    summed over pixels and channels.  Returns (loss, dL/drender) in FP64; the
    subgradient of |d| at d = 0 is taken as 0.  render, target: [H][W][3]."""
    R = np.asarray(render, np.float64)
    I = np.asarray(target, np.float64)
    diff = R - I
    gx = R[:, 1:, :] - R[:, :-1, :]
    gy = R[1:, :, :] - R[:-1, :, :]
    loss = float(np.sum(diff * diff) + lam * (np.abs(gx).sum() + np.abs(gy).sum()))
    grad = 2.0 * diff
    sx, sy = np.sign(gx), np.sign(gy)
    grad[:, 1:, :] += lam * sx
    grad[:, :-1, :] -= lam * sx
    grad[1:, :, :] += lam * sy
    grad[:-1, :, :] -= lam * sy
    return loss, grad


# ---------------------------------------------------------------------------
# Hybrid coarse-to-fine update (Sec. 3.3, Alg. 1); readings in hybrid.c
# ---------------------------------------------------------------------------

@dataclass
class Cloud:
    """Point cloud with every per-point parameter: xyz [m,3], sh [m,K,3],
    opacity [m], radius [m]."""
    xyz: np.ndarray
    sh: np.ndarray
    opacity: np.ndarray
    radius: np.ndarray

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    def astype(self, dt) -> "Cloud":
        return Cloud(*(np.ascontiguousarray(a, dtype=dt) for a in (self.xyz, self.sh, self.opacity, self.radius)))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def voxel_keys(xyz, N: int) -> np.ndarray:
    x = _f32(xyz)
    keys = np.zeros(x.shape[0], np.uint64)
    if lib().hybrid_voxel_keys(x.shape[0], _p(x), N, _p(keys)) != 0:
        raise ValueError("bad input")
    return keys


def voxel_reduce(cloud, N: int) -> Cloud:
    """Step 1 of Alg. 1: one point per non-empty voxel of an N^3 grid over the
    bounding box, the FP64 average of every parameter, in ascending voxel order."""
    c = cloud.astype(np.float32) if not isinstance(cloud, Cloud) else cloud.astype(np.float32)
    n, K = c.n, c.sh.shape[1]
    ox, os_, oo, orad = np.zeros((n, 3)), np.zeros((n, K, 3)), np.zeros(n), np.zeros(n)
    m = lib().hybrid_voxel_reduce(n, 3 * K, _p(c.xyz), _p(c.sh), _p(c.opacity), _p(c.radius), N, _p(ox), _p(os_),
                                  _p(oo), _p(orad))
    if m < 0:
        raise ValueError("bad input")
    return Cloud(ox[:m], os_[:m], oo[:m], orad[:m])


def knn(xyz, K: int):
    """Brute-force K nearest neighbours among the other points: (idx [m,K]
    with -1 past min(K, m - 1), float32 squared distances [m,K])."""
    x = _f32(xyz)
    m = x.shape[0]
    idx = np.zeros((m, K), np.int64)
    d2 = np.zeros((m, K), np.float32)
    if lib().hybrid_knn(m, _p(x), K, _p(idx), _p(d2)) != 0:
        raise ValueError("bad input")
    return idx, d2


def filter_generate(cloud, K: int, eps: float):
    """Steps 2-3 of Alg. 1 on float32 points: (keep mask, output cloud = kept
    points then one generated point per kept point)."""
    c = cloud.astype(np.float32)
    m, Kc = c.n, c.sh.shape[1]
    keep = np.zeros(m, np.int32)
    ox, os_, oo, orad = np.zeros((2 * m, 3)), np.zeros((2 * m, Kc, 3)), np.zeros(2 * m), np.zeros(2 * m)
    cnt = lib().hybrid_filter_generate(m, 3 * Kc, _p(c.xyz), _p(c.sh), _p(c.opacity), _p(c.radius), K, float(eps),
                                       _p(keep), _p(ox), _p(os_), _p(oo), _p(orad))
    if cnt < 0:
        raise ValueError("bad input")
    return keep.astype(bool), Cloud(ox[:cnt], os_[:cnt], oo[:cnt], orad[:cnt])


def hybrid_update(cloud, N: int, K: int, eps: float):
    """Alg. 1: voxel reduction, then outlier removal and point generation on the
    reduced cloud (rounded to float32, as the points are stored).  Returns
    (reduced cloud, keep mask over it, output cloud)."""
    red = voxel_reduce(cloud, N)
    keep, out = filter_generate(red.astype(np.float32), K, eps)
    return red, keep, out


# ---------------------------------------------------------------------------
# visual-hull initialisation and consistency filter (oracle/hull.c)
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 (Salmon et al., SC 2011) of a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().hull_philox(_p(c), _p(k), _p(out))
    return out


def hull_candidates(seed: int, n: int, lo, hi) -> np.ndarray:
    """The first n candidates of the rejection sampler, float32 [n, 3]."""
    lo = _f32(lo); hi = _f32(hi)
    out = np.zeros((n, 3), np.float32)
    lib().hull_candidates(int(seed), int(n), _p(lo), _p(hi), _p(out))
    return out


def _hull_tables(cams, masks):
    if len(cams) != len(masks) or not cams:
        raise ValueError("one mask per camera, at least one camera")
    cam = np.stack([cam_array(c) for c in cams]).astype(np.float32)
    ms = [np.ascontiguousarray(m, np.uint8) for m in masks]
    dims = np.array([[m.shape[1], m.shape[0]] for m in ms], np.int32)
    for c, m in zip(cams, ms):
        if (c.width, c.height) != (m.shape[1], m.shape[0]):
            raise ValueError("mask size differs from its camera's image size")
    ptrs = (ctypes.c_void_p * len(ms))(*[m.ctypes.data for m in ms])
    return cam, dims, ms, ptrs


def hull_consistent(xyz, cams, masks) -> np.ndarray:
    """CC of every point: inside the foreground of every mask (bool [n])."""
    x = _f32(xyz).reshape(-1, 3)
    cam, dims, ms, ptrs = _hull_tables(cams, masks)
    keep = np.zeros(x.shape[0], np.uint8)
    if lib().hull_consistent(x.shape[0], _p(x), len(ms), _p(cam), _p(dims), ptrs, _p(keep)) != 0:
        raise ValueError("bad input")
    return keep.astype(bool)


def hull_sample(cams, masks, lo, hi, seed: int, n: int, capacity: Optional[int] = None):
    """Rejection sampling of n candidates in [lo, hi]: (number kept, kept
    points float32 [min(kept, capacity), 3] in candidate order)."""
    lo = _f32(lo); hi = _f32(hi)
    cam, dims, ms, ptrs = _hull_tables(cams, masks)
    cap = n if capacity is None else int(capacity)
    out = np.zeros((max(cap, 1), 3), np.float32)
    kept = lib().hull_sample(len(ms), _p(cam), _p(dims), ptrs, _p(lo), _p(hi), int(seed), int(n), _p(out), cap)
    if kept < 0:
        raise ValueError("bad input")
    return int(kept), out[:min(kept, cap)]


def consistency_filter(cloud, cams, masks):
    """The points of the cloud with CC = 1, in input order: (keep [n], Cloud)."""
    c = cloud.astype(np.float32)
    keep = hull_consistent(c.xyz, cams, masks)
    return keep, Cloud(c.xyz[keep], c.sh[keep], c.opacity[keep], c.radius[keep])


# ---------------------------------------------------------------------------
# video warm start: Chamfer distance (Eq. 9), top-k SH transfer, Adam (oracle/chamfer.c)
# ---------------------------------------------------------------------------

def chamfer_nn(a, b):
    """Nearest point of b for every point of a: (index int64 [na], float32 d2 [na])."""
    a = _f32(a).reshape(-1, 3); b = _f32(b).reshape(-1, 3)
    nn = np.zeros(a.shape[0], np.int64)
    d2 = np.zeros(a.shape[0], np.float32)
    if lib().chamfer_nn(a.shape[0], _p(a), b.shape[0], _p(b), _p(nn), _p(d2)) != 0:
        raise ValueError("bad input")
    return nn, d2


def chamfer(s1, s2):
    """(CD of Eq. 9, FP64; gradient with respect to s2 positions, FP64 [n2, 3])."""
    a = _f32(s1).reshape(-1, 3); b = _f32(s2).reshape(-1, 3)
    cd = np.zeros(1, np.float64)
    g = np.zeros((b.shape[0], 3), np.float64)
    if lib().chamfer_forward_backward(a.shape[0], _p(a), b.shape[0], _p(b), _p(cd), _p(g)) != 0:
        raise ValueError("bad input")
    return float(cd[0]), g


def topk_sh(s1, sh1, s2, K: int):
    """Mean SH of each s2 point's K nearest s1 points: (FP64 [n2, C, 3], indices [n2, K], -1 past |s1|)."""
    a = _f32(s1).reshape(-1, 3); b = _f32(s2).reshape(-1, 3)
    h = _f32(sh1)
    n2 = b.shape[0]
    out = np.zeros((n2,) + h.shape[1:], np.float64)
    idx = np.zeros((n2, K), np.int64)
    k3 = int(np.prod(h.shape[1:]))
    if lib().chamfer_topk_sh(a.shape[0], _p(a), _p(h), n2, _p(b), k3, int(K), _p(out), _p(idx)) != 0:
        raise ValueError("bad input")
    return out, idx


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step in FP64, in place on p, m, v (float64 arrays)."""
    for x in (p, g, m, v):
        if x.dtype != np.float64 or not x.flags.c_contiguous:
            raise ValueError("contiguous float64 arrays required")
    if lib().adam_step(p.size, _p(p), _p(g), _p(m), _p(v), int(t), float(lr), float(b1), float(b2),
                       float(eps)) != 0:
        raise ValueError("bad input")
