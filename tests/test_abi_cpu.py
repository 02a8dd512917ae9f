"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, the ctypes structs match the C layout,
and invalid arguments are rejected before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpr.h")


@pytest.fixture(scope="module")
def abi():
    from paper_2205_14330_amd import _abi
    _abi.load()
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpr_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_are_exported(abi):
    names = declared_functions()
    assert len(names) >= 10
    lib = abi.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "dpr.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("dpr_camera %zu\ndpr_scene %zu\ndpr_view %zu\ndpr_params %zu\ndpr_plan_info %zu\n",
         sizeof(dpr_camera), sizeof(dpr_scene), sizeof(dpr_view), sizeof(dpr_params), sizeof(dpr_plan_info));
  P(dpr_view, cam); P(dpr_view, image); P(dpr_view, trans);
  P(dpr_scene, xyz); P(dpr_scene, radius);
  P(dpr_params, flags);
  P(dpr_plan_info, stats_off); P(dpr_plan_info, chunk_items);
  P(dpr_camera, width);
  return 0;
}
"""


def test_struct_layout_matches_c(abi, tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", str(src), "-o", str(exe)], check=True)
    lines = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    C = {k: int(v) for k, v in lines.items()}
    assert C["dpr_camera"] == ctypes.sizeof(abi.Camera)
    assert C["dpr_scene"] == ctypes.sizeof(abi.Scene)
    assert C["dpr_view"] == ctypes.sizeof(abi.View)
    assert C["dpr_params"] == ctypes.sizeof(abi.Params)
    assert C["dpr_plan_info"] == ctypes.sizeof(abi.PlanInfo)
    assert C["dpr_view.cam"] == abi.View.cam.offset
    assert C["dpr_view.image"] == abi.View.image.offset
    assert C["dpr_view.trans"] == abi.View.trans.offset
    assert C["dpr_scene.xyz"] == abi.Scene.xyz.offset
    assert C["dpr_scene.radius"] == abi.Scene.radius.offset
    assert C["dpr_params.flags"] == abi.Params.flags.offset
    assert C["dpr_plan_info.stats_off"] == abi.PlanInfo.stats_off.offset
    assert C["dpr_plan_info.chunk_items"] == abi.PlanInfo.chunk_items.offset
    assert C["dpr_camera.width"] == abi.Camera.width.offset


FAKE = 0x7F0000000000      # never dereferenced: every call below fails validation first


def _scene(abi, n=100, deg=2):
    return abi.Scene(n, deg, 0, FAKE, FAKE, FAKE, FAKE)


def _view(abi, scene=0, w=64, h=48, image=FAKE, trans=FAKE, fx=50.0):
    cam = abi.Camera()
    cam.R[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    cam.t[:] = [0, 0, 3]
    cam.fx = cam.fy = fx
    cam.cx, cam.cy = w / 2, h / 2
    cam.width, cam.height = w, h
    return abi.View(scene, 0, cam, image, trans)


def _params(abi, **kw):
    p = abi.Params(1e-5, 1e-5, 0.99, 0.01, 0, 0, 0, 0, 0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _plan(abi, scenes, views, params, ws=FAKE, ws_bytes=1 << 40):
    lib = abi.load()
    S = (abi.Scene * len(scenes))(*scenes)
    V = (abi.View * len(views))(*views)
    out = ctypes.c_void_p()
    rc = lib.dpr_plan_forward(S, len(scenes), V, len(views), ctypes.byref(params), ws, ws_bytes, None,
                              ctypes.byref(out))
    return rc, lib.dpr_last_error().decode(), out


@pytest.mark.parametrize("case,expect", [
    ("alpha_min", 1), ("t_min", 1), ("alpha_max", 1), ("z_near", 1), ("sh_frame", 1), ("bwd_mode", 1),
    ("flags", 1), ("max_splats", 1), ("timing_stages", 1), ("scene_index", 1), ("width", 1), ("height", 1), ("fx", 1),
    ("null_image", 1), ("sh_degree", 1), ("neg_n", 1), ("null_xyz", 1), ("mixed_degree", 4),
    ("no_views", 1), ("workspace", 2), ("null_ws", 2),
])
def test_invalid_arguments_rejected(abi, case, expect):
    scenes = [_scene(abi)]
    views = [_view(abi)]
    params = _params(abi)
    ws_bytes = 1 << 40
    ws = FAKE
    n_views_override = None
    if case == "alpha_min":
        params.alpha_min = 1.5
    elif case == "t_min":
        params.t_min = -0.1
    elif case == "alpha_max":
        params.alpha_max = 0.0
    elif case == "z_near":
        params.z_near = 0.0
    elif case == "sh_frame":
        params.sh_frame = 2
    elif case == "bwd_mode":
        params.bwd_mode = 7
    elif case == "flags":
        params.flags = 64
    elif case == "max_splats":
        params.max_splats = -1
    elif case == "timing_stages":
        params.flags = 1
        params.timing_stages = 1 << 12
    elif case == "scene_index":
        views = [_view(abi, scene=1)]
    elif case == "width":
        views = [_view(abi, w=0)]
    elif case == "height":
        views = [_view(abi, h=20000)]
    elif case == "fx":
        views = [_view(abi, fx=-1.0)]
    elif case == "null_image":
        views = [_view(abi, image=0)]
    elif case == "sh_degree":
        scenes = [_scene(abi, deg=4)]
    elif case == "neg_n":
        scenes = [_scene(abi, n=-5)]
    elif case == "null_xyz":
        scenes = [abi.Scene(10, 2, 0, 0, FAKE, FAKE, FAKE)]
    elif case == "mixed_degree":
        scenes = [_scene(abi), _scene(abi, deg=1)]
    elif case == "no_views":
        views = []
    elif case == "workspace":
        ws_bytes = 16
    elif case == "null_ws":
        ws = None
    if case == "no_views":
        lib = abi.load()
        S = (abi.Scene * 1)(*scenes)
        out = ctypes.c_void_p()
        rc = lib.dpr_plan_forward(S, 1, None, 0, ctypes.byref(params), FAKE, 1 << 40, None, ctypes.byref(out))
        msg = lib.dpr_last_error().decode()
    else:
        rc, msg, out = _plan(abi, scenes, views, params, ws, ws_bytes)
    assert rc == expect, (case, rc, msg)
    assert msg
    assert not out.value


@pytest.mark.parametrize("case", ["null_rendered", "null_fwd_ws", "bad_params"])
def test_plan_forward_render_rejects_before_device_work(abi, case):
    """The argument checks of dpr_plan_forward_render run on the host, before
    any device call (the fake workspace pointers are never touched)."""
    lib = abi.load()
    S = (abi.Scene * 1)(_scene(abi))
    V = (abi.View * 1)(_view(abi))
    params = _params(abi, alpha_min=1.5) if case == "bad_params" else _params(abi)
    out = ctypes.c_void_p()
    done = ctypes.c_int32(5)
    fwd = None if case == "null_fwd_ws" else FAKE
    rendered = None if case == "null_rendered" else ctypes.byref(done)
    rc = lib.dpr_plan_forward_render(S, 1, V, 1, ctypes.byref(params), FAKE, 1 << 40, fwd, 1 << 40, None,
                                     ctypes.byref(out), rendered)
    assert rc == 1 and lib.dpr_last_error().decode() and not out.value
    if case == "bad_params":
        assert done.value == 0


def test_plan_ws_bytes_host_only(abi):
    lib = abi.load()
    S = (abi.Scene * 1)(_scene(abi, n=5000))
    V1 = (abi.View * 1)(_view(abi))
    V2 = (abi.View * 2)(_view(abi), _view(abi, w=128, h=128))
    b1 = lib.dpr_plan_ws_bytes(S, 1, V1, 1)
    b2 = lib.dpr_plan_ws_bytes(S, 1, V2, 2)
    assert b1 > 5000 * 32 and b2 > b1 and b1 % 256 == 0
    bad = (abi.View * 1)(_view(abi, scene=3))
    assert lib.dpr_plan_ws_bytes(S, 1, bad, 1) == 0
    assert "scene" in lib.dpr_last_error().decode()


def test_injected_launch_failure(abi, monkeypatch):
    monkeypatch.setenv("DPR_FAULT", "launch")
    rc, msg, out = _plan(abi, [_scene(abi)], [_view(abi)], _params(abi))
    assert rc == 3 and "injected" in msg and not out.value


def test_null_plan_calls(abi):
    lib = abi.load()
    assert lib.dpr_workspace_bytes(None) == 0
    assert lib.dpr_backward_ws_bytes(None) == 0
    lib.dpr_plan_free(None)
    assert lib.dpr_render_forward(None, FAKE, 100, None) == 1
    info = abi.PlanInfo()
    assert lib.dpr_plan_get_info(None, ctypes.byref(info)) == 1
    assert lib.dpr_version() == 2


def test_forward_1_query_size_without_workspace(abi):
    lib = abi.load()
    sc = _scene(abi, n=1000)
    cam = _view(abi).cam
    need = ctypes.c_size_t(0)
    rc = lib.dpr_render_forward_1(ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(_params(abi)), FAKE, FAKE,
                                  None, 0, ctypes.byref(need), None)
    assert rc == 2 and need.value > 1000 * 32


def test_oracle_shares_no_code_with_hip_path():
    """The oracle and the HIP library include nothing from each other."""
    osrc = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert "dpr.h" not in osrc and "csrc" not in osrc and "paper_2205_14330_amd" not in osrc
    opy = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert "paper_2205_14330_amd" not in opy
    pkg = os.path.join(ROOT, "paper_2205_14330_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.c" not in text, f


def test_loss_workspace_sizes(abi):
    lib = abi.load()
    I = ctypes.c_int32
    W, H = (I * 2)(800, 17), (I * 2)(600, 1)
    n = lib.dpr_loss_ws_bytes(2, W, H)
    assert n >= 32 * 2 + 4 * 3 + 4 * ((800 * 600 + 1023) // 1024 + 1)
    assert lib.dpr_loss_ws_bytes(0, W, H) == 0
    assert lib.dpr_loss_ws_bytes(1, (I * 1)(0), (I * 1)(5)) == 0
    assert lib.dpr_loss_ws_bytes(1, (I * 1)(20000), (I * 1)(5)) == 0


@pytest.mark.parametrize("case,expect", [("null_render", 1), ("alias", 1), ("lambda", 1), ("nan_lambda", 1),
                                         ("workspace", 2), ("null_loss", 1), ("size", 1)])
def test_loss_invalid_arguments_rejected(abi, case, expect):
    """Every check runs on the host before anything is launched."""
    lib = abi.load()
    I = ctypes.c_int32
    W, H = (I * 1)(8), (I * 1)(4)
    r, t, g = FAKE, FAKE + 4096, FAKE + 8192
    lam, loss, ws, nb = 0.01, FAKE + 12288, FAKE + 16384, 1 << 20
    if case == "null_render":
        r = None
    elif case == "alias":
        g = r
    elif case == "lambda":
        lam = -1.0
    elif case == "nan_lambda":
        lam = float("nan")
    elif case == "workspace":
        nb = 8
    elif case == "null_loss":
        loss = None
    elif case == "size":
        W = (I * 1)(0)
    P = abi.ptr_array
    rc = lib.dpr_loss_l2_tv(1, P([r or 0]), P([t]), W, H, lam, P([g]), loss, ws, nb, None)
    assert rc == expect, lib.dpr_last_error().decode()
    assert lib.dpr_last_error().decode()


def test_hull_workspace_sizes(abi):
    lib = abi.load()
    cam = abi.Camera()
    cam.width, cam.height = 800, 600
    cams = (abi.Camera * 16)(*([cam] * 16))
    assert lib.dpr_hull_ws_bytes(0, 1, cams) > 0
    # camera table, masks packed to bits, one bitmask word per 32 items
    assert lib.dpr_hull_ws_bytes(5000, 16, cams) >= 96 * 16 + 16 * 800 * 600 // 8 + 4 * 32 * 5
    assert lib.dpr_hull_ws_bytes(-1, 1, cams) == 0
    assert lib.dpr_hull_ws_bytes(10, 0, cams) == 0
    assert lib.dpr_hull_ws_bytes(10, 5000, cams) == 0
    assert lib.dpr_hull_ws_bytes(10, 1, None) == 0
    cam.width = 0
    assert lib.dpr_hull_ws_bytes(10, 1, (abi.Camera * 1)(cam)) == 0


@pytest.mark.parametrize("case,expect", [("n_cams", 1), ("mask_size", 1), ("null_mask", 1), ("box", 1), ("nan_box", 1),
                                         ("capacity", 1), ("null_out", 1), ("workspace", 2), ("camera", 1),
                                         ("n", 1)])
def test_hull_invalid_arguments_rejected(abi, case, expect):
    """Every check of the consistency-check entry points runs on the host
    before anything is launched."""
    lib = abi.load()
    cam = abi.Camera()
    cam.R[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    cam.t[:] = [0, 0, 3]
    cam.fx = cam.fy = 50.0
    cam.cx = cam.cy = 16.0
    cam.width = cam.height = 32
    cams = (abi.Camera * 2)(cam, cam)
    masks = (abi.Mask * 2)(abi.Mask(FAKE, 32, 32), abi.Mask(FAKE + 4096, 32, 32))
    lo = (ctypes.c_float * 3)(-1, -1, -1)
    hi = (ctypes.c_float * 3)(1, 1, 1)
    n_cams, n, cap, out, ws, nb = 2, 100, 100, FAKE + 8192, FAKE + 16384, 1 << 30
    if case == "n_cams":
        n_cams = 0
    elif case == "mask_size":
        masks[1].width = 31
    elif case == "null_mask":
        masks[0].data = None
    elif case == "box":
        hi[1] = -1.0
    elif case == "nan_box":
        lo[2] = float("nan")
    elif case == "capacity":
        cap = -1
    elif case == "null_out":
        out = None
    elif case == "workspace":
        nb = 64
    elif case == "camera":
        cams[1].fx = 0.0
    elif case == "n":
        n = -5
    cnt = ctypes.c_int64(0)
    rc = lib.dpr_hull_sample(n_cams, cams, masks, lo, hi, 1, n, out, cap, ctypes.byref(cnt), ws, nb, None)
    assert rc == expect, lib.dpr_last_error()
    assert lib.dpr_last_error()
    if case in ("n_cams", "mask_size", "null_mask", "workspace", "camera"):
        keep = FAKE + 32768
        rc2 = lib.dpr_consistency(100, FAKE, n_cams, cams, masks, keep, ws, nb, None)
        assert rc2 == expect


@pytest.mark.parametrize("case", ["n1", "n2", "null_s1", "workspace", "topk_K", "topk_deg", "topk_null",
                                  "adam_t", "adam_beta", "adam_eps", "adam_null"])
def test_warm_start_invalid_arguments_rejected(abi, case):
    """Every check of the warm-start entry points runs on the host before
    anything is launched."""
    lib = abi.load()
    s1, s2, ws = FAKE, FAKE + 65536, FAKE + 131072
    if case in ("n1", "n2", "null_s1", "workspace"):
        n1, n2, nb = 100, 80, 1 << 30
        if case == "n1":
            n1 = 0
        elif case == "n2":
            n2 = -3
        elif case == "null_s1":
            s1 = None
        else:
            nb = 16
        rc = lib.dpr_chamfer(n1, s1, n2, s2, None, None, None, None, ws, nb, None)
        assert rc == (2 if case == "workspace" else 1), lib.dpr_last_error()
    elif case.startswith("topk"):
        K, deg, out = 4, 2, FAKE + 262144
        if case == "topk_K":
            K = 33
        elif case == "topk_deg":
            deg = 4
        else:
            out = None
        assert lib.dpr_topk_sh(100, s1, FAKE + 8192, 80, s2, deg, K, out, None, None) == 1
    else:
        t, b1, eps, p = 1, 0.9, 1e-8, FAKE
        if case == "adam_t":
            t = 0
        elif case == "adam_beta":
            b1 = 1.0
        elif case == "adam_eps":
            eps = 0.0
        else:
            p = None
        assert lib.dpr_adam_step(10, p, FAKE, FAKE, FAKE, t, 1e-3, b1, 0.999, eps, None) == 1
    assert lib.dpr_last_error()


def test_chamfer_workspace_sizes(abi):
    lib = abi.load()
    assert lib.dpr_chamfer_ws_bytes(1000, 2000) >= 8 * 3000 + 24 * 2000 + 4 * 2000
    assert lib.dpr_chamfer_ws_bytes(0, 5) == 0 and lib.dpr_chamfer_ws_bytes(5, 0) == 0
