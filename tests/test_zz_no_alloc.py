"""dpr_render_forward_1_noalloc (workspace in a static device array) against
dpr_render_forward_1 (workspace from the caller), both through the C ABI: two
calls in a row, the second on a smaller scene and image, each within the
image/transmittance bar of 1e-4 max-abs of the allocating entry point (the
same kernels run, so the results are expected to be bitwise equal); the
smaller call is also checked against the oracle, and an input too large for
the scratch is refused with DPR_ERR_WORKSPACE."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_14330_amd import _abi, renderer
    return torch, _abi, renderer, _abi.load()


def _inputs(torch, _abi, renderer, scene, cam):
    st = renderer.SceneTensors.from_numpy(scene, "cuda")
    c_scene = st.c_struct()
    c_cam = renderer.camera_struct(cam)
    params = renderer.RenderParams().to_c()
    return st, c_scene, c_cam, params


def _noalloc(torch, lib, c_scene, c_cam, params, cam):
    img = torch.full((cam.height, cam.width, 3), float("nan"), device="cuda")
    tr = torch.full((cam.height, cam.width), float("nan"), device="cuda")
    torch.cuda.synchronize()
    rc = lib.dpr_render_forward_1_noalloc(ctypes.byref(c_scene), ctypes.byref(c_cam), ctypes.byref(params),
                                          img.data_ptr(), tr.data_ptr(), None)
    torch.cuda.synchronize()
    return rc, img, tr


def _forward_1(torch, lib, c_scene, c_cam, params, cam):
    img = torch.empty((cam.height, cam.width, 3), device="cuda")
    tr = torch.empty((cam.height, cam.width), device="cuda")
    need = ctypes.c_size_t(0)
    rc = lib.dpr_render_forward_1(ctypes.byref(c_scene), ctypes.byref(c_cam), ctypes.byref(params),
                                  img.data_ptr(), tr.data_ptr(), None, 0, ctypes.byref(need), None)
    assert rc == 2 and need.value > 0
    for _ in range(2):      # the first query covers the plan workspace only
        ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
        rc = lib.dpr_render_forward_1(ctypes.byref(c_scene), ctypes.byref(c_cam), ctypes.byref(params),
                                      img.data_ptr(), tr.data_ptr(), ws.data_ptr(), ws.numel(),
                                      ctypes.byref(need), None)
        if rc == 0:
            break
    assert rc == 0
    torch.cuda.synchronize()
    return img, tr


def test_noalloc_matches_forward_1_on_two_calls(env):
    torch, _abi, renderer, lib = env
    cases = [(61, 40000, 1.0, 320, 240), (62, 3000, 0.5, 96, 64)]
    for k, (seed, n, extent, w, h) in enumerate(cases):
        print(f"noalloc call {k}: seed {seed}, {n} points, {w}x{h}", flush=True)
        scene = workloads.small_scene(seed, n, extent=extent)
        cam = workloads.random_sphere_camera(np.random.default_rng(seed), w, h)
        st, c_scene, c_cam, params = _inputs(torch, _abi, renderer, scene, cam)
        rc, img, tr = _noalloc(torch, lib, c_scene, c_cam, params, cam)
        assert rc == 0, lib.dpr_last_error().decode()
        ref_img, ref_tr = _forward_1(torch, lib, c_scene, c_cam, params, cam)
        ei = (img - ref_img).abs().max().item()
        et = (tr - ref_tr).abs().max().item()
        assert ei <= TOL and et <= TOL, (k, ei, et)
        print(f"  vs dpr_render_forward_1: image {ei:.3e}, trans {et:.3e}, bitwise "
              f"{bool(torch.equal(img, ref_img) and torch.equal(tr, ref_tr))}", flush=True)
        if k == 1:
            o = oracle.render(scene, cam)
            assert np.abs(img.cpu().numpy() - o.image).max() <= TOL
            assert np.abs(tr.cpu().numpy() - o.trans).max() <= TOL


def test_noalloc_refuses_inputs_beyond_the_scratch(env):
    torch, _abi, renderer, lib = env
    n = 1_500_000                    # plan workspace alone ~ 84 MB > 64 MiB
    rng = np.random.default_rng(63)
    scene = workloads.Scene(rng.uniform(-1, 1, (n, 3)).astype(np.float32),
                            (0.3 * rng.standard_normal((n, 1, 3))).astype(np.float32),
                            np.full(n, 0.5, np.float32), np.full(n, 0.02, np.float32))
    cam = workloads.random_sphere_camera(rng, 64, 64)
    st, c_scene, c_cam, params = _inputs(torch, _abi, renderer, scene, cam)
    rc, _, _ = _noalloc(torch, lib, c_scene, c_cam, params, cam)
    assert rc == _abi.DPR_ERR_WORKSPACE
    msg = lib.dpr_last_error().decode()
    assert "static scratch" in msg and str(64 << 20) in msg
    # a later small call still works
    scene = workloads.small_scene(64, 2000, extent=0.5)
    cam = workloads.random_sphere_camera(np.random.default_rng(64), 48, 40)
    st, c_scene, c_cam, params = _inputs(torch, _abi, renderer, scene, cam)
    rc, img, tr = _noalloc(torch, lib, c_scene, c_cam, params, cam)
    assert rc == 0
    o = oracle.render(scene, cam)
    assert np.abs(img.cpu().numpy() - o.image).max() <= TOL
