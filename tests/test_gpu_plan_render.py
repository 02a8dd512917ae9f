"""dpr_plan_forward_render: the plan stage and the forward in one call, the
forward queued before the wait for the pair count into a workspace laid out
for as many pairs as it can hold.

* With a large enough workspace the images and transmittance are those of
  dpr_plan_forward + dpr_render_forward bit for bit, they pass the oracle
  parity, and the backward that follows gives the same gradients (up to the
  order of its float atomics), in both backward modes.
* With a workspace too small for the pair lists, nothing is rendered (the
  images keep a sentinel: the kernels read the pair count on the device and do
  nothing), the plan reports it, and the ordinary forward then gives the same
  images.
"""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_util import compare_images, oparams, scene_tensors, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14330_amd as d
    d.load()
    return d


def _case(seed, n=20000, size=(160, 120), views=3):
    sc = workloads.small_scene(seed, n, sh_degree=2, radius=0.02)
    rng = np.random.default_rng(seed)
    cams = [workloads.random_sphere_camera(rng, *size) for _ in range(views)]
    return sc, cams


def _two_calls(dpr, st, cams, params):
    p = dpr.Plan([st], [(0, c) for c in cams], params)
    p.forward()
    return p


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_plan_render_equals_plan_then_forward(dpr, mode):
    import torch
    sc, cams = _case(71)
    st = scene_tensors(sc)
    params = dpr.RenderParams(bwd_mode=mode)
    ref = _two_calls(dpr, st, cams, params)
    ws = dpr.Workspace()
    ws.bufs["fwd"] = torch.empty(int(ref.ws.numel()) * 2, dtype=torch.uint8, device="cuda")
    p = dpr.Plan([st], [(0, c) for c in cams], params, workspace=ws, forward_now=True)
    assert p._rendered, "the workspace holds the lists: the forward must run with the plan"
    p.forward()
    torch.cuda.synchronize()
    for a, b in zip(p.images + p.trans, ref.images + ref.trans):
        assert torch.equal(a, b)
    assert p.info().pairs == ref.info().pairs
    for v, cam in enumerate(cams):
        r = oracle.render(sc, cam, oparams(params))
        compare_images(to_np(p.images[v]), to_np(p.trans[v]), r, label=f"view {v}")
    # the gradients are sums of float atomics, whose order varies from run to
    # run: equal up to that rounding
    w = [torch.randn_like(i) for i in p.images]
    g1 = p.backward(w, None)
    g0 = ref.backward(w, None)
    torch.cuda.synchronize()
    for a, b in zip(g1[0], g0[0]):
        assert float((a - b).abs().max()) <= 1e-5 * float(b.abs().max())


def test_plan_render_with_a_small_workspace_renders_nothing_then_forward_works(dpr):
    import torch
    sc, cams = _case(72)
    st = scene_tensors(sc)
    # recompute mode: the forward workspace is the pair lists and a few words,
    # so half its size holds about half the pairs and the forward is queued
    # (and must find that the lists do not fit)
    params = dpr.RenderParams(bwd_mode="recompute")
    ref = _two_calls(dpr, st, cams, params)
    sentinel = -12345.0
    images = [torch.full((c.height, c.width, 3), sentinel, device="cuda") for c in cams]
    trans = [torch.full((c.height, c.width), sentinel, device="cuda") for c in cams]
    ws = dpr.Workspace()
    ws.bufs["fwd"] = torch.empty(int(ref.ws.numel()) // 2, dtype=torch.uint8, device="cuda")
    p = dpr.Plan([st], [(0, c) for c in cams], params, images=images, trans=trans)
    p.free()
    lib = dpr._abi.load()
    import ctypes
    done = ctypes.c_int32(7)
    plan = ctypes.c_void_p()
    nbytes = lib.dpr_plan_ws_bytes(p._c_scenes, 1, p._c_views, len(cams))
    pws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    fwd = ws.bufs["fwd"]
    rc = lib.dpr_plan_forward_render(p._c_scenes, 1, p._c_views, len(cams), ctypes.byref(p._c_params),
                                     pws.data_ptr(), int(nbytes), fwd.data_ptr(), int(fwd.numel()), None,
                                     ctypes.byref(plan), ctypes.byref(done))
    assert rc == 0, lib.dpr_last_error()
    torch.cuda.synchronize()
    assert done.value == 0
    for t in images + trans:
        assert bool((t == sentinel).all()), "a forward that did not fit wrote to the outputs"
    need = int(lib.dpr_workspace_bytes(plan))
    assert need > int(fwd.numel())
    big = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert lib.dpr_render_forward(plan, big.data_ptr(), need, None) == 0
    torch.cuda.synchronize()
    for a, b in zip(images + trans, ref.images + ref.trans):
        assert torch.equal(a, b)
    lib.dpr_plan_free(plan)
