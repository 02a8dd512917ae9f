"""GPU backward parity: gradients from the HIP path (through the C ABI) against
the FP64 oracle's analytic gradients (themselves pinned to central finite
differences on the CPU).  Bar per element: |g - g*| <= 1e-3 max(|g*|, 1e-2 ||g*||_inf),
and rel-L2 <= 1e-3."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import Camera, Scene

from _gpu_util import compare_grads, compare_images, gpu_plan, oparams, random_pixels, scene_tensors, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14330_amd as d
    d.load()
    return d


def _weights(seed, cams, with_trans=True):
    rng = np.random.default_rng(seed)
    gI = [rng.standard_normal((c.height, c.width, 3)).astype(np.float32) for c in cams]
    gT = [rng.standard_normal((c.height, c.width)).astype(np.float32) for c in cams] if with_trans else None
    return gI, gT


def _gpu_grads(dpr, scenes, views, params, gI, gT):
    import torch
    plan = gpu_plan(scenes, views, params)
    gi = [torch.from_numpy(g).cuda() for g in gI]
    gt = None if gT is None else [torch.from_numpy(g).cuda() for g in gT]
    out = plan.backward(gi, gt)
    torch.cuda.synchronize()
    return plan, [(to_np(a), to_np(b), to_np(c)) for a, b, c in out]


def _check_scene(dpr, scene, cams, params, gI, gT, got, label, pixels=None):
    ref = oracle.backward(scene, cams, gI if pixels is None else [g.reshape(-1, 3)[p] for g, p in zip(gI, pixels)],
                          None if gT is None else (gT if pixels is None else [g.reshape(-1)[p] for g, p in zip(gT, pixels)]),
                          params=oparams(params), pixels=pixels)
    compare_grads(got[0], ref.xyz, f"{label} dxyz")
    compare_grads(got[1], ref.sh, f"{label} dsh")
    compare_grads(got[2], ref.opacity, f"{label} dopacity")
    return ref


@pytest.mark.parametrize("mode", ["stored", "recompute"])
@pytest.mark.parametrize("deg,frame", [(2, 0), (2, 1), (0, 0), (3, 0)])
def test_small_scene_gradients(dpr, mode, deg, frame):
    sc = workloads.small_scene(80 + deg, 1500, sh_degree=deg, extent=0.5)
    rng = np.random.default_rng(deg + 10 * frame)
    cams = [workloads.random_sphere_camera(rng, w, h) for w, h in [(48, 40), (35, 61)]]
    params = dpr.RenderParams(sh_frame=frame, bwd_mode=mode)
    gI, gT = _weights(deg, cams)
    plan, got = _gpu_grads(dpr, [sc], [(0, c) for c in cams], params, gI, gT)
    _check_scene(dpr, sc, cams, params, gI, gT, got[0], f"{mode} deg{deg} frame{frame}")


def test_image_only_loss_and_null_outputs(dpr):
    import torch
    sc = workloads.small_scene(90, 2000, extent=0.6)
    rng = np.random.default_rng(90)
    cams = [workloads.random_sphere_camera(rng, 40, 40)]
    params = dpr.RenderParams()
    gI, _ = _weights(90, cams, with_trans=False)
    plan = gpu_plan([sc], [(0, cams[0])], params)
    out = plan.backward([torch.from_numpy(gI[0]).cuda()], None, want=("sh",))
    torch.cuda.synchronize()
    assert out[0][0] is None and out[0][2] is None
    ref = oracle.backward(sc, cams, gI, None, params=oparams(params))
    compare_grads(to_np(out[0][1]), ref.sh, "dsh only")


def test_multiscene_gradients_sum_over_views(dpr):
    scenes = [workloads.small_scene(91, 1200, extent=0.6), workloads.small_scene(92, 800, extent=0.6)]
    rng = np.random.default_rng(91)
    cams = [workloads.random_sphere_camera(rng, 32, 32) for _ in range(4)]
    views = [(0, cams[0]), (1, cams[1]), (0, cams[2]), (1, cams[3])]
    params = dpr.RenderParams()
    gI, gT = _weights(91, cams)
    plan, got = _gpu_grads(dpr, scenes, views, params, gI, gT)
    _check_scene(dpr, scenes[0], [cams[0], cams[2]], params, [gI[0], gI[2]], [gT[0], gT[2]], got[0], "scene0")
    _check_scene(dpr, scenes[1], [cams[1], cams[3]], params, [gI[1], gI[3]], [gT[1], gT[3]], got[1], "scene1")


def test_stored_and_recompute_agree(dpr):
    sc = workloads.small_scene(93, 3000, extent=0.7)
    rng = np.random.default_rng(93)
    cams = [workloads.random_sphere_camera(rng, 64, 48) for _ in range(2)]
    gI, gT = _weights(93, cams)
    _, a = _gpu_grads(dpr, [sc], [(0, c) for c in cams], dpr.RenderParams(bwd_mode="stored"), gI, gT)
    _, b = _gpu_grads(dpr, [sc], [(0, c) for c in cams], dpr.RenderParams(bwd_mode="recompute"), gI, gT)
    for x, y in zip(a[0], b[0]):
        scale = np.abs(x).max()
        assert np.abs(x - y).max() <= 1e-5 * scale


def test_backward_twice_is_stable(dpr):
    import torch
    sc = workloads.small_scene(94, 2000, extent=0.6)
    rng = np.random.default_rng(94)
    cams = [workloads.random_sphere_camera(rng, 40, 40)]
    gI, gT = _weights(94, cams)
    plan = gpu_plan([sc], [(0, cams[0])], dpr.RenderParams())
    gi = [torch.from_numpy(gI[0]).cuda()]
    gt = [torch.from_numpy(gT[0]).cuda()]
    a = [to_np(t) for t in plan.backward(gi, gt)[0]]
    b = [to_np(t) for t in plan.backward(gi, gt)[0]]
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-5 * max(np.abs(x).max(), 1e-30)


def test_autograd_function_matches_oracle(dpr):
    import torch
    sc = workloads.small_scene(95, 1500, extent=0.5)
    rng = np.random.default_rng(95)
    cams = [workloads.random_sphere_camera(rng, 40, 40) for _ in range(3)]
    st = dpr.SceneTensors.from_numpy(sc)
    xyz = st.xyz.clone().requires_grad_(True)
    sh = st.sh.clone().requires_grad_(True)
    op = st.opacity.clone().requires_grad_(True)
    wrng = np.random.default_rng(96)
    w_img = wrng.standard_normal((3, 40, 40, 3)).astype(np.float32)
    w_tr = wrng.standard_normal((3, 40, 40)).astype(np.float32)
    wi, wt = torch.from_numpy(w_img).cuda(), torch.from_numpy(w_tr).cuda()
    for mode in ("stored", "recompute"):
        img, tr = dpr.render(xyz, sh, op, st.radius, cams, dpr.RenderParams(bwd_mode=mode))
        loss = (img * wi).sum() + (tr * wt).sum()      # linear: dL/dI = w_img, dL/dT = w_tr
        xyz.grad = sh.grad = op.grad = None
        loss.backward()
        torch.cuda.synchronize()
        for v in range(3):
            ref = oracle.render(sc, cams[v])
            compare_images(to_np(img[v]), to_np(tr[v]), ref, label=f"autograd fwd {v}")
        ref = oracle.backward(sc, cams, list(w_img), list(w_tr))
        compare_grads(to_np(xyz.grad), ref.xyz, f"{mode} autograd dxyz")
        compare_grads(to_np(sh.grad), ref.sh, f"{mode} autograd dsh")
        compare_grads(to_np(op.grad), ref.opacity, f"{mode} autograd dopacity")


def test_ball100k_gradients_restricted_pixels(dpr):
    """100k points, 8 views of 400x400, L2 loss against the seeded targets,
    restricted to 4096 random pixels per view (the oracle computes exactly the
    same loss); all gradients and the 256-point subset are checked."""
    import torch
    sc, cams, targets, subset = workloads.ball100k_8x400()
    views = [(0, c) for c in cams]
    params = dpr.RenderParams()
    plan = gpu_plan([sc], views, params)
    pix = [random_pixels(300 + v, c, 4096) for v, c in enumerate(cams)]
    # L2 loss gradient 2 (I - target) on the sampled pixels, from the oracle's image
    gI = []
    for v, c in enumerate(cams):
        ref_img = oracle.render(sc, c, oparams(params), pixels=pix[v]).image
        g = np.zeros((c.height * c.width, 3), np.float32)
        g[pix[v]] = (2.0 * (ref_img - targets[v].reshape(-1, 3)[pix[v]])).astype(np.float32)
        gI.append(g.reshape(c.height, c.width, 3))
    out = plan.backward([torch.from_numpy(g).cuda() for g in gI], None)
    torch.cuda.synchronize()
    got = [to_np(t) for t in out[0]]
    ref = oracle.backward(sc, cams, [g.reshape(-1, 3)[p] for g, p in zip(gI, pix)], None, params=oparams(params),
                          pixels=pix)
    compare_grads(got[0], ref.xyz, "ball100k dxyz")
    compare_grads(got[1], ref.sh, "ball100k dsh")
    compare_grads(got[2], ref.opacity, "ball100k dopacity")
    compare_grads(got[0][subset], ref.xyz[subset], "ball100k subset dxyz")
    compare_grads(got[1][subset], ref.sh[subset], "ball100k subset dsh")
    compare_grads(got[2][subset], ref.opacity[subset], "ball100k subset dopacity")


def test_workspace_reuse_matches_fresh_allocations(dpr):
    """Plans sharing one grown Workspace give the same images (bitwise) and
    gradients as plans with their own allocations, and the oracle's images;
    a plan whose Workspace went to a newer plan refuses to run."""
    import torch
    sc = workloads.small_scene(95, 3000, extent=0.7)
    st = scene_tensors(sc)
    rng = np.random.default_rng(95)
    sets = [[workloads.random_sphere_camera(rng, 24, 20)],
            [workloads.random_sphere_camera(rng, 70, 45), workloads.random_sphere_camera(rng, 33, 33)],
            [workloads.random_sphere_camera(rng, 16, 16)]]
    ws = dpr.Workspace("cuda", headroom=1.0)       # no headroom: the second set must grow it
    params = dpr.RenderParams()
    prev = None
    for k, cams in enumerate(sets):
        views = [(0, c) for c in cams]
        gI, gT = _weights(950 + k, cams)
        gi = [torch.from_numpy(g).cuda() for g in gI]
        gt = [torch.from_numpy(g).cuda() for g in gT]
        a = dpr.Plan([st], views, params, workspace=ws)
        if prev is not None:
            with pytest.raises(RuntimeError):
                prev.forward()
        a.forward()
        ga = [to_np(t) for t in a.backward(gi, gt)[0]]
        b = dpr.Plan([st], views, params)
        b.forward()
        gb = [to_np(t) for t in b.backward(gi, gt)[0]]
        for v, cam in enumerate(cams):
            assert np.array_equal(to_np(a.images[v]), to_np(b.images[v]))
            assert np.array_equal(to_np(a.trans[v]), to_np(b.trans[v]))
            ref = oracle.render(sc, cam, oparams(params))
            compare_images(to_np(a.images[v]), to_np(a.trans[v]), ref, label=f"set {k} view {v}")
        for x, y in zip(ga, gb):
            assert np.abs(x - y).max() <= 1e-5 * max(np.abs(x).max(), 1e-30)
        b.free()
        prev = a
    assert ws.reserved_bytes() > 0


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_clamped_alpha_gradients(dpr, mode):
    """Splats of opacity 0.999 centred on pixel centres: alpha is clamped to
    alpha_max there (the clamp passes no gradient to opacity or position),
    mixed with ordinary splats around them."""
    import torch
    base = workloads.small_scene(97, 1200, extent=0.5, radius=0.05)
    rng = np.random.default_rng(97)
    cam = workloads.random_sphere_camera(rng, 48, 40)
    m = 200
    u = rng.integers(0, cam.width, m) + 0.5
    v = rng.integers(0, cam.height, m) + 0.5
    Z = rng.uniform(2.6, 3.4, m)
    xc = np.stack([(u - cam.cx) * Z / cam.fx, (v - cam.cy) * Z / cam.fy, Z], 1)
    xw = (xc - np.asarray(cam.t, np.float64)) @ np.asarray(cam.R, np.float64)     # R^T (x_cam - t)
    sc = Scene(np.concatenate([base.xyz, xw.astype(np.float32)]),
               np.concatenate([base.sh, (0.3 * rng.standard_normal((m,) + base.sh.shape[1:])).astype(np.float32)]),
               np.concatenate([base.opacity, np.full(m, 0.999, np.float32)]),
               np.concatenate([base.radius, np.full(m, 0.05, np.float32)]))
    params = dpr.RenderParams(bwd_mode=mode)
    gI, gT = _weights(97, [cam])
    plan, got = _gpu_grads(dpr, [sc], [(0, cam)], params, gI, gT)
    ref = oracle.render(sc, cam, oparams(params))
    compare_images(to_np(plan.images[0]), to_np(plan.trans[0]), ref, label=f"clamped {mode}")
    _check_scene(dpr, sc, [cam], params, gI, gT, got[0], f"clamped {mode}")


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_long_lists_split_into_backward_segments(dpr, mode):
    """5000 faint, wide splats over a 40x40 view: tile lists of thousands of
    entries whose stop indices span several backward segments (256 list
    positions each), some pixels stopping inside a segment and some not
    stopping at all; full-frame gradients against the oracle."""
    import torch
    rng = np.random.default_rng(98)
    n = 5000
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz = (0.3 * d * rng.random(n)[:, None] ** (1.0 / 3.0)).astype(np.float32)
    sh = (0.3 * rng.standard_normal((n, 9, 3))).astype(np.float32)
    op = rng.uniform(0.005, 0.03, n).astype(np.float32)
    sc = Scene(xyz, sh, op, np.full(n, 0.15, np.float32))
    cams = [workloads.random_sphere_camera(rng, 40, 40), workloads.random_sphere_camera(rng, 21, 37)]
    params = dpr.RenderParams(bwd_mode=mode)
    gI, gT = _weights(98, cams)
    plan, got = _gpu_grads(dpr, [sc], [(0, c) for c in cams], params, gI, gT)
    if mode == "stored":
        inf = plan.info()
        nl = plan.ws[inf.nlast_off: inf.nlast_off + 4 * inf.pixels].view(torch.int32).cpu().numpy()
        assert nl.max() > 3 * 256 and nl.min() < nl.max()
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, oparams(params))
        compare_images(to_np(plan.images[v]), to_np(plan.trans[v]), ref, label=f"long lists {mode} view {v}")
    _check_scene(dpr, sc, cams, params, gI, gT, got[0], f"long lists {mode}")


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_backward_rejects_another_forward_workspace(dpr, mode):
    """The backward reads the tile lists (and, stored, the backward state) from
    the buffer this plan's forward wrote.  A different buffer of the same size
    is refused on the host, before any device work, with DPR_ERR_STATE; the
    right buffer still gives the oracle's gradients afterwards."""
    import torch
    from paper_2205_14330_amd import _abi
    sc = workloads.small_scene(96, 800, extent=0.6)
    rng = np.random.default_rng(96)
    cams = [workloads.random_sphere_camera(rng, 32, 24)]
    params = dpr.RenderParams(bwd_mode=mode)
    gI, gT = _weights(96, cams)
    plan = gpu_plan([sc], [(0, cams[0])], params)
    gi = [torch.from_numpy(gI[0]).cuda()]
    gt = [torch.from_numpy(gT[0]).cuda()]
    mine = plan.ws
    plan.ws = torch.zeros_like(mine)
    with pytest.raises(_abi.DprError) as err:
        plan.backward(gi, gt)
    assert err.value.code == _abi.DPR_ERR_STATE
    plan.ws = mine
    out = plan.backward(gi, gt)
    torch.cuda.synchronize()
    _check_scene(dpr, sc, cams, params, gI, gT, [to_np(t) for t in out[0]], f"{mode} after refusal")


def _sparse_hit_scene():
    """One 16x16 tile whose list is long but whose walked range holds few blended
    records: ten wide opaque splats in front (centred at pixel (12, 12)) stop
    every pixel that the 3900 narrow splats behind them reach, and 26 faint
    narrow splats at the corner pixel, one every 150 list positions, keep the
    corner pixels live deep into the list.  The backward then walks thousands
    of positions in which most 64-record chunks hold no blended record, so a
    segment's staged sums span several chunks (and are flushed before the item
    ids of a chunk two back are overwritten)."""
    W = H = 32
    f = 32.0
    cam = Camera(np.eye(3), np.zeros(3), f, f, W / 2.0, H / 2.0, W, H)
    rng = np.random.default_rng(7)
    pts = []          # (u, v, z, sigma_px, opacity)
    for k in range(10):
        pts.append((12.0, 12.0, 1.90 + 0.001 * k, 3.3, 0.99))
    for k in range(3900):
        pts.append((12.0 + rng.uniform(-0.5, 0.5), 12.0 + rng.uniform(-0.5, 0.5), 2.0 + 0.0005 * k, 0.5, 0.5))
    for j in range(26):
        pts.append((0.5, 0.5, 2.0 + 0.0005 * (150 * j + 75) + 0.0001, 0.6, 0.7))
    p = np.array(pts, np.float64)
    u, v, z, s, o = p.T
    xyz = np.stack([(u - W / 2.0) * z / f, (v - H / 2.0) * z / f, z], 1).astype(np.float32)
    sc = Scene(xyz, (0.3 * rng.standard_normal((len(p), 1, 3))).astype(np.float32), o.astype(np.float32),
               (s * z / f).astype(np.float32))
    return sc, cam


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_sparse_hits_over_long_lists(dpr, mode):
    sc, cam = _sparse_hit_scene()
    params = dpr.RenderParams(bwd_mode=mode)
    ref_img = oracle.render(sc, cam, oparams(params))
    # the scene is what it claims: the corner pixel blends its faint splats and
    # stops deep in the list, the centre stops within the wide front splats
    assert ref_img.stopped[0, 0] and 5 <= ref_img.ncontrib[0, 0] <= 26
    assert ref_img.stopped[12, 12] and ref_img.ncontrib[12, 12] <= 10
    gI, gT = _weights(11, [cam])
    plan, got = _gpu_grads(dpr, [sc], [(0, cam)], params, gI, gT)
    compare_images(to_np(plan.images[0]), to_np(plan.trans[0]), ref_img, label=f"sparse {mode}")
    _check_scene(dpr, sc, [cam], params, gI, gT, got[0], f"sparse {mode}")
