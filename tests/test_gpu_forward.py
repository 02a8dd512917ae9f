"""GPU forward parity: the HIP path (through the C ABI) against the FP64 oracle.

Image and transmittance must agree within 1e-4 max-abs per pixel; integer and
index work (depth keys, sort order, tile lists) must agree exactly.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import Camera, Scene

from _gpu_util import (IMG_TOL, compare_images, gpu_plan, oparams, random_pixels, to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14330_amd as d
    d.load()
    return d


def _scene_cam(seed, n=2000, size=(64, 48), deg=2, extent=1.0, f=None, radius=0.02):
    sc = workloads.small_scene(seed, n, sh_degree=deg, extent=extent, radius=radius)
    rng = np.random.default_rng(seed)
    W, H = size
    cam = workloads.random_sphere_camera(rng, W, H)
    if f is not None:
        cam = Camera(cam.R, cam.t, f, f, W / 2, H / 2, W, H)
    return sc, cam


def _render_check(dpr, scenes, views, params, label="", pixels_per_view=None):
    plan = gpu_plan(scenes, views, params)
    for v, (si, cam) in enumerate(views):
        pix = None
        if pixels_per_view is not None:
            pix = random_pixels(1000 + v, cam, pixels_per_view)
        ref = oracle.render(scenes[si], cam, oparams(params), pixels=pix)
        compare_images(to_np(plan.images[v]), to_np(plan.trans[v]), ref, pixels=pix, label=f"{label} view {v}")
    return plan


def test_cube4k_forward_parity(dpr):
    """4096 points, one 128x128 view at distance 3: full frame vs the oracle."""
    sc, cams = workloads.cube4k_128px()
    _render_check(dpr, [sc], [(0, cams[0])], dpr.RenderParams(), "cube4k")


@pytest.mark.parametrize("deg,frame", [(0, 0), (1, 1), (2, 0), (2, 1), (3, 0)])
def test_ragged_multiview_parity(dpr, deg, frame):
    """Three views of different, non-multiple-of-16 sizes in one launch."""
    sc = workloads.small_scene(30 + deg, 3000, sh_degree=deg)
    rng = np.random.default_rng(deg)
    views = [(0, workloads.random_sphere_camera(rng, w, h)) for w, h in [(37, 53), (64, 64), (17, 5)]]
    _render_check(dpr, [sc], views, dpr.RenderParams(sh_frame=frame), f"deg{deg} frame{frame}")


def test_multiscene_batch_parity(dpr):
    """Several scenes (different sizes, one empty) and views in one plan."""
    scenes = [workloads.small_scene(40, 1500), workloads.small_scene(41, 0), workloads.small_scene(42, 4100)]
    rng = np.random.default_rng(4)
    views = [(2, workloads.random_sphere_camera(rng, 48, 40)), (0, workloads.random_sphere_camera(rng, 33, 33)),
             (1, workloads.random_sphere_camera(rng, 20, 20)), (0, workloads.random_sphere_camera(rng, 70, 18))]
    plan = _render_check(dpr, scenes, views, dpr.RenderParams(), "multi")
    assert np.all(to_np(plan.images[2]) == 0) and np.all(to_np(plan.trans[2]) == 1)


def test_records_depth_keys_and_order(dpr):
    """Per-(view, point) records vs the oracle's per-point values; depth keys
    bitwise equal; the depth permutation exactly the oracle's (Z32, index) order."""
    torch = __import__("torch")
    sc, cam = _scene_cam(50, n=5000, size=(96, 80))
    rng = np.random.default_rng(5)
    cam2 = workloads.random_sphere_camera(rng, 40, 64)
    params = dpr.RenderParams()
    plan = gpu_plan([sc], [(0, cam), (0, cam2)], params)
    inf = plan.info()
    ws = plan.plan_ws
    M = inf.items
    rec = to_np(ws[inf.rec_off: inf.rec_off + 32 * M].view(torch.float32)).reshape(M, 8)
    skeys = to_np(ws[inf.key_off: inf.key_off + 4 * M].view(torch.int32)).view(np.uint32)
    order = to_np(ws[inf.order_off: inf.order_off + 4 * M].view(torch.int32)).view(np.uint32)
    rect = to_np(ws[inf.rect_off: inf.rect_off + 8 * M].view(torch.int32)).view(np.uint32).reshape(M, 2)
    keys = np.empty_like(skeys)
    keys[order] = skeys                  # key buffer is in sorted order, aligned with order[]
    assert np.array_equal(np.sort(order), np.arange(M, dtype=np.uint32))
    n = sc.n
    for v, c in enumerate([cam, cam2]):
        pr = oracle.project(sc, c, oparams(params))
        sl = slice(v * n, (v + 1) * n)
        r, k, rc = rec[sl], keys[sl], rect[sl]
        live = k != 0xFFFFFFFF
        nonempty = ((rc[:, 1] & 0xFFFF) > (rc[:, 0] & 0xFFFF)) & ((rc[:, 1] >> 16) > (rc[:, 0] >> 16))
        assert np.array_equal(live, nonempty)
        assert np.all(pr["valid"][live])
        # depth key: same float32 formula on both sides -> bitwise
        assert np.array_equal(k[live], pr["zkey"][live].view(np.uint32))
        np.testing.assert_allclose(r[live, 0], pr["px"][live], rtol=1e-5, atol=2e-3)
        np.testing.assert_allclose(r[live, 1], pr["py"][live], rtol=1e-5, atol=2e-3)
        a_ref = np.log2(np.e) / (2 * pr["sx"][live] ** 2)
        np.testing.assert_allclose(r[live, 2], a_ref, rtol=1e-5)
        np.testing.assert_allclose(r[live, 4], np.log2(sc.opacity[live].astype(np.float64)), rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(r[live, 5:8], pr["color"][live], atol=2e-5)
        # depth order of the view = oracle (zkey, index) order restricted to live items
        got = order[sl].astype(np.int64) - v * n
        ref = oracle.depth_order(sc, c, oparams(params))
        ref_live = ref[live[ref]]
        assert np.array_equal(got[: live.sum()], ref_live)
        assert set(got[live.sum():].tolist()) == set(np.nonzero(~live)[0].tolist())


def test_tile_lists_are_exact(dpr):
    """Each tile's list holds, in ascending (key, item) order, exactly the items
    whose tile rectangle covers the tile and whose ellipse can reach one of the
    tile's pixel centres (checked with a small margin on either side)."""
    torch = __import__("torch")
    sc, cam = _scene_cam(51, n=3000, size=(100, 70))
    params = dpr.RenderParams()
    plan = gpu_plan([sc], [(0, cam)], params)
    inf = plan.info()
    ws = plan.plan_ws
    M = inf.items
    skeys = to_np(ws[inf.key_off: inf.key_off + 4 * M].view(torch.int32)).view(np.uint32)
    order = to_np(ws[inf.order_off: inf.order_off + 4 * M].view(torch.int32)).view(np.uint32)
    keys = np.empty_like(skeys)
    keys[order] = skeys
    rect = to_np(ws[inf.rect_off: inf.rect_off + 8 * M].view(torch.int32)).view(np.uint32).reshape(M, 2)
    rec = to_np(ws[inf.rec_off: inf.rec_off + 32 * M].view(torch.float32)).reshape(M, 8).astype(np.float64)
    lam = -np.log2(params.alpha_min)
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
    rng_ = to_np(ws[inf.range_off: inf.range_off + 4 * (tx * ty + 1)].view(torch.int32)).view(np.uint32)
    pairs = to_np(plan.ws[inf.pairs_off: inf.pairs_off + 4 * inf.pairs].view(torch.int32)).view(np.uint32)
    assert rng_[-1] == inf.pairs
    cover = {t: [] for t in range(tx * ty)}
    for g in range(M):
        x0, y0 = rect[g, 0] & 0xFFFF, rect[g, 0] >> 16
        x1, y1 = rect[g, 1] & 0xFFFF, rect[g, 1] >> 16
        for yy in range(y0, y1):
            for xx in range(x0, x1):
                cover[yy * tx + xx].append((keys[g], g))

    def qmin(g, t):
        px, py, a, b, w = rec[g, :5]
        X0, Y0 = (t % tx) * 16 + 0.5, (t // tx) * 16 + 0.5
        cx, cy = min(max(px, X0), X0 + 15), min(max(py, Y0), Y0 + 15)
        return a * (cx - px) ** 2 + b * (cy - py) ** 2, w + lam

    dropped = 0
    for t in range(tx * ty):
        got = pairs[rng_[t]: rng_[t + 1]].tolist()
        full = [g for _, g in sorted(cover[t])]
        # order: a subsequence of the rect-covering list
        it = iter(full)
        assert all(g in it for g in got), t
        keep = set(got)
        for g in full:
            q, thr = qmin(g, t)
            if g in keep:
                assert q <= thr * (1 + 2e-3) + 1e-5, (t, g, q, thr)
            else:
                dropped += 1
                assert q > thr * (1 - 2e-3) - 1e-5, (t, g, q, thr)
    assert dropped > 0


def test_empty_and_culled_scenes(dpr):
    empty = workloads.small_scene(60, 0)
    cam = Camera(np.eye(3), [0, 0, 3], 50, 50, 20, 20, 40, 40)
    plan = gpu_plan([empty], [(0, cam)], dpr.RenderParams())
    assert np.all(to_np(plan.images[0]) == 0) and np.all(to_np(plan.trans[0]) == 1)
    behind = workloads.small_scene(61, 500)
    behind.xyz[:, 2] = behind.xyz[:, 2] * 0.1 - 4.0      # all at z_cam < 0
    plan = gpu_plan([behind], [(0, cam)], dpr.RenderParams())
    assert np.all(to_np(plan.images[0]) == 0) and np.all(to_np(plan.trans[0]) == 1)
    assert plan.info().pairs == 0


def test_one_pixel_and_thin_images(dpr):
    sc = workloads.small_scene(62, 800, extent=0.3)
    views = [(0, Camera(np.eye(3), [0, 0, 3], 300, 300, 0.5, 0.5, 1, 1)),
             (0, Camera(np.eye(3), [0, 0, 3], 300, 300, 100.0, 0.5, 200, 1)),
             (0, Camera(np.eye(3), [0, 0, 3], 300, 300, 0.5, 90.0, 1, 180))]
    _render_check(dpr, [sc], views, dpr.RenderParams(), "thin")


def test_equal_depth_ties_follow_index(dpr):
    """Duplicated points (identical depth keys) composite in index order."""
    base = workloads.small_scene(63, 300, extent=0.3)
    rng = np.random.default_rng(63)
    xyz = np.repeat(base.xyz, 3, axis=0)
    xyz[1::3, 0] += np.float32(0.004)                  # same depth, shifted sideways
    sh = base.sh[rng.integers(0, 300, 900)]
    op = np.clip(base.opacity[rng.integers(0, 300, 900)], 0.05, 0.95).astype(np.float32)
    sc = Scene(xyz.astype(np.float32), sh, op, np.full(900, 0.02, np.float32))
    cam = Camera(np.eye(3), [0, 0, 3], 300, 300, 32, 32, 64, 64)
    _render_check(dpr, [sc], [(0, cam)], dpr.RenderParams(), "ties")


def test_input_permutation_gives_bitwise_identical_image(dpr):
    sc, cam = _scene_cam(64, n=4000, size=(80, 80))
    zk = oracle.project(sc, cam)["zkey"]
    _, first = np.unique(zk, return_index=True)      # drop float32 depth collisions
    keep = np.sort(first)
    sc = Scene(sc.xyz[keep], sc.sh[keep], sc.opacity[keep], sc.radius[keep])
    perm = np.random.default_rng(64).permutation(sc.n)
    sp = Scene(sc.xyz[perm], sc.sh[perm], sc.opacity[perm], sc.radius[perm])
    p1 = gpu_plan([sc], [(0, cam)], dpr.RenderParams())
    p2 = gpu_plan([sp], [(0, cam)], dpr.RenderParams())
    assert np.array_equal(to_np(p1.images[0]), to_np(p2.images[0]))
    assert np.array_equal(to_np(p1.trans[0]), to_np(p2.trans[0]))


def test_view_alone_equals_view_in_batch_bitwise(dpr):
    s1 = workloads.small_scene(65, 3000)
    s2 = workloads.small_scene(66, 2000)
    rng = np.random.default_rng(65)
    c1 = workloads.random_sphere_camera(rng, 50, 40)
    c2 = workloads.random_sphere_camera(rng, 64, 64)
    alone = gpu_plan([s1], [(0, c1)], dpr.RenderParams())
    mix = gpu_plan([s2, s1], [(0, c2), (1, c1), (0, c1)], dpr.RenderParams())
    assert np.array_equal(to_np(alone.images[0]), to_np(mix.images[1]))
    assert np.array_equal(to_np(alone.trans[0]), to_np(mix.trans[1]))


def test_forward_is_deterministic_and_persistent_mode_matches(dpr):
    sc, cam = _scene_cam(67, n=6000, size=(128, 96))
    a = gpu_plan([sc], [(0, cam)], dpr.RenderParams())
    b = gpu_plan([sc], [(0, cam)], dpr.RenderParams())
    c = gpu_plan([sc], [(0, cam)], dpr.RenderParams(persistent=True))
    for p in (b, c):
        assert np.array_equal(to_np(a.images[0]), to_np(p.images[0]))
        assert np.array_equal(to_np(a.trans[0]), to_np(p.trans[0]))


def test_forward_variants_give_bitwise_identical_images(dpr):
    """The forward kernel is built with and without backward state (stored vs
    recompute mode) and with and without per-pixel counts, persistent or not;
    every variant renders the same bits.  In the second scene every seventh
    point has opacity 0.999 > alpha_max, so chunks holding one take the clamp
    path; that scene is also checked against the oracle."""
    sc, cam = _scene_cam(71, n=6000, size=(112, 80))
    op = sc.opacity.copy()
    op[::7] = np.float32(0.999)
    hot = Scene(sc.xyz, sc.sh, op, sc.radius)
    variants = (dict(bwd_mode="recompute"), dict(stats=True), dict(stats=True, bwd_mode="recompute"),
                dict(persistent=True, bwd_mode="recompute"), dict(persistent=True, stats=True))
    for scene in (sc, hot):
        ref = gpu_plan([scene], [(0, cam)], dpr.RenderParams())
        for kw in variants:
            p = gpu_plan([scene], [(0, cam)], dpr.RenderParams(**kw))
            assert np.array_equal(to_np(ref.images[0]), to_np(p.images[0])), kw
            assert np.array_equal(to_np(ref.trans[0]), to_np(p.trans[0])), kw
    plan = gpu_plan([hot], [(0, cam)], dpr.RenderParams())
    compare_images(to_np(plan.images[0]), to_np(plan.trans[0]), oracle.render(hot, cam, oparams(dpr.RenderParams())),
                   label="clamp-heavy")


def test_sh_linearity_on_gpu(dpr):
    sc, cam = _scene_cam(68, n=3000)
    s2 = Scene(sc.xyz, (sc.sh * np.float32(2.0)).astype(np.float32), sc.opacity, sc.radius)
    a = gpu_plan([sc], [(0, cam)], dpr.RenderParams())
    b = gpu_plan([s2], [(0, cam)], dpr.RenderParams())
    assert np.array_equal(to_np(a.trans[0]), to_np(b.trans[0]))
    np.testing.assert_allclose(to_np(b.images[0]), 2 * to_np(a.images[0]), rtol=1e-6, atol=1e-7)


def test_untruncated_thresholds(dpr):
    """alpha_min = t_min = 0, alpha_max = 1: the literal Eq. (6)-(7) sum."""
    sc, cam = _scene_cam(69, n=200, size=(40, 30), extent=0.4)
    p = dpr.RenderParams(alpha_min=0.0, t_min=0.0, alpha_max=1.0)
    plan = gpu_plan([sc], [(0, cam)], p)
    ref = oracle.render(sc, cam, oracle.Params.untruncated(), mode="brute")
    compare_images(to_np(plan.images[0]), to_np(plan.trans[0]), ref, label="untruncated")


def test_stats_count_blended_splats(dpr):
    torch = __import__("torch")
    sc, cam = _scene_cam(70, n=3000, size=(48, 48))
    plan = gpu_plan([sc], [(0, cam)], dpr.RenderParams(stats=True))
    inf = plan.info()
    st = to_np(plan.ws[inf.stats_off: inf.stats_off + 4 * inf.pixels].view(torch.int32)).reshape(48, 48)
    ref = oracle.render(sc, cam)
    # predicate/termination flips are allowed, but only rarely
    assert np.mean(st != ref.ncontrib) < 0.01
    assert abs(int(st.sum()) - int(ref.ncontrib.sum())) <= 0.001 * ref.ncontrib.sum() + 5


def test_blend_end_bounds_the_blends(dpr):
    """Stored-mode backward state: a pixel's blend end (one past the list
    position of the last splat it blended) is 0 exactly when it blended
    nothing, is at least its number of blended splats, and stays within its
    tile's list; also under the n = 3 cap."""
    torch = __import__("torch")
    W, H = 100, 70
    sc, cam = _scene_cam(72, n=5000, size=(W, H))
    for params in (dpr.RenderParams(stats=True), dpr.RenderParams(stats=True, max_splats=3)):
        plan = gpu_plan([sc], [(0, cam)], params)
        inf = plan.info()
        st = to_np(plan.ws[inf.stats_off: inf.stats_off + 4 * inf.pixels].view(torch.int32)).reshape(H, W)
        nl = to_np(plan.ws[inf.nlast_off: inf.nlast_off + 4 * inf.pixels].view(torch.int32)).reshape(H, W)
        tx, ty = (W + 15) // 16, (H + 15) // 16
        rng_ = to_np(plan.plan_ws[inf.range_off: inf.range_off + 4 * (tx * ty + 1)].view(torch.int32))
        tlen = np.diff(rng_.view(np.uint32).astype(np.int64))
        ys, xs = np.mgrid[0:H, 0:W]
        tl = tlen[(ys // 16) * tx + xs // 16]
        assert (st > 0).mean() > 0.3
        assert np.array_equal(st == 0, nl == 0)
        assert np.all(nl >= st)
        assert np.all(nl <= tl)
        if params.max_splats:
            assert st.max() == 3


def test_timing_of_selected_stages(dpr):
    """With timing_stages only the named stages report a time; the image is the
    same as without timing."""
    sc, cam = _scene_cam(71, n=3000, size=(48, 48))
    ref = gpu_plan([sc], [(0, cam)], dpr.RenderParams())
    for stages in (("composite_fwd",), ("depth_sort", "emit"), ()):
        plan = gpu_plan([sc], [(0, cam)], dpr.RenderParams(timing=True, timing_stages=stages))
        st = plan.stage_times()
        timed = {k for k, v in st.items() if v >= 0}
        expect = set(stages) if stages else {k for k in st if k not in ("composite_bwd", "recompute", "point_bwd")}
        assert timed == expect, (stages, st)
        assert np.array_equal(to_np(plan.images[0]), to_np(ref.images[0]))


def test_ball100k_forward_parity_sampled(dpr):
    """100k points, 8 views of 400x400: 2 full frames + 4096 pixels of every view."""
    sc, cams, _, _ = workloads.ball100k_8x400()
    views = [(0, c) for c in cams]
    plan = gpu_plan([sc], views, dpr.RenderParams())
    for v, (_, cam) in enumerate(views):
        pix = None if v < 2 else random_pixels(200 + v, cam, 4096)
        ref = oracle.render(sc, cam, pixels=pix)
        compare_images(to_np(plan.images[v]), to_np(plan.trans[v]), ref, pixels=pix, label=f"ball100k view {v}")


def test_render_forward_1_convenience(dpr):
    torch = __import__("torch")
    import ctypes
    from paper_2205_14330_amd import _abi
    sc, cam = _scene_cam(71, n=2500, size=(64, 40))
    st = dpr.SceneTensors.from_numpy(sc)
    img = torch.empty((40, 64, 3), device="cuda")
    tr = torch.empty((40, 64), device="cuda")
    lib = _abi.load()
    need = ctypes.c_size_t(0)
    params = dpr.RenderParams().to_c()
    c_sc = st.c_struct()
    c_cam = dpr.camera_struct(cam)
    rc = lib.dpr_render_forward_1(ctypes.byref(c_sc), ctypes.byref(c_cam), ctypes.byref(params),
                                  img.data_ptr(), tr.data_ptr(), None, 0, ctypes.byref(need), None)
    assert rc == 2
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    rc = lib.dpr_render_forward_1(ctypes.byref(c_sc), ctypes.byref(c_cam), ctypes.byref(params),
                                  img.data_ptr(), tr.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.byref(need), None)
    if rc == 2:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
        rc = lib.dpr_render_forward_1(ctypes.byref(c_sc), ctypes.byref(c_cam), ctypes.byref(params),
                                      img.data_ptr(), tr.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.byref(need),
                                      None)
    assert rc == 0, lib.dpr_last_error()
    torch.cuda.synchronize()
    ref = oracle.render(sc, cam)
    compare_images(to_np(img), to_np(tr), ref, label="forward_1")
