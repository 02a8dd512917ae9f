"""GPU parity at the benchmark workload: 300k points (30% on a 20-bump
surface), SH degree 2, the four 800x800 views of the first training step, in
both backward modes.  Image and transmittance of view 0 in full and of 4096
seeded pixels of each other view (max-abs 1e-4); gradients of the linear loss
sum(w I) with seeded N(0, 1) weights restricted to those same pixels (the
oracle evaluates exactly that loss) for every point's position, SH and
opacity.  Also reported: how many list positions the float32 depth key orders
differently from camera Z in float64 (near-ties, which the oracle orders by
the same key)."""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_util import compare_grads, compare_images, gpu_plan, oparams, random_pixels, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14330_amd as d
    d.load()
    return d


@pytest.fixture(scope="module")
def headline():
    scene, cams, _ = workloads.surface300k_4x800()
    cams = cams[:4]
    pix = [None] + [random_pixels(500 + v, c, 4096) for v, c in enumerate(cams) if v > 0]
    rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(3, 3)))
    w = []
    for v, c in enumerate(cams):
        full = rng.standard_normal((c.height * c.width, 3)).astype(np.float32)
        if pix[v] is not None:
            mask = np.zeros(c.height * c.width, bool)
            mask[pix[v]] = True
            full[~mask] = 0.0
        w.append(full.reshape(c.height, c.width, 3))
    return scene, cams, pix, w


def _near_tie_swaps(scene, cams):
    xyz = scene.xyz.astype(np.float64)
    swapped = 0
    for cam in cams:
        R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
        Z = xyz @ R[2] + float(np.float32(cam.t[2]))
        order = oracle.depth_order(scene, cam)
        exact = np.lexsort((order, Z[order]))
        swapped += int((order[exact] != order).sum())
    return swapped


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_surface300k_4x800_parity(dpr, headline, mode):
    import torch
    scene, cams, pix, w = headline
    print(f"headline parity, {mode}: 300k points, 4 x 800x800", flush=True)
    params = dpr.RenderParams(bwd_mode=mode)
    plan = gpu_plan([scene], [(0, c) for c in cams], params)
    for v, cam in enumerate(cams):
        ref = oracle.render(scene, cam, oparams(params), pixels=pix[v])
        compare_images(to_np(plan.images[v]), to_np(plan.trans[v]), ref, pixels=pix[v], label=f"view {v}")
    out = plan.backward([torch.from_numpy(x).cuda() for x in w], None)
    torch.cuda.synchronize()
    got = [to_np(t) for t in out[0]]
    ref = oracle.backward(scene, cams, [x.reshape(-1, 3) if p is None else x.reshape(-1, 3)[p] for x, p in zip(w, pix)],
                          None, params=oparams(params), pixels=pix)
    compare_grads(got[0], ref.xyz, f"headline {mode} dxyz")
    compare_grads(got[1], ref.sh, f"headline {mode} dsh")
    compare_grads(got[2], ref.opacity, f"headline {mode} dopacity")
    info = plan.info()
    print(f"  pairs {info.pairs}; list positions ordered differently by float32 key and float64 Z: "
          f"{_near_tie_swaps(scene, cams)} of {4 * scene.n}", flush=True)


def test_surface300k_paper_renderer_parity_outside_near_ties(dpr, headline):
    """The paper-literal renderer (n = 15 splats per pixel, normalised Eq. 5)
    at the benchmark workload.  Under the cap, a pixel whose 15th splat rests
    on a predicate within a relative 1e-4 of alpha_min has two valid results a
    whole splat apart (the oracle decides in FP64, the kernel in FP32: their
    exponents differ by up to a few 1e-5 here); the oracle flags those pixels
    (near_tie).  They must be rare, and every other pixel and the gradients of
    the loss with weight 0 on them must match."""
    import torch
    scene, cams, pix, w = headline
    params = dpr.RenderParams.paper()
    op = oparams(params)
    cams = cams[:2]
    refs = [oracle.render(scene, cam, op) for cam in cams]
    ties = [r.near_tie for r in refs]
    n_ties = sum(int(t.sum()) for t in ties)
    print(f"paper renderer at 300k x 800x800: {n_ties} near-tie pixels of {2 * 800 * 800}", flush=True)
    assert n_ties <= 1e-3 * 2 * 800 * 800
    plan = gpu_plan([scene], [(0, c) for c in cams], params)
    for v, (r, t) in enumerate(zip(refs, ties)):
        img, tr = to_np(plan.images[v]).astype(np.float64), to_np(plan.trans[v]).astype(np.float64)
        ei = float(np.abs(img - r.image)[~t].max())
        et = float(np.abs(tr - r.trans)[~t].max())
        assert ei <= 1e-4 and et <= 1e-4, (v, ei, et)
    wm = [np.where(t[..., None], np.float32(0.0), x).astype(np.float32) for x, t in zip(w[:2], ties)]
    # view 1's weights are zero outside its 4096 sampled pixels already
    out = plan.backward([torch.from_numpy(x).cuda() for x in wm], None)
    torch.cuda.synchronize()
    got = [to_np(t) for t in out[0]]
    ref = oracle.backward(scene, cams, [x.astype(np.float64) for x in wm], None, params=op)
    compare_grads(got[0], ref.xyz, "paper headline dxyz")
    compare_grads(got[1], ref.sh, "paper headline dsh")
    compare_grads(got[2], ref.opacity, "paper headline dopacity")
