"""Helpers shared by the GPU parity tests (not collected by pytest)."""
from __future__ import annotations

import numpy as np

import oracle
import workloads

IMG_TOL = 1e-4          # max-abs per pixel/channel, image and transmittance
GRAD_RTOL = 1e-3        # per element, relative to max(|g*|, 1e-2 ||g*||_inf)
GRAD_L2 = 1e-3          # ||g - g*||_2 / ||g*||_2

# (name, worst element error as a fraction of its bound, rel-L2 as a fraction of
# GRAD_L2) of every gradient comparison of the session, for the margin summary
GRAD_MARGINS = []


def torch_mod():
    import torch
    return torch


def scene_tensors(scene):
    from paper_2205_14330_amd import SceneTensors
    return SceneTensors.from_numpy(scene, "cuda")


def oparams(p) -> oracle.Params:
    return oracle.Params(p.alpha_min, p.t_min, p.alpha_max, p.z_near, p.sh_frame, int(p.max_splats),
                         int(p.kernel_norm))


def gpu_plan(scenes, views, params, run_forward=True):
    """scenes: list of numpy workloads.Scene; views: list of (scene index, camera)."""
    from paper_2205_14330_amd import Plan
    torch = torch_mod()
    st = [scene_tensors(s) for s in scenes]
    plan = Plan(st, views, params)
    if run_forward:
        plan.forward()
    torch.cuda.synchronize()
    return plan


def to_np(t):
    return t.detach().cpu().numpy()


def compare_images(img_gpu, tr_gpu, ref: oracle.RenderResult, pixels=None, tol=IMG_TOL, label=""):
    img = np.asarray(img_gpu, np.float64)
    tr = np.asarray(tr_gpu, np.float64)
    if pixels is not None:
        img = img.reshape(-1, 3)[pixels]
        tr = tr.reshape(-1)[pixels]
    ei = np.abs(img - ref.image).max() if img.size else 0.0
    et = np.abs(tr - ref.trans).max() if tr.size else 0.0
    assert ei <= tol and et <= tol, f"{label}: image err {ei:.3e}, trans err {et:.3e}"
    return ei, et


def compare_grads(g, ref, name=""):
    g = np.asarray(g, np.float64).reshape(-1)
    r = np.asarray(ref, np.float64).reshape(-1)
    if r.size == 0:
        return 0.0
    gmax = np.abs(r).max()
    if gmax == 0.0:
        assert np.abs(g).max() <= 1e-6, f"{name}: reference gradient is zero, got {np.abs(g).max()}"
        return 0.0
    bound = GRAD_RTOL * np.maximum(np.abs(r), 1e-2 * gmax)
    bad = np.abs(g - r) > bound
    l2 = np.linalg.norm(g - r) / np.linalg.norm(r)
    GRAD_MARGINS.append((name, float(np.max(np.abs(g - r) / bound)), float(l2 / GRAD_L2)))
    assert not bad.any(), (f"{name}: {bad.sum()} of {r.size} elements off; worst "
                           f"{np.max(np.abs(g - r) / bound):.3g}x the bound; rel-L2 {l2:.3e}")
    assert l2 <= GRAD_L2, f"{name}: rel-L2 {l2:.3e}"
    return l2


def random_pixels(seed, cam, count):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cam.width * cam.height, size=min(count, cam.width * cam.height), replace=False))
