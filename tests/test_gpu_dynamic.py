"""Multi-scene launch: 30 frames x 200k points, one 1024x768 view per frame,
rendered forward and backward as ONE plan (one launch per stage).  Checked on
sampled pixels of chosen frames against the oracle, and with a loss restricted
to sampled pixels for the gradients."""
import numpy as np
import pytest

import oracle
import workloads

from _gpu_util import compare_grads, compare_images, oparams, random_pixels, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frames():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14330_amd as dpr
    dpr.load()
    scenes_np, cams, _ = workloads.dynamic30x200k_1024x768()
    scenes = [dpr.SceneTensors.from_numpy(s) for s in scenes_np]
    return dpr, scenes_np, scenes, cams


@pytest.mark.parametrize("persistent", [False, True])
def test_thirty_frames_one_plan_forward(frames, persistent):
    import torch
    dpr, scenes_np, scenes, cams = frames
    plan = dpr.Plan(scenes, [(t, cams[t]) for t in range(30)], dpr.RenderParams(persistent=persistent))
    plan.forward()
    torch.cuda.synchronize()
    for t in (0, 13, 29):
        pix = random_pixels(500 + t, cams[t], 1024)
        ref = oracle.render(scenes_np[t], cams[t], pixels=pix)
        compare_images(to_np(plan.images[t]), to_np(plan.trans[t]), ref, pixels=pix, label=f"frame {t}")


def test_thirty_frames_one_plan_gradients(frames):
    import torch
    dpr, scenes_np, scenes, cams = frames
    params = dpr.RenderParams()
    plan = dpr.Plan(scenes, [(t, cams[t]) for t in range(30)], params)
    plan.forward()
    rng = np.random.default_rng(77)
    check = (4, 21)
    gI, pix = [], {}
    for t in range(30):
        g = np.zeros((cams[t].height * cams[t].width, 3), np.float32)
        if t in check:
            pix[t] = random_pixels(600 + t, cams[t], 512)
            g[pix[t]] = rng.standard_normal((512, 3)).astype(np.float32)
        gI.append(torch.from_numpy(g.reshape(cams[t].height, cams[t].width, 3)).cuda())
    out = plan.backward(gI, None)
    torch.cuda.synchronize()
    for t in check:
        ref = oracle.backward(scenes_np[t], [cams[t]], [to_np(gI[t]).reshape(-1, 3)[pix[t]]], None,
                              params=oparams(params), pixels=[pix[t]])
        compare_grads(to_np(out[t][0]), ref.xyz, f"frame {t} dxyz")
        compare_grads(to_np(out[t][1]), ref.sh, f"frame {t} dsh")
        compare_grads(to_np(out[t][2]), ref.opacity, f"frame {t} dopacity")
    # frames without loss get exactly zero gradient
    assert float(out[0][0].abs().max()) == 0.0
