"""Pins of the oracle's paper-literal variants and of the Eq. (8) loss.

* the per-pixel cap of n blended splats (Sec. 3.3 sets n = 15),
* Eq. (5) with its normalisation prefactor kept (1/sqrt(2 pi r^2), per axis
  (2 pi sx sy)^-1/2),
* the loss of Eq. (8): squared L2 plus lambda times the anisotropic total
  variation (Sec. 3.3, lambda = 0.01).
Each check is a hand-derived closed form, an identity, brute force or finite
differences — none re-types the oracle's formulas.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from workloads import Camera, Scene

SQRT_PI = math.sqrt(math.pi)
SQRT_2PI = math.sqrt(2.0 * math.pi)


def _scene(xyz, sh, opacity, radius):
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    n = xyz.shape[0]
    sh = np.asarray(sh, np.float32).reshape(n, -1, 3)
    return Scene(xyz, sh, np.asarray(opacity, np.float32).reshape(n),
                 np.broadcast_to(np.asarray(radius, np.float32), (n,)).copy())


def _cam(t=(0.0, 0.0, 3.125), f=100.0, c=8.5, size=17):
    return Camera(np.eye(3), t, f, f, c, c, size, size)


# ---------------------------------------------------------------------------
# per-pixel cap
# ---------------------------------------------------------------------------

def _three_stacked():
    """Three splats projecting onto pixel (8, 8)'s centre, sigma 1 px, at
    Z = 3.125, 6.25, 9.375, with opacities 0.5, 0.75, 0.25."""
    cols = np.array([[1.0, 0.0, 0.5], [0.0, 1.0, -0.5], [0.25, 0.25, 1.0]])
    h = cols[:, None, :] * 2 * SQRT_PI
    sc = _scene([[0, 0, 0], [0, 0, 3.125], [0, 0, 6.25]], h, [0.5, 0.75, 0.25], [0.03125, 0.0625, 0.09375])
    return sc, cols


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_cap_three_stacked_splats(n):
    """At the shared centre alpha = o exactly; capped at n the pixel composites
    the first n of them: I = sum_{i<n} a_i prod_{k<i}(1 - a_k) c_i."""
    sc, cols = _three_stacked()
    a = [0.5, 0.75, 0.25]
    r = oracle.render(sc, _cam(), oracle.Params(max_splats=n), mode="brute")
    I = np.zeros(3)
    T = 1.0
    for i in range(min(n, 3)):
        I += T * a[i] * cols[i]
        T *= 1 - a[i]
    np.testing.assert_allclose(r.image[8, 8], I, atol=1e-6)   # colours carry float32 rounding of h
    assert abs(r.trans[8, 8] - T) < 1e-12
    assert r.ncontrib[8, 8] == min(n, 3)


@pytest.mark.parametrize("rel,cap,flagged", [(3e-5, 2, True), (-3e-5, 2, True), (3e-4, 2, False),
                                              (1.0, 2, False), (3e-5, 0, False)])
def test_cap_near_tie_flag(rel, cap, flagged):
    """Under a cap, a pixel whose candidate is decided within a relative 1e-4
    of alpha_min is flagged (an evaluation in float32 may decide it the other
    way and shift the pixel's n-th splat); at the shared centre alpha = o, so
    the first splat's opacity sets that distance.  Without a cap no pixel is
    flagged, and the flag changes nothing else."""
    sc, _ = _three_stacked()
    amin = oracle.Params().alpha_min
    sc.opacity[0] = np.float32(amin * (1.0 + rel))
    r = oracle.render(sc, _cam(), oracle.Params(max_splats=cap), mode="brute")
    assert bool(r.near_tie[8, 8]) == flagged
    assert r.stopped.max() <= 1 and r.near_tie.sum() <= (1 if flagged else 0)
    ref = oracle.render(sc, _cam(), oracle.Params(max_splats=cap), mode="grid")
    assert np.array_equal(ref.image, r.image) and np.array_equal(ref.near_tie, r.near_tie)


def test_cap_above_candidate_count_is_uncapped_bitwise():
    sc = workloads.small_scene(41, 60, extent=0.2)
    rng = np.random.default_rng(41)
    cam = workloads.random_sphere_camera(rng, 24, 20)
    base = oracle.render(sc, cam, oracle.Params(), mode="brute")
    big = oracle.render(sc, cam, oracle.Params(max_splats=10 ** 6), mode="grid")
    assert np.array_equal(base.image, big.image) and np.array_equal(base.trans, big.trans)
    capped = oracle.render(sc, cam, oracle.Params(max_splats=2), mode="grid")
    assert capped.ncontrib.max() == 2 and (base.ncontrib > 2).any()
    keep = base.ncontrib <= 2                      # pixels the cap does not touch
    assert np.array_equal(capped.image[keep], base.image[keep])


def test_cap_equals_brute_force_prefix():
    """Capped at n, a pixel's result equals the uncapped render of the scene
    reduced to that pixel's first n candidates (found by rendering each point
    alone at the pixel and walking the depth order)."""
    sc = workloads.small_scene(42, 40, extent=0.15)
    rng = np.random.default_rng(42)
    cam = workloads.random_sphere_camera(rng, 16, 16)
    n = 3
    order = oracle.depth_order(sc, cam)
    capped = oracle.render(sc, cam, oracle.Params(max_splats=n), mode="brute")
    for (x, y) in [(8, 8), (3, 12), (12, 4), (0, 0)]:
        first = []
        for i in order:
            one = Scene(sc.xyz[i:i + 1], sc.sh[i:i + 1], sc.opacity[i:i + 1], sc.radius[i:i + 1])
            if oracle.render(one, cam, mode="brute").trans[y, x] < 1.0:
                first.append(i)
            if len(first) == n:
                break
        sub = Scene(sc.xyz[first], sc.sh[first], sc.opacity[first], sc.radius[first])
        ref = oracle.render(sub, cam, mode="brute")
        np.testing.assert_allclose(capped.image[y, x], ref.image[y, x], rtol=0, atol=1e-14)
        assert abs(capped.trans[y, x] - ref.trans[y, x]) < 1e-14


# ---------------------------------------------------------------------------
# Eq. (5) with the normalisation prefactor
# ---------------------------------------------------------------------------

def test_kernel_norm_hand_values():
    """sigma = 1 px: alpha = o G / sqrt(2 pi) at the pixel centres."""
    h = np.array([[1.0, 2.0, -1.0]]) * (2 * SQRT_PI)
    sc = _scene([[0, 0, 0]], h, [0.5], 0.03125)
    r = oracle.render(sc, _cam(), oracle.Params(kernel_norm=1), mode="brute")
    col = np.array([1.0, 2.0, -1.0])
    for (x, y), g in {(8, 8): 1.0, (9, 8): math.exp(-0.5), (9, 9): math.exp(-1.0), (8, 11): math.exp(-4.5)}.items():
        a = 0.5 * g / SQRT_2PI
        np.testing.assert_allclose(r.image[y, x], a * col, rtol=1e-6)
        assert abs(r.trans[y, x] - (1 - a)) < 1e-7


def test_kernel_norm_footprint_mass():
    """Untruncated, the alphas of one splat sum to o 2 pi sx sy (2 pi sx sy)^-1/2
    = o sqrt(2 pi sx sy): the normalised kernel integrates to o sqrt(2 pi) sigma
    per axis pair (sigma = 5 px here, 2 pi sigma^2 / sqrt(2 pi sigma^2))."""
    f, Z, rad = 200.0, 4.0, 0.1
    cam = Camera(np.eye(3), [0, 0, Z], f, f, 64.0, 64.0, 128, 128)
    sc = _scene([[0.0125, -0.03, 0.0]], np.array([[1, 1, 1]]) * 2 * SQRT_PI, [0.25], rad)
    p = oracle.Params.untruncated()
    p.kernel_norm = 1
    res = oracle.render(sc, cam, p, mode="brute")
    s = float(np.float32(rad)) * float(np.float32(f)) / Z
    assert abs((1.0 - res.trans).sum() - 0.25 * SQRT_2PI * s) < 1e-9


def test_kernel_norm_clamps_small_splats():
    """sigma = 0.25 px: the prefactor 1/(sqrt(2 pi) 0.25) = 1.6 pushes o G past
    alpha_max at the centre, which is then clamped to 0.99."""
    h = np.array([[1.0, 1.0, 1.0]]) * (2 * SQRT_PI)
    sc = _scene([[0, 0, 0]], h, [0.9], 0.0078125)
    r = oracle.render(sc, _cam(), oracle.Params(kernel_norm=1), mode="brute")
    assert abs(r.trans[8, 8] - 0.01) < 1e-12


# ---------------------------------------------------------------------------
# gradients of the variants: central finite differences
# ---------------------------------------------------------------------------

def _fd_check(sc, cam, params, seed):
    rng = np.random.default_rng(seed)
    npix = cam.pixels
    wI = rng.standard_normal((npix, 3))
    wT = rng.standard_normal(npix)
    xyz = sc.xyz.astype(np.float64)
    sh = sc.sh.astype(np.float64)
    op = sc.opacity.astype(np.float64)
    rad = sc.radius.astype(np.float64)
    g = oracle.backward_double(xyz, sh, op, rad, cam, wI, wT, params)

    def run():
        r = oracle.render_double(xyz, sh, op, rad, cam, params)
        class _S:
            pass
        q = _S()
        q.xyz = xyz.astype(np.float32)
        return r, oracle.depth_order(q, cam, params)

    def loss(r):
        return float((r.image.reshape(-1, 3) * wI).sum() + (r.trans.reshape(-1) * wT).sum())

    checked = kinked = 0
    for name, arr, h in (("xyz", xyz, 1e-6), ("sh", sh, 1e-3), ("opacity", op, 1e-6)):
        grad = getattr(g, name)
        gmax = np.abs(grad).max()
        flat = arr.reshape(-1)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            rp, op_ = run()
            flat[j] = old - h
            rm, om_ = run()
            flat[j] = old
            if not (np.array_equal(rp.ncontrib, rm.ncontrib) and np.array_equal(rp.stopped, rm.stopped)
                    and np.array_equal(op_, om_)):
                kinked += 1
                continue
            fd = (loss(rp) - loss(rm)) / (2 * h)
            an = grad.reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * gmax) + 1e-12, (name, j, fd, an)
            checked += 1
    assert kinked <= 0.05 * (checked + kinked)
    assert checked > 0


@pytest.mark.parametrize("params", [oracle.Params(max_splats=3), oracle.Params(kernel_norm=1),
                                    oracle.Params(max_splats=5, kernel_norm=1, sh_frame=1)],
                         ids=["cap3", "norm", "cap5-norm-world"])
def test_variant_gradients_match_central_differences(params):
    sc = workloads.small_scene(43, 24, extent=0.15)
    sc.opacity = np.minimum(sc.opacity, np.float32(0.95))
    rng = np.random.default_rng(43)
    cam = workloads.random_sphere_camera(rng, 32, 32)
    cam = Camera(cam.R, cam.t, 300.0, 300.0, 16.0, 16.0, 32, 32)
    _fd_check(sc, cam, params, 43)


# ---------------------------------------------------------------------------
# Eq. (8): squared L2 + lambda anisotropic TV
# ---------------------------------------------------------------------------

def test_loss_constant_render_has_no_tv():
    rng = np.random.default_rng(50)
    tgt = rng.standard_normal((5, 7, 3))
    R = np.full((5, 7, 3), 0.3)
    loss, g = oracle.loss_l2_tv(R, tgt, 0.01)
    assert abs(loss - ((0.3 - tgt) ** 2).sum()) < 1e-12
    np.testing.assert_allclose(g, 2 * (0.3 - tgt), atol=1e-15)


def test_loss_ramp_and_checkerboard_tv():
    """R = a x + b y per channel: TV = 3 (|a| H (W-1) + |b| W (H-1)); a 0/1
    checkerboard: every adjacent pair differs by 1."""
    H, W = 6, 9
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    R = np.repeat((0.5 * xx - 0.25 * yy)[:, :, None], 3, axis=2)
    loss, _ = oracle.loss_l2_tv(R, R, 2.0)
    assert abs(loss - 2.0 * 3 * (0.5 * H * (W - 1) + 0.25 * W * (H - 1))) < 1e-12
    cb = np.repeat(((xx + yy) % 2)[:, :, None], 3, axis=2)
    loss, g = oracle.loss_l2_tv(cb, cb, 1.0)
    assert abs(loss - 3 * (H * (W - 1) + W * (H - 1))) < 1e-12
    # an interior 1-pixel of the checkerboard: its 4 neighbours are 0, each
    # difference pulls it down by 1 -> subgradient +4 (0-pixels get -4)
    assert g[2, 3, 0] == (4.0 if cb[2, 3, 0] == 1 else -4.0)


def test_loss_lambda_zero_is_l2():
    rng = np.random.default_rng(51)
    R, T = rng.standard_normal((2, 4, 5, 3))
    loss, g = oracle.loss_l2_tv(R, T, 0.0)
    assert abs(loss - ((R - T) ** 2).sum()) < 1e-12
    np.testing.assert_allclose(g, 2 * (R - T), atol=0)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(52)
    R = rng.standard_normal((5, 6, 3))
    T = rng.standard_normal((5, 6, 3))
    lam = 0.37
    _, g = oracle.loss_l2_tv(R, T, lam)
    h = 1e-7
    for idx in np.ndindex(R.shape):
        Rp = R.copy(); Rp[idx] += h
        Rm = R.copy(); Rm[idx] -= h
        fd = (oracle.loss_l2_tv(Rp, T, lam)[0] - oracle.loss_l2_tv(Rm, T, lam)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6, (idx, fd, g[idx])
