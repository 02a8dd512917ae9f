"""Pins of the oracle's visual-hull initialisation and consistency filter
(Sec. 3.1 initialisation, appendix consistency check CC): published
known-answer vectors of the generator, exact arithmetic, hand-worked cases, and
the geometry of a sphere's visual hull.  None re-types the oracle's loops."""
import numpy as np
import pytest

import oracle
import workloads


def test_philox_known_answers():
    """Known-answer vectors published with the Philox4x32-10 reference
    implementation (Random123, Salmon et al. SC 2011)."""
    cases = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, want in cases:
        assert list(oracle.philox4x32_10(ctr, key)) == want


def test_candidates_from_the_generator_words():
    """Candidate j: u = (r >> 8) 2^-24 of the first three words of Philox at
    counter (j, 0, 0, 0) and key (seed lo, seed hi), mapped to lo + u (hi - lo)
    with one rounding.  Recomputed here in exact float64 arithmetic (the product
    of a 24-bit u and a float32 width plus a float32 lo of close exponent is
    exact in float64), then rounded to float32 once."""
    seed = (0x1234 << 32) | 0x9abcdef0
    lo = np.array([-1.5, -1.0, 0.25], np.float32)
    hi = np.array([2.0, 1.0, 0.75], np.float32)
    got = oracle.hull_candidates(seed, 50, lo, hi)
    w = (hi - lo).astype(np.float32).astype(np.float64)
    for j in range(50):
        r = oracle.philox4x32_10([j, 0, 0, 0], [seed & 0xffffffff, seed >> 32])
        u = (r[:3] >> 8).astype(np.float64) * 2.0 ** -24
        want = (u * w + lo.astype(np.float64)).astype(np.float32)
        assert np.array_equal(got[j], want), j
    assert (got >= lo).all() and (got < hi).all()


def test_candidates_are_uniform():
    got = oracle.hull_candidates(3, 200000, [0, 0, 0], [1, 1, 1])
    assert abs(got.mean() - 0.5) < 0.003
    hist = np.histogram(got[:, 0], bins=10, range=(0, 1))[0] / 200000
    assert np.abs(hist - 0.1).max() < 0.004


def _cam(fx=100.0, cx=50.0, size=100, t=(0.0, 0.0, 3.0)):
    class C:
        pass
    c = C()
    c.R = np.eye(3, dtype=np.float32).reshape(9)
    c.t = np.array(t, np.float32)
    c.fx = c.fy = fx
    c.cx = c.cy = cx
    c.width = c.height = size
    return c


def test_single_foreground_pixel():
    """R = I, t = (0, 0, 3), f = 100, c = 50: the origin projects to (50, 50),
    the corner of pixel (50, 50); x = 1e-4 stays in column 50,
    x = -1e-3 moves to column 49; a point behind the camera is outside."""
    cam = _cam()
    m = np.zeros((100, 100), np.uint8)
    m[50, 50] = 1
    pts = np.array([[0, 0, 0], [1e-4, 1e-4, 0], [-1e-3, 0, 0], [0, -1e-3, 0], [0, 0, -4], [0, 0, 1]], np.float32)
    keep = oracle.hull_consistent(pts, [cam], [m])
    assert list(keep) == [True, True, False, False, False, True]


def test_image_border_and_every_mask():
    """A point projecting outside the image is outside its mask; CC needs every
    mask."""
    cam = _cam()
    full = np.ones((100, 100), np.uint8)
    empty = np.zeros((100, 100), np.uint8)
    # px = 100 * x / 3 + 50: x = 1.5 -> 100 (just outside), x = 1.49 -> 99.67
    pts = np.array([[1.5, 0, 0], [1.49, 0, 0], [-1.5, 0, 0], [-1.49, 0, 0]], np.float32)
    assert list(oracle.hull_consistent(pts, [cam], [full])) == [False, True, True, True]
    assert not oracle.hull_consistent(pts, [cam, cam], [full, empty]).any()


def test_sphere_visual_hull():
    """Disc masks of a sphere from 12 views: every candidate well inside the
    sphere is kept, and every kept candidate lies inside every view's
    silhouette cone (an independent 3-D angle test), up to one pixel."""
    cams = workloads.disc_views(12, size=96)
    rho = 0.5
    masks = workloads.sphere_masks(cams, rho)
    lo, hi = np.array([-1, -1, -1], np.float32), np.array([1, 1, 1], np.float32)
    cand = oracle.hull_candidates(11, 60000, lo, hi)
    keep = oracle.hull_consistent(cand, cams, masks)
    r = np.linalg.norm(cand.astype(np.float64), axis=1)
    px = 1.0 / cams[0].fx                       # one pixel, in radians
    pxw = 3.0 * px                              # one pixel at the distance of the sphere
    # a point 2 px inside the silhouette is inside whatever pixel it lands on
    assert keep[r < rho - 2 * pxw].all()
    for cam in cams:
        R = np.asarray(cam.R, np.float64).reshape(3, 3)
        C = -R.T @ np.asarray(cam.t, np.float64)
        d = np.linalg.norm(C)
        v = cand[keep].astype(np.float64) - C
        ang = np.arccos(np.clip((v @ (-C / d)) / np.linalg.norm(v, axis=1), -1, 1))
        assert (ang <= np.arcsin(rho / d) + px).all()
    n, kept = oracle.hull_sample(cams, masks, lo, hi, 11, 60000)
    assert n == keep.sum() and np.array_equal(kept, cand[keep])
    frac = n / 60000
    assert 4 / 3 * np.pi * (rho - 2 * pxw) ** 3 / 8 <= frac < 1.5 * 4 / 3 * np.pi * rho ** 3 / 8


def test_sample_capacity_truncates():
    cams = workloads.disc_views(3, size=48)
    masks = workloads.sphere_masks(cams, 0.8)
    n, pts = oracle.hull_sample(cams, masks, [-1, -1, -1], [1, 1, 1], 5, 4000)
    n2, pts2 = oracle.hull_sample(cams, masks, [-1, -1, -1], [1, 1, 1], 5, 4000, capacity=10)
    assert n2 == n and pts2.shape == (10, 3) and np.array_equal(pts2, pts[:10])


def test_consistency_filter_keeps_order_and_parameters():
    cams = workloads.disc_views(5, size=64)
    masks = workloads.sphere_masks(cams, 0.6)
    rng = np.random.default_rng(2)
    xyz = rng.uniform(-1, 1, (3000, 3)).astype(np.float32)
    cloud = oracle.Cloud(xyz, *workloads.point_attributes(3000, 2, 4))
    keep, out = oracle.consistency_filter(cloud, cams, masks)
    idx = np.flatnonzero(keep)
    assert 0 < len(idx) < 3000
    assert np.array_equal(out.xyz, xyz[idx]) and np.array_equal(out.radius, cloud.radius[idx])
    assert np.array_equal(out.sh, cloud.sh[idx]) and np.array_equal(out.opacity, cloud.opacity[idx])


def test_consistency_agrees_with_plain_float32_projection_away_from_pixel_edges():
    """numpy float32 projection without fused multiply-adds gives the same
    decision wherever the projected point is not within 1e-3 px of a pixel
    edge (where the two roundings may disagree)."""
    cams = workloads.disc_views(4, size=80, seed=3)
    masks = workloads.sphere_masks(cams, 0.7)
    rng = np.random.default_rng(9)
    xyz = rng.uniform(-1, 1, (20000, 3)).astype(np.float32)
    keep = oracle.hull_consistent(xyz, cams, masks)
    ref = np.ones(len(xyz), bool)
    clear = np.ones(len(xyz), bool)
    for cam, m in zip(cams, masks):
        R = np.asarray(cam.R, np.float32).reshape(3, 3)
        X = xyz @ R.T + np.asarray(cam.t, np.float32)
        with np.errstate(divide="ignore", invalid="ignore"):
            px = np.float32(cam.fx) * (X[:, 0] / X[:, 2]) + np.float32(cam.cx)
            py = np.float32(cam.fy) * (X[:, 1] / X[:, 2]) + np.float32(cam.cy)
        inside = (X[:, 2] > 0) & (px >= 0) & (px < cam.width) & (py >= 0) & (py < cam.height)
        col = np.clip(np.floor(px), 0, cam.width - 1).astype(int)
        row = np.clip(np.floor(py), 0, cam.height - 1).astype(int)
        ref &= inside & (m[row, col] > 0)
        frac = np.minimum(np.abs(px - np.round(px)), np.abs(py - np.round(py)))
        clear &= ~(inside & (frac < 1e-3))
    assert clear.mean() > 0.97
    assert np.array_equal(keep[clear], ref[clear])
