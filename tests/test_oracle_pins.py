"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these checks re-types the oracle's generic formulas: each one is a
closed-form special case with hand-derived numbers, an identity of the
mathematics (orthonormality, Gaussian moments, telescoping of Eq. 6-7,
multiplicativity of transmittance, linearity), a library routine for a special
case (scipy's spherical harmonics), brute force, or finite differences.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from workloads import Camera, Scene

SQRT_PI = math.sqrt(math.pi)
Y00 = 1.0 / (2.0 * SQRT_PI)


def _scene(xyz, sh, opacity, radius):
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    n = xyz.shape[0]
    sh = np.asarray(sh, np.float32).reshape(n, -1, 3)
    return Scene(xyz, sh, np.asarray(opacity, np.float32).reshape(n),
                 np.broadcast_to(np.asarray(radius, np.float32), (n,)).copy())


def _cam(t=(0.0, 0.0, 3.125), f=100.0, c=8.5, size=17, R=None):
    return Camera(np.eye(3) if R is None else R, t, f, f, c, c, size, size)


# ---------------------------------------------------------------------------
# Spherical harmonics (Sec. 3.1, Eq. 4)
# ---------------------------------------------------------------------------

def test_sh_orthonormal_by_quadrature():
    """int Y_a Y_b dOmega = delta_ab over the sphere (pins the constants)."""
    xg, wg = np.polynomial.legendre.leggauss(64)      # cos(theta) nodes
    nphi = 128
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = oracle.sh_basis(3, dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def _scipy_real_sh(l, m, dirs):
    from scipy.special import sph_harm_y
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    Ylm = sph_harm_y(l, abs(m), theta, phi)
    # real form without the Condon-Shortley phase: the (-1)^m cancels scipy's
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Ylm.real
    return math.sqrt(2) * (-1) ** m * Ylm.imag


def test_sh_matches_textbook_real_basis():
    """Each Y_k, k = l^2 + l + m, equals the real SH built from scipy's
    complex ones (pins constants, signs and the index order)."""
    rng = np.random.default_rng(1)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _scipy_real_sh(l, m, d)
            assert np.abs(Y[:, l * l + l + m] - ref).max() < 1e-12, (l, m)


def test_sh_low_order_values():
    """Hand-derived values: Y00 = 1/(2 sqrt(pi)), Y1 = sqrt(3/(4 pi)) (y, z, x)."""
    d = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    Y = oracle.sh_basis(1, d)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert abs(Y[0, 0] - 0.28209479177387814) < 1e-15
    np.testing.assert_allclose(Y[:, 1:], [[0, c1, 0], [0, 0, c1], [c1, 0, 0]], atol=1e-15)
    assert abs(c1 - 0.4886025119029199) < 1e-15


def test_sh_gradient_matches_finite_difference():
    rng = np.random.default_rng(2)
    d = rng.standard_normal((50, 3))
    Y, dY = oracle.sh_basis(3, d, grad=True)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (oracle.sh_basis(3, d + e) - oracle.sh_basis(3, d - e)) / (2 * h)
        assert np.abs(fd - dY[:, :, a]).max() < 1e-8


# ---------------------------------------------------------------------------
# Projection (Sec. 3.1, Eq. 1) and colour (Eq. 3-4)
# ---------------------------------------------------------------------------

def test_projection_closed_forms():
    W = 128
    f = workloads.fov_focal(W)
    cam = Camera(np.eye(3), [0, 0, 3], f, f, 64, 64, W, W)
    xyz = np.array([[0.0, 0.0, 0.0],                                   # on axis
                    [3.0 * math.tan(math.radians(25.0)), 0.0, 0.0],    # right edge of the fov
                    [0.5, -0.25, 1.0]], np.float32)
    sc = _scene(xyz, np.zeros((3, 1, 3)), [0.5] * 3, 0.02)
    pr = oracle.project(sc, cam)
    fx = float(np.float32(f))
    assert pr["px"][0] == 64.0 and pr["py"][0] == 64.0
    assert abs(pr["px"][1] - (fx * float(xyz[1, 0]) / 3.0 + 64.0)) < 1e-12
    assert abs(pr["px"][1] - 128.0) < 1e-4
    assert abs(pr["px"][2] - (fx * 0.5 / 4.0 + 64.0)) < 1e-12
    assert abs(pr["py"][2] - (fx * -0.25 / 4.0 + 64.0)) < 1e-12
    # perspective-scaled sigma: f r / Z
    assert abs(pr["sx"][2] - fx * float(np.float32(0.02)) / 4.0) < 1e-12
    assert pr["zkey"][2] == np.float32(4.0)


def test_projection_rotated_camera():
    """A camera looking along -x from (3,0,0): X_cam = R P + t, then Eq. (1)."""
    cam = workloads.look_at_camera([3.0, 0.0, 0.0], 64, 48)
    sc = _scene([[0.0, 0.2, 0.1]], np.zeros((1, 1, 3)), [0.5], 0.02)
    pr = oracle.project(sc, cam)
    R = cam.R.astype(np.float64)
    X = R @ np.array([0.0, np.float32(0.2), np.float32(0.1)]) + cam.t.astype(np.float64)
    assert abs(X[2] - 3.0) < 1e-6                   # depth along the optical axis
    # right = f x up with f = (-1,0,0), up = z -> right = (0,1,0)... image x grows with world y
    assert pr["px"][0] > 32.0 and pr["py"][0] < 24.0   # world +z is image up (smaller row)


def test_degree0_colour_is_view_independent():
    """l_max = 0 is a single colour per point (Sec. 3.3): c = h00 / (2 sqrt(pi))."""
    rng = np.random.default_rng(3)
    sc = workloads.small_scene(3, 40, sh_degree=0)
    c1 = oracle.project(sc, workloads.random_sphere_camera(rng, 32, 32))["color"]
    c2 = oracle.project(sc, workloads.random_sphere_camera(rng, 32, 32))["color"]
    expect = sc.sh[:, 0, :].astype(np.float64) * 0.28209479177387814
    np.testing.assert_allclose(c1, expect, rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(c2, expect, rtol=1e-15, atol=1e-16)


def test_degree1_colour_closed_form_and_frames():
    rng = np.random.default_rng(4)
    sc = workloads.small_scene(4, 30, sh_degree=1)
    cam = workloads.random_sphere_camera(rng, 32, 32)
    for frame in (0, 1):
        pr = oracle.project(sc, cam, oracle.Params(sh_frame=frame))
        X = sc.xyz.astype(np.float64) @ cam.R.astype(np.float64).T + cam.t.astype(np.float64)
        v = X / np.linalg.norm(X, axis=1, keepdims=True)
        d = v if frame == 0 else v @ cam.R.astype(np.float64)
        h = sc.sh.astype(np.float64)
        c1 = 0.4886025119029199
        exp = Y00 * h[:, 0] + c1 * (h[:, 1] * d[:, 1:2] + h[:, 2] * d[:, 2:3] + h[:, 3] * d[:, 0:1])
        np.testing.assert_allclose(pr["color"], exp, atol=1e-13)


# ---------------------------------------------------------------------------
# Splatting and compositing (Sec. 3.2, Eq. 5-7)
# ---------------------------------------------------------------------------

def test_single_splat_hand_values():
    """sigma = 100 * (1/32) / 3.125 = 1 px, centre exactly on pixel (8, 8)."""
    h = np.array([[1.0, 2.0, -1.0]]) * (2 * SQRT_PI)   # colour (1, 2, -1)
    sc = _scene([[0, 0, 0]], h, [0.5], 0.03125)
    r = oracle.render(sc, _cam(), mode="brute")
    col = np.array([1.0, 2.0, -1.0])
    cases = {(8, 8): 0.5, (9, 8): 0.5 * math.exp(-0.5), (8, 10): 0.5 * math.exp(-2.0),
             (9, 9): 0.5 * math.exp(-1.0), (12, 8): 0.5 * math.exp(-8.0)}
    for (x, y), a in cases.items():
        np.testing.assert_allclose(r.image[y, x], a * col, rtol=1e-6)
        assert abs(r.trans[y, x] - (1 - a)) < 1e-7
    # 5 px away: 0.5 exp(-12.5) = 1.86e-6 < alpha_min -> not a candidate
    assert np.all(r.image[8, 13] == 0) and r.trans[8, 13] == 1.0
    # untruncated: every pixel gets its Gaussian value
    ru = oracle.render(sc, _cam(), oracle.Params.untruncated(), mode="brute")
    assert abs(ru.trans[8, 13] - (1 - 0.5 * math.exp(-12.5))) < 1e-12


def test_gaussian_footprint_moments():
    """Sum of alpha over the pixel grid = o 2 pi sx sy; centroid = projected
    point; second moments = sigma^2 (pins the 1/2 in Eq. 5, the pixel-centre
    convention and the perspective scaling of r)."""
    f, Z, r = 200.0, 4.0, 0.1                        # sigma = 5 px
    cam = Camera(np.eye(3), [0, 0, Z], f, f, 64.0, 64.0, 128, 128)
    P = np.array([[0.0125, -0.03, 0.0]], np.float32)
    sc = _scene(P, np.array([[1, 1, 1]]) * 2 * SQRT_PI, [0.25], r)
    res = oracle.render(sc, cam, oracle.Params.untruncated(), mode="brute")
    a = 1.0 - res.trans
    s = float(np.float32(r)) * float(np.float32(f)) / Z
    assert abs(a.sum() - 0.25 * 2 * math.pi * s * s) < 1e-9
    yy, xx = np.mgrid[0:128, 0:128] + 0.5
    px = float(np.float32(f)) * float(P[0, 0]) / Z + 64
    py = float(np.float32(f)) * float(P[0, 1]) / Z + 64
    assert abs((a * xx).sum() / a.sum() - px) < 1e-9
    assert abs((a * yy).sum() / a.sum() - py) < 1e-9
    assert abs((a * (xx - px) ** 2).sum() / a.sum() - s * s) < 1e-8


def test_two_splats_front_to_back():
    """Eq. (6)-(7) with two splats on one pixel: I = a1 c1 + (1 - a1) a2 c2."""
    c1 = np.array([1.0, 0.0, 0.5])
    c2 = np.array([0.0, 1.0, -0.5])
    h = np.stack([c1, c2])[:, None, :] * 2 * SQRT_PI
    # both project onto (8.5, 8.5) with sigma = 1 px; point 0 at Z=3.125, point 1 at Z=6.25
    near_far = _scene([[0, 0, 0], [0, 0, 3.125]], h, [0.5, 0.75], [0.03125, 0.0625])
    r = oracle.render(near_far, _cam(), mode="brute")
    np.testing.assert_allclose(r.image[8, 8], 0.5 * c1 + 0.5 * 0.75 * c2, atol=1e-15)
    assert abs(r.trans[8, 8] - 0.125) < 1e-15
    # swap depths: now point 1 is in front
    far_near = _scene([[0, 0, 3.125], [0, 0, 0]], h, [0.5, 0.75], [0.0625, 0.03125])
    r = oracle.render(far_near, _cam(), mode="brute")
    np.testing.assert_allclose(r.image[8, 8], 0.75 * c2 + 0.25 * 0.5 * c1, atol=1e-15)
    # equal depth: the lower index goes first
    tie = _scene([[0, 0, 0], [0, 0, 0]], h, [0.5, 0.75], [0.03125, 0.03125])
    r = oracle.render(tie, _cam(), mode="brute")
    np.testing.assert_allclose(r.image[8, 8], 0.5 * c1 + 0.5 * 0.75 * c2, atol=1e-15)
    tie2 = _scene([[0, 0, 0], [0, 0, 0]], h[::-1], [0.75, 0.5], [0.03125, 0.03125])
    r = oracle.render(tie2, _cam(), mode="brute")
    np.testing.assert_allclose(r.image[8, 8], 0.75 * c2 + 0.25 * 0.5 * c1, atol=1e-15)


def _random_view(seed, n=48, size=32, extent=0.15, f=300.0, deg=2, op_max=0.95):
    sc = workloads.small_scene(seed, n, sh_degree=deg, extent=extent)
    sc.opacity = np.minimum(sc.opacity, np.float32(op_max))
    rng = np.random.default_rng(seed)
    cam = workloads.random_sphere_camera(rng, size, size)
    cam = Camera(cam.R, cam.t, f, f, size / 2, size / 2, size, size)
    return sc, cam


def test_transmittance_is_product_of_single_splats():
    """Untruncated T(u) = prod_i (1 - alpha_i(u)); each alpha_i(u) is measured
    by rendering point i alone.  The product is taken in log space."""
    sc, cam = _random_view(5, n=20)
    full = oracle.render(sc, cam, oracle.Params.untruncated(), mode="brute")
    logT = np.zeros((cam.height, cam.width))
    for i in range(sc.n):
        one = Scene(sc.xyz[i:i + 1], sc.sh[i:i + 1], sc.opacity[i:i + 1], sc.radius[i:i + 1])
        r = oracle.render(one, cam, oracle.Params.untruncated(), mode="brute")
        logT += np.log(r.trans)
    np.testing.assert_allclose(full.trans, np.exp(logT), rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("params", [oracle.Params(), oracle.Params.untruncated(),
                                    oracle.Params(alpha_min=1e-3, t_min=0.3)])
def test_partition_of_unity(params):
    """With every colour = 1 the telescoping sum of Eq. (6)-(7) gives I = 1 - T."""
    sc, cam = _random_view(6, n=64, deg=0)
    sc.sh[:] = np.float32(2 * SQRT_PI)
    # float32(2 sqrt(pi)) / (2 sqrt(pi)) is 1 up to the float32 rounding of h
    c0 = float(np.float32(2 * SQRT_PI)) * Y00
    r = oracle.render(sc, cam, params, mode="brute")
    assert (r.trans < 0.5).any()
    for ch in range(3):
        assert np.abs(r.image[..., ch] - c0 * (1 - r.trans)).max() < 1e-12


def test_linearity_in_sh():
    sc, cam = _random_view(7, n=48)
    r1 = oracle.render(sc, cam, mode="brute")
    sc2 = Scene(sc.xyz, (sc.sh * np.float32(2.0)).astype(np.float32), sc.opacity, sc.radius)
    r2 = oracle.render(sc2, cam, mode="brute")
    assert np.array_equal(r2.trans, r1.trans)
    np.testing.assert_allclose(r2.image, 2 * r1.image, rtol=1e-13, atol=1e-15)


def test_input_permutation_invariance():
    sc, cam = _random_view(8, n=48)
    perm = np.random.default_rng(8).permutation(sc.n)
    zk = oracle.project(sc, cam)["zkey"]
    assert len(np.unique(zk)) == sc.n      # distinct depths -> unique order
    r1 = oracle.render(sc, cam, mode="brute")
    sp = Scene(sc.xyz[perm], sc.sh[perm], sc.opacity[perm], sc.radius[perm])
    r2 = oracle.render(sp, cam, mode="brute")
    assert np.array_equal(r1.image, r2.image) and np.array_equal(r1.trans, r2.trans)


@pytest.mark.parametrize("seed,size", [(9, (32, 32)), (10, (37, 21)), (11, (1, 1)), (12, (64, 9))])
def test_grid_equals_brute_force_bitwise(seed, size):
    sc, cam = _random_view(seed, n=64)
    W, H = size
    cam = Camera(cam.R, cam.t, cam.fx, cam.fy, W / 2, H / 2, W, H)
    a = oracle.render(sc, cam, mode="brute")
    b = oracle.render(sc, cam, mode="grid")
    assert np.array_equal(a.image, b.image) and np.array_equal(a.trans, b.trans)
    assert np.array_equal(a.ncontrib, b.ncontrib)


def test_pixel_subset_matches_full_frame():
    sc, cam = _random_view(13, n=64)
    full = oracle.render(sc, cam, mode="grid")
    pix = np.random.default_rng(13).choice(cam.pixels, 100, replace=False)
    sub = oracle.render(sc, cam, mode="grid", pixels=pix)
    assert np.array_equal(sub.image, full.image.reshape(-1, 3)[pix])
    assert np.array_equal(sub.trans, full.trans.reshape(-1)[pix])


def test_truncation_error_bound():
    """Defaults (alpha_min = t_min = 1e-5) vs the literal untruncated sum:
    |dI| <= 2 (m alpha_min + t_min) max|c| with m splats."""
    sc, cam = _random_view(14, n=64)
    a = oracle.render(sc, cam, mode="brute")
    b = oracle.render(sc, cam, oracle.Params.untruncated(), mode="brute")
    cmax = np.abs(oracle.project(sc, cam)["color"]).max()
    bound = 2 * (sc.n * 1e-5 + 1e-5) * cmax
    assert np.abs(a.image - b.image).max() <= bound
    assert np.abs(a.trans - b.trans).max() <= 2 * (sc.n * 1e-5 + 1e-5)


def test_early_stop_and_near_plane():
    """Opaque stack: stop once T < t_min; points behind the near plane vanish."""
    n = 12
    h = np.tile(np.array([1.0, 1.0, 1.0]) * 2 * SQRT_PI, (n, 1))[:, None, :]
    xyz = np.zeros((n, 3), np.float32)
    xyz[:, 2] = np.arange(n, dtype=np.float32) * 0.01
    sc = _scene(xyz, h, [0.9] * n, 0.03125)
    r = oracle.render(sc, _cam(), mode="brute")
    # T after k splats at the centre = 0.1^k; 0.1^5 = 1e-5 is not < 1e-5, 0.1^6 is
    assert r.ncontrib[8, 8] == 6 and r.stopped[8, 8] == 1
    behind = _scene([[0, 0, -3.2]], h[:1], [0.9], 0.03125)
    rb = oracle.render(behind, _cam(), mode="brute")
    assert np.all(rb.image == 0) and np.all(rb.trans == 1)


# ---------------------------------------------------------------------------
# Gradients: analytic backward vs central finite differences
# ---------------------------------------------------------------------------

def _loss(res, wI, wT):
    return float((res.image * wI).sum() + (res.trans * wT).sum())


@pytest.mark.parametrize("seed,frame,deg", [(20, 0, 2), (21, 1, 3), (22, 0, 1)])
def test_backward_matches_central_differences(seed, frame, deg):
    sc, cam = _random_view(seed, n=24, deg=deg)
    params = oracle.Params(sh_frame=frame)
    rng = np.random.default_rng(seed)
    npix = cam.pixels
    wI = rng.standard_normal((npix, 3))
    wT = rng.standard_normal(npix)
    xyz = sc.xyz.astype(np.float64)
    sh = sc.sh.astype(np.float64)
    op = sc.opacity.astype(np.float64)
    rad = sc.radius.astype(np.float64)
    g = oracle.backward_double(xyz, sh, op, rad, cam, wI, wT, params)

    def structure(x, s, o):
        r = oracle.render_double(x, s, o, rad, cam, params)
        class _S:
            pass
        q = _S()
        q.xyz = x.astype(np.float32)
        return r, oracle.depth_order(q, cam, params)

    base_r, base_order = structure(xyz, sh, op)
    checked = kinked = 0
    for name, arr, h in (("xyz", xyz, 1e-6), ("sh", sh, 1e-3), ("opacity", op, 1e-6)):
        grad = getattr(g, name)
        gmax = np.abs(grad).max()
        flat = arr.reshape(-1)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            rp, op_ = structure(xyz, sh, op)
            flat[j] = old - h
            rm, om_ = structure(xyz, sh, op)
            flat[j] = old
            if not (np.array_equal(rp.ncontrib, rm.ncontrib) and np.array_equal(rp.stopped, rm.stopped)
                    and np.array_equal(op_, om_)):
                kinked += 1
                continue
            fd = (_loss(rp, wI.reshape(rp.image.shape), wT) - _loss(rm, wI.reshape(rm.image.shape), wT)) / (2 * h)
            an = grad.reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * gmax) + 1e-12, (name, j, fd, an)
            checked += 1
    assert kinked <= 0.05 * (checked + kinked)
    assert checked > 0


def _clamp_pairs(xyz, op, rad, cam, alpha_max):
    """(point, pixel) pairs where o G exceeds alpha_max, from a float64
    projection of its own (Eq. 1, sigma = f r / Z).  Used only to find the
    finite-difference pairs that cross the clamp (kinks)."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    X = xyz @ R.T + np.asarray(cam.t, np.float64)
    px = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    py = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    sx = cam.fx * rad / X[:, 2]
    sy = cam.fy * rad / X[:, 2]
    ux = np.arange(cam.width) + 0.5
    uy = np.arange(cam.height) + 0.5
    q = ((px[:, None, None] - ux[None, None, :]) / sx[:, None, None]) ** 2 + \
        ((py[:, None, None] - uy[None, :, None]) / sy[:, None, None]) ** 2
    return op[:, None, None] * np.exp(-0.5 * q) > alpha_max


@pytest.mark.parametrize("seed", [30, 31])
def test_backward_with_clamped_splats_matches_central_differences(seed):
    """Splats whose o G exceeds alpha_max at a pixel centre: there alpha is the
    constant alpha_max, so the loss depends on such a splat's opacity and
    position only through the other pixels it covers, yet its colour still
    enters I and its (1 - alpha_max) still scales everything behind it.  Central
    differences pin every branch of the backward that handles a clamped splat."""
    sc, cam = _random_view(seed, n=24, deg=2)
    params = oracle.Params()
    base = oracle.project(sc, cam)
    rng = np.random.default_rng(seed)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64)
    extra = []
    # six near-opaque splats on pixel centres, each just in front of or just
    # behind one of the scene's splats, so that both orders occur
    inside = base["valid"] & (base["px"] >= 1) & (base["px"] < cam.width - 1) & \
        (base["py"] >= 1) & (base["py"] < cam.height - 1)
    for j, i in enumerate(rng.choice(np.nonzero(inside)[0], 6, replace=False)):
        ux = np.floor(base["px"][i]) + 0.5
        uy = np.floor(base["py"][i]) + 0.5
        Z = base["z"][i] + (-0.02 if j % 2 == 0 else 0.02)
        Xc = np.array([(ux - cam.cx) * Z / cam.fx, (uy - cam.cy) * Z / cam.fy, Z])
        extra.append(R.T @ (Xc - t))
    m = len(extra)
    xyz = np.concatenate([sc.xyz.astype(np.float64), np.array(extra)])
    sh = np.concatenate([sc.sh.astype(np.float64), 0.3 * rng.standard_normal((m, 9, 3))])
    op = np.concatenate([sc.opacity.astype(np.float64), np.full(m, 0.9999)])
    rad = np.concatenate([sc.radius.astype(np.float64), np.full(m, 0.02)])
    clamp0 = _clamp_pairs(xyz, op, rad, cam, params.alpha_max)
    assert clamp0[-m:].any(axis=(1, 2)).all()            # every added splat is clamped somewhere
    npix = cam.pixels
    wI = rng.standard_normal((npix, 3))
    wT = rng.standard_normal(npix)
    g = oracle.backward_double(xyz, sh, op, rad, cam, wI, wT, params)

    def structure():
        r = oracle.render_double(xyz, sh, op, rad, cam, params)

        class _S:
            pass
        q = _S()
        q.xyz = xyz.astype(np.float32)
        return r, oracle.depth_order(q, cam, params), _clamp_pairs(xyz, op, rad, cam, params.alpha_max)

    checked = kinked = 0
    checked_clamped = 0
    for name, arr, h in (("xyz", xyz, 1e-6), ("sh", sh, 1e-3), ("opacity", op, 1e-6)):
        grad = getattr(g, name)
        gmax = np.abs(grad).max()
        flat = arr.reshape(-1)
        per_point = flat.size // xyz.shape[0]
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            rp, op_, cp = structure()
            flat[j] = old - h
            rm, om_, cm = structure()
            flat[j] = old
            if not (np.array_equal(rp.ncontrib, rm.ncontrib) and np.array_equal(rp.stopped, rm.stopped)
                    and np.array_equal(op_, om_) and np.array_equal(cp, cm)):
                kinked += 1
                continue
            fd = (_loss(rp, wI.reshape(rp.image.shape), wT) - _loss(rm, wI.reshape(rm.image.shape), wT)) / (2 * h)
            an = grad.reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * gmax) + 1e-12, (name, j, fd, an)
            checked += 1
            checked_clamped += j // per_point >= xyz.shape[0] - m
    assert kinked <= 0.05 * (checked + kinked)
    assert checked_clamped >= 0.9 * m * 31


@pytest.mark.slow
@pytest.mark.parametrize("which", ["ball100k_8x400", "surface300k_4x800"])
def test_float32_depth_key_is_a_faithful_rounding_of_camera_z(which):
    """Sec. 3.2 sorts by camera-space z.  The depth order decides in float32, on
    the key fmaf(R20, x, fmaf(R21, y, fmaf(R22, z, t2))): three roundings, each
    at most half an ulp32 of a partial sum bounded by
    M = |t2| + |R22 z| + |R21 y| + |R20 x|, so |key - Z| <= e = 1.5 ulp32(M)
    against Z computed in float64 from the same float32 inputs.  Checked here
    point by point; the cull keeps exactly the points with Z > z_near; and a
    point earlier in the key order is never farther than a later one by more
    than the two points' bounds: the key order is the order of camera Z except
    between points whose Z differ by less than that (near-ties)."""
    if which == "ball100k_8x400":
        scene, cams, _, _ = workloads.ball100k_8x400()
    else:
        scene, cams, _ = workloads.surface300k_4x800()
    z_near = oracle.Params().z_near
    xyz = scene.xyz.astype(np.float64)
    swapped = 0
    for cam in cams[:4]:
        R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
        t = np.asarray(cam.t, np.float32).astype(np.float64)
        Z = xyz @ R[2] + t[2]
        M = np.abs(t[2]) + np.abs(xyz) @ np.abs(R[2])
        e = 1.5 * np.spacing(M.astype(np.float32)).astype(np.float64)
        zk = oracle.project(scene, cam)["zkey"].astype(np.float64)
        assert (np.abs(zk - Z) <= e).all()
        assert np.abs(zk - Z).max() > 0          # the key really is rounded
        order = oracle.depth_order(scene, cam)
        assert np.array_equal(np.sort(order), np.nonzero(Z > z_near)[0])
        Zo = Z[order]
        run_max = np.maximum.accumulate(Zo)
        assert (run_max[:-1] - Zo[1:] <= e.max() + e[order][1:]).all()
        exact = np.lexsort((order, Zo))           # float64 order, ties by index
        swapped += int((order[exact] != order).sum())
    print(f"{which}: {swapped} of {4 * len(xyz)} positions differ between the float32 and float64 orders")
