"""Pins of the oracle's hybrid coarse-to-fine update (Sec. 3.3, Alg. 1):
hand-worked cases, numpy/scipy reimplementations of special cases, and
invariants.  None re-types the oracle's loops."""
import numpy as np
import pytest

import oracle


def _cloud(xyz, sh=None, op=None, rad=None, k=9):
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    n = xyz.shape[0]
    rng = np.random.default_rng(n)
    sh = rng.standard_normal((n, k, 3)).astype(np.float32) if sh is None else np.asarray(sh, np.float32)
    op = rng.random(n).astype(np.float32) if op is None else np.asarray(op, np.float32)
    rad = rng.uniform(0.01, 0.03, n).astype(np.float32) if rad is None else np.asarray(rad, np.float32)
    return oracle.Cloud(xyz, sh, op, rad)


# ---------------------------------------------------------------------------
# voxel reduction
# ---------------------------------------------------------------------------

def test_voxel_reduce_hand_example():
    """bbox [0, 4]^3, N = 2 (voxel edge 2): (0,0,0), (0.5,0.5,0.5), (1.5,1.5,1.5)
    share voxel 0; (3,1,0) is voxel ix=1 -> key 1; (4,4,4) sits on the upper
    face and is clamped into voxel 7."""
    xyz = [[0, 0, 0], [0.5, 0.5, 0.5], [1.5, 1.5, 1.5], [4, 4, 4], [3, 1, 0]]
    op = [0.1, 0.2, 0.3, 0.4, 0.5]
    rad = [1, 2, 3, 4, 5]
    sh = np.arange(5 * 1 * 3, dtype=np.float32).reshape(5, 1, 3)
    red = oracle.voxel_reduce(_cloud(xyz, sh, op, rad, k=1), 2)
    assert red.n == 3
    np.testing.assert_allclose(red.xyz, [[2 / 3, 2 / 3, 2 / 3], [3, 1, 0], [4, 4, 4]], atol=1e-7)
    np.testing.assert_allclose(red.opacity, [0.2, 0.5, 0.4], atol=1e-7)
    np.testing.assert_allclose(red.radius, [2, 5, 4])
    np.testing.assert_allclose(red.sh[:, 0], [[3, 4, 5], [12, 13, 14], [9, 10, 11]])


def test_voxel_reduce_matches_numpy_grouping():
    """Per-voxel means equal numpy's bincount means over the voxel keys."""
    rng = np.random.default_rng(1)
    n = 3000
    c = _cloud(rng.uniform(-1, 2, (n, 3)))
    N = 7
    keys = oracle.voxel_keys(c.xyz, N)
    uk, inv, cnt = np.unique(keys, return_inverse=True, return_counts=True)
    red = oracle.voxel_reduce(c, N)
    assert red.n == len(uk)
    for a in range(3):
        np.testing.assert_allclose(red.xyz[:, a], np.bincount(inv, c.xyz[:, a].astype(np.float64)) / cnt, rtol=1e-12)
    np.testing.assert_allclose(red.opacity, np.bincount(inv, c.opacity.astype(np.float64)) / cnt, rtol=1e-12)
    sh = c.sh.reshape(n, -1).astype(np.float64)
    for q in range(sh.shape[1]):
        np.testing.assert_allclose(red.sh.reshape(red.n, -1)[:, q], np.bincount(inv, sh[:, q]) / cnt, rtol=1e-9,
                                   atol=1e-12)
    # keys: every coordinate's cell is floor of its normalised position
    lo, hi = c.xyz.min(0), c.xyz.max(0)
    ix = np.clip(np.floor((c.xyz - lo) * (np.float32(N) / (hi - lo))), 0, N - 1).astype(np.uint64)
    assert np.array_equal(keys, (ix[:, 2] * N + ix[:, 1]) * N + ix[:, 0])


def test_voxel_reduce_single_voxel_is_the_mean():
    rng = np.random.default_rng(2)
    c = _cloud(rng.standard_normal((100, 3)))
    red = oracle.voxel_reduce(c, 1)
    assert red.n == 1
    np.testing.assert_allclose(red.xyz[0], c.xyz.astype(np.float64).mean(0), rtol=1e-12)
    np.testing.assert_allclose(red.radius[0], c.radius.astype(np.float64).mean(), rtol=1e-12)


def test_voxel_reduce_is_permutation_invariant():
    rng = np.random.default_rng(3)
    c = _cloud(rng.random((500, 3)))
    perm = rng.permutation(500)
    p = oracle.Cloud(c.xyz[perm], c.sh[perm], c.opacity[perm], c.radius[perm])
    a, b = oracle.voxel_reduce(c, 5), oracle.voxel_reduce(p, 5)
    np.testing.assert_allclose(a.xyz, b.xyz, rtol=1e-12)
    np.testing.assert_allclose(a.sh, b.sh, rtol=1e-10, atol=1e-13)


# ---------------------------------------------------------------------------
# neighbours and the spread test
# ---------------------------------------------------------------------------

def test_knn_matches_numpy_lexsort():
    """Same float32 distance expression evaluated by numpy, ordered by
    (distance, index) with lexsort."""
    rng = np.random.default_rng(4)
    x = rng.random((300, 3)).astype(np.float32)
    x[10] = x[11]                      # an exact duplicate: distance 0 ties
    K = 7
    idx, d2 = oracle.knn(x, K)
    for i in range(300):
        d = x - x[i]
        dd = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        j = np.arange(300)
        order = np.lexsort((j, dd))
        order = order[order != i][:K]
        assert np.array_equal(idx[i], order), i
        assert np.array_equal(d2[i], dd[order])


def test_knn_on_lattice_matches_kdtree():
    """Integer lattice points with distinct distances from a query: scipy's
    KD-tree gives the same neighbour sets."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(5)
    x = rng.choice(40, size=(400, 3)).astype(np.float32) * np.array([1, 3, 7], np.float32)
    x = np.unique(x, axis=0)
    K = 5
    idx, _ = oracle.knn(x, K)
    dist, ref = cKDTree(x.astype(np.float64)).query(x.astype(np.float64), k=K + 2)
    checked = 0
    for i in range(x.shape[0]):
        # distinct distances among the first K neighbours and a strict gap to the next
        if len(np.unique(dist[i, :K + 1])) == K + 1 and dist[i, K] < dist[i, K + 1]:
            assert np.array_equal(idx[i], ref[i, 1:K + 1]), i
            checked += 1
    assert checked > x.shape[0] // 4


def test_knn_few_points():
    idx, d2 = oracle.knn(np.array([[0, 0, 0], [1, 0, 0]], np.float32), 4)
    assert list(idx[0]) == [1, -1, -1, -1] and list(idx[1]) == [0, -1, -1, -1]
    assert d2[0, 0] == 1.0


def test_spread_removes_the_outlier():
    """A ring of 8 points at radius 1 around the origin plus the origin (their
    nearest neighbours are all at comparable distances), and one far point whose
    neighbours are at distances spread far apart: only the far point has
    delta > eps, with delta equal to numpy's population std."""
    ang = np.arange(8) * np.pi / 4
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(8)], 1)
    pts = np.concatenate([ring, [[0, 0, 0]], [[10, 0, 0]]]).astype(np.float32)
    K = 4
    idx, d2 = oracle.knn(pts, K)
    far = np.sqrt(d2[9].astype(np.float64))
    delta_far = np.std(far)
    assert delta_far > 0.05
    keep, out = oracle.filter_generate(_cloud(pts), K, eps=0.05)
    assert not keep[9]
    keep2, _ = oracle.filter_generate(_cloud(pts), K, eps=float(delta_far) + 1e-3)
    assert keep2[9]


def test_spread_decisions_match_numpy_std():
    """Clusters plus scattered points: every keep/remove decision equals
    numpy's population standard deviation of the neighbour distances against
    eps (points within 1e-5 of eps are left out)."""
    rng = np.random.default_rng(7)
    centres = rng.random((6, 3))
    pts = np.concatenate([c + 0.02 * rng.standard_normal((60, 3)) for c in centres] +
                         [rng.random((40, 3))]).astype(np.float32)
    K = 6
    _, d2 = oracle.knn(pts, K)
    delta = np.std(np.sqrt(d2.astype(np.float64)), axis=1)
    eps = float(np.median(delta))
    keep, _ = oracle.filter_generate(_cloud(pts), K, eps)
    clear = np.abs(delta - eps) > 1e-5
    assert clear.sum() > 0.9 * len(pts)
    assert np.array_equal(keep[clear], (delta <= eps)[clear])
    assert 0 < keep.sum() < len(pts)


# ---------------------------------------------------------------------------
# generation
# ---------------------------------------------------------------------------

def test_generation_on_a_line():
    """Points at x = 0..9 on a line, K = 2, eps large (nothing removed): an
    interior point's neighbours are x - 1 and x + 1 (a tie at distance 1), so its
    generated point sits on it; the end points generate 1.5 and 7.5."""
    x = np.zeros((10, 3), np.float32)
    x[:, 0] = np.arange(10)
    op = np.linspace(0.1, 1.0, 10).astype(np.float32)
    keep, out = oracle.filter_generate(_cloud(x, op=op), 2, eps=1e9)
    assert keep.all() and out.n == 20
    np.testing.assert_allclose(out.xyz[:10], x)
    gx = out.xyz[10:, 0]
    np.testing.assert_allclose(gx, [1.5] + list(range(1, 9)) + [7.5])
    np.testing.assert_allclose(out.opacity[11], (op[0] + op[2]) / 2, rtol=1e-7)


def test_generated_points_use_the_kept_set_only():
    """A removed point is nobody's neighbour in the generation step."""
    ang = np.arange(8) * np.pi / 4
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(8)], 1)
    pts = np.concatenate([ring, [[0, 0, 0]], [[10, 0, 0]]]).astype(np.float32)
    keep, out = oracle.filter_generate(_cloud(pts), 4, eps=0.05)
    assert not keep[9]
    assert (out.xyz[:, 0] < 5).all()


def test_hybrid_update_composes_the_steps():
    rng = np.random.default_rng(6)
    c = _cloud(rng.random((800, 3)))
    red, keep, out = oracle.hybrid_update(c, 6, 6, 0.02)
    red32 = red.astype(np.float32)
    k2, out2 = oracle.filter_generate(red32, 6, 0.02)
    assert np.array_equal(keep, k2)
    np.testing.assert_array_equal(out.xyz, out2.xyz)
    assert out.n == keep.sum() * 2 if keep.sum() >= 2 else keep.sum()
