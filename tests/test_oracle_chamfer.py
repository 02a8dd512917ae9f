"""Pins of the video warm-start oracle (Sec. 3.4): the Chamfer distance of
Eq. (9), its gradient with respect to the next frame's positions, the top-k SH
transfer and the Adam step.  Hand-worked values, central differences, scipy's
KD-tree, numpy brute force of the same float32 distance, and Adam's closed-form
first step; none re-types the oracle's loops."""
import numpy as np
import pytest

import oracle


def test_chamfer_hand_example():
    """S1 = {0}, S2 = {(1,0,0), (0,2,0)}: term 1 = min(1, 4) = 1, term 2 =
    (1 + 4) / 2, CD = 3.5.  Gradient: y1 is the nearest of x (2/1 (y1 - x))
    and its own nearest is x (2/2 (y1 - x)): (3, 0, 0); y2: 2/2 (y2 - x) =
    (0, 2, 0)."""
    cd, g = oracle.chamfer([[0, 0, 0]], [[1, 0, 0], [0, 2, 0]])
    assert cd == pytest.approx(3.5, rel=1e-15)
    np.testing.assert_allclose(g, [[3, 0, 0], [0, 2, 0]], atol=1e-15)


def test_chamfer_of_a_cloud_with_itself_is_zero_and_symmetric():
    rng = np.random.default_rng(0)
    a = rng.random((300, 3)).astype(np.float32)
    b = rng.random((250, 3)).astype(np.float32)
    assert oracle.chamfer(a, a)[0] == 0.0
    assert oracle.chamfer(a, b)[0] == pytest.approx(oracle.chamfer(b, a)[0], rel=1e-14)


def test_chamfer_gradient_central_differences():
    """Generic positions (no near ties): each coordinate of S2 moved by +-h
    changes CD by 2 h dCD/dy up to O(h^2) (the neighbour assignments do not
    change for h far below the gaps)."""
    rng = np.random.default_rng(1)
    a = rng.random((40, 3)).astype(np.float64)
    b = rng.random((30, 3)).astype(np.float64)
    _, g = oracle.chamfer(a.astype(np.float32), b.astype(np.float32))
    h = 1e-3
    checked = 0
    for j in range(30):
        for c in range(3):
            bp, bm = b.copy(), b.copy()
            bp[j, c] += h
            bm[j, c] -= h
            fp = oracle.chamfer(a.astype(np.float32), bp.astype(np.float32))[0]
            fm = oracle.chamfer(a.astype(np.float32), bm.astype(np.float32))[0]
            # float32 positions: the step is rounded; divide by the rounded step
            step = (bp[j, c].astype(np.float32) - bm[j, c].astype(np.float32)).astype(np.float64)
            num = (fp - fm) / step
            assert num == pytest.approx(g[j, c], rel=2e-3, abs=2e-4), (j, c)
            checked += 1
    assert checked == 90


def test_nearest_neighbours_match_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(2)
    a = rng.random((2000, 3)).astype(np.float32)
    b = rng.random((1500, 3)).astype(np.float32)
    nn, d2 = oracle.chamfer_nn(a, b)
    dist, ref = cKDTree(b.astype(np.float64)).query(a.astype(np.float64), k=2)
    clear = (dist[:, 1] - dist[:, 0]) > 1e-5
    assert clear.mean() > 0.99
    assert np.array_equal(nn[clear], ref[clear, 0])
    np.testing.assert_allclose(np.sqrt(d2.astype(np.float64)), dist[:, 0], rtol=1e-6, atol=1e-7)


def test_nearest_ties_go_to_the_lower_index():
    nn, _ = oracle.chamfer_nn([[0, 0, 0]], [[1, 0, 0], [0, 1, 0], [-1, 0, 0]])
    assert nn[0] == 0


def test_topk_matches_numpy_lexsort():
    """Same float32 distance expression evaluated by numpy, ordered by
    (distance, index); the SH mean of those k in FP64."""
    rng = np.random.default_rng(3)
    s1 = rng.random((200, 3)).astype(np.float32)
    s1[7] = s1[8]                                   # an exact tie
    sh1 = rng.standard_normal((200, 9, 3)).astype(np.float32)
    s2 = rng.random((50, 3)).astype(np.float32)
    out, idx = oracle.topk_sh(s1, sh1, s2, 5)
    for i in range(50):
        d = s1 - s2[i]
        dd = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        order = np.lexsort((np.arange(200), dd))[:5]
        assert np.array_equal(idx[i], order)
        np.testing.assert_allclose(out[i], sh1[order].astype(np.float64).mean(0), rtol=1e-13, atol=1e-14)


def test_topk_with_fewer_points_than_k():
    out, idx = oracle.topk_sh([[0, 0, 0], [1, 0, 0]], np.array([[[1, 2, 3]], [[3, 4, 5]]], np.float32),
                              [[0.9, 0, 0]], 4)
    assert list(idx[0]) == [1, 0, -1, -1]
    np.testing.assert_allclose(out[0, 0], [2, 3, 4])


def test_adam_first_step_closed_form():
    """At t = 1 with zero moments, m^ = g and v^ = g^2, so the step is
    lr g / (|g| + eps): lr times the sign of g for |g| >> eps."""
    g = np.array([3.0, -0.5, 1e-3, -2e-9, 0.0])
    p = np.zeros(5); m = np.zeros(5); v = np.zeros(5)
    oracle.adam_step(p, g, m, v, 1, 0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert p[0] == pytest.approx(-0.01, rel=1e-8) and p[1] == pytest.approx(0.01, rel=1e-7)


def test_adam_minimises_the_chamfer_distance():
    """Adam on S2 positions lowers Eq. (9) (the warm-start refinement)."""
    rng = np.random.default_rng(4)
    s1 = rng.random((300, 3)).astype(np.float32)
    s2 = (s1[:250] + 0.05 * rng.standard_normal((250, 3))).astype(np.float64)
    m = np.zeros_like(s2); v = np.zeros_like(s2)
    cd0 = oracle.chamfer(s1, s2.astype(np.float32))[0]
    for t in range(1, 101):
        _, g = oracle.chamfer(s1, s2.astype(np.float32))
        oracle.adam_step(s2, np.ascontiguousarray(g), m, v, t, 2e-3)
    assert oracle.chamfer(s1, s2.astype(np.float32))[0] < 0.5 * cd0
