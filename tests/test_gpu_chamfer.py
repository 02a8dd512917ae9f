"""GPU parity of the video warm start (Sec. 3.4): Chamfer distance of
Eq. (9) and its gradient, top-k SH transfer and Adam step, through the C ABI,
against the oracle: nearest and top-k indices and SH means bit for bit (the
same float32 distances and FP64 sums in the same order); Eq. (9) to 1e-12;
gradient and Adam to float32 rounding."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_14330_amd as d
    d.load()
    from paper_2205_14330_amd import chamfer as c
    return c


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _clouds(n1, n2, seed, dup=False):
    rng = np.random.default_rng(seed)
    s1 = rng.random((n1, 3)).astype(np.float32)
    s2 = (rng.random((n2, 3)) * 1.1 - 0.05).astype(np.float32)
    if dup:
        s2[: min(n1, n2) // 3] = s1[: min(n1, n2) // 3]
        if n1 > 9:
            s1[5:9] = s1[4]
    return s1, s2


@pytest.mark.parametrize("n1,n2,dup", [(3000, 2500, False), (2000, 9000, True), (1, 700, False), (900, 1, False),
                                       (4097, 4096, True), (12000, 15000, False)])
def test_chamfer_matches_oracle(cf, n1, n2, dup):
    s1, s2 = _clouds(n1, n2, n1 + n2, dup)
    out = cf.chamfer(_t(s1), _t(s2), grad=True, nn=True)
    r12, _ = oracle.chamfer_nn(s1, s2)
    r21, _ = oracle.chamfer_nn(s2, s1)
    assert np.array_equal(out["nn12"].cpu().numpy(), r12)
    assert np.array_equal(out["nn21"].cpu().numpy(), r21)
    rcd, rg = oracle.chamfer(s1, s2)
    assert float(out["cd"].cpu()[0]) == pytest.approx(rcd, rel=1e-12)
    np.testing.assert_allclose(out["grad2"].cpu().numpy(), rg, rtol=1e-6, atol=1e-7 * np.abs(rg).max())


@pytest.mark.parametrize("n1,n2,K", [(2000, 300, 1), (2000, 300, 5), (1500, 160, 12), (1500, 129, 32), (3, 50, 8),
                                       (7, 40, 16), (6000, 1000, 4)])
def test_topk_sh_matches_oracle(cf, n1, n2, K):
    s1, s2 = _clouds(n1, n2, K, dup=True)
    sh1 = workloads.point_attributes(n1, 2, K)[0]
    out, idx = cf.topk_sh(_t(s1), _t(sh1), _t(s2), K, with_index=True)
    rout, ridx = oracle.topk_sh(s1, sh1, s2, K)
    assert np.array_equal(idx.cpu().numpy(), ridx)
    assert np.array_equal(out.cpu().numpy(), rout.astype(np.float32))


def test_adam_matches_oracle(cf):
    rng = np.random.default_rng(9)
    n = 10007
    p, g = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    m, v = (0.1 * rng.standard_normal(n)).astype(np.float32), (rng.random(n) * 0.01).astype(np.float32)
    tp, tg, tm, tv = _t(p), _t(g), _t(m), _t(v)
    cf.adam_step(tp, tg, tm, tv, 3, 1e-3)
    f = lambda x: float(np.float32(x))
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    oracle.adam_step(rp, g.astype(np.float64), rm, rv, 3, f(1e-3), f(0.9), f(0.999), f(1e-8))
    np.testing.assert_allclose(tp.cpu().numpy(), rp, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(tm.cpu().numpy(), rm, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), rv, rtol=1e-5, atol=1e-9)


def test_warm_start_lowers_the_chamfer_distance(cf):
    """Consecutive frames of the dynamic workload: the refined positions of
    frame 2 are closer to frame 1 in the sense of Eq. (9), and the autograd
    form gives the same gradient as the direct call."""
    import torch
    scenes, _, _ = workloads.dynamic30x200k_1024x768(frames=2, n=20000)
    s1 = _t(scenes[0].xyz)
    rng = np.random.default_rng(0)
    s2 = _t(scenes[1].xyz + 0.01 * rng.standard_normal(scenes[1].xyz.shape))
    cd0 = float(cf.chamfer(s1, s2)["cd"].cpu()[0])
    p, sh = cf.warm_start(s1, _t(scenes[0].sh), s2, steps=20, lr=1e-3, K=4)
    assert float(cf.chamfer(s1, p)["cd"].cpu()[0]) < cd0
    assert sh.shape == (20000, 9, 3) and torch.isfinite(sh).all()
    x = s2.clone().requires_grad_(True)
    cd = cf.ChamferFn.apply(s1, x)
    cd.backward()
    assert torch.equal(x.grad, cf.chamfer(s1, s2)["grad2"])
