"""CPU build of the video warm-start kernels (Sec. 3.4: Chamfer distance of
Eq. (9) and its gradient, top-k SH transfer, Adam step) under
AddressSanitizer and UndefinedBehaviorSanitizer, against the oracle: nearest
and top-k indices and the SH means bit for bit; Eq. (9) to 1e-12; the
gradient and the Adam step to float32 rounding.  GPU code generation is
checked by the GPU parity tests of the same cases."""
import os

import numpy as np
import pytest

import oracle
import workloads
from _hostbuild import compile_harness, run


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return compile_harness("chamfer_host", tmp_path_factory.mktemp("hostbuild"))


def _read(d, name, dtype, shape):
    return np.fromfile(os.path.join(str(d), name), dtype).reshape(shape)


def _clouds(n1, n2, seed, dup=False):
    rng = np.random.default_rng(seed)
    s1 = rng.random((n1, 3)).astype(np.float32)
    s2 = (rng.random((n2, 3)) * 1.1 - 0.05).astype(np.float32)
    if dup:
        s2[: min(n1, n2) // 3] = s1[: min(n1, n2) // 3]       # exact coincidences
        if n1 > 9:
            s1[5:9] = s1[4]                                   # ties inside s1
    return s1, s2


def check_chamfer(d, s1, s2):
    cd = float(_read(d, "cd.bin", np.float64, (1,))[0])
    g = _read(d, "grad2.bin", np.float32, (-1, 3))
    nn12 = _read(d, "nn12.bin", np.int32, (-1,))
    nn21 = _read(d, "nn21.bin", np.int32, (-1,))
    r12, _ = oracle.chamfer_nn(s1, s2)
    r21, _ = oracle.chamfer_nn(s2, s1)
    assert np.array_equal(nn12, r12) and np.array_equal(nn21, r21)
    rcd, rg = oracle.chamfer(s1, s2)
    assert cd == pytest.approx(rcd, rel=1e-12, abs=1e-300)
    np.testing.assert_allclose(g, rg, rtol=1e-6, atol=1e-7 * max(np.abs(rg).max(), 1e-30))


@pytest.mark.parametrize("n1,n2,dup", [(3000, 2500, False), (2000, 9000, True), (1, 700, False), (900, 1, False),
                                       (4097, 4096, True)])
def test_chamfer(exe, tmp_path, n1, n2, dup):
    s1, s2 = _clouds(n1, n2, n1 + n2, dup)
    run(exe, tmp_path, "chamfer", {"s1": s1, "s2": s2})
    check_chamfer(tmp_path, s1, s2)


@pytest.mark.parametrize("n1,n2,K", [(2000, 300, 1), (2000, 300, 5), (1500, 160, 12), (1500, 129, 32), (3, 50, 8),
                                       (7, 40, 16)])
def test_topk(exe, tmp_path, n1, n2, K):
    s1, s2 = _clouds(n1, n2, K, dup=True)
    sh1 = workloads.point_attributes(n1, 2, K)[0]
    run(exe, tmp_path, "topk", {"s1": s1, "sh1": sh1, "s2": s2}, 27, K)
    out = _read(tmp_path, "out_sh.bin", np.float32, (n2, 9, 3))
    idx = _read(tmp_path, "idx.bin", np.int32, (n2, K))
    rout, ridx = oracle.topk_sh(s1, sh1, s2, K)
    assert np.array_equal(idx, ridx)
    assert np.array_equal(out, rout.astype(np.float32))


def test_adam(exe, tmp_path):
    rng = np.random.default_rng(9)
    n = 1000
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = rng.random(n).astype(np.float32) * 0.01
    run(exe, tmp_path, "adam", {"p": p, "g": g, "m": m, "v": v}, 3, "0.001", "0.9", "0.999", "1e-8")
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the kernel receives the hyperparameters as float32 (1 - b rounds exactly there)
    f = lambda x: float(np.float32(x))
    oracle.adam_step(rp, g.astype(np.float64), rm, rv, 3, f(0.001), f(0.9), f(0.999), f(1e-8))
    np.testing.assert_allclose(_read(tmp_path, "p.bin", np.float32, (n,)), rp, rtol=1e-6, atol=1e-7)
    # m = b1 m + (1 - b1) g cancels where the terms have opposite signs: float32
    # rounding of the terms (|terms| <= 0.4 here), not of the result, bounds it
    np.testing.assert_allclose(_read(tmp_path, "m.bin", np.float32, (n,)), rm, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(_read(tmp_path, "v.bin", np.float32, (n,)), rv, rtol=1e-5, atol=1e-9)
