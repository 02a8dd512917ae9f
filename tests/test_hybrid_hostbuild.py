"""CPU build of the hybrid-update kernels (Sec. 3.3, Alg. 1) under
AddressSanitizer and UndefinedBehaviorSanitizer.

The kernels and host sequencing of the HIP source compile unchanged with g++
against a host stand-in of the HIP runtime (tests/hostbuild): the threads of
a block run concurrently on host threads, every scratch array is its own
allocation of exactly the size the library reserves, filled with 0xFF, and
the library's own flat scan and radix sort (sort.hip) run with their real
launch sequence.  The outputs must equal the oracle's bit for bit.

This checks the kernels' indexing, the scratch sizes and the float32 decision
arithmetic on the CPU; the GPU's own code generation is checked by the GPU
parity tests of the same cases."""
import os

import numpy as np
import pytest

import oracle
import workloads
from _hostbuild import compile_harness, run


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return compile_harness("hybrid_host", tmp_path_factory.mktemp("hostbuild"))


def _run(exe, d, mode, arrays, *args):
    run(exe, d, mode, {k: np.asarray(v, np.float32) for k, v in arrays.items()}, *args)


def _cloud(xyz, seed):
    xyz = np.asarray(xyz, np.float32)
    return oracle.Cloud(xyz, *workloads.point_attributes(xyz.shape[0], 2, seed))


def _arrays(c):
    return {"xyz": c.xyz, "sh": c.sh, "op": c.opacity, "rad": c.radius}


def _read_cloud(d, count, k3):
    r = lambda name, shape: np.fromfile(os.path.join(d, name), np.float32).reshape(shape)
    return (r("out_xyz.bin", (count, 3)), r("out_sh.bin", (count, k3 // 3, 3)), r("out_op.bin", (count,)),
            r("out_rad.bin", (count,)))


def _assert_equal(got, ref, label):
    for g, r, name in zip(got, (ref.xyz, ref.sh, ref.opacity, ref.radius), ("xyz", "sh", "opacity", "radius")):
        r32 = np.asarray(r).astype(np.float32)
        assert g.shape == r32.shape, (label, name, g.shape, r32.shape)
        bad = g != r32
        assert not bad.any(), (label, name, int(bad.sum()))


def _eps_arg(eps):
    return repr(float(np.float32(eps)))


@pytest.mark.parametrize("name", ["uniform", "clusters", "duplicates", "flat", "line"])
@pytest.mark.parametrize("K", [1, 8, 32])
def test_knn(exe, tmp_path, name, K):
    x = workloads.hybrid_clouds()[name]
    _run(exe, tmp_path, "knn", {"xyz": x}, K)
    idx = np.fromfile(tmp_path / "idx.bin", np.int32).reshape(-1, K)
    d2 = np.fromfile(tmp_path / "d2.bin", np.float32).reshape(-1, K)
    ridx, rd2 = oracle.knn(x, K)
    assert np.array_equal(idx, ridx.astype(np.int32)), name
    assert np.array_equal(d2, rd2), name


@pytest.mark.parametrize("m", [1, 2, 3, 9])
def test_knn_fewer_points_than_k(exe, tmp_path, m):
    x = np.random.default_rng(m).random((m, 3)).astype(np.float32)
    _run(exe, tmp_path, "knn", {"xyz": x}, 8)
    ridx, rd2 = oracle.knn(x, 8)
    assert np.array_equal(np.fromfile(tmp_path / "idx.bin", np.int32).reshape(-1, 8), ridx.astype(np.int32))
    assert np.array_equal(np.fromfile(tmp_path / "d2.bin", np.float32).reshape(-1, 8), rd2)


@pytest.mark.parametrize("name,N", [("uniform", 16), ("clusters", 64), ("duplicates", 8), ("flat", 32),
                                    ("line", 1000), ("uniform", 1)])
def test_voxel_reduce(exe, tmp_path, name, N):
    c = _cloud(workloads.hybrid_clouds()[name], seed=N)
    _run(exe, tmp_path, "voxel", _arrays(c), N, 27)
    m = int(open(tmp_path / "counts.txt").read().split()[0])
    ref = oracle.voxel_reduce(c, N)
    assert m == ref.n
    _assert_equal(_read_cloud(tmp_path, m, 27), ref, f"{name} N={N}")


def test_voxel_reduce_last_point_inside_a_voxel(exe, tmp_path):
    """The last point in voxel order shares its voxel with the one before it,
    so the end of the last voxel is not marked by a voxel start (the case that
    once left that end unset)."""
    x = workloads.hybrid_clouds()["uniform"]
    for N in (1, 3):
        keys = np.sort(oracle.voxel_keys(x, N))
        assert keys[-1] == keys[-2]
        c = _cloud(x, seed=N)
        _run(exe, tmp_path, "voxel", _arrays(c), N, 27)
        m = int(open(tmp_path / "counts.txt").read().split()[0])
        ref = oracle.voxel_reduce(c, N)
        assert m == ref.n
        _assert_equal(_read_cloud(tmp_path, m, 27), ref, f"N={N}")


@pytest.mark.parametrize("name,N,K,eps", [("uniform", 16, 8, 0.01), ("clusters", 48, 6, 0.004),
                                          ("duplicates", 8, 4, 0.02), ("flat", 24, 10, 0.01),
                                          ("line", 1000, 2, 1e-3), ("clusters", 32, 32, 0.02),
                                          ("clusters", 32, 32, 0.0)])
def test_hybrid_update(exe, tmp_path, name, N, K, eps):
    c = _cloud(workloads.hybrid_clouds()[name], seed=K)
    _run(exe, tmp_path, "hybrid", _arrays(c), N, K, _eps_arg(eps), 27)
    m, kept, count = (int(v) for v in open(tmp_path / "counts.txt").read().split())
    red, keep, ref = oracle.hybrid_update(c, N, K, eps)
    assert (m, kept, count) == (red.n, int(keep.sum()), ref.n)
    # eps = 0 removes every point whose neighbour distances are not all equal
    assert (kept == 0) == (eps == 0.0) and (kept < red.n or name == "line")
    _assert_equal(_read_cloud(tmp_path, count, 27), ref, f"{name} N={N} K={K}")


@pytest.mark.parametrize("deg", [0, 1, 3])
def test_hybrid_update_other_sh_degrees(exe, tmp_path, deg):
    """The row kernels have one instance per SH row length (3, 12, 27 and 48
    floats); the other cases use degree 2."""
    xyz = np.asarray(workloads.hybrid_clouds()["clusters"], np.float32)
    c = oracle.Cloud(xyz, *workloads.point_attributes(xyz.shape[0], deg, 5))
    k3 = 3 * (deg + 1) ** 2
    _run(exe, tmp_path, "hybrid", _arrays(c), 32, 8, _eps_arg(0.01), k3)
    m, kept, count = (int(v) for v in open(tmp_path / "counts.txt").read().split())
    red, keep, ref = oracle.hybrid_update(c, 32, 8, 0.01)
    assert (m, kept, count) == (red.n, int(keep.sum()), ref.n)
    _assert_equal(_read_cloud(tmp_path, count, k3), ref, f"deg={deg}")


@pytest.mark.parametrize("n", [1, 2])
def test_hybrid_update_tiny_clouds(exe, tmp_path, n):
    c = _cloud(np.arange(3 * n, dtype=np.float32).reshape(n, 3), seed=0)
    _run(exe, tmp_path, "hybrid", _arrays(c), 4, 8, _eps_arg(0.5), 27)
    m, kept, count = (int(v) for v in open(tmp_path / "counts.txt").read().split())
    red, keep, ref = oracle.hybrid_update(c, 4, 8, 0.5)
    assert count == ref.n
    _assert_equal(_read_cloud(tmp_path, count, 27), ref, f"n={n}")
