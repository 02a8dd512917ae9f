"""CPU build of the visual-hull / consistency-check kernels (Sec. 3.1
initialisation, the appendix's consistency check) under AddressSanitizer and
UndefinedBehaviorSanitizer: hull.hip compiles unchanged against the host
stand-in of the HIP runtime (tests/hostbuild); inputs, masks and outputs are
exact-size allocations and the padding after every workspace region is
poisoned.  Results must equal the oracle's bit for bit.  GPU code generation
is checked by the GPU parity tests of the same cases."""
import os

import numpy as np
import pytest

import oracle
import workloads
from _hostbuild import compile_harness, run


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return compile_harness("hull_host", tmp_path_factory.mktemp("hostbuild"))


def _tables(cams, masks):
    cam = np.stack([oracle.cam_array(c) for c in cams]).astype(np.float32)
    dims = np.array([[m.shape[1], m.shape[0]] for m in masks], np.int32)
    return {"cams": cam, "dims": dims, "masks": np.concatenate([np.ascontiguousarray(m, np.uint8).ravel()
                                                                for m in masks])}


def _noisy_masks(cams, seed, frac=0.8):
    rng = np.random.default_rng(seed)
    return [(rng.random((c.height, c.width)) < frac).astype(np.uint8) for c in cams]


def _read(d, name, dtype, shape):
    return np.fromfile(os.path.join(str(d), name), dtype).reshape(shape)


BOX = np.array([-1, -1, -1, 1, 1, 1], np.float32)


@pytest.mark.parametrize("n,capacity", [(5000, None), (5000, 7), (5000, 0), (1, None), (0, None), (1024, None)])
def test_sample(exe, tmp_path, n, capacity):
    cams = workloads.disc_views(8, size=72)
    masks = workloads.sphere_masks(cams, 0.6)
    cap = n if capacity is None else capacity
    run(exe, tmp_path, "sample", dict(_tables(cams, masks), box=BOX), 12345, n, cap)
    kept = int(open(tmp_path / "count.txt").read())
    rk, ref = oracle.hull_sample(cams, masks, BOX[:3], BOX[3:], 12345, n, capacity=cap)
    assert kept == rk
    got = _read(tmp_path, "out_xyz.bin", np.float32, (-1, 3))
    assert np.array_equal(got, ref)


def test_sample_mixed_sizes_and_noisy_masks(exe, tmp_path):
    # 37 x 29 = 1073 pixels: the last packed word of that mask is partial
    cams = workloads.disc_views(3, size=64) + workloads.disc_views(2, size=40, seed=1) + \
        [workloads.look_at_camera(np.array([0.3, -2.9, 0.5]), 37, 29)]
    masks = _noisy_masks(cams, 3, 0.9)
    seed = (7 << 40) | 99
    run(exe, tmp_path, "sample", dict(_tables(cams, masks), box=BOX), seed, 20000, 20000)
    kept = int(open(tmp_path / "count.txt").read())
    rk, ref = oracle.hull_sample(cams, masks, BOX[:3], BOX[3:], seed, 20000)
    assert kept == rk > 0
    assert np.array_equal(_read(tmp_path, "out_xyz.bin", np.float32, (-1, 3)), ref)


def test_keep(exe, tmp_path):
    cams = workloads.disc_views(6, size=64, seed=2)
    masks = workloads.sphere_masks(cams, 0.7)
    rng = np.random.default_rng(5)
    xyz = rng.uniform(-4, 4, (3001, 3)).astype(np.float32)       # some behind cameras, most outside
    xyz[:1000] = rng.uniform(-0.8, 0.8, (1000, 3))
    run(exe, tmp_path, "keep", dict(_tables(cams, masks), xyz=xyz))
    got = _read(tmp_path, "keep.bin", np.uint8, (-1,)).astype(bool)
    assert np.array_equal(got, oracle.hull_consistent(xyz, cams, masks))


def test_keep_empty_mask_rejects_all(exe, tmp_path):
    cams = workloads.disc_views(3, size=48)
    masks = workloads.sphere_masks(cams, 0.7)
    masks[1][:] = 0
    xyz = np.random.default_rng(6).uniform(-0.5, 0.5, (700, 3)).astype(np.float32)
    run(exe, tmp_path, "keep", dict(_tables(cams, masks), xyz=xyz))
    assert not _read(tmp_path, "keep.bin", np.uint8, (-1,)).any()


@pytest.mark.parametrize("n", [2500, 1, 1023, 1025])
def test_filter(exe, tmp_path, n):
    cams = workloads.disc_views(5, size=64)
    masks = workloads.sphere_masks(cams, 0.6)
    rng = np.random.default_rng(n)
    xyz = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    cloud = oracle.Cloud(xyz, *workloads.point_attributes(n, 2, 4))
    run(exe, tmp_path, "filter", dict(_tables(cams, masks), xyz=xyz, sh=cloud.sh, op=cloud.opacity,
                                      rad=cloud.radius), 27)
    kept = int(open(tmp_path / "count.txt").read())
    keep, ref = oracle.consistency_filter(cloud, cams, masks)
    assert kept == int(keep.sum())
    assert np.array_equal(_read(tmp_path, "out_xyz.bin", np.float32, (-1, 3)), ref.xyz)
    assert np.array_equal(_read(tmp_path, "out_sh.bin", np.float32, (-1, 9, 3)), ref.sh)
    assert np.array_equal(_read(tmp_path, "out_op.bin", np.float32, (-1,)), ref.opacity)
    assert np.array_equal(_read(tmp_path, "out_rad.bin", np.float32, (-1,)), ref.radius)
