"""Pins for the oracle's colour accumulation (the paper's five parallel arrays:
TSDF, weight and three colour sums): colour never changes the TSDF sums or
weights; a frame of one colour gives colour sums equal to weight x colour
exactly; a frame split into two colours adds each colour once per pair of the
pixels that carry it."""
import numpy as np

from oracle import oracle as O
from paper_2608_08287_amd import scenes as S


def frame():
    w = S.single_frame_workload()
    return w, w.depth[0], w.cameras[0]


def pack(r, g, b):
    return np.uint32(r | (g << 8) | (b << 16))


def test_colour_leaves_tsdf_and_weights_alone():
    w, d, cam = frame()
    a = O.OracleVolume(w.voxel_size, w.trunc, w.pool_capacity)
    a.fuse(d, cam)
    b = O.OracleVolume(w.voxel_size, w.trunc, w.pool_capacity)
    rgba = np.random.default_rng(5).integers(0, 1 << 24, size=d.shape).astype(np.uint32)
    b.fuse_rgb(d, rgba, cam)
    ra, rb = a.result(), b.result()
    assert np.array_equal(ra.keys, rb.keys)
    assert np.array_equal(ra.sums, rb.sums) and np.array_equal(ra.weights, rb.weights)
    assert np.all(a.colour_sums() == 0)  # fuse() adds no colour


def test_one_colour_frame_gives_weight_times_colour():
    w, d, cam = frame()
    v = O.OracleVolume(w.voxel_size, w.trunc, w.pool_capacity)
    col = (201, 17, 96)
    v.fuse_rgb(d, np.full(d.shape, pack(*col), dtype=np.uint32), cam)
    v.fuse_rgb(d, np.full(d.shape, pack(*col), dtype=np.uint32), cam)
    sums = v.colour_sums()
    weights = v.result().weights.astype(np.float64)
    for c in range(3):
        assert np.array_equal(sums[:, c, :], weights * col[c])


def test_split_frame_adds_each_colour_per_pair():
    w, d, cam = frame()
    left = d.copy()
    left[:, d.shape[1] // 2:] = 0.0
    n_left = O.frame_pairs(w.voxel_size, w.trunc, left, cam).keys.size
    n_all = O.frame_pairs(w.voxel_size, w.trunc, d, cam).keys.size
    rgba = np.full(d.shape, pack(0, 0, 255), dtype=np.uint32)
    rgba[:, :d.shape[1] // 2] = pack(255, 0, 0)
    v = O.OracleVolume(w.voxel_size, w.trunc, w.pool_capacity)
    v.fuse_rgb(d, rgba, cam)
    tot = v.colour_sums().sum(axis=(0, 2))
    assert tot[0] == 255.0 * n_left
    assert tot[1] == 0.0
    assert tot[2] == 255.0 * (n_all - n_left)
