"""GPU parity of staged accumulation (tsdf_fuse_frames_staged): tiles write one
record per contribution into staging memory, listed per block, and apply
kernels add each block's records to the pool once per launch.  Every volume
must equal the oracle's (keys and weights exact, TSDF means within 1e-5,
counters equal): on sampled room frames with one and two frames per
workgroup, with staging for every record and at the minimum (where most tiles
go to the pool directly), over several launches, on the contended plane with a
0.95 pre-fill (over 40 frames its blocks get more records than the hot-block
bound and more runs than a run table holds), under exact pool and table
overflow, on tiles that overflow the LDS key set, on ragged frames, and on the
whole 300-frame trajectory in the benchmark's configuration.  Every case prints
its name first."""
import ctypes as C
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2608_08287_amd import scenes as S
from paper_2608_08287_amd import tsdf as T

from parity import (EMPTY, SCATTER, TSDF_ATOL, add_slices, assert_parity, assert_same_volume,
                    assert_table_invariants, log, oracle_slices, result_of, run_gpu, run_workload,
                    scattered_frames, table_arrays)

pytestmark = pytest.mark.gpu

ROOM_FRAMES = [0, 1, 2, 150, 299]
BIG, MIN = 32 * 640 * 480 * 9, 1 << 16  # staging records per launch: all, and the least accepted


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the HIP path has no CPU fallback")
    T.lib()


@pytest.fixture(autouse=True)
def _announce(request):
    log(f"[gpu] {request.node.name}")
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def room():
    w = S.room_trajectory_workload(frames=ROOM_FRAMES)
    return w, O.fuse_workload(w)


@pytest.mark.parametrize("per_group", [1, 2])
@pytest.mark.parametrize("records", [BIG, MIN])
@pytest.mark.parametrize("streams", [2, 1])
def test_staged_room_frames(room, per_group, records, streams):
    w, o = room
    flags = T.FUSE_BATCH(per_group) | (T.FUSE_ONE_STREAM if streams == 1 else 0)
    g = run_workload(w, staged=records, flags=flags, keep_volume=True)
    assert_parity(g, o)
    assert g.stats.frames == len(ROOM_FRAMES) and g.stats.status == T.OK
    assert_table_invariants(g.vol, o.keys, o.keys.size)


def test_staged_several_launches_match_the_oracle():
    """70 consecutive frames: three launches (32, 32, 6), each list and count
    reset by the launch before; the oracle fuses slices of them in parallel."""
    w = S.room_trajectory_workload(frames=range(40, 110))
    g = run_workload(w, staged=BIG)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0
    parts = oracle_slices(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras,
                          max(1, min(16, os.cpu_count() or 1)))
    sums, weights, seen, points, pairs = add_slices(parts, g.keys)
    assert seen.all() and g.stats.points_valid == points and g.stats.pairs == pairs
    assert np.array_equal(g.weights, weights.astype(np.float32))
    means = np.divide(sums, weights, out=np.zeros_like(sums), where=weights > 0)
    assert float(np.abs(g.means.astype(np.float64) - means).max()) <= TSDF_ATOL


def test_staged_stress_prefilled():
    """The contended plane into a table pre-filled to load factor 0.95 (the
    long probe read-ahead): no pair dropped."""
    w = S.plane_stress_workload("A", frames=[0, 1, 2, 3])
    o = O.fuse_workload(w)
    g = run_workload(w, staged=BIG, keep_volume=True)
    assert_parity(g, o)
    assert g.stats.pairs_dropped == 0
    assert_table_invariants(g.vol, o.keys, o.keys.size)


def test_staged_stress_many_frames_hot_blocks_and_full_run_tables():
    """40 frames of the plane at 0.5 m: its blocks take more records per launch
    than one wave sums (split over waves with atomics) and more runs than a
    run table lists (those go to the pool directly); against oracle slices."""
    w = S.plane_stress_workload("A", frames=list(range(40)))
    g = run_workload(w, staged=BIG)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0
    parts = oracle_slices(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras,
                          max(1, min(16, os.cpu_count() or 1)), prefill_blocks=w.prefill_blocks)
    sums, weights, seen, points, pairs = add_slices(parts, g.keys)
    assert g.stats.points_valid == points and g.stats.pairs == pairs
    assert np.array_equal(g.weights, weights.astype(np.float32))
    means = np.divide(sums, weights, out=np.zeros_like(sums), where=weights > 0)
    assert float(np.abs(g.means.astype(np.float64) - means).max()) <= TSDF_ATOL


def test_staged_pool_exhaustion_is_exact():
    """Pool for the pre-fill plus 100 blocks: exactly the scene's keys beyond
    100 overflow, every pair of a key without a block is dropped and counted."""
    w = S.plane_stress_workload("B", frames=[0, 1])
    full = O.fuse_frames(w.voxel_size, w.trunc, 1 << 20, w.depth, w.cameras)
    g = run_workload(w, staged=BIG, keep_volume=True)
    assert g.stats.status == T.ERR_POOL_EXHAUSTED
    assert g.stats.blocks_total == w.pool_capacity
    assert g.stats.keys_pool_overflow == full.keys.size - 100
    assert g.stats.pairs == full.stats["pairs"]
    keys, blocks = table_arrays(g.vol)
    alloc = keys[(keys != EMPTY) & (blocks >= 0)]
    # the pairs that reached a block plus those dropped are all the pairs
    assert int(g.weights.sum(dtype=np.float64)) + g.stats.pairs_dropped == g.stats.pairs
    assert np.array_equal(np.sort(g.keys), np.sort(alloc))


def test_staged_table_full_is_counted_exactly():
    w = S.plane_stress_workload("C", frames=[0])
    full1 = O.fuse_frames(w.voxel_size, w.trunc, 1 << 20, w.depth, w.cameras)
    pre = np.unique(np.array([O.pack_key(*map(int, b)) for b in w.prefill_blocks],
                             dtype=np.uint64))
    g = run_workload(w, staged=BIG, keep_volume=True)
    assert g.stats.status == T.ERR_TABLE_FULL
    model = O.probe_model(np.concatenate([pre, full1.keys]), w.table_capacity)
    assert g.stats.keys_table_overflow == model.n_overflow == full1.keys.size - 50


@pytest.mark.parametrize("band", list(SCATTER))
@pytest.mark.parametrize("records", [BIG, MIN])
def test_staged_scattered_tiles(band, records):
    v, tau, opts = SCATTER[band]
    depths, cams = scattered_frames(4, seed=31, **opts)
    o = O.fuse_frames(v, tau, 1 << 20, depths, cams)
    g = run_gpu(v, tau, 1 << 21, 1 << 20, depths, cams, staged=records)
    assert_parity(g, o)


def test_staged_mixed_sizes_and_invalid_frames():
    rng = np.random.default_rng(7)
    cams, depths = [], []
    for i, (W, H) in enumerate([(13, 9), (40, 23), (1, 1), (17, 33), (0, 4), (64, 48)]):
        a, b, c = rng.uniform(-2, 2, 3)
        R = (np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
             @ np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]]))
        pose = np.concatenate([R, rng.uniform(-1, 1, (3, 1))], 1)
        cams.append(S.Camera(W, H, 20.0 + i, 18.0, W / 2, H / 2, pose.astype(np.float32)))
        d = rng.uniform(0.3, 1.2, (H, W)).astype(np.float32)
        if d.size:
            d[rng.random((H, W)) < 0.2] = np.nan
        depths.append(d)
    o = O.fuse_frames(0.01, 0.04, 1 << 14, depths, cams)
    g = run_gpu(0.01, 0.04, 1 << 15, 1 << 14, depths, cams, staged=MIN, keep_volume=True)
    assert_parity(g, o)
    assert_table_invariants(g.vol, o.keys, o.keys.size)


def test_staged_one_staging_memory_for_volumes_of_several_sizes():
    """Staging sized for a large pool serves a smaller pool too, call after call."""
    w = S.room_trajectory_workload(frames=[10, 11, 12])
    staging = T.staging_buffer(1 << 18, 1 << 20)
    big = T.Volume(w.voxel_size, w.trunc, 1 << 20, 1 << 18)
    small = T.Volume(w.voxel_size, w.trunc, 1 << 17, 1 << 16)
    d = [torch.from_numpy(x).cuda() for x in w.depth]
    for vol in (big, small, big):
        vol.fuse_frames_staged(d, w.cameras, staging)
    ref = T.Volume(w.voxel_size, w.trunc, 1 << 20, 1 << 18)
    ref.fuse_frames(d + d, w.cameras + w.cameras)
    torch.cuda.synchronize()
    assert_same_volume(big, ref)
    o = O.fuse_workload(w)
    assert_parity(result_of(small), o)


def test_staged_argument_checks():
    L = T.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    vol = T.Volume(0.01, 0.04, 1 << 12, 1 << 11)
    cam = (T.CameraC * 1)(T.CameraC(4, 4, 2.0, 2.0, 2.0, 2.0,
                                    (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)))
    depth = torch.ones((4, 4), dtype=torch.float32, device="cuda")
    ptrs = (C.c_void_p * 1)(depth.data_ptr())
    need = T.staging_bytes(1 << 11, 1 << 16)
    buf = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    p = C.c_void_p(buf.data_ptr())
    assert L.tsdf_fuse_frames_staged(vol.handle, 1, ptrs, cam, 0, p, need - 1, s) == \
        T.ERR_BUFFER_TOO_SMALL
    assert L.tsdf_fuse_frames_staged(vol.handle, 1, ptrs, cam, 0, C.c_void_p(buf.data_ptr() + 8),
                                     need, s) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frames_staged(vol.handle, 1, ptrs, cam, 0, None, need, s) == \
        T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frames_staged(vol.handle, 1, ptrs, cam, T.FUSE_XCD_REMAP, p, need, s) == \
        T.ERR_INVALID_ARGUMENT
    colour = T.Volume(0.01, 0.04, 1 << 12, 1 << 11, flags=T.VOLUME_COLOUR)
    assert L.tsdf_fuse_frames_staged(colour.handle, 1, ptrs, cam, 0, p, need, s) == \
        T.ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
    assert vol.stats().frames == 0  # nothing was enqueued
    assert L.tsdf_fuse_frames_staged(vol.handle, 1, ptrs, cam, 0, p, need, s) == T.OK
    torch.cuda.synchronize()
    st = vol.stats()
    assert st.status == T.OK and st.frames == 1 and st.points_valid == 16


@pytest.mark.parametrize("design", ["main", "slot index"])
def test_staged_full_trajectory_matches_oracle_everywhere(design):
    """All 300 frames at 640x480 in the benchmark's configuration (32 frames per
    launch, 2 per workgroup, staging for every record), against the oracle at
    every voxel, the oracle fusing slices of the trajectory in parallel."""
    w = S.room_trajectory_workload(device="cuda")
    vol = None
    P = w.pool_capacity
    if design == "slot index":
        P = w.table_capacity
        vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, P, flags=T.VOLUME_SLOT_INDEX)
    else:
        vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, P)
    d = [torch.from_numpy(x).cuda() for x in w.depth]
    vol.fuse_frames_staged(d, w.cameras, T.staging_buffer(P))
    del d
    g = result_of(vol)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0
    n_thr = max(1, min(16, os.cpu_count() or 1))
    parts = oracle_slices(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras, n_thr)
    sums, weights, seen, points, pairs = add_slices(parts, g.keys)
    assert seen.all(), "the GPU volume has blocks no slice allocated"
    assert g.stats.points_valid == points and g.stats.pairs == pairs
    assert np.array_equal(g.weights, weights.astype(np.float32)), "weights differ"
    means = np.divide(sums, weights, out=np.zeros_like(sums), where=weights > 0)
    err = float(np.abs(g.means.astype(np.float64) - means).max())
    log(f"  {g.keys.size} blocks, {pairs} pairs, max |dTSDF| {err:.2e}")
    assert err <= TSDF_ATOL, err
