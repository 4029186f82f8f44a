"""GPU parity: the HIP path through the C ABI against the sequential CPU oracle.

Block keys and per-voxel weights must match exactly, TSDF means within 1e-5;
table and pool invariants are checked against the linear-probe model.  Every
case prints its name before touching the GPU.
"""
import math

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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the HIP path has no CPU fallback")
    T.lib()


def _name(request):
    log(f"[gpu] {request.node.name}")


@pytest.fixture(autouse=True)
def _announce(request):
    _name(request)
    yield
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# The single-frame plane + sphere workload (160x120, 1 cm voxels)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def single():
    w = S.single_frame_workload()
    return w, O.fuse_workload(w)


@pytest.mark.parametrize("flags", [T.FUSE_DEFAULT, T.FUSE_TWO_PASS, T.FUSE_XCD_REMAP,
                                   T.FUSE_TWO_PASS | T.FUSE_XCD_REMAP])
def test_single_frame_parity(single, flags):
    w, o = single
    g = run_workload(w, flags=flags, keep_volume=True)
    assert_parity(g, o)
    assert g.stats.status == T.OK and g.stats.lookup_misses == 0
    assert_table_invariants(g.vol, o.keys, o.keys.size)


def test_single_frame_repeatable(single):
    w, o = single
    for _ in range(3):
        assert_parity(run_workload(w), o)


def test_reset_then_refuse_is_identical(single):
    w, o = single
    g = run_workload(w, keep_volume=True)
    g.vol.reset()
    g2 = run_gpu(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity, w.depth, w.cameras,
                 vol=g.vol)
    assert_parity(g2, o)
    assert g2.stats.frames == 1


def test_separate_stages_match_fused(single):
    w, o = single
    vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    d = torch.from_numpy(w.depth[0]).cuda()
    vol.fuse(d, w.cameras[0], T.FUSE_ALLOCATE_ONLY)
    st = vol.stats()
    assert st.blocks_total == o.keys.size and st.pairs == 0 and st.frames == 0
    vol.fuse(d, w.cameras[0], T.FUSE_INTEGRATE_ONLY)
    g = run_gpu(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity, [], [], vol=vol)
    assert_parity(g, o)


def test_extract_buffer_too_small(single):
    w, o = single
    import ctypes as C
    vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    vol.fuse(torch.from_numpy(w.depth[0]).cuda(), w.cameras[0])
    n = C.c_uint32(0)
    keys = torch.empty(10, dtype=torch.int64, device="cuda")
    st = T.lib().tsdf_extract_blocks(vol.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     10, C.c_void_p(keys.data_ptr()), None, None, C.byref(n))
    assert st == T.ERR_BUFFER_TOO_SMALL and n.value == o.keys.size


# ---------------------------------------------------------------------------
# Closed forms and tiny inputs (ragged tiles, random poses, invalid pixels)
# ---------------------------------------------------------------------------

def _rot(a, b, c):
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    return (np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]]) @ np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
            @ np.array([[1, 0, 0], [0, cc, -sc], [0, sc, cc]]))


@pytest.mark.parametrize("seed", range(6))
def test_tiny_random_frames(seed):
    rng = np.random.default_rng(100 + seed)
    W, H = [(13, 9), (1, 1), (17, 33), (16, 16), (31, 2), (40, 23)][seed]
    pose = np.concatenate([_rot(*rng.uniform(-2, 2, 3)), rng.uniform(-1, 1, (3, 1))], 1).astype(np.float32)
    cam = S.Camera(W, H, float(rng.uniform(5, 30)), float(rng.uniform(5, 30)), W / 2 - 0.3, H / 2 + 0.1, pose)
    depth = rng.uniform(0.2, 1.5, (H, W)).astype(np.float32)
    depth[rng.random((H, W)) < 0.15] = 0.0
    depth[rng.random((H, W)) < 0.05] = np.nan
    depth[rng.random((H, W)) < 0.05] = -0.5
    v, tau = [(0.01, 0.04), (0.02, 0.06), (0.005, 0.02), (0.03, 0.03), (0.01, 0.08), (0.004, 0.016)][seed]
    o = O.fuse_frames(v, tau, 1 << 14, [depth], [cam])
    g = run_gpu(v, tau, 1 << 15, 1 << 14, [depth], [cam], keep_volume=True)
    assert_parity(g, o)
    assert_table_invariants(g.vol, o.keys, o.keys.size)


@pytest.mark.parametrize("angles", [(0.0, 0.0, 0.0), (0.5, 0.3, -0.2), (-2.0, 1.1, 0.7)])
def test_fronto_parallel_plane(angles):
    R = _rot(*angles)
    pose = np.concatenate([R, np.array([[0.3], [-0.2], [1.1]])], 1).astype(np.float32)
    cam = S.Camera(97, 61, 80.0, 75.0, 48.0, 30.5, pose)
    depth = np.full((61, 97), np.float32(1.003), dtype=np.float32)
    o = O.fuse_frames(0.01, 0.04, 1 << 14, [depth], [cam])
    g = run_gpu(0.01, 0.04, 1 << 15, 1 << 14, [depth], [cam])
    assert_parity(g, o)


def test_empty_and_invalid_frames():
    cam = S.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, S.IDENTITY_POSE)
    frames = [np.zeros((48, 64), np.float32), np.full((48, 64), np.nan, np.float32),
              np.full((48, 64), -1.0, np.float32), np.full((48, 64), np.inf, np.float32)]
    g = run_gpu(0.01, 0.04, 1024, 512, frames, [cam] * 4)
    assert g.keys.size == 0 and g.stats.points_valid == 0 and g.stats.pairs == 0
    assert g.stats.status == T.OK and g.stats.frames == 4
    # a zero-sized frame is a valid no-op
    g0 = run_gpu(0.01, 0.04, 1024, 512, [np.zeros((0, 5), np.float32)],
                 [S.Camera(5, 0, 50.0, 50.0, 2.0, 0.0, S.IDENTITY_POSE)])
    assert g0.keys.size == 0 and g0.stats.frames == 1


def test_coordinates_out_of_range_are_reported():
    cam, depth = S.plane_sphere_frame()
    pose = cam.pose.copy()
    pose[0, 3] = 1.0e5
    cam2 = S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, pose)
    o = O.fuse_frames(0.01, 0.04, 4096, [depth], [cam2])
    g = run_gpu(0.01, 0.04, 8192, 4096, [depth], [cam2])
    assert_parity(g, o)
    assert g.stats.status == T.ERR_COORD_RANGE and g.stats.coord_out_of_range == 9 * 19200


def test_large_frame_1280x720():
    scene = S.room_scene(1)
    cam = S.orbit_camera(17, 300, width=1280, height=720)
    depth = S.render_depth(cam, scene, lambda z: 0.002 * z * z, 7)
    o = O.fuse_frames(0.005, 0.02, 1 << 18, [depth], [cam])
    g = run_gpu(0.005, 0.02, 1 << 20, 1 << 18, [depth], [cam])
    assert_parity(g, o)


# ---------------------------------------------------------------------------
# The room trajectory at its full frame and volume sizes (sampled frames)
# ---------------------------------------------------------------------------

ROOM_FRAMES = [0, 1, 2, 150, 299]


@pytest.fixture(scope="module")
def room():
    w = S.room_trajectory_workload(frames=ROOM_FRAMES)
    return w, O.fuse_workload(w)


def test_room_trajectory_sampled_frames(room):
    w, o = room
    g = run_workload(w, keep_volume=True)
    assert_parity(g, o)
    assert g.stats.status == T.OK
    assert_table_invariants(g.vol, o.keys, o.keys.size)


@pytest.mark.parametrize("alpha", [0.25, 0.5, 0.75, 0.9])
def test_room_load_factor_sweep(room, alpha):
    w, o = room
    C = int(math.ceil(o.keys.size / alpha))
    g = run_gpu(w.voxel_size, w.trunc, C, w.pool_capacity, w.depth, w.cameras, keep_volume=True)
    assert_parity(g, o)
    assert_table_invariants(g.vol, o.keys, o.keys.size)
    log(f"  alpha={alpha} C={C} max_probe={g.stats.max_probe}")


# ---------------------------------------------------------------------------
# Contention and overflow stress: plane at 0.5 m, table pre-filled to LF 0.95
# ---------------------------------------------------------------------------

STRESS_FRAMES = [0, 1]


@pytest.fixture(scope="module")
def stress_full():
    """Oracle with an unbounded pool: every key's true weights."""
    w = S.plane_stress_workload("plain", frames=STRESS_FRAMES)
    return w, O.fuse_workload(w)


def test_stress_plain_contention(stress_full):
    w, o = stress_full
    g = run_workload(w)
    assert_parity(g, o)


@pytest.mark.parametrize("flags", [T.FUSE_DEFAULT, T.FUSE_TWO_PASS])
def test_stress_A_prefilled_to_095_drops_nothing(stress_full, flags):
    """The pool can fill the table here, so the launches take the long probe
    read-ahead; the two-pass form runs its allocate and integrate stages."""
    w = S.plane_stress_workload("A", frames=STRESS_FRAMES)
    o = O.fuse_workload(w)
    assert o.stats["pairs_dropped"] == 0 and o.stats["pool_overflow_keys"] == 0
    g = run_workload(w, flags=flags, keep_volume=True)
    assert_parity(g, o)
    assert g.stats.pairs_dropped == 0 and g.stats.status == T.OK
    assert_table_invariants(g.vol, o.keys, o.keys.size)
    log(f"  max_probe={g.stats.max_probe}")


def test_stress_A_all_100_frames_batched_matches_oracle():
    """The stress bench's whole run: 100 plane frames through tsdf_fuse_frames
    (32 per launch, 3 per workgroup) into the table pre-filled to load factor
    0.95, against the oracle at every voxel (frame slices fused on threads,
    each after the same pre-fill, added by key)."""
    import os

    w = S.plane_stress_workload("A", device="cuda")
    g = run_workload(w, batched=True)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0
    n_thr = max(1, min(16, os.cpu_count() or 1))
    parts = oracle_slices(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras, n_thr,
                          prefill_blocks=w.prefill_blocks)
    sums, weights, seen, points, pairs = add_slices(parts, g.keys)
    assert seen.all(), "the GPU volume has blocks no slice allocated"
    assert g.stats.points_valid == points and g.stats.pairs == pairs
    assert np.array_equal(g.weights, weights.astype(np.float32)), "weights differ"
    means = np.divide(sums, weights, out=np.zeros_like(sums), where=weights > 0)
    err = float(np.abs(g.means.astype(np.float64) - means).max())
    log(f"  {g.keys.size} blocks, {pairs} pairs, max probe {g.stats.max_probe}, "
        f"max |dTSDF| {err:.2e}")
    assert err <= TSDF_ATOL, err


def _pre_keys(coords):
    return np.array([O.pack_key(*map(int, c)) for c in coords], dtype=np.uint64)


def _check_subset(g, full, allocated_scene_keys):
    """Kept scene keys carry their full weights; everything else was dropped."""
    idx = np.searchsorted(full.keys, allocated_scene_keys)
    assert np.array_equal(full.keys[idx], allocated_scene_keys)
    gi = np.searchsorted(g.keys, allocated_scene_keys)
    assert np.array_equal(g.weights[gi], full.weights[idx].astype(np.float32))
    assert float(np.abs(g.means[gi] - full.means[idx]).max(initial=0.0)) <= 1e-5
    kept_pairs = int(full.weights[idx].sum())
    assert g.stats.pairs == full.stats["pairs"]
    assert g.stats.pairs_dropped == full.stats["pairs"] - kept_pairs


def test_stress_B_pool_exhaustion_is_exact(stress_full):
    w_full, full = stress_full
    w = S.plane_stress_workload("B", frames=STRESS_FRAMES)
    pre = _pre_keys(w.prefill_blocks)
    n_scene = full.keys.size
    g = run_workload(w, keep_volume=True)
    assert g.stats.status == T.ERR_POOL_EXHAUSTED
    assert g.stats.blocks_total == w.pool_capacity
    assert g.stats.keys_pool_overflow == n_scene - 100
    table_keys, blocks = table_arrays(g.vol)
    occ = table_keys != EMPTY
    alloc_keys = table_keys[occ & (blocks >= 0)]
    scene_alloc = np.setdiff1d(alloc_keys, pre)
    assert scene_alloc.size == 100
    assert np.array_equal(np.sort(g.keys), np.sort(alloc_keys))
    _check_subset(g, full, np.sort(scene_alloc))
    assert_table_invariants(g.vol, np.union1d(pre, full.keys), w.pool_capacity)


def test_stress_C_table_full_is_reported(stress_full):
    w_full, full = stress_full
    w = S.plane_stress_workload("C", frames=STRESS_FRAMES[:1])
    full1 = O.fuse_frames(w.voxel_size, w.trunc, 1 << 20, w.depth, w.cameras)
    pre = _pre_keys(w.prefill_blocks)
    g = run_workload(w, keep_volume=True)
    assert g.stats.status == T.ERR_TABLE_FULL
    table_keys, blocks = table_arrays(g.vol)
    assert np.count_nonzero(table_keys == EMPTY) == 0
    scene_in = np.setdiff1d(table_keys, pre)
    assert scene_in.size == 50
    assert g.stats.blocks_total == pre.size + 50
    _check_subset(g, full1, np.sort(scene_in))
    # every key that found the table full is counted once: the linear-probe
    # model's overflow over the pre-fill and the scene's keys
    model = O.probe_model(np.concatenate([pre, full1.keys]), w.table_capacity)
    assert model.n_overflow == full1.keys.size - 50
    assert g.stats.keys_table_overflow == model.n_overflow
    assert g.stats.table_full_events >= g.stats.keys_table_overflow
    assert not (g.stats.status_bits & T.FLAG_OVERFLOW_RECORD_FULL)
    # the same frame again: its failing keys fail again but are not new
    events = g.stats.table_full_events
    g.vol.fuse(torch.from_numpy(w.depth[0]).cuda(), w.cameras[0])
    again = g.vol.stats()
    assert again.keys_table_overflow == model.n_overflow
    assert again.table_full_events > events and again.blocks_new == 0


def test_blocks_new_counts_since_the_previous_query(room):
    w, _ = room
    o0 = O.fuse_frames(w.voxel_size, w.trunc, w.pool_capacity, w.depth[:1], w.cameras[:1])
    o01 = O.fuse_frames(w.voxel_size, w.trunc, w.pool_capacity, w.depth[:2], w.cameras[:2])
    vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    vol.fuse(torch.from_numpy(w.depth[0]).cuda(), w.cameras[0])
    st = vol.stats()
    assert st.blocks_new == st.blocks_total == o0.keys.size
    assert vol.stats().blocks_new == 0
    vol.fuse(torch.from_numpy(w.depth[1]).cuda(), w.cameras[1])
    st = vol.stats()
    assert st.blocks_total == o01.keys.size and st.blocks_new == o01.keys.size - o0.keys.size
    vol.reset()
    assert vol.stats().blocks_new == 0


# ---------------------------------------------------------------------------
# Tiles that touch many blocks and many voxels.  "sparse": random depths seen
# through a short focal length put nearly every sample of a tile in its
# own voxel and its own block, so the LDS sums of a tile take several windows
# of blocks (and, with 8 mm blocks and a 17-sample band, the tile's 1024-key
# set overflows).  "dense": a long focal length and a 0.12 m depth spread put
# thousands of voxels of a tile in one or two hundred blocks, so a window of
# blocks takes several passes over the voxel slots.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("band", list(SCATTER))
@pytest.mark.parametrize("path", ["plain", "batch1", "batch2", "batch3", "batch4"])
def test_scattered_tiles(band, path):
    v, tau, opts = SCATTER[band]
    depths, cams = scattered_frames(4, seed=31, **opts)
    o = O.fuse_frames(v, tau, 1 << 20, depths, cams)
    if path == "plain":
        g = run_gpu(v, tau, 1 << 21, 1 << 20, depths, cams)
    else:
        g = run_gpu(v, tau, 1 << 21, 1 << 20, depths, cams, batched=True,
                    flags=T.FUSE_BATCH(int(path[-1])))
    log(f"  {o.keys.size} blocks, {o.stats['pairs']} pairs")
    assert_parity(g, o)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0


@pytest.mark.parametrize("band", list(SCATTER))
@pytest.mark.parametrize("cfg", [(16, 1, 4), (16, 1, 8), (32, 2, 8)])
def test_scattered_tiles_multi_volume(band, cfg):
    v, tau, opts = SCATTER[band]
    depths, cams = scattered_frames(2, seed=32, **opts)
    o = O.fuse_frames(v, tau, 1 << 20, depths, cams)
    vol = T.Volume(v, tau, 1 << 21, 1 << 20)
    batch = T.Batch(2)
    batch.set_config(T.BatchConfig(cfg[0], cfg[1], cfg[2], 0))
    for d, c in zip(depths, cams):
        batch.fuse([vol], [torch.from_numpy(d).cuda()], [c])
    g = result_of(vol)
    assert_parity(g, o)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0


# ---------------------------------------------------------------------------
# Probe-distance histogram (instrumented volumes)
# ---------------------------------------------------------------------------

def probe_bins(d: np.ndarray) -> np.ndarray:
    """Histogram bin of each probe distance: 0 for 0, b for [2^(b-1), 2^b)."""
    d = np.asarray(d, dtype=np.int64)
    b = np.zeros(d.shape, dtype=np.int64)
    nz = d > 0
    b[nz] = np.floor(np.log2(d[nz])).astype(np.int64) + 1
    return np.minimum(b, T.PROBE_HIST_BINS - 1)


def test_probe_histogram_of_one_tile_is_the_probe_model():
    """A 32x8 frame is one tile, so each of its distinct keys is resolved
    once, at the distance where it ends up.  Linear probing makes the total
    displacement of a key set independent of insertion order, and the
    pre-filled keys never move: so the frame's summed probe distance is the
    probe model's total over all keys less its total over the pre-fill alone,
    through a table pre-filled to a load factor near 0.95."""
    depths, cams = scattered_frames(1, W=32, H=8, seed=41, focal=20.0, lo=0.4, hi=2.0)
    v, tau, C, P = 0.004, 0.016, 4096, 8192
    prefill = S.random_block_coords(3300, seed=42)
    o = O.fuse_frames(v, tau, P, depths, cams, prefill)
    vol = T.Volume(v, tau, C, P, flags=T.VOLUME_PROBE_HISTOGRAM)
    vol.insert_blocks(torch.from_numpy(prefill.astype(np.int32)).cuda())
    vol.fuse(torch.from_numpy(depths[0]).cuda(), cams[0])
    hist, total = vol.probe_histogram()
    g = result_of(vol)
    assert_parity(g, o)
    pre = np.array([O.pack_key(*map(int, b)) for b in prefill], dtype=np.uint64)
    frame = np.setdiff1d(o.keys, pre)
    assert 100 < frame.size < 1024  # one LDS key set, no overflow
    want_total = int(O.probe_model(o.keys, C).disp_of.sum()) - int(O.probe_model(pre, C).disp_of.sum())
    log(f"  {frame.size} keys of the frame; load factor {o.keys.size / C:.3f}; total distance "
        f"{total} (model {want_total}); histogram {hist.tolist()}")
    assert int(hist.sum()) == frame.size
    assert total == want_total
    # the bins bracket the total: each resolution's distance lies in its bin
    lo = sum(int(c) * (0 if b == 0 else 1 << (b - 1)) for b, c in enumerate(hist))
    hi = sum(int(c) * (0 if b == 0 else (1 << b) - 1) for b, c in enumerate(hist))
    assert lo <= total <= hi
    top = int(np.nonzero(hist)[0].max())
    assert top == int(probe_bins(np.array([g.stats.max_probe]))[0])


def test_probe_histogram_changes_nothing_else(room):
    w, o = room
    plain = run_workload(w)
    vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity,
                   flags=T.VOLUME_PROBE_HISTOGRAM)
    for d, c in zip(w.depth, w.cameras):
        vol.fuse(torch.from_numpy(d).cuda(), c)
    g = result_of(vol)
    assert_parity(g, o)
    assert np.array_equal(g.keys, plain.keys) and np.array_equal(g.weights, plain.weights)
    hist, total = vol.probe_histogram()
    top = int(np.nonzero(hist)[0].max())
    assert top == int(probe_bins(np.array([g.stats.max_probe]))[0])
    assert int(hist.sum()) >= g.stats.blocks_total
    vol.reset()
    hist, total = vol.probe_histogram()
    assert int(hist.sum()) == 0 and total == 0
    with pytest.raises(T.TsdfError):
        T.Volume(w.voxel_size, w.trunc, 1024, 512).probe_histogram()


def test_atomic_rate_measurement_loses_no_update():
    """The measurement kernel's adds all land: the buffer sums to waves x
    instructions x rows x lanes (every float stays a small exact integer)."""
    buf = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")
    for rows, lanes in ((12, 5), (4, 16), (64, 1)):
        buf.zero_()
        T.measure_atomic_rate(buf, 1024, 8, rows, lanes)
        torch.cuda.synchronize()
        assert int(buf.double().sum().item()) == 1024 * 8 * rows * lanes
        # only the first `lanes` floats of a row are ever touched
        per_row = buf.view(-1, 16)
        assert float(per_row[:, lanes:].abs().sum()) == 0.0


# ---------------------------------------------------------------------------
# Several frames per launch (tsdf_fuse_frames)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cap", [0, 1, 2, 3, 4])
def test_batched_room_frames(room, cap):
    w, o = room
    g = run_workload(w, flags=T.FUSE_BATCH(cap), batched=True, keep_volume=True)
    assert_parity(g, o)
    assert g.stats.frames == len(ROOM_FRAMES) and g.stats.status == T.OK
    assert_table_invariants(g.vol, o.keys, o.keys.size)


def test_batched_consecutive_trajectory_frames():
    w = S.room_trajectory_workload(frames=range(40, 52))
    o = O.fuse_workload(w)
    g = run_workload(w, batched=True)
    assert_parity(g, o)


def test_batched_mixed_sizes_and_invalid_frames():
    rng = np.random.default_rng(7)
    cams, depths = [], []
    for i, (W, H) in enumerate([(13, 9), (40, 23), (1, 1), (17, 33), (0, 4), (64, 48)]):
        pose = np.concatenate([_rot(*rng.uniform(-2, 2, 3)), rng.uniform(-1, 1, (3, 1))], 1)
        cams.append(S.Camera(W, H, 20.0 + i, 18.0, W / 2, H / 2, pose.astype(np.float32)))
        d = rng.uniform(0.3, 1.2, (H, W)).astype(np.float32)
        if d.size:
            d[rng.random((H, W)) < 0.2] = np.nan
        depths.append(d)
    o = O.fuse_frames(0.01, 0.04, 1 << 14, depths, cams)
    g = run_gpu(0.01, 0.04, 1 << 15, 1 << 14, depths, cams, batched=True, keep_volume=True)
    assert_parity(g, o)
    assert_table_invariants(g.vol, o.keys, o.keys.size)


def test_batched_wide_band():
    # K = 6 (13 samples): two frames per launch
    w = S.room_trajectory_workload(frames=[3, 4, 5])
    o = O.fuse_frames(0.005, 0.03, 1 << 18, w.depth, w.cameras)
    g = run_gpu(0.005, 0.03, 1 << 20, 1 << 18, w.depth, w.cameras, batched=True)
    assert_parity(g, o)


@pytest.mark.parametrize("per_group", [1, 2, 3, 4])
def test_batched_stress_prefilled(stress_full, per_group):
    """Batched launches on the long probe read-ahead (the pool can fill the
    table), with 1 to 4 frames per workgroup."""
    w = S.plane_stress_workload("A", frames=[0, 1, 2, 3])
    o = O.fuse_workload(w)
    g = run_workload(w, batched=True, keep_volume=True, flags=T.FUSE_BATCH(per_group))
    assert_parity(g, o)
    assert g.stats.pairs_dropped == 0
    assert_table_invariants(g.vol, o.keys, o.keys.size)


# ---------------------------------------------------------------------------
# The full 300-frame trajectory in the benchmark's launch configuration
# (properties that hold at any size; the oracle covers sampled frames above)
# ---------------------------------------------------------------------------

def test_full_trajectory_batched_equals_plain():
    w = S.room_trajectory_workload(device="cuda")
    log(f"  generated {len(w.depth)} frames")
    g_b = run_workload(w, batched=True, keep_volume=True)            # tsdf_fuse_frames
    g_p = run_workload(w, flags=T.FUSE_DEFAULT, keep_volume=True)    # one launch per frame
    assert g_b.stats.status == T.OK and g_p.stats.status == T.OK
    assert g_b.stats.pairs_dropped == 0 and g_b.stats.lookup_misses == 0
    assert g_b.stats.points_valid == g_p.stats.points_valid == 300 * 640 * 480
    assert g_b.stats.pairs == g_p.stats.pairs
    assert np.array_equal(g_b.keys, g_p.keys)
    assert np.array_equal(g_b.weights, g_p.weights)
    assert float(np.abs(g_b.means - g_p.means).max()) <= 2e-5
    # every weight is an observation count: the total is the number of pairs
    assert int(g_b.weights.sum(dtype=np.float64)) == g_b.stats.pairs
    # every allocated block received a contribution (same test in both stages)
    assert np.all(g_b.weights.reshape(len(g_b.keys), -1).max(axis=1) > 0)
    assert_table_invariants(g_b.vol, g_b.keys, g_b.keys.size)
    # the frames the oracle also fused (ROOM_FRAMES, in the sampled-frames test) are
    # a subset: their keys must all be present here
    o = O.fuse_frames(w.voxel_size, w.trunc, w.pool_capacity, [w.depth[0]], [w.cameras[0]])
    assert np.all(np.isin(o.keys, g_b.keys))


def test_frames_read_from_pinned_host_memory():
    """Depth frames in pinned host memory, passed at the device addresses the
    runtime maps them to, are read by the kernels over PCIe: the plain, the
    batched and the multi-volume batch path give the same volumes as frames in
    device memory."""
    import ctypes

    w = S.room_trajectory_workload(frames=[0, 1, 2, 3, 150])
    n = len(w.depth)
    H, W = w.depth[0].shape
    host = torch.empty((n, H, W), dtype=torch.float32, pin_memory=True)
    for k in range(n):
        host[k].copy_(torch.from_numpy(w.depth[k]))
    dptr = (ctypes.c_void_p * n)()
    for k in range(n):
        dptr[k] = T.host_device_pointer(host[k].data_ptr())
        assert dptr[k]
    cams = (T.CameraC * n)(*[T.camera_struct(c) for c in w.cameras])
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = T.lib()
    ref = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    ref.fuse_frames([torch.from_numpy(d).cuda() for d in w.depth], w.cameras)
    batched = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    assert L.tsdf_fuse_frames(batched.handle, n, dptr, cams, 0, sp) == T.OK
    plain = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    for k in range(n):
        assert L.tsdf_fuse_frame(plain.handle, dptr[k], ctypes.byref(cams[k]), sp) == T.OK
    # the multi-volume batch path: each frame into its own volume, one launch
    vols = [T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity) for _ in range(n)]
    items = (T.FuseItemC * n)()
    for k in range(n):
        items[k].volume = vols[k].handle.value
        items[k].depth_dev = dptr[k]
        items[k].camera = cams[k]
    batch = T.Batch(n)
    batch.set_config(T.BatchConfig(32, 2, 8, 0))
    assert L.tsdf_batch_fuse(batch._h, items, n, 0, sp) == T.OK
    alone = [T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity) for _ in range(n)]
    for k in range(n):
        alone[k].fuse(torch.from_numpy(w.depth[k]).cuda(), w.cameras[k])
    torch.cuda.synchronize()
    st = assert_same_volume(batched, ref)
    assert_same_volume(plain, ref)
    assert st.status == T.OK and st.points_valid == n * H * W
    for k in range(n):
        assert_same_volume(vols[k], alone[k])
    del host


@pytest.mark.parametrize("design", ["main", "slot index"])
def test_full_trajectory_batched_matches_oracle_everywhere(design):
    """All 300 frames at 640x480 through the launch configuration the bench times
    (tsdf_fuse_frames, 32 frames per launch, 3 per workgroup), against the oracle
    at every voxel; for the main design (table 2^20, pool 2^18) and for the
    slot-derived block index (pool = table = 2^20), as the bench's variants.  With no pool overflow, a voxel's weight and TSDF sum are
    sums over frames, so disjoint slices of the trajectory fused into separate
    oracle volumes (in parallel: the oracle's calls release the interpreter
    lock) add up to the sequential result: weights exactly, sums up to float64
    rounding.  A block exists iff some slice allocated it."""
    import os

    w = S.room_trajectory_workload(device="cuda")
    vol = None
    if design == "slot index":
        vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.table_capacity,
                       flags=T.VOLUME_SLOT_INDEX)
    g = run_workload(w, batched=True, vol=vol)
    assert g.stats.status == T.OK and g.stats.pairs_dropped == 0
    n_thr = max(1, min(16, os.cpu_count() or 1))
    parts = oracle_slices(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras, n_thr)
    sums, weights, seen, points, pairs = add_slices(parts, g.keys)
    assert seen.all(), "the GPU volume has blocks no slice allocated"
    assert g.stats.points_valid == points and g.stats.pairs == pairs
    assert np.array_equal(g.weights, weights.astype(np.float32)), "weights differ"
    means = np.divide(sums, weights, out=np.zeros_like(sums), where=weights > 0)
    err = float(np.abs(g.means.astype(np.float64) - means).max())
    log(f"  {g.keys.size} blocks, {pairs} pairs, {n_thr} oracle slices, max |dTSDF| {err:.2e}")
    assert err <= TSDF_ATOL, err
