"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-computed
constants of the key equation (Section 2.1), textbook floor division, closed
forms of a fronto-parallel plane, the analytic sphere (Section 4.1's analytic
tier), independent brute-force fusions on tiny inputs, and known properties of
linear probing.  None of them needs a GPU.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_08287_amd import scenes as S

F = np.float32


# ---------------------------------------------------------------------------
# Section 2.1: key(x, y, z) = (x + 2^20) << 42 | (y + 2^20) << 21 | (z + 2^20)
# ---------------------------------------------------------------------------

def test_pack_key_hand_computed_values():
    # 2^20 << 42 = 2^62, 2^20 << 21 = 2^41, 2^20: origin block, worked by hand
    assert O.pack_key(0, 0, 0) == 0x4000020000100000
    assert O.pack_key(-(1 << 20), -(1 << 20), -(1 << 20)) == 0
    # the largest coordinates fill 63 bits, so bit 63 (and the all-ones EMPTY
    # word) can never be a key
    assert O.pack_key((1 << 20) - 1, (1 << 20) - 1, (1 << 20) - 1) == 0x7FFFFFFFFFFFFFFF
    assert O.pack_key(1, 0, 0) - O.pack_key(0, 0, 0) == 1 << 42
    assert O.pack_key(0, 1, 0) - O.pack_key(0, 0, 0) == 1 << 21
    assert O.pack_key(0, 0, 1) - O.pack_key(0, 0, 0) == 1
    assert O.pack_key(-1, 0, 0) == 0x4000020000100000 - (1 << 42)


def test_pack_key_unpacks_by_bit_fields():
    rng = np.random.default_rng(5)
    for b in rng.integers(-(1 << 20), 1 << 20, size=(2000, 3)):
        k = O.pack_key(int(b[0]), int(b[1]), int(b[2]))
        mask = (1 << 21) - 1
        assert ((k >> 42) & mask) - (1 << 20) == b[0]
        assert ((k >> 21) & mask) - (1 << 20) == b[1]
        assert (k & mask) - (1 << 20) == b[2]
        assert k >> 63 == 0


def test_block_of_is_floor_division():
    for v in range(-200, 201):
        assert O.block_of(v) == v // 8  # Python // is floor division
    assert O.block_of(-1) == -1 and O.block_of(-8) == -1 and O.block_of(-9) == -2
    assert O.block_of(-(1 << 23)) == -(1 << 20) and O.block_of((1 << 23) - 1) == (1 << 20) - 1


# ---------------------------------------------------------------------------
# The hash (a reading: MurmurHash3 fmix64 + Lemire range reduction)
# ---------------------------------------------------------------------------

M64 = (1 << 64) - 1


def _unfmix64(h):
    # xor-shift by 33 >= 32 is its own inverse; multiplications invert mod 2^64
    c1_inv = pow(0xFF51AFD7ED558CCD, -1, 1 << 64)
    c2_inv = pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)
    h ^= h >> 33
    h = (h * c2_inv) & M64
    h ^= h >> 33
    h = (h * c1_inv) & M64
    h ^= h >> 33
    return h


def test_fmix64_is_the_published_bijection():
    assert O.fmix64(0) == 0
    rng = np.random.default_rng(7)
    for x in rng.integers(0, 2 ** 63, size=500, dtype=np.int64):
        x = int(x) * 2 + 1
        assert _unfmix64(O.fmix64(x)) == x


def test_home_slot_range_reduction():
    rng = np.random.default_rng(8)
    for C in [1, 3, 1000, 8192, 1 << 16, 1 << 20, (1 << 32) - 1]:
        for k in rng.integers(0, 2 ** 63, size=200, dtype=np.int64):
            s = O.home_slot(int(k), C)
            assert 0 <= s < C
            assert s == ((O.fmix64(int(k)) >> 32) * C) >> 32
    # power-of-two capacities take the top bits of the hash
    k = O.pack_key(3, -4, 5)
    assert O.home_slot(k, 1 << 16) == O.fmix64(k) >> 48


def test_home_slots_of_neighbouring_blocks_are_uniform():
    C = 1024
    slots = [O.home_slot(O.pack_key(x, y, z), C) for x in range(-8, 8) for y in range(-8, 8)
             for z in range(-8, 8)]
    counts = np.bincount(slots, minlength=C)
    expected = len(slots) / C
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # chi-square with 1023 dof: mean 1023, sd ~45; 5 sd either side
    assert 800 < chi2 < 1250


# ---------------------------------------------------------------------------
# Linear-probe model
# ---------------------------------------------------------------------------

def _random_keys(n, seed):
    c = S.random_block_coords(n, seed)
    return np.array([O.pack_key(*map(int, r)) for r in c], dtype=np.uint64)


def test_probe_model_layout_invariants_and_order_independence():
    C = 4096
    keys = _random_keys(3000, 11)
    m = O.probe_model(keys, C)
    assert m.n_overflow == 0
    assert np.all(m.table[m.slot_of] == keys)
    empty = np.uint64(2 ** 64 - 1)
    for k, s, d in zip(keys[:500], m.slot_of[:500], m.disp_of[:500]):
        h = O.home_slot(int(k), C)
        assert (h + int(d)) % C == s
        for j in range(int(d)):  # no empty slot on the path home -> slot
            assert m.table[(h + j) % C] != empty
    rng = np.random.default_rng(12)
    for _ in range(3):
        perm = rng.permutation(keys.size)
        m2 = O.probe_model(keys[perm], C)
        assert np.array_equal(m2.occupied, m.occupied)
        assert int(m2.disp_of.sum()) == int(m.disp_of.sum())


def test_probe_model_duplicates_and_overflow():
    C = 64
    keys = _random_keys(100, 13)
    dup = np.concatenate([keys[:10], keys[:10]])
    m = O.probe_model(dup, C)
    assert np.array_equal(m.slot_of[:10], m.slot_of[10:])
    assert m.n_overflow == 0
    m = O.probe_model(keys, C)
    assert m.n_overflow == 100 - C
    assert np.count_nonzero(m.slot_of < 0) == 100 - C
    assert m.occupied.size == C


@pytest.mark.parametrize("alpha", [0.25, 0.5, 0.75])
def test_probe_model_matches_knuth_expected_probes(alpha):
    # successful search in linear probing: 1/2 (1 + 1/(1 - alpha)) probes on average
    C = 1 << 16
    keys = _random_keys(int(alpha * C), 14)
    m = O.probe_model(keys, C)
    mean_probes = float(m.disp_of.mean()) + 1.0
    assert mean_probes == pytest.approx(0.5 * (1 + 1 / (1 - alpha)), rel=0.04)


# ---------------------------------------------------------------------------
# Fronto-parallel plane, identity pose: separable closed form
# ---------------------------------------------------------------------------

def _axis_counts(n_pix, c, f, z, iv):
    """For one sample depth z: histogram of floor(fl(fl(a_u z) iv)) over pixels u."""
    inv_f = F(1.0) / F(f)
    a = (np.arange(n_pix).astype(F) - F(c)) * inv_f
    idx = np.floor((a * F(z)).astype(F) * F(iv)).astype(np.int64)
    vals, cnts = np.unique(idx, return_counts=True)
    return dict(zip(vals.tolist(), cnts.tolist()))


@pytest.mark.parametrize("D_layers,v,tau", [(100.3, 0.01, 0.04), (57.71, 0.005, 0.02),
                                             (121.45, 0.004, 0.016)])
def test_plane_identity_pose_closed_form(D_layers, v, tau):
    W, H, fx, fy, cx, cy = 37, 23, 30.0, 27.0, 18.3, 11.1
    D = F(D_layers * v)
    cam = S.Camera(W, H, fx, fy, cx, cy, S.IDENTITY_POSE)
    depth = np.full((H, W), D, dtype=np.float32)
    r = O.fuse_frames(v, tau, 1 << 16, [depth], [cam])
    v32, tau32 = F(v), F(tau)
    iv = F(1.0) / v32
    K = int(round(tau / v))
    expected = {}
    for k in range(2 * K + 1):
        z = F(D + F(k - K) * v32)
        iz = int(np.floor(F(z * iv)))
        zc = (F(iz) + F(0.5)) * v32
        if D - zc < -tau32:
            continue
        cx_ = _axis_counts(W, cx, fx, z, iv)
        cy_ = _axis_counts(H, cy, fy, z, iv)
        for ix, nx in cx_.items():
            for iy, ny in cy_.items():
                assert (ix, iy, iz) not in expected  # one sample per layer (D off the grid)
                expected[(ix, iy, iz)] = nx * ny
    got = {}
    for key, w, m in zip(r.keys, r.weights, r.means):
        key = int(key)
        b = [((key >> 42) & 0x1FFFFF) - (1 << 20), ((key >> 21) & 0x1FFFFF) - (1 << 20),
             (key & 0x1FFFFF) - (1 << 20)]
        for loc in np.nonzero(w)[0]:
            lx, ly, lz = loc % 8, (loc // 8) % 8, loc // 64
            vox = (8 * b[0] + int(lx), 8 * b[1] + int(ly), 8 * b[2] + int(lz))
            got[vox] = int(w[loc])
            zc = (vox[2] + 0.5) * v
            assert m[loc] == pytest.approx(min(max(float(D) - zc, -tau), tau), abs=1e-6)
            assert float(D) - zc >= -tau - 1e-6
    assert got == expected
    assert sum(got.values()) == r.stats["pairs"]


def _rot(yaw, pitch, roll):
    cy, sy, cp, sp, cr, sr = (math.cos(yaw), math.sin(yaw), math.cos(pitch), math.sin(pitch),
                              math.cos(roll), math.sin(roll))
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    Rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
    return Rz @ Ry @ Rx


@pytest.mark.parametrize("angles,t", [((0.5, 0.3, -0.2), (0.3, -0.2, 1.1)),
                                      ((-2.0, 1.1, 0.7), (-1.7, 0.4, -2.3))])
def test_plane_rotated_pose_sdf_closed_form(angles, t):
    # every pixel reads depth D: the plane z_cam = D, whatever the pose
    v, tau, D = 0.01, 0.04, F(0.8537)
    R = _rot(*angles)
    pose = np.concatenate([R, np.asarray(t)[:, None]], axis=1).astype(np.float32)
    cam = S.Camera(41, 29, 35.0, 33.0, 20.0, 14.0, pose)
    depth = np.full((29, 41), D, dtype=np.float32)
    r = O.fuse_frames(v, tau, 1 << 16, [depth], [cam])
    Rd, td = pose[:, :3].astype(np.float64), pose[:, 3].astype(np.float64)
    n_vox = 0
    for key, w, m in zip(r.keys, r.weights, r.means):
        key = int(key)
        b = np.array([((key >> 42) & 0x1FFFFF) - (1 << 20), ((key >> 21) & 0x1FFFFF) - (1 << 20),
                      (key & 0x1FFFFF) - (1 << 20)])
        for loc in np.nonzero(w)[0]:
            l = np.array([loc % 8, (loc // 8) % 8, loc // 64])
            centre = (8 * b + l + 0.5) * v
            zc = (Rd.T @ (centre - td))[2]
            assert float(D) - zc >= -tau - 2e-6
            assert m[loc] == pytest.approx(min(float(D) - zc, tau), abs=2e-6)
            n_vox += 1
    assert n_vox > 1000
    # every point contributes to between 1 and 2K+1 voxels
    pts = r.stats["points_valid"]
    assert pts == 41 * 29 and pts <= r.stats["pairs"] <= 9 * pts


# ---------------------------------------------------------------------------
# Sphere radius: the analytic tier (zero crossing within a quarter voxel)
# ---------------------------------------------------------------------------

def _zero_crossings(r, v, cols):
    """Interpolated zero crossing of the mean TSDF along world-z voxel columns."""
    vox = {}
    for key, w, m in zip(r.keys, r.weights, r.means):
        key = int(key)
        b = [((key >> 42) & 0x1FFFFF) - (1 << 20), ((key >> 21) & 0x1FFFFF) - (1 << 20),
             (key & 0x1FFFFF) - (1 << 20)]
        for loc in np.nonzero(w)[0]:
            vox[(8 * b[0] + loc % 8, 8 * b[1] + (loc // 8) % 8, 8 * b[2] + loc // 64)] = m[loc]
    out = {}
    for (ix, iy) in cols:
        zs = sorted(z for (x, y, z) in vox if x == ix and y == iy)
        for z0, z1 in zip(zs, zs[1:]):
            if z1 == z0 + 1 and vox[(ix, iy, z0)] >= 0 > vox[(ix, iy, z1)]:
                m0, m1 = vox[(ix, iy, z0)], vox[(ix, iy, z1)]
                out[(ix, iy)] = (z0 + 0.5) * v + m0 / (m0 - m1) * v
                break
    return out


def test_sphere_radius_within_quarter_voxel():
    v, tau = 0.01, 0.04
    cam, depth = S.plane_sphere_frame(noise=False)
    r = O.fuse_frames(v, tau, 4096, [depth], [cam])
    cols = [(ix, iy) for ix in range(-3, 3) for iy in range(-3, 3)]
    zc = _zero_crossings(r, v, cols)
    assert len(zc) == len(cols)
    for (ix, iy), z in zc.items():
        x, y = (ix + 0.5) * v, (iy + 0.5) * v
        z_true = 1.2 - math.sqrt(0.3 ** 2 - x * x - y * y)
        assert abs(z - z_true) < v / 4, (ix, iy, z, z_true)


def test_sphere_only_scene_radius_off_axis():
    # a larger sphere filling the view, voxel 5 mm: columns up to 4 cm off-axis
    v, tau = 0.005, 0.02
    cam = S.Camera(120, 90, 110.0, 110.0, 59.5, 44.5, S.IDENTITY_POSE)
    depth = S.render_depth(cam, [S.Sphere((0.0, 0.0, 1.0), 0.4)])
    r = O.fuse_frames(v, tau, 1 << 14, [depth], [cam])
    cols = [(ix, iy) for ix in range(-8, 8, 3) for iy in range(-8, 8, 3)]
    zc = _zero_crossings(r, v, cols)
    assert len(zc) == len(cols)
    for (ix, iy), z in zc.items():
        x, y = (ix + 0.5) * v, (iy + 0.5) * v
        z_true = 1.0 - math.sqrt(0.4 ** 2 - x * x - y * y)
        assert abs(z - z_true) < v / 4, (ix, iy, z, z_true)


# ---------------------------------------------------------------------------
# Independent brute-force fusions on tiny inputs
# ---------------------------------------------------------------------------

def _py_walk(depth, cam, v, tau):
    """Per pixel (row-major), the list of (voxel, val) a point selects.

    Float32 scalar arithmetic in the same operation order as the method's
    definition; no hash, no key packing."""
    v, tau = F(v), F(tau)
    iv = F(1.0) / v
    K = int(round(float(tau) / float(v)))
    R = cam.pose[:, :3].astype(np.float32)
    t = cam.pose[:, 3].astype(np.float32)
    ifx, ify = F(1.0) / F(cam.fx), F(1.0) / F(cam.fy)
    out = []
    H, W = depth.shape
    for y in range(H):
        for x in range(W):
            d = F(depth[y, x])
            sel, chosen = [], []
            if not (np.isfinite(d) and d > 0):
                out.append(sel)
                continue
            a = (F(x) - F(cam.cx)) * ifx
            b = (F(y) - F(cam.cy)) * ify
            for k in range(2 * K + 1):
                z = F(d + F(k - K) * v)
                if not z > 0:
                    continue
                c = [a * z, b * z, z]
                wv = [F(F(F(R[r, 0] * c[0]) + F(R[r, 1] * c[1])) + F(R[r, 2] * c[2])) + t[r]
                      for r in range(3)]
                q = [F(wv[r] * iv) for r in range(3)]
                if not all(abs(qq) < F(8388608.0) for qq in q):
                    continue
                vox = tuple(int(np.floor(qq)) for qq in q)
                if vox in chosen:
                    continue
                chosen.append(vox)
                cen = [F(F(vox[r]) + F(0.5)) * v for r in range(3)]
                zcv = F(F(R[0, 2] * F(cen[0] - t[0])) + F(R[1, 2] * F(cen[1] - t[1])))
                zcv = F(zcv + F(R[2, 2] * F(cen[2] - t[2])))
                sdf = F(d - zcv)
                if not zcv > 0 or sdf < -tau:
                    continue
                sel.append((vox, sdf if sdf < tau else tau))
            out.append(sel)
    return out


def _tiny_case(seed):
    rng = np.random.default_rng(seed)
    R = _rot(*rng.uniform(-1, 1, 3))
    pose = np.concatenate([R, rng.uniform(-0.5, 0.5, (3, 1))], axis=1).astype(np.float32)
    cam = S.Camera(13, 9, 11.0, 12.5, 6.2, 4.0, pose)
    depth = rng.uniform(0.3, 0.9, (9, 13)).astype(np.float32)
    depth[rng.random((9, 13)) < 0.1] = 0.0
    depth[0, 0] = np.nan
    return cam, depth


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_brute_force_matches(seed):
    v, tau = 0.02, 0.06
    cam, depth = _tiny_case(seed)
    sel = _py_walk(depth, cam, v, tau)
    flat = [s for p in sel for s in p]
    vox = np.array([s[0] for s in flat])
    lo = vox.min(axis=0)
    shape = tuple(vox.max(axis=0) - lo + 1)
    wsum = np.zeros(shape, dtype=np.float64)
    wcnt = np.zeros(shape, dtype=np.int64)
    for (vx, val) in flat:  # same order as the oracle's pass 2
        i = tuple(np.subtract(vx, lo))
        wsum[i] += float(val)
        wcnt[i] += 1
    r = O.fuse_frames(v, tau, 1 << 12, [depth], [cam])
    dense_sum = np.zeros(shape)
    dense_cnt = np.zeros(shape, dtype=np.int64)
    for key, w, s in zip(r.keys, r.weights, r.sums):
        key = int(key)
        b = np.array([((key >> 42) & 0x1FFFFF) - (1 << 20), ((key >> 21) & 0x1FFFFF) - (1 << 20),
                      (key & 0x1FFFFF) - (1 << 20)])
        assert w.sum() > 0  # every allocated block received a contribution
        for loc in np.nonzero(w)[0]:
            i = tuple(8 * b + np.array([loc % 8, (loc // 8) % 8, loc // 64]) - lo)
            dense_sum[i] = s[loc]
            dense_cnt[i] = w[loc]
    assert np.array_equal(dense_cnt, wcnt)
    assert np.array_equal(dense_sum, wsum)  # same summation order: bit-identical


def test_voxel_centric_brute_force_weights():
    # weight of a voxel == number of points whose walk selects it
    v, tau = 0.02, 0.06
    cam, depth = _tiny_case(4)
    sel = _py_walk(depth, cam, v, tau)
    per_pixel = [set(s[0] for s in p) for p in sel]
    allv = set().union(*per_pixel)
    lo = np.min(list(allv), axis=0) - 1
    hi = np.max(list(allv), axis=0) + 1
    r = O.fuse_frames(v, tau, 1 << 12, [depth], [cam])
    got = {}
    for key, w in zip(r.keys, r.weights):
        key = int(key)
        b = [((key >> 42) & 0x1FFFFF) - (1 << 20), ((key >> 21) & 0x1FFFFF) - (1 << 20),
             (key & 0x1FFFFF) - (1 << 20)]
        for loc in np.nonzero(w)[0]:
            got[(8 * b[0] + loc % 8, 8 * b[1] + (loc // 8) % 8, 8 * b[2] + loc // 64)] = int(w[loc])
    for x in range(lo[0], hi[0] + 1):
        for y in range(lo[1], hi[1] + 1):
            for z in range(lo[2], hi[2] + 1):
                n = sum(1 for p in per_pixel if (x, y, z) in p)
                assert got.get((x, y, z), 0) == n


# ---------------------------------------------------------------------------
# Properties: order independence, pool overflow, range, invalid points
# ---------------------------------------------------------------------------

def test_reverse_order_same_keys_weights_and_means():
    w = S.single_frame_workload()
    a = O.fuse_workload(w)
    b = O.fuse_workload(w, reverse=True)
    assert np.array_equal(a.keys, b.keys)
    assert np.array_equal(a.weights, b.weights)
    assert np.max(np.abs(a.means - b.means)) < 1e-12


def test_two_frames_commute():
    cams, depths = [], []
    for k, pose in enumerate([S.IDENTITY_POSE, S.look_at_pose((0.1, -0.05, 0.0), (0.0, 0.0, 1.3))]):
        cam, d = S.plane_sphere_frame(seed=k, pose=pose)
        cams.append(cam)
        depths.append(d)
    a = O.fuse_frames(0.01, 0.04, 4096, depths, cams)
    b = O.fuse_frames(0.01, 0.04, 4096, depths[::-1], cams[::-1])
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.weights, b.weights)
    assert np.max(np.abs(a.means - b.means)) < 1e-12


def test_slices_add_up_to_the_sequential_fusion():
    """Fusion is a sum over frames: room-orbit frames cut into slices, each fused
    into its own volume (on threads), add up to fusing them one after another.
    The GPU test of the whole 300-frame trajectory relies on this."""
    from parity import add_slices, oracle_slices

    w = S.room_trajectory_workload(frames=[0, 1, 2, 60, 61, 150])
    seq = O.fuse_workload(w)
    parts = oracle_slices(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras, 3)
    sums, weights, seen, points, pairs = add_slices(parts, seq.keys)
    assert seen.all()
    assert np.array_equal(weights, seq.weights)
    assert np.max(np.abs(sums - seq.sums)) < 1e-9
    assert points == seq.stats["points_valid"] and pairs == seq.stats["pairs"]


def test_pool_overflow_first_keys_win_and_drops_are_counted():
    w = S.single_frame_workload()
    P = 100
    pr = O.frame_pairs(w.voxel_size, w.trunc, w.depth[0], w.cameras[0])
    order = []
    seen = set()
    for k in pr.keys.tolist():
        if k not in seen:
            seen.add(k)
            order.append(k)
    winners, losers = set(order[:P]), set(order[P:])
    r = O.fuse_frames(w.voxel_size, w.trunc, P, w.depth, w.cameras)
    assert set(r.keys.tolist()) == winners
    assert set(r.pool_overflow_keys.tolist()) == losers
    assert r.stats["pairs_dropped"] == sum(1 for k in pr.keys.tolist() if k in losers)
    assert r.stats["pairs"] == pr.keys.size


def test_prefilled_blocks_take_pool_space():
    w = S.single_frame_workload()
    pre = S.random_block_coords(4000, seed=9)
    r = O.fuse_frames(w.voxel_size, w.trunc, 4096, w.depth, w.cameras, prefill_blocks=pre)
    full = O.fuse_frames(w.voxel_size, w.trunc, 1 << 16, w.depth, w.cameras)
    n_scene = full.keys.size
    assert r.stats["blocks"] == 4096
    assert r.stats["pool_overflow_keys"] == n_scene - 96


def test_coordinates_out_of_range_are_counted_not_fused():
    cam, depth = S.plane_sphere_frame()
    pose = cam.pose.copy()
    pose[0, 3] = 1.0e5  # 10^5 m / 1 cm = 10^7 voxels > 2^23
    cam2 = S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, pose)
    r = O.fuse_frames(0.01, 0.04, 4096, [depth], [cam2])
    assert r.stats["blocks"] == 0 and r.stats["pairs"] == 0
    assert r.stats["coord_out_of_range"] == 9 * r.stats["points_valid"] == 9 * 19200


def test_invalid_depths_are_not_points():
    cam, depth = S.plane_sphere_frame()
    d = depth.copy()
    d[0, :] = np.nan
    d[1, :] = np.inf
    d[2, :] = 0.0
    d[3, :] = -1.0
    d[4, :] = -np.inf
    r = O.fuse_frames(0.01, 0.04, 4096, [d], [cam])
    assert r.stats["points_valid"] == 19200 - 5 * 160
    empty = np.zeros_like(depth)
    r0 = O.fuse_frames(0.01, 0.04, 4096, [empty], [cam])
    assert r0.stats["points_valid"] == 0 and r0.stats["blocks"] == 0
