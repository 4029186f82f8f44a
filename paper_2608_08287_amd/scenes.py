"""Seeded synthetic depth inputs for hash-blocked TSDF fusion.

This module only *makes inputs*: it ray-casts analytic scenes (planes, spheres,
axis-aligned boxes) into float32 depth images for a pinhole camera and builds the
camera intrinsics and camera->world poses.  It holds none of the fusion
arithmetic, so both the GPU path and the CPU oracle can consume what it makes.

Conventions (shared by every consumer, stated here once):

* depth ``D[y, x]`` is the camera-frame z (metres) of the first surface hit by the
  ray of integer pixel ``(x, y)``; the ray direction in the camera frame is
  ``((x - cx) / fx, (y - cy) / fy, 1)``, so the ray parameter at the hit equals
  the camera-frame z.  Pixels whose ray hits nothing hold ``0`` (invalid).
* pose = camera->world ``[R | t]`` as a row-major 3x4 float32 array
  (OpenCV camera: x right, y down, z forward).
* geometry is evaluated in float64; noise is drawn with
  ``numpy.random.default_rng(seed)`` and added in float64; the result is cast to
  float32 once.

The ray caster runs on any torch device (CPU in tests, the GPU for large
trajectories).  The same array is handed to every consumer of a given run, so
the device used to make it never affects a comparison.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch


@dataclasses.dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    pose: np.ndarray  # (3, 4) float32, camera->world, row-major

    def intrinsics(self) -> Tuple[float, float, float, float]:
        return (self.fx, self.fy, self.cx, self.cy)


@dataclasses.dataclass(frozen=True)
class Plane:
    """Points p with dot(n, p) == offset (n unit, float64)."""
    normal: Tuple[float, float, float]
    offset: float


@dataclasses.dataclass(frozen=True)
class Sphere:
    center: Tuple[float, float, float]
    radius: float


@dataclasses.dataclass(frozen=True)
class Box:
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]


@dataclasses.dataclass(frozen=True)
class RoomInterior:
    """The inside faces of an axis-aligned box that contains the camera."""
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]


IDENTITY_POSE = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], dtype=np.float32)


def look_at_pose(eye: Sequence[float], target: Sequence[float],
                 up: Sequence[float] = (0.0, 1.0, 0.0)) -> np.ndarray:
    """OpenCV camera at ``eye`` looking at ``target``; world ``up`` is +y.

    R = [x | y | z] (columns) with z = normalise(target - eye),
    x = normalise(z cross up), y = z cross x.  Returned as float32 3x4.
    """
    eye = np.asarray(eye, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    pose = np.zeros((3, 4), dtype=np.float64)
    pose[:, 0], pose[:, 1], pose[:, 2], pose[:, 3] = x, y, z, eye
    return pose.astype(np.float32)


def _ray_dirs(cam: Camera, device) -> Tuple[torch.Tensor, torch.Tensor]:
    """World-frame ray directions (N, 3) with unit camera-z, and the origin (3,)."""
    ys, xs = torch.meshgrid(torch.arange(cam.height, dtype=torch.float64, device=device),
                            torch.arange(cam.width, dtype=torch.float64, device=device),
                            indexing="ij")
    dc = torch.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy,
                      torch.ones_like(xs)], dim=-1).reshape(-1, 3)
    pose = torch.as_tensor(cam.pose.astype(np.float64), device=device)
    dw = dc @ pose[:, :3].T
    return dw, pose[:, 3]


def _hit_plane(o, d, p: Plane):
    n = torch.tensor(p.normal, dtype=torch.float64, device=d.device)
    den = d @ n
    t = (p.offset - torch.dot(o, n)) / den
    return torch.where((den.abs() > 1e-12) & (t > 0), t, torch.full_like(t, math.inf))


def _hit_sphere(o, d, s: Sphere):
    c = torch.tensor(s.center, dtype=torch.float64, device=d.device)
    oc = o - c
    a = (d * d).sum(-1)
    b = d @ oc
    cc = torch.dot(oc, oc) - s.radius * s.radius
    disc = b * b - a * cc
    sq = torch.sqrt(torch.clamp(disc, min=0.0))
    t0 = (-b - sq) / a
    t1 = (-b + sq) / a
    t = torch.where(t0 > 0, t0, t1)
    return torch.where((disc >= 0) & (t > 0), t, torch.full_like(t, math.inf))


def _slab(o, d, lo, hi):
    lo = torch.tensor(lo, dtype=torch.float64, device=d.device)
    hi = torch.tensor(hi, dtype=torch.float64, device=d.device)
    inv = 1.0 / torch.where(d == 0, torch.full_like(d, 1e-300), d)
    ta = (lo - o) * inv
    tb = (hi - o) * inv
    tmin = torch.minimum(ta, tb).amax(-1)
    tmax = torch.maximum(ta, tb).amin(-1)
    return tmin, tmax


def _hit_box(o, d, b: Box):
    tmin, tmax = _slab(o, d, b.lo, b.hi)
    t = torch.where(tmin > 0, tmin, tmax)
    return torch.where((tmax >= torch.clamp(tmin, min=0.0)) & (t > 0), t, torch.full_like(t, math.inf))


def _hit_room(o, d, r: RoomInterior):
    _, tmax = _slab(o, d, r.lo, r.hi)
    return torch.where(tmax > 0, tmax, torch.full_like(tmax, math.inf))


_HITTERS = {Plane: _hit_plane, Sphere: _hit_sphere, Box: _hit_box, RoomInterior: _hit_room}


def render_depth(cam: Camera, scene: Sequence[object], noise_sigma=None,
                 seed: Optional[int] = None, device="cpu") -> np.ndarray:
    """Ray-cast ``scene`` for ``cam`` and return float32 depth of shape (H, W).

    ``noise_sigma`` is ``None`` (no noise), a float (constant sigma, metres) or a
    callable ``sigma(z)`` applied elementwise to the float64 depth.  Noise is
    standard normal from ``default_rng(seed)`` in row-major pixel order, drawn
    for every pixel (valid or not) so the stream does not depend on the scene.
    """
    d, o = _ray_dirs(cam, device)
    t = torch.full((d.shape[0],), math.inf, dtype=torch.float64, device=device)
    for prim in scene:
        t = torch.minimum(t, _HITTERS[type(prim)](o, d, prim))
    depth = t.cpu().numpy()
    hit = np.isfinite(depth)
    if noise_sigma is not None:
        rng = np.random.default_rng(seed)
        g = rng.standard_normal(depth.shape[0])
        sig = noise_sigma(depth) if callable(noise_sigma) else np.full_like(depth, noise_sigma)
        depth = np.where(hit, depth + g * np.where(hit, sig, 0.0), depth)
    depth = np.where(hit, depth, 0.0)
    return depth.astype(np.float32).reshape(cam.height, cam.width)


def render_rgbd(cam: Camera, scene: Sequence[object], colours: Sequence[Tuple[int, int, int]],
                noise_sigma=None, seed: Optional[int] = None,
                device="cpu") -> Tuple[np.ndarray, np.ndarray]:
    """Depth as ``render_depth`` (same noise stream) and a registered colour
    image: each pixel takes the 8-bit colour ``colours[i]`` of the primitive
    its ray hits first, darkened to 5/8 on alternate cells of a 10 cm checker
    in world coordinates (so colour varies across a surface).  Colour is
    packed as uint32 red | green << 8 | blue << 16; rays that hit nothing are
    black."""
    d, o = _ray_dirs(cam, device)
    t = torch.full((d.shape[0],), math.inf, dtype=torch.float64, device=device)
    which = torch.full((d.shape[0],), -1, dtype=torch.int64, device=device)
    for i, prim in enumerate(scene):
        ti = _HITTERS[type(prim)](o, d, prim)
        closer = ti < t
        which = torch.where(closer, torch.full_like(which, i), which)
        t = torch.minimum(t, ti)
    depth = render_depth(cam, scene, noise_sigma, seed, device)
    hit = torch.isfinite(t)
    p = o + d * torch.where(hit, t, torch.zeros_like(t))[:, None]
    cell = torch.floor(p / 0.1).sum(dim=1).remainder(2).cpu().numpy()
    which = which.cpu().numpy()
    hit = hit.cpu().numpy()
    table = np.asarray(colours, dtype=np.int64).reshape(-1, 3)
    rgb = np.where(hit[:, None], table[np.maximum(which, 0)], 0)
    rgb = np.where(cell[:, None] == 1, (rgb * 5) // 8, rgb)
    packed = (rgb[:, 0] | (rgb[:, 1] << 8) | (rgb[:, 2] << 16)).astype(np.uint32)
    return depth, packed.reshape(cam.height, cam.width)


def scene_colours(n: int, seed: int) -> List[Tuple[int, int, int]]:
    """``n`` seeded 8-bit colours, channels uniform on 32..255."""
    rng = np.random.default_rng(seed)
    return [tuple(int(c) for c in rng.integers(32, 256, size=3)) for _ in range(n)]


# ---------------------------------------------------------------------------
# The workloads.  Each returns (cameras, depth frames) plus the volume sizes.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    voxel_size: float
    trunc: float
    table_capacity: int
    pool_capacity: int
    cameras: List[Camera]
    depth: List[np.ndarray]
    prefill_blocks: Optional[np.ndarray] = None  # (n, 3) int32 block coords allocated before fusion


def plane_sphere_frame(noise: bool = True, seed: int = 0, width=160, height=120,
                       fx=140.0, fy=140.0, cx=80.0, cy=60.0, pose=None) -> Tuple[Camera, np.ndarray]:
    """Plane z = 1.5 m behind a sphere r = 0.3 m at (0, 0, 1.2), identity pose."""
    cam = Camera(width, height, fx, fy, cx, cy, IDENTITY_POSE if pose is None else pose)
    scene = [Plane((0.0, 0.0, 1.0), 1.5), Sphere((0.0, 0.0, 1.2), 0.3)]
    return cam, render_depth(cam, scene, 0.001 if noise else None, seed)


def single_frame_workload(noise: bool = True) -> Workload:
    """160x120 plane + sphere, 1 cm voxels, 4 cm truncation, 8192 slots, 4096 blocks."""
    cam, depth = plane_sphere_frame(noise=noise, seed=0)
    return Workload("plane_sphere_160x120", 0.01, 0.04, 8192, 4096, [cam], [depth])


def room_scene(seed: int = 1, n_objects: int = 20) -> List[object]:
    """A 4 m x 3 m x 4 m room (x, z in [-2, 2], y in [0, 3]) with seeded objects.

    Each object is a sphere (diameter ~ U(0.1, 0.6)) or an axis-aligned box (each
    side ~ U(0.1, 0.6)) with probability 1/2, centred at x, z ~ U(-1.4, 1.4),
    y ~ U(0.2, 2.0).
    """
    rng = np.random.default_rng(seed)
    scene: List[object] = [RoomInterior((-2.0, 0.0, -2.0), (2.0, 3.0, 2.0))]
    for _ in range(n_objects):
        is_sphere = rng.random() < 0.5
        c = (rng.uniform(-1.4, 1.4), rng.uniform(0.2, 2.0), rng.uniform(-1.4, 1.4))
        if is_sphere:
            scene.append(Sphere(c, 0.5 * rng.uniform(0.1, 0.6)))
        else:
            half = 0.5 * rng.uniform(0.1, 0.6, size=3)
            scene.append(Box(tuple(np.subtract(c, half)), tuple(np.add(c, half))))
    return scene


def orbit_camera(k: int, n_frames: int = 300, width=640, height=480, f=525.0,
                 radius=2.0, height_m=1.2, target=(0.0, 1.5, 0.0)) -> Camera:
    th = 2.0 * math.pi * k / n_frames
    eye = (radius * math.cos(th), height_m, radius * math.sin(th))
    return Camera(width, height, f * width / 640.0, f * width / 640.0,
                  (width - 1) / 2.0, (height - 1) / 2.0, look_at_pose(eye, target))


def room_trajectory_workload(n_frames: int = 300, frames: Optional[Sequence[int]] = None,
                             device="cpu", table_capacity=1 << 20,
                             pool_capacity=1 << 18) -> Workload:
    """Orbit (radius 2 m, height 1.2 m) of a 640x480 camera round the room centre.

    Noise sigma = 0.002 * z^2 with seed 1000 + k for frame k.  Voxel 5 mm,
    truncation 2 cm.  ``frames`` selects a subset of the ``n_frames`` orbit.
    """
    scene = room_scene(1)
    ks = range(n_frames) if frames is None else frames
    cams, depth = [], []
    for k in ks:
        cam = orbit_camera(k, n_frames)
        cams.append(cam)
        depth.append(render_depth(cam, scene, lambda z: 0.002 * z * z, 1000 + k, device))
    return Workload("room_orbit_640x480", 0.005, 0.02, table_capacity, pool_capacity, cams, depth)


def room_trajectory_rgbd(n_frames: int = 300, frames: Optional[Sequence[int]] = None,
                         device="cpu") -> Tuple[Workload, List[np.ndarray]]:
    """The room orbit of ``room_trajectory_workload`` with a colour image per
    frame (``render_rgbd``, object colours from ``scene_colours(21, 77)``);
    the depth frames are the same arrays."""
    scene = room_scene(1)
    colours = scene_colours(len(scene), 77)
    ks = range(n_frames) if frames is None else frames
    cams, depth, rgba = [], [], []
    for k in ks:
        cam = orbit_camera(k, n_frames)
        d, c = render_rgbd(cam, scene, colours, lambda z: 0.002 * z * z, 1000 + k, device)
        cams.append(cam)
        depth.append(d)
        rgba.append(c)
    w = Workload("room_orbit_rgbd_640x480", 0.005, 0.02, 1 << 20, 1 << 18, cams, depth)
    return w, rgba


def random_block_coords(n: int, seed: int, exclude_radius: int = 1 << 10) -> np.ndarray:
    """``n`` distinct int32 block coordinates (rows of (bx, by, bz)) uniform on
    [-2^20, 2^20)^3, excluding blocks with every |coordinate| < ``exclude_radius``
    (the neighbourhood the scenes occupy).  First-drawn order is kept."""
    rng = np.random.default_rng(seed)
    out = np.empty((0, 3), dtype=np.int64)
    while out.shape[0] < n:
        b = rng.integers(-(1 << 20), 1 << 20, size=(2 * (n - out.shape[0]) + 16, 3), dtype=np.int64)
        b = b[~np.all(np.abs(b) < exclude_radius, axis=1)]
        out = np.concatenate([out, b])
        _, first = np.unique(out, axis=0, return_index=True)
        out = out[np.sort(first)]
    return out[:n].astype(np.int32)


def plane_stress_workload(sub_case: str = "A", n_frames: int = 100,
                          frames: Optional[Sequence[int]] = None, device="cpu") -> Workload:
    """Contention and overflow stress: fronto-parallel plane at 0.5 m, 640x480.

    sigma = 0.5 mm (seed 2000 + k), voxel 4 mm, truncation 1.6 cm, table of 2^16
    slots pre-filled with seeded random blocks:

    * ``A``: 62,259 blocks (load factor 0.95), pool 2^16;
    * ``B``: as A with the pool 100 blocks larger than the pre-fill;
    * ``C``: 2^16 - 50 blocks, pool 2^17 (the table fills up);
    * ``plain``: no pre-fill (table 2^16, pool 2^16).
    """
    C = 1 << 16
    if sub_case == "A":
        n_pre, pool = 62259, 1 << 16
    elif sub_case == "B":
        n_pre, pool = 62259, 62259 + 100
    elif sub_case == "C":
        n_pre, pool = C - 50, 1 << 17
    elif sub_case == "plain":
        n_pre, pool = 0, 1 << 16
    else:
        raise ValueError(sub_case)
    scene = [Plane((0.0, 0.0, 1.0), 0.5)]
    ks = range(n_frames) if frames is None else frames
    cams, depth = [], []
    for k in ks:
        cam = Camera(640, 480, 525.0, 525.0, 319.5, 239.5, IDENTITY_POSE)
        cams.append(cam)
        depth.append(render_depth(cam, scene, 0.0005, 2000 + k, device))
    pre = random_block_coords(n_pre, seed=3) if n_pre else None
    return Workload(f"plane_stress_{sub_case}", 0.004, 0.016, C, pool, cams, depth, pre)


# ---------------------------------------------------------------------------
# Many independent volumes, one frame each per tick.
# ---------------------------------------------------------------------------

FRAME_SIZES = ((160, 120), (320, 240), (640, 480), (1280, 720))


@dataclasses.dataclass(frozen=True)
class VolumeSpec:
    width: int
    height: int
    voxel_size: float
    trunc: float
    table_capacity: int
    pool_capacity: int
    scene_seed: int
    orbit_offset: int   # orbit frame of tick 0
    noise_seed: int     # tick k draws its noise with seed noise_seed + k


class MultiVolumeWorkload:
    """``n_volumes`` independent reconstructions, each fed one frame per tick.

    From ``default_rng(seed)``: per volume a frame size uniform over ``sizes``,
    a voxel edge uniform over 5..10 mm (whole millimetres) and a table exponent
    e uniform over ``log2_tables[0]..log2_tables[1]``; then the drawn exponents
    are dealt to the volumes in the reverse order of their voxel edges (the
    finest voxels get the largest tables; ties keep volume order), which keeps
    every marginal uniform while giving each volume room for its surface: a
    pool that runs out turns every later new key into a probe of a full table.
    Truncation is 4 voxels, the table 2^e slots, the pool half the table.  Each
    volume has its own room scene (``room_scene`` with a drawn seed) and its own
    starting point on the 300-frame orbit; intrinsics scale with the width
    (``orbit_camera``).  Tick k gives volume i orbit frame ``orbit_offset + k``
    with noise sigma 0.002 z^2, seed ``noise_seed + k``.
    """

    def __init__(self, n_volumes: int = 64, seed: int = 3, sizes=FRAME_SIZES,
                 log2_tables=(16, 20), n_orbit: int = 300):
        rng = np.random.default_rng(seed)
        self.n_orbit = n_orbit
        size_idx = rng.integers(0, len(sizes), size=n_volumes)
        voxel_mm = rng.integers(5, 11, size=n_volumes)
        exps = rng.integers(log2_tables[0], log2_tables[1] + 1, size=n_volumes)
        scene_seeds = rng.integers(1, 1 << 30, size=n_volumes)
        offsets = rng.integers(0, n_orbit, size=n_volumes)
        exp_of = np.empty(n_volumes, dtype=np.int64)
        exp_of[np.argsort(voxel_mm, kind="stable")] = np.sort(exps)[::-1]
        self.specs: List[VolumeSpec] = []
        for i in range(n_volumes):
            w, h = sizes[int(size_idx[i])]
            v = int(voxel_mm[i]) * 1e-3
            e = int(exp_of[i])
            self.specs.append(VolumeSpec(
                width=w, height=h, voxel_size=v, trunc=4.0 * v, table_capacity=1 << e,
                pool_capacity=1 << (e - 1), scene_seed=int(scene_seeds[i]),
                orbit_offset=int(offsets[i]), noise_seed=(i + 1) * 100000))
        self._scenes = [room_scene(s.scene_seed) for s in self.specs]

    def __len__(self) -> int:
        return len(self.specs)

    def camera(self, i: int, tick: int) -> Camera:
        s = self.specs[i]
        return orbit_camera((s.orbit_offset + tick) % self.n_orbit, self.n_orbit, s.width, s.height)

    def depth(self, i: int, tick: int, device="cpu") -> np.ndarray:
        return render_depth(self.camera(i, tick), self._scenes[i], lambda z: 0.002 * z * z,
                            self.specs[i].noise_seed + tick, device)

    def pixels(self) -> int:
        return sum(s.width * s.height for s in self.specs)


class ServingWorkload:
    """Reconstruction sessions fed by Poisson frame arrivals.

    From ``default_rng(seed)``: per session a frame size uniform over
    ``sizes``, a voxel edge uniform over 5..10 mm and a pool exponent e
    uniform over ``log2_pools[0]..log2_pools[1]``; the exponents are dealt
    largest first to the sessions ordered by voxel edge, then by frame area
    from the largest (the finest voxels and, among equal voxels, the largest
    frames touch the most blocks), which keeps every marginal uniform.  Pool
    2^e blocks, table twice the pool (the paper's sizing), truncation 4 voxels,
    an own room scene and orbit start.  Arrivals form one Poisson process of
    ``rate`` frames/s (exponential gaps), each arrival going to a session drawn
    uniformly, so every session sees a Poisson process of rate / n.  A
    session's k-th frame is its orbit frame ``orbit_offset + k`` with noise
    seed ``noise_seed + k``.
    """

    def __init__(self, n_sessions: int = 256, rate: float = 3000.0, duration_s: float = 1.0,
                 seed: int = 4, sizes=FRAME_SIZES, log2_pools=(14, 18), n_orbit: int = 300):
        rng = np.random.default_rng(seed)
        self.n_orbit = n_orbit
        size_idx = rng.integers(0, len(sizes), size=n_sessions)
        voxel_mm = rng.integers(5, 11, size=n_sessions)
        exps = rng.integers(log2_pools[0], log2_pools[1] + 1, size=n_sessions)
        scene_seeds = rng.integers(1, 1 << 30, size=n_sessions)
        offsets = rng.integers(0, n_orbit, size=n_sessions)
        area = np.array([sizes[int(k)][0] * sizes[int(k)][1] for k in size_idx])
        exp_of = np.empty(n_sessions, dtype=np.int64)
        exp_of[np.lexsort((-area, voxel_mm))] = np.sort(exps)[::-1]
        self.specs: List[VolumeSpec] = []
        for i in range(n_sessions):
            w, h = sizes[int(size_idx[i])]
            v = int(voxel_mm[i]) * 1e-3
            e = int(exp_of[i])
            self.specs.append(VolumeSpec(
                width=w, height=h, voxel_size=v, trunc=4.0 * v, table_capacity=1 << (e + 1),
                pool_capacity=1 << e, scene_seed=int(scene_seeds[i]),
                orbit_offset=int(offsets[i]), noise_seed=(i + 1) * 100000 + 7))
        gaps = rng.exponential(1.0 / rate, size=int(rate * duration_s * 1.5) + 16)
        t = np.cumsum(gaps)
        t = t[t < duration_s]
        self.arrival_ns = np.round(t * 1e9).astype(np.int64)
        self.session_of = rng.integers(0, n_sessions, size=t.size)
        # frame index within its session
        self.frame_of = np.zeros(t.size, dtype=np.int64)
        seen = np.zeros(n_sessions, dtype=np.int64)
        for j, s in enumerate(self.session_of):
            self.frame_of[j] = seen[s]
            seen[s] += 1
        self._scenes = {}

    def __len__(self) -> int:
        return int(self.arrival_ns.size)

    def camera(self, session: int, k: int) -> Camera:
        s = self.specs[session]
        return orbit_camera((s.orbit_offset + k) % self.n_orbit, self.n_orbit, s.width, s.height)

    def depth(self, session: int, k: int, device="cpu") -> np.ndarray:
        if session not in self._scenes:
            self._scenes[session] = room_scene(self.specs[session].scene_seed)
        return render_depth(self.camera(session, k), self._scenes[session],
                            lambda z: 0.002 * z * z, self.specs[session].noise_seed + k, device)
