"""TEST INFRASTRUCTURE ONLY: ctypes binding of the sequential CPU oracle.

Only tests, the smoke check and the CPU-baseline leg of the benchmark use this.
The oracle's arithmetic lives in ``tsdf_oracle.cpp``; this file only marshals
numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIBRARY may name the sanitized build of the same source
_LIB_PATH = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P, U32, U64, I32, F32, I64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_float, C.c_int64
        L.ora_create.restype = P
        L.ora_create.argtypes = [F32, F32, U32]
        L.ora_destroy.argtypes = [P]
        L.ora_band_samples.argtypes = [P]
        L.ora_insert_blocks.argtypes = [P, P, U64]
        L.ora_fuse.argtypes = [P, P, U32, U32, P, P, C.c_int]
        L.ora_stats.argtypes = [P, P]
        L.ora_export.restype = U64
        L.ora_export.argtypes = [P, P, P, P, P, U64]
        L.ora_export_overflow_keys.restype = U64
        L.ora_export_overflow_keys.argtypes = [P, P, U64]
        L.ora_frame_pairs.restype = U64
        L.ora_frame_pairs.argtypes = [F32, F32, P, U32, U32, P, P, C.c_int, P, P, P, P, U64, P]
        L.ora_pack_key.restype = U64
        L.ora_pack_key.argtypes = [I32, I32, I32]
        L.ora_block_of.restype = I64
        L.ora_block_of.argtypes = [I64]
        L.ora_fmix64.restype = U64
        L.ora_fmix64.argtypes = [U64]
        L.ora_home_slot.restype = U32
        L.ora_home_slot.argtypes = [U64, U32]
        L.ora_probe_model.restype = U64
        L.ora_probe_model.argtypes = [P, U64, U32, P, P, P]
        L.ora_set_block.argtypes = [P, U64, P, P]
        L.ora_fuse_rgb.argtypes = [P, P, P, U32, U32, P, P, C.c_int]
        L.ora_export_colour.restype = U64
        L.ora_export_colour.argtypes = [P, P, U64]
        L.ora_extract_mesh.restype = U64
        L.ora_extract_mesh.argtypes = [P, P, P, P, U64]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _cam_arrays(cam):
    intr = np.asarray([cam.fx, cam.fy, cam.cx, cam.cy], dtype=np.float32)
    pose = np.ascontiguousarray(np.asarray(cam.pose, dtype=np.float32).reshape(3, 4))
    return intr, pose


@dataclass
class OracleMesh:
    ids: np.ndarray    # (T, 2) uint64: block key, cube << 4 | tetrahedron << 1 | triangle
    verts: np.ndarray  # (T, 3, 3) float64 vertex positions (metres)
    edges: np.ndarray  # (T, 3, 2, 3) int64: per vertex, the grid edge's two corners


@dataclass
class OracleResult:
    keys: np.ndarray      # (B,) uint64, ascending
    sums: np.ndarray      # (B, 512) float64
    means: np.ndarray     # (B, 512) float64, 0 where weight == 0
    weights: np.ndarray   # (B, 512) uint32
    stats: dict
    pool_overflow_keys: np.ndarray


class OracleVolume:
    """Sequential model of one TSDF volume (pool of ``pool_capacity`` blocks)."""

    def __init__(self, voxel_size: float, trunc: float, pool_capacity: int):
        self._h = lib().ora_create(voxel_size, trunc, pool_capacity)
        if not self._h:
            raise ValueError("invalid oracle volume parameters")
        self._destroy = lib().ora_destroy  # still reachable at interpreter exit

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def insert_blocks(self, coords: np.ndarray) -> None:
        c = np.ascontiguousarray(coords, dtype=np.int32).reshape(-1, 3)
        if lib().ora_insert_blocks(self._h, _ptr(c), c.shape[0]) != 0:
            raise ValueError("block coordinate outside the 21-bit range")

    def fuse(self, depth: np.ndarray, cam, reverse: bool = False) -> None:
        d = np.ascontiguousarray(depth, dtype=np.float32)
        intr, pose = _cam_arrays(cam)
        H, W = d.shape
        if lib().ora_fuse(self._h, _ptr(d), W, H, _ptr(intr), _ptr(pose), int(reverse)) != 0:
            raise ValueError("invalid frame")

    def fuse_rgb(self, depth: np.ndarray, rgba: np.ndarray, cam, reverse: bool = False) -> None:
        """As fuse, also adding each contribution's pixel colour (packed uint32
        red | green << 8 | blue << 16) to the voxel's colour sums."""
        d = np.ascontiguousarray(depth, dtype=np.float32)
        c = np.ascontiguousarray(rgba, dtype=np.uint32)
        if c.shape != d.shape:
            raise ValueError("colour image does not match the depth image")
        intr, pose = _cam_arrays(cam)
        H, W = d.shape
        if lib().ora_fuse_rgb(self._h, _ptr(d), _ptr(c), W, H, _ptr(intr), _ptr(pose),
                              int(reverse)) != 0:
            raise ValueError("invalid frame")

    def colour_sums(self) -> np.ndarray:
        """(B, 3, 512) float64 red, green, blue sums, blocks in ascending key order."""
        L = lib()
        nb = int(L.ora_export(self._h, None, None, None, None, 0))
        out = np.zeros((nb, 3, 512), dtype=np.float64)
        L.ora_export_colour(self._h, _ptr(out), nb)
        return out

    def stats(self) -> dict:
        out = np.zeros(8, dtype=np.uint64)
        lib().ora_stats(self._h, _ptr(out))
        names = ["points_valid", "pairs", "pairs_dropped", "coord_out_of_range", "blocks",
                 "pool_overflow_keys", "frames", "pool_capacity"]
        return {n: int(v) for n, v in zip(names, out)}

    def set_block(self, key: int, sums: np.ndarray, weights: np.ndarray) -> None:
        """Replace (or create) one block's 512 sums and weights (x fastest)."""
        sm = np.ascontiguousarray(sums, dtype=np.float64).reshape(512)
        w = np.ascontiguousarray(weights, dtype=np.uint32).reshape(512)
        lib().ora_set_block(self._h, int(key), _ptr(sm), _ptr(w))

    def mesh(self) -> "OracleMesh":
        """Marching-tetrahedra surface of the volume (see ora_extract_mesh)."""
        L = lib()
        n = int(L.ora_extract_mesh(self._h, None, None, None, 0))
        ids = np.zeros((n, 2), dtype=np.uint64)
        verts = np.zeros((n, 3, 3), dtype=np.float64)
        edges = np.zeros((n, 3, 2, 3), dtype=np.int64)
        L.ora_extract_mesh(self._h, _ptr(ids), _ptr(verts), _ptr(edges), n)
        return OracleMesh(ids, verts, edges)

    def result(self) -> OracleResult:
        L = lib()
        nb = int(L.ora_export(self._h, None, None, None, None, 0))
        keys = np.zeros(nb, dtype=np.uint64)
        sums = np.zeros((nb, 512), dtype=np.float64)
        means = np.zeros((nb, 512), dtype=np.float64)
        w = np.zeros((nb, 512), dtype=np.uint32)
        L.ora_export(self._h, _ptr(keys), _ptr(sums), _ptr(means), _ptr(w), nb)
        no = int(L.ora_export_overflow_keys(self._h, None, 0))
        ok = np.zeros(no, dtype=np.uint64)
        L.ora_export_overflow_keys(self._h, _ptr(ok), no)
        return OracleResult(keys, sums, means, w, self.stats(), ok)


def fuse_frames(voxel_size: float, trunc: float, pool_capacity: int, depths: Sequence[np.ndarray],
                cams: Sequence, prefill_blocks: Optional[np.ndarray] = None,
                reverse: bool = False) -> OracleResult:
    vol = OracleVolume(voxel_size, trunc, pool_capacity)
    if prefill_blocks is not None:
        vol.insert_blocks(prefill_blocks)
    order = range(len(depths) - 1, -1, -1) if reverse else range(len(depths))
    for i in order:
        vol.fuse(depths[i], cams[i], reverse=reverse)
    return vol.result()


def fuse_workload(w, reverse: bool = False) -> OracleResult:
    return fuse_frames(w.voxel_size, w.trunc, w.pool_capacity, w.depth, w.cameras,
                       w.prefill_blocks, reverse)


@dataclass
class FramePairs:
    keys: np.ndarray    # uint64
    locs: np.ndarray    # uint32
    vals: np.ndarray    # float32
    voxels: np.ndarray  # (n, 3) int32
    points_valid: int
    coord_out_of_range: int


def frame_pairs(voxel_size: float, trunc: float, depth: np.ndarray, cam,
                reverse: bool = False) -> FramePairs:
    L = lib()
    d = np.ascontiguousarray(depth, dtype=np.float32)
    intr, pose = _cam_arrays(cam)
    H, W = d.shape
    counts = np.zeros(3, dtype=np.uint64)
    n = L.ora_frame_pairs(voxel_size, trunc, _ptr(d), W, H, _ptr(intr), _ptr(pose), int(reverse),
                          None, None, None, None, 0, _ptr(counts))
    if n == 2 ** 64 - 1:
        raise ValueError("invalid parameters")
    keys = np.zeros(n, dtype=np.uint64)
    locs = np.zeros(n, dtype=np.uint32)
    vals = np.zeros(n, dtype=np.float32)
    vox = np.zeros((n, 3), dtype=np.int32)
    L.ora_frame_pairs(voxel_size, trunc, _ptr(d), W, H, _ptr(intr), _ptr(pose), int(reverse),
                      _ptr(keys), _ptr(locs), _ptr(vals), _ptr(vox), n, _ptr(counts))
    return FramePairs(keys, locs, vals, vox, int(counts[0]), int(counts[2]))


def pack_key(bx: int, by: int, bz: int) -> int:
    return int(lib().ora_pack_key(bx, by, bz))


def block_of(v: int) -> int:
    return int(lib().ora_block_of(v))


def fmix64(k: int) -> int:
    return int(lib().ora_fmix64(k))


def home_slot(key: int, C: int) -> int:
    return int(lib().ora_home_slot(key, C))


@dataclass
class ProbeModel:
    slot_of: np.ndarray    # int64 per input key (-1 = overflowed)
    disp_of: np.ndarray    # uint64 per input key
    table: np.ndarray      # uint64 (C,), EMPTY = 2^64-1
    n_overflow: int

    @property
    def occupied(self) -> np.ndarray:
        return np.nonzero(self.table != np.uint64(2 ** 64 - 1))[0]


def probe_model(keys: np.ndarray, C: int) -> ProbeModel:
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    slot = np.zeros(k.size, dtype=np.int64)
    disp = np.zeros(k.size, dtype=np.uint64)
    table = np.zeros(C, dtype=np.uint64)
    nof = lib().ora_probe_model(_ptr(k), k.size, C, _ptr(slot), _ptr(disp), _ptr(table))
    return ProbeModel(slot, disp, table, int(nof))
