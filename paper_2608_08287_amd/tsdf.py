"""Python binding of ``libtsdf.so`` (ctypes).  Argument marshalling only.

Every step of fusion runs in the HIP kernels behind the C ABI of
``include/tsdf.h``; PyTorch supplies device memory (a ``torch.uint8`` arena per
volume, depth frames, extraction outputs) and the ``hipStream_t`` to enqueue on.
There is no CPU fallback: if the library is not built, or no GPU is present,
the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# TSDF_LIBRARY may name a library built from the same sources with one design
# alternative switched on (build.py --variant), for measuring it.
LIB_PATH = os.environ.get("TSDF_LIBRARY") or os.path.join(_HERE, "libtsdf.so")

# tsdf_status
OK, ERR_INVALID_ARGUMENT, ERR_BUFFER_TOO_SMALL, ERR_POOL_EXHAUSTED, ERR_TABLE_FULL, \
    ERR_COORD_RANGE, ERR_INTERNAL, ERR_HIP, ERR_BUDGET = range(9)
FLAG_POOL_EXHAUSTED, FLAG_TABLE_FULL, FLAG_COORD_RANGE, FLAG_INTERNAL = 1, 2, 4, 8
FLAG_OVERFLOW_RECORD_FULL = 0x10
OVERFLOW_KEY_SLOTS = 8192
FUSE_DEFAULT, FUSE_TWO_PASS, FUSE_ALLOCATE_ONLY, FUSE_INTEGRATE_ONLY = 0, 1, 2, 3
FUSE_XCD_REMAP = 0x100
FUSE_ONE_STREAM = 0x200
VOLUME_SLOT_INDEX, VOLUME_COLOUR, VOLUME_PROBE_HISTOGRAM = 0x1, 0x2, 0x4
PROBE_HIST_BINS = 16


def FUSE_BATCH(m: int) -> int:
    """Flag for ``fuse_frames``: frames summed per workgroup (m = 1 to 4 -> m,
    5..15 -> 4; 0, the default, -> 3; at most 2 for bands wider than 9
    samples and for colour volumes)."""
    return (m & 0xF) << 16
BLOCK_VOXELS = 512
EMPTY_KEY = 0xFFFFFFFFFFFFFFFF

EXPORTED_SYMBOLS = (
    "tsdf_volume_bytes", "tsdf_volume_layout", "tsdf_create_volume", "tsdf_destroy_volume",
    "tsdf_reset_volume", "tsdf_fuse_frame", "tsdf_fuse_frame_ex", "tsdf_fuse_frames",
    "tsdf_fuse_frames_rgb", "tsdf_staging_bytes", "tsdf_fuse_frames_staged",
    "tsdf_query_status", "tsdf_probe_histogram", "tsdf_measure_atomic_rate",
    "tsdf_extract_blocks", "tsdf_extract_mesh", "tsdf_insert_blocks", "tsdf_status_str",
    "tsdf_fuse_frame_rgb", "tsdf_extract_colour",
    "tsdf_batch_workspace_bytes", "tsdf_batch_create", "tsdf_batch_destroy",
    "tsdf_batch_set_config", "tsdf_batch_autotune", "tsdf_batch_get_config",
    "tsdf_batch_candidates", "tsdf_batch_fuse", "tsdf_batch_fuse_static",
    "tsdf_region_create", "tsdf_region_destroy", "tsdf_region_alloc", "tsdf_region_free",
    "tsdf_region_usage",
    "tsdf_server_workspace_bytes", "tsdf_server_create", "tsdf_server_destroy", "tsdf_server_open",
    "tsdf_server_close", "tsdf_server_submit", "tsdf_server_step", "tsdf_server_completions",
    "tsdf_server_session", "tsdf_server_batch", "tsdf_server_load", "tsdf_server_replay",
)
REPLAY_SERVED, REPLAY_PLAIN = 0, 1
BATCH_NO_GRAPH = 0x1
BATCH_MAX_ITEMS = 65536
STATIC_LIST_BYTES = 1 << 20


class VolumeParams(C.Structure):
    _fields_ = [("voxel_size", C.c_float), ("trunc", C.c_float),
                ("table_capacity", C.c_uint32), ("pool_capacity", C.c_uint32),
                ("flags", C.c_uint32)]


class CameraC(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("pose", C.c_float * 12)]


class StatsC(C.Structure):
    _fields_ = [("points_valid", C.c_uint64), ("pairs", C.c_uint64),
                ("pairs_dropped", C.c_uint64), ("coord_out_of_range", C.c_uint64),
                ("blocks_total", C.c_uint32), ("blocks_new", C.c_uint32),
                ("keys_pool_overflow", C.c_uint32), ("keys_table_overflow", C.c_uint32),
                ("table_full_events", C.c_uint32), ("max_probe", C.c_uint32),
                ("lookup_misses", C.c_uint32), ("status_bits", C.c_uint32),
                ("frames", C.c_uint32), ("reserved", C.c_uint32)]


class LayoutC(C.Structure):
    _fields_ = [("counters", C.c_uint64), ("table", C.c_uint64), ("overflow_keys", C.c_uint64),
                ("block_keys", C.c_uint64),
                ("alloc_list", C.c_uint64), ("voxels", C.c_uint64), ("colour", C.c_uint64),
                ("total_bytes", C.c_uint64), ("table_capacity", C.c_uint32),
                ("pool_capacity", C.c_uint32), ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class FuseItemC(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("depth_dev", C.c_void_p), ("rgba_dev", C.c_void_p),
                ("camera", CameraC)]


class BatchConfigC(C.Structure):
    _fields_ = [("tile_width", C.c_uint32), ("pixels_per_thread", C.c_uint32),
                ("acc_blocks", C.c_uint32), ("groups_per_cu", C.c_uint32)]


class ServerParamsC(C.Structure):
    _fields_ = [("max_sessions", C.c_uint32), ("max_batch", C.c_uint32),
                ("max_inflight", C.c_uint32), ("max_queue", C.c_uint32)]


class RequestC(C.Structure):
    _fields_ = [("arrival_ns", C.c_uint64), ("session", C.c_uint32), ("reserved", C.c_uint32),
                ("depth_dev", C.c_void_p), ("camera", CameraC)]


class TsdfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


_lib = None
_hip = None


def _finalise(obj, _shutting_down=sys.is_finalizing) -> None:
    """Release an object's library handle when it is garbage-collected, but
    not during interpreter shutdown: by then the HIP runtime (or a profiler
    hooked into it) may already be torn down, so the process leaves the memory
    to the operating system.  Code that needs the memory back, or a clean exit
    under a profiler, calls close() itself.  (Bound as default arguments, this
    and the finalisers keep working while module globals are being cleared.)"""
    if _shutting_down():
        return
    try:
        obj.close()
    except Exception:
        pass


def hip_runtime() -> C.CDLL:
    """The HIP runtime this process already has loaded (torch's, which
    libtsdf.so binds to as well), never a second copy."""
    global _hip
    if _hip is None:
        lib()
        try:
            _hip = C.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_LAZY)
        except OSError as e:
            raise RuntimeError("the HIP runtime is not loaded in this process") from e
        _hip.hipHostGetDevicePointer.restype = C.c_int
        _hip.hipHostGetDevicePointer.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_uint]
    return _hip


def host_device_pointer(host_ptr: int) -> Optional[int]:
    """Device address of pinned host memory (hipHostGetDevicePointer), or None
    when the runtime gives it none."""
    dp = C.c_void_p()
    if hip_runtime().hipHostGetDevicePointer(C.byref(dp), C.c_void_p(host_ptr), 0) != 0:
        return None
    return dp.value or None


def lib() -> C.CDLL:
    """Load libtsdf.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python paper_2608_08287_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, U32, I = C.c_void_p, C.c_uint32, C.c_int
        L.tsdf_volume_bytes.restype = C.c_size_t
        L.tsdf_volume_bytes.argtypes = [C.POINTER(VolumeParams)]
        L.tsdf_volume_layout.restype = I
        L.tsdf_volume_layout.argtypes = [C.POINTER(VolumeParams), C.POINTER(LayoutC)]
        L.tsdf_create_volume.restype = I
        L.tsdf_create_volume.argtypes = [C.POINTER(VolumeParams), P, C.c_size_t, P, C.POINTER(P)]
        L.tsdf_destroy_volume.restype = I
        L.tsdf_destroy_volume.argtypes = [P]
        L.tsdf_reset_volume.restype = I
        L.tsdf_reset_volume.argtypes = [P, P]
        L.tsdf_fuse_frame.restype = I
        L.tsdf_fuse_frame.argtypes = [P, P, C.POINTER(CameraC), P]
        L.tsdf_fuse_frame_ex.restype = I
        L.tsdf_fuse_frame_ex.argtypes = [P, P, C.POINTER(CameraC), U32, P]
        L.tsdf_fuse_frames.restype = I
        L.tsdf_fuse_frames.argtypes = [P, U32, P, P, U32, P]
        L.tsdf_fuse_frames_rgb.restype = I
        L.tsdf_fuse_frames_rgb.argtypes = [P, U32, P, P, P, U32, P]
        L.tsdf_staging_bytes.restype = C.c_size_t
        L.tsdf_staging_bytes.argtypes = [U32, C.c_uint64]
        L.tsdf_fuse_frames_staged.restype = I
        L.tsdf_fuse_frames_staged.argtypes = [P, U32, P, P, U32, P, C.c_size_t, P]
        L.tsdf_query_status.restype = I
        L.tsdf_query_status.argtypes = [P, P, C.POINTER(StatsC)]
        L.tsdf_probe_histogram.restype = I
        L.tsdf_measure_atomic_rate.restype = I
        L.tsdf_measure_atomic_rate.argtypes = [P, C.c_uint64, U32, U32, U32, U32, P]
        L.tsdf_probe_histogram.argtypes = [P, P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.tsdf_extract_blocks.restype = I
        L.tsdf_extract_blocks.argtypes = [P, P, U32, P, P, P, C.POINTER(U32)]
        L.tsdf_fuse_frame_rgb.restype = I
        L.tsdf_fuse_frame_rgb.argtypes = [P, P, P, C.POINTER(CameraC), U32, P]
        L.tsdf_extract_colour.restype = I
        L.tsdf_extract_colour.argtypes = [P, P, U32, P, C.POINTER(U32)]
        L.tsdf_extract_mesh.restype = I
        L.tsdf_extract_mesh.argtypes = [P, P, U32, P, P, C.POINTER(U32)]
        L.tsdf_insert_blocks.restype = I
        L.tsdf_insert_blocks.argtypes = [P, P, U32, P]
        L.tsdf_status_str.restype = C.c_char_p
        L.tsdf_status_str.argtypes = [I]
        L.tsdf_batch_workspace_bytes.restype = C.c_size_t
        L.tsdf_batch_workspace_bytes.argtypes = [U32]
        L.tsdf_batch_create.restype = I
        L.tsdf_batch_create.argtypes = [U32, P, C.c_size_t, C.POINTER(P)]
        L.tsdf_batch_destroy.restype = I
        L.tsdf_batch_destroy.argtypes = [P]
        L.tsdf_batch_set_config.restype = I
        L.tsdf_batch_set_config.argtypes = [P, C.POINTER(BatchConfigC)]
        L.tsdf_batch_autotune.restype = I
        L.tsdf_batch_autotune.argtypes = [P, U32]
        L.tsdf_batch_get_config.restype = I
        L.tsdf_batch_get_config.argtypes = [P, C.POINTER(BatchConfigC), C.POINTER(U32)]
        L.tsdf_batch_candidates.restype = I
        L.tsdf_batch_candidates.argtypes = [P, U32, C.POINTER(BatchConfigC), C.POINTER(C.c_double),
                                            C.POINTER(U32)]
        L.tsdf_region_create.restype = I
        L.tsdf_region_create.argtypes = [P, C.c_uint64, C.POINTER(P)]
        L.tsdf_region_destroy.restype = I
        L.tsdf_region_destroy.argtypes = [P]
        L.tsdf_region_alloc.restype = I
        L.tsdf_region_alloc.argtypes = [P, C.c_uint64, C.POINTER(P)]
        L.tsdf_region_free.restype = I
        L.tsdf_region_free.argtypes = [P, P]
        L.tsdf_region_usage.restype = I
        L.tsdf_region_usage.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint64), C.POINTER(U32)]
        L.tsdf_server_workspace_bytes.restype = C.c_size_t
        L.tsdf_server_workspace_bytes.argtypes = [C.POINTER(ServerParamsC)]
        L.tsdf_server_create.restype = I
        L.tsdf_server_create.argtypes = [C.POINTER(ServerParamsC), P, C.c_size_t, P, C.c_uint64, P,
                                         C.POINTER(P)]
        L.tsdf_server_destroy.restype = I
        L.tsdf_server_destroy.argtypes = [P]
        L.tsdf_server_open.restype = I
        L.tsdf_server_open.argtypes = [P, C.POINTER(VolumeParams), C.POINTER(U32)]
        L.tsdf_server_close.restype = I
        L.tsdf_server_close.argtypes = [P, U32]
        L.tsdf_server_submit.restype = I
        L.tsdf_server_submit.argtypes = [P, U32, P, C.POINTER(CameraC), C.c_uint64]
        L.tsdf_server_step.restype = I
        L.tsdf_server_step.argtypes = [P, C.POINTER(U32)]
        L.tsdf_server_completions.restype = I
        L.tsdf_server_completions.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_int32), U32,
                                              C.POINTER(U32)]
        L.tsdf_server_session.restype = I
        L.tsdf_server_session.argtypes = [P, U32, C.POINTER(P), C.POINTER(C.c_int32)]
        L.tsdf_server_batch.restype = I
        L.tsdf_server_batch.argtypes = [P, C.POINTER(P)]
        L.tsdf_server_load.restype = I
        L.tsdf_server_load.argtypes = [P, C.POINTER(U32), C.POINTER(U32), C.POINTER(U32),
                                       C.POINTER(U32), C.POINTER(C.c_uint64)]
        L.tsdf_server_replay.restype = I
        L.tsdf_server_replay.argtypes = [P, C.POINTER(RequestC), U32, U32, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
        L.tsdf_batch_fuse.restype = I
        L.tsdf_batch_fuse.argtypes = [P, C.POINTER(FuseItemC), U32, U32, P]
        L.tsdf_batch_fuse_static.restype = I
        L.tsdf_batch_fuse_static.argtypes = [P, C.POINTER(FuseItemC), U32, P]
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().tsdf_status_str(status).decode()


def volume_params(voxel_size: float, trunc: float, table_capacity: int,
                  pool_capacity: int, flags: int = 0) -> VolumeParams:
    return VolumeParams(voxel_size, trunc, table_capacity, pool_capacity, flags)


def volume_bytes(p: VolumeParams) -> int:
    return int(lib().tsdf_volume_bytes(C.byref(p)))


def layout(p: VolumeParams) -> LayoutC:
    out = LayoutC()
    st = lib().tsdf_volume_layout(C.byref(p), C.byref(out))
    if st != OK:
        raise TsdfError(st, "tsdf_volume_layout")
    return out


def pool_voxel_order() -> np.ndarray:
    """(512,) the canonical in-block index (lz * 8 + ly) * 8 + lx of each voxel
    of a pool block, in the pool's order (the layout region ``voxels``: 64
    segments of 8 voxels, each a 4 x 1 x 2 box; segment
    g = ((ly % 4) * 2 + (lz // 2) % 2) * 8 + (lz // 4) * 4 + (ly // 4) * 2 + lx // 4
    holds voxel (lz % 2) * 4 + lx % 4 of its box)."""
    v = np.arange(512)
    word, inw, w = v >> 6, (v >> 3) & 7, v & 7
    ly = (word >> 1) + ((inw >> 1) & 1) * 4
    lz = ((word & 1) + (inw >> 2) * 2) * 2 + (w >> 2)
    lx = (inw & 1) * 4 + (w & 3)
    return (lz * 8 + ly) * 8 + lx


def staging_bytes(pool_capacity: int, records: int) -> int:
    """Bytes of staging memory for tsdf_fuse_frames_staged holding `records`
    records per launch (0 if invalid)."""
    return int(lib().tsdf_staging_bytes(pool_capacity, records))


def staging_buffer(pool_capacity: int, records: int = 32 * 640 * 480 * 9,
                   device: str | torch.device = "cuda") -> torch.Tensor:
    """A device byte tensor to hand to ``Volume.fuse_frames_staged``; the
    default holds every record of 32 frames of 640x480 with a 9-sample band."""
    n = staging_bytes(pool_capacity, records)
    if n == 0:
        raise TsdfError(ERR_INVALID_ARGUMENT, "tsdf_staging_bytes")
    return torch.empty(n, dtype=torch.uint8, device=device)


def measure_atomic_rate(buf: torch.Tensor, waves: int, iters: int, rows_per_instr: int,
                        lanes_per_row: int, stream=None) -> None:
    """Enqueue tsdf_measure_atomic_rate on a float32 device buffer (its bytes a
    multiple of 64); the caller times it."""
    st = lib().tsdf_measure_atomic_rate(C.c_void_p(buf.data_ptr()), buf.numel() * 4, waves, iters,
                                        rows_per_instr, lanes_per_row, _stream_ptr(stream))
    if st != OK:
        raise TsdfError(st, "tsdf_measure_atomic_rate")


def camera_struct(cam) -> CameraC:
    """``cam``: anything with width, height, fx, fy, cx, cy and a 3x4 pose."""
    pose = np.ascontiguousarray(np.asarray(cam.pose, dtype=np.float32).reshape(12))
    return CameraC(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                   float(cam.cy), (C.c_float * 12)(*pose.tolist()))


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class Stats:
    points_valid: int
    pairs: int
    pairs_dropped: int
    coord_out_of_range: int
    blocks_total: int
    blocks_new: int           # since the previous stats() of this volume
    keys_pool_overflow: int
    keys_table_overflow: int  # distinct keys that found the table full
    table_full_events: int
    max_probe: int
    lookup_misses: int
    status_bits: int
    frames: int
    status: int


@dataclass
class Extracted:
    keys: torch.Tensor     # (n,) int64 holding the uint64 packed keys, pool order
    tsdf: torch.Tensor     # (n, 512) float32 mean TSDF (0 where weight 0)
    weight: torch.Tensor   # (n, 512) float32


class _VolumeCalls:
    """Status and extraction calls shared by every volume handle (needs
    ``_h`` and ``device``)."""

    def stats(self, stream=None) -> Stats:
        s = StatsC()
        st = lib().tsdf_query_status(self._h, _stream_ptr(stream), C.byref(s))
        if st == ERR_HIP or st == ERR_INVALID_ARGUMENT:
            raise TsdfError(st, "tsdf_query_status")
        return Stats(s.points_valid, s.pairs, s.pairs_dropped, s.coord_out_of_range, s.blocks_total,
                     s.blocks_new, s.keys_pool_overflow, s.keys_table_overflow,
                     s.table_full_events, s.max_probe, s.lookup_misses, s.status_bits, s.frames,
                     st)

    def probe_histogram(self, stream=None) -> Tuple[np.ndarray, int]:
        """(resolutions by probe distance, bin 0: distance 0, bin b:
        [2^(b-1), 2^b); their summed distance); the volume must have been made
        with VOLUME_PROBE_HISTOGRAM."""
        out = (C.c_uint64 * PROBE_HIST_BINS)()
        total = C.c_uint64()
        st = lib().tsdf_probe_histogram(self._h, _stream_ptr(stream), out, C.byref(total))
        if st != OK:
            raise TsdfError(st, "tsdf_probe_histogram")
        return np.array(out[:], dtype=np.uint64), int(total.value)

    def extract(self, stream=None) -> Extracted:
        n = C.c_uint32(0)
        L = lib()
        st = L.tsdf_extract_blocks(self._h, _stream_ptr(stream), 0, None, None, None, C.byref(n))
        if st not in (OK, ERR_BUFFER_TOO_SMALL):
            raise TsdfError(st, "tsdf_extract_blocks")
        nb = n.value
        dev = self.device
        keys = torch.empty(nb, dtype=torch.int64, device=dev)
        tsdf = torch.empty((nb, BLOCK_VOXELS), dtype=torch.float32, device=dev)
        weight = torch.empty((nb, BLOCK_VOXELS), dtype=torch.float32, device=dev)
        st = L.tsdf_extract_blocks(self._h, _stream_ptr(stream), nb, C.c_void_p(keys.data_ptr()),
                                   C.c_void_p(tsdf.data_ptr()), C.c_void_p(weight.data_ptr()),
                                   C.byref(n))
        if st != OK:
            raise TsdfError(st, "tsdf_extract_blocks")
        return Extracted(keys, tsdf, weight)



@dataclass
class Mesh:
    verts: torch.Tensor  # (T, 3, 3) float32 vertex positions (metres), wound outwards
    ids: torch.Tensor    # (T, 2) int64: block key, cube << 4 | tetrahedron << 1 | triangle


def _extract_mesh(h, stream, device, guess: int) -> Mesh:
    L = lib()
    n = C.c_uint32(0)
    cap = max(guess, 1)
    while True:
        verts = torch.empty((cap, 3, 3), dtype=torch.float32, device=device)
        ids = torch.empty((cap, 2), dtype=torch.int64, device=device)
        st = L.tsdf_extract_mesh(h, _stream_ptr(stream), cap, C.c_void_p(verts.data_ptr()),
                                 C.c_void_p(ids.data_ptr()), C.byref(n))
        if st == OK:
            return Mesh(verts[:n.value], ids[:n.value])
        if st != ERR_BUFFER_TOO_SMALL:
            raise TsdfError(st, "tsdf_extract_mesh")
        cap = n.value


class Volume(_VolumeCalls):
    """One resident TSDF volume in a device arena owned by this object."""

    def __init__(self, voxel_size: float, trunc: float, table_capacity: int, pool_capacity: int,
                 device: str | torch.device = "cuda", stream: Optional[torch.cuda.Stream] = None,
                 flags: int = 0):
        self.params = volume_params(voxel_size, trunc, table_capacity, pool_capacity, flags)
        nbytes = volume_bytes(self.params)
        if nbytes == 0:
            raise TsdfError(ERR_INVALID_ARGUMENT, "volume parameters")
        self.layout = layout(self.params)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.device = self.arena.device
        self._h = C.c_void_p()
        st = lib().tsdf_create_volume(C.byref(self.params), C.c_void_p(self.arena.data_ptr()),
                                      nbytes, _stream_ptr(stream), C.byref(self._h))
        if st != OK:
            raise TsdfError(st, "tsdf_create_volume")

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().tsdf_destroy_volume(self._h)
            self._h = C.c_void_p()

    def __del__(self, _fin=_finalise):
        _fin(self)

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def reset(self, stream=None) -> None:
        st = lib().tsdf_reset_volume(self._h, _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_reset_volume")

    def fuse(self, depth: torch.Tensor, cam, flags: int = FUSE_DEFAULT, stream=None) -> None:
        """Enqueue the fusion of one (H, W) float32 device depth frame."""
        if depth.dtype != torch.float32 or not depth.is_cuda or not depth.is_contiguous():
            raise TypeError("depth must be a contiguous float32 device tensor")
        c = cam if isinstance(cam, CameraC) else camera_struct(cam)
        if depth.numel() != c.width * c.height:
            raise ValueError("depth size does not match the camera")
        st = lib().tsdf_fuse_frame_ex(self._h, C.c_void_p(depth.data_ptr()), C.byref(c), flags,
                                      _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_fuse_frame")

    def fuse_rgb(self, depth: torch.Tensor, rgba: torch.Tensor, cam, flags: int = FUSE_DEFAULT,
                 stream=None) -> None:
        """Colour volumes: fuse a depth frame and its packed colour image
        ((H, W) int32/uint32 holding red | green << 8 | blue << 16)."""
        if depth.dtype != torch.float32 or not depth.is_cuda or not depth.is_contiguous():
            raise TypeError("depth must be a contiguous float32 device tensor")
        if rgba.dtype not in (torch.int32, torch.uint32) or not rgba.is_cuda or \
                not rgba.is_contiguous() or rgba.shape != depth.shape:
            raise TypeError("rgba must be a contiguous 32-bit device tensor shaped like depth")
        c = cam if isinstance(cam, CameraC) else camera_struct(cam)
        if depth.numel() != c.width * c.height:
            raise ValueError("depth size does not match the camera")
        st = lib().tsdf_fuse_frame_rgb(self._h, C.c_void_p(depth.data_ptr()),
                                       C.c_void_p(rgba.data_ptr()), C.byref(c), flags,
                                       _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_fuse_frame_rgb")

    def fuse_frames(self, depths: Sequence[torch.Tensor], cams, flags: int = 0, stream=None) -> None:
        """Enqueue the fusion of several frames with as few launches as possible."""
        n = len(depths)
        structs = [c if isinstance(c, CameraC) else camera_struct(c) for c in cams]
        if len(structs) != n:
            raise ValueError("one camera per frame")
        for d, c in zip(depths, structs):
            if d.dtype != torch.float32 or not d.is_cuda or not d.is_contiguous():
                raise TypeError("depth must be a contiguous float32 device tensor")
            if d.numel() != c.width * c.height:
                raise ValueError("depth size does not match the camera")
        ptrs = (C.c_void_p * max(n, 1))(*[d.data_ptr() for d in depths])
        cam_arr = (CameraC * max(n, 1))(*structs)
        st = lib().tsdf_fuse_frames(self._h, n, ptrs, cam_arr, flags, _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_fuse_frames")

    def fuse_frames_staged(self, depths: Sequence[torch.Tensor], cams, staging: torch.Tensor,
                           flags: int = 0, stream=None) -> None:
        """tsdf_fuse_frames_staged: as fuse_frames, the per-voxel sums gathered
        per block in ``staging`` (a device byte tensor, e.g. staging_buffer)
        and added to the pool once per launch."""
        n = len(depths)
        structs = [c if isinstance(c, CameraC) else camera_struct(c) for c in cams]
        if len(structs) != n:
            raise ValueError("one camera per frame")
        for d, c in zip(depths, structs):
            if d.dtype != torch.float32 or not d.is_cuda or not d.is_contiguous():
                raise TypeError("depth must be a contiguous float32 device tensor")
            if d.numel() != c.width * c.height:
                raise ValueError("depth size does not match the camera")
        if staging.dtype != torch.uint8 or not staging.is_cuda:
            raise TypeError("staging must be a device byte tensor")
        ptrs = (C.c_void_p * max(n, 1))(*[d.data_ptr() for d in depths])
        cam_arr = (CameraC * max(n, 1))(*structs)
        st = lib().tsdf_fuse_frames_staged(self._h, n, ptrs, cam_arr, flags,
                                           C.c_void_p(staging.data_ptr()), staging.numel(),
                                           _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_fuse_frames_staged")

    def fuse_frames_rgb(self, depths: Sequence[torch.Tensor], rgbas: Sequence[torch.Tensor], cams,
                        flags: int = 0, stream=None) -> None:
        """fuse_frames for a colour volume: (H, W) int32 device colour images
        (packed red | green << 8 | blue << 16) beside the depth frames."""
        n = len(depths)
        structs = [c if isinstance(c, CameraC) else camera_struct(c) for c in cams]
        if len(structs) != n or len(rgbas) != n:
            raise ValueError("one camera and one colour image per frame")
        for d, r, c in zip(depths, rgbas, structs):
            for t in (d, r):
                if not t.is_cuda or not t.is_contiguous() or t.numel() != c.width * c.height:
                    raise TypeError("frames must be contiguous device tensors of the camera's size")
            if d.dtype != torch.float32 or r.dtype != torch.int32:
                raise TypeError("depth is float32, colour int32")
        ptrs = (C.c_void_p * max(n, 1))(*[d.data_ptr() for d in depths])
        cols = (C.c_void_p * max(n, 1))(*[r.data_ptr() for r in rgbas])
        cam_arr = (CameraC * max(n, 1))(*structs)
        st = lib().tsdf_fuse_frames_rgb(self._h, n, ptrs, cols, cam_arr, flags, _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_fuse_frames_rgb")

    def insert_blocks(self, coords: torch.Tensor, stream=None) -> None:
        """Allocate blocks for (n, 3) int32 device block coordinates."""
        if coords.dtype != torch.int32 or not coords.is_cuda or not coords.is_contiguous():
            raise TypeError("coords must be a contiguous int32 device tensor")
        n = coords.numel() // 3
        st = lib().tsdf_insert_blocks(self._h, C.c_void_p(coords.data_ptr()), n, _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_insert_blocks")

    def extract_colour(self, stream=None) -> torch.Tensor:
        """Colour volumes: (n, 512, 3) float32 mean colours, blocks in extraction order."""
        n = C.c_uint32(0)
        L = lib()
        st = L.tsdf_extract_colour(self._h, _stream_ptr(stream), 0, None, C.byref(n))
        if st not in (OK, ERR_BUFFER_TOO_SMALL):
            raise TsdfError(st, "tsdf_extract_colour")
        out = torch.empty((n.value, BLOCK_VOXELS, 3), dtype=torch.float32, device=self.device)
        st = L.tsdf_extract_colour(self._h, _stream_ptr(stream), n.value,
                                   C.c_void_p(out.data_ptr()), C.byref(n))
        if st != OK:
            raise TsdfError(st, "tsdf_extract_colour")
        return out

    def extract_mesh(self, stream=None) -> Mesh:
        """Marching-tetrahedra surface (tsdf_extract_mesh)."""
        return _extract_mesh(self._h, stream, self.device, 64 * max(self.stats(stream).blocks_total, 1))

    # Zero-copy views of the carved regions (for invariant checks and consumers).
    def table_view(self) -> torch.Tensor:
        """(C, 2) int64 view of the table: column 0 key bits, column 1 (block | pad<<32)."""
        L = self.layout
        t = self.arena[L.table:L.table + 16 * L.table_capacity]
        return t.view(torch.int64).view(L.table_capacity, 2)

    def pool_view(self) -> torch.Tensor:
        """(P, 64, 2, 8) float32 view of the voxel pool: [block, segment, (sum |
        weight), voxel of the segment]; pool_voxel_order() maps the flattened
        (segment, voxel) index to the canonical in-block index."""
        L = self.layout
        return self.arena[L.voxels:L.voxels + 4096 * L.pool_capacity].view(torch.float32).view(
            L.pool_capacity, 64, 2, 8)

    def tsdf_sum_view(self) -> torch.Tensor:
        """(P, 64, 8) strided view of the TSDF sums, in the pool's voxel order."""
        return self.pool_view()[:, :, 0, :]

    def weight_view(self) -> torch.Tensor:
        """(P, 64, 8) strided view of the weights, in the pool's voxel order."""
        return self.pool_view()[:, :, 1, :]

    def block_keys_view(self) -> torch.Tensor:
        """(P,) int64: the key of the i-th allocated block."""
        L = self.layout
        return self.arena[L.block_keys:L.block_keys + 8 * L.pool_capacity].view(torch.int64)

    def alloc_list_view(self) -> torch.Tensor:
        """(P,) int32: pool index of the i-th allocated block (slot-index volumes)."""
        L = self.layout
        if not (L.flags & VOLUME_SLOT_INDEX):
            raise ValueError("not a slot-index volume")
        return self.arena[L.alloc_list:L.alloc_list + 4 * L.pool_capacity].view(torch.int32)

    def colour_view(self) -> torch.Tensor:
        """(P, 64, 3, 8) float32 colour sums: [block, segment, (r | g | b), voxel
        of the segment], in the pool's voxel order."""
        L = self.layout
        if not (L.flags & VOLUME_COLOUR):
            raise ValueError("not a colour volume")
        return self.arena[L.colour:L.colour + 6144 * L.pool_capacity].view(torch.float32).view(
            L.pool_capacity, 64, 3, 8)


def fuse_frames(vol: Volume, depths: Sequence[torch.Tensor], cams: Sequence, flags: int = FUSE_DEFAULT,
                stream=None) -> None:
    structs = [c if isinstance(c, CameraC) else camera_struct(c) for c in cams]
    for d, c in zip(depths, structs):
        vol.fuse(d, c, flags, stream)


@dataclass(frozen=True)
class BatchConfig:
    tile_width: int         # 16, 32 or 64 pixels
    pixels_per_thread: int  # 1 or 2 (tile height pixels_per_thread * 256 / tile_width)
    acc_blocks: int         # LDS accumulator blocks per pass: 4 or 8 (8 with 2 pixels)
    groups_per_cu: int      # persistent workgroups per CU, 0 = all that fit


class Batch:
    """Multi-volume batch launcher (``tsdf_batch_*``) with its device workspace."""

    def __init__(self, max_items: int, device: str | torch.device = "cuda"):
        nbytes = int(lib().tsdf_batch_workspace_bytes(max_items))
        if nbytes == 0:
            raise TsdfError(ERR_INVALID_ARGUMENT, "tsdf_batch_workspace_bytes")
        self.max_items = max_items
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._h = C.c_void_p()
        st = lib().tsdf_batch_create(max_items, C.c_void_p(self.workspace.data_ptr()), nbytes,
                                     C.byref(self._h))
        if st != OK:
            raise TsdfError(st, "tsdf_batch_create")
        self._items = (FuseItemC * max_items)()

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().tsdf_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self, _fin=_finalise):
        _fin(self)

    def set_config(self, cfg: BatchConfig) -> None:
        c = BatchConfigC(cfg.tile_width, cfg.pixels_per_thread, cfg.acc_blocks, cfg.groups_per_cu)
        st = lib().tsdf_batch_set_config(self._h, C.byref(c))
        if st != OK:
            raise TsdfError(st, "tsdf_batch_set_config")

    def autotune(self, trials: int = 2) -> None:
        st = lib().tsdf_batch_autotune(self._h, trials)
        if st != OK:
            raise TsdfError(st, "tsdf_batch_autotune")

    def config(self) -> tuple[BatchConfig, bool]:
        c, tuned = BatchConfigC(), C.c_uint32(0)
        st = lib().tsdf_batch_get_config(self._h, C.byref(c), C.byref(tuned))
        if st != OK:
            raise TsdfError(st, "tsdf_batch_get_config")
        return (BatchConfig(c.tile_width, c.pixels_per_thread, c.acc_blocks, c.groups_per_cu),
                bool(tuned.value))

    def candidates(self) -> list[tuple[BatchConfig, float]]:
        """The tuner's candidates with the least ns per pixel measured for each."""
        n = C.c_uint32(0)
        L = lib()
        if L.tsdf_batch_candidates(self._h, 0, None, None, C.byref(n)) != OK:
            raise TsdfError(ERR_INVALID_ARGUMENT, "tsdf_batch_candidates")
        cfgs = (BatchConfigC * max(n.value, 1))()
        ns = (C.c_double * max(n.value, 1))()
        L.tsdf_batch_candidates(self._h, n.value, cfgs, ns, C.byref(n))
        return [(BatchConfig(c.tile_width, c.pixels_per_thread, c.acc_blocks, c.groups_per_cu),
                 float(t)) for c, t in zip(cfgs[:n.value], ns[:n.value])]

    def fuse(self, volumes: Sequence[Volume], depths: Sequence[torch.Tensor], cams,
             flags: int = 0, stream=None, rgbas: Optional[Sequence[torch.Tensor]] = None,
             static: bool = False) -> None:
        """Enqueue one frame into each listed volume (a volume may repeat);
        colour volumes take their colour image from ``rgbas``.  ``static``
        calls tsdf_batch_fuse_static (work list in the library's device array,
        no allocation; ``flags`` must be 0)."""
        n = len(volumes)
        if len(depths) != n or len(cams) != n or (rgbas is not None and len(rgbas) != n):
            raise ValueError("one depth frame and one camera per item")
        if n > self.max_items:
            raise ValueError("more items than the batch was made for")
        for i, (v, d, cam) in enumerate(zip(volumes, depths, cams)):
            c = cam if isinstance(cam, CameraC) else camera_struct(cam)
            if d.dtype != torch.float32 or not d.is_cuda or not d.is_contiguous():
                raise TypeError("depth must be a contiguous float32 device tensor")
            if d.numel() != c.width * c.height:
                raise ValueError("depth size does not match the camera")
            it = self._items[i]
            it.volume = v.handle.value
            it.depth_dev = d.data_ptr()
            it.rgba_dev = rgbas[i].data_ptr() if rgbas is not None and rgbas[i] is not None else None
            it.camera = c
        if static:
            if flags:
                raise ValueError("tsdf_batch_fuse_static takes no flags")
            st = lib().tsdf_batch_fuse_static(self._h, self._items, n, _stream_ptr(stream))
            if st != OK:
                raise TsdfError(st, "tsdf_batch_fuse_static")
            return
        st = lib().tsdf_batch_fuse(self._h, self._items, n, flags, _stream_ptr(stream))
        if st != OK:
            raise TsdfError(st, "tsdf_batch_fuse")


class Region:
    """Host bookkeeping of a device region (``tsdf_region_*``); no GPU needed."""

    def __init__(self, base: int, nbytes: int):
        self._h = C.c_void_p()
        st = lib().tsdf_region_create(C.c_void_p(base), nbytes, C.byref(self._h))
        if st != OK:
            raise TsdfError(st, "tsdf_region_create")

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().tsdf_region_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self, _fin=_finalise):
        _fin(self)

    def alloc(self, nbytes: int) -> Optional[int]:
        """Device address of a new range, or None when nothing fits."""
        p = C.c_void_p()
        st = lib().tsdf_region_alloc(self._h, nbytes, C.byref(p))
        if st == ERR_BUDGET:
            return None
        if st != OK:
            raise TsdfError(st, "tsdf_region_alloc")
        return p.value

    def free(self, ptr: int) -> None:
        st = lib().tsdf_region_free(self._h, C.c_void_p(ptr))
        if st != OK:
            raise TsdfError(st, "tsdf_region_free")

    def usage(self) -> tuple[int, int, int, int]:
        """(capacity, used, largest free range, live ranges)."""
        cap, used, big, n = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint32()
        st = lib().tsdf_region_usage(self._h, C.byref(cap), C.byref(used), C.byref(big), C.byref(n))
        if st != OK:
            raise TsdfError(st, "tsdf_region_usage")
        return cap.value, used.value, big.value, n.value


class SessionVolume(_VolumeCalls):
    """A session's volume as held by a server: status and extraction on the
    server's stream (the arena belongs to the server's budget)."""

    def __init__(self, handle: int, params: VolumeParams, stream: torch.cuda.Stream,
                 device: torch.device):
        self._h = C.c_void_p(handle)
        self.params = params
        self.layout = layout(params)
        self.device = device
        self._stream = stream

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def stats(self, stream=None) -> Stats:
        return super().stats(self._stream if stream is None else stream)

    def extract(self, stream=None) -> Extracted:
        out = super().extract(self._stream if stream is None else stream)
        torch.cuda.current_stream(self.device).wait_stream(self._stream)
        return out


class Server:
    """Serving loop (``tsdf_server_*``): sessions carved from one device
    budget, frames batched across sessions, on a stream of its own."""

    def __init__(self, budget_bytes: int, max_sessions: int = 256, max_batch: int = 256,
                 max_inflight: int = 1, max_queue: int = 4096, device="cuda"):
        self.params = ServerParamsC(max_sessions, max_batch, max_inflight, max_queue)
        L = lib()
        ws = int(L.tsdf_server_workspace_bytes(C.byref(self.params)))
        if ws == 0:
            raise TsdfError(ERR_INVALID_ARGUMENT, "tsdf_server_workspace_bytes")
        self.device = torch.device(device)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.region = torch.empty(budget_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        self._h = C.c_void_p()
        st = L.tsdf_server_create(C.byref(self.params), C.c_void_p(self.workspace.data_ptr()), ws,
                                  C.c_void_p(self.region.data_ptr()), budget_bytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        if st != OK:
            raise TsdfError(st, "tsdf_server_create")
        self._vol_params = {}

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().tsdf_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self, _fin=_finalise):
        _fin(self)

    def open(self, voxel_size: float, trunc: float, table_capacity: int,
             pool_capacity: int) -> Optional[int]:
        """A new session id, or None when the budget has no room."""
        p = volume_params(voxel_size, trunc, table_capacity, pool_capacity)
        sid = C.c_uint32()
        st = lib().tsdf_server_open(self._h, C.byref(p), C.byref(sid))
        if st == ERR_BUDGET:
            return None
        if st != OK:
            raise TsdfError(st, "tsdf_server_open")
        self._vol_params[sid.value] = p
        return sid.value

    def close_session(self, sid: int) -> None:
        st = lib().tsdf_server_close(self._h, sid)
        if st != OK:
            raise TsdfError(st, "tsdf_server_close")
        self._vol_params.pop(sid, None)

    def submit(self, sid: int, depth: torch.Tensor, cam, tag: int) -> int:
        """Queue a frame; returns the status (OK, ERR_BUDGET or a failure)."""
        c = cam if isinstance(cam, CameraC) else camera_struct(cam)
        if depth.numel() != c.width * c.height:
            raise ValueError("depth size does not match the camera")
        return lib().tsdf_server_submit(self._h, sid, C.c_void_p(depth.data_ptr()), C.byref(c), tag)

    def step(self) -> int:
        n = C.c_uint32()
        st = lib().tsdf_server_step(self._h, C.byref(n))
        if st != OK:
            raise TsdfError(st, "tsdf_server_step")
        return n.value

    def completions(self, max_n: int = 1024) -> list[tuple[int, int]]:
        tags = (C.c_uint64 * max_n)()
        sts = (C.c_int32 * max_n)()
        n = C.c_uint32()
        st = lib().tsdf_server_completions(self._h, tags, sts, max_n, C.byref(n))
        if st != OK:
            raise TsdfError(st, "tsdf_server_completions")
        return [(tags[i], sts[i]) for i in range(n.value)]

    def session(self, sid: int) -> tuple[SessionVolume, int]:
        h = C.c_void_p()
        fail = C.c_int32()
        st = lib().tsdf_server_session(self._h, sid, C.byref(h), C.byref(fail))
        if st != OK:
            raise TsdfError(st, "tsdf_server_session")
        return SessionVolume(h.value, self._vol_params[sid], self.stream, self.device), fail.value

    def batch_config(self, cfg: BatchConfig) -> None:
        b = C.c_void_p()
        lib().tsdf_server_batch(self._h, C.byref(b))
        c = BatchConfigC(cfg.tile_width, cfg.pixels_per_thread, cfg.acc_blocks, cfg.groups_per_cu)
        st = lib().tsdf_batch_set_config(b, C.byref(c))
        if st != OK:
            raise TsdfError(st, "tsdf_batch_set_config")

    def load(self) -> dict:
        q, f, l, s, u = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint64()
        st = lib().tsdf_server_load(self._h, C.byref(q), C.byref(f), C.byref(l), C.byref(s),
                                    C.byref(u))
        if st != OK:
            raise TsdfError(st, "tsdf_server_load")
        return {"queued": q.value, "inflight_frames": f.value, "inflight_launches": l.value,
                "sessions": s.value, "budget_used": u.value}

    def replay(self, arrivals_ns: Sequence[int], sessions: Sequence[int],
               depths: Sequence[torch.Tensor], cams, mode: int = REPLAY_SERVED):
        """Real-time replay of an arrival trace: (latency_ns array, elapsed_ns)."""
        n = len(arrivals_ns)
        reqs = (RequestC * max(n, 1))()
        for i in range(n):
            c = cams[i] if isinstance(cams[i], CameraC) else camera_struct(cams[i])
            reqs[i].arrival_ns = int(arrivals_ns[i])
            reqs[i].session = int(sessions[i])
            reqs[i].depth_dev = depths[i].data_ptr()
            reqs[i].camera = c
        lat = (C.c_double * max(n, 1))()
        el = C.c_double()
        st = lib().tsdf_server_replay(self._h, reqs, n, mode, lat, C.byref(el))
        if st != OK:
            raise TsdfError(st, "tsdf_server_replay")
        return np.array(lat[:n]), el.value
