"""The C ABI without a GPU: the library loads, exports every declared symbol, and
its host-side argument checks reject bad input before anything is enqueued."""
import ctypes as C
import os
import re
import subprocess

import pytest
import numpy as np

from paper_2608_08287_amd import tsdf as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tsdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsdf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = T.lib()
    declared = _declared_functions()
    assert set(declared) == set(T.EXPORTED_SYMBOLS)
    for name in declared:
        assert hasattr(L, name), name


def test_volume_bytes_and_layout():
    p = T.volume_params(0.01, 0.04, 8192, 4096)
    L = T.layout(p)
    assert L.table_capacity == 8192 and L.pool_capacity == 4096
    assert L.counters == 0
    for off in (L.table, L.overflow_keys, L.block_keys, L.voxels, L.total_bytes):
        assert off % 256 == 0
    assert L.overflow_keys - L.table >= 8192 * 16
    assert L.block_keys - L.overflow_keys >= T.OVERFLOW_KEY_SLOTS * 8
    assert L.voxels - L.block_keys >= 4096 * 8
    assert L.total_bytes - L.voxels == 4096 * 1024 * 4
    assert T.volume_bytes(p) == L.total_bytes
    # table 0 -> next power of two >= 2 * pool (the paper's sizing)
    assert T.layout(T.volume_params(0.01, 0.04, 0, 4096)).table_capacity == 8192
    assert T.layout(T.volume_params(0.01, 0.04, 0, 3000)).table_capacity == 8192
    assert T.layout(T.volume_params(0.01, 0.04, 0, 1)).table_capacity == 2
    # non-power-of-two tables are allowed
    assert T.layout(T.volume_params(0.005, 0.02, 123457, 1 << 18)).table_capacity == 123457
    # the configuration with a 2^20-slot table and a 2^18-block pool
    big = T.layout(T.volume_params(0.005, 0.02, 1 << 20, 1 << 18))
    assert big.total_bytes > (1 << 18) * 4096
    # regions of the variants: none without flags
    assert L.alloc_list == L.voxels and L.colour == L.total_bytes and L.flags == 0


def test_variant_layouts():
    P = 4096
    slot = T.layout(T.volume_params(0.01, 0.04, P, P, T.VOLUME_SLOT_INDEX))
    assert slot.table_capacity == P and slot.flags == T.VOLUME_SLOT_INDEX
    assert slot.voxels - slot.alloc_list >= 4 * P and slot.alloc_list % 256 == 0
    # table 0 means "as large as the pool" for slot-index volumes
    assert T.layout(T.volume_params(0.01, 0.04, 0, P, T.VOLUME_SLOT_INDEX)).table_capacity == P
    col = T.layout(T.volume_params(0.01, 0.04, 0, P, T.VOLUME_COLOUR))
    assert col.total_bytes - col.colour == P * 1536 * 4 and col.colour % 256 == 0
    both = T.layout(T.volume_params(0.01, 0.04, 0, P, T.VOLUME_SLOT_INDEX | T.VOLUME_COLOUR))
    assert both.total_bytes == slot.total_bytes + P * 1536 * 4
    # the probe histogram is instrumentation: it changes no region
    hist = T.layout(T.volume_params(0.01, 0.04, 0, P, T.VOLUME_PROBE_HISTOGRAM))
    plain = T.layout(T.volume_params(0.01, 0.04, 0, P))
    assert hist.total_bytes == plain.total_bytes and hist.flags == T.VOLUME_PROBE_HISTOGRAM
    for bad in (T.volume_params(0.01, 0.04, 2 * P, P, T.VOLUME_SLOT_INDEX),
                T.volume_params(0.01, 0.04, 0, P, 0x8)):
        assert T.volume_bytes(bad) == 0


@pytest.mark.parametrize("vs,tr,C_,P", [
    (0.0, 0.04, 8192, 4096), (-0.01, 0.04, 8192, 4096), (float("nan"), 0.04, 8192, 4096),
    (float("inf"), 0.04, 8192, 4096), (0.01, 0.0, 8192, 4096), (0.01, 0.001, 8192, 4096),
    (0.01, 0.2, 8192, 4096), (0.01, float("nan"), 8192, 4096), (0.01, 0.04, 8192, 0),
    # trunc below one voxel (K = round(0.6) = 1 would still be a valid band)
    (0.01, 0.006, 8192, 4096), (0.01, 0.0099, 8192, 4096),
    (0.01, 0.04, 8192, 1 << 22), (0.01, 0.04, 0, 0x7FFFFFFF),
])
def test_invalid_volume_params(vs, tr, C_, P):
    p = T.volume_params(vs, tr, C_, P)
    assert T.volume_bytes(p) == 0
    out = T.LayoutC()
    assert T.lib().tsdf_volume_layout(C.byref(p), C.byref(out)) == T.ERR_INVALID_ARGUMENT
    h = C.c_void_p()
    assert T.lib().tsdf_create_volume(C.byref(p), C.c_void_p(256), 1 << 40, None,
                                      C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert not h.value


def test_create_rejects_bad_arena_before_any_device_work():
    L = T.lib()
    p = T.volume_params(0.01, 0.04, 8192, 4096)
    h = C.c_void_p()
    assert L.tsdf_create_volume(C.byref(p), None, 1 << 30, None, C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_create_volume(C.byref(p), C.c_void_p(4096 + 8), 1 << 30, None,
                                C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_create_volume(C.byref(p), C.c_void_p(4096), 1024, None,
                                C.byref(h)) == T.ERR_BUFFER_TOO_SMALL
    assert L.tsdf_create_volume(C.byref(p), C.c_void_p(4096), 1 << 30, None, None) == \
        T.ERR_INVALID_ARGUMENT


def test_null_handles_are_rejected():
    L = T.lib()
    cam = T.CameraC(4, 4, 1.0, 1.0, 2.0, 2.0, (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0))
    st = T.StatsC()
    n = C.c_uint32()
    assert L.tsdf_destroy_volume(None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_reset_volume(None, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frame(None, C.c_void_p(256), C.byref(cam), None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frame_ex(None, C.c_void_p(256), C.byref(cam), 0, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_query_status(None, None, C.byref(st)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_extract_blocks(None, None, 0, None, None, None, C.byref(n)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_insert_blocks(None, C.c_void_p(256), 1, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frame_rgb(None, C.c_void_p(256), C.c_void_p(256), C.byref(cam), 0,
                                 None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frames(None, 0, None, None, 0, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_fuse_frames_rgb(None, 0, None, None, None, 0, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_extract_colour(None, None, 0, None, C.byref(n)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_extract_mesh(None, None, 0, None, None, C.byref(n)) == T.ERR_INVALID_ARGUMENT


def test_atomic_rate_measurement_rejects_bad_arguments():
    L = T.lib()
    fake = T.C.c_void_p(0x10000)  # never launched on: every call below is refused first
    for args in ((None, 64, 4, 1, 1, 1), (fake, 0, 4, 1, 1, 1), (fake, 63, 4, 1, 1, 1),
                 (fake, 64, 0, 1, 1, 1), (fake, 64, 6, 1, 1, 1), (fake, 64, 4, 0, 1, 1),
                 (fake, 64, 4, 1 << 17, 1, 1), (fake, 64, 4, 1, 0, 1), (fake, 64, 4, 1, 1, 0),
                 (fake, 64, 4, 1, 1, 17), (fake, 64, 4, 1, 5, 13), (fake, 64, 1 << 25, 1, 1, 1)):
        assert L.tsdf_measure_atomic_rate(*args, None) == T.ERR_INVALID_ARGUMENT, args


def test_status_strings():
    for s in range(9):
        assert T.status_str(s) and T.status_str(s) != "unknown status"
    assert T.status_str(99) == "unknown status"


def test_batch_workspace_bytes():
    L = T.lib()
    assert L.tsdf_batch_workspace_bytes(0) == 0
    assert L.tsdf_batch_workspace_bytes(T.BATCH_MAX_ITEMS + 1) == 0
    prev = 0
    for n in (1, 2, 64, 1000, T.BATCH_MAX_ITEMS):
        b = L.tsdf_batch_workspace_bytes(n)
        assert b % 256 == 0 and b > prev
        # per ring slot: group ranges + tile prefix sums + one 192-byte
        # descriptor per item; eight slots
        assert b % 8 == 0 and b // 8 >= 256 + 4 * (n + 1) + 192 * n
        prev = b


def test_batch_rejects_bad_arguments_before_any_device_work():
    L = T.lib()
    h = C.c_void_p()
    need = L.tsdf_batch_workspace_bytes(8)
    assert L.tsdf_batch_create(8, C.c_void_p(4096), need, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_create(0, C.c_void_p(4096), need, C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_create(T.BATCH_MAX_ITEMS + 1, C.c_void_p(4096), 1 << 40,
                               C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_create(8, None, need, C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_create(8, C.c_void_p(4096 + 16), need, C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_create(8, C.c_void_p(4096), need - 1, C.byref(h)) == T.ERR_BUFFER_TOO_SMALL
    assert not h.value
    cfg = T.BatchConfigC(16, 1, 8, 0)
    tuned = C.c_uint32()
    assert L.tsdf_batch_destroy(None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_set_config(None, C.byref(cfg)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_autotune(None, 2) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_get_config(None, C.byref(cfg), C.byref(tuned)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_fuse(None, None, 0, 0, None) == T.ERR_INVALID_ARGUMENT
    n = C.c_uint32()
    assert L.tsdf_batch_candidates(None, 0, None, None, C.byref(n)) == T.ERR_INVALID_ARGUMENT


def _c_offsets(struct: str, fields) -> dict:
    """Byte offsets and size of a C struct of include/tsdf.h, as gcc lays it out."""
    import tempfile
    body = "".join(f'printf("%zu ", offsetof({struct}, {f}));' for f in fields)
    src = ("#include <stdio.h>\n#include <stddef.h>\n#include \"tsdf.h\"\n"
           f"int main(void) {{ {body} printf(\"%zu\\n\", sizeof({struct})); return 0; }}\n")
    with tempfile.TemporaryDirectory() as d:
        c_path, exe = os.path.join(d, "t.c"), os.path.join(d, "t")
        open(c_path, "w").write(src)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c_path, "-o", exe],
                       check=True)
        vals = [int(x) for x in subprocess.run([exe], check=True, capture_output=True,
                                               text=True).stdout.split()]
    return dict(zip(list(fields) + ["sizeof"], vals))


@pytest.mark.parametrize("struct,mirror", [("tsdf_stats", "StatsC"), ("tsdf_layout", "LayoutC"),
                                           ("tsdf_volume_params", "VolumeParams"),
                                           ("tsdf_camera", "CameraC")])
def test_binding_structs_match_the_header(struct, mirror):
    """Every ctypes mirror has the C struct's fields at the C struct's offsets."""
    cls = getattr(T, mirror)
    names = [f[0] for f in cls._fields_]
    c = _c_offsets(struct, names)
    for n in names:
        assert getattr(cls, n).offset == c[n], (struct, n)
    assert C.sizeof(cls) == c["sizeof"]
    if struct == "tsdf_stats":
        assert {"blocks_new", "keys_table_overflow", "keys_pool_overflow"} <= set(names)


def test_staging_bytes_and_refusals_without_a_gpu():
    L = T.lib()
    P = 1 << 11
    r = lambda x: (x + 255) // 256 * 256

    def set_bytes(rec):
        # header, per block 8 bytes and a 128-entry run table, the work items
        # (one per 1024 records of a block: at most rec / 1024 + P + 1), the records
        items = rec // 1024 + P + 1
        return r(r(r(r(256 + 8 * P) + 8 * 128 * P) + 8 * items) + 4 * rec)
    for rec in (1 << 16, 10 ** 7):
        assert T.staging_bytes(P, rec) == 2 * set_bytes(rec)
    for pool, rec in ((0, 1 << 16), (1 << 22, 1 << 16), (P, (1 << 16) - 1), (P, 0), (P, 1 << 32)):
        assert T.staging_bytes(pool, rec) == 0, (pool, rec)
    assert L.tsdf_fuse_frames_staged(None, 0, None, None, 0, C.c_void_p(256), 1 << 30,
                                     None) == T.ERR_INVALID_ARGUMENT


def test_pool_voxel_order_is_the_documented_layout():
    """pool_voxel_order() is the header's layout: a permutation of the 512
    canonical in-block indices, each 8 consecutive pool places a 4 x 1 x 2 box
    at g = ((ly % 4) * 2 + (lz // 2) % 2) * 8 + (lz // 4) * 4 + (ly // 4) * 2 + lx // 4,
    place (lz % 2) * 4 + lx % 4."""
    order = T.pool_voxel_order()
    assert sorted(order.tolist()) == list(range(512))
    for lz in range(8):
        for ly in range(8):
            for lx in range(8):
                g = ((ly % 4) * 2 + (lz // 2) % 2) * 8 + (lz // 4) * 4 + (ly // 4) * 2 + lx // 4
                e = (lz % 2) * 4 + lx % 4
                assert order[g * 8 + e] == (lz * 8 + ly) * 8 + lx
    boxes = order.reshape(64, 8)
    for box in boxes:
        x, y, z = box % 8, (box // 8) % 8, box // 64
        assert np.ptp(x) == 3 and np.ptp(y) == 0 and np.ptp(z) == 1
