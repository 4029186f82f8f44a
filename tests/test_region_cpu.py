"""The device-region sub-allocator (tsdf_region_*) is host bookkeeping only, so
it is tested here without a GPU, against a first-fit model with merging."""
import ctypes as C

import numpy as np
import pytest

from paper_2608_08287_amd import tsdf as T

BASE = 1 << 40  # any address: the region's memory is never touched


class FirstFit:
    """Reference model: free ranges as a sorted list, first fit, full merging."""

    def __init__(self, cap):
        self.free = [(0, cap)] if cap else []
        self.live = {}

    def alloc(self, n):
        need = (n + 255) // 256 * 256
        for i, (off, size) in enumerate(self.free):
            if size >= need:
                if size == need:
                    del self.free[i]
                else:
                    self.free[i] = (off + need, size - need)
                self.live[off] = need
                return off
        return None

    def release(self, off):
        size = self.live.pop(off)
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


def test_alignment_of_the_usable_part():
    r = T.Region(BASE + 100, 10_000)
    cap, used, big, n = r.usage()
    assert cap == (10_000 - 156) // 256 * 256 and used == 0 and big == cap and n == 0
    p = r.alloc(1)
    assert p == BASE + 256
    assert r.usage()[1] == 256


@pytest.mark.parametrize("seed", range(6))
def test_random_sequences_match_first_fit(seed):
    rng = np.random.default_rng(seed)
    cap_units = int(rng.integers(50, 400))
    r = T.Region(BASE, cap_units * 256)
    model = FirstFit(cap_units * 256)
    live = []
    for _ in range(600):
        if live and rng.random() < 0.45:
            off = live.pop(int(rng.integers(0, len(live))))
            r.free(BASE + off)
            model.release(off)
        else:
            n = int(rng.integers(1, 40 * 256))
            got = r.alloc(n)
            want = model.alloc(n)
            assert (got is None) == (want is None)
            if got is not None:
                assert got - BASE == want and got % 256 == 0
                live.append(want)
        cap, used, big, nlive = r.usage()
        assert used == sum(model.live.values()) and nlive == len(model.live)
        assert big == max((s for _, s in model.free), default=0)
    for off in live:
        r.free(BASE + off)
    cap, used, big, nlive = r.usage()
    assert used == 0 and big == cap and nlive == 0


def test_bad_frees_and_arguments():
    L = T.lib()
    r = T.Region(BASE, 1 << 20)
    p = r.alloc(1000)
    with pytest.raises(T.TsdfError):
        r.free(p + 256)  # not an allocation
    r.free(p)
    with pytest.raises(T.TsdfError):
        r.free(p)  # twice
    out = C.c_void_p()
    assert L.tsdf_region_alloc(r._h, 0, C.byref(out)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_region_alloc(r._h, 1 << 21, C.byref(out)) == T.ERR_BUDGET
    assert L.tsdf_region_alloc(r._h, (1 << 64) - 1, C.byref(out)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_region_create(None, 1 << 20, C.byref(out)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_region_create(C.c_void_p(BASE), 1 << 20, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_region_free(None, C.c_void_p(BASE)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_region_usage(None, None, None, None, None) == T.ERR_INVALID_ARGUMENT
    empty = T.Region(BASE + 1, 300)  # no whole 256-byte unit after alignment
    assert empty.usage()[0] == 0 and empty.alloc(1) is None
    assert L.tsdf_region_create(C.c_void_p(BASE + 1), 100, C.byref(out)) == T.ERR_INVALID_ARGUMENT


def test_volume_sized_ranges_are_admitted_until_the_budget_is_used():
    """What a server does at admission: carve volume arenas until one fails."""
    p = T.volume_params(0.005, 0.02, 1 << 16, 1 << 15)
    need = T.volume_bytes(p)
    r = T.Region(BASE, 5 * need + need // 2)
    got = [r.alloc(need) for _ in range(6)]
    assert all(g is not None for g in got[:5]) and got[5] is None
    r.free(got[2])
    assert r.alloc(need) == got[2]


def test_server_arguments_are_checked_before_any_device_work():
    L = T.lib()
    ok = T.ServerParamsC(256, 64, 1, 1024)
    assert L.tsdf_server_workspace_bytes(C.byref(ok)) == L.tsdf_batch_workspace_bytes(64)
    for bad in (T.ServerParamsC(0, 64, 1, 1024), T.ServerParamsC(256, 0, 1, 1024),
                T.ServerParamsC(256, 64, 0, 1024), T.ServerParamsC(256, 64, 5, 1024),
                T.ServerParamsC(256, 64, 1, 32), T.ServerParamsC(70000, 64, 1, 1024)):
        assert L.tsdf_server_workspace_bytes(C.byref(bad)) == 0
    h = C.c_void_p()
    ws = L.tsdf_server_workspace_bytes(C.byref(ok))
    assert L.tsdf_server_create(C.byref(ok), C.c_void_p(BASE), ws, C.c_void_p(BASE << 1), 1 << 30,
                                None, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_create(C.byref(ok), None, ws, C.c_void_p(BASE << 1), 1 << 30, None,
                                C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_create(C.byref(ok), C.c_void_p(BASE), ws - 1, C.c_void_p(BASE << 1),
                                1 << 30, None, C.byref(h)) == T.ERR_BUFFER_TOO_SMALL
    assert L.tsdf_server_create(C.byref(ok), C.c_void_p(BASE), ws, None, 1 << 30, None,
                                C.byref(h)) == T.ERR_INVALID_ARGUMENT
    assert not h.value
    n = C.c_uint32()
    sid = C.c_uint32()
    assert L.tsdf_server_destroy(None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_open(None, None, C.byref(sid)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_close(None, 0) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_submit(None, 0, None, None, 0) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_step(None, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_completions(None, None, None, 0, C.byref(n)) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_session(None, 0, None, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_batch(None, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_load(None, None, None, None, None, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_server_replay(None, None, 0, 0, None, None) == T.ERR_INVALID_ARGUMENT
