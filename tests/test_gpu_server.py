"""GPU tests of the serving loop (tsdf_server_*): every session's result is the
one it would have alone, through continuous batching and through the replay
driver; admission against a budget; a failing session is isolated; queue and
close semantics.  Every case prints its name first."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2608_08287_amd import scenes as S
from paper_2608_08287_amd import tsdf as T

from parity import assert_parity, assert_same_volume, log, result_of

pytestmark = pytest.mark.gpu

SMALL = ((160, 120), (320, 240))


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


def budget_for(w, slack=1.05):
    return int(sum(T.volume_bytes(T.volume_params(s.voxel_size, s.trunc, s.table_capacity,
                                                  s.pool_capacity)) for s in w.specs) * slack) + (1 << 20)


def open_all(server, w):
    ids = [server.open(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity) for s in w.specs]
    assert all(i is not None for i in ids)
    return ids


def frames_of(w, device="cuda"):
    return ([torch.from_numpy(w.depth(int(s), int(k))).to(device)
             for s, k in zip(w.session_of, w.frame_of)],
            [w.camera(int(s), int(k)) for s, k in zip(w.session_of, w.frame_of)])


def alone(w, depths, cams):
    vols = [T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity) for s in w.specs]
    for s, d, c in zip(w.session_of, depths, cams):
        vols[int(s)].fuse(d, c)
    return vols


def drain(server, n, timeout_s=60.0):
    done = {}
    t0 = time.monotonic()
    while time.monotonic() - t0 < timeout_s:
        server.step()
        for tag, st in server.completions():
            done[tag] = st
        if len(done) == n:
            return done
    raise AssertionError(f"only {len(done)} of {n} frames completed")


@pytest.mark.parametrize("max_inflight,max_batch", [(1, 64), (2, 8), (4, 3)])
def test_sessions_equal_fusing_alone(max_inflight, max_batch):
    w = S.ServingWorkload(10, rate=2000.0, duration_s=0.03, seed=21, sizes=SMALL,
                          log2_pools=(15, 16))
    depths, cams = frames_of(w)
    server = T.Server(budget_for(w), max_sessions=16, max_batch=max_batch,
                      max_inflight=max_inflight, max_queue=256)
    ids = open_all(server, w)
    for j, (s, d, c) in enumerate(zip(w.session_of, depths, cams)):
        assert server.submit(ids[int(s)], d, c, j) == T.OK
        if j % 5 == 4:
            server.step()
    done = drain(server, len(w))
    assert all(st == T.OK for st in done.values())
    ref = alone(w, depths, cams)
    for i in range(len(w.specs)):
        v, fail = server.session(ids[i])
        assert fail == T.OK
        st = assert_same_volume(v, ref[i])
        assert st.frames == int(np.sum(w.session_of == i))
    log(f"  {len(w)} frames over {len(w.specs)} sessions")


def test_sessions_served_from_pinned_host_frames():
    """Frames in pinned host memory, submitted at their device addresses, are
    read by the kernels over PCIe: every session ends as when its frames are
    fused alone from device memory."""
    w = S.ServingWorkload(8, rate=2000.0, duration_s=0.03, seed=24, sizes=SMALL,
                          log2_pools=(15, 16))
    depths, cams = frames_of(w)

    class Mapped:  # a pinned frame known by its device address
        def __init__(self, t):
            self.host = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
            self.host.copy_(t)
            self.addr = T.host_device_pointer(self.host.data_ptr())
            assert self.addr

        def numel(self):
            return self.host.numel()

        def data_ptr(self):
            return self.addr

    pinned = [Mapped(d) for d in depths]
    server = T.Server(budget_for(w), max_sessions=16, max_batch=8, max_inflight=2, max_queue=256)
    ids = open_all(server, w)
    for j, (s, c) in enumerate(zip(w.session_of, cams)):
        assert server.submit(ids[int(s)], pinned[j], c, j) == T.OK
        if j % 4 == 3:
            server.step()
    done = drain(server, len(w))
    assert all(st == T.OK for st in done.values())
    ref = alone(w, depths, cams)
    for i in range(len(w.specs)):
        v, fail = server.session(ids[i])
        assert fail == T.OK
        assert_same_volume(v, ref[i])
    log(f"  {len(w)} pinned frames over {len(w.specs)} sessions")


def test_served_sessions_match_the_oracle():
    w = S.ServingWorkload(4, rate=1000.0, duration_s=0.012, seed=22, sizes=((160, 120),),
                          log2_pools=(16, 16))
    depths, cams = frames_of(w)
    server = T.Server(budget_for(w), max_sessions=4, max_batch=4)
    ids = open_all(server, w)
    for j, (s, d, c) in enumerate(zip(w.session_of, depths, cams)):
        assert server.submit(ids[int(s)], d, c, j) == T.OK
    drain(server, len(w))
    for i, spec in enumerate(w.specs):
        mine = [j for j in range(len(w)) if w.session_of[j] == i]
        if not mine:
            continue
        o = O.fuse_frames(spec.voxel_size, spec.trunc, spec.pool_capacity,
                          [depths[j].cpu().numpy() for j in mine], [cams[j] for j in mine])
        v, fail = server.session(ids[i])
        g = result_of(v)
        assert fail == T.OK and g.stats.status == T.OK
        assert_parity(g, o)


def test_full_serving_trace_sampled_sessions_match_the_oracle():
    """The serving bench's trace at full size: 256 sessions, Poisson arrivals at
    3000 frames/s for one second, replayed in real time through the served path
    in the bench's configuration (up to 256 frames per launch, 4 launches in
    flight on streams of their own, 32-pixel-wide tiles, one pixel per thread).  Every session counts
    its own frames, and 32 sessions drawn with a fixed seed match the oracle
    (fused on threads; the oracle's calls release the interpreter lock)."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    w = S.ServingWorkload(256, rate=3000.0, duration_s=1.0)
    depths = [torch.from_numpy(w.depth(int(s), int(k), device="cuda")).cuda()
              for s, k in zip(w.session_of, w.frame_of)]
    cams = [w.camera(int(s), int(k)) for s, k in zip(w.session_of, w.frame_of)]
    log(f"  rendered {len(w)} frames")
    server = T.Server(budget_for(w), max_sessions=len(w.specs), max_batch=256, max_inflight=4,
                      max_queue=max(4096, len(w)))
    server.batch_config(T.BatchConfig(32, 1, 8, 0))
    ids = open_all(server, w)
    torch.cuda.synchronize()
    lat, _ = server.replay(w.arrival_ns, [ids[int(s)] for s in w.session_of], depths, cams,
                           T.REPLAY_SERVED)
    assert lat.shape == (len(w),) and np.all(lat > 0)
    for i in range(len(w.specs)):
        v, fail = server.session(ids[i])
        assert fail == T.OK
        st = v.stats()
        assert st.status == T.OK and st.pairs_dropped == 0
        assert st.frames == int(np.sum(w.session_of == i))
    pick = sorted(np.random.default_rng(5).choice(len(w.specs), 32, replace=False).tolist())
    mine = {i: [j for j in range(len(w)) if w.session_of[j] == i] for i in pick}
    host = {i: ([depths[j].cpu().numpy() for j in mine[i]], [cams[j] for j in mine[i]])
            for i in pick}

    def oracle_of(i):
        spec = w.specs[i]
        return O.fuse_frames(spec.voxel_size, spec.trunc, spec.pool_capacity, *host[i])

    n_thr = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(n_thr) as ex:
        for i, o in zip(pick, ex.map(oracle_of, pick)):
            assert_parity(result_of(server.session(ids[i])[0]), o)
    log(f"  {len(w)} frames served; sessions {pick} match the oracle")
    server.close()
    del server, depths
    torch.cuda.empty_cache()


def test_replay_served_and_plain():
    w = S.ServingWorkload(12, rate=3000.0, duration_s=0.05, seed=23, sizes=S.FRAME_SIZES,
                          log2_pools=(16, 17))
    depths, cams = frames_of(w)
    sessions_out = {}
    for mode in (T.REPLAY_SERVED, T.REPLAY_PLAIN):
        server = T.Server(budget_for(w), max_sessions=16, max_batch=64)
        server.batch_config(T.BatchConfig(16, 1, 8, 0))
        ids = open_all(server, w)
        torch.cuda.synchronize()
        lat, elapsed = server.replay(w.arrival_ns, [ids[int(s)] for s in w.session_of], depths,
                                     cams, mode)
        assert lat.shape == (len(w),) and np.all(lat > 0)
        assert elapsed >= w.arrival_ns[-1]
        log(f"  mode {mode}: p50 {np.percentile(lat, 50) / 1e3:.1f} us, "
            f"p99 {np.percentile(lat, 99) / 1e3:.1f} us, elapsed {elapsed / 1e6:.2f} ms")
        sessions_out[mode] = (server, ids)
    (sa, ia), (sb, ib) = sessions_out[T.REPLAY_SERVED], sessions_out[T.REPLAY_PLAIN]
    for i in range(len(w.specs)):
        assert_same_volume(sa.session(ia[i])[0], sb.session(ib[i])[0])


def test_admission_against_the_budget():
    w = S.ServingWorkload(6, rate=100.0, duration_s=0.01, seed=24, sizes=SMALL,
                          log2_pools=(14, 16))
    need = [T.volume_bytes(T.volume_params(s.voxel_size, s.trunc, s.table_capacity,
                                           s.pool_capacity)) for s in w.specs]
    budget = sum(need[:4]) + 1024
    server = T.Server(budget, max_sessions=8)
    ids = [server.open(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity)
           for s in w.specs[:4]]
    assert all(i is not None for i in ids)
    load = server.load()
    assert load["sessions"] == 4 and load["budget_used"] >= sum(need[:4])
    big = max(range(6), key=lambda i: need[i])
    s = w.specs[big]
    assert server.open(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity) is None
    server.close_session(ids[0])
    server.close_session(ids[1])
    assert server.load()["sessions"] == 2
    s0 = w.specs[0]
    again = server.open(s0.voxel_size, s0.trunc, s0.table_capacity, s0.pool_capacity)
    assert again is not None
    # the reused range is reinitialised: a fresh session starts empty
    assert server.session(again)[0].stats().blocks_total == 0
    tiny = T.Server(1 << 20, max_sessions=2)
    assert tiny.open(s0.voxel_size, s0.trunc, s0.table_capacity, s0.pool_capacity) is None


def test_a_failing_session_is_isolated():
    w = S.ServingWorkload(4, rate=1000.0, duration_s=0.03, seed=25, sizes=((320, 240),),
                          log2_pools=(16, 16))
    depths, cams = frames_of(w)
    server = T.Server(budget_for(w) + (1 << 22), max_sessions=8, max_batch=4)
    ids = open_all(server, w)
    s = w.specs[0]
    weak = server.open(s.voxel_size, s.trunc, 1 << 16, 64)  # a pool of 64 blocks
    weak_frames = [(torch.from_numpy(w.depth(0, k)).cuda(), w.camera(0, k)) for k in range(3)]
    assert server.submit(weak, *weak_frames[0], 10_000) == T.OK
    drain(server, 1)
    t0 = time.monotonic()
    while server.session(weak)[1] == T.OK and time.monotonic() - t0 < 30:
        server.step()  # the status copy behind the launch lands after the frame
    assert server.session(weak)[1] == T.ERR_POOL_EXHAUSTED
    assert server.submit(weak, *weak_frames[1], 10_001) == T.ERR_POOL_EXHAUSTED
    for j, (si, d, c) in enumerate(zip(w.session_of, depths, cams)):
        assert server.submit(ids[int(si)], d, c, j) == T.OK
    done = drain(server, len(w))
    assert all(st == T.OK for st in done.values())
    ref = alone(w, depths, cams)
    for i in range(len(w.specs)):
        assert server.session(ids[i])[1] == T.OK
        assert_same_volume(server.session(ids[i])[0], ref[i])
    st = server.session(weak)[0].stats()
    assert st.status == T.ERR_POOL_EXHAUSTED and st.blocks_total == 64 and st.frames == 1


def test_queue_limit_and_close_with_queued_frames():
    w = S.ServingWorkload(2, rate=1000.0, duration_s=0.02, seed=26, sizes=((160, 120),),
                          log2_pools=(14, 14))
    depths, cams = frames_of(w)
    server = T.Server(budget_for(w), max_sessions=2, max_batch=2, max_queue=3)
    ids = open_all(server, w)
    sts = [server.submit(ids[0], depths[0], cams[0], j) for j in range(4)]
    assert sts == [T.OK, T.OK, T.OK, T.ERR_BUDGET]
    server.close_session(ids[0])
    done = dict(server.completions())
    assert done == {0: T.ERR_INVALID_ARGUMENT, 1: T.ERR_INVALID_ARGUMENT,
                    2: T.ERR_INVALID_ARGUMENT}
    assert server.load()["queued"] == 0
    assert server.submit(ids[1], depths[0], cams[0], 7) == T.OK
    assert drain(server, 1) == {7: T.OK}


def test_concurrent_launches_into_one_volume_equal_fusing_alone():
    """One session, frames launched one per launch on four streams at once:
    the launches fuse into the same volume concurrently and it ends as the
    frames fused one by one."""
    w = S.ServingWorkload(1, rate=4000.0, duration_s=0.005, seed=27, sizes=((320, 240),),
                          log2_pools=(18, 18))
    depths, cams = frames_of(w)
    server = T.Server(budget_for(w), max_sessions=2, max_batch=1, max_inflight=4, max_queue=256)
    sid = open_all(server, w)[0]
    for j, (d, c) in enumerate(zip(depths, cams)):
        assert server.submit(sid, d, c, j) == T.OK
    most = 0
    for _ in range(8):
        server.step()
        most = max(most, server.load()["inflight_launches"])
    done = drain(server, len(w))
    assert all(st == T.OK for st in done.values()) and len(w) >= 4, sorted(set(done.values()))
    assert most >= 2, "no two launches were in flight together"
    v, fail = server.session(sid)
    st = assert_same_volume(v, alone(w, depths, cams)[0])
    assert fail == T.OK and st.frames == len(w)
