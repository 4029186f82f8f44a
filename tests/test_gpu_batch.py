"""GPU parity of multi-volume batches (tsdf_batch_*): every volume of a batch
ends exactly as if its frames had been fused alone (block keys and weights
identical, TSDF means within 1e-5, counters equal), for every work-partition
configuration, through the autotuner's direct launches and through graph
replays whose work lists change from call to call; small volumes are also
checked against the CPU oracle.  Every case prints its name first."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2608_08287_amd import scenes as S
from paper_2608_08287_amd import tsdf as T

from parity import assert_parity, assert_same_volume, log, result_of

pytestmark = pytest.mark.gpu

SMALL = ((160, 120), (320, 240))
CONFIGS = ([T.BatchConfig(tw, 1, ab, gpc) for tw in (16, 32, 64) for ab in (4, 8)
            for gpc in (0, 1)]
           + [T.BatchConfig(tw, 2, 8, gpc) for tw in (16, 32, 64) for gpc in (0, 1)])


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


def make_volumes(w: S.MultiVolumeWorkload):
    return [T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity) for s in w.specs]


def frames(w: S.MultiVolumeWorkload, tick: int, which=None):
    idx = range(len(w)) if which is None else which
    return ([torch.from_numpy(w.depth(i, tick)).cuda() for i in idx],
            [w.camera(i, tick) for i in idx])


def fuse_alone(w, ticks, which_per_tick=None):
    vols = make_volumes(w)
    for k in range(ticks):
        which = range(len(w)) if which_per_tick is None else which_per_tick[k]
        d, c = frames(w, k, which)
        for i, dd, cc in zip(which, d, c):
            vols[i].fuse(dd, cc)
    return vols


def fuse_batched(w, ticks, batch, which_per_tick=None, flags=0):
    vols = make_volumes(w)
    for k in range(ticks):
        which = list(range(len(w))) if which_per_tick is None else which_per_tick[k]
        d, c = frames(w, k, which)
        batch.fuse([vols[i] for i in which], d, c, flags)
    return vols


def test_batch_matches_oracle_on_small_volumes():
    w = S.MultiVolumeWorkload(6, seed=11, sizes=SMALL, log2_tables=(16, 17))
    batch = T.Batch(16)
    vols = fuse_batched(w, 2, batch)
    for i, s in enumerate(w.specs):
        log(f"  volume {i}: {s.width}x{s.height} v={s.voxel_size} C={s.table_capacity}")
        o = O.fuse_frames(s.voxel_size, s.trunc, s.pool_capacity,
                          [w.depth(i, k) for k in range(2)], [w.camera(i, k) for k in range(2)])
        g = result_of(vols[i])
        assert g.stats.status == T.OK
        assert_parity(g, o)


def test_batch_equals_single_volume_path():
    w = S.MultiVolumeWorkload(12, seed=12, sizes=S.FRAME_SIZES, log2_tables=(17, 18))
    batch = T.Batch(12)
    a = fuse_batched(w, 3, batch)
    b = fuse_alone(w, 3)
    for i in range(len(w)):
        st = assert_same_volume(a[i], b[i])
        assert st.pairs > 0 and st.pairs_dropped == 0


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"tw{c.tile_width}_p{c.pixels_per_thread}_"
                                                      f"ab{c.acc_blocks}_g{c.groups_per_cu}")
def test_every_configuration(cfg):
    w = S.MultiVolumeWorkload(4, seed=13, sizes=S.FRAME_SIZES, log2_tables=(17, 17))
    batch = T.Batch(4)
    batch.set_config(cfg)
    assert batch.config() == (cfg, True)
    a = fuse_batched(w, 1, batch)
    b = fuse_alone(w, 1)
    for i in range(len(w)):
        assert_same_volume(a[i], b[i])


@pytest.mark.parametrize("flags", [0, T.BATCH_NO_GRAPH], ids=["graph", "direct"])
def test_replays_with_changing_work_lists(flags):
    """A fixed configuration replays one graph while the number, sizes and
    targets of the items change every call."""
    w = S.MultiVolumeWorkload(7, seed=14, sizes=S.FRAME_SIZES, log2_tables=(17, 17))
    which = [[0, 1, 2, 3, 4, 5, 6], [3], [6, 0, 2], [1, 2, 3, 4], [5, 5, 5, 1], [0, 6]]
    batch = T.Batch(8)
    batch.set_config(T.BatchConfig(16, 2, 8, 0))
    a = fuse_batched(w, len(which), batch, which, flags)
    b = fuse_alone(w, len(which), which)
    for i in range(len(w)):
        assert_same_volume(a[i], b[i])


def test_mixed_band_widths_in_one_call():
    """Volumes whose truncation spans 1..8 voxels: one kernel per band width."""
    w = S.MultiVolumeWorkload(6, seed=15, sizes=SMALL, log2_tables=(17, 17))
    Ks = [1, 2, 3, 5, 6, 8]
    vol_params = [(s.voxel_size, K * s.voxel_size, s.table_capacity, s.pool_capacity)
                  for s, K in zip(w.specs, Ks)]
    batch = T.Batch(8)
    for mode in ("tune", "graph"):
        if mode == "graph":
            batch.set_config(T.BatchConfig(32, 2, 8, 0))
        a = [T.Volume(*p) for p in vol_params]
        b = [T.Volume(*p) for p in vol_params]
        for k in range(2):
            d, c = frames(w, k)
            batch.fuse(a, d, c)
            for v, dd, cc in zip(b, d, c):
                v.fuse(dd, cc)
        for i in range(len(w)):
            assert_same_volume(a[i], b[i])


def test_repeated_volume_in_one_call():
    """Three frames of one trajectory into one volume in a single call."""
    w = S.MultiVolumeWorkload(1, seed=16, sizes=((320, 240),), log2_tables=(17, 17))
    s = w.specs[0]
    d = [torch.from_numpy(w.depth(0, k)).cuda() for k in range(3)]
    c = [w.camera(0, k) for k in range(3)]
    a = T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity)
    b = T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity)
    T.Batch(4).fuse([a, a, a], d, c)
    for dd, cc in zip(d, c):
        b.fuse(dd, cc)
    st = assert_same_volume(a, b)
    assert st.frames == 3
    o = O.fuse_frames(s.voxel_size, s.trunc, s.pool_capacity, [x.cpu().numpy() for x in d], c)
    assert_parity(result_of(a), o)


def test_autotuner_settles_and_stays_correct():
    w = S.MultiVolumeWorkload(3, seed=17, sizes=SMALL, log2_tables=(16, 16))
    batch = T.Batch(4)
    batch.autotune(1)
    cfg0, tuned0 = batch.config()
    assert not tuned0
    vols = make_volumes(w)
    ticks = 0
    tuned = False
    while not tuned:
        assert ticks < 40, "the tuner did not settle"
        d, c = frames(w, ticks)
        batch.fuse(vols, d, c)
        ticks += 1
        torch.cuda.synchronize()
        cfg, tuned = batch.config()
    assert cfg.tile_width in (16, 32, 64) and cfg.acc_blocks in (4, 8)
    assert cfg.pixels_per_thread in (1, 2)
    log(f"  tuned after {ticks} calls: {cfg}")
    cands = batch.candidates()
    assert len(cands) >= 11 and all(np.isfinite(t) and t > 0 for _, t in cands)
    assert cfg == min(cands, key=lambda ct: ct[1])[0]
    ref = fuse_alone(w, ticks)
    for i in range(len(w)):
        assert_same_volume(vols[i], ref[i])


def test_degenerate_items():
    w = S.MultiVolumeWorkload(2, seed=18, sizes=SMALL, log2_tables=(16, 16))
    s = w.specs[0]
    v = T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity)
    batch = T.Batch(4)
    batch.fuse([], [], [])  # nothing to do
    empty = S.Camera(0, 0, 100.0, 100.0, 0.0, 0.0, S.IDENTITY_POSE)
    one = S.Camera(1, 1, 100.0, 100.0, 0.0, 0.0, S.IDENTITY_POSE)
    invalid = S.Camera(64, 48, 50.0, 50.0, 31.5, 23.5, S.IDENTITY_POSE)
    depth_invalid = torch.tensor(np.array([[np.nan, -1.0, 0.0, np.inf] * 16] * 48, np.float32)).cuda()
    batch.fuse([v, v, v], [torch.empty(0, device="cuda"), torch.ones(1, 1, device="cuda"),
                           depth_invalid], [empty, one, invalid])
    st = v.stats()
    assert st.status == T.OK and st.points_valid == 1 and st.frames == 3
    assert st.blocks_total > 0


def test_batch_argument_errors():
    w = S.MultiVolumeWorkload(3, seed=19, sizes=((160, 120),), log2_tables=(16, 16))
    vols = make_volumes(w)
    d, c = frames(w, 0)
    batch = T.Batch(2)
    with pytest.raises(ValueError):
        batch.fuse(vols, d, c)  # 3 items, room for 2
    L = T.lib()
    items = (T.FuseItemC * 3)()
    assert L.tsdf_batch_fuse(batch._h, items, 3, 0, None) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_fuse(batch._h, items, 1, 0, None) == T.ERR_INVALID_ARGUMENT  # null volume
    assert L.tsdf_batch_fuse(batch._h, None, 0, 0x2, None) == T.ERR_INVALID_ARGUMENT  # unknown flag
    for bad in (T.BatchConfigC(8, 1, 8, 0), T.BatchConfigC(16, 1, 5, 0), T.BatchConfigC(16, 1, 8, 65),
                T.BatchConfigC(16, 0, 8, 0), T.BatchConfigC(16, 3, 8, 0), T.BatchConfigC(16, 2, 4, 0), T.BatchConfigC(16, 1, 16, 0)):
        assert L.tsdf_batch_set_config(batch._h, bad) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_autotune(batch._h, 0) == T.ERR_INVALID_ARGUMENT
    assert L.tsdf_batch_autotune(batch._h, 17) == T.ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
    for v in vols:
        assert v.stats().frames == 0


def test_full_size_multi_volume_tick():
    """The 64-volume workload at full size (frames 160x120 .. 1280x720, tables
    2^16..2^20): two batched ticks, first with the autotuner running, then with
    the bench's configuration (32-pixel-wide tiles, 2 pixels per thread)
    replayed as a graph, each against every volume fused alone; then every
    volume of the graph run against the oracle (volumes fused on threads)."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    w = S.MultiVolumeWorkload(64)
    dev = [frames(w, k) for k in range(2)]
    ref = make_volumes(w)
    for d, c in dev:
        for i in range(len(w)):
            ref[i].fuse(d[i], c[i])
    for mode in ("tune", "graph"):
        log(f"  {mode}")
        batch = T.Batch(64)
        if mode == "graph":
            batch.set_config(T.BatchConfig(32, 2, 8, 0))
        vols = make_volumes(w)
        for d, c in dev:
            batch.fuse(vols, d, c)
        dropped = []
        for i in range(len(w)):
            st = assert_same_volume(vols[i], ref[i])
            if st.pairs_dropped:
                dropped.append(i)
        assert dropped == [], f"pools ran out in volumes {dropped}"
        if mode == "tune":
            del vols, batch
            torch.cuda.empty_cache()
    del ref
    host = [([dev[k][0][i].cpu().numpy() for k in range(2)], [dev[k][1][i] for k in range(2)])
            for i in range(len(w))]

    def oracle_of(i):
        s = w.specs[i]
        return O.fuse_frames(s.voxel_size, s.trunc, s.pool_capacity, *host[i])

    n_thr = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(n_thr) as ex:
        for c0 in range(0, len(w), n_thr):
            ids = list(range(c0, min(c0 + n_thr, len(w))))
            for i, o in zip(ids, ex.map(oracle_of, ids)):
                assert_parity(result_of(vols[i]), o)
    log(f"  all {len(w)} volumes match the oracle")
