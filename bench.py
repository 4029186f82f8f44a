#!/usr/bin/env python
"""Throughput of hash-blocked TSDF fusion on one MI355X.

Workload: a 300-frame, 640x480 orbit through a 4 m room with 20 random boxes and
spheres (voxel 5 mm, truncation 2 cm, table of 2^20 slots, pool of 2^18 blocks).

One step = reset the volume, then fuse all frames of the trajectory into it.
Depth frames are resident in HBM before timing starts.  The headline `value` is
the trajectory fused through tsdf_fuse_frames (32 frames per launch); the plain
path (one tsdf_fuse_frame launch per frame) is timed beside it and supplies the
per-frame latency percentiles.  Also reported: the HBM roofline fraction of the
headline path's fusion kernel on algorithmic bytes, its memory-side atomic
requests against the ceiling measured in the same run, frames fused into empty
volumes (cold), the rate with frames starting in pinned host memory (uploaded
on a second stream, or read by the kernel directly), the device's state, and
the CPU oracle's throughput on a bounded sample.  Other workloads: --workload
multi / serve / stress / lf-sweep, and --variant slot / colour.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "depth points fused/s + p50/p99 frame latency, batched-served vs plain"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2608_08287_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fuse_kernel_room_orbit_640x480_traffic.json")
MULTI_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fuse_multi_kernel_64_volumes_traffic.json")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    """Hash of the device sources (so stored counter readings go stale on any change)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n_pix: int, touched_blocks: int, new_blocks: int, touched_voxels: int,
                      colour_channels: int = 0) -> int:
    """Bytes one fused frame must move at least.

    depth read (4 per pixel) + one 16-byte table entry per touched block + a new
    block's entry write and key (16 + 8) + read and write of 4-byte TSDF and weight
    per touched voxel (16); colour frames add the colour image (4 per pixel) and
    the read and write of each colour sum per touched voxel (8 per channel)."""
    extra = (4 * n_pix + 8 * colour_channels * touched_voxels) if colour_channels else 0
    return 4 * n_pix + 16 * touched_blocks + 24 * new_blocks + 16 * touched_voxels + extra


def atomic_ceiling(T, torch, stream) -> dict:
    """G requests/s that device-scope fp32 atomic adds sustain on a 1 GiB
    buffer: in the fused kernels' flush pattern (about 12 pool rows per wave
    instruction, 5 lanes per row) and in whole 64-byte rows (4 rows of 16
    lanes)."""
    buf = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    out = {}
    for name, rows, lanes in (("flush_pattern", 12, 5), ("full_rows", 4, 16)):
        waves, iters = 16384, 64
        T.measure_atomic_rate(buf, waves, iters, rows, lanes, stream)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(4):
            T.measure_atomic_rate(buf, waves, iters, rows, lanes, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = 4 * waves * iters * rows / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del buf
    return out


def tick_accounting(vols, before_blocks, before_w, n_pix) -> tuple[int, dict]:
    """Algorithmic bytes of one tick over many volumes, from weight snapshots."""
    import torch
    total, acc = 0, {"V": 0, "Bt": 0, "Bn": 0}
    for v, nb0, w0, npx in zip(vols, before_blocks, before_w, n_pix):
        nb = v.stats().blocks_total
        after = v.weight_view()[:nb].reshape(nb, 512)
        changed = after != torch.nn.functional.pad(w0, (0, 0, 0, nb - nb0))
        V = int(changed.sum())
        Bt = int(changed.any(dim=1).sum())
        Bn = nb - nb0
        total += algorithmic_bytes(npx, Bt, Bn, V)
        acc["V"] += V
        acc["Bt"] += Bt
        acc["Bn"] += Bn
    return total, acc


def bench_multi(args) -> int:
    """Many independent volumes, one frame each per tick, through tsdf_batch_fuse.

    One step = one tick: a frame into each of the volumes (64 by default, frame
    sizes 160x120 .. 1280x720, voxels 5..10 mm, truncation 4 voxels, tables
    2^16..2^20).  The autotuner runs first (untimed); then warmup ticks, then the
    timed ticks, replayed as a graph.  The same ticks are then fused into fresh
    volumes one launch per volume (the plain path) and timed the same way, every
    volume of the two runs is checked to hold the same result, and a third,
    untimed run takes the per-tick algorithmic bytes from weight snapshots.
    """
    import torch

    from paper_2608_08287_amd import scenes as S
    from paper_2608_08287_amd import tsdf as T

    torch.cuda.set_device(0)
    w = S.MultiVolumeWorkload(args.volumes)
    nv = len(w)
    n_pix = [s.width * s.height for s in w.specs]
    cache = {}

    def tick(k):
        if k not in cache:
            cache[k] = ([torch.from_numpy(w.depth(i, k, device="cuda")).cuda() for i in range(nv)],
                        [T.camera_struct(w.camera(i, k)) for i in range(nv)])
        return cache[k]

    def make():
        return [T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity) for s in w.specs]

    def points(vols):
        return sum(v.stats().points_valid for v in vols)

    # ---- batched: tune, warm up, time ----------------------------------------
    t0 = time.time()
    A = make()
    batch = T.Batch(nv)
    if args.batch_config:
        tw, ppt, ab, gpc = (int(x) for x in args.batch_config.split(","))
        batch.set_config(T.BatchConfig(tw, ppt, ab, gpc))
    else:
        batch.autotune(args.trials)
    k = 0
    tuned = batch.config()[1]
    cfg = batch.config()[0]
    while not tuned:
        d, c = tick(k)
        batch.fuse(A, d, c)
        torch.cuda.synchronize()
        k += 1
        cfg, tuned = batch.config()
        if k > 200:
            raise RuntimeError("autotuner did not settle")
    n_tune = k
    log(f"[bench] tuned after {n_tune} ticks ({time.time() - t0:.1f}s): {cfg}")
    tuning = [{"tile_width": c.tile_width, "pixels_per_thread": c.pixels_per_thread,
               "acc_blocks": c.acc_blocks, "groups_per_cu": c.groups_per_cu,
               "ns_per_pixel": t if np.isfinite(t) else None} for c, t in batch.candidates()]
    first = n_tune
    ticks = list(range(first, first + args.warmup + args.steps))
    for kk in ticks:
        tick(kk)
    log(f"[bench] rendered {len(ticks)} ticks of {nv} frames ({w.pixels()} pixels each)")
    stream = torch.cuda.current_stream()

    def batched_tick(kk):
        d, c = tick(kk)
        batch.fuse(A, d, c)

    # points fused in the timed ticks: counters before and after
    for kk in ticks[:args.warmup]:
        batched_tick(kk)
    torch.cuda.synchronize()
    pts_before = points(A)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_start = time.perf_counter()
    ev[0].record(stream)
    for j, kk in enumerate(ticks[args.warmup:]):
        batched_tick(kk)
        ev[j + 1].record(stream)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t_start
    tick_ms_b = [ev[j].elapsed_time(ev[j + 1]) for j in range(args.steps)]
    pts_timed = points(A) - pts_before
    value = pts_timed / wall_b
    log(f"[bench] batched: {wall_b / args.steps * 1e3:.3f} ms/tick, {value:.3e} points/s")

    # ---- plain: one launch per volume and frame --------------------------------
    B = make()
    for kk in range(first):
        d, c = tick(kk)
        for i in range(nv):
            B[i].fuse(d[i], c[i])
    for kk in ticks[:args.warmup]:
        d, c = tick(kk)
        for i in range(nv):
            B[i].fuse(d[i], c[i])
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_start = time.perf_counter()
    ev[0].record(stream)
    for j, kk in enumerate(ticks[args.warmup:]):
        d, c = tick(kk)
        for i in range(nv):
            B[i].fuse(d[i], c[i])
        ev[j + 1].record(stream)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t_start
    tick_ms_p = [ev[j].elapsed_time(ev[j + 1]) for j in range(args.steps)]
    plain_value = pts_timed / wall_p
    log(f"[bench] plain: {wall_p / args.steps * 1e3:.3f} ms/tick, {plain_value:.3e} points/s")

    # ---- gate: both runs hold the same volumes --------------------------------
    dropped, dropping = 0, []
    for i in range(nv):
        sa, sb = A[i].stats(), B[i].stats()
        for f in ("points_valid", "pairs", "blocks_total", "status_bits", "frames"):
            if getattr(sa, f) != getattr(sb, f):
                print(f"gate failed: volume {i} {f} {getattr(sa, f)} != {getattr(sb, f)}",
                      file=sys.stderr)
                return 1
        if sa.pairs_dropped or sb.pairs_dropped:
            # a full pool: which keys got its last blocks depends on timing, so
            # check that both runs account for every pair instead
            for v, st in ((A[i], sa), (B[i], sb)):
                wsum = int(v.extract().weight.double().sum().item())
                if wsum + st.pairs_dropped != st.pairs or st.blocks_total != v.layout.pool_capacity:
                    print(f"gate failed: volume {i} loses pairs", file=sys.stderr)
                    return 1
            dropped += sa.pairs_dropped
            dropping.append(i)
            continue
        ea, eb = A[i].extract(), B[i].extract()
        ka, ia = torch.sort(ea.keys)
        kb, ib = torch.sort(eb.keys)
        if not (torch.equal(ka, kb) and torch.equal(ea.weight[ia], eb.weight[ib])) or (
                ka.numel() and (ea.tsdf[ia] - eb.tsdf[ib]).abs().max().item() > 1e-5):
            print(f"gate failed: volume {i} differs between batched and plain", file=sys.stderr)
            return 1
    if dropping:
        # a full pool turns each later new key into a probe of a full table: the
        # run would time that failure path, not fusion
        print(f"gate failed: pools ran out in volumes {dropping} ({dropped} pairs dropped)",
              file=sys.stderr)
        return 1
    log(f"[bench] gate ok: batched == plain on all {nv} volumes, no pairs dropped")
    del A, B
    torch.cuda.empty_cache()

    # ---- algorithmic bytes of the timed ticks (untimed replay) -----------------
    Cv = make()
    tick_bytes, acc = [], {"V": 0, "Bt": 0, "Bn": 0}
    all_ticks = list(range(first)) + ticks
    for kk in all_ticks:
        timed_tick = kk in ticks[args.warmup:]
        if timed_tick:
            nb0 = [v.stats().blocks_total for v in Cv]
            w0 = [v.weight_view()[:n].reshape(n, 512).clone() for v, n in zip(Cv, nb0)]
        d, c = tick(kk)
        for i in range(nv):
            Cv[i].fuse(d[i], c[i])
        if timed_tick:
            b, a = tick_accounting(Cv, nb0, w0, n_pix)
            tick_bytes.append(b)
            for key in acc:
                acc[key] += a[key]
            del w0
    del Cv
    torch.cuda.empty_cache()
    bytes_per_tick = float(np.mean(tick_bytes))
    mean_tick_ms = float(np.mean(tick_ms_b))
    achieved = bytes_per_tick / (mean_tick_ms * 1e-3) / 1e9
    cfg_str = f"{cfg.tile_width},{cfg.pixels_per_thread},{cfg.acc_blocks},{cfg.groups_per_cu}"
    traffic = None
    if os.path.exists(MULTI_TRAFFIC_FILE) and nv == 64:
        tr = json.load(open(MULTI_TRAFFIC_FILE))
        if tr.get("kernel_sha") == kernel_sha() and tr.get("batch_config") == cfg_str:
            traffic = tr.get("bytes_per_launch")

    cpu = None
    if not args.no_cpu_baseline:
        from concurrent.futures import ThreadPoolExecutor

        from oracle import oracle as O
        # the oracle's calls release the interpreter lock, so independent
        # volumes fuse in parallel on threads (at most 16)
        n_thr = max(1, min(16, os.cpu_count() or 1))
        # every volume's tick-0 frame, rendered before any timing, largest first
        # so that the threads finish together
        items = [(w.specs[i], w.depth(i, 0, device="cuda"), w.camera(i, 0)) for i in range(nv)]
        sample = sorted(items, key=lambda it: -it[1].size)

        def fuse_one(item):
            s, d, c = item
            ov = O.OracleVolume(s.voxel_size, s.trunc, s.pool_capacity)
            ov.fuse(d, c)
            return ov.stats()["points_valid"]

        t_c0 = time.perf_counter()
        with ThreadPoolExecutor(n_thr) as ex:
            pts_n = sum(ex.map(fuse_one, sample))
        t_n = time.perf_counter() - t_c0
        # one thread: the volumes in order, for about half of --cpu-seconds
        pts, n1 = 0, 0
        t_c0 = time.perf_counter()
        for it in items:
            pts += fuse_one(it)
            n1 += 1
            if time.perf_counter() - t_c0 > args.cpu_seconds / 2:
                break
        t_1 = time.perf_counter() - t_c0
        cpu = {"value": pts_n / t_n, "unit": "points/s", "cores": n_thr, "kind": "oracle",
               "sample": f"tick 0 of all {len(sample)} volumes, each fused into its own volume "
                         f"({pts_n} points, {t_n:.2f} s), {n_thr} threads on disjoint volumes",
               "single_thread": {"value": pts / t_1, "cores": 1,
                                   "sample": f"the first {n1} of those volumes, {t_1:.1f} s"}}
        log(f"[bench] cpu oracle: {pts / t_1:.3e} points/s on one thread, "
            f"{pts_n / t_n:.3e} on {n_thr}")

    if args.profile_copy_bytes:
        src = torch.empty(args.profile_copy_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_b / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{nv} independent volumes, one frame each per tick (frames 160x120.."
                        f"1280x720, {w.pixels()} pixels per tick), voxels 5..10 mm, truncation "
                        f"4 voxels, tables 2^16..2^20 slots, pools half the table",
            "path": "tsdf_batch_fuse: one persistent launch per tick, replayed as a HIP graph",
            "batch_config": {"tile_width": cfg.tile_width,
                             "pixels_per_thread": cfg.pixels_per_thread,
                             "acc_blocks": cfg.acc_blocks, "groups_per_cu": cfg.groups_per_cu},
            "tuning_ticks": n_tune, "tuning": tuning, "points_per_step": pts_timed / args.steps,
            "parallelism": "single GPU",
        },
        "batched": {"value": value, "ms_per_tick": wall_b / args.steps * 1e3,
                    "gpu_ms_per_tick": tick_ms_b},
        "plain": {"value": plain_value, "ms_per_tick": wall_p / args.steps * 1e3,
                  "gpu_ms_per_tick": tick_ms_p, "launches_per_tick": nv},
        "speedup_vs_plain": value / plain_value,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"fuse_multi_kernel<4, {cfg.pixels_per_thread}, {cfg.acc_blocks}>",
            "algorithmic_bytes_per_launch": bytes_per_tick, "mean_launch_ms": mean_tick_ms,
            "launch_ms_includes": "the work-list copy before the launch",
            "touched_voxels_per_tick": acc["V"] / args.steps,
            "touched_blocks_per_tick": acc["Bt"] / args.steps,
            "new_blocks_per_tick": acc["Bn"] / args.steps,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_stress(args) -> int:
    """Contention stress, sub-case A: a fronto-parallel plane at 0.5 m (640x480,
    voxel 4 mm, truncation 1.6 cm), so that most lanes of a wave insert the
    same keys, fused through a table of 2^16 slots pre-filled with 62,259
    seeded random blocks (load factor 0.95), so that probe chains are long.

    One step = reset, pre-fill (untimed: the timed window opens at the first
    frame's event) and the frames fused; plain (one launch per frame) and
    batched (32 frames per launch) are timed alike.  The gate requires zero
    dropped contributions.  An untimed run on a probe-histogram volume gives
    the distribution of probe distances of the frames' key resolutions.
    """
    import torch

    from paper_2608_08287_amd import scenes as S
    from paper_2608_08287_amd import tsdf as T

    torch.cuda.set_device(0)
    t0 = time.time()
    w = S.plane_stress_workload("A", n_frames=args.frames, device="cuda")
    depth = [torch.from_numpy(d).cuda() for d in w.depth]
    cams = [T.camera_struct(c) for c in w.cameras]
    pre = torch.from_numpy(np.ascontiguousarray(w.prefill_blocks, dtype=np.int32)).cuda()
    n_pix = w.depth[0].size
    log(f"[bench] generated {len(depth)} frames in {time.time() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    L = T.lib()
    sp = T.C.c_void_p(stream.cuda_stream)

    def prepared(flags=0, vol=None):
        v = vol if vol is not None else T.Volume(w.voxel_size, w.trunc, w.table_capacity,
                                                   w.pool_capacity, flags=flags)
        v.reset()
        v.insert_blocks(pre)
        torch.cuda.synchronize()
        return v

    # ---- gate, algorithmic bytes and probe histogram (untimed) ---------------
    hv = prepared(T.VOLUME_PROBE_HISTOGRAM)
    n_pre = hv.stats().blocks_total
    acc_bytes, prev = [], n_pre
    wv = hv.weight_view()
    for k in range(len(depth)):
        before = wv[:prev].reshape(prev, 512).clone()
        hv.fuse(depth[k], w.cameras[k])
        nb = hv.stats().blocks_total
        after = wv[:nb].reshape(nb, 512)
        changed = after != torch.nn.functional.pad(before, (0, 0, 0, nb - prev))
        acc_bytes.append(algorithmic_bytes(n_pix, int(changed.any(dim=1).sum()), nb - prev,
                                           int(changed.sum())))
        prev = nb
    st = hv.stats()
    hist, hist_total = hv.probe_histogram()
    if st.status != T.OK or st.pairs_dropped or st.lookup_misses:
        print(f"correctness gate failed: {T.status_str(st.status)} dropped={st.pairs_dropped}",
              file=sys.stderr)
        return 1
    points_per_step = st.points_valid
    log(f"[bench] gate ok: {st.points_valid} points, {st.pairs} pairs, {st.blocks_total} blocks "
        f"({n_pre} pre-filled), load factor {st.blocks_total / w.table_capacity:.4f}, "
        f"max probe {st.max_probe}")

    vol = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    h = vol.handle
    ptrs = [T.C.c_void_p(d.data_ptr()) for d in depth]
    cam_refs = [T.C.byref(c) for c in cams]
    fpl = max(1, min(args.batch, 32))
    chunks = [(i, min(fpl, len(ptrs) - i)) for i in range(0, len(ptrs), fpl)]
    ptr_arr = (T.C.c_void_p * len(ptrs))(*[d.data_ptr() for d in depth])
    cam_arr = (T.CameraC * len(cams))(*cams)
    bflags = T.FUSE_BATCH(args.per_group)

    def plain(events):
        for k in range(len(ptrs)):
            events[k].record(stream)
            if L.tsdf_fuse_frame(h, ptrs[k], cam_refs[k], sp) != T.OK:
                raise RuntimeError("fuse failed")
        events[len(ptrs)].record(stream)

    def batched(events):
        for j, (i0, n) in enumerate(chunks):
            events[j].record(stream)
            p_ = T.C.cast(T.C.byref(ptr_arr, i0 * T.C.sizeof(T.C.c_void_p)), T.C.c_void_p)
            c_ = T.C.cast(T.C.byref(cam_arr, i0 * T.C.sizeof(T.CameraC)), T.C.c_void_p)
            if L.tsdf_fuse_frames(h, n, p_, c_, bflags, sp) != T.OK:
                raise RuntimeError("batched fusion failed")
        events[len(chunks)].record(stream)

    def timed(run, n_events):
        ms = []
        for step in range(args.warmup + args.steps):
            prepared(vol=vol)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_events + 1)]
            run(ev)
            torch.cuda.synchronize()
            if step >= args.warmup:
                ms.append([ev[k].elapsed_time(ev[k + 1]) for k in range(n_events)])
            s_ = vol.stats()
            if s_.status != T.OK or s_.pairs_dropped or s_.points_valid != points_per_step:
                raise RuntimeError("timed run changed the result")
        return np.array(ms)

    frame_ms = timed(plain, len(ptrs))
    launch_ms = timed(batched, len(chunks))
    step_p = float(frame_ms.sum(axis=1).mean())
    step_b = float(launch_ms.sum(axis=1).mean())
    value = points_per_step / (step_b * 1e-3)
    full = [j for j, (_, n) in enumerate(chunks) if n == fpl]
    mean_launch_ms = float(launch_ms[:, full].mean())
    bytes_per_launch = float(np.mean([sum(acc_bytes[i0:i0 + n]) for (i0, n) in chunks if n == fpl]))
    achieved = bytes_per_launch / (mean_launch_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": f"contention stress A: {len(ptrs)} frames of 640x480, fronto-parallel "
                        "plane at 0.5 m, voxel 4 mm, truncation 1.6 cm, table 2^16 slots "
                        f"pre-filled with {n_pre} random blocks (load factor 0.95), pool 2^16",
            "path": f"batched: tsdf_fuse_frames, {fpl} frames per launch, "
                    f"{args.per_group} frame(s) per workgroup",
            "points_per_step": points_per_step, "parallelism": "single GPU",
        },
        "p50_frame_ms": float(np.percentile(frame_ms, 50)),
        "p99_frame_ms": float(np.percentile(frame_ms, 99)),
        "frame_latency_path": "plain (one launch per frame)",
        "plain": {"value": points_per_step / (step_p * 1e-3), "unit": "points/s",
                  "ms_per_step": step_p, "mean_frame_ms": float(frame_ms.mean())},
        "batched": {"value": value, "unit": "points/s", "mean_launch_ms": mean_launch_ms,
                    "p99_launch_ms": float(np.percentile(launch_ms[:, full], 99))},
        "table": {
            "load_factor": st.blocks_total / w.table_capacity, "blocks_prefilled": n_pre,
            "blocks_total": st.blocks_total, "pairs_dropped": st.pairs_dropped,
            "max_probe": st.max_probe,
            "probe_histogram": {("0" if b == 0 else f"{1 << (b - 1)}-{(1 << b) - 1}"
                                 if b < T.PROBE_HIST_BINS - 1 else f">={1 << (b - 1)}"): int(c)
                                for b, c in enumerate(hist) if c},
            "resolutions": int(hist.sum()),
            "mean_probe_distance": hist_total / max(1, int(hist.sum())),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": f"fuse_kernel<4, {args.per_group}, 32, fused>",
            "algorithmic_bytes_per_launch": bytes_per_launch, "mean_launch_ms": mean_launch_ms,
        },
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args) -> int:
    """Serving: sessions fed by Poisson frame arrivals, through tsdf_server_*.

    256 sessions (frame sizes 160x120 .. 1280x720, voxels 5..10 mm, pools
    2^14..2^18 blocks, tables twice the pool) are admitted against a 200 GB
    budget.  An arrival trace of 3000 frames/s for one second is replayed in
    real time by the library's native driver twice on fresh sessions: served
    (continuous batching across sessions) and plain (one tsdf_fuse_frame per
    frame on arrival); each reports every frame's latency.  Then the same
    frames are replayed with every arrival at time zero, which measures the
    capacity (points/s) of each path.  The session counters of the served and
    plain runs must agree.
    """
    import torch

    from paper_2608_08287_amd import scenes as S
    from paper_2608_08287_amd import tsdf as T

    torch.cuda.set_device(0)
    t0 = time.time()
    w = S.ServingWorkload(args.sessions, rate=args.rate, duration_s=args.duration)
    n = len(w)
    depths = [torch.from_numpy(w.depth(int(s), int(k), device="cuda")).cuda()
              for s, k in zip(w.session_of, w.frame_of)]
    cams = [T.camera_struct(w.camera(int(s), int(k))) for s, k in zip(w.session_of, w.frame_of)]
    points = int(sum(int((d > 0).sum()) for d in depths))
    log(f"[bench] rendered {n} frames for {len(w.specs)} sessions in {time.time() - t0:.1f}s "
        f"({points} points)")
    need = sum(T.volume_bytes(T.volume_params(sp.voxel_size, sp.trunc, sp.table_capacity,
                                              sp.pool_capacity)) for sp in w.specs)
    cfg = T.BatchConfig(*(int(x) for x in args.batch_config.split(","))) if args.batch_config \
        else T.BatchConfig(32, 1, 8, 0)

    def run(mode, budget, frames=None):
        frames = depths if frames is None else frames
        server = T.Server(budget, max_sessions=len(w.specs) + 1, max_batch=args.max_batch,
                          max_inflight=args.max_inflight, max_queue=max(4096, n))
        server.batch_config(cfg)
        ids = []
        for sp in w.specs:
            sid = server.open(sp.voxel_size, sp.trunc, sp.table_capacity, sp.pool_capacity)
            if sid is None:
                raise RuntimeError("a session was not admitted")
            ids.append(sid)
        # warm the launch path (graph instantiation, first dispatches) on a
        # throwaway session
        sp = w.specs[0]
        warm = server.open(sp.voxel_size, sp.trunc, sp.table_capacity, sp.pool_capacity)
        for j in range(3):
            server.submit(warm, depths[0], cams[0], j)
        got = 0
        while got < 3:
            server.step()
            got += len(server.completions())
        server.close_session(warm)
        torch.cuda.synchronize()
        sess = [ids[int(s)] for s in w.session_of]
        lat, elapsed = server.replay(w.arrival_ns, sess, frames, cams, mode)
        _, cap_elapsed = server.replay(np.zeros(n, dtype=np.int64), sess, frames, cams, mode)
        stats = [server.session(i)[0].stats() for i in ids]
        fails = [k for k, i in enumerate(ids)
                 if server.session(i)[1] != T.OK or stats[k].status != T.OK]
        used = server.load()["budget_used"]
        server.close()
        del server
        torch.cuda.empty_cache()
        return lat, elapsed, cap_elapsed, stats, fails, used

    lat_s, el_s, cap_s, st_s, fail_s, used = run(T.REPLAY_SERVED, int(args.budget_gb * 1e9))
    log(f"[bench] served: p50 {np.percentile(lat_s, 50) / 1e3:.1f} us, "
        f"p99 {np.percentile(lat_s, 99) / 1e3:.1f} us; capacity {points / cap_s * 1e9:.3e} points/s")
    lat_p, el_p, cap_p, st_p, fail_p, _ = run(T.REPLAY_PLAIN, int(need * 1.02) + (64 << 20))
    log(f"[bench] plain: p50 {np.percentile(lat_p, 50) / 1e3:.1f} us, "
        f"p99 {np.percentile(lat_p, 99) / 1e3:.1f} us; capacity {points / cap_p * 1e9:.3e} points/s")
    # served again with every frame in pinned host memory, handed over at its
    # device address: the kernels read the depth over PCIe, nothing is uploaded
    zc = None
    total = sum(d.numel() for d in depths)
    host = torch.empty(total, dtype=torch.float32, pin_memory=True)
    hip = T.C.CDLL("libamdhip64.so.7")
    hip.hipHostGetDevicePointer.restype = T.C.c_int
    hip.hipHostGetDevicePointer.argtypes = [T.C.POINTER(T.C.c_void_p), T.C.c_void_p, T.C.c_uint]

    class _Mapped:  # a frame known by its device address
        def __init__(self, addr):
            self.addr = addr

        def data_ptr(self):
            return self.addr

    zframes, off = [], 0
    for d in depths:
        host[off:off + d.numel()].copy_(d.reshape(-1))
        dp = T.C.c_void_p()
        if hip.hipHostGetDevicePointer(T.C.byref(dp), T.C.c_void_p(host[off:].data_ptr()),
                                       0) != 0 or not dp.value:
            zframes = None  # no device address: the run is skipped, nothing launched
            break
        zframes.append(_Mapped(dp.value))
        off += d.numel()
    torch.cuda.synchronize()
    if zframes is not None:
        lat_z, el_z, cap_z, st_z, fail_z, _ = run(T.REPLAY_SERVED, int(args.budget_gb * 1e9),
                                                  frames=zframes)
        log(f"[bench] served, zero copy: p50 {np.percentile(lat_z, 50) / 1e3:.1f} us, "
            f"p99 {np.percentile(lat_z, 99) / 1e3:.1f} us; capacity "
            f"{points / cap_z * 1e9:.3e} points/s")
        for i, (a, b) in enumerate(zip(st_s, st_z)):
            for f in ("points_valid", "pairs", "pairs_dropped", "blocks_total", "frames"):
                if getattr(a, f) != getattr(b, f):
                    print(f"gate failed: zero-copy session {i} {f} {getattr(a, f)} != "
                          f"{getattr(b, f)}", file=sys.stderr)
                    return 1
        fail_s = sorted(set(fail_s) | set(fail_z))
        zc = (lat_z, el_z, cap_z)
    del host
    if fail_s or fail_p:
        bad = sorted(set(fail_s) | set(fail_p))
        print(f"gate failed: sessions whose pool or table ran out (served {fail_s}, plain "
              f"{fail_p}); status bits {[st_s[i].status_bits for i in bad]}", file=sys.stderr)
        return 1
    for i, (a, b) in enumerate(zip(st_s, st_p)):
        for f in ("points_valid", "pairs", "pairs_dropped", "blocks_total", "frames"):
            if getattr(a, f) != getattr(b, f):
                print(f"gate failed: session {i} {f} {getattr(a, f)} != {getattr(b, f)}",
                      file=sys.stderr)
                return 1
    dropped = sum(a.pairs_dropped for a in st_s)
    if fail_s or fail_p or dropped:
        print(f"gate failed: sessions failed {fail_s} / {fail_p}, {dropped} pairs dropped",
              file=sys.stderr)
        return 1
    refused = int(np.sum(lat_s < 0))
    # the capacity replay fuses every frame a second time: its points are `points` again
    value = points / (cap_s * 1e-9)
    plain_value = points / (cap_p * 1e-9)

    def pct(x, q):
        return float(np.percentile(x[x >= 0], q) / 1e6)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": cap_s * 1e-6,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{len(w.specs)} sessions, Poisson arrivals at {args.rate:g} frames/s for "
                        f"{args.duration:g} s ({n} frames, {points} points; frames 160x120.."
                        f"1280x720), voxels 5..10 mm, pools 2^14..2^18 blocks, tables 2x pool, "
                        f"budget {args.budget_gb:g} GB ({used / 1e9:.1f} GB admitted)",
            "path": f"tsdf_server: continuous batching, up to {args.max_batch} frames per launch, "
                    f"{args.max_inflight} launch(es) in flight, graph replay",
            "batch_config": {"tile_width": cfg.tile_width, "pixels_per_thread": cfg.pixels_per_thread,
                             "acc_blocks": cfg.acc_blocks, "groups_per_cu": cfg.groups_per_cu},
            "step": "every frame of the trace arriving at once (capacity)",
            "parallelism": "single GPU",
        },
        "served": {
            "p50_latency_ms": pct(lat_s, 50), "p99_latency_ms": pct(lat_s, 99),
            "max_latency_ms": pct(lat_s, 100), "refused_frames": refused,
            "sustained_points_per_s": points / (el_s * 1e-9),
            "capacity_points_per_s": value,
        },
        "plain": {
            "p50_latency_ms": pct(lat_p, 50), "p99_latency_ms": pct(lat_p, 99),
            "max_latency_ms": pct(lat_p, 100),
            "sustained_points_per_s": points / (el_p * 1e-9),
            "capacity_points_per_s": plain_value,
        },
        "capacity_vs_plain": value / plain_value,
        "served_zero_copy": None if zc is None else {
            "p50_latency_ms": pct(zc[0], 50), "p99_latency_ms": pct(zc[0], 99),
            "max_latency_ms": pct(zc[0], 100),
            "sustained_points_per_s": points / (zc[1] * 1e-9),
            "capacity_points_per_s": points / (zc[2] * 1e-9),
            "path": "served, every frame in pinned host memory at its device address (the "
                    "kernels read the depth over PCIe; no upload)"},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def device_state(torch) -> dict:
    """HBM in use on the device (by every process; the part this process's
    torch allocator holds, cached blocks included) and, where rocm-smi answers
    within a few seconds, its temperatures and clocks."""
    import subprocess
    free, total = torch.cuda.mem_get_info()
    out = {"hbm_total_gib": total / 2**30, "hbm_in_use_gib": (total - free) / 2**30,
           "torch_reserved_gib": torch.cuda.memory_reserved() / 2**30}
    preload = os.environ.get("LD_PRELOAD", "") + os.environ.get("HSA_TOOLS_LIB", "")
    if "rocprof" in preload or any(k.startswith(("ROCPROF", "ROCP_")) for k in os.environ):
        # under a profiler its preloaded library would initialise the GPU in the
        # rocm-smi launcher too, which then replaces itself with the interpreter
        out["smi_skipped"] = "profiler loaded"
        return out
    try:
        r = subprocess.run(["rocm-smi", "--showtemp", "--showclocks", "--json"],
                           capture_output=True, text=True, timeout=20)
        cards = json.loads(r.stdout) if r.returncode == 0 else {}
        card = next((v for k, v in sorted(cards.items()) if k.startswith("card")), None)
        if card:
            out["smi"] = {k: v for k, v in card.items()
                          if "temperature" in k.lower() or "clock" in k.lower()}
    except Exception as e:  # the report is informational; the bench does not depend on it
        out["smi_error"] = type(e).__name__
    return out


def check_idle(torch) -> dict:
    """HBM in use before this process allocates anything.  More than a few GiB
    means another process holds the GPU, and its work may distort the timing:
    said on stderr and in the JSON line."""
    st = device_state(torch)
    st["shared"] = st["hbm_in_use_gib"] > 4.0
    if st["shared"]:
        log(f"[bench] warning: {st['hbm_in_use_gib']:.1f} GiB of HBM in use before the run; "
            "another process may be using the GPU")
    return st


def bench_lf_sweep(args) -> int:
    """The room orbit through tables of C = ceil(N / alpha) slots, where N is
    the number of blocks the trajectory allocates and alpha in {0.25, 0.5,
    0.75, 0.9} its final load factor (C is not a power of two).  One step =
    reset + all frames through tsdf_fuse_frames (32 frames per launch, 2 per
    workgroup), timed as in the trajectory bench.  An untimed run per alpha on
    a probe-histogram volume gives the mean and longest probe distance of the
    frames' key resolutions.  `value` is the throughput at alpha = 0.9."""
    import math
    import torch

    from paper_2608_08287_amd import scenes as S
    from paper_2608_08287_amd import tsdf as T

    torch.cuda.set_device(0)
    idle = check_idle(torch)
    w = S.room_trajectory_workload(n_frames=300, frames=range(args.frames), device="cuda")
    depth = [torch.from_numpy(d).cuda() for d in w.depth]
    cams = [T.camera_struct(c) for c in w.cameras]
    stream = torch.cuda.current_stream()
    L = T.lib()
    sp = T.C.c_void_p(stream.cuda_stream)
    fpl = max(1, min(args.batch, 32))
    chunks = [(i, min(fpl, len(depth) - i)) for i in range(0, len(depth), fpl)]
    ptr_arr = (T.C.c_void_p * len(depth))(*[d.data_ptr() for d in depth])
    cam_arr = (T.CameraC * len(cams))(*cams)
    bflags = T.FUSE_BATCH(args.per_group)

    def run(vol, events=None):
        vol.reset()
        for j, (i0, n) in enumerate(chunks):
            if events is not None:
                events[j].record(stream)
            p_ = T.C.cast(T.C.byref(ptr_arr, i0 * T.C.sizeof(T.C.c_void_p)), T.C.c_void_p)
            c_ = T.C.cast(T.C.byref(cam_arr, i0 * T.C.sizeof(T.CameraC)), T.C.c_void_p)
            if L.tsdf_fuse_frames(vol.handle, n, p_, c_, bflags, sp) != T.OK:
                raise RuntimeError("batched fusion failed")
        if events is not None:
            events[len(chunks)].record(stream)

    ref = T.Volume(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity)
    run(ref)
    st0 = ref.stats()
    if st0.status != T.OK or st0.pairs_dropped:
        print("correctness gate failed at the default table", file=sys.stderr)
        return 1
    n_final, points = st0.blocks_total, st0.points_valid
    del ref
    rows = []
    for alpha in (0.25, 0.5, 0.75, 0.9):
        C = int(math.ceil(n_final / alpha))
        hv = T.Volume(w.voxel_size, w.trunc, C, w.pool_capacity, flags=T.VOLUME_PROBE_HISTOGRAM)
        run(hv)
        hst = hv.stats()
        hist, dist = hv.probe_histogram()
        del hv
        if hst.status != T.OK or hst.pairs_dropped or hst.blocks_total != n_final or \
                hst.points_valid != points:
            print(f"correctness gate failed at alpha {alpha}", file=sys.stderr)
            return 1
        vol = T.Volume(w.voxel_size, w.trunc, C, w.pool_capacity)
        for _ in range(args.warmup):
            run(vol)
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(chunks) + 1)]
            run(vol, ev)
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[-1]))
            s_ = vol.stats()
            if s_.status != T.OK or s_.pairs_dropped or s_.blocks_total != n_final:
                raise RuntimeError("timed run changed the result")
        del vol
        n_res = int(hist.sum())
        rows.append({"alpha": alpha, "table_capacity": C, "load_factor": n_final / C,
                     "points_per_s": points / (float(np.mean(ms)) * 1e-3),
                     "ms_per_step": float(np.mean(ms)), "median_ms_per_step": float(np.median(ms)),
                     "max_probe": hst.max_probe, "resolutions": n_res,
                     "mean_probe_distance": dist / max(n_res, 1)})
        log(f"[bench] alpha {alpha}: C={C} {rows[-1]['points_per_s']:.3e} points/s, "
            f"mean probe {rows[-1]['mean_probe_distance']:.2f}, max {hst.max_probe}")
    last = rows[-1]
    out = {
        "metric": METRIC, "value": last["points_per_s"], "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": last["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"room orbit, {len(depth)} frames of 640x480, voxel 5 mm, truncation "
                        f"2 cm, pool 2^18 blocks, tables of ceil({n_final} / alpha) slots",
            "path": f"batched: tsdf_fuse_frames, {fpl} frames per launch, "
                    f"{args.per_group} frame(s) per workgroup",
            "blocks": n_final, "points_per_step": points, "parallelism": "single GPU",
        },
        "sweep": rows,
        "device": {"at_start": idle, "after": device_state(torch)},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["fused", "two_pass", "fused_xcd_remap"], default="fused",
                    help="kernel structure of the plain per-frame path")
    ap.add_argument("--batch", type=int, default=32,
                    help="frames per tsdf_fuse_frames call on the headline path")
    ap.add_argument("--per-group", type=int, default=2,
                    help="frames summed per workgroup on the headline path (1, 2 or 4)")
    ap.add_argument("--profile-copy-bytes", type=int, default=0,
                    help="after the run, copy this many bytes device-to-device three times "
                         "(a kernel of known traffic for scaling hardware byte counters)")
    ap.add_argument("--variant", choices=["main", "slot", "colour"], default="main",
                    help="trajectory: the volume design (main; slot: block index = table slot, "
                         "pool = table; colour: three colour sums per voxel)")
    ap.add_argument("--workload", choices=["trajectory", "multi", "serve", "stress", "lf-sweep"],
                    default="trajectory",
                    help="trajectory: one volume, the 300-frame orbit (default); multi: many "
                         "volumes, one frame each per tick, through the batch API; serve: "
                         "sessions with Poisson arrivals through the server; stress: the "
                         "fronto-parallel plane through a table at load factor 0.95; "
                         "lf-sweep: the orbit through tables at final load factors 0.25-0.9")
    ap.add_argument("--colour-path", choices=["frames", "batch"], default="frames",
                    help="colour variant: tsdf_fuse_frames_rgb (default) or the batch API")
    ap.add_argument("--cold-volumes", type=int, default=8,
                    help="trajectory: fresh volumes for the cold-frame timing (0: skip it and "
                         "the end-to-end timing)")
    ap.add_argument("--sessions", type=int, default=256, help="serve: sessions")
    ap.add_argument("--rate", type=float, default=3000.0, help="serve: frames/s, all sessions")
    ap.add_argument("--duration", type=float, default=1.0, help="serve: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: session budget")
    ap.add_argument("--max-batch", type=int, default=256, help="serve: frames per launch")
    ap.add_argument("--max-inflight", type=int, default=4, help="serve: launches in flight, one stream each")
    ap.add_argument("--volumes", type=int, default=64, help="multi: volumes per tick")
    ap.add_argument("--trials", type=int, default=2, help="multi: autotuner trials per candidate")
    ap.add_argument("--batch-config", default="",
                    help="multi: fixed tile_width,pixels_per_thread,acc_blocks,groups_per_cu "
                         "instead of tuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the volume is not sharded across GPUs", file=sys.stderr)
        return 2
    if args.workload in ("multi", "serve", "stress", "lf-sweep"):
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 1
        if args.workload == "stress":
            args.frames = min(args.frames, 100)
            return bench_stress(args)
        if args.workload == "lf-sweep":
            return bench_lf_sweep(args)
        return bench_multi(args) if args.workload == "multi" else bench_serve(args)

    import torch

    from paper_2608_08287_amd import scenes as S
    from paper_2608_08287_amd import tsdf as T

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    flags = {"fused": T.FUSE_DEFAULT, "two_pass": T.FUSE_TWO_PASS,
             "fused_xcd_remap": T.FUSE_XCD_REMAP}[args.mode]
    idle = check_idle(torch)

    # ---- inputs, resident in HBM ---------------------------------------------
    t0 = time.time()
    colour = args.variant == "colour"
    slot = args.variant == "slot"
    if colour:
        w, rgba_np = S.room_trajectory_rgbd(n_frames=300, frames=range(args.frames), device="cuda")
        rgba = [torch.from_numpy(c.view(np.int32)).cuda() for c in rgba_np]
    else:
        w = S.room_trajectory_workload(n_frames=300, frames=range(args.frames), device="cuda")
        rgba = None
    depth = [torch.from_numpy(d).cuda() for d in w.depth]
    cams = [T.camera_struct(c) for c in w.cameras]
    n_pix = w.depth[0].size
    log(f"[bench] generated {len(depth)} frames in {time.time() - t0:.1f}s")

    vflags = (T.VOLUME_COLOUR if colour else 0) | (T.VOLUME_SLOT_INDEX if slot else 0)
    table = w.table_capacity
    pool = w.table_capacity if slot else w.pool_capacity  # one block per slot
    vol = T.Volume(w.voxel_size, w.trunc, table, pool, flags=vflags)
    L = T.lib()
    stream = torch.cuda.current_stream()
    sp = T.C.c_void_p(stream.cuda_stream)
    h = vol.handle
    ptrs = [T.C.c_void_p(d.data_ptr()) for d in depth]
    rgba_ptrs = [T.C.c_void_p(c.data_ptr()) for c in rgba] if colour else None
    cam_refs = [T.C.byref(c) for c in cams]

    def fuse_all(events=None):
        """The plain path: one launch per frame."""
        if L.tsdf_reset_volume(h, sp) != T.OK:
            raise RuntimeError("reset failed")
        for k in range(len(ptrs)):
            if events is not None:
                events[k].record(stream)
            st = (L.tsdf_fuse_frame_rgb(h, ptrs[k], rgba_ptrs[k], cam_refs[k], flags, sp) if colour
                  else L.tsdf_fuse_frame_ex(h, ptrs[k], cam_refs[k], flags, sp))
            if st != T.OK:
                raise RuntimeError("fuse failed")
        if events is not None:
            events[len(ptrs)].record(stream)

    fpl = max(1, min(args.batch, 32))  # frames per launch
    chunks = [(i, min(fpl, len(ptrs) - i)) for i in range(0, len(ptrs), fpl)]
    ptr_arr = (T.C.c_void_p * len(ptrs))(*[d.data_ptr() for d in depth])
    cam_arr = (T.CameraC * len(cams))(*cams)
    bflags = T.FUSE_BATCH(args.per_group)

    if colour:
        rgba_arr = (T.C.c_void_p * len(ptrs))(*[c.data_ptr() for c in rgba])
        # the alternative route: the batch API, fpl items of the one volume
        cbatch = T.Batch(fpl)
        cbatch.set_config(T.BatchConfig(32, 1, 4, 0))
        items = (T.FuseItemC * len(ptrs))()
        for k in range(len(ptrs)):
            items[k].volume = h.value
            items[k].depth_dev = depth[k].data_ptr()
            items[k].rgba_dev = rgba[k].data_ptr()
            items[k].camera = cams[k]

    def fuse_batched(events=None):
        """The headline path: `fpl` frames per launch (tsdf_fuse_frames, or
        tsdf_batch_fuse for colour frames)."""
        if L.tsdf_reset_volume(h, sp) != T.OK:
            raise RuntimeError("reset failed")
        for j, (i0, n) in enumerate(chunks):
            if events is not None:
                events[j].record(stream)
            if colour and args.colour_path == "batch":
                it = T.C.cast(T.C.byref(items, i0 * T.C.sizeof(T.FuseItemC)),
                              T.C.POINTER(T.FuseItemC))
                st = L.tsdf_batch_fuse(cbatch._h, it, n, 0, sp)
            elif colour:
                p = T.C.cast(T.C.byref(ptr_arr, i0 * T.C.sizeof(T.C.c_void_p)), T.C.c_void_p)
                r = T.C.cast(T.C.byref(rgba_arr, i0 * T.C.sizeof(T.C.c_void_p)), T.C.c_void_p)
                c = T.C.cast(T.C.byref(cam_arr, i0 * T.C.sizeof(T.CameraC)), T.C.c_void_p)
                st = L.tsdf_fuse_frames_rgb(h, n, p, r, c, bflags, sp)
            else:
                p = T.C.cast(T.C.byref(ptr_arr, i0 * T.C.sizeof(T.C.c_void_p)), T.C.c_void_p)
                c = T.C.cast(T.C.byref(cam_arr, i0 * T.C.sizeof(T.CameraC)), T.C.c_void_p)
                st = L.tsdf_fuse_frames(h, n, p, c, bflags, sp)
            if st != T.OK:
                raise RuntimeError("batched fusion failed")
        if events is not None:
            events[len(chunks)].record(stream)

    # ---- correctness gate and algorithmic-byte accounting (untimed) ----------
    vol.reset()
    acc_bytes, acc = [], {"V": 0, "Bt": 0, "Bn": 0}
    prev_blocks = 0
    wv = vol.weight_view()

    def listed_weights(nb):
        """(nb, 512) weights of the allocated blocks, in allocation order."""
        if slot:
            idx = vol.alloc_list_view()[:nb].long()
            return wv[idx].reshape(nb, 512)
        return wv[:nb].reshape(nb, 512)

    for k in range(len(ptrs)):
        before = listed_weights(prev_blocks).clone()
        if colour:
            vol.fuse_rgb(depth[k], rgba[k], cams[k], flags)
        else:
            vol.fuse(depth[k], cams[k], flags)
        st = vol.stats()
        nb = st.blocks_total
        after = listed_weights(nb)
        changed = after != torch.nn.functional.pad(before, (0, 0, 0, nb - prev_blocks))
        V = int(changed.sum())
        Bt = int(changed.any(dim=1).sum())
        Bn = nb - prev_blocks
        acc_bytes.append(algorithmic_bytes(n_pix, Bt, Bn, V, 3 if colour else 0))
        acc["V"] += V
        acc["Bt"] += Bt
        acc["Bn"] += Bn
        prev_blocks = nb
    st = vol.stats()
    if st.status != T.OK or st.pairs_dropped or st.lookup_misses:
        print(f"correctness gate failed: {T.status_str(st.status)} dropped={st.pairs_dropped}",
              file=sys.stderr)
        return 1
    points_per_step = st.points_valid
    log(f"[bench] gate ok: {st.points_valid} points, {st.pairs} pairs, {st.blocks_total} blocks, "
        f"max probe {st.max_probe}, load factor {st.blocks_total / w.table_capacity:.3f}")

    # ---- warmup, then the timed steps: plain path, then the headline path ----
    def timed(run, n_events):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        events = [[torch.cuda.Event(enable_timing=True) for _ in range(n_events + 1)]
                  for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            run(events[s_])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        ms = np.array([[events[s_][k].elapsed_time(events[s_][k + 1]) for k in range(n_events)]
                       for s_ in range(args.steps)])
        st_ = vol.stats()
        if st_.status != T.OK or st_.pairs_dropped or st_.points_valid != points_per_step:
            raise RuntimeError("timed run changed the result")
        return wall, ms

    wall_p, frame_ms = timed(fuse_all, len(ptrs))
    wall_b, launch_ms = timed(fuse_batched, len(chunks))
    plain_value = points_per_step * args.steps / wall_p
    value = points_per_step * args.steps / wall_b
    wall = wall_b
    # algorithmic bytes per launch of the headline path, against its mean launch time
    launch_bytes = [float(sum(acc_bytes[i0:i0 + n])) for (i0, n) in chunks]
    full = [j for j, (_, n) in enumerate(chunks) if n == fpl]
    mean_launch_ms = float(launch_ms[:, full].mean())
    bytes_per_launch = float(np.mean([launch_bytes[j] for j in full]))
    achieved = bytes_per_launch / (mean_launch_ms * 1e-3) / 1e9
    mean_frame_ms = float(frame_ms.mean())
    traffic = None
    if os.path.exists(TRAFFIC_FILE) and args.variant == "main":
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_sha") == kernel_sha() and tr.get("batch") == fpl and \
                tr.get("per_group") == args.per_group:
            traffic = tr.get("bytes_per_launch")

    # ---- memory-side atomic requests of the headline kernel and their ceiling
    atomics = None
    if args.variant == "main":
        ceiling = atomic_ceiling(T, torch, stream)
        req = None
        if os.path.exists(TRAFFIC_FILE):
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("kernel_sha") == kernel_sha() and tr.get("batch") == fpl and \
                    tr.get("per_group") == args.per_group:
                req = tr.get("atomic_requests_per_dispatch")
        atomics = {
            "unit": "G requests/s", "ceiling": ceiling["flush_pattern"],
            "ceiling_full_rows": ceiling["full_rows"],
            "requests_per_launch": req,
            "achieved": req / (mean_launch_ms * 1e-3) / 1e9 if req else None,
            "frac": (req / (mean_launch_ms * 1e-3) / 1e9) / ceiling["flush_pattern"] if req else None,
            "note": "device-scope fp32 atomic requests (TCC_EA0_ATOMIC) of one launch against the "
                    "rate tsdf_measure_atomic_rate sustains in the flush's pattern",
        }

    # ---- cold frames and the end-to-end rate (main design only) --------------
    cold = e2e = None
    if args.variant == "main" and args.cold_volumes > 0:
        # cold: one frame into a fresh volume; R volumes are reset outside the
        # timed window and fused back to back, each frame between its own events
        R = args.cold_volumes
        cvols = [T.Volume(w.voxel_size, w.trunc, table, pool) for _ in range(R)]
        cold_ms, cold_pts = [], 0
        for rep in range(args.warmup + args.steps):
            for cv in cvols:
                cv.reset()
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * R)]
            ks = [(rep * R + r) % len(ptrs) for r in range(R)]
            for r, cv in enumerate(cvols):
                ev[2 * r].record(stream)
                if L.tsdf_fuse_frame_ex(cv.handle, ptrs[ks[r]], cam_refs[ks[r]], flags, sp) != T.OK:
                    raise RuntimeError("fuse failed")
                ev[2 * r + 1].record(stream)
            torch.cuda.synchronize()
            for r, cv in enumerate(cvols):
                s_ = cv.stats()
                if s_.status != T.OK or s_.pairs_dropped:
                    raise RuntimeError("cold frame failed")
                if rep >= args.warmup:
                    cold_ms.append(ev[2 * r].elapsed_time(ev[2 * r + 1]))
                    cold_pts += s_.points_valid
        del cvols
        cold_ms = np.array(cold_ms)
        cold = {"value": cold_pts / (cold_ms.sum() * 1e-3), "unit": "points/s",
                "volumes": R, "frame_samples": int(cold_ms.size),
                "mean_frame_ms": float(cold_ms.mean()),
                "p50_frame_ms": float(np.percentile(cold_ms, 50)),
                "p99_frame_ms": float(np.percentile(cold_ms, 99)),
                "path": "plain (one launch per frame), each frame into an empty volume"}
        log(f"[bench] cold frames: mean {cold['mean_frame_ms']:.4f} ms")

        # end to end: frames start in pinned host memory; each launch's frames
        # are uploaded on a copy stream into one of two device buffers, so the
        # upload of one launch overlaps the fusion of the one before
        H_, W_ = w.depth[0].shape
        host = torch.empty((len(ptrs), H_, W_), dtype=torch.float32, pin_memory=True)
        for k in range(len(ptrs)):
            host[k].copy_(torch.from_numpy(w.depth[k]))
        bufs = [torch.empty((fpl, H_, W_), dtype=torch.float32, device="cuda") for _ in range(2)]
        buf_ptrs = [(T.C.c_void_p * fpl)(*[b[i].data_ptr() for i in range(fpl)]) for b in bufs]
        copy_stream = torch.cuda.Stream()
        free = [None, None]  # per buffer: the event after the last launch that reads it

        spans = []  # per timed step: (upload start, upload end, launch start, launch end) events

        def fuse_e2e(events=None):
            if L.tsdf_reset_volume(h, sp) != T.OK:
                raise RuntimeError("reset failed")
            if events is not None:
                events[0].record(stream)
                spans.append([])
            for j, (i0, n) in enumerate(chunks):
                b = j % 2
                ev = [torch.cuda.Event(enable_timing=events is not None) for _ in range(4)]
                if free[b] is not None:
                    copy_stream.wait_event(free[b])
                with torch.cuda.stream(copy_stream):
                    ev[0].record(copy_stream)
                    bufs[b][:n].copy_(host[i0:i0 + n], non_blocking=True)
                    ev[1].record(copy_stream)
                stream.wait_event(ev[1])
                ev[2].record(stream)
                c_ = T.C.cast(T.C.byref(cam_arr, i0 * T.C.sizeof(T.CameraC)), T.C.c_void_p)
                if L.tsdf_fuse_frames(h, n, T.C.cast(buf_ptrs[b], T.C.c_void_p), c_, bflags,
                                      sp) != T.OK:
                    raise RuntimeError("batched fusion failed")
                ev[3].record(stream)
                free[b] = ev[3]
                if events is not None:
                    spans[-1].append((ev, n))
            if events is not None:
                events[1].record(stream)

        wall_e, e2e_ms = timed(fuse_e2e, 1)
        full_spans = [(ev, n) for step in spans for (ev, n) in step if n == fpl]
        up_ms = float(np.mean([ev[0].elapsed_time(ev[1]) for ev, _ in full_spans]))
        fuse_ms = float(np.mean([ev[2].elapsed_time(ev[3]) for ev, _ in full_spans]))
        # the upload alone: all frames of a step in one pinned-to-device copy
        dev_all = torch.empty_like(host, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dev_all.copy_(host, non_blocking=True)
        e0.record(stream)
        dev_all.copy_(host, non_blocking=True)
        e1.record(stream)
        torch.cuda.synchronize()
        h2d_gbs = host.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        # zero copy: the same pinned frames read by the fusion kernel itself over
        # PCIe, through the device addresses the runtime maps them at
        hip = T.C.CDLL("libamdhip64.so.7")
        hip.hipHostGetDevicePointer.restype = T.C.c_int
        hip.hipHostGetDevicePointer.argtypes = [T.C.POINTER(T.C.c_void_p), T.C.c_void_p,
                                                T.C.c_uint]
        zptr = (T.C.c_void_p * len(ptrs))()
        mapped = True
        for k in range(len(ptrs)):
            dp = T.C.c_void_p()
            if hip.hipHostGetDevicePointer(T.C.byref(dp), T.C.c_void_p(host[k].data_ptr()),
                                           0) != 0 or not dp.value:
                mapped = False  # no device address: the leg is skipped, nothing launched
                break
            zptr[k] = dp.value

        def fuse_zero_copy(events=None):
            if L.tsdf_reset_volume(h, sp) != T.OK:
                raise RuntimeError("reset failed")
            if events is not None:
                events[0].record(stream)
            for i0, n in chunks:
                p_ = T.C.cast(T.C.byref(zptr, i0 * T.C.sizeof(T.C.c_void_p)), T.C.c_void_p)
                c_ = T.C.cast(T.C.byref(cam_arr, i0 * T.C.sizeof(T.CameraC)), T.C.c_void_p)
                if L.tsdf_fuse_frames(h, n, p_, c_, bflags, sp) != T.OK:
                    raise RuntimeError("batched fusion failed")
            if events is not None:
                events[1].record(stream)

        zero_copy = None
        if mapped:
            wall_z, z_ms = timed(fuse_zero_copy, 1)
            zero_copy = {"value": points_per_step * args.steps / wall_z, "unit": "points/s",
                         "ms_per_step": wall_z / args.steps * 1e3,
                         "median_ms_per_step": float(np.median(z_ms[:, 0])),
                         "path": "frames in pinned host memory read by the fusion kernel over "
                                 "PCIe (tsdf_fuse_frames given their device addresses), no copy"}
            log(f"[bench] zero copy: {zero_copy['value']:.3e} points/s")
        else:
            log("[bench] zero copy skipped: the pinned frames have no device address")
        del dev_all, host, bufs
        e2e = {"value": points_per_step * args.steps / wall_e, "unit": "points/s",
               "ms_per_step": wall_e / args.steps * 1e3,
               "median_ms_per_step": float(np.median(e2e_ms[:, 0])),
               "h2d_gb_per_s": h2d_gbs,
               "mean_upload_ms_overlapped": up_ms, "mean_launch_ms_overlapped": fuse_ms,
               "zero_copy": zero_copy,
               "path": f"frames in pinned host memory, {fpl} uploaded per launch on a second "
                       "stream into one of two device buffers, then tsdf_fuse_frames"}
        log(f"[bench] end to end: {e2e['value']:.3e} points/s, H2D {h2d_gbs:.1f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        n_cpu = 1
        t_c0 = time.perf_counter()
        ov = O.OracleVolume(w.voxel_size, w.trunc, w.pool_capacity)
        pts = 0
        k = 0
        while k < len(w.depth) and (k < n_cpu or time.perf_counter() - t_c0 < args.cpu_seconds):
            if colour:
                ov.fuse_rgb(w.depth[k], rgba_np[k], w.cameras[k])
            else:
                ov.fuse(w.depth[k], w.cameras[k])
            k += 1
        t_c = time.perf_counter() - t_c0
        pts = ov.stats()["points_valid"]
        cpu = {"value": pts / t_c, "unit": "points/s", "cores": 1, "kind": "oracle",
               "sample": f"first {k} of {len(w.depth)} frames fused sequentially into one volume "
                         f"({pts} points, {t_c:.1f} s, one thread)"}
        log(f"[bench] cpu oracle: {pts / t_c:.3e} points/s over {k} frames")

    if args.profile_copy_bytes:
        src = torch.empty(args.profile_copy_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"room orbit, {len(ptrs)} frames of 640x480, voxel 5 mm, truncation 2 cm, "
                        f"table 2^20 slots, pool {'2^20' if slot else '2^18'} blocks"
                        + (", colour images" if colour else ""),
            "path": (f"batched: tsdf_batch_fuse, {fpl} frames of the volume per launch"
                     if colour and args.colour_path == "batch" else
                     f"batched: tsdf_fuse_frames{'_rgb' if colour else ''}, {fpl} frames per "
                     f"launch, {args.per_group} frame(s) per workgroup"),
            "variant": {"main": "main design", "slot": "block index = table slot",
                        "colour": "TSDF, weight and three colour sums"}[args.variant],
            "frames_per_step": len(ptrs), "points_per_step": points_per_step,
            "parallelism": "single GPU",
        },
        "p50_frame_ms": float(np.percentile(frame_ms, 50)),
        "p95_frame_ms": float(np.percentile(frame_ms, 95)),
        "p99_frame_ms": float(np.percentile(frame_ms, 99)),
        "frame_latency_path": "plain (one launch per frame)",
        "plain": {
            "value": plain_value, "unit": "points/s", "mode": args.mode,
            "ms_per_step": wall_p / args.steps * 1e3, "mean_frame_ms": mean_frame_ms,
            "p50_frame_ms": float(np.percentile(frame_ms, 50)),
            "p99_frame_ms": float(np.percentile(frame_ms, 99)), "frame_samples": int(frame_ms.size),
            "median_ms_per_step": float(np.median(frame_ms.sum(axis=1))),
        },
        "batched": {
            "value": value, "unit": "points/s", "frames_per_launch": fpl,
            "frames_per_workgroup": args.per_group,
            "mean_launch_ms": mean_launch_ms,
            "p50_launch_ms": float(np.percentile(launch_ms[:, full], 50)),
            "p99_launch_ms": float(np.percentile(launch_ms[:, full], 99)),
            "ms_per_frame": mean_launch_ms / fpl,
            "median_ms_per_step": float(np.median(launch_ms.sum(axis=1))),
        },
        "cold": cold,
        "end_to_end": e2e,
        "device": {"at_start": idle, "after": device_state(torch)},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": ("fuse_multi_kernel<4, 1, 4, colour>" if colour and args.colour_path == "batch"
                       else f"fuse_kernel<4, {args.per_group}, 32, fused"
                            f"{', colour' if colour else ''}>"),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "mean_launch_ms": mean_launch_ms,
            "touched_voxels_per_frame": acc["V"] / len(ptrs),
            "touched_blocks_per_frame": acc["Bt"] / len(ptrs),
            "new_blocks_per_frame": acc["Bn"] / len(ptrs),
        },
        "atomics": atomics,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
