#!/usr/bin/env python
"""Throughput of hash-blocked TSDF fusion on one MI355X.

The default run measures three workloads and prints one JSON line:

* the headline: a 300-frame, 640x480 orbit through a 4 m room with 20 random
  boxes and spheres (voxel 5 mm, truncation 2 cm, table of 2^20 slots, pool of
  2^18 blocks).  One step = reset the volume, then fuse all frames of the
  trajectory into it.  `value` is the trajectory through tsdf_fuse_frames (32
  frames per launch); the plain path (one tsdf_fuse_frame launch per frame) is
  timed beside it and supplies the per-frame latency percentiles;
* "multi": 64 independent volumes of uneven frame sizes, one frame each per
  tick, through tsdf_batch_fuse (one graph-replayed persistent launch per
  tick) against one launch per volume;
* "served_vs_plain": 256 sessions fed by Poisson arrivals at 3000 frames/s
  through the serving loop (tsdf_server_*) against one launch per frame on
  arrival, with a sweep of the arrival rate.

Depth frames are resident in HBM before any timing starts.  Each leg first
builds and checks its inputs (untimed); then the timed parts of the legs run in
three passes, each pass taking the legs in a rotated order and the two paths of
a leg in alternating order, and every figure is the median over the passes.
Each leg reports the HBM roofline fraction of its dominant kernel on
algorithmic bytes and the CPU oracle's throughput on a bounded sample, with the
host's CPU model and count.  The run refuses to measure (exit status 3) when
another process already holds HBM.  The headline leg also reports the
memory-side atomic requests of its kernel against the ceiling measured in the
same run, frames fused into empty volumes (cold), the rate with frames starting
in pinned host memory, and the device's state.  Other workloads, alone:
--workload trajectory / multi / serve / stress / lf-sweep, and --variant
slot / colour.
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
SHARED_HBM_GIB = 4.0  # HBM in use before the run above which another process holds the GPU


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


class GateFailed(RuntimeError):
    """A leg's correctness check failed: nothing it timed is reported."""


class Leg:
    """A workload whose inputs are built once, timed in passes, then reported.

    run_pass(p) times one pass (p picks the order of the leg's two paths) and
    returns its raw figures; finish(passes) takes the medians, runs what is
    measured once, and returns the leg's JSON object; close() releases it."""

    def __init__(self, name, run_pass, finish, close):
        self.name = name
        self.run_pass = run_pass
        self.finish = finish
        self.close = close


def med(xs) -> float:
    return float(np.median(np.asarray(xs, dtype=np.float64)))


def release(torch) -> None:
    """Finish the device's work and hand cached device memory and pinned host
    blocks back, so the next leg starts from an empty allocator and nothing is
    left for the runtime to free at process exit."""
    import gc
    torch.cuda.synchronize()
    gc.collect()
    torch.cuda.empty_cache()
    torch._C._host_emptyCache()


def host_info() -> dict:
    """The host the CPU baselines ran on: CPU model and count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model}


def cpu_threads() -> int:
    """Threads for the all-core CPU baselines: the usable CPUs, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def multi_leg(args, torch, T, S) -> Leg:
    """Many independent volumes, one frame each per tick, through tsdf_batch_fuse.

    One step = one tick: a frame into each of the volumes (64 by default, frame
    sizes 160x120 .. 1280x720, voxels 5..10 mm, truncation 4 voxels, tables
    2^16..2^20, pools half the table).  Set-up (untimed): the autotuner settles
    on throwaway volumes, the ticks are rendered, and a replay of the ticks one
    launch per volume with weight snapshots gives the timed ticks' algorithmic
    bytes.  A pass: fresh volumes take the tuning and warmup ticks, then the
    timed ticks are fused batched (one graph-replayed launch per tick) and, into
    a second set of fresh volumes, plain (one launch per volume), the two in
    alternating order; every volume of the two runs must hold the same result.
    """
    w = S.MultiVolumeWorkload(args.volumes)
    nv = len(w)
    n_pix = [s.width * s.height for s in w.specs]
    cache = {}
    stream = torch.cuda.current_stream()

    def tick(k):
        if k not in cache:
            cache[k] = ([torch.from_numpy(w.depth(i, k, device="cuda")).cuda() for i in range(nv)],
                        [T.camera_struct(w.camera(i, k)) for i in range(nv)])
        return cache[k]

    def make():
        return [T.Volume(s.voxel_size, s.trunc, s.table_capacity, s.pool_capacity) for s in w.specs]

    def close_all(vols):
        for v in vols:
            v.close()

    def points(vols):
        return sum(v.stats().points_valid for v in vols)

    # ---- autotune on throwaway volumes (untimed) ------------------------------
    t0 = time.time()
    batch = T.Batch(nv)
    if args.batch_config:
        tw, ppt, ab, gpc = (int(x) for x in args.batch_config.split(","))
        batch.set_config(T.BatchConfig(tw, ppt, ab, gpc))
    else:
        batch.autotune(args.trials)
    A0 = make()
    k = 0
    cfg, tuned = batch.config()
    while not tuned:
        d, c = tick(k)
        batch.fuse(A0, d, c)
        torch.cuda.synchronize()
        k += 1
        cfg, tuned = batch.config()
        if k > 200:
            raise RuntimeError("autotuner did not settle")
    n_tune = k
    close_all(A0)
    del A0
    release(torch)
    log(f"[bench] multi: tuned after {n_tune} ticks ({time.time() - t0:.1f}s): {cfg}")
    tuning = [{"tile_width": c.tile_width, "pixels_per_thread": c.pixels_per_thread,
               "acc_blocks": c.acc_blocks, "groups_per_cu": c.groups_per_cu,
               "ns_per_pixel": t if np.isfinite(t) else None} for c, t in batch.candidates()]
    first = n_tune
    ticks = list(range(first, first + args.warmup + args.steps))
    warm, timed_ticks = ticks[:args.warmup], ticks[args.warmup:]
    for kk in ticks:
        tick(kk)
    log(f"[bench] multi: rendered {len(ticks)} ticks of {nv} frames ({w.pixels()} pixels each)")

    # ---- algorithmic bytes of the timed ticks (untimed replay) -----------------
    Cv = make()
    tick_bytes, acc = [], {"V": 0, "Bt": 0, "Bn": 0}
    for kk in list(range(first)) + ticks:
        is_timed = kk in timed_ticks
        if is_timed:
            nb0 = [v.stats().blocks_total for v in Cv]
            w0 = [v.weight_view()[:n].reshape(n, 512).clone() for v, n in zip(Cv, nb0)]
        d, c = tick(kk)
        for i in range(nv):
            Cv[i].fuse(d[i], c[i])
        if is_timed:
            b, a = tick_accounting(Cv, nb0, w0, n_pix)
            tick_bytes.append(b)
            for key in acc:
                acc[key] += a[key]
            del w0
    close_all(Cv)
    del Cv
    release(torch)
    bytes_per_tick = float(np.mean(tick_bytes))

    def run_batched():
        A = make()
        for kk in range(first):
            d, c = tick(kk)
            batch.fuse(A, d, c)
        for kk in warm:
            d, c = tick(kk)
            batch.fuse(A, d, c)
        torch.cuda.synchronize()
        pts0 = points(A)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t_start = time.perf_counter()
        ev[0].record(stream)
        for j, kk in enumerate(timed_ticks):
            d, c = tick(kk)
            batch.fuse(A, d, c)
            ev[j + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return A, wall, [ev[j].elapsed_time(ev[j + 1]) for j in range(args.steps)], points(A) - pts0

    def run_plain():
        B = make()
        for kk in list(range(first)) + warm:
            d, c = tick(kk)
            for i in range(nv):
                B[i].fuse(d[i], c[i])
        torch.cuda.synchronize()
        pts0 = points(B)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t_start = time.perf_counter()
        ev[0].record(stream)
        for j, kk in enumerate(timed_ticks):
            d, c = tick(kk)
            for i in range(nv):
                B[i].fuse(d[i], c[i])
            ev[j + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return B, wall, [ev[j].elapsed_time(ev[j + 1]) for j in range(args.steps)], points(B) - pts0

    def gate(A, B):
        """Both runs hold the same volumes, and no pool ran out."""
        for i in range(nv):
            sa, sb = A[i].stats(), B[i].stats()
            for f in ("points_valid", "pairs", "blocks_total", "status_bits", "frames"):
                if getattr(sa, f) != getattr(sb, f):
                    raise GateFailed(f"multi: volume {i} {f} {getattr(sa, f)} != {getattr(sb, f)}")
            if sa.pairs_dropped or sb.pairs_dropped:
                # a full pool turns each later new key into a probe of a full
                # table: the run would time that failure path, not fusion
                raise GateFailed(f"multi: the pool of volume {i} ran out")
            ea, eb = A[i].extract(), B[i].extract()
            ka, ia = torch.sort(ea.keys)
            kb, ib = torch.sort(eb.keys)
            if not (torch.equal(ka, kb) and torch.equal(ea.weight[ia], eb.weight[ib])) or (
                    ka.numel() and (ea.tsdf[ia] - eb.tsdf[ib]).abs().max().item() > 1e-5):
                raise GateFailed(f"multi: volume {i} differs between batched and plain")

    def run_pass(p):
        if p % 2 == 0:
            A, wall_b, ms_b, pts_b = run_batched()
            B, wall_p, ms_p, pts_p = run_plain()
        else:
            B, wall_p, ms_p, pts_p = run_plain()
            A, wall_b, ms_b, pts_b = run_batched()
        gate(A, B)
        close_all(A)
        close_all(B)
        del A, B
        release(torch)
        log(f"[bench] multi pass {p}: batched {wall_b / args.steps * 1e3:.3f} ms/tick, plain "
            f"{wall_p / args.steps * 1e3:.3f} ms/tick")
        return {"wall_b": wall_b, "tick_ms_b": ms_b, "wall_p": wall_p, "tick_ms_p": ms_p,
                "points": pts_b, "order": "batched, plain" if p % 2 == 0 else "plain, batched"}

    def cpu_baseline():
        from concurrent.futures import ThreadPoolExecutor

        from oracle import oracle as O
        # the oracle's calls release the interpreter lock, so independent
        # volumes fuse in parallel on threads
        n_thr = cpu_threads()
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
        log(f"[bench] multi cpu oracle: {pts / t_1:.3e} points/s on one thread, "
            f"{pts_n / t_n:.3e} on {n_thr}")
        return {"value": pts_n / t_n, "unit": "points/s", "cores": n_thr, "kind": "oracle",
                "sample": f"tick 0 of all {len(sample)} volumes, each fused into its own volume "
                          f"({pts_n} points, {t_n:.2f} s), {n_thr} threads on disjoint volumes",
                "host": host_info(),
                "single_thread": {"value": pts / t_1, "cores": 1,
                                  "sample": f"the first {n1} of those volumes, {t_1:.1f} s"}}

    def finish(passes):
        steps = args.steps
        vals_b = [x["points"] / x["wall_b"] for x in passes]
        vals_p = [x["points"] / x["wall_p"] for x in passes]
        value, plain_value = med(vals_b), med(vals_p)
        mean_tick_ms = med([np.mean(x["tick_ms_b"]) for x in passes])
        achieved = bytes_per_tick / (mean_tick_ms * 1e-3) / 1e9
        cfg_str = f"{cfg.tile_width},{cfg.pixels_per_thread},{cfg.acc_blocks},{cfg.groups_per_cu}"
        traffic = None
        if os.path.exists(MULTI_TRAFFIC_FILE) and nv == 64:
            tr = json.load(open(MULTI_TRAFFIC_FILE))
            if tr.get("kernel_sha") == kernel_sha() and tr.get("batch_config") == cfg_str:
                traffic = tr.get("bytes_per_launch")
        cpu = None if args.no_cpu_baseline else cpu_baseline()
        return {
            "metric": METRIC,
            "value": value,
            "unit": "points/s",
            "n_gpus": 1,
            "steps": steps,
            "warmup": args.warmup,
            "ms_per_step": med([x["wall_b"] for x in passes]) / steps * 1e3,
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
                "tuning_ticks": n_tune, "tuning": tuning,
                "points_per_step": passes[0]["points"] / steps,
                "parallelism": "single GPU",
            },
            "batched": {"value": value, "ms_per_tick": med([x["wall_b"] for x in passes]) / steps * 1e3,
                        "gpu_ms_per_tick": [x["tick_ms_b"] for x in passes]},
            "plain": {"value": plain_value,
                      "ms_per_tick": med([x["wall_p"] for x in passes]) / steps * 1e3,
                      "gpu_ms_per_tick": [x["tick_ms_p"] for x in passes], "launches_per_tick": nv},
            "speedup_vs_plain": value / plain_value,
            "passes": [{"batched": vb, "plain": vp, "order": x["order"]}
                       for vb, vp, x in zip(vals_b, vals_p, passes)],
            "roofline": {
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"fuse_multi_kernel<4, {cfg.pixels_per_thread}, {cfg.acc_blocks}>",
                "algorithmic_bytes_per_launch": bytes_per_tick, "mean_launch_ms": mean_tick_ms,
                "launch_ms_includes": "the work-list copy before the launch",
                "touched_voxels_per_tick": acc["V"] / steps,
                "touched_blocks_per_tick": acc["Bt"] / steps,
                "new_blocks_per_tick": acc["Bn"] / steps,
            },
            "cpu_baseline": cpu,
        }

    def close():
        batch.close()
        cache.clear()
        release(torch)

    return Leg("multi", run_pass, finish, close)


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


def serve_leg(args, torch, T, S) -> Leg:
    """Serving: sessions fed by Poisson frame arrivals, through tsdf_server_*.

    256 sessions (frame sizes 160x120 .. 1280x720, voxels 5..10 mm, pools
    2^14..2^18 blocks, tables twice the pool) are admitted against a 200 GB
    budget, and an arrival trace of 3000 frames/s for one second is rendered.
    Set-up (untimed): each session's frames are fused in arrival order into a
    volume of its own with weight snapshots, which gives every frame's
    algorithmic bytes.  A pass replays the trace in real time through the
    library's native driver on fresh sessions, served (continuous batching
    across sessions, up to --max-inflight launches on streams of their own) and
    plain (one tsdf_fuse_frame per frame on arrival), in alternating order, each
    reporting every frame's latency; then the same frames are replayed with
    every arrival at time zero, which measures the capacity (points/s) of each
    path.  The session counters of the served and plain runs must agree.  Once,
    after the passes: the served run with the frames in pinned host memory read
    by the kernels over PCIe, and a sweep of the arrival rate (the trace's
    arrival times scaled, which keeps it a Poisson process over the same
    frames) giving, per path, the highest swept rate whose p99 latency stays
    within each of several bounds.
    """
    t0 = time.time()
    w = S.ServingWorkload(args.sessions, rate=args.rate, duration_s=args.duration)
    n = len(w)
    depths = [torch.from_numpy(w.depth(int(s), int(k), device="cuda")).cuda()
              for s, k in zip(w.session_of, w.frame_of)]
    cams = [T.camera_struct(w.camera(int(s), int(k))) for s, k in zip(w.session_of, w.frame_of)]
    points = int(sum(int((d > 0).sum()) for d in depths))
    log(f"[bench] serve: rendered {n} frames for {len(w.specs)} sessions in "
        f"{time.time() - t0:.1f}s ({points} points)")
    need = sum(T.volume_bytes(T.volume_params(sp.voxel_size, sp.trunc, sp.table_capacity,
                                              sp.pool_capacity)) for sp in w.specs)
    cfg = T.BatchConfig(*(int(x) for x in args.batch_config.split(","))) if args.batch_config \
        else T.BatchConfig(32, 1, 8, 0)
    served_budget = int(args.budget_gb * 1e9)
    plain_budget = int(need * 1.02) + (64 << 20)

    # ---- algorithmic bytes per frame (untimed) ---------------------------------
    # first: fused into its session's fresh volume (the real-time replay);
    # again: the same frame fused a second time (the capacity replay, which
    # follows it on the same sessions and allocates nothing)
    t0 = time.time()
    first_b, again_b = np.zeros(n), np.zeros(n)
    by_session: dict = {}
    for j, s in enumerate(w.session_of):
        by_session.setdefault(int(s), []).append(j)
    for s, js in sorted(by_session.items()):
        sp = w.specs[s]
        v = T.Volume(sp.voxel_size, sp.trunc, sp.table_capacity, sp.pool_capacity)
        wv = v.weight_view()
        nb0 = 0
        for j in js:
            before = wv[:nb0].reshape(nb0, 512).clone()
            v.fuse(depths[j], cams[j])
            st = v.stats()
            if st.status != T.OK or st.pairs_dropped:
                raise GateFailed(f"serve: session {s} fails alone ({T.status_str(st.status)})")
            nb = st.blocks_total
            changed = wv[:nb].reshape(nb, 512) != torch.nn.functional.pad(before, (0, 0, 0, nb - nb0))
            V = int(changed.sum())
            Bt = int(changed.any(dim=1).sum())
            first_b[j] = algorithmic_bytes(depths[j].numel(), Bt, nb - nb0, V)
            again_b[j] = algorithmic_bytes(depths[j].numel(), Bt, 0, V)
            nb0 = nb
        v.close()
        del v, wv
    release(torch)
    log(f"[bench] serve: algorithmic bytes of the trace {first_b.sum() / 1e9:.2f} GB first, "
        f"{again_b.sum() / 1e9:.2f} GB again ({time.time() - t0:.1f}s)")

    def open_server(budget):
        server = T.Server(budget, max_sessions=len(w.specs) + 1, max_batch=args.max_batch,
                          max_inflight=args.max_inflight, max_queue=max(4096, n))
        server.batch_config(cfg)
        ids = []
        for sp in w.specs:
            sid = server.open(sp.voxel_size, sp.trunc, sp.table_capacity, sp.pool_capacity)
            if sid is None:
                server.close()
                raise GateFailed("serve: a session was not admitted")
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
        return server, ids

    def session_check(server, ids, what):
        stats = [server.session(i)[0].stats() for i in ids]
        fails = [k for k, i in enumerate(ids)
                 if server.session(i)[1] != T.OK or stats[k].status != T.OK]
        if fails:
            raise GateFailed(f"serve: {what}: sessions whose pool or table ran out {fails}; "
                             f"status bits {[stats[k].status_bits for k in fails]}")
        dropped = sum(st.pairs_dropped for st in stats)
        if dropped:
            raise GateFailed(f"serve: {what}: {dropped} pairs dropped")
        return stats

    def compare(a, b, what):
        for i, (x, y) in enumerate(zip(a, b)):
            for f in ("points_valid", "pairs", "pairs_dropped", "blocks_total", "frames"):
                if getattr(x, f) != getattr(y, f):
                    raise GateFailed(f"serve: {what}: session {i} {f} {getattr(x, f)} != "
                                     f"{getattr(y, f)}")

    def run(mode, frames=None):
        frames = depths if frames is None else frames
        server, ids = open_server(served_budget if mode == T.REPLAY_SERVED else plain_budget)
        sess = [ids[int(s)] for s in w.session_of]
        try:
            lat, elapsed = server.replay(w.arrival_ns, sess, frames, cams, mode)
            _, cap = server.replay(np.zeros(n, dtype=np.int64), sess, frames, cams, mode)
            stats = session_check(server, ids, "served" if mode == T.REPLAY_SERVED else "plain")
            used = server.load()["budget_used"]
        finally:
            server.close()
            del server
            release(torch)
        return {"lat": lat, "elapsed": elapsed, "cap": cap, "stats": stats, "used": used}

    def pct(x, q):
        return float(np.percentile(x[x >= 0], q) / 1e6)

    ref = {}

    def run_pass(p):
        modes = (T.REPLAY_SERVED, T.REPLAY_PLAIN) if p % 2 == 0 else (T.REPLAY_PLAIN, T.REPLAY_SERVED)
        res = {m: run(m) for m in modes}
        s_, p_ = res[T.REPLAY_SERVED], res[T.REPLAY_PLAIN]
        compare(s_["stats"], p_["stats"], "served vs plain")
        ref.setdefault("stats", s_["stats"])
        ref.setdefault("used", s_["used"])
        log(f"[bench] serve pass {p}: served p50 {pct(s_['lat'], 50) * 1e3:.1f} us, p99 "
            f"{pct(s_['lat'], 99) * 1e3:.1f} us, capacity {points / s_['cap'] * 1e9:.3e}; plain "
            f"p50 {pct(p_['lat'], 50) * 1e3:.1f} us, p99 {pct(p_['lat'], 99) * 1e3:.1f} us, "
            f"capacity {points / p_['cap'] * 1e9:.3e} points/s")
        return {"served": {k: s_[k] for k in ("lat", "elapsed", "cap")},
                "plain": {k: p_[k] for k in ("lat", "elapsed", "cap")},
                "order": "served, plain" if p % 2 == 0 else "plain, served"}

    def zero_copy():
        """Served again with every frame in pinned host memory, handed over at
        its device address: the kernels read the depth over PCIe."""
        total = sum(d.numel() for d in depths)
        host = torch.empty(total, dtype=torch.float32, pin_memory=True)

        class _Mapped:  # a frame known by its device address
            def __init__(self, addr):
                self.addr = addr

            def data_ptr(self):
                return self.addr

        zframes, off = [], 0
        for d in depths:
            host[off:off + d.numel()].copy_(d.reshape(-1))
            addr = T.host_device_pointer(host[off:].data_ptr())
            if addr is None:
                zframes = None  # no device address: the run is skipped, nothing launched
                break
            zframes.append(_Mapped(addr))
            off += d.numel()
        torch.cuda.synchronize()
        out = None
        if zframes is not None:
            r = run(T.REPLAY_SERVED, frames=zframes)
            compare(ref["stats"], r["stats"], "zero copy vs device frames")
            out = {"p50_latency_ms": pct(r["lat"], 50), "p99_latency_ms": pct(r["lat"], 99),
                   "max_latency_ms": pct(r["lat"], 100),
                   "sustained_points_per_s": points / (r["elapsed"] * 1e-9),
                   "capacity_points_per_s": points / (r["cap"] * 1e-9),
                   "path": "served, every frame in pinned host memory at its device address "
                           "(the kernels read the depth over PCIe; no upload)"}
            log(f"[bench] serve zero copy: p50 {out['p50_latency_ms'] * 1e3:.1f} us, p99 "
                f"{out['p99_latency_ms'] * 1e3:.1f} us")
        del zframes, host
        release(torch)
        return out

    def sweep():
        """Per path, one server whose sessions first take the whole trace once
        (so every rate sees the same volumes, with no new blocks), then the
        trace replayed at each rate."""
        rates = [float(r) for r in args.sweep_rates.split(",") if r]
        rows = {}
        for mode, name in ((T.REPLAY_SERVED, "served"), (T.REPLAY_PLAIN, "plain")):
            server, ids = open_server(served_budget if mode == T.REPLAY_SERVED else plain_budget)
            sess = [ids[int(s)] for s in w.session_of]
            try:
                server.replay(np.zeros(n, dtype=np.int64), sess, depths, cams, mode)
                rows[name] = []
                for r in rates:
                    arr = np.round(w.arrival_ns * (args.rate / r)).astype(np.int64)
                    lat, el = server.replay(arr, sess, depths, cams, mode)
                    rows[name].append({"rate": r, "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                                       "points_per_s": points / (el * 1e-9),
                                       "refused": int(np.sum(lat < 0))})
                session_check(server, ids, f"{name} sweep")
            finally:
                server.close()
                del server
                release(torch)
        table = []
        for b in (0.25, 0.5, 1.0, 2.0):
            row = {"p99_bound_ms": b}
            for name in ("served", "plain"):
                ok = [x for x in rows[name] if x["p99_ms"] <= b and x["refused"] == 0]
                top = max(ok, key=lambda x: x["rate"]) if ok else None
                row[name] = None if top is None else {
                    "rate": top["rate"], "points_per_s": top["points_per_s"], "p99_ms": top["p99_ms"]}
            table.append(row)
            log(f"[bench] serve sweep: p99 <= {b} ms: served "
                f"{row['served']['rate'] if row['served'] else None}, plain "
                f"{row['plain']['rate'] if row['plain'] else None} frames/s")
        return {"rates": rates, "served": rows["served"], "plain": rows["plain"],
                "highest_rate_within_p99": table,
                "note": "the trace's arrival times scaled by 3000/rate, on sessions that already "
                        "hold the trace once; sustained points/s over each replay"}

    def cpu_baseline():
        """The oracle on the frames of the trace's first 32 sessions, in arrival
        order, for about --cpu-seconds: each chunk of 64 arrivals is split by
        session and the sessions fuse on threads."""
        from concurrent.futures import ThreadPoolExecutor

        from oracle import oracle as O
        first_sessions = []
        for s in w.session_of:
            if int(s) not in first_sessions:
                first_sessions.append(int(s))
            if len(first_sessions) == 32:
                break
        chosen = set(first_sessions)
        js = [j for j in range(n) if int(w.session_of[j]) in chosen][:1024]
        frames = {j: depths[j].cpu().numpy() for j in js}
        cam_of = {j: w.camera(int(w.session_of[j]), int(w.frame_of[j])) for j in js}
        vols = {s: O.OracleVolume(w.specs[s].voxel_size, w.specs[s].trunc, w.specs[s].pool_capacity)
                for s in first_sessions}
        n_thr = cpu_threads()

        def fuse_group(group):
            for j in group:
                vols[int(w.session_of[j])].fuse(frames[j], cam_of[j])

        done = 0
        t_c0 = time.perf_counter()
        with ThreadPoolExecutor(n_thr) as ex:
            while done < len(js) and time.perf_counter() - t_c0 < args.cpu_seconds:
                groups: dict = {}
                for j in js[done:done + 64]:
                    groups.setdefault(int(w.session_of[j]), []).append(j)
                list(ex.map(fuse_group, groups.values()))
                done = min(len(js), done + 64)
        t_c = time.perf_counter() - t_c0
        pts = sum(v.stats()["points_valid"] for v in vols.values())
        del vols, frames
        log(f"[bench] serve cpu oracle: {pts / t_c:.3e} points/s over {done} frames")
        return {"value": pts / t_c, "unit": "points/s", "cores": n_thr, "kind": "oracle",
                "sample": f"the first {done} arrivals of the trace's first 32 sessions, fused in "
                          f"arrival order into one volume per session ({pts} points, {t_c:.1f} s), "
                          f"{n_thr} threads on disjoint sessions",
                "host": host_info()}

    def finish(passes):
        zc = zero_copy()
        sw = sweep()
        cpu = None if args.no_cpu_baseline else cpu_baseline()
        cap_s = [x["served"]["cap"] for x in passes]
        cap_p = [x["plain"]["cap"] for x in passes]
        # the capacity replay fuses every frame a second time: its points are `points` again
        value = med([points / (c * 1e-9) for c in cap_s])
        plain_value = med([points / (c * 1e-9) for c in cap_p])
        cap_ns = med(cap_s)
        achieved = float(again_b.sum()) / (cap_ns * 1e-9) / 1e9

        def path(key):
            xs = [x[key] for x in passes]
            return {"p50_latency_ms": med([pct(x["lat"], 50) for x in xs]),
                    "p99_latency_ms": med([pct(x["lat"], 99) for x in xs]),
                    "max_latency_ms": med([pct(x["lat"], 100) for x in xs]),
                    "sustained_points_per_s": med([points / (x["elapsed"] * 1e-9) for x in xs]),
                    "capacity_points_per_s": med([points / (x["cap"] * 1e-9) for x in xs])}

        served, plain = path("served"), path("plain")
        served["refused_frames"] = int(sum(np.sum(x["served"]["lat"] < 0) for x in passes))
        return {
            "metric": METRIC,
            "value": value,
            "unit": "points/s",
            "n_gpus": 1,
            "steps": 1,
            "warmup": 1,
            "ms_per_step": cap_ns * 1e-6,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {
                "workload": f"{len(w.specs)} sessions, Poisson arrivals at {args.rate:g} frames/s "
                            f"for {args.duration:g} s ({n} frames, {points} points; frames "
                            f"160x120..1280x720), voxels 5..10 mm, pools 2^14..2^18 blocks, tables "
                            f"2x pool, budget {args.budget_gb:g} GB ({ref['used'] / 1e9:.1f} GB "
                            "admitted)",
                "path": f"tsdf_server: continuous batching, up to {args.max_batch} frames per "
                        f"launch, {args.max_inflight} launch(es) in flight on streams of their "
                        "own, graph replay",
                "batch_config": {"tile_width": cfg.tile_width,
                                 "pixels_per_thread": cfg.pixels_per_thread,
                                 "acc_blocks": cfg.acc_blocks, "groups_per_cu": cfg.groups_per_cu},
                "step": "every frame of the trace arriving at once (capacity)",
                "parallelism": "single GPU",
            },
            "served": served,
            "plain": plain,
            "capacity_vs_plain": value / plain_value,
            "passes": [{"served_p99_ms": pct(x["served"]["lat"], 99),
                        "plain_p99_ms": pct(x["plain"]["lat"], 99),
                        "served_capacity": points / (x["served"]["cap"] * 1e-9),
                        "plain_capacity": points / (x["plain"]["cap"] * 1e-9),
                        "order": x["order"]} for x in passes],
            "rate_sweep": sw,
            "served_zero_copy": zc,
            "roofline": {
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": f"fuse_multi_kernel<4, {cfg.pixels_per_thread}, {cfg.acc_blocks}> "
                          "(the served capacity replay's launches)",
                "algorithmic_bytes_per_replay": float(again_b.sum()),
                "replay_ms": cap_ns * 1e-6,
                "note": "algorithmic bytes of the served capacity replay over its elapsed time: "
                        "its launches overlap on several streams, so no single launch duration "
                        "applies and this is a lower bound on the kernel's own rate",
            },
            "cpu_baseline": cpu,
        }

    def close():
        depths.clear()
        release(torch)

    return Leg("serve", run_pass, finish, close)


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
    st["shared"] = st["hbm_in_use_gib"] > SHARED_HBM_GIB
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


def trajectory_leg(args, torch, T, S) -> Leg:
    """The room orbit: one step = reset the volume, then fuse all frames.

    Set-up (untimed): the frames are rendered and fused once, frame by frame,
    with weight snapshots, which checks the result (no failure, no dropped
    contribution) and gives each frame's algorithmic bytes.  A pass times the
    plain path (one launch per frame) and the headline path (32 frames per
    launch) over --steps steps after --warmup steps each, in alternating order.
    Once, after the passes: the atomic-request ceiling, cold frames and the
    rates with frames starting in pinned host memory.
    """
    flags = {"fused": T.FUSE_DEFAULT, "two_pass": T.FUSE_TWO_PASS,
             "fused_xcd_remap": T.FUSE_XCD_REMAP}[args.mode]

    # ---- inputs, resident in HBM ---------------------------------------------
    t0 = time.time()
    colour = args.variant == "colour"
    slot = args.variant == "slot"
    if colour:
        w, rgba_np = S.room_trajectory_rgbd(n_frames=300, frames=range(args.frames), device="cuda")
        rgba = [torch.from_numpy(c.view(np.int32)).cuda() for c in rgba_np]
    else:
        w = S.room_trajectory_workload(n_frames=300, frames=range(args.frames), device="cuda")
        rgba_np = rgba = None
    depth = [torch.from_numpy(d).cuda() for d in w.depth]
    cams = [T.camera_struct(c) for c in w.cameras]
    n_pix = w.depth[0].size
    log(f"[bench] trajectory: generated {len(depth)} frames in {time.time() - t0:.1f}s")

    vflags = (T.VOLUME_COLOUR if colour else 0) | (T.VOLUME_SLOT_INDEX if slot else 0)
    table = w.table_capacity
    pool = w.table_capacity if slot else w.pool_capacity  # one block per slot
    vol = T.Volume(w.voxel_size, w.trunc, table, pool, flags=vflags)
    L = T.lib()
    stream = torch.cuda.current_stream()
    sp = T.C.c_void_p(stream.cuda_stream)
    # the upload stream of the end-to-end part, taken before any other leg
    # makes streams: the process has few hardware queues (4 by default), and
    # an upload stream that shares one with `stream` would serialise the
    # uploads behind the launches instead of overlapping them
    copy_stream = torch.cuda.Stream()
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
    full = [j for j, (_, n) in enumerate(chunks) if n == fpl]
    ptr_arr = (T.C.c_void_p * len(ptrs))(*[d.data_ptr() for d in depth])
    cam_arr = (T.CameraC * len(cams))(*cams)
    bflags = T.FUSE_BATCH(args.per_group)
    staged = args.accumulate == "staged"
    if staged and (colour or slot):
        raise GateFailed("--accumulate staged takes the main design's plain volumes only")
    # frames per workgroup as the library takes them: colour volumes and the
    # staged path sum at most two
    pg = min(args.per_group, 2) if colour or staged else args.per_group
    if staged:
        # every record of fpl frames with the band's 2K+1 samples per pixel
        stage_buf = T.staging_buffer(pool, fpl * n_pix * (2 * int(round(w.trunc / w.voxel_size)) + 1))
        stage_ptr = T.C.c_void_p(stage_buf.data_ptr())
        stage_n = stage_buf.numel()
    cbatch = None
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
                st = (L.tsdf_fuse_frames_staged(h, n, p, c, bflags, stage_ptr, stage_n, sp)
                      if staged else L.tsdf_fuse_frames(h, n, p, c, bflags, sp))
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
    del wv
    st = vol.stats()
    if st.status != T.OK or st.pairs_dropped or st.lookup_misses:
        raise GateFailed(f"trajectory: {T.status_str(st.status)} dropped={st.pairs_dropped}")
    points_per_step = st.points_valid
    log(f"[bench] trajectory gate ok: {st.points_valid} points, {st.pairs} pairs, "
        f"{st.blocks_total} blocks, max probe {st.max_probe}, load factor "
        f"{st.blocks_total / w.table_capacity:.3f}")
    launch_bytes = [float(sum(acc_bytes[i0:i0 + n])) for (i0, n) in chunks]
    bytes_per_launch = float(np.mean([launch_bytes[j] for j in full]))

    def timed(run, n_events):
        """--warmup untimed steps, then --steps steps between events: (wall s,
        per-step event intervals in ms)."""
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
            raise GateFailed("trajectory: a timed run changed the result")
        return wall, ms

    def run_pass(p):
        if p % 2 == 0:
            wall_p, frame_ms = timed(fuse_all, len(ptrs))
            wall_b, launch_ms = timed(fuse_batched, len(chunks))
        else:
            wall_b, launch_ms = timed(fuse_batched, len(chunks))
            wall_p, frame_ms = timed(fuse_all, len(ptrs))
        log(f"[bench] trajectory pass {p}: batched {wall_b / args.steps * 1e3:.3f} ms/step, "
            f"plain {wall_p / args.steps * 1e3:.3f} ms/step")
        return {"wall_p": wall_p, "frame_ms": frame_ms, "wall_b": wall_b, "launch_ms": launch_ms,
                "order": "plain, batched" if p % 2 == 0 else "batched, plain"}

    def atomics(mean_launch_ms):
        """Memory-side atomic requests of the headline kernel and their ceiling."""
        ceiling = atomic_ceiling(T, torch, stream)
        req = None
        if os.path.exists(TRAFFIC_FILE):
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("kernel_sha") == kernel_sha() and tr.get("batch") == fpl and \
                    tr.get("per_group") == pg:
                req = tr.get("atomic_requests_per_dispatch")
        return {
            "unit": "G requests/s", "ceiling": ceiling["flush_pattern"],
            "ceiling_full_rows": ceiling["full_rows"],
            "requests_per_launch": req,
            "achieved": req / (mean_launch_ms * 1e-3) / 1e9 if req else None,
            "frac": (req / (mean_launch_ms * 1e-3) / 1e9) / ceiling["flush_pattern"] if req else None,
            "note": "device-scope fp32 atomic requests (TCC_EA0_ATOMIC) of one launch against the "
                    "rate tsdf_measure_atomic_rate sustains in the flush's pattern",
        }

    def cold_frames():
        """One frame into a fresh volume; R volumes are reset outside the timed
        window and fused back to back, each frame between its own events."""
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
                    raise GateFailed("trajectory: a cold frame failed")
                if rep >= args.warmup:
                    cold_ms.append(ev[2 * r].elapsed_time(ev[2 * r + 1]))
                    cold_pts += s_.points_valid
        for cv in cvols:
            cv.close()
        del cvols
        release(torch)
        cold_ms = np.array(cold_ms)
        log(f"[bench] cold frames: mean {cold_ms.mean():.4f} ms")
        return {"value": cold_pts / (cold_ms.sum() * 1e-3), "unit": "points/s",
                "volumes": R, "frame_samples": int(cold_ms.size),
                "mean_frame_ms": float(cold_ms.mean()),
                "p50_frame_ms": float(np.percentile(cold_ms, 50)),
                "p99_frame_ms": float(np.percentile(cold_ms, 99)),
                "path": "plain (one launch per frame), each frame into an empty volume"}

    def end_to_end():
        """Frames start in pinned host memory; each launch's frames are uploaded
        on a copy stream into one of two device buffers, so the upload of one
        launch overlaps the fusion of the one before.  Then the same frames
        read by the fusion kernel itself over PCIe (zero copy)."""
        H_, W_ = w.depth[0].shape
        host = torch.empty((len(ptrs), H_, W_), dtype=torch.float32, pin_memory=True)
        for k in range(len(ptrs)):
            host[k].copy_(torch.from_numpy(w.depth[k]))
        bufs = [torch.empty((fpl, H_, W_), dtype=torch.float32, device="cuda") for _ in range(2)]
        buf_ptrs = [(T.C.c_void_p * fpl)(*[b[i].data_ptr() for i in range(fpl)]) for b in bufs]
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
        del dev_all, bufs
        # zero copy: the same pinned frames read by the fusion kernel itself over
        # PCIe, through the device addresses the runtime maps them at
        zptr = (T.C.c_void_p * len(ptrs))()
        mapped = True
        for k in range(len(ptrs)):
            addr = T.host_device_pointer(host[k].data_ptr())
            if addr is None:
                mapped = False  # no device address: the leg is skipped, nothing launched
                break
            zptr[k] = addr

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
        # the pinned frames and the events of this part go before it returns
        torch.cuda.synchronize()
        del host, free, spans, full_spans
        release(torch)
        log(f"[bench] end to end: {points_per_step * args.steps / wall_e:.3e} points/s, "
            f"H2D {h2d_gbs:.1f} GB/s")
        return {"value": points_per_step * args.steps / wall_e, "unit": "points/s",
                "ms_per_step": wall_e / args.steps * 1e3,
                "median_ms_per_step": float(np.median(e2e_ms[:, 0])),
                "h2d_gb_per_s": h2d_gbs,
                "mean_upload_ms_overlapped": up_ms, "mean_launch_ms_overlapped": fuse_ms,
                "zero_copy": zero_copy,
                "path": f"frames in pinned host memory, {fpl} uploaded per launch on a second "
                        "stream into one of two device buffers, then tsdf_fuse_frames"}

    def cpu_baseline():
        from oracle import oracle as O
        t_c0 = time.perf_counter()
        ov = O.OracleVolume(w.voxel_size, w.trunc, w.pool_capacity)
        k = 0
        while k < len(w.depth) and (k < 1 or time.perf_counter() - t_c0 < args.cpu_seconds):
            if colour:
                ov.fuse_rgb(w.depth[k], rgba_np[k], w.cameras[k])
            else:
                ov.fuse(w.depth[k], w.cameras[k])
            k += 1
        t_c = time.perf_counter() - t_c0
        pts = ov.stats()["points_valid"]
        log(f"[bench] trajectory cpu oracle: {pts / t_c:.3e} points/s over {k} frames")
        return {"value": pts / t_c, "unit": "points/s", "cores": 1, "kind": "oracle",
                "sample": f"first {k} of {len(w.depth)} frames fused sequentially into one volume "
                          f"({pts} points, {t_c:.1f} s, one thread)",
                "host": host_info()}

    def finish(passes):
        steps = args.steps
        vals_b = [points_per_step * steps / x["wall_b"] for x in passes]
        vals_p = [points_per_step * steps / x["wall_p"] for x in passes]
        value, plain_value = med(vals_b), med(vals_p)
        mean_launch_ms = med([x["launch_ms"][:, full].mean() for x in passes])
        achieved = bytes_per_launch / (mean_launch_ms * 1e-3) / 1e9
        traffic = None
        if os.path.exists(TRAFFIC_FILE) and args.variant == "main" and not staged:
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("kernel_sha") == kernel_sha() and tr.get("batch") == fpl and \
                    tr.get("per_group") == pg:
                traffic = tr.get("bytes_per_launch")
        at = atomics(mean_launch_ms) if args.variant == "main" and not staged else None
        cold = e2e = None
        if args.variant == "main" and args.cold_volumes > 0 and not staged:
            # (both time the atomic path)
            cold = cold_frames()
            e2e = end_to_end()
        cpu = None if args.no_cpu_baseline else cpu_baseline()

        def fq(q):
            return med([np.percentile(x["frame_ms"], q) for x in passes])

        return {
            "metric": METRIC,
            "value": value,
            "unit": "points/s",
            "n_gpus": 1,
            "steps": steps,
            "warmup": args.warmup,
            "ms_per_step": med([x["wall_b"] for x in passes]) / steps * 1e3,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {
                "workload": f"room orbit, {len(ptrs)} frames of 640x480, voxel 5 mm, truncation "
                            f"2 cm, table 2^20 slots, pool {'2^20' if slot else '2^18'} blocks"
                            + (", colour images" if colour else ""),
                "path": (f"batched: tsdf_batch_fuse, {fpl} frames of the volume per launch"
                         if colour and args.colour_path == "batch" else
                         f"batched: tsdf_fuse_frames{'_rgb' if colour else ''}"
                         f"{'_staged' if staged else ''}, {fpl} frames per "
                         f"launch, {pg} frame(s) per workgroup"),
                "variant": {"main": "main design", "slot": "block index = table slot",
                            "colour": "TSDF, weight and three colour sums"}[args.variant],
                "frames_per_step": len(ptrs), "points_per_step": points_per_step,
                "parallelism": "single GPU",
            },
            "p50_frame_ms": fq(50),
            "p95_frame_ms": fq(95),
            "p99_frame_ms": fq(99),
            "frame_latency_path": "plain (one launch per frame)",
            "plain": {
                "value": plain_value, "unit": "points/s", "mode": args.mode,
                "ms_per_step": med([x["wall_p"] for x in passes]) / steps * 1e3,
                "mean_frame_ms": med([x["frame_ms"].mean() for x in passes]),
                "p50_frame_ms": fq(50), "p99_frame_ms": fq(99),
                "frame_samples": int(sum(x["frame_ms"].size for x in passes)),
                "median_ms_per_step": med([np.median(x["frame_ms"].sum(axis=1)) for x in passes]),
            },
            "batched": {
                "value": value, "unit": "points/s", "frames_per_launch": fpl,
                "frames_per_workgroup": pg,
                "mean_launch_ms": mean_launch_ms,
                "p50_launch_ms": med([np.percentile(x["launch_ms"][:, full], 50) for x in passes]),
                "p99_launch_ms": med([np.percentile(x["launch_ms"][:, full], 99) for x in passes]),
                "ms_per_frame": mean_launch_ms / fpl,
                "median_ms_per_step": med([np.median(x["launch_ms"].sum(axis=1)) for x in passes]),
            },
            "passes": [{"batched": vb, "plain": vp, "order": x["order"]}
                       for vb, vp, x in zip(vals_b, vals_p, passes)],
            "cold": cold,
            "end_to_end": e2e,
            "roofline": {
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": ("fuse_multi_kernel<4, 1, 4, colour>"
                           if colour and args.colour_path == "batch"
                           else f"stage_kernel<4, {pg}> + stage_apply_kernel"
                           if staged
                           else f"fuse_kernel<4, {pg}, 32, fused"
                                f"{', colour' if colour else ''}>"),
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "mean_launch_ms": mean_launch_ms,
                "touched_voxels_per_frame": acc["V"] / len(ptrs),
                "touched_blocks_per_frame": acc["Bt"] / len(ptrs),
                "new_blocks_per_frame": acc["Bn"] / len(ptrs),
            },
            "atomics": at,
            "cpu_baseline": cpu,
        }

    def close():
        if cbatch is not None:
            cbatch.close()
        vol.close()
        depth.clear()
        if rgba is not None:
            rgba.clear()
        release(torch)

    return Leg("trajectory", run_pass, finish, close)


LEG_KEYS = {"multi": "multi", "serve": "served_vs_plain"}


def run_legs(args, names) -> int:
    """Build the legs, time them in --passes rotated passes, print one line:
    the first leg's object, the others under their keys."""
    import torch

    from paper_2608_08287_amd import scenes as S
    from paper_2608_08287_amd import tsdf as T

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    idle = check_idle(torch)
    if idle["shared"] and not args.allow_shared_gpu:
        print(f"bench.py: {idle['hbm_in_use_gib']:.1f} GiB of HBM are in use before the run: "
              "another process holds the GPU and would distort the timing; not measuring "
              "(--allow-shared-gpu measures anyway)", file=sys.stderr)
        return 3
    makers = {"trajectory": trajectory_leg, "multi": multi_leg, "serve": serve_leg}
    legs, results = [], {}
    orders = []
    try:
        for nm in names:
            legs.append(makers[nm](args, torch, T, S))
        passes = {leg.name: [] for leg in legs}
        for p in range(args.passes):
            r = p % len(legs)
            order = legs[r:] + legs[:r]
            orders.append([leg.name for leg in order])
            for leg in order:
                passes[leg.name].append(leg.run_pass(p))
        for leg in legs:
            results[leg.name] = leg.finish(passes[leg.name])
    except GateFailed as e:
        print(f"gate failed: {e}", file=sys.stderr)
        return 1
    finally:
        for leg in legs:
            leg.close()
        legs.clear()
        release(torch)

    if args.profile_copy_bytes:
        # a plain copy of known size, for scaling the memory counters
        src = torch.empty(args.profile_copy_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        release(torch)

    out = results[names[0]]
    for nm in names[1:]:
        out[LEG_KEYS[nm]] = results[nm]
    out["protocol"] = {
        "passes": args.passes, "leg_order_per_pass": orders,
        "statistic": "median over the passes of each figure; within a leg the two paths run in "
                     "alternating order from pass to pass",
    }
    out["host"] = host_info()
    out["device"] = {"at_start": idle, "after": device_state(torch)}
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--passes", type=int, default=3,
                    help="timed passes over the legs, in rotated order; figures are medians")
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bound on each CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--allow-shared-gpu", action="store_true",
                    help="measure even when another process holds HBM")
    ap.add_argument("--mode", choices=["fused", "two_pass", "fused_xcd_remap"], default="fused",
                    help="plain-path kernel")
    ap.add_argument("--batch", type=int, default=32,
                    help="frames per launch of the batched path (at most 32)")
    ap.add_argument("--per-group", type=int, default=3,
                    help="frames summed per workgroup in the batched path (1 to 4)")
    ap.add_argument("--profile-copy-bytes", type=int, default=0,
                    help="after the legs, copy this many bytes device to device three times "
                         "(the known-size reference for memory counters)")
    ap.add_argument("--variant", choices=["main", "slot", "colour"], default="main",
                    help="trajectory: main design, block index = table slot, or colour sums")
    ap.add_argument("--workload", default="all",
                    choices=["all", "trajectory", "multi", "serve", "stress", "lf-sweep"],
                    help="all: the trajectory headline with the multi and serve legs")
    ap.add_argument("--accumulate", choices=["atomic", "staged"], default="atomic",
                    help="trajectory: the headline path's accumulation: atomic adds from each "
                         "tile (tsdf_fuse_frames) or records applied once per launch "
                         "(tsdf_fuse_frames_staged)")
    ap.add_argument("--colour-path", choices=["frames", "batch"], default="frames",
                    help="colour variant: tsdf_fuse_frames_rgb or tsdf_batch_fuse")
    ap.add_argument("--cold-volumes", type=int, default=8,
                    help="trajectory: volumes for the cold-frame measurement (0: skip it and "
                         "the pinned-host legs)")
    ap.add_argument("--sessions", type=int, default=256, help="serve: sessions")
    ap.add_argument("--rate", type=float, default=3000.0, help="serve: frames/s, all sessions")
    ap.add_argument("--duration", type=float, default=1.0, help="serve: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: session budget")
    ap.add_argument("--max-batch", type=int, default=256, help="serve: frames per launch")
    ap.add_argument("--max-inflight", type=int, default=4,
                    help="serve: launches in flight, one stream each")
    ap.add_argument("--sweep-rates", default="1500,3000,6000,9000,12000,15000,18000,21000,24000",
                    help="serve: arrival rates of the sweep, frames/s")
    ap.add_argument("--volumes", type=int, default=64, help="multi: volumes per tick")
    ap.add_argument("--trials", type=int, default=2, help="multi: autotuner trials per candidate")
    ap.add_argument("--batch-config", default="",
                    help="multi/serve: fixed tile_width,pixels_per_thread,acc_blocks,groups_per_cu "
                         "instead of tuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the volume is not sharded across GPUs", file=sys.stderr)
        return 2
    if args.passes < 1 or args.steps < 1 or args.warmup < 0:
        print("bench.py: --passes and --steps must be at least 1", file=sys.stderr)
        return 2
    if args.workload in ("stress", "lf-sweep"):
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 1
        if args.workload == "stress":
            args.frames = min(args.frames, 100)
            return bench_stress(args)
        return bench_lf_sweep(args)
    names = {"all": ["trajectory", "multi", "serve"], "trajectory": ["trajectory"],
             "multi": ["multi"], "serve": ["serve"]}[args.workload]
    return run_legs(args, names)


if __name__ == "__main__":
    sys.exit(main())
