"""Helpers shared by the GPU parity tests: run a workload through the C ABI and
compare with the oracle (keys and weights exact, TSDF means within a tolerance,
table and pool invariants)."""
from __future__ import annotations

import dataclasses
import math
import sys
from typing import Optional, Sequence

import numpy as np
import torch

from oracle import oracle as O
from paper_2608_08287_amd import scenes as S
from paper_2608_08287_amd import tsdf as T

# TSDF means: float32 sums on the GPU in a racy order against float64 sums in the
# oracle.  A mean of n contributions, each |x| <= tau <= 0.04 m, carries at most
# about n * 2^-24 * tau of float32 rounding: 1e-5 holds up to n ~ 4000.
TSDF_ATOL = 1e-5
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


@dataclasses.dataclass
class GpuResult:
    keys: np.ndarray     # uint64, ascending
    means: np.ndarray    # (n, 512) float32
    weights: np.ndarray  # (n, 512) float32
    stats: T.Stats
    vol: Optional[T.Volume] = None


def run_gpu(voxel_size, trunc, table_capacity, pool_capacity, depths: Sequence[np.ndarray], cams,
            prefill_blocks=None, flags=T.FUSE_DEFAULT, keep_volume=False,
            vol: Optional[T.Volume] = None, batched: bool = False,
            staged: Optional[int] = None) -> GpuResult:
    """Fuse through one launch per frame, tsdf_fuse_frames (`batched`), or
    tsdf_fuse_frames_staged with staging for `staged` records per launch."""
    if vol is None:
        vol = T.Volume(voxel_size, trunc, table_capacity, pool_capacity)
    if prefill_blocks is not None:
        vol.insert_blocks(torch.from_numpy(np.ascontiguousarray(prefill_blocks, dtype=np.int32)).cuda())
    dev = [torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda() for d in depths]
    if staged is not None:
        vol.fuse_frames_staged(dev, cams, T.staging_buffer(pool_capacity, staged), flags)
    elif batched:
        vol.fuse_frames(dev, cams, flags)
    else:
        for d, c in zip(dev, cams):
            vol.fuse(d, c, flags)
    return result_of(vol, keep_volume)


def result_of(vol: T.Volume, keep_volume=False) -> GpuResult:
    """Stats and extracted blocks of a volume, blocks sorted by key, on the host."""
    st = vol.stats()
    ex = vol.extract()
    torch.cuda.synchronize()
    keys = ex.keys.cpu().numpy().view(np.uint64)
    order = np.argsort(keys, kind="stable")
    res = GpuResult(keys[order], ex.tsdf.cpu().numpy()[order], ex.weight.cpu().numpy()[order], st)
    if keep_volume:
        res.vol = vol
    return res


STAT_FIELDS = ("points_valid", "pairs", "pairs_dropped", "coord_out_of_range", "blocks_total",
               "keys_pool_overflow", "lookup_misses", "status_bits", "frames")


def assert_conserved(v: T.Volume, st: T.Stats) -> None:
    """Every pair that passed the walk is either in a weight or counted as
    dropped, and the pool is full whenever pairs were dropped."""
    ex = v.extract()
    assert ex.keys.numel() == st.blocks_total
    assert torch.unique(ex.keys).numel() == ex.keys.numel(), "a key owns two blocks"
    assert int(ex.weight.double().sum().item()) + st.pairs_dropped == st.pairs
    if st.pairs_dropped:
        assert st.blocks_total == v.layout.pool_capacity
        assert st.status_bits & T.FLAG_POOL_EXHAUSTED


def assert_same_volume(a: T.Volume, b: T.Volume, atol=TSDF_ATOL) -> T.Stats:
    """Two GPU volumes hold the same fusion result: block keys and weights
    identical, TSDF means within atol, counters equal.  Compared on the device
    (packed keys use 63 bits, so int64 order is key order).

    Once a pool runs out, which keys got its last blocks depends on the order
    in which workgroups reached them, so for volumes that dropped pairs only
    the order-free facts are compared (points, pairs, a full pool, status) and
    each volume must conserve its pairs."""
    sa, sb = a.stats(), b.stats()
    if sa.pairs_dropped or sb.pairs_dropped:
        for f in ("points_valid", "pairs", "coord_out_of_range", "blocks_total", "status_bits",
                  "frames"):
            assert getattr(sa, f) == getattr(sb, f), (f, getattr(sa, f), getattr(sb, f))
        assert_conserved(a, sa)
        assert_conserved(b, sb)
        return sa
    for f in STAT_FIELDS:
        assert getattr(sa, f) == getattr(sb, f), (f, getattr(sa, f), getattr(sb, f))
    ea, eb = a.extract(), b.extract()
    assert ea.keys.numel() == eb.keys.numel()
    ka, ia = torch.sort(ea.keys)
    kb, ib = torch.sort(eb.keys)
    assert torch.equal(ka, kb), "block key sets differ"
    assert torch.equal(ea.weight[ia], eb.weight[ib]), "weights differ"
    if ka.numel():
        err = (ea.tsdf[ia].double() - eb.tsdf[ib].double()).abs().max().item()
        assert err <= atol, err
    return sa


def run_workload(w, flags=T.FUSE_DEFAULT, keep_volume=False, **kw) -> GpuResult:
    return run_gpu(w.voxel_size, w.trunc, w.table_capacity, w.pool_capacity, w.depth, w.cameras,
                   w.prefill_blocks, flags, keep_volume, **kw)


def oracle_slices(voxel_size, trunc, pool_capacity, depths: Sequence[np.ndarray], cams,
                  n_slices: int, prefill_blocks=None, rgbas=None) -> list:
    """The frames cut into n_slices contiguous slices, each fused into its own
    oracle volume (after the same pre-filled blocks, if any; with the colour
    images, if given); the slices run on threads (the oracle's calls release
    the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    n = len(depths)
    bounds = [n * i // n_slices for i in range(n_slices + 1)]

    def part(i):
        ov = O.OracleVolume(voxel_size, trunc, pool_capacity)
        if prefill_blocks is not None:
            ov.insert_blocks(prefill_blocks)
        for k in range(bounds[i], bounds[i + 1]):
            if rgbas is None:
                ov.fuse(depths[k], cams[k])
            else:
                ov.fuse_rgb(depths[k], rgbas[k], cams[k])
        return ov

    with ThreadPoolExecutor(n_slices) as ex:
        return list(ex.map(part, range(n_slices)))


def add_slices(parts: list, keys: np.ndarray, colour: bool = False):
    """Sum the slices' TSDF sums and weights into (len(keys), 512) arrays over
    `keys` (ascending), dropping each slice once added.  Returns the sums, the
    weights, a mask of the keys some slice allocated, and the summed point and
    pair counts, and with `colour` also the (len(keys), 3, 512) colour sums.
    Fails if a slice dropped pairs or holds a key outside `keys`."""
    col = np.zeros((keys.size, 3, 512), dtype=np.float64) if colour else None
    sums = np.zeros((keys.size, 512), dtype=np.float64)
    weights = np.zeros((keys.size, 512), dtype=np.uint32)
    seen = np.zeros(keys.size, dtype=bool)
    points = pairs = 0
    for i in range(len(parts)):
        r = parts[i].result()
        c = parts[i].colour_sums() if colour else None
        parts[i] = None
        assert r.stats["pairs_dropped"] == 0
        idx = np.searchsorted(keys, r.keys)
        assert np.all(idx < keys.size) and np.array_equal(keys[idx], r.keys), \
            f"slice {i} holds blocks outside the key set"
        sums[idx] += r.sums
        weights[idx] += r.weights
        if colour:
            col[idx] += c
        seen[idx] = True
        points += r.stats["points_valid"]
        pairs += r.stats["pairs"]
    if colour:
        return sums, weights, seen, points, pairs, col
    return sums, weights, seen, points, pairs


def assert_parity(g: GpuResult, o: O.OracleResult, atol=TSDF_ATOL) -> None:
    assert g.keys.size == o.keys.size, (g.keys.size, o.keys.size)
    assert np.array_equal(g.keys, o.keys), "block key sets differ"
    assert np.array_equal(g.weights, o.weights.astype(np.float32)), "weights differ"
    err = np.abs(g.means.astype(np.float64) - o.means)
    assert float(err.max(initial=0.0)) <= atol, float(err.max())
    assert g.stats.points_valid == o.stats["points_valid"]
    assert g.stats.pairs == o.stats["pairs"]
    assert g.stats.pairs_dropped == o.stats["pairs_dropped"]
    assert g.stats.coord_out_of_range == o.stats["coord_out_of_range"]
    assert g.stats.blocks_total == o.stats["blocks"]
    assert g.stats.keys_pool_overflow == o.stats["pool_overflow_keys"]


def table_arrays(vol: T.Volume):
    t = vol.table_view().cpu().numpy()
    keys = t[:, 0].view(np.uint64).copy()
    blocks = (t[:, 1] & 0xFFFFFFFF).astype(np.uint32).view(np.int32)
    return keys, blocks


def assert_table_invariants(vol: T.Volume, expect_keys: np.ndarray, n_blocks: int) -> None:
    """The GPU table against the sequential linear-probe model.

    expect_keys: every key that must be in the table (allocated or pool-full).
    """
    keys, blocks = table_arrays(vol)
    C = keys.size
    occ = np.nonzero(keys != EMPTY)[0]
    tk = keys[occ]
    assert np.unique(tk).size == tk.size, "duplicate keys in the table"
    assert np.array_equal(np.sort(tk), np.sort(expect_keys)), "table key set differs"
    tb = blocks[occ]
    assert np.all((tb >= 0) | (tb == -2)), "unpublished or corrupt entry"
    alloc = np.sort(tb[tb >= 0])
    assert np.array_equal(alloc, np.arange(n_blocks)), "pool indices are not a permutation"
    bk = vol.block_keys_view()[:max(n_blocks, 0)].cpu().numpy().view(np.uint64)
    assert np.array_equal(bk[tb[tb >= 0]], tk[tb >= 0]), "block_keys does not match the table"
    model = O.probe_model(tk, C)  # any insertion order gives the same layout
    assert np.array_equal(model.occupied, occ), "occupied slots differ from the probe model"
    homes = np.array([O.home_slot(int(k), C) for k in tk], dtype=np.int64)
    disp = (occ.astype(np.int64) - homes) % C
    assert int(disp.sum()) == int(model.disp_of.sum()), "total displacement differs"
    # no empty slot between a key's home and its slot
    empty = keys == EMPTY
    cum = np.concatenate([[0], np.cumsum(np.concatenate([empty, empty]).astype(np.int64))])
    starts, ends = homes, homes + disp
    assert np.all(cum[ends] - cum[starts] == 0), "empty slot inside a probe path"


def rotation(a, b, c):
    """Rz(a) Ry(b) Rx(c)."""
    ca, sa, cb, sb, cc, sc = (math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c),
                              math.sin(c))
    return (np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
            @ np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
            @ np.array([[1, 0, 0], [0, cc, -sc], [0, sc, cc]]))


def scattered_frames(n, W=64, H=48, seed=0, focal=30.0, lo=0.3, hi=3.0, jitter=0.1):
    """n frames of depths uniform in [lo, hi] from cameras near the origin
    (rotations and offsets scaled by `jitter`): every pixel's band lands
    apart from its neighbours', so a tile touches as many voxels as it has
    samples."""
    rng = np.random.default_rng(seed)
    cams, depths = [], []
    for i in range(n):
        pose = np.concatenate([rotation(*rng.uniform(-0.3, 0.3, 3) * jitter / 0.1),
                               rng.uniform(-jitter, jitter, (3, 1))], 1)
        cams.append(S.Camera(W, H, focal, focal * 0.95, W / 2 - 0.5, H / 2 + 0.5,
                             pose.astype(np.float32)))
        depths.append(rng.uniform(lo, hi, (H, W)).astype(np.float32))
    return depths, cams


# name: (voxel, truncation, frame options)
SCATTER = {
    "sparse_4mm_K4": (0.004, 0.016, {}),
    "sparse_1mm_K8": (0.001, 0.008, {}),
    "dense_1mm_K8": (0.001, 0.008, dict(W=32, H=32, focal=1000.0, lo=1.0, hi=1.12, jitter=0.001)),
}
