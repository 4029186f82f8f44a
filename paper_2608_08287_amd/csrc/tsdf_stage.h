// Staged accumulation: the tile kernel of tsdf_fuse_frames_staged.
//
// The same walk, key set and table resolve as fuse_tile (tsdf_device.h), and
// the same per-voxel sums in LDS, but the sums do not go to the pool.  The
// integrate stage of Section 2.2 is a sum of contributions, and sums commute,
// so they can be gathered per block first and added once per launch:
//
//   1. walk   -- each lane walks its pixel's band in each of its frames and
//                keeps, per sample, the voxel's in-block index, its block's
//                LDS key-set slot and the truncated distance in registers (no
//                second walk);
//   2. resolve -- each distinct block key of the tile once against the table
//                (Section 2.3's insert protocol, resolve_key);
//   3. stage  -- each pair becomes a 4-byte record (its voxel's in-block index
//                and its truncated distance in fixed point).  The pairs of each
//                block are counted in LDS (per half wave, so that lanes of one
//                wave that hit one block contend less), a workgroup scan lays
//                the tile's blocks out one after another in LDS, one lane
//                reserves the tile's span of the launch's record array (one
//                device atomic), and one lane per block lists the block's run in
//                the block's run table (one device atomic, which also counts the
//                block's runs and records; each time a block's records pass a
//                multiple of kStageItemRecords it gains an apply work item).
//                Each pair writes its
//                record to its block's next LDS place, and the tile's records
//                are copied out as one contiguous span (coalesced stores).  A run
//                that finds its block's run table full, or a tile that finds the
//                record array full, is added to the pool directly with device
//                atomics, as the apply kernel adds everything else: all pool
//                updates commute, so this launch may even run while the
//                previous one is being applied.
//
// stage_apply_kernel (tsdf_kernels.hip) then takes the launch's work items: an
// item sums its share of a block's runs per voxel in LDS and adds the sums to
// the block's pool segments, one memory-side request per touched segment.  One
// device atomic per (tile, block) replaces one per (tile, pool segment), a
// segment takes one request per item (one per launch for most blocks) instead of one from
// every tile and frame, and the tile needs no per-voxel slots (no masks,
// prefix sums or passes): the apply kernel sums per voxel for the whole launch.
#pragma once

#include "tsdf_device.h"

namespace tsdf {
namespace {

// LDS of one staged tile: the block-key set (phases 1-2), whose room the
// tile's records take over in phase 3; the key list; per set slot the pool
// index and per half wave the count of its pairs, then the next LDS record of
// its share; per key its run in the block's area and its run in LDS.
constexpr unsigned kStageSubs = 2;  // one pair counter per half wave
template <unsigned kRecs>
struct alignas(16) StageShared {
  union {
    unsigned long long keys[kSetCap];
    unsigned recs[kRecs];
  } u;
  unsigned short list[kSetCap];
  unsigned n;  // distinct keys in the set
  unsigned wsum[kThreads / kWave];
  int blockd[kSetCap];
  unsigned bucket[kSetCap * kStageSubs];
  unsigned run_spill[kSetCap];  // 1: the run goes to the pool directly
  unsigned run_lds[kSetCap];    // first LDS record | count << 16
  unsigned base;                // the tile's first record in the launch's array
};

// A contribution as a record: the truncated distance in signed 23-bit fixed
// point of the truncation distance (|sdf| <= trunc, clamped against rounding
// at the ends), above the in-block index.
__device__ __forceinline__ unsigned stage_record(float sdf, unsigned loc, float to_fixed) {
  int q = (int)__builtin_rintf(sdf * to_fixed);
  q = q < -kStageQuantum ? -kStageQuantum : (q > kStageQuantum ? kStageQuantum : q);
  return ((unsigned)q << 9) | loc;
}

template <int K, int F>
constexpr unsigned stage_records() {
  return (unsigned)F * kThreads * (2u * K + 1u);
}

template <int K, int F, bool kLong>
__device__ __forceinline__ void stage_tile(const VolumeDev& vol, const WalkParams& wp,
                                           const FrameDev (&frs)[F], const unsigned (&px)[F],
                                           const unsigned (&py)[F], unsigned shard,
                                           const StageDev& stg,
                                           StageShared<stage_records<K, F>()>& sh) {
  constexpr int NS = 2 * K + 1;
  unsigned long long* const s_keys = sh.u.keys;
  unsigned* const s_n = &sh.n;
  int* const s_blockd = sh.blockd;
  unsigned short* const s_list = sh.list;
  unsigned* const s_bucket = sh.bucket;

  const unsigned tid = threadIdx.x;
  for (unsigned i = tid; i < kSetCap; i += kThreads) s_keys[i] = kEmptyKey;
  {
    uint4* b4 = reinterpret_cast<uint4*>(s_bucket);
    for (unsigned i = tid; i < kSetCap * kStageSubs / 4u; i += kThreads) b4[i] = make_uint4(0, 0, 0, 0);
  }
  if (tid == 0) *s_n = 0;

  float d[F];
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    const FrameDev& fr = frs[fi];
    const bool inside = px[fi] < fr.width && py[fi] < fr.height;
    d[fi] = inside ? fr.depth[(size_t)py[fi] * fr.width + px[fi]] : 0.0f;
  }
  __syncthreads();

  // ---- phase 1: walk, per-point dedupe, block keys into the LDS set --------
  unsigned st[F][NS];  // kPairValid | set slot << 9 | in-block index, or 0
  float val[F][NS];    // the pair's truncated distance
  unsigned ovf[F];     // samples whose key found the LDS set full
  unsigned n_pts = 0, n_pairs = 0, n_oor = 0;
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    const FrameDev& fr = frs[fi];
    const float df = d[fi];
    const bool point = __builtin_isfinite(df) && df > 0.0f;  // 0 outside the frame
    n_pts += point ? 1u : 0u;
    const float a = ((float)px[fi] - fr.cx) * fr.ifx;
    const float b = ((float)py[fi] - fr.cy) * fr.ify;
    bool have_prev = false;
    int pbx = 0, pby = 0, pbz = 0;
    unsigned prev_slot = kSetNone;
    ovf[fi] = 0u;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const Sample smp = walk_sample(fr, wp, df, a, b, s - K);
      const bool z_ok = point && (df + (float)(s - K) * wp.v > 0.0f);
      if (z_ok && !smp.in_range) ++n_oor;
      const bool cand = point && smp.keep;  // keep implies in range
      const int bx = smp.vx >> 3, by = smp.vy >> 3, bz = smp.vz >> 3;
      const unsigned loc = voxel_index((unsigned)smp.vx & 7u, (unsigned)smp.vy & 7u, (unsigned)smp.vz & 7u);
      // consecutive kept samples of a point mostly share a block: reuse its slot
      const bool need = cand && !(have_prev && bx == pbx && by == pby && bz == pbz);
      unsigned slot = prev_slot;
      if (need) slot = set_insert(s_keys, s_list, s_n, pack_key(bx, by, bz));
      if (cand) {
        have_prev = true;
        pbx = bx;
        pby = by;
        pbz = bz;
        prev_slot = slot;
      }
      // a voxel counts once per point (see fuse_tile)
      const unsigned word = kPairValid | (slot << 9) | loc;
      bool dup = false;
      if (cand && slot != kSetNone) {
#pragma unroll
        for (int j = 0; j < s; ++j) dup |= st[fi][j] == word;
      } else if (cand) {
        for (unsigned m = ovf[fi]; m != 0u; m &= m - 1u) {
          const Sample o = walk_sample(fr, wp, df, a, b, __builtin_ctz(m) - K);
          dup |= o.vx == smp.vx && o.vy == smp.vy && o.vz == smp.vz;
        }
      }
      const bool pair = cand && !dup;
      n_pairs += pair ? 1u : 0u;
      const bool spilled = pair && slot == kSetNone;
      ovf[fi] |= spilled ? (1u << s) : 0u;
      st[fi][s] = (pair && !spilled) ? word : 0u;
      val[fi][s] = smp.val;
    }
  }
  // phase 1's counts, fixed here rather than at the end of the tile (see fuse_tile)
  asm volatile("" : "+v"(n_pts), "+v"(n_pairs), "+v"(n_oor));
  __syncthreads();

  // ---- phase 2: resolve each distinct key of the tile once; count pairs ----
  const unsigned n_keys = *s_n;
  unsigned my_probe_max = 0, my_missing = 0;
  for (unsigned base = 0; base < n_keys; base += kThreads) {
    const unsigned j = base + tid;
    const bool act = j < n_keys;
    const unsigned h = act ? s_list[j] : 0u;
    const unsigned long long key = act ? s_keys[h] : kEmptyKey;
    unsigned probes = 0;
    bool missing = false;
    const int blk = resolve_key<true, kLong>(vol, key, act, probes, missing);
    if (act) {
      s_blockd[h] = blk;
      my_probe_max = probes > my_probe_max ? probes : my_probe_max;
      my_missing += missing ? 1u : 0u;
      if (vol.probe_hist) count_probe(vol, probes);
    }
  }
  // the pairs of each (set slot, half wave)
  const unsigned sub = (lane_id() >> 5) & (kStageSubs - 1u);
#pragma unroll
  for (int fi = 0; fi < F; ++fi)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const unsigned w = st[fi][s];
      if (w & kPairValid)
        __hip_atomic_fetch_add(s_bucket + ((w >> 9) & 0x3FFu) * kStageSubs + sub, 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  __syncthreads();

  // ---- phase 3: runs laid out, listed, records placed and copied out -------
  // Thread t takes keys 4t .. 4t+3: a workgroup scan over the keys' pair
  // counts lays their runs out in LDS (the half-wave counters become the next
  // record of each half's share), and thread 0 reserves the tile's span of the
  // launch's record array.
  constexpr unsigned kPer = kSetCap / kThreads;
  unsigned tile_total = 0;
  {
    unsigned mine = 0;
#pragma unroll
    for (unsigned i = 0; i < kPer; ++i) {
      const unsigned j = tid * kPer + i;
      if (j < n_keys) {
        const unsigned h = s_list[j];
        const unsigned total =
            s_blockd[h] >= 0 ? s_bucket[h * kStageSubs] + s_bucket[h * kStageSubs + 1] : 0u;
        sh.run_lds[j] = total << 16;  // the LDS place follows the scan
        mine += total;
      }
    }
    const unsigned incl = wave_inclusive_scan(mine);
    if (lane_id() == kWave - 1) sh.wsum[tid / kWave] = incl;
    __syncthreads();
    unsigned at = incl - mine;
#pragma unroll
    for (unsigned wv = 0; wv < kThreads / kWave; ++wv) {
      const unsigned ws = sh.wsum[wv];
      at += wv < tid / kWave ? ws : 0u;
      tile_total += ws;
    }
#pragma unroll
    for (unsigned i = 0; i < kPer; ++i) {
      const unsigned j = tid * kPer + i;
      if (j < n_keys) {
        const unsigned total = sh.run_lds[j] >> 16;
        sh.run_lds[j] = at | (total << 16);
        if (total) {
          const unsigned h = s_list[j];
          const unsigned lo = s_bucket[h * kStageSubs];
          s_bucket[h * kStageSubs] = at;
          s_bucket[h * kStageSubs + 1] = at + lo;
        }
        at += total;
      }
    }
    if (tid == 0) sh.base = tile_total ? add_u32(stg.head + 1, tile_total) : 0u;
  }
  __syncthreads();
  // the tile's runs into their blocks' run tables; a block gains a work item
  // each time its records pass a multiple of kStageItemRecords
  const unsigned base = sh.base;
  const bool tile_fits = (unsigned long long)base + tile_total <= stg.rec_cap;
#pragma unroll
  for (unsigned i = 0; i < kPer; ++i) {
    const unsigned j = tid * kPer + i;
    const unsigned rl = j < n_keys ? sh.run_lds[j] : 0u;
    const unsigned total = rl >> 16;
    const int blk = total ? s_blockd[s_list[j]] : -1;
    bool spill = !tile_fits;
    unsigned item0 = 0, n_items = 0;
    if (total && tile_fits) {
      const unsigned long long old =
          __hip_atomic_fetch_add(stg.block_stat + blk, (1ull << 32) | total, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      const unsigned r = (unsigned)(old >> 32), before = (unsigned)old;
      spill = r >= kStageRuns;
      if (!spill)
        stg.runs[(size_t)blk * kStageRuns + r] =
            (unsigned long long)(base + (rl & 0xFFFFu)) | ((unsigned long long)total << 32);
      item0 = (before + kStageItemRecords - 1) / kStageItemRecords;
      n_items = (before + total + kStageItemRecords - 1) / kStageItemRecords - item0;
    }
    if (j < n_keys) sh.run_spill[j] = (total && spill) ? 1u : 0u;
    const unsigned incl = wave_inclusive_scan(n_items);
    const unsigned wave_items = (unsigned)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    if (wave_items) {
      unsigned at = 0;
      if (lane_id() == 0) at = add_u32(stg.head + 2, wave_items);
      at = (unsigned)__builtin_amdgcn_readfirstlane((int)at) + incl - n_items;
      for (unsigned k = 0; k < n_items; ++k) {
        if (at + k < stg.item_cap) {
          stg.items[2u * (at + k)] = (unsigned)blk;
          stg.items[2u * (at + k) + 1u] = item0 + k;
        }
      }
    }
  }

  unsigned n_drop = 0;
  unsigned* const s_recs = sh.u.recs;  // the key set is no longer read
#pragma unroll
  for (int fi = 0; fi < F; ++fi)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const unsigned w = st[fi][s];
      if (w & kPairValid) {
        const unsigned h = (w >> 9) & 0x3FFu;
        if (s_blockd[h] < 0) {
          ++n_drop;  // the pool had no block for this key
        } else {
          const unsigned p = __hip_atomic_fetch_add(s_bucket + h * kStageSubs + sub, 1u,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          s_recs[p] = stage_record(val[fi][s], w & 511u, stg.to_fixed);
        }
      }
      // one pair at a time: hoisting every pair's LDS reservation ahead
      // would hold all their results in registers at once
      __builtin_amdgcn_sched_barrier(0);
    }
  __syncthreads();
  // the tile's records out as one span; runs that could not be listed are
  // added to the pool directly
  if (tile_fits)
    for (unsigned p = tid; p < tile_total; p += kThreads) stg.recs[base + p] = s_recs[p];
  for (unsigned j = tid / kWave; j < n_keys; j += kThreads / kWave) {
    if (!sh.run_spill[j]) continue;
    const unsigned rl = sh.run_lds[j];
    const unsigned total = rl >> 16, first = rl & 0xFFFFu;
    float* const bp = vol.voxels + (size_t)s_blockd[s_list[j]] * kBlockFloats;
    for (unsigned i = lane_id(); i < total; i += kWave) {
      const unsigned rec = s_recs[first + i], loc = rec & 511u;
      add_f32(bp + pool_tsdf_index(loc), (float)((int)rec >> 9) * stg.to_metres);
      add_f32(bp + pool_weight_index(loc), 1.0f);
    }
  }
  // Pairs whose key did not fit the LDS set (a tile of more than kSetCap
  // blocks): resolved one by one and added to the pool directly.
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    const FrameDev& fr = frs[fi];
    const float a = ((float)px[fi] - fr.cx) * fr.ifx;
    const float b = ((float)py[fi] - fr.cy) * fr.ify;
    for (unsigned m = ovf[fi]; m != 0u; m &= m - 1u) {
      const int s = __builtin_ctz(m);
      const Sample smp = walk_sample(fr, wp, d[fi], a, b, s - K);
      unsigned probes = 0;
      bool missing = false;
      const int blk = resolve_key<true, kLong>(vol, pack_key(smp.vx >> 3, smp.vy >> 3, smp.vz >> 3),
                                               true, probes, missing);
      my_missing += missing ? 1u : 0u;
      if (vol.probe_hist) count_probe(vol, probes);
      if (blk >= 0) {
        const unsigned loc = voxel_index((unsigned)smp.vx & 7u, (unsigned)smp.vy & 7u, (unsigned)smp.vz & 7u);
        float* bp = vol.voxels + (size_t)blk * kBlockFloats;
        add_f32(bp + pool_tsdf_index(loc), smp.val);
        add_f32(bp + pool_weight_index(loc), 1.0f);
      } else {
        ++n_drop;
      }
    }
  }

  // ---- counters: one atomic per wave, spread over shards -------------------
  const unsigned wave = tid / kWave;
  const bool leader = lane_id() == 0;
  const unsigned pts_w = wave_sum(n_pts);
  const unsigned pairs_w = wave_sum(n_pairs);
  const unsigned sh_i = (shard * 4u + wave) & (kCounterShards - 1);
  if (leader && pts_w) add_u64(&vol.ctr->points_valid[sh_i], pts_w);
  if (leader && pairs_w) add_u64(&vol.ctr->pairs[sh_i], pairs_w);
  if (__ballot(n_drop)) {
    const unsigned dw = wave_sum(n_drop);
    if (leader) add_u64(&vol.ctr->pairs_dropped, dw);
  }
  if (__ballot(n_oor)) {
    const unsigned ow = wave_sum(n_oor);
    if (leader) add_u64(&vol.ctr->coord_out_of_range, ow);
  }
  if (__ballot(my_missing)) {
    const unsigned mw = wave_sum(my_missing);
    if (leader) add_u32(&vol.ctr->lookup_misses, mw);
  }
  if (__ballot(my_probe_max)) {
    const unsigned pm = wave_max(my_probe_max);
    if (leader && pm > *(volatile unsigned*)&vol.ctr->max_probe)
      __hip_atomic_fetch_max(&vol.ctr->max_probe, pm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int NB>
struct StageArgs {
  VolumeDev vol;
  WalkParams wp;
  StageDev stg;
  FrameDev f[NB];
  unsigned n_frames, tiles_x, n_tiles, pad;
};

// One workgroup = one 32x8 tile of F consecutive frames of the launch, as
// fuse_kernel.  Frames and parameters are read from the argument segment.
template <int K, int F, int NB, bool kLong>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(F == 2 ? 4 : 1)))
void stage_kernel(StageArgs<NB> args) {
  __shared__ StageShared<stage_records<K, F>()> ss;
  const StageArgs<NB>& A =
      *(const StageArgs<NB>*)(ConstPtr<StageArgs<NB>>)__builtin_amdgcn_kernarg_segment_ptr();
  const unsigned n_tiles = A.n_tiles, tiles_x = A.tiles_x;
  const unsigned group = blockIdx.x / n_tiles;
  const unsigned tile = blockIdx.x % n_tiles;
  const unsigned x = (tile % tiles_x) * kTileW + (threadIdx.x % kTileW);
  const unsigned y = (tile / tiles_x) * kTileH + (threadIdx.x / kTileW);
  FrameDev frs[F];
  unsigned px[F], py[F];
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    const unsigned idx = group * F + fi;
    const bool in_batch = idx < A.n_frames;
    frs[fi] = A.f[in_batch ? idx : 0u];
    if (!in_batch) frs[fi].width = frs[fi].height = 0;
    px[fi] = x;
    py[fi] = y;
  }
  stage_tile<K, F, kLong>(A.vol, A.wp, frs, px, py, blockIdx.x, A.stg, ss);
}

template <int K, int F, bool kLong>
hipError_t launch_stage_kf(const VolumeDev& vol, const WalkParams& wp, const FrameDev* frames,
                           int n, const StageDev& stg, hipStream_t s) {
  StageArgs<kMaxBatchFrames> args;
  args.vol = vol;
  args.wp = wp;
  args.stg = stg;
  unsigned w = 0, h = 0;
  for (int i = 0; i < kMaxBatchFrames; ++i) {
    args.f[i] = frames[i < n ? i : 0];
    if (i < n) {
      w = frames[i].width > w ? frames[i].width : w;
      h = frames[i].height > h ? frames[i].height : h;
    }
  }
  const unsigned tx = (w + kTileW - 1) / kTileW, ty = (h + kTileH - 1) / kTileH;
  const unsigned n_tiles = tx * ty;
  if (n_tiles == 0) return hipSuccess;
  args.n_frames = (unsigned)n;
  args.tiles_x = tx;
  args.n_tiles = n_tiles;
  args.pad = 0;
  const unsigned groups = ((unsigned)n + F - 1) / F;
  hipLaunchKernelGGL((stage_kernel<K, F, kMaxBatchFrames, kLong>), dim3(n_tiles * groups),
                     dim3(kThreads), 0, s, args);
  return hipGetLastError();
}

template <int K>
hipError_t launch_stage_k(const VolumeDev& vol, const WalkParams& wp, const FrameDev* frames, int n,
                          int frames_per_group, const StageDev& stg, hipStream_t s) {
  if (n < 1 || n > kMaxBatchFrames) return hipErrorInvalidValue;
  const bool lp = long_probe(vol);
  if (frames_per_group != 1 && frames_per_group != 2) return hipErrorInvalidValue;
  if constexpr (2 * K + 1 <= 9) {  // two frames' records of a tile fit LDS up to K = 4
    if (frames_per_group == 2)
      return lp ? launch_stage_kf<K, 2, true>(vol, wp, frames, n, stg, s)
                : launch_stage_kf<K, 2, false>(vol, wp, frames, n, stg, s);
  }
  return lp ? launch_stage_kf<K, 1, true>(vol, wp, frames, n, stg, s)
            : launch_stage_kf<K, 1, false>(vol, wp, frames, n, stg, s);
}

}  // namespace
}  // namespace tsdf
