// Host half of libtsdf.so: argument checking, arena carving, launches and
// status read-back for the volume calls of the C ABI declared in
// include/tsdf.h (multi-volume batches are in tsdf_batch.cpp).
//
// Every entry point validates on the host and returns before enqueuing anything
// if an argument is wrong.  No entry point allocates device memory; the only
// host allocation is the volume handle.

#include <cstddef>
#include <cstdlib>
#include <mutex>

#include "tsdf_host.h"

namespace {

using namespace tsdf_host;

uint32_t next_pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p > 0xFFFFFFFFull ? 0u : (uint32_t)p;
}

// Fills `out` for valid params; returns false otherwise.
bool make_layout(const tsdf_volume_params* p, tsdf_layout* out) {
  if (!p) return false;
  if (!finite(p->voxel_size) || !(p->voxel_size > 0.0f)) return false;
  // Section 2.2: the band reaches at least one voxel either side of the surface
  if (!finite(p->trunc) || !(p->trunc >= p->voxel_size)) return false;
  const int K = band_half(*p);
  if (K < 1 || K > TSDF_MAX_BAND_HALF) return false;
  if (p->pool_capacity < 1 || p->pool_capacity > TSDF_MAX_POOL_BLOCKS) return false;
  if ((p->flags & ~(TSDF_VOLUME_SLOT_INDEX | TSDF_VOLUME_COLOUR | TSDF_VOLUME_PROBE_HISTOGRAM)) != 0)
    return false;
  const bool slot_index = (p->flags & TSDF_VOLUME_SLOT_INDEX) != 0;
  const bool colour = (p->flags & TSDF_VOLUME_COLOUR) != 0;
  uint32_t C = p->table_capacity;
  if (C == 0) C = slot_index ? p->pool_capacity : next_pow2_at_least(2ull * p->pool_capacity);
  if (C == 0) return false;
  if (slot_index && C != p->pool_capacity) return false;  // one block per slot
  const uint64_t P = p->pool_capacity;
  tsdf_layout L;
  std::memset(&L, 0, sizeof(L));
  uint64_t off = 0;
  L.counters = off;
  off = align_up(off + tsdf::kCountersBytes);
  L.table = off;
  off = align_up(off + (uint64_t)C * sizeof(tsdf::TableEntry));
  L.overflow_keys = off;
  off = align_up(off + (uint64_t)TSDF_OVERFLOW_KEY_SLOTS * 8ull);
  L.block_keys = off;
  off = align_up(off + P * 8ull);
  L.alloc_list = off;
  off = align_up(off + (slot_index ? P * 4ull : 0ull));
  L.voxels = off;
  off = align_up(off + P * tsdf::kBlockFloats * 4ull);
  L.colour = off;
  off = align_up(off + (colour ? P * tsdf::kColourFloats * 4ull : 0ull));
  L.total_bytes = off;
  L.table_capacity = C;
  L.pool_capacity = p->pool_capacity;
  L.flags = p->flags;
  *out = L;
  return true;
}

tsdf_status init_table_and_counters(tsdf_volume* v, hipStream_t s) {
  const tsdf_layout& L = v->layout;
  hipError_t e = tsdf::launch_fill_u32(v->dev.table, 0xFFFFFFFFu,
                                        (size_t)L.table_capacity * (sizeof(tsdf::TableEntry) / 4), s);
  if (e == hipSuccess)
    e = tsdf::launch_fill_u32(v->dev.overflow_keys, 0xFFFFFFFFu, TSDF_OVERFLOW_KEY_SLOTS * 2ull, s);
  if (e == hipSuccess) e = tsdf::launch_fill_u32(v->dev.ctr, 0u, tsdf::kCountersBytes / 4, s);
  return hip_status(e);
}

}  // namespace

extern "C" {

size_t tsdf_volume_bytes(const tsdf_volume_params* params) {
  tsdf_layout L;
  return make_layout(params, &L) ? (size_t)L.total_bytes : 0;
}

tsdf_status tsdf_volume_layout(const tsdf_volume_params* params, tsdf_layout* out) {
  if (!out) return TSDF_ERR_INVALID_ARGUMENT;
  return make_layout(params, out) ? TSDF_OK : TSDF_ERR_INVALID_ARGUMENT;
}

tsdf_status tsdf_create_volume(const tsdf_volume_params* params, void* dev_arena,
                               size_t arena_bytes, void* hip_stream, tsdf_volume** out) {
  if (!out) return TSDF_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  tsdf_layout L;
  if (!make_layout(params, &L)) return TSDF_ERR_INVALID_ARGUMENT;
  if (!dev_arena || ((uintptr_t)dev_arena % kAlign) != 0) return TSDF_ERR_INVALID_ARGUMENT;
  if (arena_bytes < L.total_bytes) return TSDF_ERR_BUFFER_TOO_SMALL;
  tsdf_volume* v = static_cast<tsdf_volume*>(std::malloc(sizeof(tsdf_volume)));
  if (!v) return TSDF_ERR_INTERNAL;
  v->params = *params;
  v->layout = L;
  v->frames = 0;
  v->blocks_seen = 0;
  char* base = static_cast<char*>(dev_arena);
  v->dev.ctr = reinterpret_cast<tsdf::DevCounters*>(base + L.counters);
  v->dev.table = reinterpret_cast<tsdf::TableEntry*>(base + L.table);
  v->dev.overflow_keys = reinterpret_cast<unsigned long long*>(base + L.overflow_keys);
  v->dev.pad[0] = v->dev.pad[1] = 0u;
  v->dev.block_keys = reinterpret_cast<unsigned long long*>(base + L.block_keys);
  v->dev.voxels = reinterpret_cast<float*>(base + L.voxels);
  const bool slot_index = (L.flags & TSDF_VOLUME_SLOT_INDEX) != 0;
  const bool colour = (L.flags & TSDF_VOLUME_COLOUR) != 0;
  v->dev.alloc_list = slot_index ? reinterpret_cast<unsigned*>(base + L.alloc_list) : nullptr;
  v->dev.colour = colour ? reinterpret_cast<float*>(base + L.colour) : nullptr;
  v->dev.table_capacity = L.table_capacity;
  v->dev.pool_capacity = L.pool_capacity;
  v->dev.slot_index = slot_index ? 1u : 0u;
  v->dev.probe_hist = (L.flags & TSDF_VOLUME_PROBE_HISTOGRAM) ? 1u : 0u;
  hipStream_t s = as_stream(hip_stream);
  tsdf_status st = init_table_and_counters(v, s);
  const size_t pool_words = (size_t)L.pool_capacity * tsdf::kBlockFloats;
  if (st == TSDF_OK) st = hip_status(tsdf::launch_fill_u32(v->dev.voxels, 0u, pool_words, s));
  if (st == TSDF_OK)
    st = hip_status(tsdf::launch_fill_u32(v->dev.block_keys, 0xFFFFFFFFu,
                                          (size_t)L.pool_capacity * 2, s));
  if (st == TSDF_OK && v->dev.colour)
    st = hip_status(tsdf::launch_fill_u32(v->dev.colour, 0u,
                                          (size_t)L.pool_capacity * tsdf::kColourFloats, s));
  if (st != TSDF_OK) {
    std::free(v);
    return st;
  }
  *out = v;
  return TSDF_OK;
}

tsdf_status tsdf_destroy_volume(tsdf_volume* vol) {
  if (!vol) return TSDF_ERR_INVALID_ARGUMENT;
  std::free(vol);
  return TSDF_OK;
}

tsdf_status tsdf_reset_volume(tsdf_volume* vol, void* hip_stream) {
  if (!vol) return TSDF_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(hip_stream);
  // the used-block clear reads the bump counter, so it runs before the counters
  // are zeroed (same stream, in order)
  tsdf_status st = hip_status(tsdf::launch_reset_used(vol->dev, s));
  if (st == TSDF_OK) st = init_table_and_counters(vol, s);
  if (st == TSDF_OK) {
    vol->frames = 0;
    vol->blocks_seen = 0;
  }
  return st;
}

namespace {

tsdf_status fuse_one(tsdf_volume* vol, const float* depth_dev, const uint32_t* rgba_dev,
                     const tsdf_camera* cam, uint32_t flags, void* hip_stream) {
  if (!vol || !valid_camera(cam)) return TSDF_ERR_INVALID_ARGUMENT;
  if ((flags & ~(TSDF_FUSE_MODE_MASK | TSDF_FUSE_XCD_REMAP)) != 0)
    return TSDF_ERR_INVALID_ARGUMENT;
  const uint64_t n_pix = (uint64_t)cam->width * cam->height;
  if (n_pix > 0 && !depth_dev) return TSDF_ERR_INVALID_ARGUMENT;
  if (n_pix > 0 && vol->dev.colour && !rgba_dev) return TSDF_ERR_INVALID_ARGUMENT;
  const tsdf::FrameDev f = frame_dev(depth_dev, cam, vol->dev.colour ? rgba_dev : nullptr);
  const tsdf::WalkParams wp = walk_params(vol);
  const bool remap = (flags & TSDF_FUSE_XCD_REMAP) != 0;
  hipStream_t s = as_stream(hip_stream);
  hipError_t e = hipSuccess;
  if (n_pix > 0) {
    switch (flags & TSDF_FUSE_MODE_MASK) {
      case TSDF_FUSE_DEFAULT:
        e = tsdf::launch_fuse(vol->dev, wp, &f, 1, 1, tsdf::FuseMode::kFused, remap, s);
        break;
      case TSDF_FUSE_TWO_PASS:
        e = tsdf::launch_fuse(vol->dev, wp, &f, 1, 1, tsdf::FuseMode::kAllocate, remap, s);
        if (e == hipSuccess)
          e = tsdf::launch_fuse(vol->dev, wp, &f, 1, 1, tsdf::FuseMode::kIntegrate, remap, s);
        break;
      case TSDF_FUSE_ALLOCATE_ONLY:
        e = tsdf::launch_fuse(vol->dev, wp, &f, 1, 1, tsdf::FuseMode::kAllocate, remap, s);
        break;
      case TSDF_FUSE_INTEGRATE_ONLY:
        e = tsdf::launch_fuse(vol->dev, wp, &f, 1, 1, tsdf::FuseMode::kIntegrate, remap, s);
        break;
    }
  }
  if (e != hipSuccess) return TSDF_ERR_HIP;
  if ((flags & TSDF_FUSE_MODE_MASK) != TSDF_FUSE_ALLOCATE_ONLY) vol->frames++;
  return TSDF_OK;
}

}  // namespace

tsdf_status tsdf_fuse_frame_ex(tsdf_volume* vol, const float* depth_dev, const tsdf_camera* cam,
                               uint32_t flags, void* hip_stream) {
  if (vol && vol->dev.colour) return TSDF_ERR_INVALID_ARGUMENT;  // colour needs an image
  return fuse_one(vol, depth_dev, nullptr, cam, flags, hip_stream);
}

tsdf_status tsdf_fuse_frame_rgb(tsdf_volume* vol, const float* depth_dev, const uint32_t* rgba_dev,
                                const tsdf_camera* cam, uint32_t flags, void* hip_stream) {
  if (vol && !vol->dev.colour) return TSDF_ERR_INVALID_ARGUMENT;
  return fuse_one(vol, depth_dev, rgba_dev, cam, flags, hip_stream);
}

namespace {

// Several frames of one volume, up to kMaxBatchFrames per launch; rgba_devs is
// null for plain volumes and required (per frame with pixels) for colour ones.
tsdf_status fuse_frames_impl(tsdf_volume* vol, uint32_t n_frames, const float* const* depth_devs,
                             const uint32_t* const* rgba_devs, const tsdf_camera* cams,
                             uint32_t flags, void* hip_stream) {
  if (n_frames > 0 && (!depth_devs || !cams)) return TSDF_ERR_INVALID_ARGUMENT;
  if ((flags & ~(TSDF_FUSE_XCD_REMAP | TSDF_FUSE_BATCH_MASK)) != 0) return TSDF_ERR_INVALID_ARGUMENT;
  const bool colour = vol->dev.colour != nullptr;
  if (colour && n_frames > 0 && !rgba_devs) return TSDF_ERR_INVALID_ARGUMENT;
  for (uint32_t i = 0; i < n_frames; ++i) {
    if (!valid_camera(&cams[i])) return TSDF_ERR_INVALID_ARGUMENT;
    if ((uint64_t)cams[i].width * cams[i].height > 0 &&
        (!depth_devs[i] || (colour && !rgba_devs[i])))
      return TSDF_ERR_INVALID_ARGUMENT;
  }
  const tsdf::WalkParams wp = walk_params(vol);
  // frames summed per workgroup: the TSDF_FUSE_BATCH(m) request, at most 4 (3
  // when m = 0, the measured best), capped for wide bands and, for colour
  // volumes, at 2
  const uint32_t asked = (flags & TSDF_FUSE_BATCH_MASK) >> TSDF_FUSE_BATCH_SHIFT;
  int per_group = asked == 0 ? 3 : asked >= 4 ? 4 : (int)asked;
  const int cap = colour ? 2 : tsdf::max_frames_per_group(wp.K);
  if (per_group > cap) per_group = cap;
  const bool remap = (flags & TSDF_FUSE_XCD_REMAP) != 0;
  hipStream_t s = as_stream(hip_stream);
  tsdf::FrameDev batch[tsdf::kMaxBatchFrames];
  uint32_t done = 0;
  while (done < n_frames) {
    const uint32_t left = n_frames - done;
    const int n = left < (uint32_t)tsdf::kMaxBatchFrames ? (int)left : tsdf::kMaxBatchFrames;
    uint64_t pix = 0;
    for (int i = 0; i < n; ++i) {
      batch[i] = frame_dev(depth_devs[done + i], &cams[done + i],
                           colour ? rgba_devs[done + i] : nullptr);
      pix += (uint64_t)cams[done + i].width * cams[done + i].height;
    }
    if (pix > 0 && tsdf::launch_fuse(vol->dev, wp, batch, n, n > 1 ? per_group : 1,
                                     tsdf::FuseMode::kFused, remap, s) != hipSuccess)
      return TSDF_ERR_HIP;
    done += (uint32_t)n;
    vol->frames += (uint32_t)n;
  }
  return TSDF_OK;
}

}  // namespace

namespace {

// Staging memory of tsdf_fuse_frames_staged: two sets, used by alternate
// launches.  A set: four list heads in a 256-byte header, per pool block its
// run and record counts (8 bytes) and a run table of kStageRuns 8-byte entries,
// the work items (8 bytes each), then the records (4 bytes each).
struct StageLayout {
  uint64_t block_stat, runs, items, recs, set_bytes;
  uint64_t item_cap;
};
StageLayout stage_layout(uint64_t pool, uint64_t records) {
  StageLayout L;
  L.item_cap = records / tsdf::kStageItemRecords + pool + 1;  // enough for any launch
  L.block_stat = kAlign;
  L.runs = align_up(L.block_stat + 8 * pool);
  L.items = align_up(L.runs + 8ull * tsdf::kStageRuns * pool);
  L.recs = align_up(L.items + 8 * L.item_cap);
  L.set_bytes = align_up(L.recs + 4 * records);
  return L;
}
constexpr uint64_t kMinStageRecords = 1ull << 16;
constexpr uint64_t kMaxStageRecords = 0xFFFFFFFFull;

// The apply kernels of a call run on a second stream of the device, ordered
// against the caller's stream by events; the stream and events are made on
// first use and kept for the life of the process.  A call enqueues its whole
// sequence holding the device's lock.
constexpr int kMaxStageDevices = 64;
struct StageStreams {
  hipStream_t aux = nullptr;
  hipEvent_t tile_done[2] = {nullptr, nullptr};
  hipEvent_t apply_done[2] = {nullptr, nullptr};
};
std::mutex g_stage_mu;
StageStreams g_stage[kMaxStageDevices];

hipError_t stage_streams(StageStreams** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxStageDevices) return hipErrorInvalidDevice;
  StageStreams& ss = g_stage[dev];
  if (!ss.aux) {
    hipStream_t aux = nullptr;
    e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&ss.tile_done[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.apply_done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) return e;
    ss.aux = aux;
  }
  *out = &ss;
  return hipSuccess;
}

}  // namespace

size_t tsdf_staging_bytes(uint32_t pool_capacity, uint64_t records) {
  if (pool_capacity < 1 || pool_capacity > TSDF_MAX_POOL_BLOCKS) return 0;
  if (records < kMinStageRecords || records > kMaxStageRecords) return 0;
  return (size_t)(2 * stage_layout(pool_capacity, records).set_bytes);
}

tsdf_status tsdf_fuse_frames_staged(tsdf_volume* vol, uint32_t n_frames,
                                    const float* const* depth_devs, const tsdf_camera* cams,
                                    uint32_t flags, void* staging_dev, size_t staging_bytes,
                                    void* hip_stream) {
  if (!vol || vol->dev.colour) return TSDF_ERR_INVALID_ARGUMENT;
  if (n_frames > 0 && (!depth_devs || !cams)) return TSDF_ERR_INVALID_ARGUMENT;
  if ((flags & ~(TSDF_FUSE_BATCH_MASK | TSDF_FUSE_ONE_STREAM)) != 0)
    return TSDF_ERR_INVALID_ARGUMENT;
  for (uint32_t i = 0; i < n_frames; ++i) {
    if (!valid_camera(&cams[i])) return TSDF_ERR_INVALID_ARGUMENT;
    if ((uint64_t)cams[i].width * cams[i].height > 0 && !depth_devs[i])
      return TSDF_ERR_INVALID_ARGUMENT;
  }
  if (!staging_dev || ((uintptr_t)staging_dev % kAlign) != 0) return TSDF_ERR_INVALID_ARGUMENT;
  const uint64_t P = vol->layout.pool_capacity;
  if (staging_bytes < tsdf_staging_bytes((uint32_t)P, kMinStageRecords))
    return TSDF_ERR_BUFFER_TOO_SMALL;
  // the most records whose two sets fit
  uint64_t lo = kMinStageRecords, hi = kMaxStageRecords;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (2 * stage_layout(P, mid).set_bytes <= staging_bytes) lo = mid;
    else hi = mid - 1;
  }
  const StageLayout L = stage_layout(P, lo);
  // frames per workgroup: TSDF_FUSE_BATCH(1) -> 1, anything else -> 2
  const uint32_t asked = (flags & TSDF_FUSE_BATCH_MASK) >> TSDF_FUSE_BATCH_SHIFT;
  const int per_group = asked == 1 ? 1 : 2;
  const tsdf::WalkParams wp = walk_params(vol);
  hipStream_t s = as_stream(hip_stream);
  tsdf::StageDev set[2];
  for (int k = 0; k < 2; ++k) {
    char* base = static_cast<char*>(staging_dev) + k * L.set_bytes;
    std::memset(&set[k], 0, sizeof(set[k]));
    set[k].head = reinterpret_cast<unsigned*>(base);
    set[k].block_stat = reinterpret_cast<unsigned long long*>(base + L.block_stat);
    set[k].runs = reinterpret_cast<unsigned long long*>(base + L.runs);
    set[k].items = reinterpret_cast<unsigned*>(base + L.items);
    set[k].recs = reinterpret_cast<unsigned*>(base + L.recs);
    set[k].rec_cap = (unsigned)lo;
    set[k].item_cap = (unsigned)L.item_cap;
    set[k].to_fixed = (float)tsdf::kStageQuantum / wp.trunc;
    set[k].to_metres = wp.trunc / (float)tsdf::kStageQuantum;
  }
  const bool one_stream = (flags & TSDF_FUSE_ONE_STREAM) != 0;
  std::lock_guard<std::mutex> lock(g_stage_mu);
  StageStreams* ss = nullptr;
  if (!one_stream && stage_streams(&ss) != hipSuccess) return TSDF_ERR_HIP;
  hipStream_t aux = one_stream ? s : ss->aux;
  tsdf::FrameDev batch[tsdf::kMaxBatchFrames];
  uint32_t done = 0, launch = 0;
  hipError_t e = hipSuccess;
  while (done < n_frames && e == hipSuccess) {
    const uint32_t left = n_frames - done;
    const int n = left < (uint32_t)tsdf::kMaxBatchFrames ? (int)left : tsdf::kMaxBatchFrames;
    uint64_t pix = 0;
    for (int i = 0; i < n; ++i) {
      batch[i] = frame_dev(depth_devs[done + i], &cams[done + i]);
      pix += (uint64_t)cams[done + i].width * cams[done + i].height;
    }
    if (pix > 0) {
      const int k = (int)(launch & 1u);
      // the set is free once the launch two back has been applied; its heads
      // and block counts start at zero
      if (!one_stream && launch >= 2) e = hipStreamWaitEvent(s, ss->apply_done[k], 0);
      if (e == hipSuccess) e = tsdf::launch_fill_u32(set[k].head, 0u, L.runs / 4, s);
      if (e == hipSuccess) e = tsdf::launch_stage(vol->dev, wp, batch, n, per_group, set[k], s);
      if (!one_stream) {
        if (e == hipSuccess) e = hipEventRecord(ss->tile_done[k], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux, ss->tile_done[k], 0);
      }
      if (e == hipSuccess) e = tsdf::launch_stage_apply(vol->dev, set[k], aux);
      if (!one_stream && e == hipSuccess) e = hipEventRecord(ss->apply_done[k], aux);
      ++launch;
    }
    done += (uint32_t)n;
    vol->frames += (uint32_t)n;
  }
  // the caller's stream resumes after every apply of the call
  for (uint32_t k = 0; !one_stream && k < 2 && k < launch && e == hipSuccess; ++k)
    e = hipStreamWaitEvent(s, ss->apply_done[k], 0);
  return e == hipSuccess ? TSDF_OK : TSDF_ERR_HIP;
}

tsdf_status tsdf_fuse_frames(tsdf_volume* vol, uint32_t n_frames, const float* const* depth_devs,
                             const tsdf_camera* cams, uint32_t flags, void* hip_stream) {
  if (!vol) return TSDF_ERR_INVALID_ARGUMENT;
  if (vol->dev.colour) return TSDF_ERR_INVALID_ARGUMENT;  // colour frames: _rgb or batches
  return fuse_frames_impl(vol, n_frames, depth_devs, nullptr, cams, flags, hip_stream);
}

tsdf_status tsdf_fuse_frames_rgb(tsdf_volume* vol, uint32_t n_frames,
                                 const float* const* depth_devs,
                                 const uint32_t* const* rgba_devs, const tsdf_camera* cams,
                                 uint32_t flags, void* hip_stream) {
  if (!vol || !vol->dev.colour) return TSDF_ERR_INVALID_ARGUMENT;
  return fuse_frames_impl(vol, n_frames, depth_devs, rgba_devs, cams, flags, hip_stream);
}

tsdf_status tsdf_fuse_frame(tsdf_volume* vol, const float* depth_dev, const tsdf_camera* cam,
                            void* hip_stream) {
  return tsdf_fuse_frame_ex(vol, depth_dev, cam, TSDF_FUSE_DEFAULT, hip_stream);
}

tsdf_status tsdf_query_status(tsdf_volume* vol, void* hip_stream, tsdf_stats* out) {
  if (!vol) return TSDF_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(hip_stream);
  tsdf::DevCounters c;
  if (hipMemcpyAsync(&c, vol->dev.ctr, sizeof(c), hipMemcpyDeviceToHost, s) != hipSuccess)
    return TSDF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TSDF_ERR_HIP;
  uint32_t bits = c.status_bits;
  if (c.coord_out_of_range) bits |= TSDF_FLAG_COORD_RANGE;
  if (out) {
    std::memset(out, 0, sizeof(*out));
    for (unsigned i = 0; i < tsdf::kCounterShards; ++i) {
      out->points_valid += c.points_valid[i];
      out->pairs += c.pairs[i];
    }
    out->pairs_dropped = c.pairs_dropped;
    out->coord_out_of_range = c.coord_out_of_range;
    out->blocks_total = c.block_count < vol->layout.pool_capacity ? c.block_count
                                                                  : vol->layout.pool_capacity;
    out->blocks_new = out->blocks_total - vol->blocks_seen;
    vol->blocks_seen = out->blocks_total;
    out->keys_pool_overflow = c.keys_pool_overflow;
    out->keys_table_overflow = c.keys_table_overflow;
    out->table_full_events = c.table_full_events;
    out->max_probe = c.max_probe;
    out->lookup_misses = c.lookup_misses;
    out->status_bits = bits;
    out->frames = vol->frames;
  }
  if (bits & TSDF_FLAG_INTERNAL) return TSDF_ERR_INTERNAL;
  if (bits & TSDF_FLAG_TABLE_FULL) return TSDF_ERR_TABLE_FULL;
  if (bits & TSDF_FLAG_POOL_EXHAUSTED) return TSDF_ERR_POOL_EXHAUSTED;
  if (bits & TSDF_FLAG_COORD_RANGE) return TSDF_ERR_COORD_RANGE;
  return TSDF_OK;
}

tsdf_status tsdf_probe_histogram(tsdf_volume* vol, void* hip_stream, uint64_t* bins,
                                 uint64_t* total_distance) {
  if (!vol || !bins || !vol->dev.probe_hist) return TSDF_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(hip_stream);
  unsigned long long h[TSDF_PROBE_HIST_BINS + 1];  // the bins, then the sum
  static_assert(offsetof(tsdf::DevCounters, probe_sum) ==
                    offsetof(tsdf::DevCounters, probe_hist) + 8 * TSDF_PROBE_HIST_BINS,
                "the sum follows the bins");
  if (hipMemcpyAsync(h, vol->dev.ctr->probe_hist, sizeof(h), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return TSDF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TSDF_ERR_HIP;
  for (unsigned i = 0; i < TSDF_PROBE_HIST_BINS; ++i) bins[i] = h[i];
  if (total_distance) *total_distance = h[TSDF_PROBE_HIST_BINS];
  return TSDF_OK;
}

tsdf_status tsdf_measure_atomic_rate(float* buf_dev, uint64_t bytes, uint32_t waves,
                                     uint32_t iters, uint32_t rows_per_instr,
                                     uint32_t lanes_per_row, void* hip_stream) {
  if (!buf_dev || bytes < 64 || bytes % 64 != 0 || bytes / 64 > 0xFFFFFFFFull) return TSDF_ERR_INVALID_ARGUMENT;
  if (waves == 0 || waves % 4 != 0 || waves > (1u << 24) || iters == 0 || iters > (1u << 16))
    return TSDF_ERR_INVALID_ARGUMENT;
  if (lanes_per_row < 1 || lanes_per_row > 16 || rows_per_instr < 1 ||
      rows_per_instr * lanes_per_row > 64)
    return TSDF_ERR_INVALID_ARGUMENT;
  return hip_status(tsdf::launch_atomic_rate(buf_dev, (unsigned)(bytes / 64), waves, iters,
                                             rows_per_instr, lanes_per_row,
                                             as_stream(hip_stream)));
}

tsdf_status tsdf_extract_blocks(tsdf_volume* vol, void* hip_stream, uint32_t max_blocks,
                                uint64_t* keys_dev, float* tsdf_dev, float* weight_dev,
                                uint32_t* n_blocks_out) {
  if (!vol || !n_blocks_out) return TSDF_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(hip_stream);
  unsigned count = 0;
  if (hipMemcpyAsync(&count, &vol->dev.ctr->block_count, sizeof(count), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return TSDF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TSDF_ERR_HIP;
  const uint32_t n = count < vol->layout.pool_capacity ? count : vol->layout.pool_capacity;
  *n_blocks_out = n;
  if (n > max_blocks) return TSDF_ERR_BUFFER_TOO_SMALL;
  return hip_status(tsdf::launch_extract(vol->dev, n, reinterpret_cast<unsigned long long*>(keys_dev),
                                         tsdf_dev, weight_dev, s));
}

tsdf_status tsdf_extract_colour(tsdf_volume* vol, void* hip_stream, uint32_t max_blocks,
                                float* rgb_dev, uint32_t* n_blocks_out) {
  if (!vol || !n_blocks_out || !vol->dev.colour) return TSDF_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(hip_stream);
  unsigned count = 0;
  if (hipMemcpyAsync(&count, &vol->dev.ctr->block_count, sizeof(count), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return TSDF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TSDF_ERR_HIP;
  const uint32_t n = count < vol->layout.pool_capacity ? count : vol->layout.pool_capacity;
  *n_blocks_out = n;
  if (n > max_blocks) return TSDF_ERR_BUFFER_TOO_SMALL;
  if (n > 0 && !rgb_dev) return TSDF_ERR_INVALID_ARGUMENT;
  return hip_status(tsdf::launch_extract_colour(vol->dev, n, rgb_dev, s));
}

tsdf_status tsdf_extract_mesh(tsdf_volume* vol, void* hip_stream, uint32_t max_triangles,
                              float* vertices_dev, uint64_t* ids_dev, uint32_t* n_triangles_out) {
  if (!vol || !n_triangles_out || (max_triangles > 0 && !vertices_dev))
    return TSDF_ERR_INVALID_ARGUMENT;
  hipStream_t s = as_stream(hip_stream);
  unsigned count = 0;
  if (hipMemcpyAsync(&count, &vol->dev.ctr->block_count, sizeof(count), hipMemcpyDeviceToHost,
                     s) != hipSuccess)
    return TSDF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TSDF_ERR_HIP;
  const uint32_t n_blocks = count < vol->layout.pool_capacity ? count : vol->layout.pool_capacity;
  unsigned* counter = &vol->dev.ctr->mesh_triangles;
  hipError_t e = tsdf::launch_fill_u32(counter, 0u, 1, s);
  if (e == hipSuccess)
    e = tsdf::launch_mesh(vol->dev, walk_params(vol), n_blocks, counter, max_triangles,
                          vertices_dev, reinterpret_cast<unsigned long long*>(ids_dev), s);
  unsigned tris = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&tris, counter, sizeof(tris), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return TSDF_ERR_HIP;
  *n_triangles_out = tris;
  return tris > max_triangles ? TSDF_ERR_BUFFER_TOO_SMALL : TSDF_OK;
}

tsdf_status tsdf_insert_blocks(tsdf_volume* vol, const int32_t* block_coords_dev, uint32_t n,
                               void* hip_stream) {
  if (!vol || (n > 0 && !block_coords_dev)) return TSDF_ERR_INVALID_ARGUMENT;
  return hip_status(tsdf::launch_insert_blocks(vol->dev, block_coords_dev, n, as_stream(hip_stream)));
}

const char* tsdf_status_str(tsdf_status status) {
  switch (status) {
    case TSDF_OK: return "ok";
    case TSDF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case TSDF_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case TSDF_ERR_POOL_EXHAUSTED: return "voxel pool exhausted";
    case TSDF_ERR_TABLE_FULL: return "hash table full";
    case TSDF_ERR_COORD_RANGE: return "voxel coordinate outside the key range";
    case TSDF_ERR_INTERNAL: return "internal invariant violated";
    case TSDF_ERR_HIP: return "HIP runtime error";
    case TSDF_ERR_BUDGET: return "no room in the region, queue or session table";
    case TSDF_STATUS_RANGE_: break;
  }
  return "unknown status";
}

}  // extern "C"
