// Internal declarations shared by the host half (tsdf_api.cpp) and the device
// half (tsdf_kernels.hip) of libtsdf.so.  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tsdf.h"

namespace tsdf {

// One hash-table slot (Section 2.1): 64-bit packed key, 32-bit pool index,
// 4 bytes of padding -> 16 bytes, read with one 128-bit load.
struct alignas(16) TableEntry {
  unsigned long long key;
  int block;
  unsigned pad;
};
static_assert(sizeof(TableEntry) == 16, "16-byte entries");

constexpr int kBlockPublishing = -1;  // key claimed, pool index not yet stored
constexpr int kBlockPoolFull = -2;    // key claimed, the pool had no block left
constexpr int kBlockTableFull = -3;   // (never stored) resolution failed: table full
constexpr unsigned long long kEmptyKey = ~0ull;

// Device counters.  The 512-byte header holds the allocation state and the loss
// counters on separate 128-byte lines; the per-frame traffic counters, which
// every wave adds to, are spread over kCounterShards lines' worth of slots so
// that no single address takes one atomic per wave of the whole grid.
constexpr unsigned kCounterShards = 256;
struct DevCounters {
  // line 0: allocation
  unsigned block_count;         // pool bump allocator (may run past the capacity)
  unsigned status_bits;         // sticky TSDF_FLAG_*
  unsigned keys_pool_overflow;
  unsigned table_full_events;
  unsigned max_probe;
  unsigned lookup_misses;
  unsigned mesh_triangles;      // surface extraction: triangles found
  unsigned keys_table_overflow; // distinct keys recorded in the overflow set
  unsigned pad0[24];
  // line 1: losses
  unsigned long long pairs_dropped;
  unsigned long long coord_out_of_range;
  unsigned long long pad1[14];
  // probe-histogram volumes: (tile, key) resolutions by probe distance, bin
  // 0 for distance 0 and bin b >= 1 for distances in [2^(b-1), 2^b), the last
  // bin open-ended
  unsigned long long probe_hist[TSDF_PROBE_HIST_BINS];
  unsigned long long probe_sum;  // and their summed probe distance
  unsigned long long pad2[31 - TSDF_PROBE_HIST_BINS];
  // sharded traffic counters (summed on the host)
  unsigned long long points_valid[kCounterShards];
  unsigned long long pairs[kCounterShards];
};
static_assert(sizeof(DevCounters) == 512 + 2 * 8 * kCounterShards, "counter layout");
constexpr size_t kCountersBytes = 8192;
static_assert(sizeof(DevCounters) <= kCountersBytes, "counters fit their region");

// Voxel pool layout: block b owns 1024 floats at b * kBlockFloats, as 64
// segments of 64 bytes.  A segment holds 8 voxels, 4 along x by 2 along z
// (segment (lx / 4, ly, lz / 2)), as their 8 TSDF sums then their 8 weights,
// so one memory-side atomic request carries both accumulators of 8 voxels.
// Device code numbers a block's voxels segment by segment (voxel_index);
// outputs use the canonical in-block order (lz * 8 + ly) * 8 + lx.  On the room
// orbit a tile's contributions touch about 10 % fewer such segments than
// x-rows of 8: the camera turns about the vertical axis, so the surfaces it
// sees extend along both x and z.  (Measured against x-rows: room orbit 3 %
// faster batched and 5 % one frame per launch; the multi-volume kernel 2-3 %
// slower.)
constexpr unsigned kBlockFloats = 1024;
__host__ __device__ constexpr unsigned voxel_index(unsigned lx, unsigned ly, unsigned lz) {
  // segment (sx, ly, sz) = (lx / 4, ly, lz / 2); phase 3 marks voxels in 64-bit
  // words of 8 segments (index / 64), keyed by (ly % 4, sz % 2) so that the
  // lanes of a wave, which touch neighbouring voxels, mark different words
  return ((((ly & 3u) * 2u + ((lz >> 1) & 1u)) * 8u + (lz >> 2) * 4u + (ly >> 2) * 2u +
           (lx >> 2))
          << 3) |
         ((lz & 1u) << 2) | (lx & 3u);
}
// The canonical in-block index of device voxel index v.
__host__ __device__ constexpr unsigned canonical_index(unsigned v) {
  return ((((v >> 6) & 1u) * 2u + (v >> 5 & 1u) * 4u + ((v >> 2) & 1u)) * 8u +
          (v >> 7) + ((v >> 4) & 1u) * 4u) *
             8u +
         ((v >> 3) & 1u) * 4u + (v & 3u);
}
__host__ __device__ constexpr unsigned pool_tsdf_index(unsigned v) {
  return (v >> 3) * 16u + (v & 7u);
}
__host__ __device__ constexpr unsigned pool_weight_index(unsigned v) {
  return (v >> 3) * 16u + 8u + (v & 7u);
}
static_assert(voxel_index(7, 7, 7) == 511 && canonical_index(voxel_index(5, 3, 6)) == (6 * 8 + 3) * 8 + 5 &&
                  canonical_index(voxel_index(2, 0, 1)) == 66 && voxel_index(4, 0, 0) == 8,
              "segment-major voxel numbering");

// Colour volumes: per block 64 segments of 24 floats (the segment's 8 red, 8
// green, 8 blue sums), in the same voxel numbering.
constexpr unsigned kColourFloats = 1536;
__host__ __device__ constexpr unsigned colour_index(unsigned v, unsigned channel) {
  return (v >> 3) * 24u + channel * 8u + (v & 7u);
}

struct VolumeDev {
  DevCounters* ctr;
  TableEntry* table;
  unsigned long long* overflow_keys;  // TSDF_OVERFLOW_KEY_SLOTS keys that found the table full
  unsigned long long* block_keys;  // key of the i-th allocated block
  float* voxels;                   // pool_capacity * kBlockFloats
  unsigned* alloc_list;            // slot-index volumes: pool index of the i-th allocated block
  float* colour;                   // colour volumes: pool_capacity * kColourFloats
  unsigned table_capacity;
  unsigned pool_capacity;
  unsigned slot_index;             // 1: a block's pool index is its table slot
  unsigned probe_hist;             // 1: count resolutions by probe distance
  unsigned pad[2];                 // keeps the struct a whole number of 16-byte units
};
static_assert(sizeof(VolumeDev) % 16 == 0, "volume descriptors stay 16-byte aligned");

// Pool index of the i-th allocated block.
__host__ __device__ inline unsigned allocated_block(const VolumeDev& vol, unsigned i) {
  return vol.slot_index ? vol.alloc_list[i] : i;
}

struct FrameDev {
  const float* depth;
  const unsigned* rgba;    // colour volumes: packed 8-bit red | green << 8 | blue << 16
  unsigned width, height;
  float cx, cy, ifx, ify;  // 1/fx, 1/fy rounded once to float32
  float R[9];              // camera->world rotation, row-major
  float t[3];
};

struct WalkParams {
  float v, iv, trunc;  // voxel edge, 1/v (float32), truncation
  int K;               // band half-width in samples
};

// Frames fused by one launch of tsdf_fuse_frames.
constexpr int kMaxBatchFrames = 32;

enum class FuseMode : int { kFused = 0, kAllocate = 1, kIntegrate = 2 };

// One item of a multi-volume batch: a frame and the volume it goes into, as
// the persistent kernel reads it from the device workspace.
struct BatchItem {
  VolumeDev vol;
  WalkParams wp;
  FrameDev fr;
  unsigned tiles_x;  // tiles per row of this frame for the launch's tile width
  unsigned pad;
};
static_assert(sizeof(BatchItem) % 16 == 0, "items stay 16-byte aligned");

// The work list of one batch launch, in the device workspace.  Items are
// sorted by group g = batch_group(K, colour) (band half-width K, colour or
// not); the items of g are k_begin[g] .. k_begin[g+1]-1 and their tiles are
// the global tile indices tile_start[first] .. tile_start[last]-1 (tile_start
// is the exclusive prefix sum of tile counts).
constexpr int kBatchGroups = 32;  // k_begin entries (groups 0 .. 19 used)
__host__ __device__ constexpr int batch_group(int K, bool colour) { return K + (colour ? 10 : 0); }
struct BatchWork {
  const unsigned* k_begin;
  const unsigned* tile_start;
  const BatchItem* items;
};

// Staged accumulation (tsdf_fuse_frames_staged).  The tiles of a launch do not
// add their contributions to the pool.  Each tile writes one record per
// contribution, grouped by block, into a launch-wide record array (one device
// atomic per tile reserves its span), and lists each of its (tile, block) runs
// in the block's run table (one device atomic per tile and block, which also
// counts the block's runs and records).  A block is cut into one work item per
// kStageItemRecords records; the apply kernel takes items from a queue, sums
// an item's share of the block's runs per voxel in LDS and adds the sums to
// the block's pool segments with device atomics, one request per touched
// segment.
//
// A record is one contribution in 32 bits: its voxel's in-block index (bits
// 0..8) and its truncated distance in signed 23-bit fixed point of the
// truncation distance (bits 9..31): q = round(sdf * kStageQuantum / trunc),
// |q| <= kStageQuantum, so sdf is carried to within trunc / 2^23 (2.4e-9 m at
// trunc = 2 cm).
constexpr int kStageQuantum = (1 << 22) - 1;
constexpr unsigned kStageRuns = 128;          // run table entries per block and launch
constexpr unsigned kStageItemRecords = 1024;  // records per apply work item
// One set of staging buffers (a launch uses one set; two sets alternate so
// that a launch's tile kernel may run while the previous launch is applied).
struct StageDev {
  unsigned* head;                  // [0] blocks listed, [1] records reserved, [2] items,
                                   // [3] items taken by the apply kernel
  unsigned long long* block_stat;  // per pool block: runs << 32 | records
  unsigned long long* runs;        // per pool block: kStageRuns (first record | count << 32)
  unsigned* items;                 // work items: (block, part)
  unsigned* recs;                  // the launch's records
  unsigned rec_cap;                // records the array holds
  unsigned item_cap;               // work items the list holds
  float to_fixed;                  // kStageQuantum / trunc
  float to_metres;                 // trunc / kStageQuantum
  unsigned pad[2];
};
static_assert(sizeof(StageDev) % 16 == 0, "stage descriptors stay 16-byte aligned");

hipError_t launch_fill_u32(void* ptr, unsigned value, size_t n_words, hipStream_t s);
hipError_t launch_reset_used(VolumeDev vol, hipStream_t s);
hipError_t launch_atomic_rate(float* p, unsigned n_rows, unsigned waves, unsigned iters,
                              unsigned rows, unsigned lanes, hipStream_t s);
// Fuse n_frames (1..kMaxBatchFrames) frames in one launch, frames_per_group of
// them summed per workgroup (1 to 4, at most max_frames_per_group(K)).
hipError_t launch_fuse(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n_frames,
                       int frames_per_group, FuseMode mode, bool xcd_remap, hipStream_t s);
int max_frames_per_group(int K);
// one per band half-width K, each in its own translation unit
hipError_t launch_fuse_band1(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band2(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band3(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band4(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band5(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band6(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band7(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
hipError_t launch_fuse_band8(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s);
// The tile kernel of staged accumulation: n frames (1..kMaxBatchFrames) of one
// volume in one launch, frames_per_group (1 or 2) of them per workgroup; then
// the apply kernel, which consumes the launch's work items.  A set's heads and
// block counts must be zero before its tile kernel runs.
hipError_t launch_stage(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                        int frames_per_group, const StageDev& stage, hipStream_t s);
hipError_t launch_stage_band1(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band2(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band3(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band4(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band5(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band6(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band7(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_band8(VolumeDev, const WalkParams&, const FrameDev*, int, int,
                              const StageDev&, hipStream_t);
hipError_t launch_stage_apply(VolumeDev vol, const StageDev& stage, hipStream_t s);
// The persistent multi-volume kernel for band half-width K taking
// pixels_per_thread (1 or 2) pixels per thread and accumulating acc_blocks
// (4 or 8; 8 with 2 pixels) blocks in LDS per pass, as a host
// function pointer for hipLaunchKernel / graph kernel nodes; nullptr for
// other values.  Colour volumes have one shape: 1 pixel, 4 blocks.  Its
// arguments are (BatchWork work, unsigned tile_width_log2).
const void* multi_kernel(int K, int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band1(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band2(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band3(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band4(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band5(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band6(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band7(int pixels_per_thread, int acc_blocks, bool colour);
const void* multi_kernel_band8(int pixels_per_thread, int acc_blocks, bool colour);
// out[i] = the sticky status bits of the volume whose counters ctrs[i] points
// to (0 for a null pointer), i < n.  ctrs and out may be host-mapped memory.
// The device address and size of the process-lifetime work-list array of
// tsdf_batch_fuse_static on the current device (looked up on first use).
hipError_t static_scratch(void** ptr, size_t* bytes);
hipError_t launch_gather_status(DevCounters* const* ctrs, unsigned n, unsigned* out, hipStream_t s);
// Marching-tetrahedra surface of the first n_blocks pool blocks; counter
// (zeroed by the caller) receives the triangle count; at most max_tris
// triangles are written (9 floats in verts, 2 ids in ids, ids may be null).
hipError_t launch_mesh(VolumeDev vol, const WalkParams& wp, unsigned n_blocks, unsigned* counter,
                       unsigned max_tris, float* verts, unsigned long long* ids, hipStream_t s);
hipError_t launch_insert_blocks(VolumeDev vol, const int* coords, unsigned n, hipStream_t s);
hipError_t launch_extract(VolumeDev vol, unsigned n_blocks, unsigned long long* keys,
                          float* tsdf, float* weight, hipStream_t s);
hipError_t launch_extract_colour(VolumeDev vol, unsigned n_blocks, float* rgb, hipStream_t s);

}  // namespace tsdf
