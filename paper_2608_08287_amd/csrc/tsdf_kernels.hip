// Device half of libtsdf.so, part 1: the small kernels (table insert of given
// blocks, fills, reset of used blocks, extraction) and the dispatch of the fused
// kernel to its per-K translation units.

#include <mutex>

#include "tsdf_device.h"

namespace tsdf {
namespace {

__global__ __launch_bounds__(256) void insert_blocks_kernel(VolumeDev vol, const int* coords,
                                                            unsigned n) {
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  bool act = i < n;
  int bx = 0, by = 0, bz = 0;
  if (act) {
    bx = coords[3 * (size_t)i];
    by = coords[3 * (size_t)i + 1];
    bz = coords[3 * (size_t)i + 2];
  }
  const bool in_range = bx >= -(1 << 20) && bx < (1 << 20) && by >= -(1 << 20) &&
                        by < (1 << 20) && bz >= -(1 << 20) && bz < (1 << 20);
  if (act && !in_range) add_u64(&vol.ctr->coord_out_of_range, 1ull);
  act = act && in_range;
  unsigned probes = 0;
  bool missing = false;
  resolve_key<true>(vol, pack_key(bx, by, bz), act, probes, missing);
  if (act && probes > *(volatile unsigned*)&vol.ctr->max_probe)
    __hip_atomic_fetch_max(&vol.ctr->max_probe, probes, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned* p, unsigned value, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256u;
  const size_t n4 = n / 4;
  uint4* p4 = reinterpret_cast<uint4*>(p);
  const uint4 v4 = make_uint4(value, value, value, value);
  for (size_t i = blockIdx.x * 256u + threadIdx.x; i < n4; i += stride) p4[i] = v4;
  for (size_t i = n4 * 4 + blockIdx.x * 256u + threadIdx.x; i < n; i += stride) p[i] = value;
}

// Zero the pool blocks handed out since the last reset (the others are zero),
// and their colour sums.
__global__ __launch_bounds__(256) void reset_used_kernel(VolumeDev vol) {
  unsigned used = *(volatile unsigned*)&vol.ctr->block_count;
  used = used < vol.pool_capacity ? used : vol.pool_capacity;
  constexpr unsigned kQuads = kBlockFloats / 4, kColourQuads = kColourFloats / 4;
  const size_t stride = (size_t)gridDim.x * 256u;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  float4* v4 = reinterpret_cast<float4*>(vol.voxels);
  for (size_t i = blockIdx.x * 256u + threadIdx.x; i < (size_t)used * kQuads; i += stride)
    v4[(size_t)allocated_block(vol, (unsigned)(i / kQuads)) * kQuads + i % kQuads] = z;
  if (vol.colour) {
    float4* c4 = reinterpret_cast<float4*>(vol.colour);
    for (size_t i = blockIdx.x * 256u + threadIdx.x; i < (size_t)used * kColourQuads; i += stride)
      c4[(size_t)allocated_block(vol, (unsigned)(i / kColourQuads)) * kColourQuads +
         i % kColourQuads] = z;
  }
}

// One thread per pool segment of 8 voxels (4 along x by 2 along z): read its
// 64 bytes, write the 8 means and 8 weights at their canonical places, two runs
// of 4 consecutive x in flat (lz * 8 + ly) * 8 + lx order.
__global__ __launch_bounds__(256) void extract_kernel(VolumeDev vol, unsigned n_blocks,
                                                      unsigned long long* keys, float* tsdf,
                                                      float* weight) {
  const size_t n_segs = (size_t)n_blocks * (TSDF_BLOCK_VOXELS / 8);
  const size_t stride = (size_t)gridDim.x * 256u;
  const float4* v4 = reinterpret_cast<const float4*>(vol.voxels);
  for (size_t r = blockIdx.x * 256u + threadIdx.x; r < n_segs; r += stride) {
    const size_t src = (size_t)allocated_block(vol, (unsigned)(r / 64)) * 64 + r % 64;
    // float4 q of the segment: sums of (lz even, odd), then weights of the same
    const float4 s0 = v4[4 * src], s1 = v4[4 * src + 1], w0 = v4[4 * src + 2],
                 w1 = v4[4 * src + 3];
    // canonical index of the segment's first voxel (lz even); lz odd is 64 on
    const size_t base = (r / 64) * TSDF_BLOCK_VOXELS + canonical_index((unsigned)(r % 64) * 8u);
    if (tsdf) {
      float4 m0, m1;
      m0.x = w0.x > 0.f ? s0.x / w0.x : 0.f;
      m0.y = w0.y > 0.f ? s0.y / w0.y : 0.f;
      m0.z = w0.z > 0.f ? s0.z / w0.z : 0.f;
      m0.w = w0.w > 0.f ? s0.w / w0.w : 0.f;
      m1.x = w1.x > 0.f ? s1.x / w1.x : 0.f;
      m1.y = w1.y > 0.f ? s1.y / w1.y : 0.f;
      m1.z = w1.z > 0.f ? s1.z / w1.z : 0.f;
      m1.w = w1.w > 0.f ? s1.w / w1.w : 0.f;
      reinterpret_cast<float4*>(tsdf + base)[0] = m0;
      reinterpret_cast<float4*>(tsdf + base + 64)[0] = m1;
    }
    if (weight) {
      reinterpret_cast<float4*>(weight + base)[0] = w0;
      reinterpret_cast<float4*>(weight + base + 64)[0] = w1;
    }
  }
  if (keys)
    for (size_t i = blockIdx.x * 256u + threadIdx.x; i < n_blocks; i += stride)
      keys[i] = vol.block_keys[i];
}

// One thread per voxel: its mean colour = colour sums / weight, 3 floats.
__global__ __launch_bounds__(256) void extract_colour_kernel(VolumeDev vol, unsigned n_blocks,
                                                             float* rgb) {
  const size_t n = (size_t)n_blocks * TSDF_BLOCK_VOXELS;
  const size_t stride = (size_t)gridDim.x * 256u;
  for (size_t v = blockIdx.x * 256u + threadIdx.x; v < n; v += stride) {
    const unsigned c = (unsigned)(v % TSDF_BLOCK_VOXELS);  // canonical in-block index
    const unsigned loc = voxel_index(c & 7u, (c >> 3) & 7u, c >> 6);
    const size_t blk = allocated_block(vol, (unsigned)(v / TSDF_BLOCK_VOXELS));
    const float w = vol.voxels[blk * kBlockFloats + pool_weight_index(loc)];
    const float* cp = vol.colour + blk * kColourFloats;
#pragma unroll
    for (unsigned c = 0; c < 3; ++c)
      rgb[v * 3 + c] = w > 0.f ? cp[colour_index(loc, c)] / w : 0.f;
  }
}

unsigned grid_for(size_t work, unsigned cap) {
  const size_t g = (work + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_fill_u32(void* ptr, unsigned value, size_t n_words, hipStream_t s) {
  if (n_words == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n_words / 4 + 1, 8192)), dim3(256), 0, s,
                     static_cast<unsigned*>(ptr), value, n_words);
  return hipGetLastError();
}

// Measurement: device-scope fp32 atomic adds in the pattern of the fused
// kernels' flush.  Each wave instruction adds 1.0 to `lanes` consecutive
// floats at the start of each of `rows` 64-byte rows, the rows picked by a
// per-wave linear congruential sequence among the buffer's n_rows rows.
__global__ __launch_bounds__(256) void atomic_rate_kernel(float* p, unsigned n_rows, unsigned iters,
                                                          unsigned rows, unsigned lanes) {
  const unsigned gid = blockIdx.x * 256u + threadIdx.x;
  const unsigned wave = gid >> 6, lane = gid & 63u;
  const unsigned r = lane / lanes, e = lane % lanes;
  const bool act = r < rows;
  unsigned long long h = (unsigned long long)(wave + 1u) * 0x9E3779B97F4A7C15ull;
  for (unsigned it = 0; it < iters; ++it) {
    h = h * 6364136223846793005ull + 1442695040888963407ull;
    // row r of this instruction: the sequence's value plus r golden-ratio steps
    const unsigned long long hr = (h >> 16) + (unsigned long long)r * 0x9E3779B9ull;
    const unsigned row = (unsigned)(hr % n_rows);
    if (act) add_f32(p + (size_t)row * 16u + e, 1.0f);
  }
}

hipError_t launch_atomic_rate(float* p, unsigned n_rows, unsigned waves, unsigned iters,
                              unsigned rows, unsigned lanes, hipStream_t s) {
  hipLaunchKernelGGL(atomic_rate_kernel, dim3(waves / 4u), dim3(256), 0, s, p, n_rows, iters, rows,
                     lanes);
  return hipGetLastError();
}

hipError_t launch_reset_used(VolumeDev vol, hipStream_t s) {
  hipLaunchKernelGGL(reset_used_kernel,
                     dim3(grid_for((size_t)vol.pool_capacity * (kBlockFloats / 4), 8192)),
                     dim3(256), 0, s, vol);
  return hipGetLastError();
}

// Staged accumulation, the apply kernels.  A block's records are its runs (one
// per tile that touched it), each a contiguous span of the launch's record
// array; its run table lists them.
//
// Sum a block's runs r = part, part + step, ... into a wave's LDS sums and
// counts (512 of each, zeroed here).  The run descriptors are read by the
// lanes together; then the runs are taken four at a time, each run's records
// by consecutive lanes, with the four runs' loads issued before any is added
// (four memory latencies overlapped, not four in a row).
__device__ void stage_sum_runs(const StageDev& stg, unsigned blk, unsigned n_runs, unsigned part,
                               unsigned step, float* sum, unsigned* cnt) {
  const unsigned lane = lane_id();
#pragma unroll
  for (unsigned i = 0; i < TSDF_BLOCK_VOXELS / (4u * kWave); ++i) {
    reinterpret_cast<float4*>(sum)[lane + i * kWave] = make_float4(0.f, 0.f, 0.f, 0.f);
    reinterpret_cast<uint4*>(cnt)[lane + i * kWave] = make_uint4(0u, 0u, 0u, 0u);
  }
  const unsigned long long* const runs = stg.runs + (size_t)blk * kStageRuns;
  constexpr unsigned kAhead = 4;
  for (unsigned r0 = part; r0 < n_runs; r0 += step * kWave) {
    const unsigned rr = r0 + lane * step;
    const unsigned long long mine = rr < n_runs ? runs[rr] : 0ull;
    const unsigned here = (n_runs - r0 + step - 1) / step;  // runs of this round
    for (unsigned k = 0; k < kWave && k < here; k += kAhead) {
      unsigned first[kAhead], count[kAhead], longest = 0;
#pragma unroll
      for (unsigned j = 0; j < kAhead; ++j) {
        const int src = (int)(k + j < here ? k + j : k);
        first[j] = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)mine, src);
        count[j] = k + j < here
                       ? (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(mine >> 32), src)
                       : 0u;
        longest = count[j] > longest ? count[j] : longest;
      }
      for (unsigned i0 = 0; i0 < longest; i0 += kWave) {
        unsigned rec[kAhead];
        bool in[kAhead];
#pragma unroll
        for (unsigned j = 0; j < kAhead; ++j) {
          in[j] = i0 + lane < count[j];
          rec[j] = in[j] ? stg.recs[first[j] + i0 + lane] : 0u;
        }
#pragma unroll
        for (unsigned j = 0; j < kAhead; ++j) {
          if (in[j]) {
            const unsigned loc = rec[j] & 511u;
            __hip_atomic_fetch_add(sum + loc, (float)((int)rec[j] >> 9) * stg.to_metres,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            __hip_atomic_fetch_add(cnt + loc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
          }
        }
      }
    }
  }
}

// The work items of a launch, taken by waves from a queue (one device atomic
// per eight items).  Item (block, k) of a block with n records (parts = ceil(n /
// kStageItemRecords) items, appended by the tile kernel) sums the block's runs
// k, k + parts, ... per voxel in LDS and adds the sums to the block's pool
// segments with device atomics: a segment's 8 sums and 8 weights by 16 lanes of
// one instruction, one memory-side request per touched segment.  Items of one
// block, the tile kernel's direct additions and the items of an earlier launch
// may all update a segment at once: every update is an atomic add.
constexpr unsigned kApplyWaves = kThreads / kWave;

__global__ __launch_bounds__(kThreads) void stage_apply_kernel(VolumeDev vol, StageDev stg) {
  __shared__ float s_sum[kApplyWaves][TSDF_BLOCK_VOXELS];
  __shared__ unsigned s_cnt[kApplyWaves][TSDF_BLOCK_VOXELS];
  const unsigned wv = threadIdx.x / kWave, lane = lane_id();
  const unsigned n_items = stg.head[2] < stg.item_cap ? stg.head[2] : stg.item_cap;
  float* const sum = s_sum[wv];
  unsigned* const cnt = s_cnt[wv];
  constexpr unsigned kGrab = 8;  // items per queue atomic: one counter serves every wave
  for (;;) {
    unsigned t0 = 0;
    if (lane == 0) t0 = add_u32(stg.head + 3, kGrab);
    t0 = (unsigned)__builtin_amdgcn_readfirstlane((int)t0);
    if (t0 >= n_items) break;
    for (unsigned t = t0; t < t0 + kGrab && t < n_items; ++t) {
    const unsigned blk = stg.items[2u * t], part = stg.items[2u * t + 1u];
    const unsigned long long stat = stg.block_stat[blk];
    const unsigned runs_listed = (unsigned)(stat >> 32);
    const unsigned n_runs = runs_listed < kStageRuns ? runs_listed : kStageRuns;
    const unsigned parts = ((unsigned)stat + kStageItemRecords - 1) / kStageItemRecords;
    stage_sum_runs(stg, blk, n_runs, part, parts, sum, cnt);
    float* const bp = vol.voxels + (size_t)blk * kBlockFloats;
#pragma unroll
    for (unsigned q = 0; q < 16; ++q) {
      const unsigned row = q * 4u + (lane >> 4), e = lane & 15u;  // segment; e < 8: sums, else weights
      const unsigned loc = row * 8u + (e & 7u);
      const unsigned c = cnt[loc];
      if (c) add_f32(bp + row * 16u + e, e < 8u ? sum[loc] : (float)c);
    }
    }
  }
}

hipError_t launch_stage_apply(VolumeDev vol, const StageDev& stage, hipStream_t s) {
  // a fixed grid of resident workgroups (16 KiB of LDS each, eight per CU)
  // taking items until the queue is empty
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)(n_cu > 0 ? n_cu : 1) * 8u;
  hipLaunchKernelGGL(stage_apply_kernel, dim3(grid), dim3(kThreads), 0, s, vol, stage);
  return hipGetLastError();
}

hipError_t launch_stage(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                        int frames_per_group, const StageDev& stage, hipStream_t s) {
  switch (wp.K) {
    case 1: return launch_stage_band1(vol, wp, frames, n, frames_per_group, stage, s);
    case 2: return launch_stage_band2(vol, wp, frames, n, frames_per_group, stage, s);
    case 3: return launch_stage_band3(vol, wp, frames, n, frames_per_group, stage, s);
    case 4: return launch_stage_band4(vol, wp, frames, n, frames_per_group, stage, s);
    case 5: return launch_stage_band5(vol, wp, frames, n, frames_per_group, stage, s);
    case 6: return launch_stage_band6(vol, wp, frames, n, frames_per_group, stage, s);
    case 7: return launch_stage_band7(vol, wp, frames, n, frames_per_group, stage, s);
    case 8: return launch_stage_band8(vol, wp, frames, n, frames_per_group, stage, s);
    default: return hipErrorInvalidValue;
  }
}

int max_frames_per_group(int K) {
  return K >= 1 && K <= TSDF_MAX_BAND_HALF ? max_frames_for(K) : 0;
}

hipError_t launch_fuse(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                       int frames_per_group, FuseMode mode, bool remap, hipStream_t s) {
  switch (wp.K) {
    case 1: return launch_fuse_band1(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 2: return launch_fuse_band2(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 3: return launch_fuse_band3(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 4: return launch_fuse_band4(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 5: return launch_fuse_band5(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 6: return launch_fuse_band6(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 7: return launch_fuse_band7(vol, wp, frames, n, frames_per_group, mode, remap, s);
    case 8: return launch_fuse_band8(vol, wp, frames, n, frames_per_group, mode, remap, s);
    default: return hipErrorInvalidValue;
  }
}

__global__ __launch_bounds__(256) void gather_status_kernel(DevCounters* const* ctrs, unsigned n, unsigned* out) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const DevCounters* c = ctrs[i];
  const unsigned bits =
      c ? __hip_atomic_load(&c->status_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
  __hip_atomic_store(&out[i], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_gather_status(DevCounters* const* ctrs, unsigned n, unsigned* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_status_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctrs, n, out);
  return hipGetLastError();
}

// The work list of tsdf_batch_fuse_static: a device array the library holds
// for the whole process on every device it runs on, so that the call needs no
// caller memory and allocates nothing.  Host code never uses the array's name
// as an address (on the host it is only a stand-in for the symbol): its device
// address is looked up once per device, with that device current, and kept.
namespace {
constexpr size_t kStaticListBytes = TSDF_STATIC_LIST_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticListBytes];
}  // namespace

hipError_t static_scratch(void** ptr, size_t* bytes) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  static std::mutex mu;
  static void* by_device[kMaxDevices];
  std::lock_guard<std::mutex> lock(mu);
  if (!by_device[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    by_device[dev] = p;
  }
  *ptr = by_device[dev];
  *bytes = kStaticListBytes;
  return hipSuccess;
}

const void* multi_kernel(int K, int pixels_per_thread, int acc_blocks, bool colour) {
  switch (K) {
    case 1: return multi_kernel_band1(pixels_per_thread, acc_blocks, colour);
    case 2: return multi_kernel_band2(pixels_per_thread, acc_blocks, colour);
    case 3: return multi_kernel_band3(pixels_per_thread, acc_blocks, colour);
    case 4: return multi_kernel_band4(pixels_per_thread, acc_blocks, colour);
    case 5: return multi_kernel_band5(pixels_per_thread, acc_blocks, colour);
    case 6: return multi_kernel_band6(pixels_per_thread, acc_blocks, colour);
    case 7: return multi_kernel_band7(pixels_per_thread, acc_blocks, colour);
    case 8: return multi_kernel_band8(pixels_per_thread, acc_blocks, colour);
    default: return nullptr;
  }
}

hipError_t launch_insert_blocks(VolumeDev vol, const int* coords, unsigned n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(insert_blocks_kernel, dim3((n + 255) / 256), dim3(256), 0, s, vol, coords, n);
  return hipGetLastError();
}

hipError_t launch_extract_colour(VolumeDev vol, unsigned n_blocks, float* rgb, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(extract_colour_kernel, dim3(grid_for((size_t)n_blocks * 512, 8192)),
                     dim3(256), 0, s, vol, n_blocks, rgb);
  return hipGetLastError();
}

hipError_t launch_extract(VolumeDev vol, unsigned n_blocks, unsigned long long* keys,
                          float* tsdf, float* weight, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(extract_kernel, dim3(grid_for((size_t)n_blocks * 64, 8192)), dim3(256), 0,
                     s, vol, n_blocks, keys, tsdf, weight);
  return hipGetLastError();
}

}  // namespace tsdf
