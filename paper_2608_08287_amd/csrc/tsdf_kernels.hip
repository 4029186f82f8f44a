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

// One thread per x-row of 8 voxels: read the row's 64-byte segment, write the
// 8 means and 8 weights in flat x-fastest order.
__global__ __launch_bounds__(256) void extract_kernel(VolumeDev vol, unsigned n_blocks,
                                                      unsigned long long* keys, float* tsdf,
                                                      float* weight) {
  const size_t n_rows = (size_t)n_blocks * (TSDF_BLOCK_VOXELS / 8);
  const size_t stride = (size_t)gridDim.x * 256u;
  const float4* v4 = reinterpret_cast<const float4*>(vol.voxels);
  for (size_t r = blockIdx.x * 256u + threadIdx.x; r < n_rows; r += stride) {
    const size_t src = (size_t)allocated_block(vol, (unsigned)(r / 64)) * 64 + r % 64;
    const float4 s0 = v4[4 * src], s1 = v4[4 * src + 1], w0 = v4[4 * src + 2],
                 w1 = v4[4 * src + 3];
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
      reinterpret_cast<float4*>(tsdf)[2 * r] = m0;
      reinterpret_cast<float4*>(tsdf)[2 * r + 1] = m1;
    }
    if (weight) {
      reinterpret_cast<float4*>(weight)[2 * r] = w0;
      reinterpret_cast<float4*>(weight)[2 * r + 1] = w1;
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
    const unsigned loc = (unsigned)(v % TSDF_BLOCK_VOXELS);
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
