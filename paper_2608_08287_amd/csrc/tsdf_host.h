// Host-side internals shared by the translation units of the C ABI
// (tsdf_api.cpp: volumes; tsdf_batch.cpp: multi-volume batches).  Not part of
// the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/tsdf.h"
#include "tsdf_internal.h"

struct tsdf_volume {
  tsdf_volume_params params;
  tsdf_layout layout;
  tsdf::VolumeDev dev;
  uint32_t frames;
  uint32_t blocks_seen;  // blocks_total at the previous tsdf_query_status
};

namespace tsdf_host {

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline bool finite(float x) { return std::isfinite(x); }

// K = round(trunc / voxel_size): the band takes 2K + 1 samples (Section 2.2).
inline int band_half(const tsdf_volume_params& p) {
  return (int)std::llround((double)p.trunc / (double)p.voxel_size);
}

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

inline tsdf_status hip_status(hipError_t e) { return e == hipSuccess ? TSDF_OK : TSDF_ERR_HIP; }

inline bool valid_camera(const tsdf_camera* c) {
  if (!c) return false;
  if ((uint64_t)c->width * (uint64_t)c->height > (1ull << 31)) return false;
  if (!finite(c->fx) || !finite(c->fy) || !finite(c->cx) || !finite(c->cy)) return false;
  if (c->fx == 0.0f || c->fy == 0.0f) return false;
  for (int i = 0; i < 12; ++i)
    if (!finite(c->pose[i])) return false;
  return true;
}

inline tsdf::FrameDev frame_dev(const float* depth_dev, const tsdf_camera* cam,
                                const uint32_t* rgba_dev = nullptr) {
  tsdf::FrameDev f;
  f.depth = depth_dev;
  f.rgba = rgba_dev;
  f.width = cam->width;
  f.height = cam->height;
  f.cx = cam->cx;
  f.cy = cam->cy;
  f.ifx = 1.0f / cam->fx;
  f.ify = 1.0f / cam->fy;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) f.R[3 * r + c] = cam->pose[4 * r + c];
    f.t[r] = cam->pose[4 * r + 3];
  }
  return f;
}

inline tsdf::WalkParams walk_params(const tsdf_volume* vol) {
  tsdf::WalkParams wp;
  wp.v = vol->params.voxel_size;
  wp.iv = 1.0f / vol->params.voxel_size;
  wp.trunc = vol->params.trunc;
  wp.K = band_half(vol->params);
  return wp;
}

}  // namespace tsdf_host
