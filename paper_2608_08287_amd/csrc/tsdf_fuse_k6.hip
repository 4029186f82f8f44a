// The fused kernels (one volume; many volumes) and the staged tile kernel for
// a band of 2K + 1 samples, K = 6.
#include "tsdf_stage.h"

namespace tsdf {

hipError_t launch_fuse_band6(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                             int frames_per_group, FuseMode mode, bool remap, hipStream_t s) {
  return launch_fuse_k<6>(vol, wp, frames, n, frames_per_group, mode, remap, s);
}

hipError_t launch_stage_band6(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                              int frames_per_group, const StageDev& stage, hipStream_t s) {
  return launch_stage_k<6>(vol, wp, frames, n, frames_per_group, stage, s);
}

const void* multi_kernel_band6(int pixels_per_thread, int acc_blocks, bool colour) {
  return multi_kernel_k<6>(pixels_per_thread, acc_blocks, colour);
}

}  // namespace tsdf
