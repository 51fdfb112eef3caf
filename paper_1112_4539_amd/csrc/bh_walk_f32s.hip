// bh_walk_f32s.hip -- the FP32 walk's instrumented kernels (counts and list hashes, list dumps).
#include "bh_walk_impl.h"

namespace bh {

hipError_t walk_f32_stats(int mode, const WalkArgs& a, hipStream_t st) {
  return mode == kWalkDump ? launch_walk_mode<false, kWalkDump>(a, st) : launch_walk_mode<false, kWalkStats>(a, st);
}

const void* walk_f32_stats_fn(int mode, bool quad, bool soft, bool group_theta, int targets_per_lane) {
  return mode == kWalkDump ? walk_persistent_fn<false, kWalkDump>(quad, soft, group_theta, targets_per_lane)
                           : walk_persistent_fn<false, kWalkStats>(quad, soft, group_theta, targets_per_lane);
}

}  // namespace bh
