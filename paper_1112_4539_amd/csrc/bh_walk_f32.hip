// bh_walk_f32.hip -- the FP32 force walk's kernels (forces only).
#include "bh_walk_impl.h"

namespace bh {

hipError_t walk_f32_forces(const WalkArgs& a, hipStream_t st) { return launch_walk_mode<false, kWalkForces>(a, st); }

const void* walk_f32_forces_fn(bool quad, bool soft, bool group_theta, int targets_per_lane) {
  return walk_persistent_fn<false, kWalkForces>(quad, soft, group_theta, targets_per_lane);
}

}  // namespace bh
