// bh_walk_f64.hip -- the FP64 force walk's kernels (forces only).
#include "bh_walk_impl.h"

namespace bh {

hipError_t walk_f64_forces(const WalkArgs& a, hipStream_t st) { return launch_walk_mode<true, kWalkForces>(a, st); }

const void* walk_f64_forces_fn(bool quad, bool soft, bool group_theta, int targets_per_lane) {
  return walk_persistent_fn<true, kWalkForces>(quad, soft, group_theta, targets_per_lane);
}

}  // namespace bh
