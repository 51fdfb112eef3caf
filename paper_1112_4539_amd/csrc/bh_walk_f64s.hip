// bh_walk_f64s.hip -- the FP64 walk's instrumented kernels (counts and list hashes, list dumps).
#include "bh_walk_impl.h"

namespace bh {

hipError_t walk_f64_stats(int mode, const WalkArgs& a, hipStream_t st) {
  return mode == kWalkDump ? launch_walk_mode<true, kWalkDump>(a, st) : launch_walk_mode<true, kWalkStats>(a, st);
}

const void* walk_f64_stats_fn(int mode, bool quad, bool soft, bool group_theta, int targets_per_lane) {
  return mode == kWalkDump ? walk_persistent_fn<true, kWalkDump>(quad, soft, group_theta, targets_per_lane)
                           : walk_persistent_fn<true, kWalkStats>(quad, soft, group_theta, targets_per_lane);
}

}  // namespace bh
