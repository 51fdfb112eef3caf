// bh_walk.hip -- walk copies of the nodes, and the dispatch of the force walk
// (the walk itself is in bh_walk_impl.h, instantiated by bh_walk_f32.hip,
// bh_walk_f32s.hip, bh_walk_f64.hip and bh_walk_f64s.hip).
#include "bh_walk_impl.h"

namespace bh {

// The opening size S = (l/theta + s)^2 of a node is precomputed per node for a
// uniform theta (one pass per call) or formed on the fly from a per-group theta.
__global__ __launch_bounds__(256) void k_mac_size(const Node* __restrict__ nodes, const Counts* __restrict__ cnt,
                                                  int cap, double inv_theta, WalkNode* __restrict__ wnodes) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cap || c >= cnt->n_nodes) return;
  const Node nd = nodes[c];
  const double u = fma(nd.l, inv_theta, nd.s);
  WalkNode w;
  // A leaf's S is 0: every other particle passes (d^2 > 0, since particles at
  // the same position share a leaf of several particles), and the target's own
  // leaf fails (its position is the target's, exactly: d^2 = 0).
  w.cx = nd.cx;
  w.cy = nd.cy;
  w.cz = nd.cz;
  w.M = nd.M;
  w.S = (nd.meta & 1) ? 0.0 : u * u;
  w.M32 = (float)nd.M;
  w.pad = 0;
  // next(c) kept inside (c, cap]: the walk then moves forward and reads at
  // most one record past the last without checking
  w.next = min(max(nd.next, c + 1), cap);
  w.first = nd.first;
  w.count = nd.count;
  w.meta = nd.meta;
  wnodes[c] = w;
}

hipError_t launch_mac_size(const Node* nodes, const Counts* counts, int cap, double inv_theta,
                           WalkNode* wnodes, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  k_mac_size<<<(cap + 255) / 256, 256, 0, st>>>(nodes, counts, cap, inv_theta, wnodes);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_theta_copy(const Node* __restrict__ nodes, const Counts* __restrict__ cnt,
                                                    int cap, ThetaNode* __restrict__ tnodes) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cap || c >= cnt->n_nodes) return;
  const Node nd = nodes[c];
  const bool leaf = nd.meta & 1;
  ThetaNode w;
  w.cx = nd.cx;
  w.cy = nd.cy;
  w.cz = nd.cz;
  w.l = leaf ? 0.0 : nd.l;
  w.M32 = (float)nd.M;
  w.next = min(max(nd.next, c + 1), cap);  // as in the uniform-theta copy
  w.first = nd.first;
  w.count = nd.count;
  w.s = leaf ? 0.0 : nd.s;
  w.meta = nd.meta;
  w.pad = 0;
  tnodes[c] = w;
}

hipError_t launch_theta_copy(const Node* nodes, const Counts* counts, int cap, ThetaNode* tnodes, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  k_theta_copy<<<(cap + 255) / 256, 256, 0, st>>>(nodes, counts, cap, tnodes);
  return hipGetLastError();
}

// Workgroups of the persistent walk that are resident on the chip at once (0 if
// the runtime cannot tell).
int persistent_grid(bool f64, int mode, bool soft, bool group_theta, int waves_per_block, int targets_per_lane) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const bool quad = (mode & kWalkQuad) != 0;
  const int m = mode & 3;
  const void* fn = f64 ? (m == kWalkForces ? walk_f64_forces_fn(quad, soft, group_theta, targets_per_lane)
                                           : walk_f64_stats_fn(m, quad, soft, group_theta, targets_per_lane))
                       : (m == kWalkForces ? walk_f32_forces_fn(quad, soft, group_theta, targets_per_lane)
                                           : walk_f32_stats_fn(m, quad, soft, group_theta, targets_per_lane));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, waves_per_block * kWave, 0) != hipSuccess) return 0;
  return cus * per_cu;
}

hipError_t launch_walk(bool f64, int mode, const WalkArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  // (the order-2 bit of the mode is carried by a.qrec)
  const int m = mode & 3;
  if (f64) return m == kWalkForces ? walk_f64_forces(a, st) : walk_f64_stats(m, a, st);
  return m == kWalkForces ? walk_f32_forces(a, st) : walk_f32_stats(m, a, st);
}

}  // namespace bh
