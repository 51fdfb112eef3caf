// bh_common.h -- shared definitions of the gfx950 Barnes-Hut library (device and host side).
//
// Data layout in HBM (one tree of n particles; every array lives in the
// caller's workspace):
//   * particles, Morton order:  float4/double4 (x, y, z, m) per particle, plus
//     perm[k] = caller index of the k-th particle in Morton order.
//   * nodes, depth-first preorder (Sec. 4.4 next/more pointers): one 64-byte
//     Node per cell or leaf.  more(c) is implicitly c+1; next(c) is stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bh {

constexpr int kLevels = 21;                 // bits per axis of the Morton grid (63-bit keys)
constexpr uint32_t kGrid = 1u << kLevels;   // cells per axis at the finest level
constexpr int kWave = 64;                   // CDNA wavefront width

// One node of the tree, 64 bytes, read by the walk with scalar loads.
//   com   : centre of mass (a one-particle leaf: the particle's position, exact)
//   M     : total mass (FP64 sum, children folded left in octant order)
//   l     : side of the cell, L * 2^-level
//   s     : |geometric centre - com| (Eq. (2) of the paper), 0 for leaves
//   next  : preorder id of the first node after this subtree
//   first : Morton position of the first particle of the subtree
//   count : number of particles in the subtree
//   meta  : bit 0 = leaf, bit 1 = leaf holding several particles (coincident
//           keys), bits 8..15 = level
struct alignas(64) Node {
  double cx, cy, cz;
  double M;
  double l;
  double s;
  int32_t next;
  int32_t first;
  int32_t count;
  int32_t meta;
};
static_assert(sizeof(Node) == 64, "Node must be 64 bytes");

// The walk's copy of a node for one uniform theta: a cell carries its squared
// opening size S = (l/theta + s)^2 (a leaf 0), and the mass also rounded to
// FP32.  The fields one FP32 step reads (centre, S, M32, next, first, count,
// meta) are the first 52 bytes, the FP32 mass beside the integers, so that
// they arrive in one batch of scalar loads.
struct alignas(64) WalkNode {
  double cx, cy, cz;
  double S;
  float M32;
  int32_t next;
  int32_t first;
  int32_t count;
  int32_t meta;
  int32_t pad;
  double M;
};
static_assert(sizeof(WalkNode) == 64, "WalkNode must be 64 bytes");

// The walk's copy of a node for per-group theta (FP32 walks): the opening size
// is formed per step from l and s, S = (l/theta + s)^2; a leaf carries l = s =
// 0, so S = 0 < d^2 for every particle but the target itself.  The fields of a
// step are the first 56 bytes.
struct alignas(64) ThetaNode {
  double cx, cy, cz;
  double l;
  float M32;
  int32_t next;
  int32_t first;
  int32_t count;
  double s;
  int32_t meta;
  int32_t pad;
};
static_assert(sizeof(ThetaNode) == 64, "ThetaNode must be 64 bytes");

// Second moments of a node for walks of order 2 (quadrupole cell terms):
// B_ab = sum over the node's particles of m (x_a - com_a)(x_b - com_b), FP64,
// with T = Bxx + Byy + Bzz kept as T/2 (exact) and -3T/2, the two forms the
// term uses.  A one-particle leaf has B = 0.  Read by the walk beside the
// node's walk record, with the same index.
struct alignas(64) QuadRec {
  double bxx, bxy, bxz, byy, byz, bzz;
  double t05;    // T / 2
  double nt15;   // -3T / 2
};
static_assert(sizeof(QuadRec) == 64, "QuadRec must be 64 bytes");

// Root cube and Morton quantisation, computed on the device by the bbox pass.
struct Cube {
  double lo[3];   // coordinate-wise minimum of the particles
  double L;       // largest extent (1 if every particle coincides)
  double scale;   // 2^21 / L
  double pad[3];
};

// Device-side counters of one build.
struct Counts {
  int32_t n_unique;     // U: distinct Morton keys (= leaves)
  int32_t n_internal;   // I: internal nodes
  int32_t n_nodes;      // U + I
  int32_t bad_input;    // nonzero if a coordinate or mass was not finite
  int32_t bad_theta;    // nonzero if the last per-group-theta walk met an invalid theta
  int32_t pad[3];
};

// Opening parameters: a walk accepts theta in (0, 2/sqrt(3)) (beyond that a cell
// holding the target could pass Eq. (2)); a per-group theta outside that range
// or not finite is replaced by kThetaFallback and reported.
constexpr double kThetaMax = 1.1547005383792515;  // 2/sqrt(3)
constexpr float kThetaFallback = 0.5f;

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroups are dispatched to the 8 XCDs round-robin.  The logical index of
// workgroup b of nb gives each XCD runs of `chunk` consecutive indices (whose
// work shares data in that XCD's L2: tree nodes for neighbouring walk groups,
// source lines for neighbouring gathers), interleaving the runs across XCDs to
// keep the load even.  A run is at most a 64th of the grid, so that every XCD
// takes at least 8 runs and a few heavy runs do not leave the others idle.
__device__ __forceinline__ int remap_block(int b, int nb, int chunk) {
  if (chunk <= 0) return b;
  chunk = min(chunk, max(1, nb >> 6));
  const int full = (nb / (8 * chunk)) * 8 * chunk;
  if (b >= full) return b;
  const int k = b >> 3, x = b & 7;
  return ((k / chunk) * 8 + x) * chunk + (k % chunk);
}

}  // namespace bh
