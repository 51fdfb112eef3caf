// bh_internal.h -- launch-side declarations shared by the library's translation units.
#pragma once
#include "bh_common.h"

namespace bh {

// scans: 256 threads x 16 items per tile
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
// radix sort: 256 threads x 16 keys per tile, 8-bit digits
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kBboxBlocks = 1024;

// Mass and first moments (sum of m x) of a node, FP64: what a parent's moment
// pass reads of each child, in one aligned 32-byte record.
struct alignas(32) Mom {
  double M, X, Y, Z;
};

// Views into the caller's workspace used by one build.  A build covers K >= 1
// independent clusters (a forest): cluster k is the caller's particles
// [off[k], off[k+1]) and gets its own root cube, keys and tree.  The sort puts
// the clusters one after the other in Morton order, so every cluster keeps its
// particle range, and its subtree is the preorder node range [croot[k],
// croot[k+1]).  A single tree is the forest with K = 1.
// The moment passes fold every subtree that lies inside one chunk of kChunk
// consecutive preorder nodes in a workgroup's LDS.  The internal nodes whose
// subtree crosses the chunk's end are ancestors of the next chunk's first node
// that start in the chunk, so a chunk has at most one per level: they are kept
// in kLevels x (number of chunks) slots, each with its children.
constexpr int kChunk = 512;
constexpr int kChunkThreads = 256;  // workgroup of the chunk launches: kChunk / kChunkThreads nodes per thread
inline int64_t n_chunks(int64_t n) { return (2 * (n > 0 ? n : 1) + kChunk - 1) / kChunk; }

struct BuildWs {
  Cube* cube;               // [K] root cube per cluster
  Counts* counts;
  int n_seg;                // K
  const int64_t* seg_off;   // [K+1] cluster offsets (device; the caller's or own_off)
  int64_t* own_off;         // [2] offsets {0, n} of a single tree
  int32_t* seg;             // [n] caller index -> cluster
  int32_t* scid;            // [n] Morton position -> cluster
  int32_t* ucid;            // [n] unique key -> cluster
  int32_t* croot;           // [K+1] preorder id of each cluster's root; croot[K] = node count
  double* bbox_part;        // [kBboxBlocks][6]
  int n_bbox_blocks;
  uint64_t *key_a, *key_b;  // [n]
  int32_t *idx_a, *idx_b;   // [n]; idx_a ends as perm (Morton position -> caller index)
  int32_t* hist;            // [256 * ntiles]
  int32_t* scan_tiles;      // scan scratch
  void* ps;                 // [n] float4 or double4 (x, y, z, m) in Morton order
  int32_t *flag, *uid;      // [n]
  uint64_t* ukey;           // [n]
  int32_t* ustart;          // [n + 1]
  int32_t *split, *pf, *pl; // [n]
  int32_t *ilevel, *ifirst, *ilast;  // [n]
  int32_t *nstart, *nexcl;  // [n + 1]
  uint32_t* lmask;          // [n + 1]
  Node* nodes;              // [2n]
  Mom* mom;                 // [2n] mass and first moments of every node, for the moment passes
  int32_t* nx;              // [2n] next(c) of every node, for the moment passes
  uint8_t* nlev;            // [2n] level of every node, for the moment passes
  int32_t* obkt;            // [kLevels][n_chunks] the straddling node of each level and chunk, or -1
  int32_t* okids;           // [kLevels][n_chunks][8] their children in octant order, -1 after the last
  WalkNode* wnodes;         // [2n] walk copy of the nodes for the last uniform theta
  int32_t* horder;          // [n] Morton positions in the Hilbert walk order (filled on demand)
  uint64_t *hkey_a, *hkey_b;  // [n] sort buffers of the Hilbert order (its own: it may run beside the build)
  int32_t* hidx;            // [n]
  int32_t* hhist;           // [256 * ntiles]
  int32_t* hscan;           // scan scratch
  QuadRec* qrec;            // [2n + 1] second moments of every node (walks of order 2; filled on demand)
};

// A second stream for a build: the Hilbert walk order, which needs only the
// sorted particles, is formed there while the build goes on (fork is recorded
// on the build's stream after the particles are sorted, join on the second
// stream after the order; the build's stream waits for join before it returns).
struct BuildFork {
  hipStream_t side;
  hipEvent_t fork, join;
};

hipError_t scan_excl(const int32_t* in, int32_t* out, int n, int32_t* tile_buf, int32_t* total, hipStream_t st);
hipError_t build_tree_f32(const float* pos, const float* mass, int n, const BuildWs& w, const BuildFork* fork,
                          hipStream_t st);
hipError_t build_tree_f64(const double* pos, const double* mass, int n, const BuildWs& w, const BuildFork* fork,
                          hipStream_t st);
hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
// Walk order of the targets (w.horder): Morton positions sorted by cluster and
// the Hilbert index of their cell a few levels below the cluster's root cube.
// Reads the sorted particles (w.ps, w.scid) and the cubes; its scratch arrays
// are its own.
hipError_t hilbert_order(bool f64, int n, const BuildWs& w, hipStream_t st);
// The targets' walk order as caller indices (order: Morton positions, null =
// Morton order).
hipError_t launch_walk_order(const int32_t* order, const int32_t* perm, int n, int32_t* out, hipStream_t st);
// Second moments of every node about its centre of mass (w.qrec), for walks of
// order 2; runs after the build (reads its nodes and topology arrays).
hipError_t quad_moments(bool f64, int n, const BuildWs& w, hipStream_t st);

// Tree walk launch.  Targets are processed in groups of 64 (one wavefront);
// group g holds the targets at positions [64g, 64g+64) of `order` (Morton
// positions; null = Morton order itself).
struct WalkArgs {
  const Node* nodes;
  const Counts* cnt;           // the build's counters (leaf count)
  int32_t* bad_theta;          // per-group theta walks: set to 1 if a theta was replaced
  const void* ps;              // float4 / double4 particles in Morton order
  const int32_t* perm;         // Morton position -> caller index
  const int32_t* order;        // optional target order (Morton positions), may be null
  const int32_t* scid;         // Morton position -> cluster (null for a single tree)
  const int32_t* croot;        // [K+1] preorder range of each cluster's subtree
  const int64_t* seg_off;      // [K+1] caller offsets of the clusters (list words are cluster-relative)
  int n_seg;
  int n;
  double eps2;
  double inv_theta;            // 1/theta when theta_group is null
  const WalkNode* wnodes;      // uniform theta: walk copy of the nodes (S and M32 precomputed)
  const ThetaNode* tnodes;     // per-group theta, FP32: walk copy with l and s (same memory as wnodes)
  const float* theta_group;    // theta per walk group (64 targets of the walk order), may be null
  const QuadRec* qrec;         // order 2: second moments of every node (cell terms with the quadrupole)
  void* acc;                   // [n][3] caller order
  void* pot;                   // [n] caller order
  int32_t* counts;             // stats: [n][2] = (particle terms, cell terms), caller order
  uint64_t* hash;              // stats: [n] ordered-list hash, caller order
  int64_t* lists;              // dump: [n][maxlen] list words, caller order
  int64_t maxlen;
  int32_t* group_steps;        // stats: [ceil(n/64)] nodes visited per group, may be null
  int xcd_chunk;               // workgroups per XCD chunk of the block remap (0 = identity)
  int lds_share64;             // waves (out of 64) that read nodes through LDS copies
  int waves_per_block;         // 1, 2 or 4
  int persistent;              // 0: one wave per group; 1: waves pull groups from `queue`
  int32_t* queue;              // persistent: group counter, zeroed before the launch
  int grid;                    // persistent: workgroups launched
  int targets_per_lane;        // 1 or 2: a wave walks 64 or 128 targets
};

enum WalkMode { kWalkForces = 0, kWalkStats = 1, kWalkDump = 2 };
// Added to a mode: cell terms of order 2 (monopole plus quadrupole correction).
constexpr int kWalkQuad = 4;

hipError_t launch_walk(bool f64, int mode, const WalkArgs& a, hipStream_t st);

// Workgroups of the persistent walk resident on the current device at once.
int persistent_grid(bool f64, int mode, bool soft, bool group_theta, int waves_per_block, int targets_per_lane);

// Walk copy of the nodes for one uniform theta: every record with its side l
// replaced by S = (l/theta + s)^2 (Eq. (2) squared, the S_effective of Sec. 4.4)
// and its mass also in FP32.
hipError_t launch_mac_size(const Node* nodes, const Counts* counts, int cap, double inv_theta,
                           WalkNode* wnodes, hipStream_t st);

// ---- learned opening parameter (bh_learn.hip)
// Flat FP32 parameters of the MLP 8 -> 64 -> 64 -> 1: W1 [64][8], b1 [64],
// W2 [64][64], b2 [64], w3 [64], b3; a gradient vector has one more entry
// (the batch loss).  bf16 weight copies: W1, W2, W2 transposed, w3.
constexpr int kMlpW1 = 0, kMlpB1 = 512, kMlpW2 = 576, kMlpB2 = 4672, kMlpw3 = 4736, kMlpB3 = 4800;
constexpr int kMlpParams = 4801;
constexpr int kMlpGradLen = kMlpParams + 1;
constexpr int kMlpW1b = 0, kMlpW2b = 512, kMlpW2Tb = 4608, kMlpw3b = 8704, kMlpWb = 8768;
constexpr int kMlpMaxParts = 1024;  // workgroups (partial gradients) of one gradient pass

// Learned theta: per walk group g, the 64 Morton positions order[64g, 64g+64)
// (order null: Morton groups).
hipError_t launch_features(bool f64, const Node* nodes, const void* ps, const Cube* cubes, const int32_t* scid,
                           const int32_t* croot, const int64_t* seg_off, int n_seg, int n, const int32_t* order,
                           float* X, hipStream_t st);
hipError_t launch_group_error(bool f64, const void* acc, const double* ref, const int32_t* perm,
                              const int32_t* order, int n, double theta, double target, double* rms, float* label,
                              hipStream_t st);
hipError_t launch_mlp_prepare(const float* P, uint16_t* wb, hipStream_t st);
hipError_t launch_mlp_infer(const float* P, const uint16_t* wb, const float* norm, const float* X, int64_t rows,
                            float alpha, float fallback, float cap, float* theta, hipStream_t st);
int mlp_grad_parts(int batch);
hipError_t launch_mlp_grad(const float* P, const uint16_t* wb, const float* norm, const float* X, const float* T,
                           const int32_t* idx, int batch, float* partial, float* grad, hipStream_t st);
hipError_t launch_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, uint16_t* wb, hipStream_t st);

// Walk copy of the nodes for per-group theta (FP32 walks).
hipError_t launch_theta_copy(const Node* nodes, const Counts* counts, int cap, ThetaNode* tnodes, hipStream_t st);

// Neighbour search (the general tree walk of Fig. 4): per target the particles
// within `radius`, their ordered hash, optional lists and the SPH density.
// `copy` receives the walk copy (2n + 1 records; the force walk's buffer).
hipError_t launch_neighbours(bool f64, const Node* nodes, const Counts* counts, WalkNode* copy, const void* ps,
                             const int32_t* perm, const int32_t* order, const int32_t* scid, const int32_t* croot,
                             const int64_t* seg_off, int n_seg, int n, double radius, int32_t* count,
                             uint64_t* hash, int64_t* lists, int64_t maxlen, void* rho, int xcd_chunk,
                             hipEvent_t ev0, hipEvent_t ev1, hipStream_t st);

// Time loop (bh_step.hip): leapfrog updates and the Morton reorder of the state.
hipError_t launch_kick_drift(bool f64, void* pos, void* vel, const void* acc, int n, double dt, hipStream_t st);
hipError_t launch_kick(bool f64, void* vel, const void* acc, int n, double dt, hipStream_t st);
hipError_t launch_reorder(bool f64, const int32_t* perm, int n, void* pos, void* vel, void* mass, void* acc,
                          void* pot, int64_t* ids, void* tmp, hipStream_t st);

// Direct sum of Eq. (1) for a list of targets (caller indices).
hipError_t launch_direct(bool f64, const void* pos, const void* mass, int n, const int64_t* targets, int nt,
                         double eps, void* acc, void* pot, hipStream_t st);

}  // namespace bh
