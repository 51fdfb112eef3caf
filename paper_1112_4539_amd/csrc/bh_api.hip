// bh_api.hip -- host side of the C ABI declared in include/bh.h.
//
// Argument checks, workspace carving, and the launch sequences of the build,
// the walk and the direct sum.  Device memory is never allocated here: every
// array is a view into the caller's workspace.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/bh.h"
#include "bh_internal.h"

namespace bh {
hipError_t make_rank(const int32_t* perm, int n, int32_t* rank, hipStream_t st);
}

struct bh_tree {
  int64_t n = 0;
  int64_t n_seg = 1;
  int prec = BH_FP32;
  const void* pos = nullptr;       // build inputs, kept for graph replays
  const void* mass = nullptr;
  bh::BuildWs w{};
  int32_t* rank = nullptr;  // caller index -> Morton position (filled on demand)
  mutable bool rank_ready = false;
  int32_t* queue = nullptr; // group counter of the persistent walk
  int waves_per_block = 1;
  int xcd_chunk = -1;  // -1: 1024 for FP32 trees (about the one-wave workgroups an XCD holds), 0 for FP64
  int target_order = 2;
  mutable bool horder_ready = false;  // w.horder holds the Hilbert order of the current build
  int order = 1;                      // cell terms: 1 monopole, 2 with the quadrupole correction
  mutable bool quad_ready = false;    // w.qrec holds the second moments of the current build
  int lds_share64 = 0;
  int persistent = 0;
  int targets_per_lane = 1;
  bool timing = false;
  bool timed = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct bh_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(BH_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// (node and record indices are int32: 2n + 1 walk records must fit)
constexpr int64_t kMaxN = (int64_t(1) << 30) - 1;
constexpr int64_t kMaxClusters = int64_t(1) << 24;
constexpr size_t kAlign = 256;
using bh::kThetaMax;
const double kThetaCap = 1.15;  // largest learned theta handed to the walk (below 2/sqrt(3))

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves the workspace; with base == nullptr it only measures.
size_t layout(int64_t n, int64_t K, int prec, char* base, bh::BuildWs* w, int32_t** rank, int32_t** queue) {
  const size_t N = (size_t)(n > 0 ? n : 1);
  const size_t nodes = 2 * N;
  const size_t sort_tiles = (N + bh::kSortTile - 1) / bh::kSortTile;
  const size_t hist = 256 * sort_tiles;
  const size_t max_scan = hist > N + 1 ? hist : N + 1;
  const size_t scan_tiles = (max_scan + bh::kScanTile - 1) / bh::kScanTile + 16;
  const size_t ps = (prec == BH_FP64 ? 32 : 16) * N;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += up(bytes);
    return p;
  };
  bh::BuildWs t{};
  t.n_seg = (int)K;
  t.cube = reinterpret_cast<bh::Cube*>(take(sizeof(bh::Cube) * (size_t)K));
  t.counts = reinterpret_cast<bh::Counts*>(take(sizeof(bh::Counts)));
  t.own_off = reinterpret_cast<int64_t*>(take(2 * sizeof(int64_t)));
  t.seg_off = t.own_off;
  t.croot = reinterpret_cast<int32_t*>(take(4 * ((size_t)K + 1)));
  int32_t* q = reinterpret_cast<int32_t*>(take(4));
  t.seg = reinterpret_cast<int32_t*>(take(4 * N));
  t.scid = reinterpret_cast<int32_t*>(take(4 * N));
  t.ucid = reinterpret_cast<int32_t*>(take(4 * N));
  t.bbox_part = reinterpret_cast<double*>(take(sizeof(double) * 6 * bh::kBboxBlocks));
  t.n_bbox_blocks = bh::kBboxBlocks;
  t.key_a = reinterpret_cast<uint64_t*>(take(8 * N));
  t.key_b = reinterpret_cast<uint64_t*>(take(8 * N));
  t.ukey = reinterpret_cast<uint64_t*>(take(8 * N));
  t.idx_a = reinterpret_cast<int32_t*>(take(4 * N));
  t.idx_b = reinterpret_cast<int32_t*>(take(4 * N));
  t.hist = reinterpret_cast<int32_t*>(take(4 * hist));
  t.scan_tiles = reinterpret_cast<int32_t*>(take(4 * scan_tiles));
  t.ps = take(ps);
  t.flag = reinterpret_cast<int32_t*>(take(4 * N));
  t.uid = reinterpret_cast<int32_t*>(take(4 * N));
  t.ustart = reinterpret_cast<int32_t*>(take(4 * (N + 1)));
  t.split = reinterpret_cast<int32_t*>(take(4 * N));
  t.pf = reinterpret_cast<int32_t*>(take(4 * N));
  t.pl = reinterpret_cast<int32_t*>(take(4 * N));
  t.ilevel = reinterpret_cast<int32_t*>(take(4 * N));
  t.ifirst = reinterpret_cast<int32_t*>(take(4 * N));
  t.ilast = reinterpret_cast<int32_t*>(take(4 * N));
  t.nstart = reinterpret_cast<int32_t*>(take(4 * (N + 1)));
  t.nexcl = reinterpret_cast<int32_t*>(take(4 * (N + 1)));
  t.lmask = reinterpret_cast<uint32_t*>(take(4 * (N + 1)));
  t.nodes = reinterpret_cast<bh::Node*>(take(sizeof(bh::Node) * nodes));
  t.mom = reinterpret_cast<bh::Mom*>(take(sizeof(bh::Mom) * nodes));
  t.nx = reinterpret_cast<int32_t*>(take(4 * nodes));
  t.nlev = reinterpret_cast<uint8_t*>(take(nodes));
  t.obkt = reinterpret_cast<int32_t*>(take(4 * bh::kLevels * (size_t)bh::n_chunks((int64_t)N)));
  t.okids = reinterpret_cast<int32_t*>(take(32 * bh::kLevels * (size_t)bh::n_chunks((int64_t)N)));
  // (one spare record past the last: the walk reads the record after its
  // cursor's last position before it tests the loop bound)
  t.wnodes = reinterpret_cast<bh::WalkNode*>(take(sizeof(bh::WalkNode) * (nodes + 1)));
  t.horder = reinterpret_cast<int32_t*>(take(4 * N));
  t.hkey_a = reinterpret_cast<uint64_t*>(take(8 * N));
  t.hkey_b = reinterpret_cast<uint64_t*>(take(8 * N));
  t.hidx = reinterpret_cast<int32_t*>(take(4 * N));
  t.hhist = reinterpret_cast<int32_t*>(take(4 * hist));
  t.hscan = reinterpret_cast<int32_t*>(take(4 * scan_tiles));
  t.qrec = reinterpret_cast<bh::QuadRec*>(take(sizeof(bh::QuadRec) * (nodes + 1)));
  int32_t* r = reinterpret_cast<int32_t*>(take(4 * N));
  if (w) *w = t;
  if (rank) *rank = r;
  if (queue) *queue = q;
  return off;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int check_theta_eps(double theta, double eps) {
  if (!(theta > 0.0 && theta < kThetaMax))
    return fail(BH_EINVAL, "theta must be in (0, 2/sqrt(3)); got %g", theta);
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BH_EINVAL, "eps must be finite and >= 0; got %g", eps);
  return BH_OK;
}

int sync_counts(const bh_tree* t, hipStream_t st, bh::Counts* c) {
  hipError_t e = hipMemcpyAsync(c, t->w.counts, sizeof(bh::Counts), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "reading tree counters");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "synchronising the stream");
  return BH_OK;
}

constexpr int kMaxDevices = 64;

// One second stream per device (default priority), with its two events, for
// the Hilbert order beside the build; created on first use, kept until the
// process ends.  Builds that use it hold g_side_mu while they enqueue.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
SideStream g_side[kMaxDevices];

hipError_t side_stream(SideStream** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  SideStream& ss = g_side[dev];
  if (!ss.s) {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (b) (void)hipEventDestroy(b);
      if (a) (void)hipEventDestroy(a);
      if (s) (void)hipStreamDestroy(s);
      return e;
    }
    ss.s = s;
    ss.fork = a;
    ss.join = b;
  }
  *out = &ss;
  return hipSuccess;
}

hipError_t build_on(const bh_tree* t, const bh::BuildFork* fork, hipStream_t st) {
  const int n = (int)t->n;
  return t->prec == BH_FP64
             ? bh::build_tree_f64(static_cast<const double*>(t->pos), static_cast<const double*>(t->mass), n, t->w,
                                  fork, st)
             : bh::build_tree_f32(static_cast<const float*>(t->pos), static_cast<const float*>(t->mass), n, t->w,
                                  fork, st);
}

// Enqueues the build.  With may_fork, a tree that walks in Hilbert order gets
// that order formed on the second stream beside the build (not while st is
// being captured into a graph: the capture then holds the plain sequence).
hipError_t enqueue_build(const bh_tree* t, hipStream_t st, bool may_fork = true) {
  t->horder_ready = false;
  t->quad_ready = false;
  t->rank_ready = false;
  bool fork = may_fork && t->target_order == 2 && t->n > 0;
  if (fork) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    fork = hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
  }
  if (!fork) return build_on(t, nullptr, st);
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStream* ss = nullptr;
  if (side_stream(&ss) != hipSuccess) return build_on(t, nullptr, st);
  const bh::BuildFork bf{ss->s, ss->fork, ss->join};
  hipError_t e = build_on(t, &bf, st);
  if (e == hipSuccess) t->horder_ready = true;
  return e;
}

// Morton positions in the walk's target order (null: Morton order), once
// ensure_target_order has formed it.
const int32_t* walk_order_of(const bh_tree* t) {
  return t->target_order == 1 ? t->rank : t->target_order == 2 ? t->w.horder : nullptr;
}

// The walk order of the targets for the current build, formed on first use.
hipError_t ensure_target_order(const bh_tree* t, hipStream_t st) {
  if (t->n == 0) return hipSuccess;
  if (t->target_order == 1 && !t->rank_ready) {
    hipError_t e = bh::make_rank(t->w.idx_a, (int)t->n, t->rank, st);
    if (e != hipSuccess) return e;
    t->rank_ready = true;
  }
  if (t->target_order == 2 && !t->horder_ready) {
    hipError_t e = bh::hilbert_order(t->prec == BH_FP64, (int)t->n, t->w, st);
    if (e != hipSuccess) return e;
    t->horder_ready = true;
  }
  return hipSuccess;
}

int run_walk(const bh_tree* t, double theta, const float* theta_group, double eps, void* acc, void* pot,
             int mode, int32_t* counts, uint64_t* hash, int64_t* lists, int64_t maxlen, int32_t* group_steps,
             hipStream_t st, bool allow_timing = true) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (!theta_group) {
    int rc = check_theta_eps(theta, eps);
    if (rc) return rc;
  } else if (!(eps >= 0.0) || !std::isfinite(eps)) {
    return fail(BH_EINVAL, "eps must be finite and >= 0; got %g", eps);
  }
  if (t->n == 0) return BH_OK;
  const size_t el = t->prec == BH_FP64 ? 8 : 4;
  if (!acc || !pot || !aligned(acc, el) || !aligned(pot, el))
    return fail(BH_EINVAL, "acc/pot must be non-null device arrays aligned to %zu bytes", el);
  if (mode != bh::kWalkForces && (!counts || !hash || !aligned(counts, 4) || !aligned(hash, 8)))
    return fail(BH_EINVAL, "counts/hash must be non-null aligned device arrays");
  if (mode == bh::kWalkDump && (!lists || maxlen <= 0 || !aligned(lists, 8)))
    return fail(BH_EINVAL, "lists must be a non-null aligned device array with maxlen > 0");
  if (!theta_group) {
    hipError_t e = bh::launch_mac_size(t->w.nodes, t->w.counts, (int)(2 * t->n), 1.0 / theta, t->w.wnodes, st);
    if (e != hipSuccess) return hip_fail(e, "launching the opening-size pass");
  } else {
    // the flag reports this walk's per-group values only
    hipError_t e = bh::fill_i32(&t->w.counts->bad_theta, 1, 0, st);
    if (e != hipSuccess) return hip_fail(e, "clearing the theta flag");
  }
  if (theta_group && t->prec == BH_FP32) {
    hipError_t e = bh::launch_theta_copy(t->w.nodes, t->w.counts, (int)(2 * t->n),
                                         reinterpret_cast<bh::ThetaNode*>(t->w.wnodes), st);
    if (e != hipSuccess) return hip_fail(e, "launching the per-group walk copy");
  }
  {
    // (once per build; a graph that captures the build captures this too)
    hipError_t e = ensure_target_order(t, st);
    if (e != hipSuccess) return hip_fail(e, "launching the target order");
  }
  if (t->order == 2 && !t->quad_ready) {
    // (once per build, like the Hilbert order)
    hipError_t e = bh::quad_moments(t->prec == BH_FP64, (int)t->n, t->w, st);
    if (e != hipSuccess) return hip_fail(e, "launching the second-moment passes");
    t->quad_ready = true;
  }
  bh::WalkArgs a{};
  a.nodes = t->w.nodes;
  a.qrec = t->order == 2 ? t->w.qrec : nullptr;
  a.cnt = t->w.counts;
  a.bad_theta = &t->w.counts->bad_theta;
  a.wnodes = t->w.wnodes;
  a.tnodes = reinterpret_cast<const bh::ThetaNode*>(t->w.wnodes);
  a.ps = t->w.ps;
  a.perm = t->w.idx_a;
  a.order = walk_order_of(t);
  a.scid = t->n_seg > 1 ? t->w.scid : nullptr;  // (a single tree keeps no cluster ids)
  a.croot = t->w.croot;
  a.seg_off = t->w.seg_off;
  a.n_seg = (int)t->n_seg;
  a.n = (int)t->n;
  a.eps2 = eps * eps;
  a.inv_theta = theta_group ? 0.0 : 1.0 / theta;
  a.theta_group = theta_group;
  a.acc = acc;
  a.pot = pot;
  a.counts = counts;
  a.hash = hash;
  a.lists = lists;
  a.maxlen = maxlen;
  a.group_steps = group_steps;
  a.xcd_chunk = t->xcd_chunk >= 0 ? t->xcd_chunk : (t->prec == BH_FP64 ? 0 : 1024);
  a.lds_share64 = t->lds_share64;
  a.waves_per_block = t->waves_per_block;
  a.persistent = t->persistent;
  a.targets_per_lane = t->order == 2 ? 1 : t->targets_per_lane;  // (order 2: one target per lane)
  a.queue = t->queue;
  if (a.persistent) {
    a.grid = bh::persistent_grid(t->prec == BH_FP64, t->order == 2 ? (mode | bh::kWalkQuad) : mode, eps * eps > 0.0,
                                 theta_group != nullptr, t->waves_per_block, a.targets_per_lane);
    if (a.grid <= 0) return fail(BH_EHIP, "cannot size the persistent walk grid");
  }
  bh_tree* mt = const_cast<bh_tree*>(t);
  const bool timing = t->timing && allow_timing;
  if (timing) {
    hipError_t e = hipEventRecord(t->ev0, st);
    if (e != hipSuccess) return hip_fail(e, "recording the walk start event");
  }
  hipError_t e = bh::launch_walk(t->prec == BH_FP64, t->order == 2 ? (mode | bh::kWalkQuad) : mode, a, st);
  if (e != hipSuccess) return hip_fail(e, "launching the tree walk");
  if (timing) {
    e = hipEventRecord(t->ev1, st);
    if (e != hipSuccess) return hip_fail(e, "recording the walk end event");
    mt->timed = true;
  }
  return BH_OK;
}

// ---- the allocation-free entry point (bh_forces_noalloc)
// Its workspace is this file-scope device array: each GPU the library runs on
// holds its own copy, allocated when the code object is loaded there and kept
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not a device address: the device address comes from hipGetSymbolAddress,
// once per device with that device current, and is the only one ever handed
// to kernels.
static_assert(BH_NOALLOC_SCRATCH_BYTES % kAlign == 0, "scratch size must keep the workspace alignment");
static __device__ __align__(256) unsigned char scratch[BH_NOALLOC_SCRATCH_BYTES];

std::mutex g_noalloc_mu;                 // guards the two tables below (host state only)
void* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device
bh_tree g_noalloc_tree[kMaxDevices];     // host handle of the tree built in `scratch`, per device

// Device address of this device's scratch array (looked up on the device's first call).
// The caller holds g_noalloc_mu.
int scratch_address(int dev, void** out) {
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "locating the static scratch array");
    if (!p || !aligned(p, kAlign)) return fail(BH_EHIP, "the static scratch array is not 256-byte aligned");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return BH_OK;
}

}  // namespace

extern "C" {

const char* bh_last_error(void) { return g_err; }

int bh_version(void) { return 3; }

int64_t bh_forest_workspace_bytes(int64_t n, int64_t n_clusters, int prec) {
  if (n < 0 || n > kMaxN || n_clusters < 1 || n_clusters > kMaxClusters || (prec != BH_FP32 && prec != BH_FP64))
    return -1;
  return (int64_t)layout(n, n_clusters, prec, nullptr, nullptr, nullptr, nullptr);
}

int64_t bh_workspace_bytes(int64_t n, int prec) { return bh_forest_workspace_bytes(n, 1, prec); }

int bh_build_forest(const void* pos, const void* mass, const int64_t* offsets, int64_t n_clusters, int64_t n,
                    int prec, void* workspace, int64_t ws_bytes, void* stream, bh_tree** out) {
  if (!out) return fail(BH_EINVAL, "out must not be null");
  *out = nullptr;
  if (n < 0 || n > kMaxN) return fail(BH_EINVAL, "n must be in [0, 2^30 - 1]; got %lld", (long long)n);
  if (n_clusters < 1 || n_clusters > kMaxClusters)
    return fail(BH_EINVAL, "n_clusters must be in [1, 2^24]; got %lld", (long long)n_clusters);
  if (prec != BH_FP32 && prec != BH_FP64) return fail(BH_EINVAL, "prec must be BH_FP32 or BH_FP64");
  const size_t el = prec == BH_FP64 ? 8 : 4;
  if (n > 0 && (!pos || !mass || !aligned(pos, el) || !aligned(mass, el)))
    return fail(BH_EINVAL, "pos/mass must be non-null device arrays aligned to %zu bytes", el);
  if (offsets && !aligned(offsets, 8)) return fail(BH_EINVAL, "offsets must be 8-byte aligned");
  if (!offsets && n_clusters != 1) return fail(BH_EINVAL, "offsets are required for more than one cluster");
  const int64_t need = bh_forest_workspace_bytes(n, n_clusters, prec);
  if (!workspace || ws_bytes < need)
    return fail(BH_ENOSPC, "workspace of %lld bytes needed, %lld given", (long long)need, (long long)ws_bytes);
  if (!aligned(workspace, kAlign)) return fail(BH_EINVAL, "workspace must be 256-byte aligned");
  bh_tree* t = new (std::nothrow) bh_tree();
  if (!t) return fail(BH_EINVAL, "out of host memory");
  t->n = n;
  t->n_seg = n_clusters;
  t->prec = prec;
  t->pos = pos;
  t->mass = mass;
  layout(n, n_clusters, prec, static_cast<char*>(workspace), &t->w, &t->rank, &t->queue);
  if (offsets) t->w.seg_off = offsets;
  hipError_t e = enqueue_build(t, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "launching the tree build");
  }
  *out = t;
  return BH_OK;
}

int bh_build_tree(const void* pos, const void* mass, int64_t n, int prec, void* workspace, int64_t ws_bytes,
                  void* stream, bh_tree** out) {
  return bh_build_forest(pos, mass, nullptr, 1, n, prec, workspace, ws_bytes, stream, out);
}

int bh_tree_check(const bh_tree* t, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  bh::Counts c{};
  int rc = sync_counts(t, static_cast<hipStream_t>(stream), &c);
  if (rc) return rc;
  if (c.bad_input) return fail(BH_EINVAL, "non-finite particle coordinate or mass");
  if (c.bad_theta)
    return fail(BH_EINVAL, "a per-group theta was not finite or outside (0, 2/sqrt(3)); %g was used in its place",
                (double)bh::kThetaFallback);
  return BH_OK;
}

int bh_tree_stats(const bh_tree* t, void* stream, int64_t* n_nodes, int64_t* n_leaves, int64_t* n_internal) {
  if (!t) return fail(BH_EINVAL, "null tree");
  bh::Counts c{};
  int rc = sync_counts(t, static_cast<hipStream_t>(stream), &c);
  if (rc) return rc;
  if (n_nodes) *n_nodes = t->n ? c.n_nodes : 0;
  if (n_leaves) *n_leaves = t->n ? c.n_unique : 0;
  if (n_internal) *n_internal = t->n ? c.n_internal : 0;
  return BH_OK;
}

int bh_forces(const bh_tree* t, double theta, double eps, void* acc, void* pot, void* stream) {
  return run_walk(t, theta, nullptr, eps, acc, pot, bh::kWalkForces, nullptr, nullptr, nullptr, 0,
                  nullptr, static_cast<hipStream_t>(stream));
}

int bh_forces_theta(const bh_tree* t, const float* theta_group, double eps, void* acc, void* pot, void* stream) {
  if (!theta_group) return fail(BH_EINVAL, "theta_group must not be null");
  return run_walk(t, 0.0, theta_group, eps, acc, pot, bh::kWalkForces, nullptr, nullptr, nullptr, 0,
                  nullptr, static_cast<hipStream_t>(stream));
}

int bh_forces_noalloc(const void* pos, const void* mass, int64_t n, int prec, double theta, double eps, void* acc,
                      void* pot, void* stream) {
  if (n < 0 || n > BH_NOALLOC_MAX_N)
    return fail(BH_EINVAL, "n must be in [0, %d] for bh_forces_noalloc; got %lld (use bh_build_tree with a "
                "workspace for larger sets)", BH_NOALLOC_MAX_N, (long long)n);
  if (prec != BH_FP32 && prec != BH_FP64) return fail(BH_EINVAL, "prec must be BH_FP32 or BH_FP64");
  int rc = check_theta_eps(theta, eps);
  if (rc) return rc;
  if (n == 0) return BH_OK;
  const size_t el = prec == BH_FP64 ? 8 : 4;
  if (!pos || !mass || !acc || !pot || !aligned(pos, el) || !aligned(mass, el) || !aligned(acc, el) ||
      !aligned(pot, el))
    return fail(BH_EINVAL, "pos/mass/acc/pot must be non-null device arrays aligned to %zu bytes", el);
  const size_t need = layout(n, 1, prec, nullptr, nullptr, nullptr, nullptr);
  if (need > (size_t)BH_NOALLOC_SCRATCH_BYTES)
    return fail(BH_ENOSPC, "%zu bytes of scratch needed, %d held", need, BH_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "reading the current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(BH_EINVAL, "device %d beyond the %d this entry serves", dev,
                                                 kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  void* base = nullptr;
  if ((rc = scratch_address(dev, &base)) != BH_OK) return rc;
  // the same handle each call: default walk shape, fields reset (no events, no timing)
  bh_tree& t = g_noalloc_tree[dev];
  t = bh_tree{};
  t.n = n;
  t.n_seg = 1;
  t.prec = prec;
  t.pos = pos;
  t.mass = mass;
  layout(n, 1, prec, static_cast<char*>(base), &t.w, &t.rank, &t.queue);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // every array the build and the walk read is written by them first (counters
  // and flags by fill kernels), so the previous call's contents do not matter
  e = enqueue_build(&t, st, false);
  if (e != hipSuccess) return hip_fail(e, "launching the tree build");
  return run_walk(&t, theta, nullptr, eps, acc, pot, bh::kWalkForces, nullptr, nullptr, nullptr, 0, nullptr, st,
                  false);
}

int bh_walk_stats(const bh_tree* t, double theta, const float* theta_group, double eps, void* acc, void* pot,
                  int32_t* counts, uint64_t* hash, int64_t* lists, int64_t maxlen, int32_t* group_steps,
                  void* stream) {
  if (group_steps && !aligned(group_steps, 4)) return fail(BH_EINVAL, "group_steps must be 4-byte aligned");
  return run_walk(t, theta, theta_group, eps, acc, pot, lists ? bh::kWalkDump : bh::kWalkStats, counts, hash,
                  lists, maxlen, group_steps, static_cast<hipStream_t>(stream));
}

int bh_tree_export(const bh_tree* t, void* nodes, int32_t* perm, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  hipStream_t st = static_cast<hipStream_t>(stream);
  bh::Counts c{};
  int rc = sync_counts(t, st, &c);
  if (rc) return rc;
  if (t->n == 0) return BH_OK;
  hipError_t e;
  if (nodes) {
    e = hipMemcpyAsync(nodes, t->w.nodes, sizeof(bh::Node) * (size_t)c.n_nodes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copying nodes");
  }
  if (perm) {
    e = hipMemcpyAsync(perm, t->w.idx_a, 4 * (size_t)t->n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copying perm");
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "synchronising the stream");
  return BH_OK;
}

int bh_leapfrog_step(void* pos, void* vel, void* mass, void* acc, void* pot, int64_t* ids, int64_t n, int prec,
                     double dt, double theta, double eps, int order, int reorder, void* workspace, int64_t ws_bytes,
                     void* stream) {
  if (n < 0 || n > kMaxN) return fail(BH_EINVAL, "n must be in [0, 2^30 - 1]; got %lld", (long long)n);
  if (prec != BH_FP32 && prec != BH_FP64) return fail(BH_EINVAL, "prec must be BH_FP32 or BH_FP64");
  if (!std::isfinite(dt)) return fail(BH_EINVAL, "dt must be finite");
  if (order != 1 && order != 2) return fail(BH_EINVAL, "order must be 1 or 2");
  if (reorder != 0 && reorder != 1) return fail(BH_EINVAL, "reorder must be 0 or 1");
  int rc = check_theta_eps(theta, eps);
  if (rc) return rc;
  if (n == 0) return BH_OK;
  const size_t el = prec == BH_FP64 ? 8 : 4;
  if (!pos || !vel || !mass || !acc || !pot || !aligned(pos, el) || !aligned(vel, el) || !aligned(mass, el) ||
      !aligned(acc, el) || !aligned(pot, el) || (ids && !aligned(ids, 8)))
    return fail(BH_EINVAL, "pos/vel/mass/acc/pot must be non-null device arrays aligned to %zu bytes", el);
  const int64_t need = bh_workspace_bytes(n, prec);
  if (!workspace || ws_bytes < need)
    return fail(BH_ENOSPC, "workspace of %lld bytes needed, %lld given", (long long)need, (long long)ws_bytes);
  if (!aligned(workspace, kAlign)) return fail(BH_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool f64 = prec == BH_FP64;
  bh_tree t;
  t.n = n;
  t.n_seg = 1;
  t.prec = prec;
  t.pos = pos;
  t.mass = mass;
  t.order = order;
  layout(n, 1, prec, static_cast<char*>(workspace), &t.w, &t.rank, &t.queue);
  // kick and drift with the forces of the current positions, rebuild, new forces, kick
  hipError_t e = bh::launch_kick_drift(f64, pos, vel, acc, (int)n, dt, st);
  if (e != hipSuccess) return hip_fail(e, "launching the kick-drift pass");
  e = enqueue_build(&t, st);
  if (e != hipSuccess) return hip_fail(e, "launching the tree build");
  rc = run_walk(&t, theta, nullptr, eps, acc, pot, bh::kWalkForces, nullptr, nullptr, nullptr, 0, nullptr, st, false);
  if (rc) return rc;
  e = bh::launch_kick(f64, vel, acc, (int)n, dt, st);
  if (e != hipSuccess) return hip_fail(e, "launching the kick pass");
  if (reorder) {
    // (the walk copy of the nodes is free once the walk is done: 128 bytes per particle)
    e = bh::launch_reorder(f64, t.w.idx_a, (int)n, pos, vel, mass, acc, pot, ids, t.w.wnodes, st);
    if (e != hipSuccess) return hip_fail(e, "launching the Morton reorder");
  }
  return BH_OK;
}

int bh_neighbours(const bh_tree* t, double radius, int32_t* count, uint64_t* hash, int64_t* lists, int64_t maxlen,
                  void* rho, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (!(radius > 0.0) || !std::isfinite(radius)) return fail(BH_EINVAL, "radius must be finite and > 0; got %g", radius);
  if (t->n == 0) return BH_OK;
  if (!count || !hash || !aligned(count, 4) || !aligned(hash, 8))
    return fail(BH_EINVAL, "count/hash must be non-null aligned device arrays");
  if (lists && (maxlen <= 0 || !aligned(lists, 8)))
    return fail(BH_EINVAL, "lists must be an aligned device array with maxlen > 0");
  const size_t el = t->prec == BH_FP64 ? 8 : 4;
  if (rho && !aligned(rho, el)) return fail(BH_EINVAL, "rho must be aligned to %zu bytes", el);
  hipStream_t st = static_cast<hipStream_t>(stream);
  {
    hipError_t e = ensure_target_order(t, st);
    if (e != hipSuccess) return hip_fail(e, "launching the target order");
  }
  const int32_t* order = walk_order_of(t);
  const int chunk = t->xcd_chunk >= 0 ? t->xcd_chunk : (t->prec == BH_FP64 ? 0 : 1024);
  hipError_t e = bh::launch_neighbours(t->prec == BH_FP64, t->w.nodes, t->w.counts, t->w.wnodes, t->w.ps, t->w.idx_a,
                                       order, t->n_seg > 1 ? t->w.scid : nullptr, t->w.croot, t->w.seg_off,
                                       (int)t->n_seg, (int)t->n, radius, count, hash, lists, lists ? maxlen : 0, rho,
                                       chunk, t->timing ? t->ev0 : nullptr, t->timing ? t->ev1 : nullptr, st);
  if (e != hipSuccess) return hip_fail(e, "launching the neighbour walk");
  if (t->timing) const_cast<bh_tree*>(t)->timed = true;
  return BH_OK;
}

int bh_walk_order(const bh_tree* t, int32_t* order, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (t->n == 0) return BH_OK;
  if (!order || !aligned(order, 4)) return fail(BH_EINVAL, "order must be a non-null device array of int32");
  hipStream_t st = static_cast<hipStream_t>(stream);
  {
    hipError_t e = ensure_target_order(t, st);
    if (e != hipSuccess) return hip_fail(e, "launching the target order");
  }
  const int32_t* pos_order = walk_order_of(t);
  hipError_t e = bh::launch_walk_order(pos_order, t->w.idx_a, (int)t->n, order, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "writing the walk order");
  return BH_OK;
}

int bh_tree_moments2(const bh_tree* t, double* B, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  hipStream_t st = static_cast<hipStream_t>(stream);
  bh::Counts c{};
  int rc = sync_counts(t, st, &c);
  if (rc) return rc;
  if (t->n == 0) return BH_OK;
  if (!B || !aligned(B, 8)) return fail(BH_EINVAL, "B must be a non-null device array of doubles");
  if (!t->quad_ready) {
    hipError_t e = bh::quad_moments(t->prec == BH_FP64, (int)t->n, t->w, st);
    if (e != hipSuccess) return hip_fail(e, "launching the second-moment passes");
    t->quad_ready = true;
  }
  // (the records hold B in their first 48 bytes)
  hipError_t e = hipMemcpy2DAsync(B, 6 * sizeof(double), t->w.qrec, sizeof(bh::QuadRec), 6 * sizeof(double),
                                  (size_t)c.n_nodes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "copying the second moments");
  return BH_OK;
}

int bh_set_walk_config(bh_tree* t, int waves_per_block, int xcd_chunk, int target_order, int lds_share,
                       int persistent, int targets_per_lane) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(BH_EINVAL, "waves_per_block must be 1, 2 or 4");
  if (xcd_chunk < -1) return fail(BH_EINVAL, "xcd_chunk must be >= -1");
  if (target_order < 0 || target_order > 2) return fail(BH_EINVAL, "target_order must be 0, 1 or 2");
  if (lds_share < 0 || lds_share > 64) return fail(BH_EINVAL, "lds_share must be in [0, 64]");
  if (persistent != 0 && persistent != 1) return fail(BH_EINVAL, "persistent must be 0 or 1");
  if (targets_per_lane != 1 && targets_per_lane != 2) return fail(BH_EINVAL, "targets_per_lane must be 1 or 2");
  t->lds_share64 = lds_share;
  t->persistent = persistent;
  t->targets_per_lane = targets_per_lane;
  t->waves_per_block = waves_per_block;
  t->xcd_chunk = xcd_chunk;
  t->target_order = target_order;
  return BH_OK;
}

int bh_set_expansion_order(bh_tree* t, int order) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (order != 1 && order != 2) return fail(BH_EINVAL, "order must be 1 (monopole) or 2 (quadrupole)");
  t->order = order;
  return BH_OK;
}

int bh_set_timing(bh_tree* t, int enable) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (enable && !t->ev0) {
    hipError_t e = hipEventCreate(&t->ev0);
    if (e == hipSuccess) e = hipEventCreate(&t->ev1);
    if (e != hipSuccess) return hip_fail(e, "creating timing events");
  }
  t->timing = enable != 0;
  t->timed = false;
  return BH_OK;
}

int bh_walk_time_ms(const bh_tree* t, float* ms) {
  if (!t || !ms) return fail(BH_EINVAL, "null argument");
  if (!t->timed) return fail(BH_EINVAL, "no timed walk since timing was enabled");
  hipError_t e = hipEventSynchronize(t->ev1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, t->ev0, t->ev1);
  if (e != hipSuccess) return hip_fail(e, "reading the walk timing events");
  return BH_OK;
}

void bh_tree_release(bh_tree* t) {
  if (!t) return;
  if (t->ev0) (void)hipEventDestroy(t->ev0);
  if (t->ev1) (void)hipEventDestroy(t->ev1);
  delete t;
}

int bh_direct(const void* pos, const void* mass, int64_t n, int prec, const int64_t* targets, int64_t nt,
              double eps, void* acc, void* pot, void* stream) {
  if (n < 0 || n > kMaxN || nt < 0 || nt > kMaxN) return fail(BH_EINVAL, "n and nt must be in [0, 2^30 - 1]");
  if (prec != BH_FP32 && prec != BH_FP64) return fail(BH_EINVAL, "prec must be BH_FP32 or BH_FP64");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BH_EINVAL, "eps must be finite and >= 0; got %g", eps);
  if (nt == 0) return BH_OK;
  const size_t el = prec == BH_FP64 ? 8 : 4;
  if (!pos || !mass || !targets || !acc || !pot || !aligned(pos, el) || !aligned(mass, el) ||
      !aligned(targets, 8) || !aligned(acc, el) || !aligned(pot, el))
    return fail(BH_EINVAL, "null or misaligned device array");
  hipError_t e = bh::launch_direct(prec == BH_FP64, pos, mass, (int)n, targets, (int)nt, eps, acc, pot,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the direct sum");
  return BH_OK;
}

int bh_forest_roots(const bh_tree* t, int32_t* roots, void* stream) {
  if (!t || !roots || !aligned(roots, 4)) return fail(BH_EINVAL, "null tree or misaligned roots array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(roots, t->w.croot, 4 * (size_t)(t->n_seg + 1), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "copying cluster roots");
  return BH_OK;
}

int bh_graph_create(bh_tree* t, double theta, double eps, void* acc, void* pot, void* stream, bh_graph** out) {
  if (!out) return fail(BH_EINVAL, "out must not be null");
  *out = nullptr;
  if (!t) return fail(BH_EINVAL, "null tree");
  int rc = check_theta_eps(theta, eps);
  if (rc) return rc;
  const size_t el = t->prec == BH_FP64 ? 8 : 4;
  if (t->n > 0 && (!acc || !pot || !aligned(acc, el) || !aligned(pot, el)))
    return fail(BH_EINVAL, "acc/pot must be non-null device arrays aligned to %zu bytes", el);
  // Capture needs a stream of its own (the caller's may be the null stream);
  // the first use on it waits for the caller's pending work.
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "creating the capture stream");
  e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  bh_graph* g = nullptr;
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t eb = enqueue_build(t, cs);
    int wrc = eb == hipSuccess ? run_walk(t, theta, nullptr, eps, acc, pot, bh::kWalkForces, nullptr, nullptr,
                                          nullptr, 0, nullptr, cs, false)
                               : BH_OK;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    // nothing captured has run: an eager walk before the first replay must
    // form the target order and the second moments itself
    t->horder_ready = false;
    t->quad_ready = false;
    t->rank_ready = false;
    if (eb != hipSuccess) e = eb;
    if (e == hipSuccess && wrc != BH_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipStreamDestroy(cs);
      return wrc;
    }
    if (e == hipSuccess) {
      g = new (std::nothrow) bh_graph();
      if (!g) {
        (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        return fail(BH_EINVAL, "out of host memory");
      }
      g->graph = graph;
      e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        g = nullptr;
      }
    }
  }
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return hip_fail(e, "capturing the force pipeline");
  *out = g;
  return BH_OK;
}

int bh_graph_launch(bh_graph* g, void* stream) {
  if (!g || !g->exec) return fail(BH_EINVAL, "null graph");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the captured pipeline");
  return BH_OK;
}

void bh_graph_release(bh_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

int bh_autotune(bh_tree* t, double theta, double eps, void* acc, void* pot, int reps, void* stream,
                bh_walk_config* best, bh_walk_config* tried, int max_tried, int* n_tried) {
  if (!t || !best) return fail(BH_EINVAL, "null tree or result");
  if (reps < 1 || reps > 100) return fail(BH_EINVAL, "reps must be in [1, 100]");
  if (tried && max_tried < 0) return fail(BH_EINVAL, "max_tried must be >= 0");
  int rc = check_theta_eps(theta, eps);
  if (rc) return rc;
  if (n_tried) *n_tried = 0;
  const bool was_timing = t->timing;
  if ((rc = bh_set_timing(t, 1)) != BH_OK) return rc;
  bh_walk_config cur{t->waves_per_block, t->xcd_chunk, t->lds_share64, t->persistent, t->targets_per_lane, 0.f};
  auto measure = [&](bh_walk_config& c) -> int {
    t->waves_per_block = c.waves_per_block;
    t->xcd_chunk = c.xcd_chunk;
    t->lds_share64 = c.lds_share;
    t->persistent = c.persistent;
    t->targets_per_lane = c.targets_per_lane;
    float bestms = 0.f;
    for (int r = 0; r < reps; ++r) {
      int q = bh_forces(t, theta, eps, acc, pot, stream);
      if (q != BH_OK) return q;
      float ms = 0.f;
      if ((q = bh_walk_time_ms(t, &ms)) != BH_OK) return q;
      if (r == 0 || ms < bestms) bestms = ms;
    }
    c.ms = bestms;
    if (tried && n_tried && *n_tried < max_tried) tried[*n_tried] = c;
    if (n_tried) ++*n_tried;
    return BH_OK;
  };
  // coordinate search: one knob at a time, keeping the best so far
  if ((rc = measure(cur)) != BH_OK) return rc;
  static const int kTargets[] = {1, 2};
  static const int kPersistent[] = {0, 1};
  static const int kWpb[] = {1, 2, 4};
  static const int kShare[] = {0, 8, 16, 32};
  static const int kChunk[] = {0, 8, 256, 1024};
  for (int stage = 0; stage < 5 && rc == BH_OK; ++stage) {
    const int* vals = stage == 0 ? kTargets : stage == 1 ? kPersistent : stage == 2 ? kWpb : stage == 3 ? kShare
                                                                                                        : kChunk;
    const int nv = stage == 0 ? 2 : stage == 1 ? 2 : stage == 2 ? 3 : stage == 3 ? 4 : 4;
    if (stage == 4 && cur.persistent) break;  // the block remap does not apply to the persistent walk
    bh_walk_config stage_best = cur;
    for (int v = 0; v < nv; ++v) {
      bh_walk_config c = cur;
      int* knob = stage == 0 ? &c.targets_per_lane : stage == 1 ? &c.persistent : stage == 2 ? &c.waves_per_block
                  : stage == 3 ? &c.lds_share : &c.xcd_chunk;
      if (*knob == vals[v]) continue;
      *knob = vals[v];
      if ((rc = measure(c)) != BH_OK) break;
      if (c.ms < stage_best.ms) stage_best = c;
    }
    cur = stage_best;
  }
  t->waves_per_block = cur.waves_per_block;
  t->xcd_chunk = cur.xcd_chunk;
  t->lds_share64 = cur.lds_share;
  t->persistent = cur.persistent;
  t->targets_per_lane = cur.targets_per_lane;
  (void)bh_set_timing(t, was_timing ? 1 : 0);
  if (rc != BH_OK) return rc;
  *best = cur;
  return BH_OK;
}

/* ---- learned opening parameter */

int bh_features(const bh_tree* t, float* X, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (t->n == 0) return BH_OK;
  if (!X || !aligned(X, 4)) return fail(BH_EINVAL, "X must be a non-null device array of floats");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = ensure_target_order(t, st);
  if (e != hipSuccess) return hip_fail(e, "launching the target order");
  e = bh::launch_features(t->prec == BH_FP64, t->w.nodes, t->w.ps, t->w.cube, t->n_seg > 1 ? t->w.scid : nullptr,
                          t->w.croot, t->w.seg_off, (int)t->n_seg, (int)t->n, walk_order_of(t), X, st);
  if (e != hipSuccess) return hip_fail(e, "launching the feature pass");
  return BH_OK;
}

int bh_group_error(const bh_tree* t, const void* acc, const double* acc_ref, double theta, double target,
                   double* rms, float* label, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (t->n == 0) return BH_OK;
  const size_t el = t->prec == BH_FP64 ? 8 : 4;
  if (!acc || !acc_ref || !aligned(acc, el) || !aligned(acc_ref, 8))
    return fail(BH_EINVAL, "acc/acc_ref must be non-null aligned device arrays");
  if ((rms && !aligned(rms, 8)) || (label && !aligned(label, 4)))
    return fail(BH_EINVAL, "rms/label must be aligned device arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = ensure_target_order(t, st);
  if (e != hipSuccess) return hip_fail(e, "launching the target order");
  e = bh::launch_group_error(t->prec == BH_FP64, acc, acc_ref, t->w.idx_a, walk_order_of(t), (int)t->n, theta,
                             target, rms, label, st);
  if (e != hipSuccess) return hip_fail(e, "launching the group error pass");
  return BH_OK;
}

int bh_mlp_sizes(int64_t batch, int64_t* n_param, int64_t* n_grad, int64_t* n_wbf16, int64_t* n_partial) {
  if (batch < 0 || batch > kMaxN) return fail(BH_EINVAL, "batch must be in [0, 2^30 - 1]");
  if (n_param) *n_param = bh::kMlpParams;
  if (n_grad) *n_grad = bh::kMlpGradLen;
  if (n_wbf16) *n_wbf16 = bh::kMlpWb;
  if (n_partial) *n_partial = (int64_t)bh::mlp_grad_parts((int)(batch > 0 ? batch : 1)) * bh::kMlpGradLen;
  return BH_OK;
}

int bh_mlp_prepare(const float* params, uint16_t* wbf16, void* stream) {
  if (!params || !wbf16 || !aligned(params, 4) || !aligned(wbf16, 16))
    return fail(BH_EINVAL, "params (4-byte) and wbf16 (16-byte aligned) must be device arrays");
  hipError_t e = bh::launch_mlp_prepare(params, wbf16, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the weight copy");
  return BH_OK;
}

int bh_mlp_infer(const float* params, const uint16_t* wbf16, const float* norm, const float* X, int64_t rows,
                 float alpha, float theta_fallback, float* theta, void* stream) {
  if (rows < 0 || rows > kMaxN) return fail(BH_EINVAL, "rows must be in [0, 2^30 - 1]");
  if (rows == 0) return BH_OK;
  if (!params || !wbf16 || !norm || !X || !theta || !aligned(wbf16, 16) || !aligned(X, 4) || !aligned(theta, 4))
    return fail(BH_EINVAL, "null or misaligned device array");
  if (!(alpha > 0.f) || !std::isfinite(alpha)) return fail(BH_EINVAL, "alpha must be finite and > 0");
  if (!(theta_fallback > 0.f && theta_fallback < kThetaMax))
    return fail(BH_EINVAL, "theta_fallback must be in (0, 2/sqrt(3))");
  hipError_t e = bh::launch_mlp_infer(params, wbf16, norm, X, rows, alpha, theta_fallback, (float)kThetaCap, theta,
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the MLP");
  return BH_OK;
}

int bh_mlp_grad(const float* params, const uint16_t* wbf16, const float* norm, const float* X, const float* target,
                const int32_t* rows_idx, int64_t batch, float* partial, float* grad, void* stream) {
  if (batch < 1 || batch > kMaxN) return fail(BH_EINVAL, "batch must be in [1, 2^30 - 1]");
  if (!params || !wbf16 || !norm || !X || !target || !rows_idx || !partial || !grad || !aligned(wbf16, 16) ||
      !aligned(rows_idx, 4) || !aligned(partial, 4) || !aligned(grad, 4))
    return fail(BH_EINVAL, "null or misaligned device array");
  hipError_t e = bh::launch_mlp_grad(params, wbf16, norm, X, target, rows_idx, (int)batch, partial, grad,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the MLP gradient");
  return BH_OK;
}

int bh_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                float beta2, float eps, uint16_t* wbf16, void* stream) {
  if (!params || !grad || !m || !v || !wbf16 || !aligned(wbf16, 16)) return fail(BH_EINVAL, "null device array");
  if (step < 1) return fail(BH_EINVAL, "step counts from 1");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(BH_EINVAL, "invalid Adam hyper-parameters");
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipError_t e = bh::launch_mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, c1, c2, wbf16,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the Adam step");
  return BH_OK;
}

}  // extern "C"
