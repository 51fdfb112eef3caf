// bh_api.hip -- host side of the C ABI declared in include/bh.h.
//
// Argument checks, workspace carving, and the launch sequences of the build,
// the walk and the direct sum.  Device memory is never allocated here: every
// array is a view into the caller's workspace.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/bh.h"
#include "bh_internal.h"

namespace bh {
hipError_t make_rank(const int32_t* perm, int n, int32_t* rank, hipStream_t st);
}

struct bh_tree {
  int64_t n = 0;
  int prec = BH_FP32;
  bh::BuildWs w{};
  int32_t* rank = nullptr;  // caller index -> Morton position
  int waves_per_block = 4;
  int xcd_chunk = 0;
  int target_order = 0;
  int lds_share64 = 16;
  bool timing = false;
  bool timed = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
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

constexpr int64_t kMaxN = int64_t(1) << 30;
constexpr size_t kAlign = 256;
const double kThetaMax = 2.0 / std::sqrt(3.0);

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves the workspace; with base == nullptr it only measures.
size_t layout(int64_t n, int prec, char* base, bh::BuildWs* w, int32_t** rank) {
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
  t.cube = reinterpret_cast<bh::Cube*>(take(sizeof(bh::Cube)));
  t.counts = reinterpret_cast<bh::Counts*>(take(sizeof(bh::Counts)));
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
  t.ipre = reinterpret_cast<int32_t*>(take(4 * N));
  t.nstart = reinterpret_cast<int32_t*>(take(4 * (N + 1)));
  t.nexcl = reinterpret_cast<int32_t*>(take(4 * (N + 1)));
  t.lmask = reinterpret_cast<uint32_t*>(take(4 * (N + 1)));
  t.nodes = reinterpret_cast<bh::Node*>(take(sizeof(bh::Node) * nodes));
  t.Mx = reinterpret_cast<double*>(take(24 * nodes));
  t.wnodes = reinterpret_cast<bh::WalkNode*>(take(sizeof(bh::WalkNode) * nodes));
  int32_t* r = reinterpret_cast<int32_t*>(take(4 * N));
  if (w) *w = t;
  if (rank) *rank = r;
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

int run_walk(const bh_tree* t, double theta, const float* theta_group, double eps, void* acc, void* pot,
             int mode, int32_t* counts, uint64_t* hash, int64_t* lists, int64_t maxlen, int32_t* group_steps,
             hipStream_t st) {
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
  }
  bh::WalkArgs a{};
  a.nodes = t->w.nodes;
  a.wnodes = t->w.wnodes;
  a.ps = t->w.ps;
  a.perm = t->w.idx_a;
  a.order = t->target_order == 1 ? t->rank : nullptr;
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
  a.xcd_chunk = t->xcd_chunk;
  a.lds_share64 = t->lds_share64;
  a.waves_per_block = t->waves_per_block;
  bh_tree* mt = const_cast<bh_tree*>(t);
  if (t->timing) {
    hipError_t e = hipEventRecord(t->ev0, st);
    if (e != hipSuccess) return hip_fail(e, "recording the walk start event");
  }
  hipError_t e = bh::launch_walk(t->prec == BH_FP64, mode, a, st);
  if (e != hipSuccess) return hip_fail(e, "launching the tree walk");
  if (t->timing) {
    e = hipEventRecord(t->ev1, st);
    if (e != hipSuccess) return hip_fail(e, "recording the walk end event");
    mt->timed = true;
  }
  return BH_OK;
}

}  // namespace

extern "C" {

const char* bh_last_error(void) { return g_err; }

int bh_version(void) { return 1; }

int64_t bh_workspace_bytes(int64_t n, int prec) {
  if (n < 0 || n > kMaxN || (prec != BH_FP32 && prec != BH_FP64)) return -1;
  return (int64_t)layout(n, prec, nullptr, nullptr, nullptr);
}

int bh_build_tree(const void* pos, const void* mass, int64_t n, int prec, void* workspace, int64_t ws_bytes,
                  void* stream, bh_tree** out) {
  if (!out) return fail(BH_EINVAL, "out must not be null");
  *out = nullptr;
  if (n < 0 || n > kMaxN) return fail(BH_EINVAL, "n must be in [0, 2^30]; got %lld", (long long)n);
  if (prec != BH_FP32 && prec != BH_FP64) return fail(BH_EINVAL, "prec must be BH_FP32 or BH_FP64");
  const size_t el = prec == BH_FP64 ? 8 : 4;
  if (n > 0 && (!pos || !mass || !aligned(pos, el) || !aligned(mass, el)))
    return fail(BH_EINVAL, "pos/mass must be non-null device arrays aligned to %zu bytes", el);
  const int64_t need = bh_workspace_bytes(n, prec);
  if (!workspace || ws_bytes < need)
    return fail(BH_ENOSPC, "workspace of %lld bytes needed, %lld given", (long long)need, (long long)ws_bytes);
  if (!aligned(workspace, kAlign)) return fail(BH_EINVAL, "workspace must be 256-byte aligned");
  bh_tree* t = new (std::nothrow) bh_tree();
  if (!t) return fail(BH_EINVAL, "out of host memory");
  t->n = n;
  t->prec = prec;
  layout(n, prec, static_cast<char*>(workspace), &t->w, &t->rank);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = prec == BH_FP64
                     ? bh::build_tree_f64(static_cast<const double*>(pos), static_cast<const double*>(mass), (int)n,
                                          t->w, st)
                     : bh::build_tree_f32(static_cast<const float*>(pos), static_cast<const float*>(mass), (int)n,
                                          t->w, st);
  if (e == hipSuccess && n > 0) e = bh::make_rank(t->w.idx_a, (int)n, t->rank, st);
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "launching the tree build");
  }
  *out = t;
  return BH_OK;
}

int bh_tree_check(const bh_tree* t, void* stream) {
  if (!t) return fail(BH_EINVAL, "null tree");
  bh::Counts c{};
  int rc = sync_counts(t, static_cast<hipStream_t>(stream), &c);
  if (rc) return rc;
  if (c.bad_input) return fail(BH_EINVAL, "non-finite particle coordinate or mass");
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

int bh_set_walk_config(bh_tree* t, int waves_per_block, int xcd_chunk, int target_order, int lds_share) {
  if (!t) return fail(BH_EINVAL, "null tree");
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(BH_EINVAL, "waves_per_block must be 1, 2 or 4");
  if (xcd_chunk < 0) return fail(BH_EINVAL, "xcd_chunk must be >= 0");
  if (target_order != 0 && target_order != 1) return fail(BH_EINVAL, "target_order must be 0 or 1");
  if (lds_share < 0 || lds_share > 64) return fail(BH_EINVAL, "lds_share must be in [0, 64]");
  t->lds_share64 = lds_share;
  t->waves_per_block = waves_per_block;
  t->xcd_chunk = xcd_chunk;
  t->target_order = target_order;
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
  if (n < 0 || n > kMaxN || nt < 0 || nt > kMaxN) return fail(BH_EINVAL, "n and nt must be in [0, 2^30]");
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

}  // extern "C"
