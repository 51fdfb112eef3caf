// bh_walk.hip -- the force walk (gfx950), the hot loop of the method.
//
// What is computed (per target particle i) is the iterative walk of Sec. 4.4
// (Fig. 5, next/more pointers) with the opening test of Eq. (2)/(3):
//   * at a leaf: a particle-particle term of Eq. (1) with every particle j != i;
//   * at a cell that does not hold i and satisfies d^2 > (l/theta + s)^2:
//     a particle-cell term with (M, centre of mass), same softened kernel,
//     then continue at next(c);
//   * otherwise open the cell: continue at more(c) = c + 1.
//
// How it runs on CDNA: one wavefront walks 64 Morton-consecutive targets
// together.  The wave keeps one cursor c over the preorder node array; lane i
// is active at c iff c >= skip_i, where skip_i = next of the last cell lane i
// accepted.  At an internal node every active lane evaluates the opening test;
// accepting lanes add the cell term (masked) and set skip_i = next(c).  The
// cursor goes to c+1 if any active lane opened c (wave ballot), else to
// next(c).  Every lane therefore meets exactly the nodes of its own
// single-particle walk, in the same order, so lists and summation order do not
// depend on how targets are grouped.  Node records are wave-uniform and are
// read with scalar loads; there is no divergence in the traversal itself.
//
// Precision (FP32 variant): positions and masses are FP32.  The opening test
// runs in FP64 on the FP64 centre of mass and the exactly widened position,
// d^2 = fma(dz,dz,fma(dy,dy,dx*dx)), so the interaction lists are those of
// the FP64 reference walk.  The same FP64 offset and d^2 feed the term:
// r^2 + eps^2 is rounded once to FP32, the inverse square root is v_rsq_f32,
// and the contributions are accumulated in FP64 (on CDNA4 FP64 add and FMA
// issue at the unpacked FP32 rate).  The FP64 variant evaluates every term
// exactly as the reference definition (IEEE sqrt and division, no
// contraction) and accumulates in FP64.
#include "bh_internal.h"

namespace bh {

__device__ __forceinline__ int remap_block(int b, int nb, int chunk) {
  // Workgroups are dispatched to the 8 XCDs round-robin.  Give each XCD runs of
  // `chunk` consecutive workgroups (Morton-adjacent groups share tree nodes in
  // that XCD's L2), interleaving the runs across XCDs to keep the load even.
  if (chunk <= 0) return b;
  const int full = (nb / (8 * chunk)) * 8 * chunk;
  if (b >= full) return b;
  const int k = b >> 3, x = b & 7;
  return ((k / chunk) * 8 + x) * chunk + (k % chunk);
}

// FP32 term, FP64 sums.  The offset dx and d^2 = |dx|^2 come exact (FP64
// from FP32 input) or once-rounded from the opening test; r^2 + eps^2 is
// rounded once to FP32, r^-1 is the hardware v_rsq_f32, m r^-1 and m r^-3 are
// FP32 products, and the contributions m r^-3 dx and -m r^-1 are accumulated
// in FP64 (CDNA4 issues FP64 add and FMA at the FP32 rate, so this costs no
// more than FP32 sums with periodic compensation, and leaves no summation
// error worth counting).
struct AccMixed {
  double ax, ay, az, p;
  __device__ void init() { ax = ay = az = p = 0.0; }
  template <bool kSoft>
  __device__ __forceinline__ void term(double dx, double dy, double dz, double d2, float m, double eps2) {
    const float r2 = (float)(d2 + eps2);
    // r2 == 0 only for a coincident pair without softening: that pair adds nothing
    const float ri = kSoft ? __builtin_amdgcn_rsqf(r2) : ((r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f);
    const float mr = m * ri;
    const double mr3 = (double)((mr * ri) * ri);
    ax = fma(mr3, dx, ax);
    ay = fma(mr3, dy, ay);
    az = fma(mr3, dz, az);
    p -= (double)mr;
  }
};

struct AccF64 {
  double ax, ay, az, p;
  __device__ void init() { ax = ay = az = p = 0.0; }
  // Same operations and order as the reference pair term: r2 = dx*dx + dy*dy +
  // dz*dz + eps2, rinv = 1/sqrt(r2), m*(rinv*rinv*rinv).
  __device__ __forceinline__ void term(double dx, double dy, double dz, double m, double eps2) {
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    if (r2 == 0.0) return;
    const double rinv = 1.0 / sqrt(r2);
    const double mr3 = m * (rinv * rinv * rinv);
    ax += mr3 * dx;
    ay += mr3 * dy;
    az += mr3 * dz;
    p -= m * rinv;
  }
};

constexpr uint64_t kFnvOffset = 14695981039346656037ull;
constexpr uint64_t kFnvPrime = 1099511628211ull;

// The opening size S = (l/theta + s)^2 of a node is precomputed per node for a
// uniform theta (one pass per call) or formed on the fly from a per-group theta.
__global__ __launch_bounds__(256) void k_mac_size(const Node* __restrict__ nodes, const Counts* __restrict__ cnt,
                                                  int cap, double inv_theta, WalkNode* __restrict__ wnodes) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cap || c >= cnt->n_nodes) return;
  const Node nd = nodes[c];
  const double u = fma(nd.l, inv_theta, nd.s);
  WalkNode w;
  w.cx = nd.cx;
  w.cy = nd.cy;
  w.cz = nd.cz;
  w.M = nd.M;
  w.S = u * u;
  w.M32 = (float)nd.M;
  w.pad = 0;
  w.next = nd.next;
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

// What a step needs of a node, from the walk copy (uniform theta) or from the
// plain node (per-group theta: S formed from l and s per lane).
template <bool kPlain>
struct StepNode;
// Records are read through the constant address space: the node arrays are
// not written while a walk runs, and saying so lets the compiler keep the
// wave-uniform record loads on the scalar path even in loops that also store
// results or take work from a counter.
#define BH_CONST __attribute__((address_space(4)))
template <typename Rec>
__device__ __forceinline__ Rec const_load(const Rec* base, int c) {
  const BH_CONST Rec* p = (const BH_CONST Rec*)(uintptr_t)base + c;
  Rec r;
  if constexpr (sizeof(Rec) == sizeof(WalkNode) && std::is_same<Rec, WalkNode>::value) {
    r.cx = p->cx; r.cy = p->cy; r.cz = p->cz; r.M = p->M; r.S = p->S; r.M32 = p->M32; r.pad = 0;
  } else {
    r.cx = p->cx; r.cy = p->cy; r.cz = p->cz; r.M = p->M; r.l = p->l; r.s = p->s;
  }
  r.next = p->next; r.first = p->first; r.count = p->count; r.meta = p->meta;
  return r;
}
template <>
struct StepNode<false> {
  const WalkNode* base;
  __device__ __forceinline__ WalkNode load(int c) const { return const_load(base, c); }
};
template <>
struct StepNode<true> {
  const Node* base;
  __device__ __forceinline__ Node load(int c) const { return const_load(base, c); }
};

// One walk: a cursor over the preorder node array shared by the wave, and the
// per-lane state of the lane's target.
template <bool kF64>
struct Cursor {
  using R = typename std::conditional<kF64, double, float>::type;
  typename std::conditional<kF64, AccF64, AccMixed>::type acc;
  double xi, yi, zi;   // target position (exactly widened)
  double inv_theta;
  int i;               // Morton position of the target, -1 for an idle lane
  int slot;            // position of the target in the walk order
  int c;               // wave-uniform cursor
  int skip;            // the lane is active at c iff skip <= c
  int k, kend;         // position inside a leaf of several particles
  int steps;
  int node0;           // preorder id of the root of the target's cluster (list words are relative)
  int idx0;            // caller index of the first particle of the target's cluster
  int32_t n_pp, n_pc;
  uint64_t h;
  int64_t len;
  int64_t* list;
};

// One step of a walk at node `cur` (index cur_c = C.c).  kGuard: some target
// of the wave has theta > 1, so a cell holding the target must be excluded
// explicitly (for theta <= 1 such a cell fails the opening test by itself:
// d <= (sqrt(3)/2) l + s < l/theta + s, a margin of 0.13 l that no rounding
// reaches).
//
// Each step produces one source for the shared term: the cell (after the
// opening test), the particle of a one-particle leaf, or one particle of a
// leaf of coincident-key particles (the cursor stays on such a leaf until its
// particles are done).  One term site keeps the sums in place.
template <bool kF64, int kMode, bool kSoft, bool kPlain, bool kGuard, typename Rec>
__device__ __forceinline__ void walk_step(const WalkArgs& a, Cursor<kF64>& C, const Rec& rec) {
  // The record was read from LDS by every lane; its integer fields steer the
  // wave's control flow, so take them as wave-uniform values.
  Rec cur = rec;
  cur.next = uniform(rec.next);
  cur.first = uniform(rec.first);
  cur.count = uniform(rec.count);
  cur.meta = uniform(rec.meta);
  using R = typename Cursor<kF64>::R;
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  constexpr bool kStats = kMode != kWalkForces;
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);
  const int c = C.c;
  const int i = C.i;
  if constexpr (kStats) ++C.steps;
  const int nnext = max(cur.next, c + 1);
  const int kind = cur.meta & 3;  // 0 cell, 1 one-particle leaf, 3 several-particle leaf
  const bool act = C.skip <= c;
  const uint64_t m_act = ballot(act);
  // Offset to the node's position (cell: centre of mass; one-particle leaf:
  // its particle), formed in FP64.  For FP32 input the FP64 difference of the
  // widened coordinates is exact, so its FP32 rounding equals a direct FP32
  // subtraction; a cell's offset is rounded once.  Formed for every node so
  // that the whole record is read at the top of the step.
  double dx = cur.cx - C.xi, dy = cur.cy - C.yi, dz = cur.cz - C.zi;
  // Opening test of Eq. (2) in FP64, also evaluated (and ignored) for leaves
  // so that no field load is left for later in the step.
  double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
  double S;
  if constexpr (kPlain) {
    const double u = fma(cur.l, C.inv_theta, cur.s);
    S = u * u;
  } else {
    S = cur.S;
  }
  bool pass = d2 > S;
  if constexpr (kGuard) pass = pass && !((unsigned)(i - cur.first) < (unsigned)cur.count);
  // (a ballot is convergent: it keeps the test, and the loads it needs, here)
  const uint64_t m_pass = ballot(pass);
  R tm;
  bool use;
  uint64_t m_use;
  int cnext = nnext;
  int src = cur.first;  // Morton position of a particle source
  if (kind == 0) {
    // Cell: a cell term for the lanes that accept it.
    use = act && pass;
    m_use = m_act & m_pass;
    if (m_act & ~m_pass) cnext = c + 1;
    if constexpr (kF64 || kPlain) tm = (R)cur.M; else tm = (R)cur.M32;
  } else if (kind == 1) {
    // One-particle leaf: a particle term unless the particle is i.
    use = act && cur.first != i;
    m_use = m_act & ballot(cur.first != i);
    if constexpr (kF64 || kPlain) tm = (R)cur.M; else tm = (R)cur.M32;
  } else {
    // Leaf of coincident-key particles: one of its particles per step.
    if (C.kend == 0) {
      C.k = min(max(cur.first, 0), a.n);
      C.kend = C.k + min(max(cur.count, 0), a.n - C.k);
    }
    const int kk = min(C.k, a.n - 1);
    src = kk;
    const R4 q = ps[kk];
    use = act && C.k < C.kend && kk != i;
    m_use = m_act & ballot(C.k < C.kend && kk != i);
    // the step's source is this particle: its offset replaces the node's
    dx = (double)q.x - C.xi;
    dy = (double)q.y - C.yi;
    dz = (double)q.z - C.zi;
    d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    tm = q.w;
    if (++C.k < C.kend) {
      cnext = c;
    } else {
      C.k = C.kend = 0;
    }
  }
  if (m_use) {
    if (use) {
      if constexpr (kF64) {
        C.acc.term(dx, dy, dz, tm, a.eps2);
      } else {
        C.acc.template term<kSoft>(dx, dy, dz, d2, tm, a.eps2);
      }
      if (kind == 0) C.skip = nnext;
      if constexpr (kStats) {
        const uint64_t wd = kind == 0 ? (((uint64_t)(c - C.node0) << 1) | 1ull)
                                      : ((uint64_t)(a.perm[src] - C.idx0) << 1);
        if (kind == 0) ++C.n_pc; else ++C.n_pp;
        C.h = (C.h ^ wd) * kFnvPrime;
        if (kMode == kWalkDump && C.len < a.maxlen) C.list[C.len] = (int64_t)wd;
        ++C.len;
      }
    }
  }
  C.c = cnext;
}

// Node records reach the walk through LDS.  The walk reads one record per
// step and nearly every record misses the small scalar cache, whose miss
// handling then sets the pace; the vector path has the throughput but a
// longer latency.  So each step copies both possible successors of the
// current node (c+1 and next(c)) with the LDS-DMA load (global_load_lds_dwordx4:
// lanes 0-3 bring the four 16-byte quarters of one record, lanes 4-7 those
// of the other) into the wave's spare buffer, and the next step reads the one
// it needs with broadcast LDS reads.  The copy's latency overlaps one step.
typedef __attribute__((address_space(3))) void lds_void;

template <typename Rec>
__device__ __forceinline__ void fetch_pair(const Rec* base, int ca, int cb, int lane, uint4* dst) {
  if (lane < 8) {
    const int r = lane < 4 ? ca : cb;
    const char* src = reinterpret_cast<const char*>(base + r) + (lane & 3) * 16;
    __builtin_amdgcn_global_load_lds(src, (lds_void*)dst, 16, 0, 0);
  }
}

// The plain form: each step reads its node with scalar loads (the record is
// wave-uniform), one round trip per step.
// Both forms walk the subtree [C.c, end) of one cluster; `end` is clamped to
// the node capacity, so a corrupted record can never send the cursor out of the
// array, and every step moves the cursor forward or stays on a leaf for at most
// its particle count.
template <bool kF64, int kMode, bool kSoft, bool kPlain, bool kGuard>
__device__ __forceinline__ void walk_loop_scalar(const WalkArgs& a, StepNode<kPlain> wn, Cursor<kF64>& C,
                                                 int end) {
  while (C.c < end) walk_step<kF64, kMode, kSoft, kPlain, kGuard>(a, C, wn.load(C.c));
}

template <bool kF64, int kMode, bool kSoft, bool kPlain, bool kGuard>
__device__ __forceinline__ void walk_loop_lds(const WalkArgs& a, StepNode<kPlain> wn, Cursor<kF64>& C,
                                              uint4 (*pf)[8], int end) {
  using Rec = decltype(wn.load(0));
  const int cap = 2 * a.n;
  const int lane = __lane_id();
  int buf = 0, slot = 0;  // LDS buffer and slot holding the current record
  fetch_pair(wn.base, C.c, C.c, lane, pf[0]);
  while (C.c < end) {
    const int c = C.c;
    // The copy issued last step is the only vector memory operation in flight
    // here; the compiler does not order LDS-DMA writes before later LDS reads,
    // so wait for it explicitly (s_waitcnt vmcnt(0)).
    __builtin_amdgcn_s_waitcnt(0x0f70);
    const Rec rec = reinterpret_cast<const Rec*>(pf[buf])[slot];
    const int nnext = max(uniform(rec.next), c + 1);
    fetch_pair(wn.base, min(c + 1, cap - 1), min(nnext, cap - 1), lane, pf[buf ^ 1]);
    walk_step<kF64, kMode, kSoft, kPlain, kGuard>(a, C, rec);
    if (C.c != c) {  // moved on (a leaf of several particles keeps the cursor)
      slot = C.c == c + 1 ? 0 : 1;
      buf ^= 1;
    }
  }
}

// The clusters klo..khi of a wave, one subtree after the other; lanes of the
// other clusters stay idle (skip past the subtree).
template <bool kF64, int kMode, bool kSoft, bool kPlain, bool kGuard, bool kLds>
__device__ __forceinline__ void walk_clusters(const WalkArgs& a, StepNode<kPlain> wn, Cursor<kF64>& C,
                                              uint4 (*pf)[8], bool valid, int kc, int klo, int khi) {
  const int cap = 2 * a.n;
  for (int k = klo; k <= khi; ++k) {
    const int r0 = min(max(uniform(a.croot[k]), 0), cap);
    const int r1 = min(max(uniform(a.croot[k + 1]), r0), cap);
    C.c = r0;
    C.k = C.kend = 0;
    C.skip = (valid && kc == k) ? r0 : 0x7fffffff;
    if (r0 >= r1) continue;
    if constexpr (kLds)
      walk_loop_lds<kF64, kMode, kSoft, kPlain, kGuard>(a, wn, C, pf, r1);
    else
      walk_loop_scalar<kF64, kMode, kSoft, kPlain, kGuard>(a, wn, C, r1);
  }
}

// The walk of one group of 64 targets (one wavefront).
// kSoft: eps > 0, so r^2 + eps^2 > 0 and the FP32 term needs no zero test.
// kGroupTheta: theta per 64-particle Morton group instead of one uniform theta
// (uniform theta walks the copy with S precomputed).
template <bool kF64, int kMode, bool kSoft, bool kGroupTheta>
__device__ __forceinline__ void walk_group(const WalkArgs& a, int group, uint4 (*pf)[8]) {
  using R = typename Cursor<kF64>::R;
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  constexpr bool kStats = kMode != kWalkForces;
  const int lane = __lane_id();
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);

  Cursor<kF64> C;
  C.slot = group * kWave + lane;
  const bool valid = C.slot < a.n;
  C.i = valid ? (a.order ? a.order[C.slot] : C.slot) : -1;
  R4 me;
  if (valid) {
    me = ps[C.i];
  } else {
    me.x = me.y = me.z = me.w = (R)0;
  }
  C.xi = (double)me.x;
  C.yi = (double)me.y;
  C.zi = (double)me.z;
  C.inv_theta = kGroupTheta ? 1.0 / (double)a.theta_group[valid ? (C.i >> 6) : 0] : a.inv_theta;
  C.acc.init();
  C.k = C.kend = 0;
  C.steps = 0;
  C.n_pp = C.n_pc = 0;
  C.h = kFnvOffset;
  C.len = 0;
  C.list = (kMode == kWalkDump && valid) ? a.lists + (int64_t)a.perm[C.i] * a.maxlen : nullptr;
  const bool guard = ballot(valid && C.inv_theta < 1.0) != 0ull;
  // Clusters of the wave's targets: a wave usually lies inside one cluster; one
  // that straddles cluster edges walks each cluster's subtree in turn.
  const int kc = valid ? min(max(a.scid[C.i], 0), a.n_seg - 1) : 0;
  int klo = valid ? kc : 0x7fffffff, khi = valid ? kc : -1;
  for (int o = 32; o > 0; o >>= 1) {
    klo = min(klo, __shfl_xor(klo, o, 64));
    khi = max(khi, __shfl_xor(khi, o, 64));
  }
  klo = uniform(klo);
  khi = uniform(khi);
  C.node0 = valid ? a.croot[kc] : 0;
  C.idx0 = valid ? (int)a.seg_off[kc] : 0;
  StepNode<kGroupTheta> wn;
  if constexpr (kGroupTheta) wn.base = a.nodes; else wn.base = a.wnodes;
  // Waves split between the two node paths (scalar cache / LDS copies) so
  // that neither the scalar cache nor instruction issue alone sets the pace;
  // the share taking the LDS path is a launch parameter (results identical).
  // (taken as a wave-uniform value: the compiler cannot tell that the wave
  // index is uniform, and a branch it took for divergent would turn the walk
  // state that crosses it into per-lane values)
  const bool lds_path = uniform(((group * 37) & 63) < a.lds_share64 ? 1 : 0) != 0;
  // (one cluster loop per path and guard: the LDS path's copies must not share
  // a loop with the scalar path's loads, or the compiler stops treating the
  // node array as unwritten and drops the scalar loads)
  if (lds_path) {
    if (guard)
      walk_clusters<kF64, kMode, kSoft, kGroupTheta, true, true>(a, wn, C, pf, valid, kc, klo, khi);
    else
      walk_clusters<kF64, kMode, kSoft, kGroupTheta, false, true>(a, wn, C, pf, valid, kc, klo, khi);
  } else {
    if (guard)
      walk_clusters<kF64, kMode, kSoft, kGroupTheta, true, false>(a, wn, C, pf, valid, kc, klo, khi);
    else
      walk_clusters<kF64, kMode, kSoft, kGroupTheta, false, false>(a, wn, C, pf, valid, kc, klo, khi);
  }

  if (kStats && a.group_steps && lane == 0 && valid) a.group_steps[group] = C.steps;
  if (!valid) return;
  const int o = a.perm[C.i];
  R* accp = reinterpret_cast<R*>(a.acc);
  R* potp = reinterpret_cast<R*>(a.pot);
  accp[3 * (int64_t)o] = (R)C.acc.ax;
  accp[3 * (int64_t)o + 1] = (R)C.acc.ay;
  accp[3 * (int64_t)o + 2] = (R)C.acc.az;
  potp[o] = (R)C.acc.p;
  if constexpr (kStats) {
    a.counts[2 * (int64_t)o] = C.n_pp;
    a.counts[2 * (int64_t)o + 1] = C.n_pc;
    a.hash[o] = C.h;
  }
}

// One wavefront per group; workgroups of waves_per_block waves.
template <bool kF64, int kMode, bool kSoft, bool kGroupTheta>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
  __shared__ uint4 pf_lds[4][2][8];  // per wave: two buffers of two 64-byte node records
  const int wv = threadIdx.x >> 6;
  const int blk = remap_block(blockIdx.x, gridDim.x, a.xcd_chunk);
  // (a wave past the last target has no valid lane and walks nothing)
  walk_group<kF64, kMode, kSoft, kGroupTheta>(a, blk * a.waves_per_block + wv, pf_lds[wv]);
}

// Persistent form: a grid that fits on the chip at once; every wave takes the
// next group from a device counter until none is left, so the load balances
// itself and no workgroup waits for a dispatch slot.  Every wave leaves once
// the counter passes the last group.
template <bool kF64, int kMode, bool kSoft, bool kGroupTheta>
__global__ __launch_bounds__(256) void k_walk_persistent(WalkArgs a) {
  __shared__ uint4 pf_lds[4][2][8];
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int groups = (a.n + kWave - 1) / kWave;
  for (;;) {
    int g = 0;
    if (lane == 0) g = atomicAdd(a.queue, 1);
    g = __shfl(g, 0, 64);
    if (g >= groups) break;
    walk_group<kF64, kMode, kSoft, kGroupTheta>(a, g, pf_lds[wv]);
  }
}

template <bool kF64, int kMode, bool kSoft, bool kGroupTheta>
static hipError_t launch_t(const WalkArgs& a, hipStream_t st) {
  const int groups = (a.n + kWave - 1) / kWave;
  const int wpb = a.waves_per_block;
  const int blocks = (groups + wpb - 1) / wpb;
  if (a.persistent) {
    hipError_t e = fill_i32(a.queue, 1, 0, st);
    if (e != hipSuccess) return e;
    k_walk_persistent<kF64, kMode, kSoft, kGroupTheta><<<max(1, min(a.grid, blocks)), wpb * kWave, 0, st>>>(a);
  } else {
    k_walk<kF64, kMode, kSoft, kGroupTheta><<<blocks, wpb * kWave, 0, st>>>(a);
  }
  return hipGetLastError();
}

template <bool kF64, int kMode>
static const void* persistent_fn(bool soft, bool group_theta) {
  if (soft)
    return group_theta ? reinterpret_cast<const void*>(&k_walk_persistent<kF64, kMode, true, true>)
                       : reinterpret_cast<const void*>(&k_walk_persistent<kF64, kMode, true, false>);
  return group_theta ? reinterpret_cast<const void*>(&k_walk_persistent<kF64, kMode, false, true>)
                     : reinterpret_cast<const void*>(&k_walk_persistent<kF64, kMode, false, false>);
}

// Workgroups of the persistent walk that are resident on the chip at once (0 if
// the runtime cannot tell).
int persistent_grid(bool f64, int mode, bool soft, bool group_theta, int waves_per_block) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn;
  if (f64)
    fn = mode == kWalkForces ? persistent_fn<true, kWalkForces>(soft, group_theta)
       : mode == kWalkStats  ? persistent_fn<true, kWalkStats>(soft, group_theta)
                             : persistent_fn<true, kWalkDump>(soft, group_theta);
  else
    fn = mode == kWalkForces ? persistent_fn<false, kWalkForces>(soft, group_theta)
       : mode == kWalkStats  ? persistent_fn<false, kWalkStats>(soft, group_theta)
                             : persistent_fn<false, kWalkDump>(soft, group_theta);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, waves_per_block * kWave, 0) != hipSuccess) return 0;
  return cus * per_cu;
}

template <bool kF64, int kMode>
static hipError_t launch_mode(const WalkArgs& a, hipStream_t st) {
  const bool soft = a.eps2 > 0.0;
  if (a.theta_group)
    return soft ? launch_t<kF64, kMode, true, true>(a, st) : launch_t<kF64, kMode, false, true>(a, st);
  return soft ? launch_t<kF64, kMode, true, false>(a, st) : launch_t<kF64, kMode, false, false>(a, st);
}

hipError_t launch_walk(bool f64, int mode, const WalkArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (f64) {
    if (mode == kWalkForces) return launch_mode<true, kWalkForces>(a, st);
    if (mode == kWalkStats) return launch_mode<true, kWalkStats>(a, st);
    return launch_mode<true, kWalkDump>(a, st);
  }
  if (mode == kWalkForces) return launch_mode<false, kWalkForces>(a, st);
  if (mode == kWalkStats) return launch_mode<false, kWalkStats>(a, st);
  return launch_mode<false, kWalkDump>(a, st);
}

}  // namespace bh
