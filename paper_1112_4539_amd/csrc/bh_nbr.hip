// bh_nbr.hip -- the general tree walk of Sec. 4.3 (Fig. 4) as a neighbour search.
//
// Per target particle i and search radius r, the walk of Fig. 4 with
//   * proc_particle: particle j != i is a neighbour iff |x_j - x_i|^2 < r^2;
//     its work here is the SPH density sum rho_i += m_j W(|x_j - x_i|, r/2),
//     W the M4 cubic spline of support 2h = r (Monaghan & Lattanzio 1985);
//   * distance_test: a cell is skipped when it cannot hold a point within r;
//   * proc_cell: nothing.
// It runs on the force walk's machinery: one wavefront walks 64 targets of
// the walk order with a shared cursor over the depth-first preorder, a target
// being active at node c iff c >= its skip pointer.  The walk copy carries,
// per cell, R2 = ((r + s + (sqrt(3)/2) l)(1 + 2^-40))^2: every point of the
// cell's cube lies within (sqrt(3)/2) l of the cube's centre, itself s from
// the centre of mass, so a target whose squared distance to the centre of
// mass is at least R2 has no neighbour in the cell (the factor keeps the
// bound safe under rounding).  A leaf of one particle carries r^2, the exact
// test, so cells and leaves take the same test.  A cell of at most kNbrGroup
// particles is a group: when a lane can reach it, the wave tests its
// particles directly, read in Morton order from the particle array (which is
// the depth-first order of its leaves), and moves on past its subtree; a leaf
// of several particles (coincident Morton keys) is a group that every active
// lane enters.  The neighbour sets therefore equal the definition's, and each
// target meets its neighbours in depth-first (Morton) order whatever the
// grouping.
#include "bh_walk_impl.h"

namespace bh {

namespace {

// One node of the neighbour walk, 64 bytes, read with scalar loads.
//   cx, cy, cz : centre of mass (a one-particle leaf: its particle, exact)
//   R2         : squared skip radius (cell), r^2 (one-particle leaf), +inf
//                (leaf of several particles)
//   m          : mass (a one-particle leaf: its particle's, exact)
//   next       : first node after the subtree, in (c, cap]
//   first      : Morton position of the first particle
//   count      : particles in the subtree
//   tag        : -1 cell, >= 0 the caller index of a one-particle leaf's
//                particle, -2 a group: a cell of at most kNbrGroup particles
//                or a leaf of several, whose particles are tested directly
struct alignas(64) NbrRec {
  double cx, cy, cz, R2, m;
  int32_t next, first, count, tag;
};
static_assert(sizeof(NbrRec) == 64, "NbrRec must be 64 bytes");
static_assert(sizeof(NbrRec) == sizeof(WalkNode), "the neighbour walk copy shares the walk copy's storage");
constexpr int32_t kTagCell = -1, kTagGroup = -2;
// Cells of at most this many particles are walked as groups: their particles
// are tested directly, four (FP32) or two (FP64) per round trip, instead of
// one dependent record load per node of their subtree.  On the clumpy 4M
// field at r = 2e-3 the search takes 8.7 ms with no groups, 6.8 ms with
// groups of 8, 6.0 ms with 24-32 and 6.3 ms with 64.
constexpr int kNbrGroup = 32;

template <bool kOff32>
__device__ __forceinline__ NbrRec nbr_load(const NbrRec* base, int c) {
  const BH_CONST char* b = kOff32 ? rec_at32(base, c) : (const BH_CONST char*)(uintptr_t)base + (uint64_t)c * 64u;
  const v8u_t w0 = *(const BH_CONST v8u_t*)b;             // cx, cy, cz, R2
  const v2u_t w1 = *(const BH_CONST v2u_t*)(b + 32);      // m
  const v2u_t w2 = *(const BH_CONST v2u_t*)(b + 40);      // next, first
  const v2u_t w3 = *(const BH_CONST v2u_t*)(b + 48);      // count, tag
  NbrRec r;
  r.cx = f64_of(w0.s01);
  r.cy = f64_of(w0.s23);
  r.cz = f64_of(w0.s45);
  r.R2 = f64_of(w0.s67);
  r.m = f64_of(w1);
  r.next = (int)w2.x;
  r.first = (int)w2.y;
  r.count = (int)w3.x;
  r.tag = (int)w3.y;
  return r;
}

__device__ __forceinline__ NbrRec nbr_record(const Node& nd, int c, const int32_t* __restrict__ perm, int cap,
                                             double radius, int group_max) {
  NbrRec w;
  w.cx = nd.cx;
  w.cy = nd.cy;
  w.cz = nd.cz;
  if (!(nd.meta & 1)) {
    const double u = (radius + nd.s + 0.8660254037844387 * nd.l) * (1.0 + 0x1p-40);
    w.R2 = u * u;
    w.tag = nd.count <= group_max ? kTagGroup : kTagCell;
  } else if (nd.count == 1) {
    w.R2 = radius * radius;
    w.tag = perm[nd.first];
  } else {
    w.R2 = __builtin_huge_val();
    w.tag = kTagGroup;
  }
  w.m = nd.M;
  w.next = min(max(nd.next, c + 1), cap);
  w.first = nd.first;
  w.count = nd.count;
  return w;
}

// The walk reads the records of the cluster roots, of the cells it descends
// (cells of more than group_max particles: every node it visits below a root
// has only such cells above it) and of their children, and never a node
// inside a group.  So each such cell writes its own record and those of its
// children that are groups or leaves (a child that is itself such a cell
// writes its own), and k_nbr_roots writes the roots; the records of nodes
// inside groups are left as they are.  (Every next pointer the walk follows
// leads to a sibling of a visited node or of one of its ancestors, a child of
// a descended cell, or to the end of the cluster's range.)
__global__ __launch_bounds__(256) void k_nbr_copy(const Node* __restrict__ nodes, const Counts* __restrict__ cnt,
                                                  const int32_t* __restrict__ perm, int cap, double radius,
                                                  int group_max, NbrRec* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int nn = min(cap, cnt->n_nodes);
  if (c >= nn) return;
  const Node nd = nodes[c];
  if ((nd.meta & 1) || nd.count <= group_max) return;
  out[c] = nbr_record(nd, c, perm, cap, radius, group_max);
  const int end = min(max(nd.next, c + 1), nn);
  int ch = c + 1;
  for (int k = 0; k < 8 && ch < end; ++k) {
    const Node cd = nodes[ch];
    if ((cd.meta & 1) || cd.count <= group_max) out[ch] = nbr_record(cd, ch, perm, cap, radius, group_max);
    ch = min(max(cd.next, ch + 1), end);
  }
}

__global__ __launch_bounds__(64) void k_nbr_roots(const Node* __restrict__ nodes, const Counts* __restrict__ cnt,
                                                  const int32_t* __restrict__ perm, const int32_t* __restrict__ croot,
                                                  int n_seg, int cap, double radius, int group_max,
                                                  NbrRec* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_seg) return;
  const int c = croot[k];
  if (c < 0 || c >= min(cap, cnt->n_nodes)) return;
  out[c] = nbr_record(nodes[c], c, perm, cap, radius, group_max);
}

struct NbrArgs {
  const NbrRec* wn;            // neighbour walk copy [2n + 1]
  const void* ps;              // float4 / double4 particles in Morton order
  const int32_t* perm;         // Morton position -> caller index
  const int32_t* order;        // walk order of the targets (Morton positions), may be null
  const int32_t* scid;         // Morton position -> cluster (forest), may be null
  const int32_t* croot;        // [K + 1] preorder range of each cluster's subtree
  const int64_t* seg_off;      // [K + 1] caller offsets of the clusters
  int n_seg;
  int n;
  double r2;                   // r^2
  double inv_h;                // 1/h, h = r/2
  double sig;                  // 1/(pi h^3), the spline's normalisation
  int32_t* count;              // [n] neighbours, caller order
  uint64_t* hash;              // [n] ordered hash of the neighbours' (cluster-relative) caller indices
  int64_t* lists;              // [n][maxlen], may be null
  int64_t maxlen;
  void* rho;                   // [n] SPH density, may be null
  int xcd_chunk;
};

struct NbrTarget {
  double xi, yi, zi;
  double wsum;         // m_i + sum over neighbours of m_j w(q_j); the density is sig * wsum
  int i, skip, idx0;
  int32_t count;
  uint64_t h;
  int64_t* list;
};

// w(q) = W(|d|, h) / sig of the M4 cubic spline in three dimensions, from
// d^2 >= 0, in its truncated-power form: w = (2 - q)_+^3 / 4 - (1 - q)_+^3
// (equal to 1 - 3/2 q^2 + 3/4 q^3 for q < 1, (2 - q)^3 / 4 for 1 <= q < 2 and
// 0 beyond, q = |d|/h), which needs no branch or select.  |d| = sqrt(d^2) by
// Goldschmidt's iteration from the hardware reciprocal square root (one
// refinement of the root and of the half reciprocal, then a residual
// correction: within an ulp or two of the rounded root, far inside the
// density's tolerance).  2^-1000 is added to d^2, so that the iteration never
// meets 0 * inf: the sum is d^2 itself for d^2 > 2^-947, and below that q is
// ~1e-142 or less, where w = 1 to the last bit whatever the root.
__device__ __forceinline__ double sph_w2(double d2, double inv_h) {
  const double d2g = d2 + 0x1p-1000;
  const double y = __builtin_amdgcn_rsq(d2g);
  double g = d2g * y, hh = 0.5 * y;
  const double e = fma(-g, hh, 0.5);
  g = fma(g, e, g);
  hh = fma(hh, e, hh);
  g = fma(fma(-g, g, d2g), hh, g);
  const double q = g * inv_h;
  const double u = fmax(2.0 - q, 0.0), b = fmax(1.0 - q, 0.0);
  return fma(0.25, (u * u) * u, -((b * b) * b));
}

template <bool kLists>
__device__ __forceinline__ void nbr_pair(const NbrArgs& a, NbrTarget& T, int caller, double m, double d2) {
  // (j, the caller index relative to the cluster, is in [0, n) with n < 2^30,
  // so j << 1 is exact in 32 bits and leaves the hash's high word alone)
  const uint32_t j = (uint32_t)(caller - T.idx0);
  if constexpr (kLists) {
    if (T.count < a.maxlen) T.list[T.count] = (int64_t)j;
  }
  ++T.count;
  T.h = (T.h ^ (uint64_t)(j << 1)) * kFnvPrime;
  T.wsum = fma(m, sph_w2(d2, a.inv_h), T.wsum);
}

// The particles [first, first + count) of a group, in Morton (depth-first)
// order, against the lanes `in` (active, and within reach of the group).
// Their positions, masses and caller indices are read with scalar loads a few
// at a time, all loads of a batch in flight together (the last particle is
// re-read to fill a batch, never one past it).
template <bool kF64, bool kLists, bool kOff32>
__device__ __forceinline__ void nbr_group(const NbrArgs& a, NbrTarget& T, bool in, int first, int count) {
  typedef float v4f_t __attribute__((ext_vector_type(4)));
  typedef double v4d_t __attribute__((ext_vector_type(4)));
  using V4 = typename std::conditional<kF64, v4d_t, v4f_t>::type;
  constexpr int kBatch = kF64 ? 2 : 4;   // 64 bytes of particles per batch
  const int end = first + count;
  for (int k0 = first; k0 < end; k0 += kBatch) {
    V4 q[kBatch];
    int caller[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const uint32_t k = (uint32_t)min(k0 + j, end - 1);
      if constexpr (kOff32) {
        // (32-bit byte offsets: the loads take them in a scalar register)
        q[j] = *(const BH_CONST V4*)((const BH_CONST char*)(uintptr_t)a.ps + k * (uint32_t)sizeof(V4));
        caller[j] = *(const BH_CONST int32_t*)((const BH_CONST char*)(uintptr_t)a.perm + k * 4u);
      } else {
        q[j] = *((const BH_CONST V4*)(uintptr_t)a.ps + k);
        caller[j] = *((const BH_CONST int32_t*)(uintptr_t)a.perm + k);
      }
    }
    // (every value of the batch taken here, in scalar registers: one wait for
    // the whole batch, instead of loads sunk into the per-particle branches)
#pragma unroll
    for (int j = 0; j < kBatch; ++j) asm volatile("" ::"s"(q[j].x), "s"(q[j].y), "s"(q[j].z), "s"(q[j].w), "s"(caller[j]));
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      if (k0 + j < end) {
        const double dx = (double)q[j].x - T.xi, dy = (double)q[j].y - T.yi, dz = (double)q[j].z - T.zi;
        const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
        if (in && d2 < a.r2 && k0 + j != T.i) nbr_pair<kLists>(a, T, caller[j], (double)q[j].w, d2);
      }
    }
  }
}

// One step at node c: the test (cell or group: can the target reach it;
// one-particle leaf: is its particle a neighbour), the successor's record
// requested as soon as the wave knows it, then the neighbour work.  The walk
// descends into a cell that a lane can reach; a group is never descended:
// when a lane can reach it, its particles are tested directly, and the walk
// goes on after its subtree.
template <bool kF64, bool kLists, bool kOff32, typename Fetch>
__device__ __forceinline__ void nbr_step(const NbrArgs& a, NbrTarget& T, int& c, const NbrRec& rec, Fetch fetch) {
  const int nnext = uniform(rec.next), first = uniform(rec.first), tag = uniform(rec.tag);
  // (the mass goes with the step's first batch of scalar loads: a load left to
  // the leaf's branch would cost the step a second round trip)
  asm volatile("" ::"s"(rec.m));
  const bool act = T.skip <= c;
  const double dx = rec.cx - T.xi, dy = rec.cy - T.yi, dz = rec.cz - T.zi;
  const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const bool in = d2 < rec.R2;
  // (the lanes that enter, as the AND of two compare masks: a ballot of the
  // combined flag would first turn it into a number)
  const uint64_t m_in = ballot(act) & __builtin_amdgcn_fcmp(d2, rec.R2, 4);  // ordered <
  const bool cell = tag == kTagCell;
  // (next pointers exceed c in every record the walk reads; the max keeps the
  // cursor moving forward whatever a record holds)
  const int cn = max((m_in && cell) ? c + 1 : nnext, c + 1);
  fetch(cn);
  if (cell) {
    if (act && !in) T.skip = nnext;
  } else if (m_in) {
    // (a group is not descended: every lane active here is active after it)
    if (tag >= 0) {
      if (act && in && first != T.i) nbr_pair<kLists>(a, T, tag, rec.m, d2);
    } else {
      nbr_group<kF64, kLists, kOff32>(a, T, act && in, first, uniform(rec.count));
    }
  }
  c = cn;
}

// The subtree [c, end) of one cluster.  The copy has a spare record at
// cap = 2n and every next pointer is at most cap, so the look-ahead read stays
// inside it.
template <bool kF64, bool kLists, bool kOff32>
__device__ void nbr_subtree(const NbrArgs& a, NbrTarget& T, int c, int end) {
  NbrRec cur = nbr_load<kOff32>(a.wn, c);
  while (c < end) {
    NbrRec nx;
    nbr_step<kF64, kLists, kOff32>(a, T, c, cur, [&](int cn) { nx = nbr_load<kOff32>(a.wn, cn); });
    cur = nx;
  }
}

// kLists: the caller asked for neighbour lists (a.lists non-null).
template <bool kF64, bool kLists>
__global__ __launch_bounds__(64) void k_nbr(NbrArgs a) {
  using T4 = typename std::conditional<kF64, double4, float4>::type;
  using R = typename std::conditional<kF64, double, float>::type;
  const int group = remap_block(blockIdx.x, gridDim.x, a.xcd_chunk);
  const int lane = __lane_id();
  const int slot = group * kWave + lane;
  const bool valid = slot < a.n;
  NbrTarget T;
  T.i = valid ? (a.order ? a.order[slot] : slot) : -1;
  T4 me;
  if (valid) {
    me = reinterpret_cast<const T4*>(a.ps)[T.i];
  } else {
    me.x = me.y = me.z = me.w = 0;
  }
  T.xi = (double)me.x;
  T.yi = (double)me.y;
  T.zi = (double)me.z;
  T.wsum = (double)me.w;   // the target's own term, w(0) = 1
  T.count = 0;
  T.h = kFnvOffset;
  T.list = (kLists && valid) ? a.lists + (int64_t)a.perm[T.i] * a.maxlen : nullptr;
  const int kc = (valid && a.scid) ? min(max(a.scid[T.i], 0), a.n_seg - 1) : 0;
  T.idx0 = valid ? (int)a.seg_off[kc] : 0;
  int klo = valid ? kc : 0x7fffffff, khi = valid ? kc : -1;
  for (int o = 32; o > 0; o >>= 1) {
    klo = min(klo, __shfl_xor(klo, o, 64));
    khi = max(khi, __shfl_xor(khi, o, 64));
  }
  klo = uniform(klo);
  khi = uniform(khi);
  const int cap = 2 * a.n;
  const bool off32 = a.n < kOff32MaxN;
  for (int k = klo; k <= khi; ++k) {
    const int r0 = min(max(uniform(a.croot[k]), 0), cap);
    const int r1 = min(max(uniform(a.croot[k + 1]), r0), cap);
    T.skip = (valid && kc == k) ? r0 : 0x7fffffff;
    if (r0 >= r1) continue;
    if (off32)
      nbr_subtree<kF64, kLists, true>(a, T, r0, r1);
    else
      nbr_subtree<kF64, kLists, false>(a, T, r0, r1);
  }
  if (!valid) return;
  const int o = a.perm[T.i];
  a.count[o] = T.count;
  a.hash[o] = T.h;
  if (a.rho) reinterpret_cast<R*>(a.rho)[o] = (R)(a.sig * T.wsum);
}

}  // namespace

hipError_t launch_neighbours(bool f64, const Node* nodes, const Counts* counts, WalkNode* copy, const void* ps,
                             const int32_t* perm, const int32_t* order, const int32_t* scid, const int32_t* croot,
                             const int64_t* seg_off, int n_seg, int n, double radius, int32_t* count,
                             uint64_t* hash, int64_t* lists, int64_t maxlen, void* rho, int xcd_chunk,
                             hipEvent_t ev0, hipEvent_t ev1, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int cap = 2 * n;
  NbrRec* rec = reinterpret_cast<NbrRec*>(copy);
  k_nbr_copy<<<(cap + 255) / 256, 256, 0, st>>>(nodes, counts, perm, cap, radius, kNbrGroup, rec);
  k_nbr_roots<<<(n_seg + 63) / 64, 64, 0, st>>>(nodes, counts, perm, croot, n_seg, cap, radius, kNbrGroup, rec);
  NbrArgs a{};
  a.wn = rec;
  a.ps = ps;
  a.perm = perm;
  a.order = order;
  a.scid = scid;
  a.croot = croot;
  a.seg_off = seg_off;
  a.n_seg = n_seg;
  a.n = n;
  a.r2 = radius * radius;
  const double h = 0.5 * radius;
  a.inv_h = 1.0 / h;
  a.sig = 1.0 / (3.141592653589793 * h * h * h);
  a.count = count;
  a.hash = hash;
  a.lists = lists;
  a.maxlen = maxlen;
  a.rho = rho;
  a.xcd_chunk = xcd_chunk;
  const int groups = (n + kWave - 1) / kWave;
  // (ev0/ev1, when given, bracket the walk kernel alone)
  if (ev0) {
    const hipError_t e = hipEventRecord(ev0, st);
    if (e != hipSuccess) return e;
  }
  if (f64) {
    if (lists) k_nbr<true, true><<<groups, kWave, 0, st>>>(a); else k_nbr<true, false><<<groups, kWave, 0, st>>>(a);
  } else {
    if (lists) k_nbr<false, true><<<groups, kWave, 0, st>>>(a); else k_nbr<false, false><<<groups, kWave, 0, st>>>(a);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ev1) return e;
  return hipEventRecord(ev1, st);
}

}  // namespace bh
