// bh_walk_impl.h -- the force walk (gfx950), the hot loop of the method.
//
// What is computed (per target particle i) is the iterative walk of Sec. 4.4
// (Fig. 5, next/more pointers) with the opening test of Eq. (2)/(3):
//   * at a leaf: a particle-particle term of Eq. (1) with every particle j != i;
//   * at a cell that does not hold i and satisfies d^2 > (l/theta + s)^2:
//     a particle-cell term with (M, centre of mass), same softened kernel,
//     then continue at next(c);
//   * otherwise open the cell: continue at more(c) = c + 1.
//
// How it runs on CDNA: one wavefront walks 64 (or 128: two per lane)
// Morton-consecutive targets together.  The wave keeps one cursor c over the
// preorder node array; a target is active at c iff c >= its skip pointer, the
// next of the last cell it accepted.  Every active target evaluates the
// opening test; the ones that pass add the term (masked) and skip the node's
// subtree.  The cursor goes to c+1 if an active target opened c (a lane mask
// from the compare), else to next(c).  Every target therefore meets exactly
// the nodes of its own single-particle walk, in the same order, so lists and
// summation order do not depend on how targets are grouped.  Node records are
// wave-uniform and are read with scalar loads, the next one as soon as the
// opening masks fix the cursor, so that its latency overlaps the terms; there
// is no divergence in the traversal itself.  In a forest a wave walks, in
// turn, the subtree of every cluster its targets belong to.
//
// Precision (FP32 variant): positions and masses are FP32.  The opening test
// runs in FP64 on the FP64 centre of mass and the exactly widened position,
// d^2 = fma(dz,dz,fma(dy,dy,dx*dx)), so the interaction lists are those of
// the FP64 reference walk.  The same FP64 offset and d^2 feed the term:
// r^2 + eps^2 is rounded once to FP32, the inverse square root is v_rsq_f32,
// and the contributions are accumulated in FP64 (on CDNA4 FP64 add and FMA
// issue at nearly the unpacked FP32 rate).  The FP64 variant evaluates every
// term exactly as the reference definition (IEEE sqrt and division, no
// contraction) and accumulates in FP64.
#pragma once
#include <type_traits>

#include "bh_internal.h"

namespace bh {


// FP32 term, FP64 sums.  The offset dx and d^2 = |dx|^2 come exact (FP64
// from FP32 input) or once-rounded from the opening test; r^2 + eps^2 is
// rounded once to FP32, r^-1 is the hardware v_rsq_f32, m r^-1 and m r^-3 are
// FP32 products, and the contributions m r^-3 dx and -m r^-1 are accumulated
// in FP64 (CDNA4 issues FP64 add and FMA at the FP32 rate, so this costs no
// more than FP32 sums with periodic compensation, and leaves no summation
// error worth counting).
struct MixedTerm {
  double mr3, mr;  // m r^-3 and m r^-1
  float ri;        // r^-1 (softened)
  double r2;       // r^2 + eps^2 before its FP32 rounding
};

// Quadrupole correction of a cell term (walks of order 2): the second-order
// part of the Taylor expansion of the cell's softened potential about its
// centre of mass.  With d = com - x_i (FP64), rho^-1 = ri, second moments B
// and T = tr B:
//   acc += rho^-5 (7.5 dBd rho^-2 - 1.5 T) d - 3 rho^-5 B d
//   pot += rho^-3 (T/2 - 1.5 dBd rho^-2)
// evaluated in FP64 (it is a small correction to the monopole; FP64 costs the
// FP32 rate here and needs no conversions of d), in fused form.
struct QuadPart {
  double c;            // coefficient of d
  double k;            // coefficient of B d (-3 rho^-5)
  double pq;           // potential correction
  double bx, by, bz;   // B d
};
__device__ __forceinline__ QuadPart quad_part(double dx, double dy, double dz, double ri, const QuadRec& q) {
  QuadPart r;
  r.bx = fma(q.bxz, dz, fma(q.bxy, dy, q.bxx * dx));
  r.by = fma(q.byz, dz, fma(q.byy, dy, q.bxy * dx));
  r.bz = fma(q.bzz, dz, fma(q.byz, dy, q.bxz * dx));
  const double dbd = fma(dz, r.bz, fma(dy, r.by, dx * r.bx));
  const double ri2 = ri * ri;
  const double ri3 = ri * ri2;
  const double ri5 = ri3 * ri2;
  r.c = ri5 * fma(7.5 * dbd, ri2, q.nt15);
  r.k = -3.0 * ri5;
  r.pq = ri3 * fma(-1.5 * dbd, ri2, q.t05);
  return r;
}

struct AccMixed {
  double ax, ay, az, p;
  __device__ void init() { ax = ay = az = p = 0.0; }
  template <bool kSoft>
  static __device__ __forceinline__ MixedTerm prep(double d2, float m, double eps2) {
    const float r2 = (float)(d2 + eps2);
    // r2 == 0 only for a coincident pair without softening: that pair adds nothing
    const float ri = kSoft ? __builtin_amdgcn_rsqf(r2) : ((r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f);
    const float mr = m * ri;
    return MixedTerm{(double)((mr * ri) * ri), (double)mr, ri, d2 + eps2};
  }
  // (the monopole potential's m r^-1 is taken as (m r^-3)(r^2 + eps^2) in one
  // FP64 fused multiply-add, which spares the term a conversion: with r^-1 from
  // v_rsq_f32 good to about 1e-7, the product carries about three times that
  // relative error, far inside the FP32 tolerance)
  __device__ __forceinline__ void add(const MixedTerm& q, double dx, double dy, double dz) {
    ax = fma(q.mr3, dx, ax);
    ay = fma(q.mr3, dy, ay);
    az = fma(q.mr3, dz, az);
    p = fma(-q.mr3, q.r2, p);
  }
  // a cell term of order 2: the monopole factors of `q` plus the correction `u`
  __device__ __forceinline__ void add_quad(const MixedTerm& q, const QuadPart& u, double dx, double dy, double dz) {
    const double c = q.mr3 + u.c;
    ax = fma(c, dx, ax);
    ay = fma(c, dy, ay);
    az = fma(c, dz, az);
    ax = fma(u.k, u.bx, ax);
    ay = fma(u.k, u.by, ay);
    az = fma(u.k, u.bz, az);
    p = fma(-q.mr3, q.r2, p + u.pq);
  }
  template <bool kSoft>
  __device__ __forceinline__ void term(double dx, double dy, double dz, double d2, float m, double eps2) {
    add(prep<kSoft>(d2, m, eps2), dx, dy, dz);
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
  // Order-2 cell term, in the reference expression's operations and order.
  __device__ __forceinline__ void term_quad(double dx, double dy, double dz, double m, double eps2,
                                            const QuadRec& q) {
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    if (r2 == 0.0) return;
    const double ri = 1.0 / sqrt(r2);
    const double ri2 = ri * ri;
    const double ri3 = ri * ri2;
    const double ri5 = ri3 * ri2;
    const double ri7 = ri5 * ri2;
    const double bx = q.bxx * dx + q.bxy * dy + q.bxz * dz;
    const double by = q.bxy * dx + q.byy * dy + q.byz * dz;
    const double bz = q.bxz * dx + q.byz * dy + q.bzz * dz;
    const double dbd = dx * bx + dy * by + dz * bz;
    const double T = 2.0 * q.t05;
    const double g = 7.5 * dbd * ri7 - 1.5 * T * ri5;
    ax += m * ri3 * dx - 3.0 * ri5 * bx + g * dx;
    ay += m * ri3 * dy - 3.0 * ri5 * by + g * dy;
    az += m * ri3 * dz - 3.0 * ri5 * bz + g * dz;
    p += -m * ri + 0.5 * (T * ri3 - 3.0 * dbd * ri5);
  }
};

// The second-moment record of node c (walks of order 2), through the constant
// address space like the walk records.
__device__ __forceinline__ QuadRec quad_load(const QuadRec* base, int c) {
  const __attribute__((address_space(4))) QuadRec* p =
      (const __attribute__((address_space(4))) QuadRec*)(uintptr_t)base + (uint32_t)c;
  QuadRec r;
  r.bxx = p->bxx; r.bxy = p->bxy; r.bxz = p->bxz; r.byy = p->byy; r.byz = p->byz; r.bzz = p->bzz;
  r.t05 = p->t05; r.nt15 = p->nt15;
  return r;
}

constexpr uint64_t kFnvOffset = 14695981039346656037ull;
constexpr uint64_t kFnvPrime = 1099511628211ull;

// What a step needs of a node: the walk copy for one theta (S and the FP32
// mass precomputed), the per-group-theta copy (FP32: l, s and the FP32 mass),
// or the plain node (FP64 per-group theta).
template <bool kF64, bool kPlain>
struct StepNode;
// Records are read through the constant address space: the node arrays are
// not written while a walk runs, and saying so lets the compiler keep the
// wave-uniform record loads on the scalar path even in loops that also store
// results or take work from a counter.
#define BH_CONST __attribute__((address_space(4)))
template <typename Rec>
__device__ __forceinline__ Rec const_load(const Rec* base, int c) {
  const BH_CONST Rec* p = (const BH_CONST Rec*)(uintptr_t)base + (uint32_t)c;
  Rec r;
  if constexpr (std::is_same<Rec, WalkNode>::value) {
    r.cx = p->cx; r.cy = p->cy; r.cz = p->cz; r.S = p->S; r.M32 = p->M32; r.pad = 0; r.M = p->M;
  } else if constexpr (std::is_same<Rec, ThetaNode>::value) {
    r.cx = p->cx; r.cy = p->cy; r.cz = p->cz; r.l = p->l; r.M32 = p->M32; r.s = p->s; r.pad = 0;
  } else {
    r.cx = p->cx; r.cy = p->cy; r.cz = p->cz; r.M = p->M; r.l = p->l; r.s = p->s;
  }
  r.next = p->next; r.first = p->first; r.count = p->count; r.meta = p->meta;
  return r;
}
// The same loads with a 32-bit byte offset (walk copies below 4 GiB): the
// scalar load then takes the offset in an SGPR, and the step saves the 64-bit
// address arithmetic.  The record is read as vectors of dwords (a struct read
// through a byte offset is split into many small loads); pieces a walk does
// not use are dropped by the compiler.
typedef unsigned v8u_t __attribute__((ext_vector_type(8)));
typedef unsigned v2u_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double f64_of(v2u_t w) { return __builtin_bit_cast(double, w); }
__device__ __forceinline__ const BH_CONST char* rec_at32(const void* base, int c) {
  return (const BH_CONST char*)(uintptr_t)base + (uint32_t)c * 64u;
}
__device__ __forceinline__ WalkNode load32(const WalkNode* base, int c) {
  const BH_CONST char* b = rec_at32(base, c);
  const v8u_t w0 = *(const BH_CONST v8u_t*)b;             // cx, cy, cz, S
  const v2u_t w1 = *(const BH_CONST v2u_t*)(b + 32);      // M32, next
  const v2u_t w2 = *(const BH_CONST v2u_t*)(b + 40);      // first, count
  const v2u_t w3 = *(const BH_CONST v2u_t*)(b + 48);      // meta, pad
  const v2u_t w4 = *(const BH_CONST v2u_t*)(b + 56);      // M
  WalkNode r;
  r.cx = f64_of(w0.s01);
  r.cy = f64_of(w0.s23);
  r.cz = f64_of(w0.s45);
  r.S = f64_of(w0.s67);
  r.M32 = __builtin_bit_cast(float, w1.x);
  r.next = (int)w1.y;
  r.first = (int)w2.x;
  r.count = (int)w2.y;
  r.meta = (int)w3.x;
  r.pad = 0;
  r.M = f64_of(w4);
  return r;
}
__device__ __forceinline__ ThetaNode load32(const ThetaNode* base, int c) {
  const BH_CONST char* b = rec_at32(base, c);
  const v8u_t w0 = *(const BH_CONST v8u_t*)b;             // cx, cy, cz, l
  const v2u_t w1 = *(const BH_CONST v2u_t*)(b + 32);      // M32, next
  const v2u_t w2 = *(const BH_CONST v2u_t*)(b + 40);      // first, count
  const v2u_t w3 = *(const BH_CONST v2u_t*)(b + 48);      // s
  const v2u_t w4 = *(const BH_CONST v2u_t*)(b + 56);      // meta, pad
  ThetaNode r;
  r.cx = f64_of(w0.s01);
  r.cy = f64_of(w0.s23);
  r.cz = f64_of(w0.s45);
  r.l = f64_of(w0.s67);
  r.M32 = __builtin_bit_cast(float, w1.x);
  r.next = (int)w1.y;
  r.first = (int)w2.x;
  r.count = (int)w2.y;
  r.s = f64_of(w3);
  r.meta = (int)w4.x;
  r.pad = 0;
  return r;
}
static_assert(sizeof(WalkNode) == 64 && sizeof(ThetaNode) == 64, "load32 assumes 64-byte records");
// Walk copies of n particles hold 2n + 1 records of 64 bytes: below 4 GiB for
// n < 2^25.
constexpr int kOff32MaxN = 1 << 25;

template <bool kF64>
struct StepNode<kF64, false> {
  const WalkNode* base;
  __device__ __forceinline__ WalkNode load(int c) const { return const_load(base, c); }
  template <bool kOff32>
  __device__ __forceinline__ WalkNode load_at(int c) const {
    if constexpr (kOff32) return load32(base, c); else return const_load(base, c);
  }
};
template <>
struct StepNode<false, true> {
  const ThetaNode* base;
  __device__ __forceinline__ ThetaNode load(int c) const { return const_load(base, c); }
  template <bool kOff32>
  __device__ __forceinline__ ThetaNode load_at(int c) const {
    if constexpr (kOff32) return load32(base, c); else return const_load(base, c);
  }
};
template <>
struct StepNode<true, true> {
  const Node* base;
  __device__ __forceinline__ Node load(int c) const { return const_load(base, c); }
  template <bool kOff32>
  __device__ __forceinline__ Node load_at(int c) const { return const_load(base, c); }
};

// Per-target state of a walk.
template <bool kF64>
struct Target {
  typename std::conditional<kF64, AccF64, AccMixed>::type acc;
  double xi, yi, zi;   // target position (exactly widened)
  double inv_theta;
  int i;               // Morton position of the target, -1 for an idle slot
  int slot;            // position of the target in the walk order
  int skip;            // the target is active at c iff skip <= c
  int node0;           // preorder id of the root of the target's cluster (list words are relative)
  int idx0;            // caller index of the first particle of the target's cluster
  int32_t n_pp, n_pc;
  uint64_t h;
  int64_t len;
  int64_t* list;
};

// One walk: a cursor over the preorder node array shared by the wave, and the
// kT targets of each lane (a wave walks 64 kT Morton-consecutive targets: lane
// l holds targets l, 64 + l, ...).
template <bool kF64, int kT>
struct Cursor {
  using R = typename std::conditional<kF64, double, float>::type;
  Target<kF64> t[kT];
  int c;               // wave-uniform cursor
  int k, kend;         // position inside a leaf of several particles
  int steps;
};

// A step at a leaf of several coincident-key particles (rare): one of its
// particles per step, the cursor staying on the leaf until they are done.
template <bool kF64, int kT, int kMode, bool kSoft, typename Rec, typename Fetch>
__device__ __forceinline__ void bucket_step(const WalkArgs& a, Cursor<kF64, kT>& C, const Rec& cur, Fetch&& fetch) {
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  constexpr bool kStats = (kMode & 3) != kWalkForces;
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);
  constexpr int kBase = kMode & 3;
  const int c = C.c;
  if (C.kend == 0) {
    C.k = min(max(cur.first, 0), a.n);
    C.kend = C.k + min(max(cur.count, 0), a.n - C.k);
  }
  const int kk = min(C.k, a.n - 1);
  const bool more = C.k + 1 < C.kend;
  fetch(more ? c : c + 1);
  const R4 q = ps[kk];
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    Target<kF64>& T = C.t[t];
    if (T.skip <= c && C.k < C.kend && kk != T.i) {
      const double dx = (double)q.x - T.xi, dy = (double)q.y - T.yi, dz = (double)q.z - T.zi;
      if constexpr (kF64) {
        T.acc.term(dx, dy, dz, q.w, a.eps2);
      } else {
        T.acc.template term<kSoft>(dx, dy, dz, fma(dz, dz, fma(dy, dy, dx * dx)), q.w, a.eps2);
      }
      if constexpr (kStats) {
        const uint64_t wd = (uint64_t)(a.perm[kk] - T.idx0) << 1;
        ++T.n_pp;
        T.h = (T.h ^ wd) * kFnvPrime;
        if (kBase == kWalkDump && T.len < a.maxlen) T.list[T.len] = (int64_t)wd;
        ++T.len;
      }
    }
  }
  if (more) {
    ++C.k;
    C.c = c;
  } else {
    C.k = C.kend = 0;
    C.c = c + 1;
  }
}

// One step of a walk at node `cur` (index C.c).  A cell and a one-particle
// leaf take the same path, and the opening test alone decides: the walk copies
// give a leaf S = 0, which every other particle passes (d^2 > 0) and the
// target's own leaf fails (d^2 = 0 exactly); a cell that holds the target
// fails the test when theta <= 1 (d <= (sqrt(3)/2) l + s < l/theta + s, a
// margin of 0.13 l that no rounding reaches).  kGuard: some target of the wave
// has theta > 1, so a cell holding the target is excluded by its particle range.
//
// A target that uses the node adds its term and skips the node's subtree
// (next(c); for a leaf that is c + 1 anyway); the cursor moves to c + 1 if an
// active target did not use the node, else to next(c).
//
// `fetch` is called with the next cursor as soon as the opening decisions fix
// it, before the terms are evaluated: the caller issues the next record's load
// there, and its latency overlaps the terms instead of heading the next step.
template <bool kF64, int kT, int kMode, bool kSoft, bool kPlain, bool kGuard, bool kBucket, typename Rec,
          typename Fetch>
__device__ __forceinline__ void walk_step(const WalkArgs& a, Cursor<kF64, kT>& C, const Rec& rec, const QuadRec& qd,
                                          Fetch&& fetch) {
  // On the LDS route the record was read by every lane; its integer fields
  // steer the wave's control flow, so take them as wave-uniform values (on the
  // scalar route they already are, and this costs nothing).
  Rec cur = rec;
  cur.next = uniform(rec.next);
  cur.first = uniform(rec.first);
  cur.count = uniform(rec.count);
  cur.meta = uniform(rec.meta);
  using R = typename Cursor<kF64, kT>::R;
  constexpr bool kStats = (kMode & 3) != kWalkForces;
  constexpr bool kQuad = (kMode & kWalkQuad) != 0;
  const int c = C.c;
  if constexpr (kStats) ++C.steps;
  // (the walk copies hold next(c) in (c, cap] already; the plain nodes of the
  // FP64 per-group-theta walk are taken as they are and clamped here)
  constexpr bool kRaw = std::is_same<Rec, Node>::value;
  const int nnext = kRaw ? max(cur.next, c + 1) : cur.next;
  constexpr bool kTheta = std::is_same<Rec, ThetaNode>::value;
  if constexpr (!kF64) {
    // Keep the FP32 mass in the step's first batch of scalar loads: it is used
    // only by the term, and a load left to the term's branch would cost the
    // step a second memory round trip.  (An empty statement that takes the
    // value in a scalar register; it emits no instruction.)
    asm volatile("" ::"s"(cur.M32));
  }
  bool use[kT];
  uint64_t m_open = 0;
  double dx[kT], dy[kT], dz[kT], d2[kT];
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    const Target<kF64>& T = C.t[t];
    const bool act = T.skip <= c;
    const uint64_t m_act = ballot(act);
    // Offset to the node's position (cell: centre of mass; leaf: its
    // particle), formed in FP64.  For FP32 input the FP64 difference of the
    // widened coordinates is exact, so its FP32 rounding equals a direct FP32
    // subtraction; a cell's offset is rounded once.
    dx[t] = cur.cx - T.xi;
    dy[t] = cur.cy - T.yi;
    dz[t] = cur.cz - T.zi;
    // Opening test of Eq. (2) in FP64.
    d2[t] = fma(dz[t], dz[t], fma(dy[t], dy[t], dx[t] * dx[t]));
    double S;
    if constexpr (kTheta) {
      const double u = fma(cur.l, T.inv_theta, cur.s);  // a leaf: l = s = 0, S = 0
      S = u * u;
    } else if constexpr (kPlain) {
      const double u = fma(cur.l, T.inv_theta, cur.s);
      S = (cur.meta & 1) ? 0.0 : u * u;
    } else {
      S = cur.S;
    }
    const bool pd = d2[t] > S;
    // the same test as a lane mask, straight from the compare (ordered >) --
    // a ballot of a combined flag would first turn it into a number
    uint64_t m_pass = __builtin_amdgcn_fcmp(d2[t], S, 2);
    if constexpr (kGuard) {
      const bool ns = (unsigned)(T.i - cur.first) >= (unsigned)cur.count;
      use[t] = act && pd && ns;
      m_pass &= __builtin_amdgcn_uicmp((unsigned)(T.i - cur.first), (unsigned)cur.count, 35);  // unsigned >=
    } else {
      use[t] = act && pd;
    }
    m_open |= m_act & ~m_pass;
  }
  // (the test above runs for every node, so that the whole record is read at
  // the top of the step; a leaf of several particles then goes its own way --
  // kBucket: the tree has such leaves, known per walk from the build's counts)
  if (kBucket && (cur.meta & 2)) {
    bucket_step<kF64, kT, kMode, kSoft>(a, C, cur, fetch);
  } else {
    const int cn = m_open ? c + 1 : nnext;
    fetch(cn);
    // A step whose node no active target uses (every one opens it) skips the
    // terms: a wave-uniform branch on the use mask.
    uint64_t m_use = 0;
#pragma unroll
    for (int t = 0; t < kT; ++t) m_use |= ballot(use[t]);
    if (m_use) {
    R tm;
    if constexpr (kF64) tm = (R)cur.M; else tm = (R)cur.M32;
    // (the walk copies mark a leaf by S = 0, resp. l = 0, so their steps need
    // no meta word to tell cells from leaves)
    bool cell;
    if constexpr (std::is_same<Rec, WalkNode>::value) cell = __builtin_bit_cast(uint64_t, cur.S) != 0;
    else if constexpr (std::is_same<Rec, ThetaNode>::value) cell = __builtin_bit_cast(uint64_t, cur.l) != 0;
    else cell = (cur.meta & 1) == 0;
    // FP32: the term's factors are formed for every lane ahead of the masked
    // sums (a VALU instruction costs the same with lanes masked off), so
    // that they overlap the cursor's scalar work instead of following it.
    MixedTerm q[kT];
    if constexpr (!kF64) {
#pragma unroll
      for (int t = 0; t < kT; ++t) {
        q[t] = AccMixed::prep<kSoft>(d2[t], tm, a.eps2);
        asm volatile("" : "+v"(q[t].mr3), "+v"(q[t].r2));
      }
    }
    // Order 2: a cell (not a leaf: its second moments vanish) adds the
    // quadrupole correction.  Whether the node is a cell is wave-uniform.
    QuadPart u[kT];
    const bool quad = kQuad && cell;
    if constexpr (kQuad && !kF64) {
      if (quad) {
#pragma unroll
        for (int t = 0; t < kT; ++t) u[t] = quad_part(dx[t], dy[t], dz[t], (double)q[t].ri, qd);
      }
    }
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      Target<kF64>& T = C.t[t];
      if (use[t]) {
        if constexpr (kF64) {
          if (quad)
            T.acc.term_quad(dx[t], dy[t], dz[t], tm, a.eps2, qd);
          else
            T.acc.term(dx[t], dy[t], dz[t], tm, a.eps2);
        } else {
          if (quad)
            T.acc.add_quad(q[t], u[t], dx[t], dy[t], dz[t]);
          else
            T.acc.add(q[t], dx[t], dy[t], dz[t]);
        }
        T.skip = nnext;
        if constexpr (kStats) {
          const uint64_t wd = cell ? (((uint64_t)(c - T.node0) << 1) | 1ull)
                                   : ((uint64_t)(a.perm[cur.first] - T.idx0) << 1);
          if (cell) ++T.n_pc; else ++T.n_pp;
          T.h = (T.h ^ wd) * kFnvPrime;
          if ((kMode & 3) == kWalkDump && T.len < a.maxlen) T.list[T.len] = (int64_t)wd;
          ++T.len;
        }
      }
    }
    }
    C.c = cn;
  }
}

// A second route for node records, a launch option (a share of the waves
// takes it): through LDS.  Each step copies both possible successors of the
// current node (c+1 and next(c)) with the LDS-DMA load (global_load_lds_dwordx4:
// lanes 0-3 bring the four 16-byte quarters of one record, lanes 4-7 those
// of the other) into the wave's spare buffer, and the next step reads the one
// it needs with broadcast LDS reads.  The copy's latency overlaps one step.
// On the measured workloads the scalar route with its look-ahead load is the
// faster one.
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
// wave-uniform), one round trip per step, issued by the previous step as soon
// as it knows the cursor.
// Both forms walk the subtree [C.c, end) of one cluster; `end` is clamped to
// the node capacity, so a corrupted record can never send the cursor out of the
// array, and every step moves the cursor forward or stays on a leaf for at most
// its particle count.
template <bool kF64, int kT, int kMode, bool kSoft, bool kPlain, bool kGuard, bool kBucket, bool kOff32>
__device__ __forceinline__ void walk_loop_scalar(const WalkArgs& a, StepNode<kF64, kPlain> wn, Cursor<kF64, kT>& C,
                                                 int end) {
  using Rec = decltype(wn.load(0));
  // The next record is read before the loop test: the walk copies have a spare
  // record at index cap = 2n (their next pointers stay <= cap); the plain node
  // array is read at most at its last record.
  constexpr bool kRaw = std::is_same<Rec, Node>::value;
  const int last = 2 * a.n - 1;
  // (two steps per iteration, the records alternating between two sets of
  // registers, so that no step has to move the next record into place)
  // (order 2: the node's second-moment record is read beside its walk record)
  constexpr bool kQuad = (kMode & kWalkQuad) != 0;
  Rec ra = wn.template load_at<kOff32>(C.c), rb;
  QuadRec qa{}, qb{};
  if constexpr (kQuad) qa = quad_load(a.qrec, C.c);
  while (C.c < end) {
    walk_step<kF64, kT, kMode, kSoft, kPlain, kGuard, kBucket>(a, C, ra, qa, [&](int cn) {
      const int ci = kRaw ? min(cn, last) : cn;
      rb = wn.template load_at<kOff32>(ci);
      if constexpr (kQuad) qb = quad_load(a.qrec, ci);
    });
    if (C.c >= end) break;
    walk_step<kF64, kT, kMode, kSoft, kPlain, kGuard, kBucket>(a, C, rb, qb, [&](int cn) {
      const int ci = kRaw ? min(cn, last) : cn;
      ra = wn.template load_at<kOff32>(ci);
      if constexpr (kQuad) qa = quad_load(a.qrec, ci);
    });
  }
}

template <bool kF64, int kT, int kMode, bool kSoft, bool kPlain, bool kGuard, bool kBucket>
__device__ __forceinline__ void walk_loop_lds(const WalkArgs& a, StepNode<kF64, kPlain> wn, Cursor<kF64, kT>& C,
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
    walk_step<kF64, kT, kMode, kSoft, kPlain, kGuard, kBucket>(a, C, rec, QuadRec{}, [](int) {});
    if (C.c != c) {  // moved on (a leaf of several particles keeps the cursor)
      slot = C.c == c + 1 ? 0 : 1;
      buf ^= 1;
    }
  }
}

// The clusters klo..khi of a wave, one subtree after the other; targets of the
// other clusters stay idle (skip past the subtree).
template <bool kF64, int kT, int kMode, bool kSoft, bool kPlain, bool kGuard, bool kBucket, bool kLds>
__device__ __forceinline__ void walk_clusters(const WalkArgs& a, StepNode<kF64, kPlain> wn, Cursor<kF64, kT>& C,
                                              uint4 (*pf)[8], const int (&kc)[kT], int klo, int khi) {
  const int cap = 2 * a.n;
  // (the plain nodes of the FP64 per-group-theta walk keep 64-bit addressing)
  constexpr bool kRaw = kF64 && kPlain;
  const bool off32 = !kRaw && a.n < kOff32MaxN;
  for (int k = klo; k <= khi; ++k) {
    const int r0 = min(max(uniform(a.croot[k]), 0), cap);
    const int r1 = min(max(uniform(a.croot[k + 1]), r0), cap);
    C.c = r0;
    C.k = C.kend = 0;
#pragma unroll
    for (int t = 0; t < kT; ++t) C.t[t].skip = (C.t[t].i >= 0 && kc[t] == k) ? r0 : 0x7fffffff;
    if (r0 >= r1) continue;
    if constexpr (kLds && (kMode & kWalkQuad) == 0)
      walk_loop_lds<kF64, kT, kMode, kSoft, kPlain, kGuard, kBucket>(a, wn, C, pf, r1);
    else if (off32)
      walk_loop_scalar<kF64, kT, kMode, kSoft, kPlain, kGuard, kBucket, true>(a, wn, C, r1);
    else
      walk_loop_scalar<kF64, kT, kMode, kSoft, kPlain, kGuard, kBucket, false>(a, wn, C, r1);
  }
}

// The walk of one group of 64 kT targets (one wavefront).
// kSoft: eps > 0, so r^2 + eps^2 > 0 and the FP32 term needs no zero test.
// kGroupTheta: theta per walk group (64 targets) instead of one uniform theta
// (uniform theta walks the copy with S precomputed).
template <bool kF64, int kT, int kMode, bool kSoft, bool kGroupTheta>
__device__ __forceinline__ void walk_group(const WalkArgs& a, int group, uint4 (*pf)[8]) {
  using R = typename Cursor<kF64, kT>::R;
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  constexpr bool kStats = (kMode & 3) != kWalkForces;
  const int lane = __lane_id();
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);

  Cursor<kF64, kT> C;
  C.k = C.kend = 0;
  C.steps = 0;
  bool guard_l = false;
  int kc[kT];
  int klo = 0x7fffffff, khi = -1;
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    Target<kF64>& T = C.t[t];
    T.slot = (group * kT + t) * kWave + lane;
    const bool valid = T.slot < a.n;
    T.i = valid ? (a.order ? a.order[T.slot] : T.slot) : -1;
    R4 me;
    if (valid) {
      me = ps[T.i];
    } else {
      me.x = me.y = me.z = me.w = (R)0;
    }
    T.xi = (double)me.x;
    T.yi = (double)me.y;
    T.zi = (double)me.z;
    if constexpr (kGroupTheta) {
      // theta of the target's walk group (the 64 targets at [64g, 64g + 64) of
      // the walk order); one that is not finite or outside (0, 2/sqrt(3)) is
      // replaced by the fallback and reported
      float th = valid ? a.theta_group[T.slot >> 6] : kThetaFallback;
      if (!(th > 0.f && (double)th < kThetaMax)) {
        th = kThetaFallback;
        atomicOr(a.bad_theta, 1);
      }
      T.inv_theta = 1.0 / (double)th;
    } else {
      T.inv_theta = a.inv_theta;
    }
    T.acc.init();
    T.n_pp = T.n_pc = 0;
    T.h = kFnvOffset;
    T.len = 0;
    T.list = ((kMode & 3) == kWalkDump && valid) ? a.lists + (int64_t)a.perm[T.i] * a.maxlen : nullptr;
    guard_l = guard_l || (valid && T.inv_theta < 1.0);
    // Clusters of the wave's targets: a wave usually lies inside one cluster;
    // one that straddles cluster edges walks each cluster's subtree in turn.
    kc[t] = (valid && a.scid) ? min(max(a.scid[T.i], 0), a.n_seg - 1) : 0;
    if (valid) {
      klo = min(klo, kc[t]);
      khi = max(khi, kc[t]);
    }
    T.node0 = valid ? a.croot[kc[t]] : 0;
    T.idx0 = valid ? (int)a.seg_off[kc[t]] : 0;
  }
  const bool guard = ballot(guard_l) != 0ull;
  for (int o = 32; o > 0; o >>= 1) {
    klo = min(klo, __shfl_xor(klo, o, 64));
    khi = max(khi, __shfl_xor(khi, o, 64));
  }
  klo = uniform(klo);
  khi = uniform(khi);
  StepNode<kF64, kGroupTheta> wn;
  if constexpr (kGroupTheta && kF64) wn.base = a.nodes;
  else if constexpr (kGroupTheta) wn.base = a.tnodes;
  else wn.base = a.wnodes;
  // Waves split between the two node paths (scalar cache / LDS copies) so
  // that neither the scalar cache nor instruction issue alone sets the pace;
  // the share taking the LDS path is a launch parameter (results identical).
  // (taken as a wave-uniform value: the compiler cannot tell that the wave
  // index is uniform, and a branch it took for divergent would turn the walk
  // state that crosses it into per-lane values)
  // (walks of order 2 take the scalar route only)
  const bool lds_path = (kMode & kWalkQuad) == 0 && uniform(((group * 37) & 63) < a.lds_share64 ? 1 : 0) != 0;
  // (one cluster loop per path and guard: the LDS path's copies must not share
  // a loop with the scalar path's loads, or the compiler stops treating the
  // node array as unwritten and drops the scalar loads)
  // Leaves of several coincident-key particles exist iff some keys repeat
  // (fewer leaves than particles); without them the step needs no branch for
  // them.
  const bool buckets = uniform(a.cnt->n_unique < a.n ? 1 : 0) != 0;
  if (lds_path) {
    if (buckets) {
      if (guard)
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, true, true, true>(a, wn, C, pf, kc, klo, khi);
      else
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, false, true, true>(a, wn, C, pf, kc, klo, khi);
    } else {
      if (guard)
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, true, false, true>(a, wn, C, pf, kc, klo, khi);
      else
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, false, false, true>(a, wn, C, pf, kc, klo, khi);
    }
  } else {
    if (buckets) {
      if (guard)
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, true, true, false>(a, wn, C, pf, kc, klo, khi);
      else
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, false, true, false>(a, wn, C, pf, kc, klo, khi);
    } else {
      if (guard)
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, true, false, false>(a, wn, C, pf, kc, klo, khi);
      else
        walk_clusters<kF64, kT, kMode, kSoft, kGroupTheta, false, false, false>(a, wn, C, pf, kc, klo, khi);
    }
  }

#pragma unroll
  for (int t = 0; t < kT; ++t) {
    const Target<kF64>& T = C.t[t];
    if (T.i < 0) continue;
    if (kStats && a.group_steps && lane == 0) a.group_steps[T.slot >> 6] = C.steps;
    const int o = a.perm[T.i];
    R* accp = reinterpret_cast<R*>(a.acc);
    R* potp = reinterpret_cast<R*>(a.pot);
    accp[3 * (int64_t)o] = (R)T.acc.ax;
    accp[3 * (int64_t)o + 1] = (R)T.acc.ay;
    accp[3 * (int64_t)o + 2] = (R)T.acc.az;
    potp[o] = (R)T.acc.p;
    if constexpr (kStats) {
      a.counts[2 * (int64_t)o] = T.n_pp;
      a.counts[2 * (int64_t)o + 1] = T.n_pc;
      a.hash[o] = T.h;
    }
  }
}

// One wavefront per group of 64 kT targets; workgroups of waves_per_block waves.
template <bool kF64, int kT, int kMode, bool kSoft, bool kGroupTheta>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
  __shared__ uint4 pf_lds[4][2][8];  // per wave: two buffers of two 64-byte node records
  const int wv = threadIdx.x >> 6;
  const int blk = remap_block(blockIdx.x, gridDim.x, a.xcd_chunk);
  // (a wave past the last target has no valid lane and walks nothing)
  walk_group<kF64, kT, kMode, kSoft, kGroupTheta>(a, blk * a.waves_per_block + wv, pf_lds[wv]);
}

// Persistent form: a grid that fits on the chip at once; every wave takes the
// next group from a device counter until none is left, so the load balances
// itself and no workgroup waits for a dispatch slot.  Every wave leaves once
// the counter passes the last group.
// The group loop keeps the launch arguments in scalar registers; left alone
// the compiler takes 106 of them, which caps the kernel at 7 waves per SIMD
// (the plain form runs 8).  The FP32 uniform-theta force kernels of one target
// per lane are asked for 8 waves: their spare scalars then go to VGPR lanes
// outside the step loop.  (The others would spill vector registers to memory.)
template <bool kF64, int kT, int kMode, bool kSoft, bool kGroupTheta>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(!kF64 && kT == 1 && kMode == kWalkForces && !kGroupTheta ? 8 : 1)))  // (not order 2)
void k_walk_persistent(WalkArgs a) {
  __shared__ uint4 pf_lds[4][2][8];
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int groups = (a.n + kT * kWave - 1) / (kT * kWave);
  for (;;) {
    int g = 0;
    if (lane == 0) g = atomicAdd(a.queue, 1);
    g = __shfl(g, 0, 64);
    if (g >= groups) break;
    walk_group<kF64, kT, kMode, kSoft, kGroupTheta>(a, g, pf_lds[wv]);
  }
}

template <bool kF64, int kT, int kMode, bool kSoft, bool kGroupTheta>
static hipError_t launch_t(const WalkArgs& a, hipStream_t st) {
  const int groups = (a.n + kT * kWave - 1) / (kT * kWave);
  const int wpb = a.waves_per_block;
  const int blocks = (groups + wpb - 1) / wpb;
  if (a.persistent) {
    hipError_t e = fill_i32(a.queue, 1, 0, st);
    if (e != hipSuccess) return e;
    k_walk_persistent<kF64, kT, kMode, kSoft, kGroupTheta><<<max(1, min(a.grid, blocks)), wpb * kWave, 0, st>>>(a);
  } else {
    k_walk<kF64, kT, kMode, kSoft, kGroupTheta><<<blocks, wpb * kWave, 0, st>>>(a);
  }
  return hipGetLastError();
}

template <bool kF64, int kT, int kMode>
static hipError_t launch_mode(const WalkArgs& a, hipStream_t st) {
  const bool soft = a.eps2 > 0.0;
  if (a.theta_group)
    return soft ? launch_t<kF64, kT, kMode, true, true>(a, st) : launch_t<kF64, kT, kMode, false, true>(a, st);
  return soft ? launch_t<kF64, kT, kMode, true, false>(a, st) : launch_t<kF64, kT, kMode, false, false>(a, st);
}

template <bool kF64, int kT, int kMode>
static const void* persistent_fn(bool soft, bool group_theta) {
  if (soft)
    return group_theta ? reinterpret_cast<const void*>(&k_walk_persistent<kF64, kT, kMode, true, true>)
                       : reinterpret_cast<const void*>(&k_walk_persistent<kF64, kT, kMode, true, false>);
  return group_theta ? reinterpret_cast<const void*>(&k_walk_persistent<kF64, kT, kMode, false, true>)
                     : reinterpret_cast<const void*>(&k_walk_persistent<kF64, kT, kMode, false, false>);
}

// One translation unit per (precision, mode) instantiates its kernels through
// these two, so that the walk's many variants compile side by side.
// (walks of order 2 take one target per lane)
template <bool kF64, int kMode>
static hipError_t launch_walk_mode(const WalkArgs& a, hipStream_t st) {
  if (a.qrec) return launch_mode<kF64, 1, kMode | kWalkQuad>(a, st);
  if (a.targets_per_lane == 2) return launch_mode<kF64, 2, kMode>(a, st);
  return launch_mode<kF64, 1, kMode>(a, st);
}

template <bool kF64, int kMode>
static const void* walk_persistent_fn(bool quad, bool soft, bool group_theta, int targets_per_lane) {
  if (quad) return persistent_fn<kF64, 1, kMode | kWalkQuad>(soft, group_theta);
  return targets_per_lane == 2 ? persistent_fn<kF64, 2, kMode>(soft, group_theta)
                               : persistent_fn<kF64, 1, kMode>(soft, group_theta);
}

// Defined in bh_walk_<precision><mode>.hip.
hipError_t walk_f32_forces(const WalkArgs& a, hipStream_t st);
hipError_t walk_f32_stats(int mode, const WalkArgs& a, hipStream_t st);
hipError_t walk_f64_forces(const WalkArgs& a, hipStream_t st);
hipError_t walk_f64_stats(int mode, const WalkArgs& a, hipStream_t st);
const void* walk_f32_forces_fn(bool quad, bool soft, bool group_theta, int targets_per_lane);
const void* walk_f32_stats_fn(int mode, bool quad, bool soft, bool group_theta, int targets_per_lane);
const void* walk_f64_forces_fn(bool quad, bool soft, bool group_theta, int targets_per_lane);
const void* walk_f64_stats_fn(int mode, bool quad, bool soft, bool group_theta, int targets_per_lane);

}  // namespace bh
