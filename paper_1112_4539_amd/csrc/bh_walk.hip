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

// Per-lane state of one walk.
template <bool kF64>
struct Lane {
  using R = typename std::conditional<kF64, double, float>::type;
  typename std::conditional<kF64, AccF64, AccMixed>::type acc;
  int32_t n_pp, n_pc;
  uint64_t h;
  int64_t len;
};

// What a step needs of a node, from the walk copy (uniform theta) or from the
// plain node (per-group theta: S formed from l and s per lane).
template <bool kPlain>
struct StepNode;
template <>
struct StepNode<false> {
  const WalkNode* base;
  __device__ __forceinline__ WalkNode load(int c) const { return base[c]; }
};
template <>
struct StepNode<true> {
  const Node* base;
  __device__ __forceinline__ Node load(int c) const { return base[c]; }
};

// The walk loop of one wavefront.  kGuard: some target of the wave has
// theta > 1, so a cell holding the target must be excluded explicitly (for
// theta <= 1 such a cell fails the opening test by itself: d <= (sqrt(3)/2) l
// + s < l/theta + s, a margin of 0.13 l that no rounding reaches).
// kPlain: read the plain nodes (per-group theta) rather than the walk copy.
//
// Each step produces one source for the shared term: the cell (opening test
// first), the particle of a one-particle leaf, or one particle of a leaf of
// coincident-key particles (the cursor stays on such a leaf until its
// particles are done).  One term site keeps the accumulators in place.
template <bool kF64, int kMode, bool kSoft, bool kPlain, bool kGuard>
__device__ __forceinline__ void walk_loop(const WalkArgs& a, StepNode<kPlain> wn, int i, int lane_valid,
                                          double xi, double yi, double zi, float xf, float yf, float zf,
                                          double inv_theta, Lane<kF64>& L, int64_t* mylist, int& steps) {
  using R = typename Lane<kF64>::R;
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  constexpr bool kStats = kMode != kWalkForces;
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);
  const R eps2 = (R)a.eps2;
  const int cap = 2 * a.n;
  // next(root) is the node count; clamp it to the capacity so that a corrupted
  // record can never send the cursor out of the array, and force progress.
  const int n_nodes = min(uniform(wn.load(0).next), cap);
  int skip = lane_valid ? 0 : 0x7fffffff;
  int c = 0;
  int k = 0, kend = 0;  // position inside a leaf of several particles
  while (c < n_nodes) {
    if constexpr (kStats) ++steps;
    const auto cur = wn.load(c);
    const int nnext = max(cur.next, c + 1);
    const int kind = cur.meta & 3;  // 0 cell, 1 one-particle leaf, 3 several-particle leaf
    const bool act = skip <= c;
    const uint64_t m_act = ballot(act);
    // Offset to the node's position (cell: centre of mass; one-particle leaf:
    // its particle), formed in FP64.  For FP32 input the FP64 difference of the
    // widened coordinates is exact, so its FP32 rounding equals a direct FP32
    // subtraction; a cell's offset is rounded once.  Formed for every node so
    // that the whole record is read at the top of the step.
    double dx = cur.cx - xi, dy = cur.cy - yi, dz = cur.cz - zi;
    // Opening test of Eq. (2) in FP64, also evaluated (and ignored) for leaves
    // so that no field load is left for later in the step.
    double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double S;
    if constexpr (kPlain) {
      const double u = fma(cur.l, inv_theta, cur.s);
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
      if (kend == 0) {
        k = min(max(cur.first, 0), a.n);
        kend = k + min(max(cur.count, 0), a.n - k);
      }
      const int kk = min(k, a.n - 1);
      src = kk;
      const R4 q = ps[kk];
      use = act && k < kend && kk != i;
      m_use = m_act & ballot(k < kend && kk != i);
      // the step's source is this particle: its offset replaces the node's
      dx = (double)q.x - xi;
      dy = (double)q.y - yi;
      dz = (double)q.z - zi;
      d2 = fma(dz, dz, fma(dy, dy, dx * dx));
      tm = q.w;
      if (++k < kend) {
        cnext = c;
      } else {
        k = kend = 0;
      }
    }
    if (m_use) {
      if (use) {
        if constexpr (kF64) {
          L.acc.term(dx, dy, dz, tm, eps2);
        } else {
          L.acc.template term<kSoft>(dx, dy, dz, d2, tm, a.eps2);
        }
        if (kind == 0) skip = nnext;
        if constexpr (kStats) {
          const uint64_t wd = kind == 0 ? (((uint64_t)c << 1) | 1ull) : ((uint64_t)a.perm[src] << 1);
          if (kind == 0) ++L.n_pc; else ++L.n_pp;
          L.h = (L.h ^ wd) * kFnvPrime;
          if (kMode == kWalkDump && L.len < a.maxlen) mylist[L.len] = (int64_t)wd;
          ++L.len;
        }
      }
    }
    c = cnext;
  }
}

// kSoft: eps > 0, so r^2 + eps^2 > 0 and the FP32 term needs no zero test.
// kGroupTheta: theta per 64-particle Morton group instead of one uniform theta
// (uniform theta walks the copy with S precomputed).
template <bool kF64, int kMode, bool kSoft, bool kGroupTheta>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
  using R = typename Lane<kF64>::R;
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  constexpr bool kStats = kMode != kWalkForces;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int blk = remap_block(blockIdx.x, gridDim.x, a.xcd_chunk);
  const int slot = (blk * a.waves_per_block + wv) * kWave + lane;
  const bool valid = slot < a.n;
  const int i = valid ? (a.order ? a.order[slot] : slot) : -1;  // Morton position of the target
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);

  R4 me;
  if (valid) {
    me = ps[i];
  } else {
    me.x = me.y = me.z = me.w = (R)0;
  }
  const double xi = (double)me.x, yi = (double)me.y, zi = (double)me.z;
  const double inv_theta = kGroupTheta ? 1.0 / (double)a.theta_group[valid ? (i >> 6) : 0] : a.inv_theta;
  const bool guard = ballot(valid && inv_theta < 1.0) != 0ull;
  StepNode<kGroupTheta> wn;
  if constexpr (kGroupTheta) wn.base = a.nodes; else wn.base = a.wnodes;

  Lane<kF64> L;
  L.acc.init();
  L.n_pp = L.n_pc = 0;
  L.h = kFnvOffset;
  L.len = 0;
  int64_t* mylist = nullptr;
  if (kMode == kWalkDump && valid) mylist = a.lists + (int64_t)a.perm[i] * a.maxlen;
  int steps = 0;
  const float xf = (float)me.x, yf = (float)me.y, zf = (float)me.z;
  if (guard)
    walk_loop<kF64, kMode, kSoft, kGroupTheta, true>(a, wn, i, valid, xi, yi, zi, xf, yf, zf, inv_theta, L, mylist,
                                                     steps);
  else
    walk_loop<kF64, kMode, kSoft, kGroupTheta, false>(a, wn, i, valid, xi, yi, zi, xf, yf, zf, inv_theta, L, mylist,
                                                      steps);

  if (kStats && a.group_steps && lane == 0 && valid) a.group_steps[slot >> 6] = steps;
  if (!valid) return;
  const int o = a.perm[i];
  R* accp = reinterpret_cast<R*>(a.acc);
  R* potp = reinterpret_cast<R*>(a.pot);
  if constexpr (kF64) {
    accp[3 * (int64_t)o] = L.acc.ax;
    accp[3 * (int64_t)o + 1] = L.acc.ay;
    accp[3 * (int64_t)o + 2] = L.acc.az;
    potp[o] = L.acc.p;
  } else {
    accp[3 * (int64_t)o] = (float)L.acc.ax;
    accp[3 * (int64_t)o + 1] = (float)L.acc.ay;
    accp[3 * (int64_t)o + 2] = (float)L.acc.az;
    potp[o] = (float)L.acc.p;
  }
  if constexpr (kStats) {
    a.counts[2 * (int64_t)o] = L.n_pp;
    a.counts[2 * (int64_t)o + 1] = L.n_pc;
    a.hash[o] = L.h;
  }
}

template <bool kF64, int kMode, bool kSoft, bool kGroupTheta>
static hipError_t launch_t(const WalkArgs& a, hipStream_t st) {
  const int groups = (a.n + kWave - 1) / kWave;
  const int wpb = a.waves_per_block;
  const int blocks = (groups + wpb - 1) / wpb;
  k_walk<kF64, kMode, kSoft, kGroupTheta><<<blocks, wpb * kWave, 0, st>>>(a);
  return hipGetLastError();
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
