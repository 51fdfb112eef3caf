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
// Precision (FP32 variant): the opening test is done in FP64 on the FP64
// centre of mass and the exactly widened FP32 position, d^2 =
// fma(dz,dz,fma(dy,dy,dx*dx)); the cell offset COM - x_i is formed in FP64 and
// rounded once to FP32 (CDNA4 issues FP64 add/fma at the same rate as
// unpacked FP32); particle offsets x_j - x_i are single FP32 roundings.  The
// kernel itself is FP32 (v_rsq_f32), accumulated in plain FP32 partial sums
// that are folded every kFlush terms into a (hi, lo) pair with Knuth's TwoSum.
// The FP64 variant evaluates every term exactly as the reference definition
// (IEEE sqrt and division, no contraction) and accumulates in FP64.
#include "bh_internal.h"

namespace bh {

constexpr int kFlush = 32;  // FP32 terms per lane between compensated folds

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

__device__ __forceinline__ void two_sum(float& hi, float& lo, float v) {
  const float s = hi + v;
  const float bb = s - hi;
  const float err = (hi - (s - bb)) + (v - bb);
  hi = s;
  lo += err;
}

struct AccF32 {
  float ax, ay, az, p;          // current partial sums
  float hx, hy, hz, hp;         // compensated totals
  float lx, ly, lz, lp;
  int cnt;
  __device__ void init() {
    ax = ay = az = p = 0.f;
    hx = hy = hz = hp = 0.f;
    lx = ly = lz = lp = 0.f;
    cnt = 0;
  }
  __device__ __forceinline__ void term(float dx, float dy, float dz, float m, float eps2) {
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    const float ri = (r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f;
    const float mr = m * ri;
    const float mr3 = (mr * ri) * ri;
    ax = fmaf(mr3, dx, ax);
    ay = fmaf(mr3, dy, ay);
    az = fmaf(mr3, dz, az);
    p -= mr;
    ++cnt;
  }
  __device__ __forceinline__ void fold() {
    two_sum(hx, lx, ax);
    two_sum(hy, ly, ay);
    two_sum(hz, lz, az);
    two_sum(hp, lp, p);
    ax = ay = az = p = 0.f;
    cnt = 0;
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

template <bool kF64, int kMode>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
  using R = typename std::conditional<kF64, double, float>::type;
  using R4 = typename std::conditional<kF64, double4, float4>::type;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int blk = remap_block(blockIdx.x, gridDim.x, a.xcd_chunk);
  const int slot = (blk * a.waves_per_block + wv) * kWave + lane;
  const bool valid = slot < a.n;
  const int i = valid ? (a.order ? a.order[slot] : slot) : -1;  // Morton position of the target
  const R4* __restrict__ ps = reinterpret_cast<const R4*>(a.ps);
  const Node* __restrict__ nodes = a.nodes;

  R4 me;
  if (valid) {
    me = ps[i];
  } else {
    me.x = me.y = me.z = me.w = (R)0;
  }
  const double xi = (double)me.x, yi = (double)me.y, zi = (double)me.z;
  const double inv_theta = a.theta_group ? 1.0 / (double)a.theta_group[valid ? (i >> 6) : 0] : a.inv_theta;
  const R eps2 = (R)a.eps2;

  typename std::conditional<kF64, AccF64, AccF32>::type acc;
  acc.init();
  int32_t n_pp = 0, n_pc = 0;
  uint64_t h = kFnvOffset;
  int64_t len = 0;
  int64_t* mylist = nullptr;
  if (kMode == kWalkDump && valid) mylist = a.lists + (int64_t)a.perm[i] * a.maxlen;

  int skip = valid ? 0 : 0x7fffffff;
  // next(root) is the node count; clamp it to the capacity so that a corrupted
  // record can never send the cursor out of the array, and force progress.
  const int n_nodes = min(uniform(nodes[0].next), 2 * a.n);
  int c = 0;
  while (c < n_nodes) {
    Node nd = nodes[c];
    nd.next = max(nd.next, c + 1);
    nd.first = min(max(nd.first, 0), a.n);
    nd.count = min(max(nd.count, 0), a.n - nd.first);
    const bool act = skip <= c;
    if (nd.meta & 1) {
      // leaf: particle-particle terms with every particle in it except i
      if (nd.count == 1) {
        if (act && nd.first != i) {
          acc.term((R)nd.cx - me.x, (R)nd.cy - me.y, (R)nd.cz - me.z, (R)nd.M, eps2);
          if (kMode != kWalkForces) {
            ++n_pp;
            const uint64_t wd = (uint64_t)a.perm[nd.first] << 1;
            h = (h ^ wd) * kFnvPrime;
            if (kMode == kWalkDump && len < a.maxlen) mylist[len] = (int64_t)wd;
            ++len;
          }
        }
      } else {
        for (int k = nd.first; k < nd.first + nd.count; ++k) {
          const R4 q = ps[k];
          if (act && k != i) {
            acc.term(q.x - me.x, q.y - me.y, q.z - me.z, q.w, eps2);
            if (kMode != kWalkForces) {
              ++n_pp;
              const uint64_t wd = (uint64_t)a.perm[k] << 1;
              h = (h ^ wd) * kFnvPrime;
              if (kMode == kWalkDump && len < a.maxlen) mylist[len] = (int64_t)wd;
              ++len;
            }
          }
        }
      }
      c = nd.next;
    } else {
      const bool inside = (unsigned)(i - nd.first) < (unsigned)nd.count;
      const double dx = nd.cx - xi, dy = nd.cy - yi, dz = nd.cz - zi;
      const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
      const double u = fma(nd.l, inv_theta, nd.s);
      const bool take = act && !inside && d2 > u * u;
      if (ballot(take)) {
        if (take) {
          acc.term((R)dx, (R)dy, (R)dz, (R)nd.M, eps2);
          if (kMode != kWalkForces) {
            ++n_pc;
            const uint64_t wd = ((uint64_t)c << 1) | 1ull;
            h = (h ^ wd) * kFnvPrime;
            if (kMode == kWalkDump && len < a.maxlen) mylist[len] = (int64_t)wd;
            ++len;
          }
        }
      }
      skip = take ? nd.next : skip;
      c = ballot(act && !take) ? c + 1 : nd.next;
    }
    if constexpr (!kF64) {
      if (ballot(acc.cnt >= kFlush)) {
        if (acc.cnt >= kFlush) acc.fold();
      }
    }
  }
  if (!valid) return;
  const int o = a.perm[i];
  R* accp = reinterpret_cast<R*>(a.acc);
  R* potp = reinterpret_cast<R*>(a.pot);
  if constexpr (kF64) {
    accp[3 * (int64_t)o] = acc.ax;
    accp[3 * (int64_t)o + 1] = acc.ay;
    accp[3 * (int64_t)o + 2] = acc.az;
    potp[o] = acc.p;
  } else {
    acc.fold();
    accp[3 * (int64_t)o] = acc.hx + acc.lx;
    accp[3 * (int64_t)o + 1] = acc.hy + acc.ly;
    accp[3 * (int64_t)o + 2] = acc.hz + acc.lz;
    potp[o] = acc.hp + acc.lp;
  }
  if (kMode != kWalkForces) {
    a.counts[2 * (int64_t)o] = n_pp;
    a.counts[2 * (int64_t)o + 1] = n_pc;
    a.hash[o] = h;
  }
}

template <bool kF64, int kMode>
static hipError_t launch_t(const WalkArgs& a, hipStream_t st) {
  const int groups = (a.n + kWave - 1) / kWave;
  const int wpb = a.waves_per_block;
  const int blocks = (groups + wpb - 1) / wpb;
  k_walk<kF64, kMode><<<blocks, wpb * kWave, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_walk(bool f64, int mode, const WalkArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (f64) {
    if (mode == kWalkForces) return launch_t<true, kWalkForces>(a, st);
    if (mode == kWalkStats) return launch_t<true, kWalkStats>(a, st);
    return launch_t<true, kWalkDump>(a, st);
  }
  if (mode == kWalkForces) return launch_t<false, kWalkForces>(a, st);
  if (mode == kWalkStats) return launch_t<false, kWalkStats>(a, st);
  return launch_t<false, kWalkDump>(a, st);
}

}  // namespace bh
