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
// bound safe under rounding).  A leaf carries r^2, the exact test.  The
// neighbour sets therefore equal the definition's, and each target meets its
// neighbours in depth-first (Morton) order whatever the grouping.
#include "bh_walk_impl.h"

namespace bh {

namespace {

// W(r, h) of the M4 cubic spline in three dimensions.
__device__ __forceinline__ double sph_w(double r, double h) {
  const double q = r / h;
  const double sig = 1.0 / (3.141592653589793 * h * h * h);
  if (q < 1.0) return sig * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
  if (q < 2.0) {
    const double u = 2.0 - q;
    return sig * 0.25 * u * u * u;
  }
  return 0.0;
}

__global__ __launch_bounds__(256) void k_nbr_copy(const Node* __restrict__ nodes, const Counts* __restrict__ cnt,
                                                  int cap, double radius, WalkNode* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cap || c >= cnt->n_nodes) return;
  const Node nd = nodes[c];
  WalkNode w;
  w.cx = nd.cx;
  w.cy = nd.cy;
  w.cz = nd.cz;
  if (nd.meta & 1) {
    w.S = radius * radius;
  } else {
    const double u = (radius + nd.s + 0.8660254037844387 * nd.l) * (1.0 + 0x1p-40);
    w.S = u * u;
  }
  w.M32 = (float)nd.M;
  w.pad = 0;
  w.next = min(max(nd.next, c + 1), cap);
  w.first = nd.first;
  w.count = nd.count;
  w.meta = nd.meta;
  w.M = nd.M;
  out[c] = w;
}

struct NbrArgs {
  const WalkNode* wn;          // neighbour walk copy [2n + 1]
  const void* ps;              // float4 / double4 particles in Morton order
  const int32_t* perm;         // Morton position -> caller index
  const int32_t* order;        // walk order of the targets (Morton positions), may be null
  const int32_t* scid;         // Morton position -> cluster (forest), may be null
  const int32_t* croot;        // [K + 1] preorder range of each cluster's subtree
  const int64_t* seg_off;      // [K + 1] caller offsets of the clusters
  int n_seg;
  int n;
  double r2, h;
  int32_t* count;              // [n] neighbours, caller order
  uint64_t* hash;              // [n] ordered hash of the neighbours' (cluster-relative) caller indices
  int64_t* lists;              // [n][maxlen], may be null
  int64_t maxlen;
  void* rho;                   // [n] SPH density, may be null
  int xcd_chunk;
};

struct NbrTarget {
  double xi, yi, zi, rho;
  int i, skip, idx0;
  int32_t count;
  uint64_t h;
  int64_t len;
  int64_t* list;
};

template <typename T4>
__device__ __forceinline__ void nbr_particle(const NbrArgs& a, NbrTarget& T, int k, const T4& q) {
  const double dx = (double)q.x - T.xi, dy = (double)q.y - T.yi, dz = (double)q.z - T.zi;
  const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
  if (k != T.i && d2 < a.r2) {
    const int64_t j = (int64_t)a.perm[k] - T.idx0;
    ++T.count;
    T.h = (T.h ^ ((uint64_t)j << 1)) * kFnvPrime;
    if (T.list && T.len < a.maxlen) T.list[T.len] = j;
    ++T.len;
    T.rho += (double)q.w * sph_w(sqrt(d2), a.h);
  }
}

template <bool kF64, bool kOff32>
__device__ void nbr_subtree(const NbrArgs& a, NbrTarget& T, int c, int end) {
  using T4 = typename std::conditional<kF64, double4, float4>::type;
  const T4* __restrict__ ps = reinterpret_cast<const T4*>(a.ps);
  StepNode<kF64, false> wn;
  wn.base = a.wn;
  while (c < end) {
    const WalkNode cur = wn.template load_at<kOff32>(c);
    const int nnext = uniform(cur.next);
    const int first = uniform(cur.first), count = uniform(cur.count), meta = uniform(cur.meta);
    const bool act = T.skip <= c;
    if (meta & 1) {
      // a leaf: proc_particle for its particle(s)
      if (act) {
        if (count == 1) {
          // (a one-particle leaf sits at its particle, and carries its mass exactly)
          T4 q;
          q.x = cur.cx;
          q.y = cur.cy;
          q.z = cur.cz;
          q.w = cur.M;
          nbr_particle(a, T, first, q);
        } else {
          for (int k = first; k < first + count; ++k) nbr_particle(a, T, k, ps[k]);
        }
      }
      c = c + 1;
    } else {
      // a cell: distance_test; lanes that cannot reach it skip its subtree
      const double dx = cur.cx - T.xi, dy = cur.cy - T.yi, dz = cur.cz - T.zi;
      const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
      const bool far = !(d2 < cur.S);
      if (act && far) T.skip = nnext;
      const uint64_t m_open = ballot(act && !far);
      c = m_open ? c + 1 : nnext;
    }
  }
}

template <bool kF64>
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
  T.rho = valid ? (double)me.w * sph_w(0.0, a.h) : 0.0;
  T.count = 0;
  T.h = kFnvOffset;
  T.len = 0;
  T.list = (a.lists && valid) ? a.lists + (int64_t)a.perm[T.i] * a.maxlen : nullptr;
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
      nbr_subtree<kF64, true>(a, T, r0, r1);
    else
      nbr_subtree<kF64, false>(a, T, r0, r1);
  }
  if (!valid) return;
  const int o = a.perm[T.i];
  a.count[o] = T.count;
  a.hash[o] = T.h;
  if (a.rho) reinterpret_cast<R*>(a.rho)[o] = (R)T.rho;
}

}  // namespace

hipError_t launch_neighbours(bool f64, const Node* nodes, const Counts* counts, WalkNode* copy, const void* ps,
                             const int32_t* perm, const int32_t* order, const int32_t* scid, const int32_t* croot,
                             const int64_t* seg_off, int n_seg, int n, double radius, int32_t* count,
                             uint64_t* hash, int64_t* lists, int64_t maxlen, void* rho, int xcd_chunk,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int cap = 2 * n;
  k_nbr_copy<<<(cap + 255) / 256, 256, 0, st>>>(nodes, counts, cap, radius, copy);
  NbrArgs a{};
  a.wn = copy;
  a.ps = ps;
  a.perm = perm;
  a.order = order;
  a.scid = scid;
  a.croot = croot;
  a.seg_off = seg_off;
  a.n_seg = n_seg;
  a.n = n;
  a.r2 = radius * radius;
  a.h = 0.5 * radius;
  a.count = count;
  a.hash = hash;
  a.lists = lists;
  a.maxlen = maxlen;
  a.rho = rho;
  a.xcd_chunk = xcd_chunk;
  const int groups = (n + kWave - 1) / kWave;
  if (f64)
    k_nbr<true><<<groups, kWave, 0, st>>>(a);
  else
    k_nbr<false><<<groups, kWave, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace bh
