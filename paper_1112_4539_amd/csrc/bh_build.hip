// bh_build.hip -- tree construction on the GPU (gfx950).
//
// The paper builds the oct-tree on the host (Sec. 4.1, and steps 1-3 of the
// flow listed at the end of Sec. 4.4) and suggests parallelising that part
// (Sec. 7).  Here every step runs on the device, as a pipeline of HBM-bound
// passes with no host round trip:
//
//   bbox     root cube: coordinate-wise min, largest extent L       (Sec. 4.1)
//   keys     63-bit Morton key on the 2^21 grid of the cube         (Sec. 5)
//   sort     stable LSD radix sort of (key, index), 8 x 8-bit digits (Sec. 5,
//            localized particle ordering), then gather to Morton order
//   topology compressed oct-tree read off the sorted unique keys; nodes are
//            numbered in depth-first preorder, so more(c) = c+1 and
//            next(c) = c + subtree size (Sec. 4.4, next/more pointers)
//   moments  FP64 mass and centre of mass, children folded left in octant
//            order, one pass per tree level, deepest first (Sec. 4.4), and
//            the distance s of Eq. (2)
//
// Determinism: integer work is exact; the FP64 sums have a fixed order and use
// only correctly rounded +, *, /, sqrt and fma, so the node set and every node
// value are bit-identical from run to run and independent of launch shapes.
#include "bh_internal.h"

namespace bh {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive block scan of one value per thread (blockDim.x = nwaves*64).
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* lds, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = wave_incl_scan(v, lane);
  if (lane == 63) lds[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    int s = lds[k];
    pre += (k < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------- scan (int32)
// Device-wide exclusive scan: tile sums, scan of tile sums, per-tile apply.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* __restrict__ in, int n,
                                                               int32_t* __restrict__ tile_sums) {
  __shared__ int lds[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll 4
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kScanThreads + threadIdx.x;
    s += (i < n) ? in[i] : 0;
  }
  int tot;
  block_excl_scan<kScanThreads>(s, lds, &tot);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the tile sums in place; total to *total.
__global__ __launch_bounds__(1024) void k_scan_tiles(int32_t* __restrict__ sums, int ntiles,
                                                     int32_t* __restrict__ total) {
  __shared__ int lds[16];
  const int t = threadIdx.x;
  int per = (ntiles + 1023) / 1024;
  int b = t * per, e = min(ntiles, b + per);
  int s = 0;
  for (int k = b; k < e; ++k) s += sums[k];
  int tot;
  int pre = block_excl_scan<1024>(s, lds, &tot);
  for (int k = b; k < e; ++k) {
    int v = sums[k];
    sums[k] = pre;
    pre += v;
  }
  if (t == 0 && total) *total = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* __restrict__ in, int n,
                                                              const int32_t* __restrict__ tile_offs,
                                                              int32_t* __restrict__ out) {
  __shared__ int tile[kScanTile];
  __shared__ int lds[kScanThreads / 64];
  const int t = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kScanThreads + t;
    tile[r * kScanThreads + t] = (i < n) ? in[i] : 0;
  }
  __syncthreads();
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) s += tile[t * kScanItems + k];
  int tot;
  int pre = block_excl_scan<kScanThreads>(s, lds, &tot) + tile_offs[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    int v = tile[t * kScanItems + k];
    tile[t * kScanItems + k] = pre;
    pre += v;
  }
  __syncthreads();
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kScanThreads + t;
    if (i < n) out[i] = tile[r * kScanThreads + t];
  }
}

// k_scan_apply for at most kScanFuseTiles tiles, without the pass over the
// tile sums: each block adds up the sums of the tiles before it itself (at most
// kScanFuseTiles / kScanThreads loads per thread), which saves a launch.
constexpr int kScanFuseTiles = 2048;
__global__ __launch_bounds__(kScanThreads) void k_scan_apply_sum(const int32_t* __restrict__ in, int n,
                                                                  const int32_t* __restrict__ tile_sums,
                                                                  int32_t* __restrict__ out,
                                                                  int32_t* __restrict__ total) {
  __shared__ int tile[kScanTile];
  __shared__ int lds[kScanThreads / 64];
  const int t = threadIdx.x;
  int o = 0;
  for (int k = t; k < (int)blockIdx.x; k += kScanThreads) o += tile_sums[k];
  int off;
  block_excl_scan<kScanThreads>(o, lds, &off);
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kScanThreads + t;
    tile[r * kScanThreads + t] = (i < n) ? in[i] : 0;
  }
  __syncthreads();
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) s += tile[t * kScanItems + k];
  int tot;
  int pre = block_excl_scan<kScanThreads>(s, lds, &tot) + off;
  for (int k = 0; k < kScanItems; ++k) {
    int v = tile[t * kScanItems + k];
    tile[t * kScanItems + k] = pre;
    pre += v;
  }
  __syncthreads();
  for (int r = 0; r < kScanItems; ++r) {
    int64_t i = base + r * kScanThreads + t;
    if (i < n) out[i] = tile[r * kScanThreads + t];
  }
  if (total && t == 0 && blockIdx.x == gridDim.x - 1) *total = off + tot;
}

hipError_t scan_excl(const int32_t* in, int32_t* out, int n, int32_t* tile_buf, int32_t* total,
                     hipStream_t st) {
  int ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles == 0) ntiles = 1;
  k_scan_reduce<<<ntiles, kScanThreads, 0, st>>>(in, n, tile_buf);
  if (ntiles <= kScanFuseTiles) {
    k_scan_apply_sum<<<ntiles, kScanThreads, 0, st>>>(in, n, tile_buf, out, total);
  } else {
    k_scan_tiles<<<1, 1024, 0, st>>>(tile_buf, ntiles, total);
    k_scan_apply<<<ntiles, kScanThreads, 0, st>>>(in, n, tile_buf, out);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- bbox
template <typename T>
__global__ __launch_bounds__(256) void k_bbox_partial(const T* __restrict__ pos, const T* __restrict__ mass,
                                                      int64_t n, double* __restrict__ part,
                                                      Counts* __restrict__ cnt) {
  __shared__ double red[6][4];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = (double)pos[3 * i + d];
      if (!isfinite(v)) {
        bad = true;
      } else {
        mn[d] = fmin(mn[d], v);
        mx[d] = fmax(mx[d], v);
      }
    }
    if (!isfinite((double)mass[i])) bad = true;
  }
  if (__any(bad) && lane_id() == 0) atomicOr(&cnt->bad_input, 1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double a = mn[d], b = mx[d];
    for (int o = 32; o > 0; o >>= 1) {
      a = fmin(a, __shfl_xor(a, o, 64));
      b = fmax(b, __shfl_xor(b, o, 64));
    }
    if (lane == 0) {
      red[d][w] = a;
      red[3 + d][w] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    int k = threadIdx.x;
    double v = red[k][0];
    for (int q = 1; q < 4; ++q) v = (k < 3) ? fmin(v, red[k][q]) : fmax(v, red[k][q]);
    part[blockIdx.x * 6 + k] = v;
  }
}

// Root cube from the coordinate-wise extremes: lo = minimum corner, side L =
// largest extent (1 if every particle coincides or there is none).
__device__ void finish_cube(double lo[3], double hi[3], Cube* __restrict__ cube) {
  double L = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (!(lo[d] <= hi[d])) {  // no finite particle at all
      lo[d] = 0.0;
      hi[d] = 0.0;
    }
    double e = hi[d] - lo[d];
    if (e > L) L = e;
  }
  if (L == 0.0) L = 1.0;
  for (int d = 0; d < 3; ++d) cube->lo[d] = lo[d];
  cube->L = L;
  cube->scale = (double)kGrid / L;
}

// One wave folds the per-block extremes (min and max are exact, so the order
// does not matter).
__global__ __launch_bounds__(64) void k_bbox_final(const double* __restrict__ part, int nb, Cube* __restrict__ cube) {
  const int lane = threadIdx.x;
  double v[6];
  for (int k = 0; k < 6; ++k) v[k] = k < 3 ? INFINITY : -INFINITY;
  for (int b = lane; b < nb; b += 64)
    for (int k = 0; k < 6; ++k) v[k] = k < 3 ? fmin(v[k], part[b * 6 + k]) : fmax(v[k], part[b * 6 + k]);
  for (int k = 0; k < 6; ++k)
    for (int o = 32; o > 0; o >>= 1) {
      double u = __shfl_xor(v[k], o, 64);
      v[k] = k < 3 ? fmin(v[k], u) : fmax(v[k], u);
    }
  if (lane == 0) finish_cube(v, v + 3, cube);
}

// Offsets of a forest: off[0] = 0, nondecreasing, off[K] = n.  A violation is
// reported through bad_input; every later pass clamps ranges to [0, n], so a bad
// offset array can give wrong trees but never an access out of bounds.
__global__ __launch_bounds__(256) void k_seg_check(const int64_t* __restrict__ off, int K, int64_t n,
                                                   Counts* __restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  const int64_t v = off[k];
  bool bad = v < 0 || v > n || (k == 0 && v != 0) || (k == K && v != n) || (k < K && off[k + 1] < v);
  if (bad) atomicOr(&cnt->bad_input, 2);
}

__global__ void k_single_off(int64_t* __restrict__ off, int64_t n) {
  if (threadIdx.x == 0) {
    off[0] = 0;
    off[1] = n;
  }
}

__device__ __forceinline__ int64_t clamp_off(int64_t v, int64_t n) { return v < 0 ? 0 : (v > n ? n : v); }

// Cluster of caller index i: the k with off[k] <= i < off[k+1] (off in global
// memory or in an LDS copy).
template <typename P>
__device__ __forceinline__ int seg_of(P off, int K, int64_t i) {
  int lo = 0, hi = K;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Root cube of every cluster of a forest: one workgroup per cluster.
template <typename T>
__global__ __launch_bounds__(256) void k_bbox_seg(const T* __restrict__ pos, const T* __restrict__ mass,
                                                  const int64_t* __restrict__ off, int64_t n,
                                                  Cube* __restrict__ cube, Counts* __restrict__ cnt) {
  __shared__ double red[6][4];
  const int k = blockIdx.x;
  const int64_t b = clamp_off(off[k], n), e = max(b, clamp_off(off[k + 1], n));
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      double x = (double)pos[3 * i + d];
      if (!isfinite(x)) {
        bad = true;
      } else {
        v[d] = fmin(v[d], x);
        v[3 + d] = fmax(v[3 + d], x);
      }
    }
    if (!isfinite((double)mass[i])) bad = true;
  }
  if (__any(bad) && lane_id() == 0) atomicOr(&cnt->bad_input, 1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = 0; q < 6; ++q) {
    for (int o = 32; o > 0; o >>= 1) {
      double u = __shfl_xor(v[q], o, 64);
      v[q] = q < 3 ? fmin(v[q], u) : fmax(v[q], u);
    }
    if (lane == 0) red[q][w] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < 6; ++q)
      for (int r = 1; r < 4; ++r) red[q][0] = q < 3 ? fmin(red[q][0], red[q][r]) : fmax(red[q][0], red[q][r]);
    double lo[3] = {red[0][0], red[1][0], red[2][0]}, hi[3] = {red[3][0], red[4][0], red[5][0]};
    finish_cube(lo, hi, cube + k);
  }
}

// ---------------------------------------------------------------- Morton keys
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return (uint32_t)v;
}

// q_d = clamp(floor((x_d - lo_d) * 2^21/L), 0, 2^21-1); key interleaves the
// bits with x as the most significant bit of each triplet, so the octant of a
// child is 4*bx + 2*by + bz and key order is depth-first (Morton) order.
template <typename T>
__global__ __launch_bounds__(256) void k_keys(const T* __restrict__ pos, int n, const Cube* __restrict__ cubes,
                                              const int64_t* __restrict__ off, int K, int32_t* __restrict__ seg,
                                              uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = K > 1 ? seg_of(off, K, i) : 0;
  if (seg) seg[i] = k;
  const Cube* cube = cubes + k;
  const double sc = cube->scale;
  uint64_t q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double t = floor(((double)pos[3 * (int64_t)i + d] - cube->lo[d]) * sc);
    if (!(t >= 0.0)) t = 0.0;  // also maps a non-finite input to 0 (flagged by bbox)
    if (t > (double)(kGrid - 1)) t = (double)(kGrid - 1);
    q[d] = (uint64_t)t;
  }
  keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  idx[i] = i;
}

// ---------------------------------------------------------------- radix sort
// Digit sources of a pass: 8 bits of the key, or 8 bits of the item's cluster.
// The cluster of caller index v is a search over the cluster offsets, staged in
// LDS when they fit (the offsets are sorted and caller order keeps each cluster
// contiguous), else the per-index cluster array, which the key passes leave in
// no useful order, so that lookup is a scattered read.
enum SortDigit { kDigKey = 0, kDigSegLds = 1, kDigSegIdx = 2 };
constexpr int kSegLds = 2048;  // most cluster offsets (K + 1) staged in LDS

template <int kDig>
struct SegTable {
  // off[0..K] when the offsets sit in LDS
  int64_t off[kDig == kDigSegLds ? kSegLds : 1];
  __device__ __forceinline__ void load(const int64_t* __restrict__ g, int K) {
    if constexpr (kDig == kDigSegLds) {
      for (int k = threadIdx.x; k <= K; k += blockDim.x) off[k] = g[k];
    }
  }
  __device__ __forceinline__ uint32_t digit(uint64_t key, int32_t val, const int32_t* __restrict__ seg, int K,
                                            int shift) const {
    if constexpr (kDig == kDigKey) return (uint32_t)(key >> shift) & 255u;
    if constexpr (kDig == kDigSegLds) return ((uint32_t)seg_of(off, K, val) >> shift) & 255u;
    return ((uint32_t)seg[val] >> shift) & 255u;
  }
};

template <int kDig>
__global__ __launch_bounds__(kSortThreads) void k_rs_hist(const uint64_t* __restrict__ keys,
                                                          const int32_t* __restrict__ vals,
                                                          const int32_t* __restrict__ seg,
                                                          const int64_t* __restrict__ seg_off, int K, int n,
                                                          int shift, int32_t* __restrict__ hist, int ntiles) {
  __shared__ uint32_t h[256];
  __shared__ SegTable<kDig> tab;
  h[threadIdx.x] = 0;
  tab.load(seg_off, K);
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[tab.digit(kDig == kDigKey ? keys[i] : 0ull, kDig == kDigKey ? 0 : vals[i], seg, K, shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = (int32_t)h[threadIdx.x];
}

// Stable scatter through LDS.  Each wave takes a contiguous quarter of the
// tile and ranks its items in input order (the rank among equal digits within
// 64 items comes from 8 ballots, one per digit bit), after per-wave digit
// counts have given every wave its starting slot per digit; the items are
// placed in LDS sorted by digit, and the tile then leaves in that order, so
// that consecutive lanes write consecutive addresses of one digit's run
// instead of 8- and 4-byte pieces all over the output.
template <int kDig>
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                             const int32_t* __restrict__ vin,
                                                             const int32_t* __restrict__ seg,
                                                             const int64_t* __restrict__ seg_off, int K,
                                                             uint64_t* __restrict__ kout,
                                                             int32_t* __restrict__ vout, int n, int shift,
                                                             const int32_t* __restrict__ offs, int ntiles) {
  constexpr int kWaves = kSortThreads / 64;
  constexpr int kPerWave = kSortTile / kWaves;
  __shared__ uint64_t lkey[kSortTile];
  __shared__ int32_t lval[kSortTile];
  __shared__ uint8_t ldig[kSortTile];
  __shared__ uint32_t goff[256];          // output position of the tile's first item of each digit
  __shared__ uint32_t loff[256];          // tile position of the first item of each digit
  __shared__ uint32_t wslot[kWaves][256]; // per wave: its counts, then its next slot per digit
  __shared__ uint32_t wsum[kWaves];
  __shared__ SegTable<kDig> tab;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const int m = (int)min((int64_t)kSortTile, (int64_t)n - tile0);  // items in this tile
  goff[t] = (uint32_t)offs[(int64_t)t * ntiles + blockIdx.x];
#pragma unroll
  for (int k = 0; k < kWaves; ++k) wslot[k][t] = 0;
  tab.load(seg_off, K);
  __syncthreads();
  // per-wave digit counts
  for (int r = 0; r < kPerWave / 64; ++r) {
    const int j = w * kPerWave + r * 64 + lane;
    if (j < m) {
      const int64_t i = tile0 + j;
      atomicAdd(&wslot[w][tab.digit(kDig == kDigKey ? kin[i] : 0ull, kDig == kDigKey ? 0 : vin[i], seg, K, shift)], 1u);
    }
  }
  __syncthreads();
  {
    // digit t: tile total, exclusive scan over digits, then each wave's first slot
    uint32_t cw[kWaves];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      cw[k] = wslot[k][t];
      c += cw[k];
    }
    uint32_t x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    const uint32_t first = before + x - c;
    loff[t] = first;
    uint32_t run = first;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      wslot[k][t] = run;
      run += cw[k];
    }
  }
  __syncthreads();
  // each wave places its items in input order; the slots it advances are its own
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint64_t le = lt | (1ull << lane);
  for (int r = 0; r < kPerWave / 64; ++r) {
    const int j = w * kPerWave + r * 64 + lane;
    const bool valid = j < m;
    const int64_t i = tile0 + j;
    const uint64_t key = valid ? kin[i] : 0ull;
    const int32_t val = valid ? vin[i] : 0;
    const uint32_t d = valid ? tab.digit(key, val, seg, K, shift) : 0u;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t mk = ballot(bit);
      peers &= bit ? mk : ~mk;
    }
    if (valid) {
      const uint32_t q = wslot[w][d] + (uint32_t)__popcll(peers & lt);
      lkey[q] = key;
      lval[q] = val;
      ldig[q] = (uint8_t)d;
    }
    // (the wave's LDS operations take effect in program order: every lane has
    // read its slot above before the last lane of each digit advances it)
    if (valid && (peers & ~le) == 0ull) wslot[w][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // the tile in digit order: position j holds the (j - loff[d])-th item of digit d
  for (int r = 0; r < kSortItems; ++r) {
    const int j = r * kSortThreads + t;
    if (j < m) {
      const uint32_t d = ldig[j];
      const uint32_t q = goff[d] + (uint32_t)j - loff[d];
      kout[q] = lkey[j];
      vout[q] = lval[j];
    }
  }
}

__global__ __launch_bounds__(256) void k_copy_kv(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                 uint64_t* __restrict__ kout, int32_t* __restrict__ vout, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  kout[i] = kin[i];
  vout[i] = vin[i];
}

// ---------------------------------------------------------------- gather
template <typename T, typename T4>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ pos, const T* __restrict__ mass,
                                                const int32_t* __restrict__ perm, const int32_t* __restrict__ seg,
                                                int n, T4* __restrict__ ps, int32_t* __restrict__ scid) {
  // (Morton neighbours often sit close together in the caller's order, e.g.
  // particles of one cluster: runs of consecutive blocks per XCD keep their
  // source lines in one L2)
  const int k = remap_block(blockIdx.x, gridDim.x, 64) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int64_t j = perm[k];
  if (scid) scid[k] = seg[j];
  T4 v;
  v.x = pos[3 * j];
  v.y = pos[3 * j + 1];
  v.z = pos[3 * j + 2];
  v.w = mass[j];
  ps[k] = v;
}

// ---------------------------------------------------------------- unique keys
// A leaf per distinct (cluster, key).
__global__ __launch_bounds__(256) void k_unique_flags(const uint64_t* __restrict__ keys,
                                                      const int32_t* __restrict__ scid, int n,
                                                      int32_t* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || keys[i] != keys[i - 1] || (scid && scid[i] != scid[i - 1])) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_unique_write(const uint64_t* __restrict__ keys,
                                                      const int32_t* __restrict__ scid, int n,
                                                      const int32_t* __restrict__ flag,
                                                      const int32_t* __restrict__ uid,
                                                      uint64_t* __restrict__ ukey, int32_t* __restrict__ ustart,
                                                      int32_t* __restrict__ ucid, Counts* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) {
    ukey[uid[i]] = keys[i];
    ustart[uid[i]] = i;
    if (ucid) ucid[uid[i]] = scid[i];
  }
  if (i == n - 1) {
    int U = uid[i] + flag[i];
    ustart[U] = n;
    cnt->n_unique = U;
  }
}

// First unique key of every cluster (the sort keeps cluster k at Morton
// positions [off[k], off[k+1])); U for an empty trailing cluster.
__global__ __launch_bounds__(256) void k_croot_first(const int64_t* __restrict__ off, int K, int n,
                                                     const int32_t* __restrict__ uid,
                                                     const Counts* __restrict__ cnt, int32_t* __restrict__ croot) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  const int64_t b = clamp_off(off[k], n);
  croot[k] = b < n ? uid[b] : cnt->n_unique;
}

// Preorder id of the cluster's root: the shallowest node starting at its first
// unique key u, u + #internal nodes starting before u; for k = K the node count.
__global__ __launch_bounds__(256) void k_croot_final(int K, const int32_t* __restrict__ nexcl,
                                                     int32_t* __restrict__ croot) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  const int u = croot[k];
  croot[k] = u + nexcl[u];
}

// ---------------------------------------------------------------- topology
// Level of the deepest cell that holds both keys: 3*level leading bits of the
// 63-bit keys agree.  For distinct keys this is the level of the oct-tree cell
// whose children separate them.
__device__ __forceinline__ int split_level(uint64_t a, uint64_t b) {
  int lcp = __clzll((long long)(a ^ b)) - 1;  // bit 63 is always 0
  return lcp / 3;
}

__device__ __forceinline__ bool same_cell(uint64_t a, uint64_t b, int level) {
  return level == 0 || ((a ^ b) >> (63 - 3 * level)) == 0ull;
}

// For each pair of adjacent unique keys j, j+1 with split level s, the
// oct-tree cell (s, prefix) exists and has j|j+1 as one of its child
// boundaries.  Its key range [f, l] is found by galloping + binary search
// (keys are sorted, so a range shares a prefix iff its ends do).  The pair is
// the cell's representative iff it is the first child boundary in the range.
//
// Keys of different clusters share no cell: such a pair gets split level -1 and
// bounds every search.
//
// The keys of the block's 256 pairs and of kPairHalo keys on either side are
// staged in LDS first: most cells are small, so most searches stay in the
// tile, and only those that run past it read the key array in memory.
constexpr int kPairHalo = 512;
__global__ __launch_bounds__(256) void k_pairs(const uint64_t* __restrict__ ukey, const int32_t* __restrict__ ucid,
                                               const Counts* __restrict__ cnt,
                                               int32_t* __restrict__ split, int32_t* __restrict__ rep,
                                               int32_t* __restrict__ pf, int32_t* __restrict__ pl, int nmax) {
  __shared__ uint64_t tile[256 + 2 * kPairHalo];
  const int U = cnt->n_unique;
  const int j0 = blockIdx.x * blockDim.x;
  const int tlo = max(j0 - kPairHalo, 0), thi = min(j0 + (int)blockDim.x + kPairHalo, U);  // keys [tlo, thi)
  for (int t = threadIdx.x; t < thi - tlo; t += blockDim.x) tile[t] = ukey[tlo + t];
  __syncthreads();
  auto key = [&](int m) { return (m >= tlo && m < thi) ? tile[m - tlo] : ukey[m]; };
  int j = j0 + threadIdx.x;
  if (j >= nmax) return;
  if (j >= U - 1) {
    rep[j] = 0;
    return;
  }
  const int cj = ucid ? ucid[j] : 0;
  if (ucid && ucid[j + 1] != cj) {
    split[j] = -1;
    rep[j] = 0;
    return;
  }
  const uint64_t kj = key(j), kj1 = key(j + 1);
  const int s = split_level(kj, kj1);
  split[j] = s;
  auto in_cell = [&](int m, uint64_t ref) { return (!ucid || ucid[m] == cj) && same_cell(key(m), ref, s); };
  // first key of the cell: smallest f <= j with same_cell(ukey[f], kj, s)
  int lo = j, step = 1;
  while (true) {
    int cand = j - step;
    if (cand < 0 || !in_cell(cand, kj)) break;
    lo = cand;
    step <<= 1;
  }
  int hi_bad = j - step;  // < 0 or outside the cell
  int a = hi_bad, b = lo;  // invariant: a outside (or -1), b inside
  if (a < -1) a = -1;
  while (b - a > 1) {
    int m = a + (b - a) / 2;
    if (in_cell(m, kj)) b = m; else a = m;
  }
  const int f = b;
  // last key of the cell: largest l >= j+1 with same_cell(ukey[l], kj1, s)
  int up = j + 1;
  step = 1;
  while (true) {
    int cand = j + 1 + step;
    if (cand >= U || !in_cell(cand, kj1)) break;
    up = cand;
    step <<= 1;
  }
  int c = up, d = j + 1 + step;  // c inside, d outside (or U)
  if (d > U) d = U;
  while (d - c > 1) {
    int m = c + (d - c) / 2;
    if (in_cell(m, kj1)) c = m; else d = m;
  }
  const int l = c;
  bool is_rep = (f == j) || (s < kLevels - 1 && same_cell(key(f), kj, s + 1));
  rep[j] = is_rep ? 1 : 0;
  pf[j] = f;
  pl[j] = l;
}

__global__ __launch_bounds__(256) void k_internal_write(const int32_t* __restrict__ rep,
                                                        const int32_t* __restrict__ irank,
                                                        const int32_t* __restrict__ split,
                                                        const int32_t* __restrict__ pf, const int32_t* __restrict__ pl,
                                                        Counts* __restrict__ cnt, int32_t* __restrict__ ilevel,
                                                        int32_t* __restrict__ ifirst, int32_t* __restrict__ ilast,
                                                        int32_t* __restrict__ nstart, uint32_t* __restrict__ lmask,
                                                        int nmax) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nmax) return;
  const int U = cnt->n_unique;
  if (j == 0) {
    int I = (U >= 2) ? irank[U - 2] + rep[U - 2] : 0;
    cnt->n_internal = I;
    cnt->n_nodes = U + I;
  }
  if (j >= U - 1 || !rep[j]) return;
  int v = irank[j];
  int s = split[j], f = pf[j];
  ilevel[v] = s;
  ifirst[v] = f;
  ilast[v] = pl[j];
  atomicAdd(&nstart[f], 1);
  atomicOr(&lmask[f], 1u << s);
}

// Preorder: for each unique-key position x, the internal nodes whose first key
// is x (a chain of nested cells, shallowest first) come before leaf x.
//   pre(internal v) = f + #internal nodes starting before f + #shallower nodes starting at f
//   pre(leaf x)     = x + #internal nodes starting at or before x
//   next(v)         = pre(leaf last(v)) + 1
template <typename T4>
__global__ __launch_bounds__(256) void k_nodes_internal(const Counts* __restrict__ cnt, const Cube* __restrict__ cubes,
                                                        const int32_t* __restrict__ ucid,
                                                        const int32_t* __restrict__ ilevel,
                                                        const int32_t* __restrict__ ifirst,
                                                        const int32_t* __restrict__ ilast,
                                                        const int32_t* __restrict__ nstart,
                                                        const int32_t* __restrict__ nexcl,
                                                        const uint32_t* __restrict__ lmask,
                                                        const int32_t* __restrict__ ustart,
                                                        const uint64_t* __restrict__ ukey, Node* __restrict__ nodes,
                                                        int32_t* __restrict__ nx, uint8_t* __restrict__ nlev,
                                                        int nmax) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nmax || v >= cnt->n_internal) return;
  const int s = ilevel[v], f = ifirst[v], l = ilast[v];
  const int pre = f + nexcl[f] + __popc(lmask[f] & ((1u << s) - 1u));
  const Cube* cube = cubes + (ucid ? ucid[f] : 0);
  Node nd;
  nd.l = ldexp(cube->L, -s);
  // the cube's centre, in the centre-of-mass fields until the moment passes
  // replace it (they need it for s, and for the centre of a massless cell)
  const uint64_t prefix = (s == 0) ? 0ull : (ukey[f] >> (63 - 3 * s));
  nd.cx = cube->lo[0] + ((double)compact3(prefix >> 2) + 0.5) * nd.l;
  nd.cy = cube->lo[1] + ((double)compact3(prefix >> 1) + 0.5) * nd.l;
  nd.cz = cube->lo[2] + ((double)compact3(prefix) + 0.5) * nd.l;
  nd.M = 0.0;
  nd.s = 0.0;
  nd.next = l + nexcl[l] + nstart[l] + 1;
  nd.first = ustart[f];
  nd.count = ustart[l + 1] - ustart[f];
  nd.meta = s << 8;
  nodes[pre] = nd;
  nx[pre] = nd.next;
  nlev[pre] = (uint8_t)s;
}

template <typename T4>
__global__ __launch_bounds__(256) void k_nodes_leaf(const Counts* __restrict__ cnt, const Cube* __restrict__ cubes,
                                                    const int32_t* __restrict__ ucid,
                                                    const int32_t* __restrict__ split,
                                                    const int32_t* __restrict__ nstart,
                                                    const int32_t* __restrict__ nexcl,
                                                    const int32_t* __restrict__ ustart, const T4* __restrict__ ps,
                                                    Node* __restrict__ nodes, Mom* __restrict__ mom,
                                                    int32_t* __restrict__ nx, uint8_t* __restrict__ nlev, int nmax) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int U = cnt->n_unique;
  if (x >= nmax || x >= U) return;
  const int pre = x + nexcl[x] + nstart[x];
  const int first = ustart[x], count = ustart[x + 1] - first;
  const Cube* cube = cubes + (ucid ? ucid[x] : 0);
  // a leaf sits one level below the deeper of its two neighbour splits (split
  // -1 marks a cluster edge, so a cluster's only key is its level-0 root)
  int level;
  if (count > 1) {
    level = kLevels;
  } else {
    int sl = (x > 0) ? split[x - 1] : -1;
    int sr = (x < U - 1) ? split[x] : -1;
    level = 1 + max(sl, sr);
  }
  Node nd;
  double M = 0.0, X = 0.0, Y = 0.0, Z = 0.0;
  for (int k = first; k < first + count; ++k) {
    T4 p = ps[k];
    double m = (double)p.w;
    M += m;
    X += m * (double)p.x;
    Y += m * (double)p.y;
    Z += m * (double)p.z;
  }
  if (count == 1) {
    T4 p = ps[first];
    nd.cx = (double)p.x;
    nd.cy = (double)p.y;
    nd.cz = (double)p.z;
  } else if (M != 0.0) {
    nd.cx = X / M;
    nd.cy = Y / M;
    nd.cz = Z / M;
  } else {
    // massless bucket: sit at the cell centre
    const double l = ldexp(cube->L, -level);
    T4 p = ps[first];
    double c[3] = {(double)p.x, (double)p.y, (double)p.z};
    double ctr[3];
    for (int d = 0; d < 3; ++d) {
      double q = floor((c[d] - cube->lo[d]) * cube->scale);
      if (!(q >= 0.0)) q = 0.0;
      if (q > (double)(kGrid - 1)) q = (double)(kGrid - 1);
      ctr[d] = cube->lo[d] + (q + 0.5) * l;
    }
    nd.cx = ctr[0];
    nd.cy = ctr[1];
    nd.cz = ctr[2];
  }
  nd.M = M;
  nd.l = ldexp(cube->L, -level);
  nd.s = 0.0;
  nd.next = pre + 1;
  nd.first = first;
  nd.count = count;
  nd.meta = 1 | (count > 1 ? 2 : 0) | (level << 8);
  nodes[pre] = nd;
  mom[pre] = Mom{M, X, Y, Z};
  nx[pre] = pre + 1;
  nlev[pre] = (uint8_t)level;
}

// ---------------------------------------------------------------- moments
// The moments of an internal node fold its children's, in octant order (the
// preorder of the children p+1, next(p+1), ... < next(p)).  The fold runs
// bottom-up in two launches, with the same arithmetic for every node:
//  * k_moments_chunk: a workgroup loads a chunk of kChunk consecutive preorder
//    nodes (next, level, the leaves' moments) into LDS and folds there, level
//    by level (deepest first), every internal node whose subtree ends inside
//    the chunk.  The others, at most one per level, go to the chunk's slot of
//    their level's list, and k_open_kids lists their children (along next,
//    which past the chunk's end continues in memory);
//  * k_moments_top: one launch per level folds that level's listed nodes
//    from their children's records in memory.
// A node's children are deeper than it, so each fold reads finished values.

// Per-chunk index in LDS: next of every node, and the internal nodes whose
// subtree ends in the chunk grouped by level.
struct ChunkIndex {
  int32_t nx[kChunk];
  int16_t ord[kChunk];         // chunk offsets of the closed internal nodes, by level
  uint8_t lv[kChunk];
  int32_t start[kLevels + 2];  // ord range of each level
  int32_t fill[kLevels + 1];
  int32_t levels[kLevels + 1]; // the levels that have closed internal nodes, deepest first
  int32_t n_levels;
};

__device__ __forceinline__ bool chunk_leaf(const ChunkIndex& ci, int c0, int i) { return ci.nx[i] == c0 + i + 1; }

// Groups the chunk's closed internal nodes by level (ci.nx and ci.lv loaded,
// then a barrier, by the caller).  Ends with a barrier.
__device__ void chunk_sort(ChunkIndex& ci, int c0, int cn) {
  const int tid = threadIdx.x, c1 = c0 + cn;
  if (tid <= kLevels) ci.fill[tid] = 0;
  __syncthreads();
  for (int i = tid; i < cn; i += blockDim.x)
    if (!chunk_leaf(ci, c0, i) && ci.nx[i] <= c1) atomicAdd(&ci.fill[ci.lv[i]], 1);
  __syncthreads();
  if (tid < kWave) {
    // (one wave: an exclusive scan of the level counts, and the non-empty
    // levels, deepest first)
    const int cntL = tid <= kLevels ? ci.fill[tid] : 0;
    int incl = cntL;
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(incl, o, kWave);
      if (tid >= o) incl += u;
    }
    if (tid <= kLevels) ci.start[tid] = incl - cntL;
    if (tid == kLevels) ci.start[kLevels + 1] = incl;
    const uint64_t ne = __ballot(tid <= kLevels && cntL > 0);
    if (tid <= kLevels && cntL > 0) ci.levels[__popcll(ne >> (tid + 1))] = tid;
    if (tid == 0) ci.n_levels = __popcll(ne);
  }
  __syncthreads();
  if (tid <= kLevels) ci.fill[tid] = 0;
  __syncthreads();
  for (int i = tid; i < cn; i += blockDim.x) {
    if (chunk_leaf(ci, c0, i) || ci.nx[i] > c1) continue;
    const int L = ci.lv[i];
    ci.ord[ci.start[L] + atomicAdd(&ci.fill[L], 1)] = (int16_t)i;
  }
  __syncthreads();
}

__device__ __forceinline__ void add_mom(Mom& s, const Mom& q) {
  s.M += q.M;
  s.X += q.X;
  s.Y += q.Y;
  s.Z += q.Z;
}

// Centre of mass and s of node p from its folded moments q and its cube's
// centre ctr (which the node record holds until here).
__device__ __forceinline__ void finish_node(int p, const Mom& q, const double ctr[3], Node* __restrict__ nodes,
                                            Mom* __restrict__ mom) {
  double com[3];
  if (q.M != 0.0) {
    com[0] = q.X / q.M;
    com[1] = q.Y / q.M;
    com[2] = q.Z / q.M;
  } else {
    com[0] = ctr[0];
    com[1] = ctr[1];
    com[2] = ctr[2];
  }
  const double dx = ctr[0] - com[0], dy = ctr[1] - com[1], dz = ctr[2] - com[2];
  nodes[p].cx = com[0];
  nodes[p].cy = com[1];
  nodes[p].cz = com[2];
  nodes[p].M = q.M;
  nodes[p].s = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
  mom[p] = q;
}

__global__ __launch_bounds__(kChunkThreads) void k_moments_chunk(const Counts* __restrict__ cnt,
                                                                 const int32_t* __restrict__ nx,
                                                                 const uint8_t* __restrict__ nlev,
                                                                 Node* __restrict__ nodes, Mom* __restrict__ mom,
                                                                 int32_t* __restrict__ obkt, int nchunks) {
  constexpr int kItems = kChunk / kChunkThreads;
  __shared__ ChunkIndex ci;
  __shared__ Mom sm[kChunk];
  const int n_nodes = cnt->n_nodes;
  const int c0 = blockIdx.x * kChunk;
  if (c0 >= n_nodes) return;
  const int cn = min(kChunk, n_nodes - c0), c1 = c0 + cn;
  const int tid = threadIdx.x;
  int nxt[kItems];
#pragma unroll
  for (int t = 0; t < kItems; ++t) {
    const int i = tid + t * kChunkThreads;
    nxt[t] = i < cn ? nx[c0 + i] : 0;
  }
#pragma unroll
  for (int t = 0; t < kItems; ++t) {
    const int i = tid + t * kChunkThreads;
    if (i >= cn) continue;
    ci.nx[i] = nxt[t];
    ci.lv[i] = (uint8_t)min((int)nlev[c0 + i], kLevels);
    if (nxt[t] == c0 + i + 1) sm[i] = mom[c0 + i];  // a leaf
  }
  // the cube centres of this thread's closed internal nodes, for the end
  double ctr[kItems][3];
#pragma unroll
  for (int t = 0; t < kItems; ++t) {
    const int i = tid + t * kChunkThreads;
    const bool closed = i < cn && nxt[t] != c0 + i + 1 && nxt[t] <= c1;
    ctr[t][0] = closed ? nodes[c0 + i].cx : 0.0;
    ctr[t][1] = closed ? nodes[c0 + i].cy : 0.0;
    ctr[t][2] = closed ? nodes[c0 + i].cz : 0.0;
  }
  // this chunk's slot of each level's list of straddling nodes: none yet
  if (tid < kLevels) obkt[tid * nchunks + blockIdx.x] = -1;
  __syncthreads();
  chunk_sort(ci, c0, cn);
  for (int t = 0; t < ci.n_levels; ++t) {
    const int L = ci.levels[t];
    for (int j = ci.start[L] + tid; j < ci.start[L + 1]; j += kChunkThreads) {
      const int i = ci.ord[j];
      const int end = ci.nx[i] - c0;
      Mom q{0.0, 0.0, 0.0, 0.0};
      int c = i + 1;
      for (int k = 0; k < 8 && c < end; ++k, c = max(ci.nx[c] - c0, c + 1)) add_mom(q, sm[c]);
      sm[i] = q;
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < kItems; ++t) {
    const int i = tid + t * kChunkThreads;
    if (i >= cn || nxt[t] == c0 + i + 1) continue;
    if (nxt[t] <= c1) {
      finish_node(c0 + i, sm[i], ctr[t], nodes, mom);
    } else {
      // crosses the chunk's end (an ancestor of the next chunk's first node,
      // the only one of its level here): list it for its level's pass
      obkt[min((int)ci.lv[i], kLevels - 1) * nchunks + blockIdx.x] = c0 + i;
    }
  }
}

// Children of the listed straddling nodes, along next (past the chunk's end
// the chain continues in memory), -1 after the last.
__global__ __launch_bounds__(256) void k_open_kids(const Counts* __restrict__ cnt, const int32_t* __restrict__ obkt,
                                                   const int32_t* __restrict__ nx, int nchunks,
                                                   int32_t* __restrict__ okids) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (int64_t)kLevels * nchunks) return;
  const int L = (int)(slot / nchunks), j = (int)(slot - (int64_t)L * nchunks);
  const int n_nodes = cnt->n_nodes;
  if ((int64_t)j * kChunk >= n_nodes) return;  // a chunk past the last node
  const int p = obkt[slot];
  if (p < 0) return;
  int k = 0;
  if (p < n_nodes) {
    const int end = min(nx[p], n_nodes);
    for (int c = p + 1; k < 8 && c < end; ++k, c = max(nx[c], c + 1)) okids[8 * slot + k] = c;
  }
  for (; k < 8; ++k) okids[8 * slot + k] = -1;
}

__global__ __launch_bounds__(256) void k_moments_top(const Counts* __restrict__ cnt, const int32_t* __restrict__ obkt,
                                                     const int32_t* __restrict__ okids, int nchunks,
                                                     Node* __restrict__ nodes, Mom* __restrict__ mom, int L) {
  const int n_nodes = cnt->n_nodes;
  {
    const int m = min((n_nodes + kChunk - 1) / kChunk, nchunks);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
      const int slot = L * nchunks + j;
      const int p = obkt[slot];
      if (p < 0 || p >= n_nodes) continue;
      Mom q{0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < 8; ++k) {
        const int c = okids[8 * slot + k];
        if (c <= p || c >= n_nodes) break;
        add_mom(q, mom[c]);
      }
      const double ctr[3] = {nodes[p].cx, nodes[p].cy, nodes[p].cz};
      finish_node(p, q, ctr, nodes, mom);
    }
  }
}

// ---------------------------------------------------------------- driver
static inline int nblk(int64_t n, int t) { return (int)((n + t - 1) / t) > 0 ? (int)((n + t - 1) / t) : 1; }

template <typename T4>
static hipError_t hilbert_impl(int n, const BuildWs& w, hipStream_t st);

template <typename T, typename T4>
static hipError_t build_impl(const T* pos, const T* mass, int n, const BuildWs& w, const BuildFork* fork,
                             hipStream_t st) {
  hipError_t e;
  const int K = w.n_seg;
  k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(w.counts), sizeof(Counts) / 4, 0);
  if (w.seg_off == w.own_off) k_single_off<<<1, 64, 0, st>>>(w.own_off, n);
  k_seg_check<<<nblk(K + 1, 256), 256, 0, st>>>(w.seg_off, K, n, w.counts);
  // cluster roots for an empty build: every cluster starts and ends at node 0
  k_fill_i32<<<nblk(K + 1, 256), 256, 0, st>>>(w.croot, K + 1, 0);
  if (n == 0) return hipGetLastError();
  // root cubes
  if (K == 1) {
    const int nbb = w.n_bbox_blocks;
    k_bbox_partial<T><<<nbb, 256, 0, st>>>(pos, mass, n, w.bbox_part, w.counts);
    k_bbox_final<<<1, 64, 0, st>>>(w.bbox_part, nbb, w.cube);
  } else {
    k_bbox_seg<T><<<K, 256, 0, st>>>(pos, mass, w.seg_off, n, w.cube, w.counts);
  }
  // keys and stable sort by (cluster, key): 8 key passes, then the cluster digits
  // cluster ids are kept only for a forest (a single tree's are all 0)
  int32_t* seg = K > 1 ? w.seg : nullptr;
  int32_t* scid = K > 1 ? w.scid : nullptr;
  int32_t* ucid = K > 1 ? w.ucid : nullptr;
  k_keys<T><<<nblk(n, 256), 256, 0, st>>>(pos, n, w.cube, w.seg_off, K, seg, w.key_a, w.idx_a);
  const int ntiles = (n + kSortTile - 1) / kSortTile;
  int seg_passes = 0;
  for (unsigned r = (unsigned)(K - 1); r; r >>= 8) ++seg_passes;
  uint64_t *kin = w.key_a, *kout = w.key_b;
  int32_t *vin = w.idx_a, *vout = w.idx_b;
  const bool seg_lds = K + 1 <= kSegLds;
  for (int pass = 0; pass < 8 + seg_passes; ++pass) {
    const bool segp = pass >= 8;
    const int shift = segp ? 8 * (pass - 8) : 8 * pass;
    if (!segp)
      k_rs_hist<kDigKey><<<ntiles, kSortThreads, 0, st>>>(kin, vin, w.seg, w.seg_off, K, n, shift, w.hist, ntiles);
    else if (seg_lds)
      k_rs_hist<kDigSegLds><<<ntiles, kSortThreads, 0, st>>>(kin, vin, w.seg, w.seg_off, K, n, shift, w.hist, ntiles);
    else
      k_rs_hist<kDigSegIdx><<<ntiles, kSortThreads, 0, st>>>(kin, vin, w.seg, w.seg_off, K, n, shift, w.hist, ntiles);
    if ((e = scan_excl(w.hist, w.hist, 256 * ntiles, w.scan_tiles, nullptr, st)) != hipSuccess) return e;
    if (!segp)
      k_rs_scatter<kDigKey><<<ntiles, kSortThreads, 0, st>>>(kin, vin, w.seg, w.seg_off, K, kout, vout, n, shift,
                                                             w.hist, ntiles);
    else if (seg_lds)
      k_rs_scatter<kDigSegLds><<<ntiles, kSortThreads, 0, st>>>(kin, vin, w.seg, w.seg_off, K, kout, vout, n, shift,
                                                                w.hist, ntiles);
    else
      k_rs_scatter<kDigSegIdx><<<ntiles, kSortThreads, 0, st>>>(kin, vin, w.seg, w.seg_off, K, kout, vout, n, shift,
                                                                w.hist, ntiles);
    uint64_t* tk = kin; kin = kout; kout = tk;
    int32_t* tv = vin; vin = vout; vout = tv;
  }
  // the sorted data must end in key_a / idx_a
  if (kin != w.key_a) k_copy_kv<<<nblk(n, 256), 256, 0, st>>>(kin, vin, w.key_a, w.idx_a, n);
  k_gather<T, T4><<<nblk(n, 256), 256, 0, st>>>(pos, mass, w.idx_a, seg, n, reinterpret_cast<T4*>(w.ps), scid);
  if (fork) {
    if ((e = hipEventRecord(fork->fork, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(fork->side, fork->fork, 0)) != hipSuccess) return e;
    if ((e = hilbert_impl<T4>(n, w, fork->side)) != hipSuccess) return e;
    if ((e = hipEventRecord(fork->join, fork->side)) != hipSuccess) return e;
  }
  // unique (cluster, key) pairs
  k_unique_flags<<<nblk(n, 256), 256, 0, st>>>(w.key_a, scid, n, w.flag);
  if ((e = scan_excl(w.flag, w.uid, n, w.scan_tiles, nullptr, st)) != hipSuccess) return e;
  k_unique_write<<<nblk(n, 256), 256, 0, st>>>(w.key_a, scid, n, w.flag, w.uid, w.ukey, w.ustart, ucid,
                                               w.counts);
  k_croot_first<<<nblk(K + 1, 256), 256, 0, st>>>(w.seg_off, K, n, w.uid, w.counts, w.croot);
  // internal nodes
  k_pairs<<<nblk(n, 256), 256, 0, st>>>(w.ukey, ucid, w.counts, w.split, w.flag, w.pf, w.pl, n);
  if ((e = scan_excl(w.flag, w.uid, n, w.scan_tiles, nullptr, st)) != hipSuccess) return e;
  k_fill_i32<<<nblk(n + 1, 256), 256, 0, st>>>(w.nstart, n + 1, 0);
  k_fill_i32<<<nblk(n + 1, 256), 256, 0, st>>>(reinterpret_cast<int32_t*>(w.lmask), n + 1, 0);
  k_internal_write<<<nblk(n, 256), 256, 0, st>>>(w.flag, w.uid, w.split, w.pf, w.pl, w.counts, w.ilevel, w.ifirst,
                                                 w.ilast, w.nstart, w.lmask, n);
  if ((e = scan_excl(w.nstart, w.nexcl, n + 1, w.scan_tiles, nullptr, st)) != hipSuccess) return e;
  k_croot_final<<<nblk(K + 1, 256), 256, 0, st>>>(K, w.nexcl, w.croot);
  k_nodes_internal<T4><<<nblk(n, 256), 256, 0, st>>>(w.counts, w.cube, ucid, w.ilevel, w.ifirst, w.ilast,
                                                     w.nstart, w.nexcl, w.lmask, w.ustart, w.ukey, w.nodes, w.nx,
                                                     w.nlev, n);
  k_nodes_leaf<T4><<<nblk(n, 256), 256, 0, st>>>(w.counts, w.cube, ucid, w.split, w.nstart, w.nexcl, w.ustart,
                                                 reinterpret_cast<const T4*>(w.ps), w.nodes, w.mom, w.nx, w.nlev, n);
  // moments: chunks of the preorder (2n nodes at most), then the straddling
  // internal nodes
  const int nch = (int)n_chunks(n);
  k_moments_chunk<<<nch, kChunkThreads, 0, st>>>(w.counts, w.nx, w.nlev, w.nodes, w.mom, w.obkt, nch);
  k_open_kids<<<nblk((int64_t)kLevels * nch, 256), 256, 0, st>>>(w.counts, w.obkt, w.nx, nch, w.okids);
  const int tg = nblk(nch, 256);
  for (int L = kLevels - 1; L >= 0; --L)
    k_moments_top<<<tg, 256, 0, st>>>(w.counts, w.obkt, w.okids, nch, w.nodes, w.mom, L);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (fork) return hipStreamWaitEvent(st, fork->join, 0);
  return hipSuccess;
}

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  k_fill_i32<<<nblk(n, 256), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rank(const int32_t* __restrict__ perm, int n, int32_t* __restrict__ rank) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) rank[perm[k]] = k;
}

hipError_t make_rank(const int32_t* perm, int n, int32_t* rank, hipStream_t st) {
  k_rank<<<nblk(n, 256), 256, 0, st>>>(perm, n, rank);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Hilbert walk order
// The walk's targets go in groups of 64 consecutive positions of an order.  In
// Morton order a group that straddles the edge of a large cell is split between
// distant cells, which widens the group's union walk; in Hilbert order a group
// is a face-connected run of cells.  Only the coarse levels matter (measured:
// 10 levels give the full-depth order's walk on a clumpy 4M field), so the
// order sorts Morton positions by (cluster, Hilbert index of the cell
// hilbert_levels(K) below the cluster's root cube), ties in Morton order, in as
// few 8-bit passes as the key needs.

// Hilbert index of the cell (x, y, z) of a 2^b grid, by Skilling's transform
// ("Programming the Hilbert curve", AIP Conf. Proc. 707, 2004): undo the
// excess work of the Gray-code walk level by level, Gray-encode, then
// interleave with x as the most significant bit of each triplet.
__device__ __forceinline__ uint32_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int b) {
  uint32_t X[3] = {x, y, z};
  const uint32_t top = 1u << (b - 1);
  for (uint32_t q = top; q > 1; q >>= 1) {
    const uint32_t low = q - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (X[i] & q) {
        X[0] ^= low;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & low;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t q = top; q > 1; q >>= 1)
    if (X[2] & q) t ^= q - 1;
  uint32_t h = 0;
  for (int j = b - 1; j >= 0; --j)
    h = (h << 3) | ((((X[0] ^ t) >> j) & 1u) << 2) | ((((X[1] ^ t) >> j) & 1u) << 1) | (((X[2] ^ t) >> j) & 1u);
  return h;
}

static int bits_of(unsigned v) {
  int b = 0;
  for (; v; v >>= 1) ++b;
  return b;
}

// Levels of the Hilbert cells: 10 for a single tree (four passes; 8 levels in
// three passes walked 2 % slower), fewer in a forest so that the cluster id and
// the index share 32 bits where they can.
static int hilbert_levels(int K) {
  const int cbits = bits_of((unsigned)(K - 1));
  return max(5, min(10, (32 - cbits) / 3));
}

// Sort key of Morton position k: its cluster above the Hilbert index of its
// particle's cell `levels` below the cluster's root cube (the grid coordinates
// are those of the Morton keys).
template <typename T4>
__global__ __launch_bounds__(256) void k_hkeys(const T4* __restrict__ ps, int n, const Cube* __restrict__ cubes,
                                               const int32_t* __restrict__ scid, int levels,
                                               uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int cl = scid ? scid[k] : 0;
  const Cube* cube = cubes + cl;
  const T4 p = ps[k];
  const double c[3] = {(double)p.x, (double)p.y, (double)p.z};
  uint32_t q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double t = floor((c[d] - cube->lo[d]) * cube->scale);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(kGrid - 1)) t = (double)(kGrid - 1);
    q[d] = (uint32_t)t >> (kLevels - levels);
  }
  keys[k] = ((uint64_t)(uint32_t)cl << (3 * levels)) | hilbert3(q[0], q[1], q[2], levels);
  idx[k] = k;
}

template <typename T4>
static hipError_t hilbert_impl(int n, const BuildWs& w, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int K = w.n_seg;
  const int levels = hilbert_levels(K);
  const int passes = (3 * levels + bits_of((unsigned)(K - 1)) + 7) / 8;
  k_hkeys<T4><<<nblk(n, 256), 256, 0, st>>>(reinterpret_cast<const T4*>(w.ps), n, w.cube, K > 1 ? w.scid : nullptr,
                                            levels, w.hkey_a, w.horder);
  const int ntiles = (n + kSortTile - 1) / kSortTile;
  uint64_t *kin = w.hkey_a, *kout = w.hkey_b;
  int32_t *vin = w.horder, *vout = w.hidx;
  hipError_t e;
  for (int pass = 0; pass < passes; ++pass) {
    k_rs_hist<kDigKey><<<ntiles, kSortThreads, 0, st>>>(kin, vin, nullptr, w.seg_off, K, n, 8 * pass, w.hhist, ntiles);
    if ((e = scan_excl(w.hhist, w.hhist, 256 * ntiles, w.hscan, nullptr, st)) != hipSuccess) return e;
    k_rs_scatter<kDigKey><<<ntiles, kSortThreads, 0, st>>>(kin, vin, nullptr, w.seg_off, K, kout, vout, n, 8 * pass,
                                                           w.hhist, ntiles);
    uint64_t* tk = kin; kin = kout; kout = tk;
    int32_t* tv = vin; vin = vout; vout = tv;
  }
  if (vin != w.horder) k_copy_kv<<<nblk(n, 256), 256, 0, st>>>(kin, vin, kout, w.horder, n);
  return hipGetLastError();
}

// The walk order of the targets as caller indices: out[k] = perm[order[k]]
// (order: Morton positions in walk order; null = Morton order itself).
__global__ __launch_bounds__(256) void k_walk_order(const int32_t* __restrict__ order, const int32_t* __restrict__ perm,
                                                    int n, int32_t* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = perm[order ? order[k] : k];
}

hipError_t launch_walk_order(const int32_t* order, const int32_t* perm, int n, int32_t* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_walk_order<<<nblk(n, 256), 256, 0, st>>>(order, perm, n, out);
  return hipGetLastError();
}

hipError_t hilbert_order(bool f64, int n, const BuildWs& w, hipStream_t st) {
  return f64 ? hilbert_impl<double4>(n, w, st) : hilbert_impl<float4>(n, w, st);
}

// ---------------------------------------------------------------- second moments
// Quadrupole cell terms (walks of order 2) need each node's second moments
// about its centre of mass.  A leaf sums over its particles (one particle: 0);
// a cell takes its children's moments shifted to its own centre of mass by the
// parallel-axis theorem, B = sum_c (B_c + M_c d_c d_c^T) with d_c = com_c -
// com, children in octant order, one pass per level, deepest first.
__device__ __forceinline__ void put_quad(QuadRec* __restrict__ qr, int p, const double b[6]) {
  QuadRec q;
  q.bxx = b[0];
  q.bxy = b[1];
  q.bxz = b[2];
  q.byy = b[3];
  q.byz = b[4];
  q.bzz = b[5];
  const double T = b[0] + b[3] + b[5];
  q.t05 = 0.5 * T;
  q.nt15 = -1.5 * T;
  qr[p] = q;
}

// Second moments of leaf c (over its particles; one particle: zero).
template <typename T4>
__device__ __forceinline__ void leaf_quad(const Node& nd, const T4* __restrict__ ps, double b[6]) {
  for (int t = 0; t < 6; ++t) b[t] = 0.0;
  if (nd.count <= 1) return;
  for (int k = nd.first; k < nd.first + nd.count; ++k) {
    const T4 q = ps[k];
    const double m = (double)q.w;
    const double y0 = (double)q.x - nd.cx, y1 = (double)q.y - nd.cy, y2 = (double)q.z - nd.cz;
    b[0] += m * y0 * y0;
    b[1] += m * y0 * y1;
    b[2] += m * y0 * y2;
    b[3] += m * y1 * y1;
    b[4] += m * y1 * y2;
    b[5] += m * y2 * y2;
  }
}

// Child c's term of the parallel-axis fold into a parent with centre of mass
// (px, py, pz).
__device__ __forceinline__ void quad_fold(double b[6], const double cb[6], double cx, double cy, double cz, double cM,
                                          double px, double py, double pz) {
  const double d0 = cx - px, d1 = cy - py, d2 = cz - pz;
  const double m0 = cM * d0, m1 = cM * d1, m2 = cM * d2;
  b[0] += cb[0] + m0 * d0;
  b[1] += cb[1] + m0 * d1;
  b[2] += cb[2] + m0 * d2;
  b[3] += cb[3] + m1 * d1;
  b[4] += cb[4] + m1 * d2;
  b[5] += cb[5] + m2 * d2;
}

// The two launches of the first moments (k_moments_chunk, k_moments_top), for
// the second, over the same chunks: the chunk launch forms the leaves' moments
// from their particles and folds the chunk's closed nodes in LDS; the
// straddling nodes and their children are the lists the build made.
template <typename T4>
__global__ __launch_bounds__(kChunkThreads) void k_quad_chunk(const Counts* __restrict__ cnt, const int32_t* __restrict__ nx,
                                                    const uint8_t* __restrict__ nlev, const Node* __restrict__ nodes,
                                                    const T4* __restrict__ ps, QuadRec* __restrict__ qr) {
  __shared__ ChunkIndex ci;
  __shared__ double sb[kChunk][6];
  __shared__ double sc[kChunk][4];
  const int n_nodes = cnt->n_nodes;
  const int c0 = blockIdx.x * kChunk;
  if (c0 >= n_nodes) return;
  const int cn = min(kChunk, n_nodes - c0), c1 = c0 + cn;
  const int tid = threadIdx.x;
  for (int i = tid; i < cn; i += blockDim.x) {
    const int nxt = nx[c0 + i];
    const Node nd = nodes[c0 + i];
    ci.nx[i] = nxt;
    ci.lv[i] = (uint8_t)min((int)nlev[c0 + i], kLevels);
    sc[i][0] = nd.cx;
    sc[i][1] = nd.cy;
    sc[i][2] = nd.cz;
    sc[i][3] = nd.M;
    if (nxt == c0 + i + 1) {
      double b[6];
      leaf_quad(nd, ps, b);
      for (int t = 0; t < 6; ++t) sb[i][t] = b[t];
      put_quad(qr, c0 + i, b);
    }
  }
  __syncthreads();
  chunk_sort(ci, c0, cn);
  for (int t = 0; t < ci.n_levels; ++t) {
    const int L = ci.levels[t];
    for (int j = ci.start[L] + tid; j < ci.start[L + 1]; j += kChunkThreads) {
      const int i = ci.ord[j];
      const int end = ci.nx[i] - c0;
      double b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int c = i + 1;
      for (int k = 0; k < 8 && c < end; ++k, c = max(ci.nx[c] - c0, c + 1))
        quad_fold(b, sb[c], sc[c][0], sc[c][1], sc[c][2], sc[c][3], sc[i][0], sc[i][1], sc[i][2]);
      for (int q = 0; q < 6; ++q) sb[i][q] = b[q];
    }
    __syncthreads();
  }
  for (int i = tid; i < cn; i += blockDim.x)
    if (!chunk_leaf(ci, c0, i) && ci.nx[i] <= c1) put_quad(qr, c0 + i, sb[i]);
}

__global__ __launch_bounds__(256) void k_quad_top(const Counts* __restrict__ cnt, const int32_t* __restrict__ obkt,
                                                  const int32_t* __restrict__ okids, int nchunks,
                                                  const Node* __restrict__ nodes, QuadRec* __restrict__ qr, int L) {
  const int n_nodes = cnt->n_nodes;
  {
    const int m = min((n_nodes + kChunk - 1) / kChunk, nchunks);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
      const int slot = L * nchunks + j;
      const int p = obkt[slot];
      if (p < 0 || p >= n_nodes) continue;
      const Node np = nodes[p];
      double b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < 8; ++k) {
        const int c = okids[8 * slot + k];
        if (c <= p || c >= n_nodes) break;
        const Node nc = nodes[c];
        const QuadRec q = qr[c];
        const double cb[6] = {q.bxx, q.bxy, q.bxz, q.byy, q.byz, q.bzz};
        quad_fold(b, cb, nc.cx, nc.cy, nc.cz, nc.M, np.cx, np.cy, np.cz);
      }
      put_quad(qr, p, b);
    }
  }
}

template <typename T4>
static hipError_t quad_impl(int n, const BuildWs& w, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int nch = (int)n_chunks(n);
  k_quad_chunk<T4><<<nch, kChunkThreads, 0, st>>>(w.counts, w.nx, w.nlev, w.nodes, reinterpret_cast<const T4*>(w.ps),
                                                  w.qrec);
  const int tg = nblk(nch, 256);
  for (int L = kLevels - 1; L >= 0; --L)
    k_quad_top<<<tg, 256, 0, st>>>(w.counts, w.obkt, w.okids, nch, w.nodes, w.qrec, L);
  return hipGetLastError();
}

hipError_t quad_moments(bool f64, int n, const BuildWs& w, hipStream_t st) {
  return f64 ? quad_impl<double4>(n, w, st) : quad_impl<float4>(n, w, st);
}

hipError_t build_tree_f32(const float* pos, const float* mass, int n, const BuildWs& w, const BuildFork* fork,
                          hipStream_t st) {
  return build_impl<float, float4>(pos, mass, n, w, fork, st);
}

hipError_t build_tree_f64(const double* pos, const double* mass, int n, const BuildWs& w, const BuildFork* fork,
                          hipStream_t st) {
  return build_impl<double, double4>(pos, mass, n, w, fork, st);
}

}  // namespace bh
