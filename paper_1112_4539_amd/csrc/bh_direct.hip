// bh_direct.hip -- brute-force O(N^2) sum of Eq. (1) for a list of targets (gfx950).
//
// Used as the accuracy judge of the tree walk (the paper compares its tree
// forces with a brute-force sum, Sec. 5, Eq. (4)) and for the tree versus
// brute-force crossover.  Sources are staged through LDS in tiles of 256;
// each thread owns one target and runs over the tile from LDS (broadcast
// reads).  The FP64 variant keeps the reference order (ascending source
// index, j == i skipped) and the reference expression, so it reproduces the
// CPU definition; the FP32 variant uses v_rsq_f32 and FMA.
#include "bh_internal.h"

namespace bh {

constexpr int kDirectThreads = 256;

template <bool kF64>
__global__ __launch_bounds__(kDirectThreads) void k_direct(const void* __restrict__ posv, const void* __restrict__ massv,
                                                           int n, const int64_t* __restrict__ targets, int nt,
                                                           double eps2, void* __restrict__ accv,
                                                           void* __restrict__ potv) {
  using R = typename std::conditional<kF64, double, float>::type;
  const R* pos = reinterpret_cast<const R*>(posv);
  const R* mass = reinterpret_cast<const R*>(massv);
  __shared__ R sx[kDirectThreads], sy[kDirectThreads], sz[kDirectThreads], sm[kDirectThreads];
  const int t = blockIdx.x * kDirectThreads + threadIdx.x;
  const int64_t ti = t < nt ? targets[t] : -1;
  const bool in_range = ti >= 0 && ti < n;   // an index outside [0, n) yields NaN outputs
  const bool valid = t < nt && in_range;
  const int64_t i = valid ? ti : -1;
  R xi = 0, yi = 0, zi = 0;
  if (valid) {
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
  }
  R ax = 0, ay = 0, az = 0, p = 0;
  const R e2 = (R)eps2;
  for (int base = 0; base < n; base += kDirectThreads) {
    const int j = base + threadIdx.x;
    if (j < n) {
      sx[threadIdx.x] = pos[3 * (int64_t)j];
      sy[threadIdx.x] = pos[3 * (int64_t)j + 1];
      sz[threadIdx.x] = pos[3 * (int64_t)j + 2];
      sm[threadIdx.x] = mass[j];
    }
    __syncthreads();
    const int cnt = min(kDirectThreads, n - base);
    for (int k = 0; k < cnt; ++k) {
      if (base + k == i) continue;
      const R dx = sx[k] - xi, dy = sy[k] - yi, dz = sz[k] - zi;
      if constexpr (kF64) {
        const double r2 = dx * dx + dy * dy + dz * dz + e2;
        if (r2 == 0.0) continue;
        const double rinv = 1.0 / sqrt(r2);
        const double mr3 = sm[k] * (rinv * rinv * rinv);
        ax += mr3 * dx;
        ay += mr3 * dy;
        az += mr3 * dz;
        p -= sm[k] * rinv;
      } else {
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, e2)));
        const float ri = (r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f;
        const float mr = sm[k] * ri;
        const float mr3 = (mr * ri) * ri;
        ax = fmaf(mr3, dx, ax);
        ay = fmaf(mr3, dy, ay);
        az = fmaf(mr3, dz, az);
        p -= mr;
      }
    }
    __syncthreads();
  }
  if (t >= nt) return;
  R* acc = reinterpret_cast<R*>(accv);
  R* pot = reinterpret_cast<R*>(potv);
  if (!valid) {
    const R nan = (R)NAN;
    ax = ay = az = p = nan;
  }
  acc[3 * (int64_t)t] = ax;
  acc[3 * (int64_t)t + 1] = ay;
  acc[3 * (int64_t)t + 2] = az;
  pot[t] = p;
}

hipError_t launch_direct(bool f64, const void* pos, const void* mass, int n, const int64_t* targets, int nt,
                         double eps, void* acc, void* pot, hipStream_t st) {
  if (nt <= 0) return hipSuccess;
  const int blocks = (nt + kDirectThreads - 1) / kDirectThreads;
  if (f64)
    k_direct<true><<<blocks, kDirectThreads, 0, st>>>(pos, mass, n, targets, nt, eps * eps, acc, pot);
  else
    k_direct<false><<<blocks, kDirectThreads, 0, st>>>(pos, mass, n, targets, nt, eps * eps, acc, pot);
  return hipGetLastError();
}

}  // namespace bh
