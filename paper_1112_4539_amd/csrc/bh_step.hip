// bh_step.hip -- the time loop around the force walk (Sec. 1: forces, orbit
// integration, repeat): kick-drift-kick leapfrog updates, and the reorder of
// the particle state into the new tree's Morton order.
//
// Sec. 5 notes that a code which rebuilds the tree every step gets the
// localized (Morton) particle order for free.  After a step the state arrays
// can be permuted into the order of the tree just built; the next step's
// build then reads nearly sorted keys and gathers nearly in place, and the
// walk's targets in input order are nearly Morton-ordered.
#include "bh_internal.h"

namespace bh {

namespace {

inline int nblk(int64_t n, int t) { return (int)((n + t - 1) / t) > 0 ? (int)((n + t - 1) / t) : 1; }

// v += dt/2 a, then x += dt v (the first kick and the drift); FP64 arithmetic,
// one rounding to the state's precision per update.
template <typename T>
__global__ __launch_bounds__(256) void k_kick_drift(T* __restrict__ pos, T* __restrict__ vel,
                                                    const T* __restrict__ acc, int64_t n3, double dt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n3) return;
  const T v = (T)((double)vel[k] + 0.5 * dt * (double)acc[k]);
  vel[k] = v;
  pos[k] = (T)((double)pos[k] + dt * (double)v);
}

// v += dt/2 a (the second kick).
template <typename T>
__global__ __launch_bounds__(256) void k_kick(T* __restrict__ vel, const T* __restrict__ acc, int64_t n3, double dt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n3) return;
  vel[k] = (T)((double)vel[k] + 0.5 * dt * (double)acc[k]);
}

// tmp[k] = src[perm[k]] for elements of `width` words of type W.
template <typename W>
__global__ __launch_bounds__(256) void k_gather_rows(const W* __restrict__ src, const int32_t* __restrict__ perm,
                                                     int n, int width, W* __restrict__ tmp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * width) return;
  const int k = (int)(t / width), c = (int)(t - (int64_t)k * width);
  tmp[t] = src[(int64_t)perm[k] * width + c];
}

template <typename W>
__global__ __launch_bounds__(256) void k_copy_rows(const W* __restrict__ tmp, int64_t m, W* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) dst[t] = tmp[t];
}

template <typename W>
hipError_t permute_rows(W* a, const int32_t* perm, int n, int width, W* tmp, hipStream_t st) {
  if (!a) return hipSuccess;
  const int64_t m = (int64_t)n * width;
  k_gather_rows<W><<<nblk(m, 256), 256, 0, st>>>(a, perm, n, width, tmp);
  k_copy_rows<W><<<nblk(m, 256), 256, 0, st>>>(tmp, m, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_kick_drift(bool f64, void* pos, void* vel, const void* acc, int n, double dt, hipStream_t st) {
  const int64_t n3 = 3 * (int64_t)n;
  if (n3 == 0) return hipSuccess;
  if (f64)
    k_kick_drift<double><<<nblk(n3, 256), 256, 0, st>>>(static_cast<double*>(pos), static_cast<double*>(vel),
                                                         static_cast<const double*>(acc), n3, dt);
  else
    k_kick_drift<float><<<nblk(n3, 256), 256, 0, st>>>(static_cast<float*>(pos), static_cast<float*>(vel),
                                                        static_cast<const float*>(acc), n3, dt);
  return hipGetLastError();
}

hipError_t launch_kick(bool f64, void* vel, const void* acc, int n, double dt, hipStream_t st) {
  const int64_t n3 = 3 * (int64_t)n;
  if (n3 == 0) return hipSuccess;
  if (f64)
    k_kick<double><<<nblk(n3, 256), 256, 0, st>>>(static_cast<double*>(vel), static_cast<const double*>(acc), n3, dt);
  else
    k_kick<float><<<nblk(n3, 256), 256, 0, st>>>(static_cast<float*>(vel), static_cast<const float*>(acc), n3, dt);
  return hipGetLastError();
}

// Permute the state into Morton order: a[k] = a_old[perm[k]] for every array
// given (null ones are skipped).  tmp holds at least 24 n bytes.
hipError_t launch_reorder(bool f64, const int32_t* perm, int n, void* pos, void* vel, void* mass, void* acc,
                          void* pot, int64_t* ids, void* tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (f64) {
    double* t = static_cast<double*>(tmp);
    if (e == hipSuccess) e = permute_rows<double>(static_cast<double*>(pos), perm, n, 3, t, st);
    if (e == hipSuccess) e = permute_rows<double>(static_cast<double*>(vel), perm, n, 3, t, st);
    if (e == hipSuccess) e = permute_rows<double>(static_cast<double*>(acc), perm, n, 3, t, st);
    if (e == hipSuccess) e = permute_rows<double>(static_cast<double*>(mass), perm, n, 1, t, st);
    if (e == hipSuccess) e = permute_rows<double>(static_cast<double*>(pot), perm, n, 1, t, st);
  } else {
    float* t = static_cast<float*>(tmp);
    if (e == hipSuccess) e = permute_rows<float>(static_cast<float*>(pos), perm, n, 3, t, st);
    if (e == hipSuccess) e = permute_rows<float>(static_cast<float*>(vel), perm, n, 3, t, st);
    if (e == hipSuccess) e = permute_rows<float>(static_cast<float*>(acc), perm, n, 3, t, st);
    if (e == hipSuccess) e = permute_rows<float>(static_cast<float*>(mass), perm, n, 1, t, st);
    if (e == hipSuccess) e = permute_rows<float>(static_cast<float*>(pot), perm, n, 1, t, st);
  }
  if (e == hipSuccess) e = permute_rows<int64_t>(ids, perm, n, 1, static_cast<int64_t*>(tmp), st);
  return e;
}

}  // namespace bh
