// bh_learn.hip -- the learned opening parameter (gfx950): group features, the
// per-group force error that labels them, and the small MLP that maps features
// to theta, with its training step.  None of this is in the paper: the paper
// uses one fixed theta (Eq. (2)); here each walk group of 64 targets may get
// its own, predicted from the group's geometry and the tree around it.
//
// MLP: 8 -> 64 -> 64 -> 1, tanh-form GELU, theta = 0.2 + 0.8 sigmoid(z).
// Matrix products run on the matrix cores (v_mfma_f32_16x16x32_bf16): bf16
// operands, FP32 accumulation.  Weights are kept in FP32 (Adam state) and
// rounded to bf16 copies after every step; biases stay FP32.  One wavefront
// handles a tile of 32 rows (two 16-row MFMA blocks), staging activations and
// their transposes in LDS so that every operand fragment is one 16-byte read.
#include "bh_internal.h"

namespace bh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- bf16
// Round to nearest bfloat16, ties to even (NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 frag(const uint16_t* p) {  // 8 consecutive bf16, 16-byte aligned
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// D += A B for 16x16 tiles with K = 32.  Lane l supplies A[l%16][k], B[k][l%16]
// for its eight k of the lane group l/16 (the same k for A and B), and holds
// D[4 (l/16) + i][l%16], i = 0..3.
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;
__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + tanhf(kGeluC * (x + kGeluA * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
  const float t = tanhf(kGeluC * (x + kGeluA * x * x * x));
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * x * x);
}

// ---------------------------------------------------------------- features
// Eight scale-free descriptors of walk group g (the Morton positions at
// [64g, 64g+64) of the walk order `order`; null: the positions themselves):
//   0 log2(h / h_typ), h the AABB half-width, h_typ = L (64/N)^(1/3) / 2
//   1 |centre of mass - centre of mass of c| / l_c, c the smallest cell
//     holding the group, l_c its side
//   2 the same against the ancestor of c three levels up (or the root)
//   3 mass-weighted RMS radius about the centre of mass, / h
//   4 |centre of mass - AABB centre| / h
//   5 log10(density of the smallest cell holding the group / M_tot L^-3)
//   6 the same for that cell's parent
//   7 log2(side of that cell / h)
// N, L, M_tot are those of the cluster of the group's first Morton position
// (the whole set for one tree).
template <typename T4>
__global__ __launch_bounds__(256) void k_features(const Node* __restrict__ nodes, const T4* __restrict__ ps,
                                                  const Cube* __restrict__ cubes, const int32_t* __restrict__ scid,
                                                  const int32_t* __restrict__ croot,
                                                  const int64_t* __restrict__ seg_off, int n_seg, int n,
                                                  const int32_t* __restrict__ order, float* __restrict__ X) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = 64 * g;
  if (s0 >= n) return;
  const int s1 = min(n, s0 + 64);
  auto member = [&](int s) { return order ? min(max(order[s], 0), n - 1) : s; };
  // the group's Morton range [a, b)
  int a = n, b = 0;
  for (int s = s0; s < s1; ++s) {
    const int q = member(s);
    a = min(a, q);
    b = max(b, q + 1);
  }
  const int k = scid ? min(max(scid[a], 0), n_seg - 1) : 0;
  const double L = cubes[k].L;
  const int64_t nk64 = seg_off[k + 1] - seg_off[k];
  const double Nk = (double)(nk64 > 0 ? nk64 : 1);
  const int cap = 2 * n;
  const int root = min(max(croot[k], 0), cap - 1);
  const double Mtot = nodes[root].M;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
  for (int s = s0; s < s1; ++s) {
    const T4 p = ps[member(s)];
    const double x = (double)p.x, y = (double)p.y, z = (double)p.z, m = (double)p.w;
    lo[0] = fmin(lo[0], x); hi[0] = fmax(hi[0], x);
    lo[1] = fmin(lo[1], y); hi[1] = fmax(hi[1], y);
    lo[2] = fmin(lo[2], z); hi[2] = fmax(hi[2], z);
    M += m;
    Sx += m * x; Sy += m * y; Sz += m * z;
  }
  double h = fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]) * 0.5;
  h = fmax(h, ldexp(L, -22));
  const double gc[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
  double com[3] = {gc[0], gc[1], gc[2]};
  if (M > 0.0) {
    com[0] = Sx / M; com[1] = Sy / M; com[2] = Sz / M;
  }
  double R2 = 0.0;
  for (int s = s0; s < s1; ++s) {
    const T4 p = ps[member(s)];
    const double dx = (double)p.x - com[0], dy = (double)p.y - com[1], dz = (double)p.z - com[2];
    R2 += (double)p.w * (dx * dx + dy * dy + dz * dz);
  }
  const double rms = M > 0.0 ? sqrt(R2 / M) : 0.0;
  // smallest cell holding the group's Morton range [a, b): descend from the cluster's root while a
  // child holds the whole range (at most 21 levels of at most 8 children)
  // (path[0] = c, path[1] = its parent, ... path[3] = three levels up)
  int path[4] = {root, root, root, root};
  int c = root;
  const Node& r0 = nodes[root];
  if (r0.first <= a && r0.first + r0.count >= b) {
    for (int depth = 0; depth < 2 * kLevels && !(nodes[c].meta & 1); ++depth) {
      const int end = min(nodes[c].next, cap);
      int ch = c + 1, found = -1;
      for (int s = 0; s < 8 && ch < end; ++s) {
        const Node& nd = nodes[ch];
        if (nd.first <= a && nd.first + nd.count >= b) {
          found = ch;
          break;
        }
        ch = max(nd.next, ch + 1);
      }
      if (found < 0) break;
      path[3] = path[2];
      path[2] = path[1];
      path[1] = c;
      c = found;
      path[0] = c;
    }
  }
  const int par = path[1], anc = path[3];
  const double rho_mean = fmax(Mtot, 1e-300) / (L * L * L);
  const double lc = nodes[c].l, lp = nodes[par].l;
  float* o = X + 8 * (int64_t)g;
  o[0] = (float)log2(h / (0.5 * L * cbrt(64.0 / Nk)));
  {
    const Node& nc = nodes[c];
    const Node& na = nodes[anc];
    const double cx = com[0] - nc.cx, cy = com[1] - nc.cy, cz = com[2] - nc.cz;
    const double ax = com[0] - na.cx, ay = com[1] - na.cy, az = com[2] - na.cz;
    o[1] = (float)(sqrt(cx * cx + cy * cy + cz * cz) / nc.l);
    o[2] = (float)(sqrt(ax * ax + ay * ay + az * az) / na.l);
  }
  o[3] = (float)(rms / h);
  const double ex = com[0] - gc[0], ey = com[1] - gc[1], ez = com[2] - gc[2];
  o[4] = (float)(sqrt(ex * ex + ey * ey + ez * ez) / h);
  o[5] = (float)log10(fmax(nodes[c].M, 1e-300) / (lc * lc * lc) / rho_mean);
  o[6] = (float)log10(fmax(nodes[par].M, 1e-300) / (lp * lp * lp) / rho_mean);
  o[7] = (float)log2(lc / h);
}

hipError_t launch_features(bool f64, const Node* nodes, const void* ps, const Cube* cubes, const int32_t* scid,
                           const int32_t* croot, const int64_t* seg_off, int n_seg, int n, const int32_t* order,
                           float* X, hipStream_t st) {
  const int G = (n + 63) / 64;
  if (G == 0) return hipSuccess;
  if (f64)
    k_features<double4><<<(G + 255) / 256, 256, 0, st>>>(nodes, static_cast<const double4*>(ps), cubes, scid,
                                                         croot, seg_off, n_seg, n, order, X);
  else
    k_features<float4><<<(G + 255) / 256, 256, 0, st>>>(nodes, static_cast<const float4*>(ps), cubes, scid, croot,
                                                        seg_off, n_seg, n, order, X);
  return hipGetLastError();
}

// ---------------------------------------------------------------- group error
// RMS over walk group g's particles (as in k_features) of |a - a_ref| / |a_ref|;
// where it is within `target`, label[g] = max(label[g], theta) (labels start
// at the grid minimum).
template <typename R>
__global__ __launch_bounds__(256) void k_group_error(const R* __restrict__ acc, const double* __restrict__ ref,
                                                     const int32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ order, int n, double theta,
                                                     double target, double* __restrict__ rms,
                                                     float* __restrict__ label) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = 64 * g;
  if (s0 >= n) return;
  const int s1 = min(n, s0 + 64);
  // (a particle whose reference force is exactly zero has no relative error:
  // it is left out, and a group of only such particles has RMS 0)
  double s = 0.0;
  int m = 0;
  for (int j = s0; j < s1; ++j) {
    const int64_t o = perm[order ? min(max(order[j], 0), n - 1) : j];
    const double rx = ref[3 * o], ry = ref[3 * o + 1], rz = ref[3 * o + 2];
    const double dx = (double)acc[3 * o] - rx, dy = (double)acc[3 * o + 1] - ry, dz = (double)acc[3 * o + 2] - rz;
    const double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 > 0.0) {
      s += (dx * dx + dy * dy + dz * dz) / r2;
      ++m;
    }
  }
  const double r = m > 0 ? sqrt(s / (double)m) : 0.0;
  if (rms) rms[g] = r;
  if (label && r <= target) label[g] = fmaxf(label[g], (float)theta);
}

hipError_t launch_group_error(bool f64, const void* acc, const double* ref, const int32_t* perm,
                              const int32_t* order, int n, double theta, double target, double* rms, float* label,
                              hipStream_t st) {
  const int G = (n + 63) / 64;
  if (G == 0) return hipSuccess;
  if (f64)
    k_group_error<double><<<(G + 255) / 256, 256, 0, st>>>(static_cast<const double*>(acc), ref, perm, order, n,
                                                           theta, target, rms, label);
  else
    k_group_error<float><<<(G + 255) / 256, 256, 0, st>>>(static_cast<const float*>(acc), ref, perm, order, n,
                                                          theta, target, rms, label);
  return hipGetLastError();
}

// ---------------------------------------------------------------- MLP
struct MlpArgs {
  const float* P;        // [kMlpParams] FP32 master parameters
  const uint16_t* wb;    // [kMlpWb] bf16 copies: W1, W2, W2^T, w3
  const float* norm;     // [16]: mu[8], 1/sd[8]
};

// LDS of one wavefront: a 32-row tile, row-major and transposed copies.
struct alignas(16) TileLds {
  uint16_t xb[32][8];
  uint16_t xT[8][32];
  uint16_t h1[32][64];
  uint16_t h1T[64][32];
  uint16_t h2[32][64];
  uint16_t dp2[32][64];
  uint16_t dp2T[64][32];
  uint16_t dp1T[64][32];
  float gd1[32][64];   // gelu'(pre-activation) of the two hidden layers (gradient pass)
  float gd2[32][64];
  float dz[32];
  float tgt[32];
};

// Normalised bf16 inputs of the tile's rows (lanes 0..31 take one row each;
// rows past `rows` are zero).
template <bool kT>
__device__ __forceinline__ void load_rows(const MlpArgs& w, const float* __restrict__ X, int64_t rows, int64_t row0,
                                          const int32_t* __restrict__ idx, TileLds& s, int lane,
                                          const float* __restrict__ T) {
  if (lane < 32) {
    const int64_t row = row0 + lane;
    const bool valid = row < rows;
    const int64_t src = valid ? (idx ? (int64_t)idx[row] : row) : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float v = valid ? (X[8 * src + k] - w.norm[k]) * w.norm[8 + k] : 0.0f;
      const uint16_t hb = valid ? to_bf16(v) : (uint16_t)0;
      s.xb[lane][k] = hb;
      if constexpr (kT) s.xT[k][lane] = hb;
    }
    if constexpr (kT) s.tgt[lane] = valid ? T[src] : 0.0f;
  }
}

// Forward pass of rows 16h..16h+15 of the tile: hidden states (and, for the
// gradient pass, their transposes and the GELU slopes) to LDS; z in the lanes
// with l%16 == 0 (rows 16h + 4(l/16) + i).
template <bool kT>
__device__ __forceinline__ void fwd_half(const MlpArgs& w, TileLds& s, int h, int lane, f32x4& z) {
  const int r = lane & 15, g = lane >> 4;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // layer 1: K = 8 features, padded to 32 with zeros
  const bf16x8 ax = g == 0 ? frag(&s.xb[16 * h + r][0]) : zero8();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const bf16x8 bw = g == 0 ? frag(w.wb + kMlpW1b + (16 * nt + r) * 8) : zero8();
    const f32x4 d = mma(ax, bw, zero);
    const int col = 16 * nt + r;
    const float bias = w.P[kMlpB1 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * h + 4 * g + i;
      const float v = d[i] + bias;
      const uint16_t hb = to_bf16(gelu(v));
      s.h1[row][col] = hb;
      if constexpr (kT) {
        s.h1T[col][row] = hb;
        s.gd1[row][col] = gelu_grad(v);
      }
    }
  }
  __syncthreads();
  // layer 2: K = 64
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 d = zero;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      d = mma(frag(&s.h1[16 * h + r][32 * ks + 8 * g]), frag(w.wb + kMlpW2b + (16 * nt + r) * 64 + 32 * ks + 8 * g), d);
    const int col = 16 * nt + r;
    const float bias = w.P[kMlpB2 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float v = d[i] + bias;
      s.h2[16 * h + 4 * g + i][col] = to_bf16(gelu(v));
      if constexpr (kT) s.gd2[16 * h + 4 * g + i][col] = gelu_grad(v);
    }
  }
  __syncthreads();
  // layer 3: one output column (B is zero outside column 0)
  f32x4 d = zero;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
    d = mma(frag(&s.h2[16 * h + r][32 * ks + 8 * g]), r == 0 ? frag(w.wb + kMlpw3b + 32 * ks + 8 * g) : zero8(), d);
  const float b3 = w.P[kMlpB3];
#pragma unroll
  for (int i = 0; i < 4; ++i) z[i] = d[i] + b3;
}

// theta for every row of X: 0.2 + 0.8 sigmoid(z), times alpha, at most `cap`;
// a non-finite result is replaced by `fallback`.
__global__ __launch_bounds__(64) void k_mlp_infer(MlpArgs w, const float* __restrict__ X, int64_t rows, float alpha,
                                                  float fallback, float cap, float* __restrict__ theta) {
  __shared__ TileLds s;
  const int lane = threadIdx.x;
  const int r = lane & 15, g = lane >> 4;
  for (int64_t tile = blockIdx.x; tile * 32 < rows; tile += gridDim.x) {
    load_rows<false>(w, X, rows, tile * 32, nullptr, s, lane, nullptr);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x4 z;
      fwd_half<false>(w, s, h, lane, z);
      if (r == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t row = tile * 32 + 16 * h + 4 * g + i;
          if (row < rows) {
            float th = (0.2f + 0.8f / (1.0f + expf(-z[i]))) * alpha;
            if (!isfinite(th)) th = fallback;
            theta[row] = fminf(th, cap);
          }
        }
      }
      __syncthreads();
    }
  }
}

// Gradient of the batch loss mean((sigmoid(z) - t)^2) over the rows idx[0..B):
// every workgroup accumulates its tiles' contributions (weight gradients in
// MFMA accumulators) and writes one partial vector; k_mlp_reduce sums them in
// a fixed order.
__global__ __launch_bounds__(64) void k_mlp_grad(MlpArgs w, const float* __restrict__ X, const float* __restrict__ T,
                                                 const int32_t* __restrict__ idx, int batch,
                                                 float* __restrict__ partial) {
  __shared__ TileLds s;
  const int lane = threadIdx.x;
  const int r = lane & 15, g = lane >> 4;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gW2[4][4], gW1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW1[a] = zero;
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[a][b] = zero;
  }
  float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f};
  float gw3 = 0.f, gb3 = 0.f, loss = 0.f;
  const float scale = 2.0f / (float)batch;
  for (int64_t tile = blockIdx.x; tile * 32 < batch; tile += gridDim.x) {
    load_rows<true>(w, X, batch, tile * 32, idx, s, lane, T);
    __syncthreads();
    f32x4 z[2];
    fwd_half<true>(w, s, 0, lane, z[0]);
    fwd_half<true>(w, s, 1, lane, z[1]);
    // output error
    if (r == 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * h + 4 * g + i;
          const bool valid = tile * 32 + row < batch;
          const float y = 1.0f / (1.0f + expf(-z[h][i]));
          const float e = y - s.tgt[row];
          s.dz[row] = valid ? scale * e * y * (1.0f - y) : 0.0f;
          loss += valid ? e * e : 0.0f;
        }
    }
    __syncthreads();
    // last layer: lane l owns w3[l]
    for (int row = 0; row < 32; ++row) gw3 += s.dz[row] * from_bf16(s.h2[row][lane]);
    if (lane == 0)
      for (int row = 0; row < 32; ++row) gb3 += s.dz[row];
    // error of the second hidden layer
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int col = 16 * nt + r;
        const float w3c = from_bf16(w.wb[kMlpw3b + col]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * h + 4 * g + i;
          const float dp = s.dz[row] * w3c * s.gd2[row][col];
          gb2[nt] += dp;
          const uint16_t hb = to_bf16(dp);
          s.dp2[row][col] = hb;
          s.dp2T[col][row] = hb;
        }
      }
    __syncthreads();
    // error of the first hidden layer: dh1 = bf16(dpre2) W2
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 d = zero;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          d = mma(frag(&s.dp2[16 * h + r][32 * ks + 8 * g]),
                  frag(w.wb + kMlpW2Tb + (16 * nt + r) * 64 + 32 * ks + 8 * g), d);
        const int col = 16 * nt + r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * h + 4 * g + i;
          const float dp = d[i] * s.gd1[row][col];
          gb1[nt] += dp;
          s.dp1T[col][row] = to_bf16(dp);
        }
      }
    // dW2 += bf16(dpre2)^T h1 (contraction over the tile's 32 rows)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        gW2[mt][nt] = mma(frag(&s.dp2T[16 * mt + r][8 * g]), frag(&s.h1T[16 * nt + r][8 * g]), gW2[mt][nt]);
    __syncthreads();
    // dW1 += bf16(dpre1)^T x'
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
      gW1[mt] = mma(frag(&s.dp1T[16 * mt + r][8 * g]), r < 8 ? frag(&s.xT[r][8 * g]) : zero8(), gW1[mt]);
    __syncthreads();
  }
  // this workgroup's partial gradient
  float* out = partial + (int64_t)blockIdx.x * kMlpGradLen;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 16 * mt + 4 * g + i;
      if (r < 8) out[kMlpW1 + o * 8 + r] = gW1[mt][i];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) out[kMlpW2 + o * 64 + 16 * nt + r] = gW2[mt][nt][i];
    }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    float b1 = gb1[nt], b2 = gb2[nt];
    b1 += __shfl_xor(b1, 16, 64);
    b1 += __shfl_xor(b1, 32, 64);
    b2 += __shfl_xor(b2, 16, 64);
    b2 += __shfl_xor(b2, 32, 64);
    if (g == 0) {
      out[kMlpB1 + 16 * nt + r] = b1;
      out[kMlpB2 + 16 * nt + r] = b2;
    }
  }
  out[kMlpw3 + lane] = gw3;
  loss += __shfl_xor(loss, 16, 64);
  loss += __shfl_xor(loss, 32, 64);
  if (lane == 0) {
    out[kMlpB3] = gb3;
    out[kMlpParams] = loss;
  }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int nparts, int batch,
                                                    float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpGradLen) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += (double)partial[(int64_t)b * kMlpGradLen + p];
  grad[p] = (float)(p == kMlpParams ? s / (double)batch : s);
}

// bf16 copies of the weights (W1, W2, W2 transposed, w3) from the FP32 masters.
__device__ __forceinline__ void write_bf16_copy(const float* __restrict__ P, uint16_t* __restrict__ wb, int p) {
  if (p < kMlpB1) {
    wb[kMlpW1b + p] = to_bf16(P[p]);
  } else if (p >= kMlpW2 && p < kMlpB2) {
    const int q = p - kMlpW2, o = q / 64, i = q % 64;
    const uint16_t v = to_bf16(P[p]);
    wb[kMlpW2b + q] = v;
    wb[kMlpW2Tb + i * 64 + o] = v;
  } else if (p >= kMlpw3 && p < kMlpB3) {
    wb[kMlpw3b + (p - kMlpw3)] = to_bf16(P[p]);
  }
}

__global__ __launch_bounds__(256) void k_mlp_prepare(const float* __restrict__ P, uint16_t* __restrict__ wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpParams) write_bf16_copy(P, wb, p);
}

// One Adam step (Kingma & Ba): c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ P, const float* __restrict__ grad,
                                                  float* __restrict__ m, float* __restrict__ v, float lr, float beta1,
                                                  float beta2, float eps, float c1, float c2,
                                                  uint16_t* __restrict__ wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float gr = grad[p];
  const float mm = beta1 * m[p] + (1.0f - beta1) * gr;
  const float vv = beta2 * v[p] + (1.0f - beta2) * gr * gr;
  m[p] = mm;
  v[p] = vv;
  P[p] = P[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  write_bf16_copy(P, wb, p);
}

static inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

hipError_t launch_mlp_prepare(const float* P, uint16_t* wb, hipStream_t st) {
  k_mlp_prepare<<<blocks(kMlpParams, 256), 256, 0, st>>>(P, wb);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* P, const uint16_t* wb, const float* norm, const float* X, int64_t rows,
                            float alpha, float fallback, float cap, float* theta, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  MlpArgs w{P, wb, norm};
  const int64_t tiles = (rows + 31) / 32;
  const int grid = (int)(tiles < 4096 ? tiles : 4096);
  k_mlp_infer<<<grid, 64, 0, st>>>(w, X, rows, alpha, fallback, cap, theta);
  return hipGetLastError();
}

int mlp_grad_parts(int batch) {
  const int tiles = (batch + 31) / 32;
  return tiles < kMlpMaxParts ? tiles : kMlpMaxParts;
}

hipError_t launch_mlp_grad(const float* P, const uint16_t* wb, const float* norm, const float* X, const float* T,
                           const int32_t* idx, int batch, float* partial, float* grad, hipStream_t st) {
  MlpArgs w{P, wb, norm};
  const int parts = mlp_grad_parts(batch);
  k_mlp_grad<<<parts, 64, 0, st>>>(w, X, T, idx, batch, partial);
  k_mlp_reduce<<<blocks(kMlpGradLen, 256), 256, 0, st>>>(partial, parts, batch, grad);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, uint16_t* wb, hipStream_t st) {
  k_mlp_adam<<<blocks(kMlpParams, 256), 256, 0, st>>>(P, grad, m, v, lr, beta1, beta2, eps, c1, c2, wb);
  return hipGetLastError();
}

}  // namespace bh
