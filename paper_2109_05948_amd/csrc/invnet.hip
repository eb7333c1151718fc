// The paper's colour-invariant network (Section 2.3) and its training.
//
// A colouring enters as k one-hot class vectors over the n vertices; a batch
// of B colourings is an (B k) x n matrix, one row per (colouring, class).
// Layer j maps rows of width l_in to l_out:
//   Z = X Lambda + broadcast_over_classes(R Gamma) + beta,  R = class mean of X
//   hidden:  X' = LReLU_0.2(BN(Z)), BN over the B k rows per feature (batch
//            statistics in training, running estimates with momentum 0.1 in
//            evaluation; learnable scale and shift per feature)
//   output (width 1):  f = class mean of Z.
// The products of the hidden layers are GEMMs (BF16 operands, FP32
// accumulation and output) on the MFMA kernels of gemm.hip; the width-1 output layer's
// products (matrix-vector, FP32 weights), the one-hot input, class means,
// broadcasts, normalisation, activation, loss, their backward steps and
// Adam are the kernels below.  All reductions run in a fixed order.
#include <vector>

#include "gemm.h"

namespace dlm {

constexpr float kInvSlope = 0.2f;
constexpr float kBnEps = 1e-5f;
constexpr float kBnMomentum = 0.1f;

__device__ __forceinline__ uint16_t to_bf16(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// X0[(c k + i) n + v] = 1 if colour i holds vertex v in colouring c
__global__ __launch_bounds__(256) void inv_onehot_kernel(const int16_t* __restrict__ colors, int32_t n, int32_t k,
                                                         uint16_t* __restrict__ x0) {
  const int64_t row = blockIdx.x;  // c k + i
  const int c = (int)(row / k), i = (int)(row - (int64_t)c * k);
  for (int v = threadIdx.x; v < n; v += blockDim.x)
    x0[row * n + v] = colors[(size_t)c * n + v] == i ? (uint16_t)0x3f80u : (uint16_t)0u;
}

// R[c][f] = (1/k) sum_i X[c k + i][f], BF16 out
__global__ __launch_bounds__(256) void inv_class_mean_kernel(const uint16_t* __restrict__ x, int32_t k, int32_t l,
                                                             uint16_t* __restrict__ r) {
  const int c = blockIdx.y;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= l) return;
  float s = 0.f;
  for (int i = 0; i < k; ++i) s += from_bf16(x[((size_t)c * k + i) * l + f]);
  r[(size_t)c * l + f] = to_bf16(s / (float)k);
}

// Per-colouring kernels: a block of four waves covers 64 V features of one
// colouring c (V consecutive features per lane, V = 4, 2 or 1 as the layer
// width allows aligned vector access); wave w takes the class rows
// i = w, w + 4, ... and the four partial sums are combined in wave order
// through LDS.
constexpr int kTileF = 64;

template <int V>
struct vec {
  float x[V];
};

template <int V>
__device__ __forceinline__ vec<V> ldv(const float* __restrict__ p) {
  vec<V> r;
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    r.x[0] = t.x, r.x[1] = t.y, r.x[2] = t.z, r.x[3] = t.w;
  } else if constexpr (V == 2) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    r.x[0] = t.x, r.x[1] = t.y;
  } else {
    r.x[0] = *p;
  }
  return r;
}

template <int V>
__device__ __forceinline__ void stv(float* __restrict__ p, const vec<V>& v) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v.x[0], v.x[1], v.x[2], v.x[3]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(v.x[0], v.x[1]);
  } else {
    *p = v.x[0];
  }
}

// BF16 store of V values; returns the rounded values
template <int V>
__device__ __forceinline__ vec<V> stv_bf16(uint16_t* __restrict__ p, const vec<V>& v) {
  vec<V> r;
  uint16_t b[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    b[e] = to_bf16(v.x[e]);
    r.x[e] = from_bf16(b[e]);
  }
  if constexpr (V == 4) {
    *reinterpret_cast<uint2*>(p) = make_uint2((uint32_t)b[0] | ((uint32_t)b[1] << 16),
                                              (uint32_t)b[2] | ((uint32_t)b[3] << 16));
  } else if constexpr (V == 2) {
    *reinterpret_cast<uint32_t*>(p) = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
  } else {
    *p = b[0];
  }
  return r;
}

// sum over the four waves, in wave order, of the values each lane left in sh
template <int V>
__device__ __forceinline__ vec<V> sum4(float (*sh)[kTileF * 4], int lane) {
  vec<V> r;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int o = lane * V + e;
    r.x[e] = (sh[0][o] + sh[1][o]) + (sh[2][o] + sh[3][o]);
  }
  return r;
}

template <int V>
__device__ __forceinline__ void put(float (*sh)[kTileF * 4], int w, int lane, const vec<V>& v) {
#pragma unroll
  for (int e = 0; e < V; ++e) sh[w][lane * V + e] = v.x[e];
}

template <int V>
__device__ __forceinline__ vec<V> zero() {
  vec<V> r;
#pragma unroll
  for (int e = 0; e < V; ++e) r.x[e] = 0.f;
  return r;
}

// Forward normalisation statistics of colouring c over its k class rows of
// v = z + u[c] + beta: the mean and the sum of squared deviations (two
// passes; the second re-reads the block's rows from cache).
template <int V>
__global__ __launch_bounds__(256) void inv_fwd_stats_kernel(const float* __restrict__ z, const float* __restrict__ u,
                                                            const float* __restrict__ beta, int32_t k, int32_t l,
                                                            float* __restrict__ pmean, float* __restrict__ pm2) {
  __shared__ float sh[4][kTileF * 4];
  const int c = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int f = (blockIdx.x * kTileF + lane) * V;
  const bool ok = f < l;
  vec<V> add = zero<V>(), s = zero<V>(), q = zero<V>();
  const float* zc = z + (size_t)c * k * l + f;
  if (ok) {
    const vec<V> uu = ldv<V>(u + (size_t)c * l + f), bb = ldv<V>(beta + f);
#pragma unroll
    for (int e = 0; e < V; ++e) add.x[e] = uu.x[e] + bb.x[e];
#pragma unroll 4
    for (int i = w; i < k; i += 4) {
      const vec<V> t = ldv<V>(zc + (size_t)i * l);
#pragma unroll
      for (int e = 0; e < V; ++e) s.x[e] += t.x[e];
    }
  }
  put<V>(sh, w, lane, s);
  __syncthreads();
  vec<V> m = sum4<V>(sh, lane);
#pragma unroll
  for (int e = 0; e < V; ++e) m.x[e] = m.x[e] / (float)k + add.x[e];
  if (ok)
#pragma unroll 4
    for (int i = w; i < k; i += 4) {
      const vec<V> t = ldv<V>(zc + (size_t)i * l);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const float d = t.x[e] + add.x[e] - m.x[e];
        q.x[e] += d * d;
      }
    }
  __syncthreads();
  put<V>(sh, w, lane, q);
  __syncthreads();
  if (w == 0 && ok) {
    stv<V>(pmean + (size_t)c * l + f, m);
    stv<V>(pm2 + (size_t)c * l + f, sum4<V>(sh, lane));
  }
}

// Column reductions over the B colourings: a block of 16 waves covers 64
// features; wave w sums the colourings of the w-th of 16 contiguous slices
// in order, and the slices are combined in order.
constexpr int kColWaves = 16;

__device__ __forceinline__ float col_slice_sum(const float* __restrict__ p, int B, int l, int f, int w) {
  const int c0 = (int)((int64_t)B * w / kColWaves), c1 = (int)((int64_t)B * (w + 1) / kColWaves);
  float s = 0.f;
#pragma unroll 4
  for (int c = c0; c < c1; ++c) s += p[(size_t)c * l + f];
  return s;
}

__device__ __forceinline__ float col_combine(float (*sh)[kTileF], int lane) {
  float t = 0.f;
  for (int w = 0; w < kColWaves; ++w) t += sh[w][lane];
  return t;
}

// The B groups of k rows merged (equal group sizes): mean = average of the
// group means, M2 = sum of the group M2 plus k sum (group mean - mean)^2;
// biased variance M2 / (B k).  With update, the running estimates move by
// the momentum towards (mean, unbiased variance).
__global__ __launch_bounds__(1024) void inv_fwd_stats_final_kernel(const float* __restrict__ pmean,
                                                                   const float* __restrict__ pm2, int32_t B,
                                                                   int32_t k, int32_t l, float* __restrict__ mean,
                                                                   float* __restrict__ var, float* __restrict__ rm,
                                                                   float* __restrict__ rv, int32_t update) {
  __shared__ float sh[kColWaves][kTileF];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int f = blockIdx.x * kTileF + lane;
  const bool ok = f < l;
  sh[w][lane] = ok ? col_slice_sum(pmean, B, l, f, w) : 0.f;
  __syncthreads();
  const float m = col_combine(sh, lane) / (float)B;
  float q = 0.f, d2 = 0.f;
  if (ok) {
    const int c0 = (int)((int64_t)B * w / kColWaves), c1 = (int)((int64_t)B * (w + 1) / kColWaves);
    for (int c = c0; c < c1; ++c) {
      const float d = pmean[(size_t)c * l + f] - m;
      q += pm2[(size_t)c * l + f];
      d2 += d * d;
    }
  }
  __syncthreads();
  sh[w][lane] = q + (float)k * d2;
  __syncthreads();
  if (w == 0 && ok) {
    const float N = (float)B * (float)k;
    const float v = col_combine(sh, lane) / N;
    mean[f] = m;
    var[f] = v;
    if (update) {
      rm[f] = (1.f - kBnMomentum) * rm[f] + kBnMomentum * m;
      rv[f] = (1.f - kBnMomentum) * rv[f] + kBnMomentum * v * (N / (N - 1.f));
    }
  }
}

// o1[f] = sum_c p1[c][f] and o2[f] = sum_c p2[c][f] (o2 may be null)
__global__ __launch_bounds__(1024) void inv_colsum_kernel(const float* __restrict__ p1, const float* __restrict__ p2,
                                                          int32_t B, int32_t l, float* __restrict__ o1,
                                                          float* __restrict__ o2) {
  __shared__ float sh[kColWaves][kTileF];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int f = blockIdx.x * kTileF + lane;
  const bool ok = f < l;
  sh[w][lane] = ok ? col_slice_sum(p1, B, l, f, w) : 0.f;
  __syncthreads();
  if (w == 0 && ok) o1[f] = col_combine(sh, lane);
  if (!p2) return;  // uniform over the block
  __syncthreads();
  sh[w][lane] = ok ? col_slice_sum(p2, B, l, f, w) : 0.f;
  __syncthreads();
  if (w == 0 && ok) o2[f] = col_combine(sh, lane);
}

// Normalise, scale, shift and activate the k class rows of colouring c:
// X'[c k + i][f] = LReLU((z + u[c] + beta - mean) / sqrt(var + eps) gamma + mu)
// in BF16, and the class mean of the next layer R'[c][f] from those values.
template <int V>
__global__ __launch_bounds__(256) void inv_fwd_apply_kernel(const float* __restrict__ z, const float* __restrict__ u,
                                                            const float* __restrict__ beta,
                                                            const float* __restrict__ mean,
                                                            const float* __restrict__ var,
                                                            const float* __restrict__ gamma,
                                                            const float* __restrict__ mu, int32_t k, int32_t l,
                                                            uint16_t* __restrict__ xn, uint16_t* __restrict__ rn) {
  __shared__ float sh[4][kTileF * 4];
  const int c = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int f = (blockIdx.x * kTileF + lane) * V;
  const bool ok = f < l;
  vec<V> r = zero<V>();
  if (ok) {
    vec<V> a, rs, g, sf;
    const vec<V> uu = ldv<V>(u + (size_t)c * l + f), bb = ldv<V>(beta + f), mm = ldv<V>(mean + f),
                 vv = ldv<V>(var + f), gg = ldv<V>(gamma + f), ss = ldv<V>(mu + f);
#pragma unroll
    for (int e = 0; e < V; ++e) {
      a.x[e] = uu.x[e] + bb.x[e];
      rs.x[e] = 1.f / sqrtf(vv.x[e] + kBnEps);
      g.x[e] = gg.x[e];
      sf.x[e] = ss.x[e];
    }
    const size_t base = (size_t)c * k * l + f;
#pragma unroll 4
    for (int i = w; i < k; i += 4) {
      const vec<V> t = ldv<V>(z + base + (size_t)i * l);
      vec<V> y;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const float zh = (t.x[e] + a.x[e] - mm.x[e]) * rs.x[e];
        const float yy = zh * g.x[e] + sf.x[e];
        y.x[e] = yy > 0.f ? yy : kInvSlope * yy;
      }
      const vec<V> xb = stv_bf16<V>(xn + base + (size_t)i * l, y);
#pragma unroll
      for (int e = 0; e < V; ++e) r.x[e] += xb.x[e];
    }
  }
  put<V>(sh, w, lane, r);
  __syncthreads();
  if (w == 0 && ok) {
    vec<V> t = sum4<V>(sh, lane);
#pragma unroll
    for (int e = 0; e < V; ++e) t.x[e] /= (float)k;
    stv_bf16<V>(rn + (size_t)c * l + f, t);
  }
}

// Output layer (width 1), one block per colouring c: z_i = X[c k + i] . lambda
// for the k class rows (four waves, rows split round-robin, lanes over the
// features), u = R[c] . gamma, and f[c] = (1/k) sum_i z_i + u + beta.  The
// weights are the FP32 trainables; sums run in a fixed order.
__global__ __launch_bounds__(256) void inv_out_fwd_kernel(const uint16_t* __restrict__ x,
                                                          const uint16_t* __restrict__ r,
                                                          const float* __restrict__ lam,
                                                          const float* __restrict__ gam,
                                                          const float* __restrict__ beta, int32_t k, int32_t l,
                                                          float* __restrict__ out) {
  __shared__ float part[5];
  const int c = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float acc = 0.f;
  for (int i = w; i < k; i += 4) {
    const uint16_t* row = x + ((size_t)c * k + i) * l;
    float z = 0.f;
    for (int f = lane; f < l; f += 64) z += from_bf16(row[f]) * lam[f];
    acc += z;
  }
  float u = 0.f;
  if (w == 0)
    for (int f = lane; f < l; f += 64) u += from_bf16(r[(size_t)c * l + f]) * gam[f];
  for (int o = 32; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o);
    u += __shfl_xor(u, o);
  }
  if (lane == 0) {
    part[w] = acc;
    if (w == 0) part[4] = u;
  }
  __syncthreads();
  if (threadIdx.x == 0) out[c] = (part[0] + part[1] + part[2] + part[3]) / (float)k + part[4] + beta[0];
}

// MSE on one batch: df[c] = 2 (f - t) / B, loss = mean (f - t)^2, and the
// output bias gradient sum_c df[c] (one block, fixed order)
__global__ __launch_bounds__(256) void inv_mse_kernel(const float* __restrict__ f, const float* __restrict__ t,
                                                      int32_t B, float* __restrict__ df, float* __restrict__ loss,
                                                      float* __restrict__ dbeta) {
  __shared__ float part[256], pd[256];
  float s = 0.f, sd = 0.f;
  for (int c = threadIdx.x; c < B; c += 256) {
    const float d = f[c] - t[c];
    df[c] = 2.f * d / (float)B;
    s += d * d;
    sd += 2.f * d / (float)B;
  }
  part[threadIdx.x] = s;
  pd[threadIdx.x] = sd;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      part[threadIdx.x] += part[threadIdx.x + w];
      pd[threadIdx.x] += pd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (loss) *loss = part[0] / (float)B;
    *dbeta = pd[0];
  }
}

// Output layer weight gradients, per (colouring c, feature f): with
// dz = df[c] / k on every class row and du = df[c],
//   pa[c][f] = (df[c] / k) sum_i X[c k + i][f]   (summed over c: d lambda)
//   pb[c][f] = df[c] R[c][f]                      (summed over c: d gamma)
__global__ __launch_bounds__(256) void inv_out_grad_kernel(const uint16_t* __restrict__ x,
                                                           const uint16_t* __restrict__ r,
                                                           const float* __restrict__ df, int32_t k, int32_t l,
                                                           float* __restrict__ pa, float* __restrict__ pb) {
  const int c = blockIdx.y;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= l) return;
  float sx = 0.f;
  for (int i = 0; i < k; ++i) sx += from_bf16(x[((size_t)c * k + i) * l + f]);
  const float d = df[c];
  pa[(size_t)c * l + f] = d / (float)k * sx;
  pb[(size_t)c * l + f] = d * from_bf16(r[(size_t)c * l + f]);
}

// Output layer input gradients: dX[c k + i][f] = (df[c] / k) lambda[f] and
// dR[c][f] = df[c] gamma[f]
__global__ __launch_bounds__(256) void inv_out_dx_kernel(const float* __restrict__ df, const float* __restrict__ lam,
                                                         const float* __restrict__ gam, int32_t k, int32_t l,
                                                         float* __restrict__ dx, float* __restrict__ dr) {
  const int c = blockIdx.y;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= l) return;
  const float d = df[c], v = d / (float)k * lam[f];
  for (int i = 0; i < k; ++i) dx[((size_t)c * k + i) * l + f] = v;
  dr[(size_t)c * l + f] = d * gam[f];
}

// Backward through LReLU and the normalisation of a hidden layer, pass 1,
// per colouring c: with zhat recomputed from the stored z and
// dY = (dX + dR[c] / k) LReLU'(zhat gamma + mu) over the k class rows (the
// dR / k term is the class-mean path of the layer above), the partial sums
// of dY and dY zhat; summed over colourings these are the gradients of mu
// and gamma.
template <int V>
struct bn_lane {  // per-feature constants of the normalisation backward
  vec<V> a, m, rs, g, sf, drk;
};

template <int V>
__device__ __forceinline__ bn_lane<V> bn_load(const float* u, const float* beta, const float* mean, const float* var,
                                              const float* gamma, const float* mu, const float* dr, int c, int k,
                                              int l, int f) {
  bn_lane<V> b;
  const vec<V> uu = ldv<V>(u + (size_t)c * l + f), bb = ldv<V>(beta + f), vv = ldv<V>(var + f),
               dd = ldv<V>(dr + (size_t)c * l + f);
  b.m = ldv<V>(mean + f);
  b.g = ldv<V>(gamma + f);
  b.sf = ldv<V>(mu + f);
#pragma unroll
  for (int e = 0; e < V; ++e) {
    b.a.x[e] = uu.x[e] + bb.x[e];
    b.rs.x[e] = 1.f / sqrtf(vv.x[e] + kBnEps);
    b.drk.x[e] = dd.x[e] / (float)k;
  }
  return b;
}

template <int V>
__global__ __launch_bounds__(256) void inv_bwd_stats_kernel(const float* __restrict__ dx, const float* __restrict__ dr,
                                                            const float* __restrict__ z, const float* __restrict__ u,
                                                            const float* __restrict__ beta,
                                                            const float* __restrict__ mean,
                                                            const float* __restrict__ var,
                                                            const float* __restrict__ gamma,
                                                            const float* __restrict__ mu, int32_t k, int32_t l,
                                                            float* __restrict__ p1, float* __restrict__ p2) {
  __shared__ float sh1[4][kTileF * 4], sh2[4][kTileF * 4];
  const int c = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int f = (blockIdx.x * kTileF + lane) * V;
  const bool ok = f < l;
  vec<V> s1 = zero<V>(), s2 = zero<V>();
  if (ok) {
    const bn_lane<V> b = bn_load<V>(u, beta, mean, var, gamma, mu, dr, c, k, l, f);
    const size_t base = (size_t)c * k * l + f;
#pragma unroll 4
    for (int i = w; i < k; i += 4) {
      const vec<V> t = ldv<V>(z + base + (size_t)i * l), d = ldv<V>(dx + base + (size_t)i * l);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const float zh = (t.x[e] + b.a.x[e] - b.m.x[e]) * b.rs.x[e];
        const float y = zh * b.g.x[e] + b.sf.x[e];
        const float dy = (d.x[e] + b.drk.x[e]) * (y > 0.f ? 1.f : kInvSlope);
        s1.x[e] += dy;
        s2.x[e] += dy * zh;
      }
    }
  }
  put<V>(sh1, w, lane, s1);
  put<V>(sh2, w, lane, s2);
  __syncthreads();
  if (w == 0 && ok) {
    stv<V>(p1 + (size_t)c * l + f, sum4<V>(sh1, lane));
    stv<V>(p2 + (size_t)c * l + f, sum4<V>(sh2, lane));
  }
}

// Pass 2: dZ = gamma (N dY - sum dY - zhat sum dY zhat) / (N sqrt(var + eps))
// in BF16 for the products below, and per colouring dU[c][f] = sum_i dZ (BF16
// for the Gamma products, FP32 partial for the bias gradient).
template <int V>
__global__ __launch_bounds__(256) void inv_bwd_apply_kernel(const float* __restrict__ dx, const float* __restrict__ dr,
                                                            const float* __restrict__ z, const float* __restrict__ u,
                                                            const float* __restrict__ beta,
                                                            const float* __restrict__ mean,
                                                            const float* __restrict__ var,
                                                            const float* __restrict__ gamma,
                                                            const float* __restrict__ mu,
                                                            const float* __restrict__ dmu,
                                                            const float* __restrict__ dgamma, int32_t B, int32_t k,
                                                            int32_t l, uint16_t* __restrict__ dzb,
                                                            uint16_t* __restrict__ dub, float* __restrict__ pdu) {
  __shared__ float shu[4][kTileF * 4];
  const int c = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int f = (blockIdx.x * kTileF + lane) * V;
  const bool ok = f < l;
  vec<V> du = zero<V>();
  if (ok) {
    const bn_lane<V> b = bn_load<V>(u, beta, mean, var, gamma, mu, dr, c, k, l, f);
    const vec<V> s1 = ldv<V>(dmu + f), s2 = ldv<V>(dgamma + f);
    const float N = (float)B * (float)k;
    vec<V> scale;
#pragma unroll
    for (int e = 0; e < V; ++e) scale.x[e] = b.g.x[e] * b.rs.x[e] / N;
    const size_t base = (size_t)c * k * l + f;
#pragma unroll 4
    for (int i = w; i < k; i += 4) {
      const vec<V> t = ldv<V>(z + base + (size_t)i * l), d = ldv<V>(dx + base + (size_t)i * l);
      vec<V> v;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const float zh = (t.x[e] + b.a.x[e] - b.m.x[e]) * b.rs.x[e];
        const float y = zh * b.g.x[e] + b.sf.x[e];
        const float dy = (d.x[e] + b.drk.x[e]) * (y > 0.f ? 1.f : kInvSlope);
        v.x[e] = scale.x[e] * (N * dy - s1.x[e] - zh * s2.x[e]);
        du.x[e] += v.x[e];
      }
      stv_bf16<V>(dzb + base + (size_t)i * l, v);
    }
  }
  put<V>(shu, w, lane, du);
  __syncthreads();
  if (w == 0 && ok) {
    const vec<V> t = sum4<V>(shu, lane);
    stv_bf16<V>(dub + (size_t)c * l + f, t);
    stv<V>(pdu + (size_t)c * l + f, t);
  }
}

// Where each layer's trainables start in the packed FP32 array, where its
// Lambda and Gamma end (beta follows them), and where their BF16 copy starts
constexpr int kMaxLayers = 64;
struct inv_layout {
  int64_t start[kMaxLayers + 1];  // start[nl] = total
  int64_t lg_end[kMaxLayers];
  int64_t bf[kMaxLayers];
  int32_t nl;
};

__device__ __forceinline__ float adam_one(float p, float& m, float& v, float g, float lr, float bc1, float bc2) {
  m = 0.9f * m + 0.1f * g;
  v = 0.999f * v + 0.001f * g * g;
  return p - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
}

// Adam over all trainables, four consecutive values per thread (16-byte
// accesses; the array is 256-byte aligned); a value of some Lambda or Gamma
// also refreshes its BF16 copy
__global__ __launch_bounds__(256) void inv_adam_kernel(float* __restrict__ P, float* __restrict__ M,
                                                       float* __restrict__ V, const float* __restrict__ G, int64_t total,
                                                       float lr, float bc1, float bc2, uint16_t* __restrict__ pb,
                                                       const inv_layout lay) {
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (e0 >= total) return;
  float p[4], m[4], v[4], g[4];
  const int cnt = total - e0 >= 4 ? 4 : (int)(total - e0);
  if (cnt == 4) {
    const float4 tp = *reinterpret_cast<const float4*>(P + e0), tm = *reinterpret_cast<const float4*>(M + e0),
                 tv = *reinterpret_cast<const float4*>(V + e0), tg = *reinterpret_cast<const float4*>(G + e0);
    p[0] = tp.x, p[1] = tp.y, p[2] = tp.z, p[3] = tp.w;
    m[0] = tm.x, m[1] = tm.y, m[2] = tm.z, m[3] = tm.w;
    v[0] = tv.x, v[1] = tv.y, v[2] = tv.z, v[3] = tv.w;
    g[0] = tg.x, g[1] = tg.y, g[2] = tg.z, g[3] = tg.w;
  } else {
    for (int q = 0; q < cnt; ++q) p[q] = P[e0 + q], m[q] = M[e0 + q], v[q] = V[e0 + q], g[q] = G[e0 + q];
  }
  int j = 0;
  while (j + 1 < lay.nl && lay.start[j + 1] <= e0) ++j;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q >= cnt) break;
    const int64_t e = e0 + q;
    while (j + 1 < lay.nl && lay.start[j + 1] <= e) ++j;
    p[q] = adam_one(p[q], m[q], v[q], g[q], lr, bc1, bc2);
    if (e < lay.lg_end[j]) pb[lay.bf[j] + (e - lay.start[j])] = to_bf16(p[q]);
  }
  if (cnt == 4) {
    *reinterpret_cast<float4*>(P + e0) = make_float4(p[0], p[1], p[2], p[3]);
    *reinterpret_cast<float4*>(M + e0) = make_float4(m[0], m[1], m[2], m[3]);
    *reinterpret_cast<float4*>(V + e0) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    for (int q = 0; q < cnt; ++q) P[e0 + q] = p[q], M[e0 + q] = m[q], V[e0 + q] = v[q];
  }
}

__global__ __launch_bounds__(256) void inv_to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                          int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = to_bf16(src[e]);
}

// dst[c][r] = src[r][c] for a rows x cols BF16 matrix: a 64 x 64 tile per
// workgroup through LDS (the hidden layers' Lambda^T and Gamma^T, which make
// both operands of the forward products K-contiguous)
__global__ __launch_bounds__(256) void inv_transpose_kernel(const uint16_t* __restrict__ src, int32_t rows,
                                                            int32_t cols, uint16_t* __restrict__ dst) {
  __shared__ uint16_t t[64][66];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    if (r0 + r < rows && c0 + c < cols) t[r][c] = src[(int64_t)(r0 + r) * cols + c0 + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int c = e >> 6, r = e & 63;
    if (r0 + r < rows && c0 + c < cols) dst[(int64_t)(c0 + c) * rows + r0 + r] = t[r][c];
  }
}

}  // namespace dlm

using namespace dlm;

struct dlm_invnet {
  int n = 0, k = 0, nl = 0, max_batch = 0, device = 0;
  std::vector<int> lin, lout;
  // packed FP32 trainables per layer: L, G, beta, then gamma, mu (hidden layers)
  std::vector<int64_t> oL, oG, ob, og, om, oLb, oGb, orm, orv;
  std::vector<int> vw;  // vector width of each hidden layer's per-colouring kernels
  inv_layout layout;    // the packed trainables, for the Adam kernel
  int64_t total = 0, nrun = 0;
  float *P = nullptr, *M = nullptr, *V = nullptr, *Gr = nullptr, *run = nullptr;
  uint16_t* Pb = nullptr;  // BF16 copies of every L and G
  uint16_t* PbT = nullptr;  // BF16 Lambda^T and Gamma^T of the hidden layers ([l_out][l_in])
  bool t_fresh = false;     // PbT matches Pb (refreshed after training, not after every Adam step)
  std::vector<int64_t> oLT, oGT;  // their offsets (multiples of 8 values)
  // activations for max_batch colourings
  std::vector<uint16_t*> X;  // X[j]: BF16 [N][lin[j]]
  std::vector<uint16_t*> R;  // R[j]: BF16 [B][lin[j]]
  std::vector<float*> Z;     // Z[j]: FP32 [N][lout[j]], X Lambda before bias and normalisation
  std::vector<float*> U;     // U[j]: FP32 [B][lout[j]], R Gamma
  std::vector<float*> mean, var;  // the batch statistics of the last training forward
  float *dX = nullptr, *dR = nullptr, *df = nullptr, *fout = nullptr;
  float *pa = nullptr, *pb = nullptr;  // per-colouring partial sums [B][lmax]
  uint16_t *dZb = nullptr, *dUb = nullptr;
  // split-K partials of the products on each stream (they run concurrently)
  void *gw = nullptr, *gw_side = nullptr;
  int64_t gw_bytes = 0, gw_side_bytes = 0;
  int adam_t = 0;
  void* ws = nullptr;
  hipStream_t stream = nullptr;  // the stream of the call in progress
  // the class-mean products (one row per colouring) run on a second stream,
  // beside the class-row products of the same layer
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

// the products run on the network's current stream, the class-mean ones
// (side) on its second stream
// row-major C[rows][cols] = A[rows][inner] W[inner][cols]: from WT = W^T
// [cols][inner] when the transposed copies are fresh (both operands
// K-contiguous), else from W
int mm_rows(dlm_invnet* s, const uint16_t* A, const uint16_t* W, const uint16_t* WT, int rows, int inner, int cols,
            float* C, bool side = false) {
  if (s->t_fresh)
    return gemm_bf16(true, A, inner, true, WT, inner, C, cols, rows, cols, inner, 0, 0, side ? s->gw_side : s->gw,
                     side ? s->gw_side_bytes : s->gw_bytes, side ? s->side : s->stream);
  return gemm_bf16(true, A, inner, false, W, cols, C, cols, rows, cols, inner, 0, 0, side ? s->gw_side : s->gw,
                   side ? s->gw_side_bytes : s->gw_bytes, side ? s->side : s->stream);
}
// row-major C[inner][cols] = A[rows][inner]^T D[rows][cols]
int mm_at(dlm_invnet* s, const uint16_t* A, const uint16_t* D, int rows, int inner, int cols, float* C,
          bool side = false) {
  return gemm_bf16(false, A, inner, false, D, cols, C, cols, inner, cols, rows, 0, 0, side ? s->gw_side : s->gw,
                   side ? s->gw_side_bytes : s->gw_bytes, side ? s->side : s->stream);
}
// row-major C[rows][inner] = D[rows][cols] W[inner][cols]^T
int mm_wt(dlm_invnet* s, const uint16_t* D, const uint16_t* W, int rows, int inner, int cols, float* C,
          bool side = false) {
  return gemm_bf16(true, D, cols, true, W, cols, C, inner, rows, inner, cols, 0, 0, side ? s->gw_side : s->gw,
                   side ? s->gw_side_bytes : s->gw_bytes, side ? s->side : s->stream);
}

// the side stream starts after everything issued on st so far; st later
// waits for everything issued on the side stream so far
int fork_side(dlm_invnet* s, hipStream_t st) {
  DLM_HIP(hipEventRecord(s->ev_fork, st));
  DLM_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
  return DLM_OK;
}
int join_side(dlm_invnet* s, hipStream_t st) {
  DLM_HIP(hipEventRecord(s->ev_join, s->side));
  DLM_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
  return DLM_OK;
}

unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }
unsigned col_blocks(int64_t l) { return (unsigned)((l + kTileF - 1) / kTileF); }

// launch a per-colouring kernel with the layer's vector width (4, 2 or 1)
#define INV_VLAUNCH(kern, V, l, B, st, ...)                                                                  \
  do {                                                                                                      \
    if ((V) == 4)                                                                                           \
      hipLaunchKernelGGL(kern<4>, dim3((unsigned)(((l) + 4 * kTileF - 1) / (4 * kTileF)), (unsigned)(B)), \
                         dim3(256), 0, st, __VA_ARGS__);                                                    \
    else if ((V) == 2)                                                                                      \
      hipLaunchKernelGGL(kern<2>, dim3((unsigned)(((l) + 2 * kTileF - 1) / (2 * kTileF)), (unsigned)(B)), \
                         dim3(256), 0, st, __VA_ARGS__);                                                    \
    else                                                                                                    \
      hipLaunchKernelGGL(kern<1>, dim3((unsigned)(((l) + kTileF - 1) / kTileF), (unsigned)(B)), dim3(256), \
                         0, st, __VA_ARGS__);                                                               \
  } while (0)

// forward of a batch of B colourings; train: BN from the batch statistics
// (and, with update, the running estimates moved), else from the running
// estimates
int inv_forward(dlm_invnet* s, const int16_t* colors, int B, bool train, bool update, hipStream_t st) {
  const int k = s->k;
  const int64_t N = (int64_t)B * k;
  hipLaunchKernelGGL(inv_onehot_kernel, dim3((unsigned)N), dim3(256), 0, st, colors, s->n, k, s->X[0]);
  for (int j = 0; j < s->nl; ++j) {
    const int li = s->lin[j], lo = s->lout[j];
    if (j == 0)  // deeper class means come with the layer below's activation
      hipLaunchKernelGGL(inv_class_mean_kernel, dim3((unsigned)((li + 255) / 256), (unsigned)B), dim3(256), 0, st,
                         s->X[0], k, li, s->R[0]);
    if (j == s->nl - 1) {  // width 1: matrix-vector products, no GEMM
      hipLaunchKernelGGL(inv_out_fwd_kernel, dim3((unsigned)B), dim3(256), 0, st, s->X[j], s->R[j], s->P + s->oL[j],
                         s->P + s->oG[j], s->P + s->ob[j], k, li, s->fout);
      break;
    }
    if (!train && s->t_fresh && k >= 32) {
      // evaluation: U = R Gamma first, then X Lambda with the layer's bias,
      // normalisation (running estimates), scale, shift and LReLU applied
      // as its results are stored (BF16 X of the next layer, no FP32 Z),
      // then the class means of the new activations
      int rc = mm_rows(s, s->R[j], s->Pb + s->oGb[j], s->PbT + s->oGT[j], B, li, lo, s->U[j]);
      const GemmEval ev{s->U[j], s->P + s->ob[j], s->run + s->orm[j], s->run + s->orv[j], s->P + s->og[j],
                        s->P + s->om[j], k, kInvSlope, kBnEps, s->X[j + 1]};
      if (rc == DLM_OK)
        rc = gemm_bf16(true, s->X[j], li, true, s->PbT + s->oLT[j], li, nullptr, lo, (int)N, lo, li, 0, 0, nullptr, 0,
                       st, &ev);
      if (rc != DLM_OK) return rc;
      hipLaunchKernelGGL(inv_class_mean_kernel, dim3((unsigned)((lo + 255) / 256), (unsigned)B), dim3(256), 0, st,
                         s->X[j + 1], k, lo, s->R[j + 1]);
      continue;
    }
    int rc = fork_side(s, st);
    if (rc == DLM_OK) rc = mm_rows(s, s->R[j], s->Pb + s->oGb[j], s->PbT + s->oGT[j], B, li, lo, s->U[j], true);
    if (rc == DLM_OK) rc = mm_rows(s, s->X[j], s->Pb + s->oLb[j], s->PbT + s->oLT[j], (int)N, li, lo, s->Z[j]);
    if (rc == DLM_OK) rc = join_side(s, st);
    if (rc != DLM_OK) return rc;
    const float* mean = s->run + s->orm[j];
    const float* var = s->run + s->orv[j];
    if (train) {
      INV_VLAUNCH(inv_fwd_stats_kernel, s->vw[j], lo, B, st, s->Z[j], s->U[j], s->P + s->ob[j], k, lo, s->pa, s->pb);
      hipLaunchKernelGGL(inv_fwd_stats_final_kernel, dim3(col_blocks(lo)), dim3(1024), 0, st, s->pa, s->pb, B, k, lo,
                         s->mean[j], s->var[j], s->run + s->orm[j], s->run + s->orv[j], update ? 1 : 0);
      mean = s->mean[j];
      var = s->var[j];
    }
    INV_VLAUNCH(inv_fwd_apply_kernel, s->vw[j], lo, B, st, s->Z[j], s->U[j], s->P + s->ob[j], mean, var,
                s->P + s->og[j], s->P + s->om[j], k, lo, s->X[j + 1], s->R[j + 1]);
  }
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

// gradients of the batch MSE into s->Gr (after a training forward)
int inv_backward(dlm_invnet* s, const float* targets, int B, float* loss, hipStream_t st) {
  const int k = s->k;
  const int64_t N = (int64_t)B * k;
  const int jo = s->nl - 1;
  hipLaunchKernelGGL(inv_mse_kernel, dim3(1), dim3(256), 0, st, s->fout, targets, B, s->df, loss, s->Gr + s->ob[jo]);
  for (int j = jo; j >= 0; --j) {
    const int li = s->lin[j], lo = s->lout[j];
    const dim3 tiles((unsigned)((li + 255) / 256), (unsigned)B);
    if (j == jo) {  // width 1: no GEMM
      hipLaunchKernelGGL(inv_out_grad_kernel, tiles, dim3(256), 0, st, s->X[j], s->R[j], s->df, k, li, s->pa, s->pb);
      hipLaunchKernelGGL(inv_colsum_kernel, dim3(col_blocks(li)), dim3(1024), 0, st, s->pa, s->pb, B, li,
                         s->Gr + s->oL[j], s->Gr + s->oG[j]);
      if (j == 0) break;
      hipLaunchKernelGGL(inv_out_dx_kernel, tiles, dim3(256), 0, st, s->df, s->P + s->oL[j], s->P + s->oG[j], k, li,
                         s->dX, s->dR);
    } else {
      int rc = fork_side(s, st);
      if (rc == DLM_OK) rc = mm_at(s, s->R[j], s->dUb, B, li, lo, s->Gr + s->oG[j], true);
      if (rc == DLM_OK && j > 0) rc = mm_wt(s, s->dUb, s->Pb + s->oGb[j], B, li, lo, s->dR, true);
      if (rc == DLM_OK) rc = mm_at(s, s->X[j], s->dZb, (int)N, li, lo, s->Gr + s->oL[j]);
      if (rc == DLM_OK && j > 0) rc = mm_wt(s, s->dZb, s->Pb + s->oLb[j], (int)N, li, lo, s->dX);
      if (rc == DLM_OK) rc = join_side(s, st);
      if (rc != DLM_OK) return rc;
      if (j == 0) break;
    }
    // through LReLU and the normalisation of layer j - 1 (width li)
    const int p = j - 1;
    float* dmu = s->Gr + s->om[p];
    float* dgamma = s->Gr + s->og[p];
    INV_VLAUNCH(inv_bwd_stats_kernel, s->vw[p], li, B, st, s->dX, s->dR, s->Z[p], s->U[p], s->P + s->ob[p],
                s->mean[p], s->var[p], s->P + s->og[p], s->P + s->om[p], k, li, s->pa, s->pb);
    hipLaunchKernelGGL(inv_colsum_kernel, dim3(col_blocks(li)), dim3(1024), 0, st, s->pa, s->pb, B, li, dmu, dgamma);
    INV_VLAUNCH(inv_bwd_apply_kernel, s->vw[p], li, B, st, s->dX, s->dR, s->Z[p], s->U[p], s->P + s->ob[p],
                s->mean[p], s->var[p], s->P + s->og[p], s->P + s->om[p], dmu, dgamma, B, k, li, s->dZb, s->dUb,
                s->pa);
    hipLaunchKernelGGL(inv_colsum_kernel, dim3(col_blocks(li)), dim3(1024), 0, st, s->pa, (const float*)nullptr, B, li,
                       s->Gr + s->ob[p], (float*)nullptr);
  }
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

// Lambda^T and Gamma^T of the hidden layers from their BF16 copies
int inv_refresh_transposed(dlm_invnet* s, hipStream_t st) {
  for (int j = 0; j + 1 < s->nl; ++j) {
    const int li = s->lin[j], lo = s->lout[j];
    const dim3 grid((unsigned)((lo + 63) / 64), (unsigned)((li + 63) / 64));
    hipLaunchKernelGGL(inv_transpose_kernel, grid, dim3(256), 0, st, s->Pb + s->oLb[j], li, lo, s->PbT + s->oLT[j]);
    hipLaunchKernelGGL(inv_transpose_kernel, grid, dim3(256), 0, st, s->Pb + s->oGb[j], li, lo, s->PbT + s->oGT[j]);
  }
  DLM_HIP(hipGetLastError());
  s->t_fresh = true;
  return DLM_OK;
}

int inv_refresh_bf16(dlm_invnet* s, hipStream_t st) {
  for (int j = 0; j < s->nl; ++j) {
    const int64_t c = (int64_t)s->lin[j] * s->lout[j];
    hipLaunchKernelGGL(inv_to_bf16_kernel, dim3(blocks(c)), dim3(256), 0, st, s->P + s->oL[j], s->Pb + s->oLb[j], c);
    hipLaunchKernelGGL(inv_to_bf16_kernel, dim3(blocks(c)), dim3(256), 0, st, s->P + s->oG[j], s->Pb + s->oGb[j], c);
  }
  DLM_HIP(hipGetLastError());
  return inv_refresh_transposed(s, st);
}

int set_stream(dlm_invnet* s, hipStream_t st) {
  s->stream = st;
  return DLM_OK;
}

}  // namespace

extern "C" {

int dlm_invnet_create(int32_t n, int32_t k, int32_t nl, const int32_t* widths, const float* params_host,
                      int32_t max_batch, dlm_invnet** out) {
  if (!out || !widths || !params_host) return set_error(DLM_E_INVAL, "dlm_invnet_create: null argument");
  *out = nullptr;
  if (n < 1 || n > 32767 || k < 2 || k > 32767 || nl < 1 || nl > 64 || max_batch < 1 || max_batch > 65535)
    return set_error(DLM_E_INVAL, "dlm_invnet_create: n=%d k=%d layers=%d max_batch=%d", n, k, nl, max_batch);
  if (widths[nl - 1] != 1) return set_error(DLM_E_INVAL, "dlm_invnet_create: the last layer must have width 1");
  for (int j = 0; j < nl; ++j)
    if (widths[j] < 1 || widths[j] > 65536) return set_error(DLM_E_INVAL, "dlm_invnet_create: width %d", widths[j]);
  if ((int64_t)max_batch * k > 0x7fffffffll)  // class rows of one pass: a 32-bit GEMM dimension and grid size
    return set_error(DLM_E_INVAL, "dlm_invnet_create: max_batch * k too large");
  int device = 0;
  DLM_HIP(hipGetDevice(&device));
  dlm_invnet* s = new dlm_invnet();
  s->n = n;
  s->k = k;
  s->nl = nl;
  s->max_batch = max_batch;
  s->device = device;
  int64_t o = 0, ob16 = 0, orun = 0, lmax = n;
  for (int j = 0; j < nl; ++j) {
    const int li = j ? widths[j - 1] : n, lo = widths[j];
    s->lin.push_back(li);
    s->lout.push_back(lo);
    lmax = lmax > lo ? lmax : lo;
    s->oL.push_back(o);
    o += (int64_t)li * lo;
    s->oG.push_back(o);
    o += (int64_t)li * lo;
    s->ob.push_back(o);
    o += lo;
    s->oLb.push_back(ob16);
    ob16 += (int64_t)li * lo;
    s->oGb.push_back(ob16);
    ob16 += (int64_t)li * lo;
    if (j < nl - 1) {
      s->og.push_back(o);
      o += lo;
      s->om.push_back(o);
      o += lo;
      s->orm.push_back(orun);
      orun += lo;
      s->orv.push_back(orun);
      orun += lo;
    } else {
      s->og.push_back(-1);
      s->om.push_back(-1);
      s->orm.push_back(-1);
      s->orv.push_back(-1);
    }
  }
  s->total = o;
  s->nrun = orun;
  s->layout.nl = nl;
  for (int j = 0; j < nl; ++j) {
    s->layout.start[j] = s->oL[j];
    s->layout.lg_end[j] = s->ob[j];  // Lambda and Gamma precede beta
    s->layout.bf[j] = s->oLb[j];
  }
  s->layout.start[nl] = o;
  // vector width per hidden layer: the widest of 4, 2, 1 that divides the
  // width and every packed offset the per-colouring kernels read or write
  // (activation buffers are 256-byte aligned and their rows l values long)
  for (int j = 0; j < nl; ++j) {
    int v = 1;
    if (j < nl - 1)
      for (int c : {4, 2}) {
        const int64_t offs[] = {s->lout[j], s->ob[j], s->og[j], s->om[j], s->orm[j], s->orv[j]};
        bool fit = true;
        for (int64_t x : offs) fit = fit && x % c == 0;
        if (fit) {
          v = c;
          break;
        }
      }
    s->vw.push_back(v);
  }
  const int64_t B = max_batch, N = B * k;
  // one allocation: P, M, V, Gr, run (FP32), Pb (BF16), activations, backward buffers
  std::vector<std::pair<void**, int64_t>> parts;
  parts.push_back({(void**)&s->P, 4 * o});
  parts.push_back({(void**)&s->M, 4 * o});
  parts.push_back({(void**)&s->V, 4 * o});
  parts.push_back({(void**)&s->Gr, 4 * o});
  parts.push_back({(void**)&s->run, 4 * std::max<int64_t>(orun, 1)});
  parts.push_back({(void**)&s->Pb, 2 * ob16});
  int64_t obt = 0;
  for (int j = 0; j < nl; ++j) {
    const int64_t c = (int64_t)s->lin[j] * s->lout[j];
    s->oLT.push_back(obt);
    obt += (c + 7) & ~7ll;
    s->oGT.push_back(obt);
    obt += (c + 7) & ~7ll;
  }
  parts.push_back({(void**)&s->PbT, 2 * std::max<int64_t>(obt, 8)});
  s->X.assign(nl, nullptr);
  s->R.assign(nl, nullptr);
  s->Z.assign(nl, nullptr);
  s->U.assign(nl, nullptr);
  s->mean.assign(nl, nullptr);
  s->var.assign(nl, nullptr);
  for (int j = 0; j < nl; ++j) {
    parts.push_back({(void**)&s->X[j], 2 * N * s->lin[j]});
    parts.push_back({(void**)&s->R[j], 2 * B * s->lin[j]});
    parts.push_back({(void**)&s->Z[j], 4 * N * s->lout[j]});
    parts.push_back({(void**)&s->U[j], 4 * B * s->lout[j]});
    parts.push_back({(void**)&s->mean[j], 4 * s->lout[j]});
    parts.push_back({(void**)&s->var[j], 4 * s->lout[j]});
  }
  parts.push_back({(void**)&s->dX, 4 * N * lmax});
  parts.push_back({(void**)&s->pa, 4 * B * lmax});
  parts.push_back({(void**)&s->pb, 4 * B * lmax});
  parts.push_back({(void**)&s->dR, 4 * B * lmax});
  parts.push_back({(void**)&s->df, 4 * B});
  parts.push_back({(void**)&s->fout, 4 * B});
  parts.push_back({(void**)&s->dZb, 2 * N * lmax});
  parts.push_back({(void**)&s->dUb, 2 * B * lmax});
  // the weight gradients X^T dZ (K = the batch's class rows) may cut K into
  // chunks when their tile grid is small; size both streams' partials
  for (int j = 0; j + 1 < nl; ++j) {
    const int li = s->lin[j], lo = s->lout[j];
    s->gw_bytes = std::max(s->gw_bytes, gemm_workspace_bytes(li, lo, (int)N));
    s->gw_bytes = std::max(s->gw_bytes, gemm_workspace_bytes((int)N, lo, li));
    if (j > 0) s->gw_bytes = std::max(s->gw_bytes, gemm_workspace_bytes((int)N, li, lo));
    s->gw_side_bytes = std::max(s->gw_side_bytes, gemm_workspace_bytes(li, lo, (int)B));
    s->gw_side_bytes = std::max(s->gw_side_bytes, gemm_workspace_bytes((int)B, lo, li));
    if (j > 0) s->gw_side_bytes = std::max(s->gw_side_bytes, gemm_workspace_bytes((int)B, li, lo));
  }
  parts.push_back({&s->gw, std::max<int64_t>(s->gw_bytes, 256)});
  parts.push_back({&s->gw_side, std::max<int64_t>(s->gw_side_bytes, 256)});
  int64_t bytes = 0;
  for (auto& p : parts) bytes += (p.second + 255) & ~255ll;
  hipError_t e = hipMalloc(&s->ws, (size_t)bytes);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMalloc (invnet)");
  }
  int64_t off = 0;
  for (auto& p : parts) {
    *p.first = (unsigned char*)s->ws + off;
    off += (p.second + 255) & ~255ll;
  }
  if (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming) != hipSuccess) {
    dlm_invnet_destroy(s);
    return set_error(DLM_E_HIP, "dlm_invnet_create: second stream set-up failed");
  }
  // host parameters: the trainables, then the running estimates
  int rc = DLM_OK;
  if (hipMemcpy(s->P, params_host, 4 * o, hipMemcpyHostToDevice) != hipSuccess ||
      (orun && hipMemcpy(s->run, params_host + o, 4 * orun, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemset(s->M, 0, 4 * o) != hipSuccess || hipMemset(s->V, 0, 4 * o) != hipSuccess)
    rc = set_error(DLM_E_HIP, "dlm_invnet_create: upload failed");
  if (rc == DLM_OK) rc = inv_refresh_bf16(s, nullptr);
  if (rc == DLM_OK && hipDeviceSynchronize() != hipSuccess) rc = set_error(DLM_E_HIP, "dlm_invnet_create: sync");
  if (rc != DLM_OK) {
    dlm_invnet_destroy(s);
    return rc;
  }
  *out = s;
  return DLM_OK;
}

int dlm_invnet_destroy(dlm_invnet* s) {
  if (!s) return DLM_OK;
  if (s->side) (void)hipStreamSynchronize(s->side);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->side) (void)hipStreamDestroy(s->side);
  (void)hipFree(s->ws);
  delete s;
  return DLM_OK;
}

int dlm_invnet_num_params(const dlm_invnet* s, int64_t* trainable, int64_t* running) {
  if (!s || !trainable || !running) return set_error(DLM_E_INVAL, "dlm_invnet_num_params: null argument");
  *trainable = s->total;
  *running = s->nrun;
  return DLM_OK;
}

int dlm_invnet_get_params(const dlm_invnet* s, float* params_dev, void* stream) {
  if (!s || !params_dev) return set_error(DLM_E_INVAL, "dlm_invnet_get_params: null argument");
  hipStream_t st = (hipStream_t)stream;
  DLM_HIP(hipMemcpyAsync(params_dev, s->P, 4 * s->total, hipMemcpyDeviceToDevice, st));
  if (s->nrun) DLM_HIP(hipMemcpyAsync(params_dev + s->total, s->run, 4 * s->nrun, hipMemcpyDeviceToDevice, st));
  return DLM_OK;
}

int dlm_invnet_forward(dlm_invnet* s, const int16_t* colors, int32_t count, float* out, void* stream) {
  if (!s || count < 0 || (count > 0 && (!colors || !out))) return set_error(DLM_E_INVAL, "dlm_invnet_forward: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  int rc = set_stream(s, st);
  for (int32_t c0 = 0; rc == DLM_OK && c0 < count; c0 += s->max_batch) {
    const int B = std::min(s->max_batch, count - c0);
    rc = inv_forward(s, colors + (size_t)c0 * s->n, B, false, false, st);
    if (rc == DLM_OK) DLM_HIP(hipMemcpyAsync(out + c0, s->fout, 4 * (size_t)B, hipMemcpyDeviceToDevice, st));
  }
  return rc;
}

int dlm_invnet_grad(dlm_invnet* s, const int16_t* colors, const float* targets, int32_t count, float* grad,
                    float* loss, void* stream) {
  if (!s || count < 1 || count > s->max_batch || !colors || !targets)
    return set_error(DLM_E_INVAL, "dlm_invnet_grad: count=%d (need 1..max_batch) or null buffer", count);
  hipStream_t st = (hipStream_t)stream;
  int rc = set_stream(s, st);
  if (rc == DLM_OK) rc = inv_forward(s, colors, count, true, false, st);
  if (rc == DLM_OK) rc = inv_backward(s, targets, count, loss, st);
  if (rc == DLM_OK && grad) DLM_HIP(hipMemcpyAsync(grad, s->Gr, 4 * s->total, hipMemcpyDeviceToDevice, st));
  return rc;
}

int dlm_invnet_train(dlm_invnet* s, const int16_t* colors, const float* targets, int32_t count, int32_t batch,
                     int32_t epochs, float lr, float* losses, void* stream) {
  if (!s || count < 0 || batch < 1 || batch > s->max_batch || epochs < 0 || !(lr > 0.f))
    return set_error(DLM_E_INVAL, "dlm_invnet_train: count=%d batch=%d epochs=%d", count, batch, epochs);
  if (count > 0 && (!colors || !targets)) return set_error(DLM_E_INVAL, "dlm_invnet_train: null buffer");
  hipStream_t st = (hipStream_t)stream;
  int rc = set_stream(s, st);
  int step = 0;
  for (int ep = 0; rc == DLM_OK && ep < epochs; ++ep)
    for (int32_t c0 = 0; rc == DLM_OK && c0 < count; c0 += batch) {
      const int B = std::min(batch, count - c0);
      rc = inv_forward(s, colors + (size_t)c0 * s->n, B, true, true, st);
      if (rc == DLM_OK) rc = inv_backward(s, targets + c0, B, losses ? losses + step : nullptr, st);
      if (rc != DLM_OK) break;
      ++s->adam_t;
      const float bc1 = 1.f - powf(0.9f, (float)s->adam_t), bc2 = 1.f - powf(0.999f, (float)s->adam_t);
      hipLaunchKernelGGL(inv_adam_kernel, dim3(blocks((s->total + 3) / 4)), dim3(256), 0, st, s->P, s->M, s->V,
                         s->Gr, s->total, lr, bc1, bc2, s->Pb, s->layout);
      DLM_HIP(hipGetLastError());
      s->t_fresh = false;  // the next training forward reads Lambda itself
      ++step;
    }
  if (rc == DLM_OK && !s->t_fresh) rc = inv_refresh_transposed(s, st);
  return rc;
}

}  // extern "C"
