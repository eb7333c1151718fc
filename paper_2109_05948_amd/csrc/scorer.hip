// Offspring scorer: the colour-permutation-invariant regressor of Section 2.3
// in per-class MLP form, with BF16 MFMA inference and training (FP32
// accumulation, FP32 master weights, Adam).
//
//   a1_i = b1 + V_i W1   (V_i = indicator of colour class i; computed as the
//                          sum of the W1 rows of the class's vertices)
//   h1_i = LReLU(a1_i)   a2_i = b2 + h1_i W2   h2_i = LReLU(a2_i)
//   z = sum_i h2_i       a3 = b3 + z W3        h3 = LReLU(a3)
//   y = h3 . w4 + b4                 LReLU(x) = max(0.2 x, x)
//
// H1 = 256, H2 = 128, H3 = 64.  Layer 2 and its two backward products run
// on v_mfma_f32_32x32x16_bf16; layer 1 is a gather of FP32 W1 rows (a dense
// one-hot product would cost n/k times more, and FP32 keeps the LeakyReLU
// branch of a1 exact to FP32 rounding); the head is plain FP32.
//
// MFMA 32x32x16 (bf16) operand layout, lane l of a wave:
//   A (32 x 16): A[l % 32][8 (l / 32) + j], j = 0..7
//   B (16 x 32): B[8 (l / 32) + j][l % 32]
//   D (32 x 32): D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32], r = 0..15
#include <math.h>
#include <string.h>

#include <vector>

#include "dlm_common.h"

namespace dlm {

constexpr int H1 = 256, H2 = 128, H3 = 64;
constexpr float kSlope = 0.2f;
constexpr int kRowPadH1 = H1 + 8;  // LDS row stride (bf16) of h1, breaks bank aliasing
constexpr int kRowPadH2 = H2 + 8;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float lrelu(float x) { return x > 0.f ? x : kSlope * x; }
__device__ __forceinline__ float dlrelu(float h) { return h > 0.f ? 1.f : kSlope; }

// gfx950's 32x32x16 BF16 MFMA: lane l supplies row l % 32 of A (of B^T)
// with the eight K values 8 (l / 32) .. 8 (l / 32) + 7; the 32x32 FP32
// result is spread as for every 32x32 MFMA (16 values per lane)
__device__ __forceinline__ f16v mfma(bf8 a, bf8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf8 ld_b8(const uint16_t* p) {  // 16-byte aligned
  return *reinterpret_cast<const bf8*>(p);
}

// Offsets (in floats) of the packed FP32 parameter vector.
struct ParamLayout {
  int64_t W1, b1, W2, b2, W3, b3, w4, b4, total;
};
inline ParamLayout param_layout(int n) {
  ParamLayout p;
  int64_t o = 0;
  p.W1 = o; o += (int64_t)n * H1;
  p.b1 = o; o += H1;
  p.W2 = o; o += (int64_t)H1 * H2;
  p.b2 = o; o += H2;
  p.W3 = o; o += (int64_t)H2 * H3;
  p.b3 = o; o += H3;
  p.w4 = o; o += H3;
  p.b4 = o; o += 1;
  p.total = o;
  return p;
}

struct ScorerDev {
  const float* P;            // FP32 master parameters
  const uint16_t* W2b;       // bf16 [H1][H2]
  const uint16_t* W2t;       // bf16 [H2][H1]
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, ow4, ob4;
  int32_t n, k, kpad;
};

// Per-colouring activations kept for the backward pass.
struct TrainBufs {
  uint16_t* h1t;  // bf16 [B][H1][kpad]  (K-contiguous for the weight-gradient product)
  uint16_t* h2;   // bf16 [B][kpad][H2]
  float* z;       // [B][H2]
  float* a3;      // [B][H3]
  float* y;       // [B]
  uint16_t* da2t; // bf16 [B][H2][kpad]
  float* da1;     // [B][kpad][H1]
  float* da3;     // [B][H3]
  float* dy;      // [B]
  float* part;    // [nchunk][H1][H2] partial sums of dW2
  float* p1;      // [B][H1] per-colouring sum over classes of da1
  float* p2;      // [B][H2] per-colouring sum over classes of da2
};

// ---------------------------------------------------------------------------
// Forward, one workgroup (4 waves) per colouring.
//   layer 1: wave w takes classes i = w, w+4, ...; it lists the class's
//            vertices in ascending order (ballot) and sums their W1 rows, lane l
//            owning features 4l..4l+3 (deterministic order)
//   layer 2: wave w computes the output columns 32w..32w+31 for every row tile
//   pool + head: column sums over the valid rows, then the FP32 head
template <bool TRAIN>
__global__ __launch_bounds__(256) void scorer_fwd_kernel(ScorerDev s, const int16_t* __restrict__ colors,
                                                         int32_t count, float* __restrict__ out,
                                                         TrainBufs tb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int n = s.n, k = s.k, kpad = s.kpad;
  const int64_t b = blockIdx.x;
  uint16_t* h1 = reinterpret_cast<uint16_t*>(smem);                       // [kpad][kRowPadH1]
  int16_t* col = reinterpret_cast<int16_t*>(smem + (size_t)kpad * kRowPadH1 * 2);
  uint16_t* lists = reinterpret_cast<uint16_t*>(col + ((n + 7) & ~7));   // [4][n]
  float* zs = reinterpret_cast<float*>(lists + 4 * ((n + 7) & ~7));       // [H2]
  float* hs = zs + H2;                                                    // [H3]

  const int16_t* cb = colors + b * n;
  for (int v = tid; v < n; v += 256) col[v] = cb[v];
  // rows k..kpad-1 are zero
  for (int i = k + wid; i < kpad; i += 4)
    for (int f = lane; f < H1; f += 64) h1[i * kRowPadH1 + f] = 0;
  __syncthreads();

  // ---- layer 1 (gather) + LReLU -> h1 (bf16, LDS)
  uint16_t* mylist = lists + wid * ((n + 7) & ~7);
  const float* b1 = s.P + s.ob1;
  for (int i = wid; i < k; i += 4) {
    int cnt = 0;
    for (int v0 = 0; v0 < n; v0 += 64) {
      const int v = v0 + lane;
      const bool in = v < n && col[v] == i;
      const uint64_t m = __ballot(in);
      if (in) mylist[cnt + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)v;
      cnt += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float a0 = b1[4 * lane], a1v = b1[4 * lane + 1], a2v = b1[4 * lane + 2], a3v = b1[4 * lane + 3];
    const float* W1 = s.P + s.oW1 + 4 * lane;
    for (int q = 0; q < cnt; ++q) {
      const float4 wrow = *reinterpret_cast<const float4*>(W1 + (size_t)mylist[q] * H1);
      a0 += wrow.x;
      a1v += wrow.y;
      a2v += wrow.z;
      a3v += wrow.w;
    }
    uint16_t* row = h1 + i * kRowPadH1 + 4 * lane;
    row[0] = f2bf(lrelu(a0));
    row[1] = f2bf(lrelu(a1v));
    row[2] = f2bf(lrelu(a2v));
    row[3] = f2bf(lrelu(a3v));
  }
  __syncthreads();
  if (TRAIN) {  // h1 transposed for the weight-gradient product: h1t[b][f][i]
    uint16_t* dst = tb.h1t + b * (int64_t)H1 * kpad;
    for (int e = tid; e < H1 * kpad; e += 256) {
      const int f = e / kpad, i = e - (e / kpad) * kpad;
      dst[e] = h1[i * kRowPadH1 + f];
    }
  }

  // ---- layer 2 on MFMA: wave w -> columns n0 = 32 w
  const int n0 = 32 * wid;
  const float bias2 = s.P[s.ob2 + n0 + (lane & 31)];
  float zc = 0.f;  // this lane's share of z[n0 + lane % 32]
  for (int m0 = 0; m0 < kpad; m0 += 32) {
    f16v acc = {};
    const uint16_t* arow = h1 + (m0 + (lane & 31)) * kRowPadH1 + 8 * (lane >> 5);
    const uint16_t* brow = s.W2t + (size_t)(n0 + (lane & 31)) * H1 + 8 * (lane >> 5);
#pragma unroll 4
    for (int k0 = 0; k0 < H1; k0 += 16) acc = mfma(ld_b8(arow + k0), ld_b8(brow + k0), acc);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const float h = lrelu(acc[r] + bias2);
      if (i < k) zc += h;
      if (TRAIN) tb.h2[(b * kpad + i) * H2 + n0 + (lane & 31)] = i < k ? f2bf(h) : (uint16_t)0;
    }
  }
  zc += __shfl_xor(zc, 32);
  if (lane < 32) zs[n0 + lane] = zc;
  __syncthreads();

  // ---- head
  if (tid < H3) {
    const float* W3 = s.P + s.oW3;
    float a = s.P[s.ob3 + tid];
    for (int q = 0; q < H2; ++q) a += zs[q] * W3[q * H3 + tid];
    hs[tid] = a;
    if (TRAIN) tb.a3[b * H3 + tid] = a;
  }
  __syncthreads();
  if (wid == 0) {
    float p = lrelu(hs[lane]) * s.P[s.ow4 + lane];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o);
    if (lane == 0) {
      const float y = p + s.P[s.ob4];
      out[b] = y;
      if (TRAIN) tb.y[b] = y;
    }
  }
  if (TRAIN)
    for (int q = tid; q < H2; q += 256) tb.z[b * H2 + q] = zs[q];
}

// ---------------------------------------------------------------------------
// Backward per colouring: head, dz, da2 = dz * LReLU'(a2), dh1 = da2 W2^T on
// MFMA, da1 = dh1 * LReLU'(a1).
__global__ __launch_bounds__(256) void scorer_bwd_kernel(ScorerDev s, const float* __restrict__ targets,
                                                         int32_t count, float scale, TrainBufs tb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int k = s.k, kpad = s.kpad;
  const int64_t b = blockIdx.x;
  uint16_t* da2 = reinterpret_cast<uint16_t*>(smem);  // [kpad][kRowPadH2]
  float* dz = reinterpret_cast<float*>(smem + (size_t)kpad * kRowPadH2 * 2);
  float* da3s = dz + H2;
  const float dy = scale * (tb.y[b] - targets[b]);
  if (tid < H3) {
    const float a = tb.a3[b * H3 + tid];
    const float d = dy * s.P[s.ow4 + tid] * (a > 0.f ? 1.f : kSlope);
    da3s[tid] = d;
    tb.da3[b * H3 + tid] = d;
  }
  if (tid == 0) tb.dy[b] = dy;
  __syncthreads();
  if (tid < H2) {
    const float* W3 = s.P + s.oW3;
    float a = 0.f;
    for (int j = 0; j < H3; ++j) a += W3[tid * H3 + j] * da3s[j];
    dz[tid] = a;
  }
  __syncthreads();
  // da2 rows (bf16, LDS), its transposed copy for the weight gradient, and
  // its sum over the classes (bias gradient)
  uint16_t* dt = tb.da2t + b * (int64_t)H2 * kpad;
  if (tid < H2) {
    const int q = tid;
    float sum = 0.f;
    for (int i = 0; i < kpad; ++i) {
      const float h = bf2f(tb.h2[(b * kpad + i) * H2 + q]);
      const uint16_t d = i < k ? f2bf(dz[q] * dlrelu(h)) : (uint16_t)0;
      da2[i * kRowPadH2 + q] = d;
      dt[q * kpad + i] = d;
      sum += bf2f(d);
    }
    tb.p2[b * H2 + q] = sum;
  }
  __syncthreads();
  // dh1 = da2 (kpad x H2) . W2^T (H2 x H1): wave w -> column tiles w and w + 4
  const uint16_t* h1t = tb.h1t + b * (int64_t)H1 * kpad;
  float colsum = 0.f;
  for (int nt = wid; nt < H1 / 32; nt += 4) {
    const int f0 = 32 * nt;
    for (int m0 = 0; m0 < kpad; m0 += 32) {
      f16v acc = {};
      const uint16_t* arow = da2 + (m0 + (lane & 31)) * kRowPadH2 + 8 * (lane >> 5);
      const uint16_t* brow = s.W2b + (size_t)(f0 + (lane & 31)) * H2 + 8 * (lane >> 5);
#pragma unroll 4
      for (int k0 = 0; k0 < H2; k0 += 16) acc = mfma(ld_b8(arow + k0), ld_b8(brow + k0), acc);
      const int f = f0 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const float h = bf2f(h1t[(int64_t)f * kpad + i]);
        const float d = i < k ? acc[r] * dlrelu(h) : 0.f;
        tb.da1[(b * kpad + i) * H1 + f] = d;
        colsum += d;
      }
    }
    colsum += __shfl_xor(colsum, 32);
    if (lane < 32) tb.p1[b * H1 + f0 + lane] = colsum;
    colsum = 0.f;
  }
}

// dW2 partial sums: chunk c of CB colourings; out[f][q] = sum h1[b][i][f] da2[b][i][q]
constexpr int kChunkB = 4;
__global__ __launch_bounds__(256) void scorer_dw2_kernel(int32_t count, int32_t kpad, TrainBufs tb) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int c = blockIdx.x;
  const int q0 = 32 * wid;  // wave w: columns q0..q0+31, all 8 row tiles f
  f16v acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f16v{};
  const int b_end = min(count, (c + 1) * kChunkB);
  for (int b = c * kChunkB; b < b_end; ++b) {
    const uint16_t* A = tb.h1t + (int64_t)b * H1 * kpad;
    const uint16_t* B = tb.da2t + (int64_t)b * H2 * kpad + (int64_t)(q0 + (lane & 31)) * kpad + 8 * (lane >> 5);
    for (int k0 = 0; k0 < kpad; k0 += 16) {
      const bf8 bf = ld_b8(B + k0);
#pragma unroll
      for (int t = 0; t < 8; ++t)
        acc[t] = mfma(ld_b8(A + (int64_t)(32 * t + (lane & 31)) * kpad + 8 * (lane >> 5) + k0), bf, acc[t]);
    }
  }
  float* out = tb.part + (int64_t)c * H1 * H2;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      out[(int64_t)f * H2 + q0 + (lane & 31)] = acc[t][r];
    }
}

// Small gradients and the dW2 reduction (fixed summation order).
__global__ __launch_bounds__(256) void scorer_grad_small_kernel(ScorerDev s, int32_t count,
                                                                int32_t nchunk, TrainBufs tb,
                                                                float* __restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t o = e;
  if (o < H1 * H2) {  // dW2
    float a = 0.f;
    for (int c = 0; c < nchunk; ++c) a += tb.part[(int64_t)c * H1 * H2 + o];
    g[s.oW2 + o] = a;
    return;
  }
  o -= H1 * H2;
  if (o < H1) {  // db1
    float a = 0.f;
    for (int b = 0; b < count; ++b) a += tb.p1[(int64_t)b * H1 + o];
    g[s.ob1 + o] = a;
    return;
  }
  o -= H1;
  if (o < H2) {  // db2
    float a = 0.f;
    for (int b = 0; b < count; ++b) a += tb.p2[(int64_t)b * H2 + o];
    g[s.ob2 + o] = a;
    return;
  }
  o -= H2;
  if (o < H2 * H3) {  // dW3
    const int q = (int)(o / H3), j = (int)(o % H3);
    float a = 0.f;
    for (int b = 0; b < count; ++b) a += tb.z[(int64_t)b * H2 + q] * tb.da3[(int64_t)b * H3 + j];
    g[s.oW3 + o] = a;
    return;
  }
  o -= H2 * H3;
  if (o < H3) {  // db3 and dw4
    float a = 0.f, w = 0.f;
    for (int b = 0; b < count; ++b) {
      a += tb.da3[(int64_t)b * H3 + o];
      w += tb.dy[b] * lrelu(tb.a3[(int64_t)b * H3 + o]);
    }
    g[s.ob3 + o] = a;
    g[s.ow4 + o] = w;
    return;
  }
  o -= H3;
  if (o == 0) {  // db4
    float a = 0.f;
    for (int b = 0; b < count; ++b) a += tb.dy[b];
    g[s.ob4] = a;
  }
}

// dW1[v][f] = sum_b da1[b][col_b v][f]  (fixed order over b)
__global__ __launch_bounds__(256) void scorer_dw1_kernel(ScorerDev s, const int16_t* __restrict__ colors,
                                                         int32_t count, TrainBufs tb, float* __restrict__ g) {
  const int v = blockIdx.x, f = threadIdx.x;
  float a = 0.f;
  for (int b = 0; b < count; ++b) {
    const int c = colors[(int64_t)b * s.n + v];
    a += tb.da1[((int64_t)b * s.kpad + c) * H1 + f];
  }
  g[s.oW1 + (int64_t)v * H1 + f] = a;
}

__global__ __launch_bounds__(256) void scorer_loss_kernel(const float* __restrict__ y,
                                                          const float* __restrict__ t, int32_t count,
                                                          float* __restrict__ loss) {
  __shared__ float red[4];
  float a = 0.f;
  for (int b = threadIdx.x; b < count; b += 256) {
    const float r = y[b] - t[b];
    a += r * r;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (red[0] + red[1] + red[2] + red[3]) / (float)count;
}

// Adam (Kingma and Ba, with bias correction) on the FP32 master weights.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ P, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g,
                                                   int64_t total, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 working copies of W2 for the MFMA products: W2b [H1][H2], W2t [H2][H1]
__global__ __launch_bounds__(256) void scorer_cast_kernel(const float* __restrict__ P, int64_t oW2,
                                                          uint16_t* __restrict__ W2b,
                                                          uint16_t* __restrict__ W2t) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < H1 * H2) {
    const uint16_t x = f2bf(P[oW2 + j]);
    W2b[j] = x;
    W2t[(j % H2) * H1 + j / H2] = x;
  }
}

}  // namespace dlm

using namespace dlm;

struct dlm_scorer {
  int32_t n = 0, k = 0, kpad = 0, max_batch = 0;
  int64_t step = 0;
  ParamLayout L{};
  float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t *W2b = nullptr, *W2t = nullptr;
  TrainBufs tb{};
  void* ws = nullptr;
  ScorerDev dev() const {
    return ScorerDev{P, W2b, W2t, L.W1, L.b1, L.W2, L.b2, L.W3, L.b3, L.w4, L.b4, n, k, kpad};
  }
};

namespace {
size_t fwd_lds(int n, int kpad) {
  const size_t np = (size_t)((n + 7) & ~7);
  return (size_t)kpad * kRowPadH1 * 2 + np * 2 + 4 * np * 2 + (H2 + H3) * 4;
}
size_t bwd_lds(int kpad) { return (size_t)kpad * kRowPadH2 * 2 + (H2 + H3) * 4; }

int cast_weights(dlm_scorer* s, hipStream_t st) {
  hipLaunchKernelGGL(scorer_cast_kernel, dim3((H1 * H2 + 255) / 256), dim3(256), 0, st, s->P, s->L.W2, s->W2b,
                     s->W2t);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

// forward (train) + backward + gradient of the mean loss over `count` examples into s->g
int grad_pass(dlm_scorer* s, const int16_t* colors, const float* targets, int32_t count,
              float* loss, hipStream_t st) {
  const ScorerDev d = s->dev();
  const size_t lf = fwd_lds(s->n, s->kpad), lb = bwd_lds(s->kpad);
  hipLaunchKernelGGL(scorer_fwd_kernel<true>, dim3(count), dim3(256), lf, st, d, colors, count, s->tb.y, s->tb);
  DLM_HIP(hipGetLastError());
  if (loss) {
    hipLaunchKernelGGL(scorer_loss_kernel, dim3(1), dim3(256), 0, st, s->tb.y, targets, count, loss);
    DLM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(scorer_bwd_kernel, dim3(count), dim3(256), lb, st, d, targets, count, 2.f / (float)count,
                     s->tb);
  DLM_HIP(hipGetLastError());
  const int nchunk = (count + kChunkB - 1) / kChunkB;
  hipLaunchKernelGGL(scorer_dw2_kernel, dim3(nchunk), dim3(256), 0, st, count, s->kpad, s->tb);
  DLM_HIP(hipGetLastError());
  const int64_t small = (int64_t)H1 * H2 + H1 + H2 + H2 * H3 + H3 + 1;
  hipLaunchKernelGGL(scorer_grad_small_kernel, dim3((unsigned)((small + 255) / 256)), dim3(256), 0, st, d, count,
                     nchunk, s->tb, s->g);
  DLM_HIP(hipGetLastError());
  hipLaunchKernelGGL(scorer_dw1_kernel, dim3(s->n), dim3(H1), 0, st, d, colors, count, s->tb, s->g);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int check_colors_arg(const dlm_scorer* s, const void* p, int32_t count, const char* fn) {
  if (!s) return set_error(DLM_E_INVAL, "%s: scorer is NULL", fn);
  if (count < 0) return set_error(DLM_E_INVAL, "%s: count < 0", fn);
  if (count > 0 && !p) return set_error(DLM_E_INVAL, "%s: null buffer", fn);
  return DLM_OK;
}
}  // namespace

extern "C" {

int dlm_scorer_create(int32_t n, int32_t k, int32_t h1, int32_t h2, int32_t h3, int32_t max_batch,
                      const float* params_host, dlm_scorer** out) {
  if (!out) return set_error(DLM_E_INVAL, "dlm_scorer_create: out is NULL");
  *out = nullptr;
  if (h1 != H1 || h2 != H2 || h3 != H3)
    return set_error(DLM_E_UNSUPPORTED, "dlm_scorer_create: widths %d,%d,%d (only 256,128,64 are built)", h1,
                     h2, h3);
  if (n < 1 || n > 32767 || k < 1 || k > 256)
    return set_error(DLM_E_INVAL, "dlm_scorer_create: n=%d k=%d (need 1<=n<=32767, 1<=k<=256)", n, k);
  if (max_batch < 0 || max_batch > (1 << 20))
    return set_error(DLM_E_INVAL, "dlm_scorer_create: max_batch=%d", max_batch);
  if (!params_host) return set_error(DLM_E_INVAL, "dlm_scorer_create: params is NULL");
  dlm_scorer* s = new dlm_scorer();
  s->n = n;
  s->k = k;
  s->kpad = (k + 31) & ~31;
  s->max_batch = max_batch;
  s->L = param_layout(n);
  const int64_t P = s->L.total;
  const int64_t B = max_batch, kp = s->kpad;
  const int64_t nchunk = (B + kChunkB - 1) / kChunkB;
  // one allocation for everything the scorer owns
  const int64_t bytes_f =
      4 * (4 * P + B * H2 + B * H3 + B + B * kp * H1 + B * H3 + B + nchunk * H1 * H2 + B * (H1 + H2));
  const int64_t bytes_h = 2 * (2 * H1 * H2 + B * H1 * kp + B * kp * H2 + B * H2 * kp);
  const int64_t bytes = bytes_f + bytes_h + 256;
  hipError_t e = hipMalloc(&s->ws, (size_t)bytes);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMalloc (scorer)");
  }
  float* f = (float*)s->ws;
  s->P = f; f += P;
  s->m = f; f += P;
  s->v = f; f += P;
  s->g = f; f += P;
  s->tb.z = f; f += B * H2;
  s->tb.a3 = f; f += B * H3;
  s->tb.y = f; f += B;
  s->tb.da1 = f; f += B * kp * H1;
  s->tb.da3 = f; f += B * H3;
  s->tb.dy = f; f += B;
  s->tb.part = f; f += nchunk * H1 * H2;
  s->tb.p1 = f; f += B * H1;
  s->tb.p2 = f; f += B * H2;
  // the BF16 region starts on a 16-byte boundary: its rows are read 8 values at a time
  uint16_t* h = (uint16_t*)(((uintptr_t)f + 15) & ~(uintptr_t)15);
  s->W2b = h; h += H1 * H2;
  s->W2t = h; h += H1 * H2;
  s->tb.h1t = h; h += B * H1 * kp;
  s->tb.h2 = h; h += B * kp * H2;
  s->tb.da2t = h; h += B * H2 * kp;
  if ((e = hipMemcpy(s->P, params_host, sizeof(float) * P, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(s->m, 0, sizeof(float) * 2 * P)) != hipSuccess) {
    (void)hipFree(s->ws);
    delete s;
    return hip_fail(e, "scorer upload");
  }
  int rc = cast_weights(s, nullptr);
  if (rc == DLM_OK && (e = hipDeviceSynchronize()) != hipSuccess) rc = hip_fail(e, "scorer init");
  if (rc != DLM_OK) {
    (void)hipFree(s->ws);
    delete s;
    return rc;
  }
  *out = s;
  return DLM_OK;
}

int dlm_scorer_destroy(dlm_scorer* s) {
  if (!s) return DLM_OK;
  (void)hipFree(s->ws);
  delete s;
  return DLM_OK;
}

int dlm_scorer_num_params(const dlm_scorer* s, int64_t* count) {
  if (!s || !count) return set_error(DLM_E_INVAL, "dlm_scorer_num_params: null argument");
  *count = s->L.total;
  return DLM_OK;
}

int dlm_scorer_get_params(const dlm_scorer* s, float* params_dev, void* stream) {
  if (!s || !params_dev) return set_error(DLM_E_INVAL, "dlm_scorer_get_params: null argument");
  DLM_HIP(hipMemcpyAsync(params_dev, s->P, sizeof(float) * s->L.total, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return DLM_OK;
}

int dlm_score_offspring(const dlm_scorer* s, const int16_t* colors, int32_t count, float* scores,
                        void* stream) {
  int rc = check_colors_arg(s, colors, count, "dlm_score_offspring");
  if (rc != DLM_OK) return rc;
  if (count == 0) return DLM_OK;
  if (!scores) return set_error(DLM_E_INVAL, "dlm_score_offspring: scores is NULL");
  const size_t lds = fwd_lds(s->n, s->kpad);
  if ((int64_t)lds > device_lds_limit())
    return set_error(DLM_E_UNSUPPORTED, "dlm_score_offspring: %zu bytes of LDS needed", lds);
  DLM_HIP(hipFuncSetAttribute((const void*)scorer_fwd_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  hipLaunchKernelGGL(scorer_fwd_kernel<false>, dim3(count), dim3(256), lds, (hipStream_t)stream, s->dev(), colors,
                     count, scores, s->tb);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_scorer_grad(dlm_scorer* s, const int16_t* colors, const float* targets, int32_t count,
                    float* grad_dev, float* loss_dev, void* stream) {
  int rc = check_colors_arg(s, colors, count, "dlm_scorer_grad");
  if (rc != DLM_OK) return rc;
  if (count < 1 || count > s->max_batch)
    return set_error(DLM_E_INVAL, "dlm_scorer_grad: count=%d outside [1, max_batch=%d]", count, s->max_batch);
  if (!targets) return set_error(DLM_E_INVAL, "dlm_scorer_grad: targets is NULL");
  hipStream_t st = (hipStream_t)stream;
  DLM_HIP(hipFuncSetAttribute((const void*)scorer_fwd_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)fwd_lds(s->n, s->kpad)));
  if ((rc = grad_pass(s, colors, targets, count, loss_dev, st)) != DLM_OK) return rc;
  if (grad_dev)
    DLM_HIP(hipMemcpyAsync(grad_dev, s->g, sizeof(float) * s->L.total, hipMemcpyDeviceToDevice, st));
  return DLM_OK;
}

int dlm_scorer_train(dlm_scorer* s, const int16_t* colors, const float* targets, int32_t count,
                     int32_t batch, int32_t epochs, float lr, float* loss_dev, void* stream) {
  int rc = check_colors_arg(s, colors, count, "dlm_scorer_train");
  if (rc != DLM_OK) return rc;
  if (batch < 1 || batch > s->max_batch)
    return set_error(DLM_E_INVAL, "dlm_scorer_train: batch=%d outside [1, max_batch=%d]", batch, s->max_batch);
  if (epochs < 0 || !(lr > 0.f)) return set_error(DLM_E_INVAL, "dlm_scorer_train: epochs=%d lr=%g", epochs, lr);
  if (count == 0 || epochs == 0) return DLM_OK;
  if (!targets) return set_error(DLM_E_INVAL, "dlm_scorer_train: targets is NULL");
  hipStream_t st = (hipStream_t)stream;
  DLM_HIP(hipFuncSetAttribute((const void*)scorer_fwd_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)fwd_lds(s->n, s->kpad)));
  const double beta1 = 0.9, beta2 = 0.999;
  int64_t li = 0;
  for (int ep = 0; ep < epochs; ++ep)
    for (int32_t s0 = 0; s0 < count; s0 += batch) {
      const int32_t cnt = count - s0 < batch ? count - s0 : batch;
      rc = grad_pass(s, colors + (int64_t)s0 * s->n, targets + s0, cnt, loss_dev ? loss_dev + li : nullptr, st);
      if (rc != DLM_OK) return rc;
      ++li;
      s->step += 1;
      const float bc1 = (float)(1.0 - pow(beta1, (double)s->step));
      const float bc2 = (float)(1.0 - pow(beta2, (double)s->step));
      hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((s->L.total + 255) / 256)), dim3(256), 0, st, s->P, s->m,
                         s->v, s->g, s->L.total, lr, (float)beta1, (float)beta2, 1e-8f, bc1, bc2);
      DLM_HIP(hipGetLastError());
      if ((rc = cast_weights(s, st)) != DLM_OK) return rc;
    }
  return DLM_OK;
}

}  // extern "C"
