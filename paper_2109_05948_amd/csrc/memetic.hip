// Device steps of the memetic generation (Algorithm 1) around the tabu search
// and the scorer: gathering selected offspring, standardising the training
// targets, random parent pairing and the (mu + lambda) population update.
#include "dlm_common.h"

namespace dlm {

constexpr uint32_t kDomPair = 0x80000009u;
constexpr uint32_t kDomSelGroup = 0x8000000Au;
constexpr uint32_t kDomReduce = 0x8000000Bu;

__global__ __launch_bounds__(256) void gather_rows_kernel(const int16_t* __restrict__ src, int32_t rows,
                                                          int32_t n, const int32_t* __restrict__ idx,
                                                          int16_t* __restrict__ dst) {
  const int64_t r = blockIdx.x;
  const int32_t s = idx[r];
  const bool ok = s >= 0 && s < rows;
  for (int v = threadIdx.x; v < n; v += 256) dst[r * n + v] = ok ? src[(int64_t)s * n + v] : (int16_t)-1;
}

// mean and standard deviation in FP64, fixed order, one workgroup
// out[i] = f[i], or the largest f below 0x7fffffff (the worst legal score)
// where f[i] = 0x7fffffff (no legal colouring met); *any = 1 if some f[i]
// is legal, else 0 (and out is left as f).  One workgroup.
__global__ __launch_bounds__(256) void wvcp_targets_kernel(const int32_t* __restrict__ f, int32_t count,
                                                           int32_t* __restrict__ out, int32_t* __restrict__ any) {
  __shared__ int32_t red[256];
  int32_t w = INT32_MIN;
  for (int i = threadIdx.x; i < count; i += 256)
    if (f[i] != 0x7fffffff) w = max(w, f[i]);
  red[threadIdx.x] = w;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const int32_t worst = red[0];
  const bool ok = worst != INT32_MIN;
  for (int i = threadIdx.x; i < count; i += 256) out[i] = (ok && f[i] == 0x7fffffff) ? worst : f[i];
  if (threadIdx.x == 0) any[0] = ok ? 1 : 0;
}

__global__ __launch_bounds__(256) void standardize_kernel(const int32_t* __restrict__ f, int32_t count,
                                                          float* __restrict__ out) {
  __shared__ double red[256];
  __shared__ double s_mean, s_inv;
  double a = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) a += (double)f[i];
  red[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += red[i];
    s_mean = t / count;
  }
  __syncthreads();
  const double mean = s_mean;
  double q = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) {
    const double d = (double)f[i] - mean;
    q += d * d;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += red[i];
    const double sd = sqrt(t / count);
    s_inv = sd > 0.0 ? 1.0 / sd : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += 256) out[i] = (float)(((double)f[i] - mean) * s_inv);
}

// pairs[i] = (i, j), j uniform over the other members:
// j = floor(w0 (pop - 1) / 2^32), w0 = Philox(seed; i, gen, 0, pair domain), j += (j >= i)
__global__ __launch_bounds__(256) void random_pairs_kernel(int32_t pop, Key key, uint32_t gen,
                                                           int32_t* __restrict__ pairs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pop) return;
  int j = 0;
  if (pop > 1) {
    j = (int)lemire(philox_w0((uint32_t)i, gen, 0u, kDomPair, key), (uint32_t)(pop - 1));
    j += j >= i;
  }
  pairs[2 * i] = i;
  pairs[2 * i + 1] = j;
}

// keys of the merged pool: parents 0..pop-1, offspring pop..2pop-1
__global__ __launch_bounds__(256) void merge_keys_kernel(const int32_t* __restrict__ fpar,
                                                         const int32_t* __restrict__ foff, int32_t pop,
                                                         uint64_t* __restrict__ keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * pop) return;
  const int32_t f = i < pop ? fpar[i] : foff[i - pop];
  keys[i] = ((uint64_t)(uint32_t)(f ^ 0x80000000) << 32) | (uint32_t)i;  // signed order
}

__global__ __launch_bounds__(256) void merge_rank_kernel(const uint64_t* __restrict__ keys, int32_t total,
                                                         int32_t keep, int32_t* __restrict__ pick) {
  __shared__ uint64_t tile[1024];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t mine = i < total ? keys[i] : ~0ull;
  uint32_t rank = 0;
  for (int base = 0; base < total; base += 1024) {
    const int m = min(1024, total - base);
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += blockDim.x) tile[j] = keys[base + j];
    __syncthreads();
    for (int j = 0; j < m; ++j) rank += tile[j] < mine;
  }
  if (i < total && rank < (uint32_t)keep) pick[rank] = i;
}

__global__ __launch_bounds__(256) void merge_copy_kernel(const int16_t* __restrict__ par,
                                                         const int32_t* __restrict__ fpar,
                                                         const int16_t* __restrict__ off,
                                                         const int32_t* __restrict__ foff, int32_t pop,
                                                         int32_t n, const int32_t* __restrict__ pick,
                                                         int16_t* __restrict__ out, int32_t* __restrict__ fout) {
  const int64_t r = blockIdx.x;
  const int32_t s = pick[r];
  const int16_t* src = s < pop ? par + (int64_t)s * n : off + (int64_t)(s - pop) * n;
  for (int v = threadIdx.x; v < n; v += 256) out[r * n + v] = src[v];
  if (threadIdx.x == 0) fout[r] = s < pop ? fpar[s] : foff[s - pop];
}

// one child per group of K consecutive children: the smallest score (ties
// by index) or a Philox draw
__global__ __launch_bounds__(256) void select_groups_kernel(const float* __restrict__ scores, int32_t groups,
                                                            int32_t K, int32_t mode, Key key, uint32_t gen,
                                                            int32_t* __restrict__ idx) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= groups) return;
  int best = 0;
  if (mode == DLM_SELECT_TOP) {
    const float* s = scores + (size_t)g * K;
    float bs = s[0];
    for (int j = 1; j < K; ++j) {
      const float x = s[j];
      if (x < bs) {
        bs = x;
        best = j;
      }
    }
  } else {
    best = (int)lemire(philox_w0((uint32_t)g, gen, 0u, kDomSelGroup, key), (uint32_t)K);
  }
  idx[g] = g * K + best;
}

// k -> k - 1 colours, one workgroup per row (in place): the class sizes in
// LDS, the smallest class (ties by colour) by a block minimum of
// size << 15 | colour, then its vertices redrawn and the classes above it
// moved down by one.  A row with a colour outside [0, k) becomes all -1.
__global__ __launch_bounds__(256) void reduce_colours_kernel(int16_t* __restrict__ colors, int32_t n, int32_t k,
                                                             Key key, uint32_t step) {
  extern __shared__ __align__(16) uint32_t sizes[];  // k counters
  __shared__ uint32_t wmin[4];
  const int r = blockIdx.x, tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  int16_t* row = colors + (size_t)r * n;
  for (int c = tid; c < k; c += blockDim.x) sizes[c] = 0u;
  __syncthreads();
  int bad = 0;
  for (int v = tid; v < n; v += blockDim.x) {
    const int c = row[v];
    if (c < 0 || c >= k)
      bad = 1;
    else
      atomicAdd(&sizes[c], 1u);
  }
  if (__syncthreads_or(bad)) {
    for (int v = tid; v < n; v += blockDim.x) row[v] = -1;
    return;
  }
  uint32_t best = 0xffffffffu;
  for (int c = tid; c < k; c += blockDim.x) best = min(best, (sizes[c] << 15) | (uint32_t)c);
  best = wave_min_u32(best);
  if (lane == 0) wmin[wid] = best;
  __syncthreads();
  best = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
  const int gone = (int)(best & 0x7fffu);
  for (int v = tid; v < n; v += blockDim.x) {
    const int c = row[v];
    row[v] = (int16_t)(c == gone ? (int)lemire(philox_w0((uint32_t)r, step, (uint32_t)v, kDomReduce, key), (uint32_t)(k - 1))
                                 : c - (c > gone));
  }
}

}  // namespace dlm

using namespace dlm;

extern "C" {

int dlm_gather_rows(const int16_t* src, int32_t rows, int32_t n, const int32_t* idx, int32_t count,
                    int16_t* dst, void* stream) {
  if (rows < 0 || n < 1 || count < 0) return set_error(DLM_E_INVAL, "dlm_gather_rows: rows=%d n=%d count=%d", rows, n, count);
  if (count == 0) return DLM_OK;
  if (!src || !idx || !dst) return set_error(DLM_E_INVAL, "dlm_gather_rows: null buffer");
  hipLaunchKernelGGL(gather_rows_kernel, dim3(count), dim3(256), 0, (hipStream_t)stream, src, rows, n, idx, dst);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_standardize(const int32_t* f, int32_t count, float* out, void* stream) {
  if (count < 1 || !f || !out) return set_error(DLM_E_INVAL, "dlm_standardize: bad arguments");
  hipLaunchKernelGGL(standardize_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, f, count, out);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_wvcp_targets(const int32_t* f, int32_t count, int32_t* out, int32_t* any_legal, void* stream) {
  if (count < 1 || !f || !out || !any_legal) return set_error(DLM_E_INVAL, "dlm_wvcp_targets: bad arguments");
  hipLaunchKernelGGL(wvcp_targets_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, f, count, out, any_legal);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_random_pairs(int32_t pop, uint64_t seed, uint32_t gen, int32_t* pairs, void* stream) {
  if (pop < 0 || (pop > 0 && !pairs)) return set_error(DLM_E_INVAL, "dlm_random_pairs: bad arguments");
  if (pop == 0) return DLM_OK;
  hipLaunchKernelGGL(random_pairs_kernel, dim3((pop + 255) / 256), dim3(256), 0, (hipStream_t)stream, pop,
                     make_key(seed), gen, pairs);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_select_groups(const float* scores, int32_t groups, int32_t K, int32_t mode, uint64_t seed, uint32_t gen,
                      int32_t* idx, void* stream) {
  if (groups < 0 || K < 1 || (mode != DLM_SELECT_TOP && mode != DLM_SELECT_RANDOM) ||
      (int64_t)groups * K > 0x7fffffffll)
    return set_error(DLM_E_INVAL, "dlm_select_groups: groups=%d K=%d mode=%d", groups, K, mode);
  if (groups == 0) return DLM_OK;
  if (!idx || (mode == DLM_SELECT_TOP && !scores)) return set_error(DLM_E_INVAL, "dlm_select_groups: null buffer");
  hipLaunchKernelGGL(select_groups_kernel, dim3((groups + 255) / 256), dim3(256), 0, (hipStream_t)stream, scores,
                     groups, K, mode, make_key(seed), gen, idx);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_reduce_colours(int16_t* colors, int32_t pop, int32_t n, int32_t k, uint64_t seed, uint32_t step,
                       void* stream) {
  if (pop < 0 || n < 1 || n > 32767 || k < 2 || k > 32767)
    return set_error(DLM_E_INVAL, "dlm_reduce_colours: pop=%d n=%d k=%d", pop, n, k);
  if (pop == 0) return DLM_OK;
  if (!colors) return set_error(DLM_E_INVAL, "dlm_reduce_colours: null buffer");
  const size_t lds = (size_t)k * 4u;
  DLM_HIP(hipFuncSetAttribute((const void*)reduce_colours_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  hipLaunchKernelGGL(reduce_colours_kernel, dim3(pop), dim3(256), lds, (hipStream_t)stream, colors, n, k,
                     make_key(seed), step);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_pop_update(const int16_t* parents, const int32_t* f_parents, const int16_t* offspring,
                   const int32_t* f_offspring, int32_t pop, int32_t n, int16_t* out, int32_t* f_out,
                   void* workspace, void* stream) {
  if (pop < 0 || n < 1) return set_error(DLM_E_INVAL, "dlm_pop_update: pop=%d n=%d", pop, n);
  if (pop == 0) return DLM_OK;
  if (!parents || !f_parents || !offspring || !f_offspring || !out || !f_out || !workspace)
    return set_error(DLM_E_INVAL, "dlm_pop_update: null buffer");
  hipStream_t s = (hipStream_t)stream;
  uint64_t* keys = (uint64_t*)workspace;
  int32_t* pick = (int32_t*)(keys + 2 * (int64_t)pop);
  const unsigned g2 = (unsigned)((2 * pop + 255) / 256);
  hipLaunchKernelGGL(merge_keys_kernel, dim3(g2), dim3(256), 0, s, f_parents, f_offspring, pop, keys);
  DLM_HIP(hipGetLastError());
  hipLaunchKernelGGL(merge_rank_kernel, dim3(g2), dim3(256), 0, s, keys, 2 * pop, pop, pick);
  DLM_HIP(hipGetLastError());
  hipLaunchKernelGGL(merge_copy_kernel, dim3(pop), dim3(256), 0, s, parents, f_parents, offspring, f_offspring,
                     pop, n, pick, out, f_out);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

}  // extern "C"
