// Greedy partition crossover (GPX; Sections 1 and 2.6 of the paper: the
// offspring inherits alternately the largest remaining colour class of each
// parent, the individual itself being the first parent) and the offspring
// selection of eq. (select_cross), population-wide.
#include "dlm_common.h"

namespace dlm {

// One workgroup per child.  Step l takes parent A when l is even, B when odd;
// the class with the most unassigned vertices wins, ties going to the
// smallest Philox word of (child, l, lowest unassigned vertex of the class),
// then to that vertex.  Its unassigned vertices get colour l.  After k steps
// the vertices left get a uniform colour (Philox (child, 0, v, fill domain)).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void gpx_kernel(int32_t n, int32_t k, int32_t pop,
                                                    const int16_t* __restrict__ parents,
                                                    const int32_t* __restrict__ pairs,
                                                    int32_t per_pair, uint32_t child_base, Key key,
                                                    int16_t* __restrict__ children) {
  constexpr int NW = BLOCK / kWave;
  extern __shared__ __align__(16) unsigned char smem[];
  int16_t* pa = reinterpret_cast<int16_t*>(smem);
  int16_t* pb = pa + n;
  int16_t* out = pb + n;  // -1 = unassigned
  uint32_t* size = reinterpret_cast<uint32_t*>(smem + align16(6u * n));
  uint32_t* minv = size + k;
  __shared__ uint32_t s_max[NW], s_cnt[NW];
  __shared__ uint64_t s_key[NW];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int64_t child = blockIdx.x;
  const int64_t p = child / per_pair;
  const uint32_t cid = child_base + (uint32_t)child;
  const int32_t ia = pairs[2 * p], ib = pairs[2 * p + 1];
  if (ia < 0 || ia >= pop || ib < 0 || ib >= pop) {  // bad pair: child marked invalid
    for (int v = tid; v < n; v += BLOCK) children[child * n + v] = -1;
    return;
  }
  const int16_t* A = parents + (int64_t)ia * n;
  const int16_t* B = parents + (int64_t)ib * n;
  int bad = 0;
  for (int v = tid; v < n; v += BLOCK) {
    const int16_t ca = A[v], cb = B[v];
    bad |= (ca < 0) | (ca >= k) | (cb < 0) | (cb >= k);
    pa[v] = ca;
    pb[v] = cb;
    out[v] = -1;
  }
  if (__syncthreads_or(bad)) {  // a parent colour outside [0, k): child marked invalid
    for (int v = tid; v < n; v += BLOCK) children[child * n + v] = -1;
    return;
  }
  for (int l = 0; l < k; ++l) {
    const int16_t* P = (l & 1) ? pb : pa;
    for (int c = tid; c < k; c += BLOCK) {
      size[c] = 0;
      minv[c] = (uint32_t)n;
    }
    __syncthreads();
    for (int v = tid; v < n; v += BLOCK)
      if (out[v] < 0) {
        atomicAdd(&size[P[v]], 1u);
        atomicMin(&minv[P[v]], (uint32_t)v);
      }
    __syncthreads();
    // largest class size and how many classes have it
    uint32_t m = 0, cnt = 0;
    for (int c = tid; c < k; c += BLOCK) {
      const uint32_t s = size[c];
      if (s > m) {
        m = s;
        cnt = 1;
      } else if (s == m) {
        ++cnt;
      }
    }
    const uint32_t wm = wave_max_u32(m);
    const uint32_t wc = wave_sum_u32(m == wm ? cnt : 0u);
    if (lane == 0) {
      s_max[wid] = wm;
      s_cnt[wid] = wc;
    }
    __syncthreads();
    uint32_t gm = 0, gc = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) gm = max(gm, s_max[w]);
#pragma unroll
    for (int w = 0; w < NW; ++w) gc += s_max[w] == gm ? s_cnt[w] : 0u;
    if (gm == 0) break;  // every vertex assigned (uniform)
    // winner: the tied class with the smallest (hash, lowest unassigned vertex)
    uint64_t best = ~0ull;
    for (int c = tid; c < k; c += BLOCK)
      if (size[c] == gm) {
        const uint32_t mv = minv[c];
        const uint32_t h = gc > 1 ? philox_w0(cid, (uint32_t)l, mv, kDomGpxTie, key) : 0u;
        best = umin64(best, ((uint64_t)h << 32) | mv);
      }
    best = wave_min_u64(best);
    if (lane == 0) s_key[wid] = best;
    __syncthreads();
    uint64_t gb = s_key[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) gb = umin64(gb, s_key[w]);
    const int cw = P[(uint32_t)gb];
    for (int v = tid; v < n; v += BLOCK)
      if (out[v] < 0 && P[v] == cw) out[v] = (int16_t)l;
    __syncthreads();
  }
  int16_t* dst = children + child * n;
  for (int v = tid; v < n; v += BLOCK) {
    int16_t c = out[v];
    if (c < 0) c = (int16_t)lemire(philox_w0(cid, 0u, (uint32_t)v, kDomGpxFill, key), (uint32_t)k);
    dst[v] = c;
  }
}

// ---------------------------------------------------------------------------
// Selection: rank of element i = #{j : key_j < key_i or (key_j == key_i and
// j < i)}; the first `keep` ranks are written in rank order.
__device__ __forceinline__ uint32_t float_order_key(float x) {
  const uint32_t u = __float_as_uint(x);
  if (x != x) return 0xffffffffu;  // NaN last
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(256) void select_keys_kernel(const float* __restrict__ scores,
                                                          int32_t count, int32_t mode, Key key,
                                                          uint32_t gen, uint64_t* __restrict__ keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t k32 = mode == 0 ? float_order_key(scores[i])
                                 : philox_w0((uint32_t)i, gen, 0u, kDomSelect, key);
  keys[i] = ((uint64_t)k32 << 32) | (uint32_t)i;
}

__global__ __launch_bounds__(256) void select_rank_kernel(const uint64_t* __restrict__ keys,
                                                          int32_t count, int32_t keep,
                                                          int32_t* __restrict__ idx_out) {
  __shared__ uint64_t tile[1024];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t mine = i < count ? keys[i] : ~0ull;
  uint32_t rank = 0;
  for (int base = 0; base < count; base += 1024) {
    const int m = min(1024, count - base);
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += blockDim.x) tile[j] = keys[base + j];
    __syncthreads();
    for (int j = 0; j < m; ++j) rank += tile[j] < mine;
  }
  if (i < count && rank < (uint32_t)keep) idx_out[rank] = i;
}

}  // namespace dlm

using namespace dlm;

extern "C" int dlm_gpx_batch(const dlm_graph* g, int32_t k, const int16_t* parents, int32_t pop,
                             const int32_t* pairs, int32_t npairs, int32_t per_pair,
                             uint64_t seed, uint32_t child_base, int16_t* children,
                             void* stream) {
  if (!g) return set_error(DLM_E_INVAL, "dlm_gpx_batch: graph is NULL");
  if (k < 1 || k > 32767) return set_error(DLM_E_INVAL, "dlm_gpx_batch: k=%d outside [1, 32767]", k);
  if (pop < 1 || npairs < 0 || per_pair < 1)
    return set_error(DLM_E_INVAL, "dlm_gpx_batch: pop=%d npairs=%d per_pair=%d", pop, npairs, per_pair);
  const int64_t nchild = (int64_t)npairs * per_pair;
  if (nchild > 0x7fffffffll) return set_error(DLM_E_INVAL, "dlm_gpx_batch: too many children");
  if (nchild == 0) return DLM_OK;
  if (!parents || !pairs || !children) return set_error(DLM_E_INVAL, "dlm_gpx_batch: null buffer");
  const size_t lds = align16(6u * g->n) + 8u * k;
  if ((int64_t)lds > device_lds_limit())
    return set_error(DLM_E_UNSUPPORTED, "dlm_gpx_batch: %zu bytes of LDS needed", lds);
  auto kern = gpx_kernel<256>;
  DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3((unsigned)nchild), dim3(256), lds, (hipStream_t)stream, g->n, k,
                     pop, parents, pairs, per_pair, child_base, make_key(seed), children);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

extern "C" int dlm_select(const float* scores, int32_t count, int32_t keep, int32_t mode,
                          uint64_t seed, uint32_t gen, int32_t* idx_out, void* workspace,
                          void* stream) {
  if (count < 0 || keep < 0 || keep > count)
    return set_error(DLM_E_INVAL, "dlm_select: count=%d keep=%d", count, keep);
  if (mode != 0 && mode != 1) return set_error(DLM_E_INVAL, "dlm_select: mode=%d", mode);
  if (count == 0 || keep == 0) return DLM_OK;
  if ((mode == 0 && !scores) || !idx_out || !workspace)
    return set_error(DLM_E_INVAL, "dlm_select: null buffer");
  hipStream_t s = (hipStream_t)stream;
  uint64_t* keys = (uint64_t*)workspace;
  const unsigned grid = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(select_keys_kernel, dim3(grid), dim3(256), 0, s, scores, count, mode,
                     make_key(seed), gen, keys);
  DLM_HIP(hipGetLastError());
  hipLaunchKernelGGL(select_rank_kernel, dim3(grid), dim3(256), 0, s, keys, count, keep, idx_out);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}
