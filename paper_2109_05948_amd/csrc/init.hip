// Population initialisation (Section 2.7: uniform random colours for k-COL;
// Section 2.1: randomized greedy for the weighted problem).
#include <algorithm>
#include <numeric>
#include <vector>

#include "dlm_common.h"

namespace dlm {

__global__ __launch_bounds__(256) void init_random_kernel(int32_t n, int32_t k, int64_t total,
                                                          Key key, int32_t ind_base,
                                                          int16_t* __restrict__ colors) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int32_t i = (int32_t)(idx / n), v = (int32_t)(idx - (int64_t)i * n);
  const uint32_t w = philox_w0((uint32_t)(ind_base + i), 0u, (uint32_t)v, kDomInit, key);
  colors[idx] = (int16_t)lemire(w, (uint32_t)k);
}

// One workgroup per individual; vertices are coloured one after another in
// the fixed greedy order, the neighbour scan of each vertex is parallel.
__global__ __launch_bounds__(256) void init_greedy_kernel(const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col_idx,
                                                          const int32_t* __restrict__ order,
                                                          int32_t n, Key key, int32_t ind_base,
                                                          int16_t* __restrict__ colors,
                                                          int32_t* __restrict__ k_used) {
  extern __shared__ __align__(16) unsigned char smem[];
  int16_t* col = reinterpret_cast<int16_t*>(smem);
  uint32_t* blocked = reinterpret_cast<uint32_t*>(smem + align16(2u * n));  // ceil((n+1)/32) words
  __shared__ int32_t s_used;
  const int tid = threadIdx.x;
  const int32_t ind = ind_base + (int32_t)blockIdx.x;
  for (int v = tid; v < n; v += blockDim.x) col[v] = -1;
  if (tid == 0) s_used = 0;
  __syncthreads();
  for (int a = 0; a < n; ++a) {
    const int v = order[a];
    const int used = s_used;
    const int nwords = (used + 31) >> 5;
    for (int w = tid; w < nwords; w += blockDim.x) blocked[w] = 0;
    __syncthreads();
    for (int e = row_ptr[v] + tid; e < row_ptr[v + 1]; e += blockDim.x) {
      const int cu = col[col_idx[e]];
      if (cu >= 0) atomicOr(&blocked[cu >> 5], 1u << (cu & 31));
    }
    __syncthreads();
    if (tid == 0) {
      int nf = 0;
      for (int w = 0; w < nwords; ++w) {
        const uint32_t valid = (w == nwords - 1 && (used & 31)) ? ((1u << (used & 31)) - 1u) : 0xffffffffu;
        nf += __popc(~blocked[w] & valid);
      }
      if (nf == 0) {
        col[v] = (int16_t)used;
        s_used = used + 1;
      } else {
        int r = (int)lemire(philox_w0((uint32_t)ind, 0u, (uint32_t)v, kDomGreedy, key), (uint32_t)nf);
        for (int w = 0; w < nwords; ++w) {
          const uint32_t valid = (w == nwords - 1 && (used & 31)) ? ((1u << (used & 31)) - 1u) : 0xffffffffu;
          uint32_t free_bits = ~blocked[w] & valid;
          const int cnt = __popc(free_bits);
          if (r < cnt) {
            for (int s = 0; s < r; ++s) free_bits &= free_bits - 1;  // drop the r lowest free colours
            col[v] = (int16_t)(w * 32 + __ffs(free_bits) - 1);
            break;
          }
          r -= cnt;
        }
      }
    }
    __syncthreads();
  }
  const int64_t base = (int64_t)blockIdx.x * n;
  for (int v = tid; v < n; v += blockDim.x) colors[base + v] = col[v];
  if (tid == 0 && k_used) k_used[blockIdx.x] = s_used;
}

__global__ void fill_i32_kernel(int32_t* p, int32_t n, int32_t value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

}  // namespace dlm

using namespace dlm;

extern "C" int dlm_init_population(const dlm_graph* g, int32_t k, int32_t pop, uint64_t seed,
                                   int32_t ind_base, int32_t mode, int16_t* colors,
                                   int32_t* k_used, void* stream) {
  if (!g) return set_error(DLM_E_INVAL, "dlm_init_population: graph is NULL");
  if (pop < 0) return set_error(DLM_E_INVAL, "dlm_init_population: pop < 0");
  if (ind_base < 0 || (int64_t)ind_base + pop > 0x7fffffffll)
    return set_error(DLM_E_INVAL, "dlm_init_population: ind_base + pop exceeds 2^31");
  if (pop == 0) return DLM_OK;
  if (!colors) return set_error(DLM_E_INVAL, "dlm_init_population: colors is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (mode == DLM_INIT_RANDOM) {
    if (k < 1 || k > 32767) return set_error(DLM_E_INVAL, "dlm_init_population: k=%d outside [1, 32767]", k);
    const int64_t total = (int64_t)pop * g->n;
    hipLaunchKernelGGL(init_random_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g->n,
                       k, total, make_key(seed), ind_base, colors);
    DLM_HIP(hipGetLastError());
    if (k_used) {
      hipLaunchKernelGGL(fill_i32_kernel, dim3((pop + 255) / 256), dim3(256), 0, s, k_used, pop, k);
      DLM_HIP(hipGetLastError());
    }
    return DLM_OK;
  }
  if (mode != DLM_INIT_GREEDY) return set_error(DLM_E_INVAL, "dlm_init_population: unknown mode %d", mode);
  if (!g->weights) return set_error(DLM_E_INVAL, "dlm_init_population: greedy mode needs vertex weights");
  // the greedy order (weight descending, degree descending, index ascending)
  // was computed when the graph was created
  const size_t lds = align16(2u * g->n) + 4u * ((g->n + 32) / 32 + 1);
  hipLaunchKernelGGL(init_greedy_kernel, dim3(pop), dim3(256), lds, s, g->row_ptr, g->col_idx, g->order,
                     g->n, make_key(seed), ind_base, colors, k_used);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}
