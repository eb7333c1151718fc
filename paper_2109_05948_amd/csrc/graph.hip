// Library core: error reporting, graph ingest (validation + upload) and the
// score kernels (conflicts, eq. (f); weighted score, eq. (score_WVCP)).
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

#include "dlm_common.h"

namespace dlm {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? DLM_E_NOMEM : DLM_E_HIP, "%s failed: %s", what,
                   hipGetErrorString(e));
}

int device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

int device_lds_per_cu() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || v <= 0)
    return 65536;
  return v;
}

int device_cu_count() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return v;
}

// ---------------------------------------------------------------------------
// Scores: one workgroup per colouring.
__global__ __launch_bounds__(256) void evaluate_kernel(const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       const int32_t* __restrict__ erow,
                                                       const int32_t* __restrict__ weights,
                                                       int32_t n, int32_t k,
                                                       const int16_t* __restrict__ colors,
                                                       int32_t* __restrict__ conflicts,
                                                       int32_t* __restrict__ wscore) {
  extern __shared__ __align__(16) unsigned char smem[];
  int16_t* col = reinterpret_cast<int16_t*>(smem);
  uint32_t* cmax = reinterpret_cast<uint32_t*>(smem + align16(2u * n));
  uint32_t* red = cmax + (wscore ? k : 0);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t row = blockIdx.x;
  int bad = 0;
  for (int v = tid; v < n; v += blockDim.x) {
    const int c = colors[row * n + v];
    bad |= (c < 0) | (c >= k);
    col[v] = (int16_t)c;
  }
  if (wscore)
    for (int c = tid; c < k; c += blockDim.x) cmax[c] = 0;
  if (__syncthreads_or(bad)) {  // a colour outside [0, k): no score
    if (tid == 0) {
      conflicts[row] = -1;
      if (wscore) wscore[row] = -1;
    }
    return;
  }
  uint32_t same = 0;
  const int32_t nnz = row_ptr[n];
  for (int e = tid; e < nnz; e += blockDim.x) {
    const int u = erow[e], v = col_idx[e];
    same += (u < v) & (col[u] == col[v]);
  }
  if (wscore)
    for (int v = tid; v < n; v += blockDim.x) atomicMax(&cmax[col[v]], (uint32_t)weights[v]);
  uint32_t s = wave_sum_u32(same);
  if (lane == 0) red[wid] = s;
  __syncthreads();
  uint32_t ws = 0;
  if (wscore)
    for (int c = tid; c < k; c += blockDim.x) ws += cmax[c];
  ws = wave_sum_u32(ws);
  if (lane == 0) red[8 + wid] = ws;
  __syncthreads();
  if (tid == 0) {
    uint32_t a = 0, b = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += red[w];
      b += red[8 + w];
    }
    conflicts[row] = (int32_t)a;
    if (wscore) wscore[row] = (int32_t)b;
  }
}

}  // namespace dlm

using namespace dlm;

extern "C" {

int dlm_abi_version(void) { return DLM_ABI_VERSION; }

const char* dlm_last_error(void) { return g_last_error.c_str(); }

int dlm_graph_create(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                     const int32_t* weights, uint32_t flags, void* stream, dlm_graph** out) {
  if (!out) return set_error(DLM_E_INVAL, "dlm_graph_create: out is NULL");
  *out = nullptr;
  if (flags & ~(uint32_t)DLM_G_BITSET) return set_error(DLM_E_INVAL, "dlm_graph_create: unknown flags 0x%x", flags);
  if (flags & DLM_G_BITSET)
    return set_error(DLM_E_UNSUPPORTED, "dlm_graph_create: bitset adjacency rows are not built by this library");
  if (n < 1 || n > 32767) return set_error(DLM_E_INVAL, "dlm_graph_create: n=%d outside [1, 32767]", n);
  if (!row_ptr) return set_error(DLM_E_INVAL, "dlm_graph_create: row_ptr is NULL");
  if (row_ptr[0] != 0) return set_error(DLM_E_INVAL, "dlm_graph_create: row_ptr[0] != 0");
  int32_t max_deg = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t d = row_ptr[v + 1] - row_ptr[v];
    if (d < 0) return set_error(DLM_E_INVAL, "dlm_graph_create: row_ptr decreases at %d", v);
    if (d > max_deg) max_deg = d;
  }
  const int64_t nnz = row_ptr[n];
  if (nnz > 0 && !col_idx) return set_error(DLM_E_INVAL, "dlm_graph_create: col_idx is NULL");
  std::vector<int32_t> erow((size_t)nnz);
  for (int32_t v = 0; v < n; ++v) {
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int32_t u = col_idx[e];
      if (u < 0 || u >= n)
        return set_error(DLM_E_INVAL, "dlm_graph_create: col_idx[%d]=%d out of range", e, u);
      if (u == v) return set_error(DLM_E_INVAL, "dlm_graph_create: self loop at vertex %d", v);
      if (e > row_ptr[v] && col_idx[e - 1] >= u)
        return set_error(DLM_E_INVAL, "dlm_graph_create: row %d not strictly ascending", v);
      erow[(size_t)e] = v;
    }
  }
  // symmetry: u in N(v) => v in N(u), by binary search in the sorted row of u
  for (int32_t v = 0; v < n; ++v)
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int32_t u = col_idx[e];
      int32_t lo = row_ptr[u], hi = row_ptr[u + 1];
      bool found = false;
      while (lo < hi) {
        const int32_t mid = (lo + hi) / 2;
        if (col_idx[mid] == v) {
          found = true;
          break;
        }
        if (col_idx[mid] < v) lo = mid + 1;
        else hi = mid;
      }
      if (!found)
        return set_error(DLM_E_INVAL, "dlm_graph_create: edge (%d,%d) has no reverse", v, u);
    }
  int32_t max_w = 0;
  if (weights)
    for (int32_t v = 0; v < n; ++v) {
      if (weights[v] <= 0)
        return set_error(DLM_E_INVAL, "dlm_graph_create: weight of vertex %d is %d (must be > 0)", v,
                         weights[v]);
      if (weights[v] > max_w) max_w = weights[v];
    }
  if (weights && (int64_t)max_w * n > (1ll << 30))
    return set_error(DLM_E_UNSUPPORTED, "dlm_graph_create: n * max weight exceeds 2^30");

  // greedy WVCP start (Section 2.1): vertices by weight descending, then
  // degree descending, then index ascending; a property of the graph, so it
  // is computed once here
  std::vector<int32_t> order;
  if (weights) {
    order.resize((size_t)n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      if (weights[a] != weights[b]) return weights[a] > weights[b];
      const int32_t da = row_ptr[a + 1] - row_ptr[a], db = row_ptr[b + 1] - row_ptr[b];
      if (da != db) return da > db;
      return a < b;
    });
  }

  dlm_graph* g = new dlm_graph();
  g->n = n;
  g->nnz = nnz;
  g->max_deg = max_deg;
  g->max_w = max_w;
  (void)hipGetDevice(&g->device);
  hipStream_t s = (hipStream_t)stream;
  auto fail = [&](hipError_t e, const char* what) {
    (void)hipStreamSynchronize(s);  // no copy may still read or write g's buffers
    dlm_graph_destroy(g);
    return hip_fail(e, what);
  };
  auto upload = [&](int32_t** dst, const int32_t* src, int64_t count) -> hipError_t {
    hipError_t e = hipMalloc(dst, sizeof(int32_t) * (size_t)(count > 0 ? count : 1));
    if (e == hipSuccess && count > 0)
      e = hipMemcpyAsync(*dst, src, sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice, s);
    return e;
  };
  hipError_t e;
  if ((e = upload(&g->row_ptr, row_ptr, n + 1)) != hipSuccess) return fail(e, "graph upload (row_ptr)");
  if ((e = upload(&g->col_idx, col_idx, nnz)) != hipSuccess) return fail(e, "graph upload (col_idx)");
  if ((e = upload(&g->erow, erow.data(), nnz)) != hipSuccess) return fail(e, "graph upload (erow)");
  if (weights) {
    if ((e = upload(&g->weights, weights, n)) != hipSuccess) return fail(e, "graph upload (weights)");
    if ((e = upload(&g->order, order.data(), n)) != hipSuccess) return fail(e, "graph upload (order)");
  }
  // the host arrays (the caller's and the local ones) are read synchronously
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "hipStreamSynchronize");
  *out = g;
  return DLM_OK;
}

int dlm_graph_destroy(dlm_graph* g) {
  if (!g) return DLM_OK;
  (void)hipFree(g->row_ptr);
  (void)hipFree(g->col_idx);
  (void)hipFree(g->erow);
  (void)hipFree(g->weights);
  (void)hipFree(g->order);
  delete g;
  return DLM_OK;
}

int dlm_graph_info(const dlm_graph* g, int32_t* n, int64_t* nnz, int32_t* max_deg) {
  if (!g) return set_error(DLM_E_INVAL, "dlm_graph_info: graph is NULL");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_deg) *max_deg = g->max_deg;
  return DLM_OK;
}

int dlm_evaluate(const dlm_graph* g, int32_t k, const int16_t* colors, int32_t count,
                 int32_t* conflicts, int32_t* wscore, void* stream) {
  if (!g) return set_error(DLM_E_INVAL, "dlm_evaluate: graph is NULL");
  if (count < 0) return set_error(DLM_E_INVAL, "dlm_evaluate: count < 0");
  if (count == 0) return DLM_OK;
  if (!colors || !conflicts) return set_error(DLM_E_INVAL, "dlm_evaluate: null buffer");
  if (k < 1 || k > 32767) return set_error(DLM_E_INVAL, "dlm_evaluate: k=%d outside [1, 32767]", k);
  if (wscore && !g->weights) return set_error(DLM_E_INVAL, "dlm_evaluate: wscore needs vertex weights");
  const size_t lds = align16(2u * g->n) + 4u * (wscore ? k : 0) + 4u * 16;
  if ((int)lds > device_lds_limit())
    return set_error(DLM_E_UNSUPPORTED, "dlm_evaluate: %zu bytes of LDS needed", lds);
  hipLaunchKernelGGL(evaluate_kernel, dim3(count), dim3(256), lds, (hipStream_t)stream, g->row_ptr,
                     g->col_idx, g->erow, g->weights, g->n, k, colors, conflicts, wscore);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

}  // extern "C"
