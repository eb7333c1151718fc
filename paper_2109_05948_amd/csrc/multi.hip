// Uneven batches: populations of many graphs (different n, k, budgets) in one
// persistent launch, captured once into a hipGraph and replayed.
//
// Work items are (graph, individual) pairs ordered longest-first (graphs by
// n * k * iterations, descending).  The grid holds as many workgroups as the
// device keeps resident at the launch's LDS size; each workgroup pops items
// from an atomic counter until the queue is empty, so every workgroup exits.
// A graph whose table fits the launch's LDS budget runs the LDS16 table, one
// whose byte gamma alone fits runs the SPLIT8 table (expiries in device
// memory, a rerun with the device-memory table in the same slot if a colour
// class would pass 255 vertices), the others the device-memory table; device
// storage is one slot per workgroup.  The search itself is the same function
// as dlm_tabu_batch's, so trajectories are identical to single-graph runs
// with the same seeds and indices.
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "tabu_body.h"

namespace dlm {

struct MultiDesc {
  TabuArgs a;
  int32_t tier;        // 0 = LDS16, 1 = GLOBAL16, 3 = SPLIT8 (GLOBAL16 rerun past 255 per class)
  int32_t first_item;  // items [first_item, first_item + pop) belong to this graph
  int32_t pop;
  int32_t pad;
};

__global__ void fill_u32_kernel(uint32_t* p, int32_t n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void tabu_multi_kernel(const MultiDesc* __restrict__ descs, int32_t ndesc,
                                                           int32_t total, uint32_t* __restrict__ queue,
                                                           uint32_t* __restrict__ gslots, int64_t slot_words) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_item;
  unsigned char* gtab =
      gslots ? reinterpret_cast<unsigned char*>(gslots + (size_t)blockIdx.x * (size_t)slot_words) : nullptr;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(queue, 1u);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= total) break;  // uniform: every workgroup reaches this exit
    int g = 0;
    while (g + 1 < ndesc && descs[g + 1].first_item <= item) ++g;
    const MultiDesc& d = descs[g];
    const int li = item - d.first_item;
    if (d.tier == 0) {
      tabu_individual<BLOCK, TabLds16>(d.a, li, nullptr, smem);
    } else if (d.tier == 3) {
      // byte gamma; the start colouring waits behind the slot's table for a
      // 16-bit rerun if a colour class would pass 255 vertices
      const int n = d.a.n;
      int16_t* gcol = d.a.colors + (size_t)li * n;
      int16_t* save = reinterpret_cast<int16_t*>(gtab + tab_entries(n, d.a.k) * TabGlobal16::kGlobalBytes);
      for (int v = threadIdx.x; v < n; v += BLOCK) save[v] = gcol[v];
      __syncthreads();
      tabu_individual<BLOCK, TabSplit8>(d.a, li, gtab, smem);
      __syncthreads();
      if (d.a.iters[li] == -2) {
        for (int v = threadIdx.x; v < n; v += BLOCK) gcol[v] = save[v];
        __syncthreads();
        tabu_individual<BLOCK, TabGlobal16>(d.a, li, gtab, smem);
      }
    } else {
      tabu_individual<BLOCK, TabGlobal16>(d.a, li, gtab, smem);
    }
  }
}

}  // namespace dlm

using namespace dlm;

struct dlm_multi_plan {
  int32_t block = 256, lds_budget = 0, grid = 0, total = 0, ndesc = 0, n_global = 0;
  size_t lds = 0;
  int64_t slot_words = 0;
  MultiDesc* d_descs = nullptr;
  uint32_t* d_queue = nullptr;
  uint32_t* d_slots = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int validate_items(const dlm_multi_item* items, int32_t count) {
  if (count < 1 || !items) return set_error(DLM_E_INVAL, "dlm_multi: count=%d", count);
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    const dlm_multi_item& it = items[i];
    if (!it.g) return set_error(DLM_E_INVAL, "dlm_multi: item %d has no graph", i);
    if (it.k < 1 || it.k > 32767 || it.max_iters < 0 || it.max_iters > (1 << 30) || it.pop < 0 ||
        it.ten_den <= 0 || it.ten_num < 0 || it.ten_num > 32767 || it.ten_rand < 1 || it.ten_rand > 1024 ||
        it.ind_base < 0 || (int64_t)it.ind_base + it.pop > 0x7fffffffll || it.reserved != 0)
      return set_error(DLM_E_INVAL, "dlm_multi: item %d has invalid parameters", i);
    if (it.pop > 0 && (!it.colors_dev || !it.f_best_dev || !it.iters_dev))
      return set_error(DLM_E_INVAL, "dlm_multi: item %d has a null output buffer", i);
    total += it.pop;
  }
  if (total > 0x7fffffffll) return set_error(DLM_E_INVAL, "dlm_multi: too many individuals");
  return DLM_OK;
}

template <int BLOCK>
int occupancy(size_t lds, int* per_cu) {
  DLM_HIP(hipFuncSetAttribute((const void*)tabu_multi_kernel<BLOCK>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  DLM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, tabu_multi_kernel<BLOCK>, BLOCK, lds));
  return DLM_OK;
}

int launch_persistent(const dlm_multi_plan* p, hipStream_t s) {
  switch (p->block) {
#define DLM_CASE(B)                                                                                       \
  case B:                                                                                                 \
    hipLaunchKernelGGL(tabu_multi_kernel<B>, dim3(p->grid), dim3(B), p->lds, s, p->d_descs, p->ndesc,     \
                       p->total, p->d_queue, p->d_slots, p->slot_words);                                  \
    break;
    DLM_CASE(64)
    DLM_CASE(128)
    DLM_CASE(256)
    DLM_CASE(512)
#undef DLM_CASE
    default:
      return set_error(DLM_E_INVAL, "dlm_multi: block=%d not in {64,128,256,512}", p->block);
  }
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

void free_plan(dlm_multi_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  (void)hipFree(p->d_descs);
  (void)hipFree(p->d_queue);
  (void)hipFree(p->d_slots);
  delete p;
}

}  // namespace

extern "C" {

int dlm_multi_plan_create(const dlm_multi_item* items, int32_t count, const dlm_multi_config* cfg,
                          void* stream, dlm_multi_plan** out) {
  if (!out) return set_error(DLM_E_INVAL, "dlm_multi_plan_create: out is NULL");
  *out = nullptr;
  int rc = validate_items(items, count);
  if (rc != DLM_OK) return rc;
  const int block = cfg && cfg->block ? cfg->block : 256;
  if (block != 64 && block != 128 && block != 256 && block != 512)
    return set_error(DLM_E_INVAL, "dlm_multi_plan_create: block=%d not in {64,128,256,512}", block);
  const int nw = block / kWave;
  const int64_t lds_max = device_lds_limit();
  const int64_t budget = cfg && cfg->lds_budget ? std::min<int64_t>(cfg->lds_budget, lds_max) : lds_max;
  // longest first
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ca = (double)items[a].g->n * items[a].k * items[a].max_iters;
    const double cb = (double)items[b].g->n * items[b].k * items[b].max_iters;
    return ca > cb;
  });
  dlm_multi_plan* p = new dlm_multi_plan();
  p->block = block;
  p->lds_budget = (int32_t)budget;
  std::vector<MultiDesc> descs;
  int32_t first = 0;
  size_t lds = tabu_layout(1, 1, nw, 0).bytes;
  for (int oi : order) {
    const dlm_multi_item& it = items[oi];
    if (it.pop == 0) continue;
    const int n = it.g->n;
    MultiDesc d{};
    d.a = TabuArgs{it.g->row_ptr, it.g->col_idx, it.g->erow, it.colors_dev, it.f_best_dev, it.iters_dev,
                   it.stats_dev, it.hash_dev, nullptr, nullptr, make_key(it.seed), n, it.k, it.max_iters,
                   it.ten_num, it.ten_den, it.ten_rand, it.ind_base, 0};
    const uint64_t lds16 = tabu_layout(n, it.k, nw, TabLds16::kLdsBytes).bytes;
    const uint64_t lds8 = tabu_layout(n, it.k, nw, TabSplit8::kLdsBytes).bytes;
    if ((int64_t)lds16 <= budget) {
      d.tier = 0;
      lds = std::max<size_t>(lds, lds16);
    } else if ((int64_t)lds8 <= budget) {
      d.tier = 3;
      ++p->n_global;
      lds = std::max<size_t>(lds, lds8);
      // packed 16-bit table for a rerun (the byte run's expiries use the first half) + the start colouring
      p->slot_words = std::max<int64_t>(p->slot_words, (int64_t)tab_entries(n, it.k) + (n + 1) / 2);
    } else {
      d.tier = 1;
      ++p->n_global;
      lds = std::max<size_t>(lds, tabu_layout(n, it.k, nw, 0).bytes);
      p->slot_words = std::max<int64_t>(p->slot_words, (int64_t)tab_entries(n, it.k));
    }
    d.first_item = first;
    d.pop = it.pop;
    first += it.pop;
    descs.push_back(d);
  }
  p->slot_words = (p->slot_words + 3) & ~int64_t(3);  // 16-byte aligned slots
  p->total = first;
  p->ndesc = (int32_t)descs.size();
  p->lds = lds;
  if ((int64_t)lds > lds_max) {
    free_plan(p);
    return set_error(DLM_E_UNSUPPORTED, "dlm_multi_plan_create: %zu bytes of LDS needed", lds);
  }
  int per_cu = 0;
  switch (block) {
    case 64: rc = occupancy<64>(lds, &per_cu); break;
    case 128: rc = occupancy<128>(lds, &per_cu); break;
    case 256: rc = occupancy<256>(lds, &per_cu); break;
    default: rc = occupancy<512>(lds, &per_cu); break;
  }
  if (rc != DLM_OK) {
    free_plan(p);
    return rc;
  }
  p->grid = std::max(1, std::min(per_cu * device_cu_count(), std::max(p->total, 1)));
  hipStream_t s = (hipStream_t)stream;
  auto fail = [&](hipError_t e, const char* what) {
    free_plan(p);
    return hip_fail(e, what);
  };
  hipError_t e;
  if ((e = hipMalloc(&p->d_descs, sizeof(MultiDesc) * std::max<size_t>(descs.size(), 1))) != hipSuccess)
    return fail(e, "hipMalloc");
  if ((e = hipMalloc(&p->d_queue, 256)) != hipSuccess) return fail(e, "hipMalloc");
  if (p->slot_words > 0 &&
      (e = hipMalloc(&p->d_slots, sizeof(uint32_t) * (size_t)p->slot_words * p->grid)) != hipSuccess)
    return fail(e, "hipMalloc");
  if (!descs.empty() &&
      (e = hipMemcpy(p->d_descs, descs.data(), sizeof(MultiDesc) * descs.size(), hipMemcpyHostToDevice)) !=
          hipSuccess)
    return fail(e, "hipMemcpy");
  // capture: queue reset (a fill kernel, no memset node) + the persistent kernel
  hipStream_t cs;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return fail(e, "hipStreamCreate");
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(e, "hipStreamBeginCapture");
  }
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, cs, p->d_queue, 1, 0u);
  rc = p->total > 0 ? launch_persistent(p, cs) : DLM_OK;
  e = hipStreamEndCapture(cs, &p->graph);
  (void)hipStreamDestroy(cs);
  if (rc != DLM_OK) {
    free_plan(p);
    return rc;
  }
  if (e != hipSuccess) return fail(e, "hipStreamEndCapture");
  if ((e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess)
    return fail(e, "hipGraphInstantiate");
  (void)s;
  *out = p;
  return DLM_OK;
}

int dlm_multi_plan_launch(dlm_multi_plan* p, void* stream) {
  if (!p) return set_error(DLM_E_INVAL, "dlm_multi_plan_launch: plan is NULL");
  DLM_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
  return DLM_OK;
}

int dlm_multi_plan_info(const dlm_multi_plan* p, int32_t* grid, int32_t* lds_bytes, int32_t* n_global,
                        int32_t* total_items) {
  if (!p) return set_error(DLM_E_INVAL, "dlm_multi_plan_info: plan is NULL");
  if (grid) *grid = p->grid;
  if (lds_bytes) *lds_bytes = (int32_t)p->lds;
  if (n_global) *n_global = p->n_global;
  if (total_items) *total_items = p->total;
  return DLM_OK;
}

int dlm_multi_plan_destroy(dlm_multi_plan* p) {
  free_plan(p);
  return DLM_OK;
}

// Calibration: each candidate (block, LDS budget) runs the batch on scratch
// copies of the colourings with `calib_iters` iterations per individual;
// the fastest in iterations per second wins.  Results are cached per
// (device, item shapes).
int dlm_multi_autotune(const dlm_multi_item* items, int32_t count, int32_t calib_iters,
                       dlm_multi_config* best, float* rates, void* stream) {
  int rc = validate_items(items, count);
  if (rc != DLM_OK) return rc;
  if (!best || calib_iters < 1) return set_error(DLM_E_INVAL, "dlm_multi_autotune: bad arguments");
  static std::mutex mu;
  static std::map<std::vector<int64_t>, dlm_multi_config> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<int64_t> key{dev, calib_iters};
  for (int i = 0; i < count; ++i) {
    key.push_back(items[i].g->n);
    key.push_back(items[i].g->nnz);
    key.push_back(items[i].k);
    key.push_back(items[i].pop);
  }
  const int blocks[] = {64, 128, 256, 512};
  const int64_t lds_max = device_lds_limit();
  const int64_t budgets[] = {lds_max / 4, lds_max / 2, lds_max};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto hit = cache.find(key);
    if (hit != cache.end() && !rates) {
      *best = hit->second;
      return DLM_OK;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  // scratch copies and outputs
  std::vector<dlm_multi_item> cal(items, items + count);
  std::vector<void*> bufs;
  auto cleanup = [&]() {
    for (void* b : bufs) (void)hipFree(b);
  };
  int64_t total_iters_bound = 0;
  for (int i = 0; i < count; ++i) {
    dlm_multi_item& c = cal[i];
    if (c.pop == 0) continue;
    const size_t cb = sizeof(int16_t) * (size_t)c.pop * c.g->n;
    void *col, *fb, *it;
    hipError_t e;
    if ((e = hipMalloc(&col, cb)) != hipSuccess || (e = hipMalloc(&fb, 4 * (size_t)c.pop)) != hipSuccess ||
        (e = hipMalloc(&it, 4 * (size_t)c.pop)) != hipSuccess) {
      cleanup();
      return hip_fail(e, "hipMalloc (autotune)");
    }
    bufs.push_back(col);
    bufs.push_back(fb);
    bufs.push_back(it);
    c.colors_dev = (int16_t*)col;
    c.f_best_dev = (int32_t*)fb;
    c.iters_dev = (int32_t*)it;
    c.stats_dev = nullptr;
    c.hash_dev = nullptr;
    c.max_iters = std::min(c.max_iters, calib_iters);
    total_iters_bound += (int64_t)c.pop * c.max_iters;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float best_rate = -1.f;
  dlm_multi_config best_cfg{256, 0};
  int ci = 0;
  for (int b : blocks)
    for (int64_t bud : budgets) {
      dlm_multi_config cfg{b, (int32_t)bud};
      for (int i = 0; i < count; ++i)
        if (cal[i].pop)
          (void)hipMemcpyAsync(cal[i].colors_dev, items[i].colors_dev,
                               sizeof(int16_t) * (size_t)cal[i].pop * cal[i].g->n, hipMemcpyDeviceToDevice, s);
      dlm_multi_plan* p = nullptr;
      float rate = 0.f;
      if (dlm_multi_plan_create(cal.data(), count, &cfg, stream, &p) == DLM_OK) {
        (void)hipEventRecord(e0, s);
        rc = dlm_multi_plan_launch(p, stream);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // iterations actually run (early stops at f = 0 count as run iterations)
        int64_t iters = 0;
        for (int i = 0; i < count; ++i) {
          if (!cal[i].pop) continue;
          std::vector<int32_t> h(cal[i].pop);
          (void)hipMemcpy(h.data(), cal[i].iters_dev, 4 * (size_t)cal[i].pop, hipMemcpyDeviceToHost);
          for (int32_t x : h) iters += x;
        }
        rate = ms > 0.f && rc == DLM_OK ? (float)(iters / (ms * 1e-3)) : 0.f;
        dlm_multi_plan_destroy(p);
      }
      if (rates) rates[ci] = rate;
      ++ci;
      if (rate > best_rate) {
        best_rate = rate;
        best_cfg = cfg;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  (void)total_iters_bound;
  if (best_rate <= 0.f) return set_error(DLM_E_HIP, "dlm_multi_autotune: no configuration ran");
  *best = best_cfg;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = best_cfg;
  return DLM_OK;
}

}  // extern "C"
