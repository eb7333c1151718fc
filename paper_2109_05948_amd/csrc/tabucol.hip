// Population TabuCol for k-COL (Section 2.7 of the paper: TabuCol with the
// gamma table of its efficient implementation), one workgroup per individual.
//
// Per individual (the search body and the table tiers are in tabu_body.h):
//   tab[v*kp + c]  gamma[v][c] (neighbours of v coloured c) and the tabu
//                  expiry of (v, c), rows padded to kp = k rounded up to 4;
//                  LDS16 packs both into a 32-bit LDS word, LDS32 keeps two,
//                  SPLIT16 / SPLIT8 keep 16- / 8-bit gamma in LDS and the
//                  expiries in device memory, GLOBAL16 keeps the packed word
//                  in device memory
//   cg[v]          colour of v (low 16) | gamma[v][col v] (high 16)
//   list, pos      the conflicting vertices (with tombstones), kept in place
//
// One iteration:
//   scan      every thread takes (list entry, colour quad) pairs strided by
//             the block size and keeps its three smallest admissible
//             candidate keys (biased delta << 16 | the thread's candidate
//             number);
//   wave      DPP minimum; the moves tied at the wave's minimum are hashed
//             (Philox of (ind, t, v, c)) unless another wave already
//             published a better delta;
//   reduce    one barrier, then the (delta, hash, v, c) minimum over the
//             waves' slots;
//   apply     all threads update the gamma rows of v*'s neighbours (CSR row
//             from device memory) and the conflict list; wave 0 writes the
//             tabu entries, v*'s state and the lazily kept best colouring.
//
// The byte-gamma tier gives up on an individual whose colour classes would
// pass 255 vertices; a rerun kernel repeats those from their start colouring
// with the 16-bit device table, so every tier returns the same result.
#include <mutex>

#include "tabu_body.h"
#include "tabu_wave.h"

namespace dlm {

template <int BLOCK, class Tab>
__global__ __launch_bounds__(BLOCK) void tabucol_kernel(TabuArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int li = blockIdx.x;
  unsigned char* gtab =
      a.gtab ? a.gtab + (size_t)li * (size_t)tab_entries(a.n, a.k) * Tab::kGlobalBytes : nullptr;
  tabu_individual<BLOCK, Tab>(a, li, gtab, smem);
}

// Byte-gamma runs that gave up (iters = -2: a colour class would pass 255
// vertices) start again from their saved start colouring with the packed
// 16-bit table in device memory.  A persistent grid walks the population;
// every workgroup owns one table slot and skips the individuals that
// finished.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void tabucol_rerun_kernel(TabuArgs a, const int16_t* __restrict__ start,
                                                              unsigned char* __restrict__ slots, int32_t pop) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* slot = slots + (size_t)blockIdx.x * (size_t)tab_entries(a.n, a.k) * TabGlobal16::kGlobalBytes;
  for (int li = blockIdx.x; li < pop; li += gridDim.x) {
    if (a.iters[li] != -2) continue;
    int16_t* gcol = a.colors + (size_t)li * a.n;
    for (int v = threadIdx.x; v < a.n; v += BLOCK) gcol[v] = start[(size_t)li * a.n + v];
    __syncthreads();
    tabu_individual<BLOCK, TabGlobal16>(a, li, slot, smem);
    __syncthreads();
  }
}

// WAVE8: one wavefront per individual (tabu_wave.h)
template <int KQ>
__global__ __launch_bounds__(64) void tabucol_w8_kernel(TabuArgs a, int32_t acap) {
  extern __shared__ __align__(16) unsigned char smem[];
  tabu_w8_individual<KQ>(a, blockIdx.x, acap, smem);
}

template <int KQ>
static int launch_w8_kq(const TabuArgs& a, int pop, int acap, size_t lds, hipStream_t s) {
  auto kern = tabucol_w8_kernel<KQ>;
  DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(pop), dim3(64), lds, s, a, acap);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

static int launch_w8(const TabuArgs& a, int pop, int acap, size_t lds, hipStream_t s) {
  switch (w8_bucket(a.k)) {
    case 8: return launch_w8_kq<8>(a, pop, acap, lds, s);
    case 16:  // rows of 9 to 15 and 17 to 23 dwords get a kernel of their exact width
      switch (tab_stride(a.k) >> 2) {
        case 9: return launch_w8_kq<9>(a, pop, acap, lds, s);
        case 10: return launch_w8_kq<10>(a, pop, acap, lds, s);
        case 11: return launch_w8_kq<11>(a, pop, acap, lds, s);
        case 12: return launch_w8_kq<12>(a, pop, acap, lds, s);
        case 13: return launch_w8_kq<13>(a, pop, acap, lds, s);
        case 14: return launch_w8_kq<14>(a, pop, acap, lds, s);
        case 15: return launch_w8_kq<15>(a, pop, acap, lds, s);
        default: return launch_w8_kq<16>(a, pop, acap, lds, s);
      }
    case 24:
      switch (tab_stride(a.k) >> 2) {
        case 17: return launch_w8_kq<17>(a, pop, acap, lds, s);
        case 18: return launch_w8_kq<18>(a, pop, acap, lds, s);
        case 19: return launch_w8_kq<19>(a, pop, acap, lds, s);
        case 20: return launch_w8_kq<20>(a, pop, acap, lds, s);
        case 21: return launch_w8_kq<21>(a, pop, acap, lds, s);
        case 22: return launch_w8_kq<22>(a, pop, acap, lds, s);
        case 23: return launch_w8_kq<23>(a, pop, acap, lds, s);
        default: return launch_w8_kq<24>(a, pop, acap, lds, s);
      }
    case 32: return launch_w8_kq<32>(a, pop, acap, lds, s);
    case 64: return launch_w8_kq<64>(a, pop, acap, lds, s);
  }
  return set_error(DLM_E_UNSUPPORTED, "dlm_tabu_batch: k=%d too large for the wave table", a.k);
}

__global__ void copy_i16_kernel(const int16_t* __restrict__ src, int16_t* __restrict__ dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

struct Rerun {
  const int16_t* start;
  unsigned char* slots;
  int32_t grid;
};

template <int BLOCK, class Tab>
static int launch_block(const TabuArgs& a, int pop, size_t lds, hipStream_t s, const Rerun* rr) {
  if (rr) {
    auto kern = tabucol_rerun_kernel<BLOCK>;
    DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(rr->grid), dim3(BLOCK), lds, s, a, rr->start, rr->slots, pop);
  } else {
    auto kern = tabucol_kernel<BLOCK, Tab>;
    DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(pop), dim3(BLOCK), lds, s, a);
  }
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

// resident workgroups per CU of the search kernel at this LDS size (0 if unknown)
template <int BLOCK, class Tab>
static int resident_b(size_t lds) {
  int nb = 0;
  auto kern = tabucol_kernel<BLOCK, Tab>;
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, BLOCK, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <class Tab>
static int resident(int block, size_t lds) {
  switch (block) {
    case 64: return resident_b<64, Tab>(lds);
    case 128: return resident_b<128, Tab>(lds);
    case 256: return resident_b<256, Tab>(lds);
    case 512: return resident_b<512, Tab>(lds);
    case 1024: return resident_b<1024, Tab>(lds);
  }
  return 0;
}

// rr != nullptr launches the 16-bit rerun pass instead of the search
template <class Tab>
static int launch_tab(const TabuArgs& a, int pop, int block, size_t lds, hipStream_t s,
                      const Rerun* rr = nullptr) {
  switch (block) {
    case 64: return launch_block<64, Tab>(a, pop, lds, s, rr);
    case 128: return launch_block<128, Tab>(a, pop, lds, s, rr);
    case 256: return launch_block<256, Tab>(a, pop, lds, s, rr);
    case 512: return launch_block<512, Tab>(a, pop, lds, s, rr);
    case 1024: return launch_block<1024, Tab>(a, pop, lds, s, rr);
  }
  return set_error(DLM_E_INVAL, "dlm_tabu_batch: block=%d not in {64,128,256,512,1024}", block);
}


// How a call runs: the table tier and block (AUTO resolved), the LDS of the
// search (and rerun) kernel, and the caller-owned workspace it needs.
struct TabuPlan {
  int table = 0, block = 0;
  uint64_t lds = 0, lds_rr = 0;
  uint64_t gtab_bytes = 0;    // device-memory table part of every individual
  uint64_t start_bytes = 0;   // SPLIT8: copy of the start colourings
  uint64_t slot_bytes = 0;    // SPLIT8: one rerun slot (packed 16-bit table)
  int64_t slots = 0;          // SPLIT8: rerun slots
  int32_t acap = 0;           // WAVE8: tabu pairs each individual's LDS holds
  uint64_t ws_bytes = 0;      // total, each part on a 256-byte boundary
};

static uint64_t align256(uint64_t x) { return (x + 255u) & ~255ull; }

static int tabu_check(const char* fn, const dlm_graph* g, const dlm_tabu_params* p, int32_t pop) {
  if (!g || !p) return set_error(DLM_E_INVAL, "%s: graph or params is NULL", fn);
  if (pop < 0) return set_error(DLM_E_INVAL, "%s: pop < 0", fn);
  if (p->k < 1 || p->k > 32767) return set_error(DLM_E_INVAL, "%s: k=%d outside [1, 32767]", fn, p->k);
  if (p->max_iters < 0 || p->max_iters > (1 << 30))
    return set_error(DLM_E_INVAL, "%s: max_iters=%d outside [0, 2^30]", fn, p->max_iters);
  if (p->ten_den <= 0 || p->ten_num < 0 || p->ten_num > 32767)
    return set_error(DLM_E_INVAL, "%s: tenure slope %d/%d invalid", fn, p->ten_num, p->ten_den);
  if (p->ten_rand < 1 || p->ten_rand > 1024)
    return set_error(DLM_E_INVAL, "%s: ten_rand=%d outside [1, 1024]", fn, p->ten_rand);
  if (p->ind_base < 0 || (int64_t)p->ind_base + pop > 0x7fffffffll)
    return set_error(DLM_E_INVAL, "%s: ind_base + pop exceeds 2^31", fn);
  if (p->trace_cap < 0) return set_error(DLM_E_INVAL, "%s: trace_cap=%d < 0", fn, p->trace_cap);
  if (p->reserved != 0) return set_error(DLM_E_INVAL, "%s: reserved must be 0", fn);
  return DLM_OK;
}

static int tabu_plan(const char* fn, const dlm_graph* g, const dlm_tabu_params* p, int32_t pop, TabuPlan& P) {
  const int n = g->n, k = p->k;
  const int64_t lds_max = device_lds_limit();
  // automatic table with an automatic (or 64-thread) block: the wave table
  // whenever it holds the individual (it beat the block kernels at every
  // measured shape, one individual per CU included)
  const bool wave_auto = p->table == DLM_TABLE_AUTO && (p->block == 0 || p->block == 64) && w8_bucket(k) != 0 &&
                         (uint64_t)n * (uint64_t)tab_stride(k) <= (1ull << 17) &&
                         w8_layout(n, k, 0).bytes + 4u * kWave <= (uint64_t)lds_max;
  if (p->table == DLM_TABLE_WAVE8 || wave_auto) {
    if (p->block != 0 && p->block != 64)
      return set_error(DLM_E_INVAL, "%s: the wave table runs 64 threads per individual (block=%d)", fn, p->block);
    const uint64_t kp = (uint64_t)tab_stride(k);
    if (w8_bucket(k) == 0 || (uint64_t)n * kp > (1ull << 17))
      return set_error(DLM_E_UNSUPPORTED, "%s: n=%d, k=%d outside the wave table (k <= 256, n*kp <= 2^17)", fn, n, k);
    const uint64_t base = w8_layout(n, k, 0).bytes;
    const int64_t lds_cu = device_lds_per_cu();
    if (base + 4u * kWave > (uint64_t)lds_max)
      return set_error(DLM_E_UNSUPPORTED, "%s: %llu bytes of LDS needed, %lld available", fn,
                       (unsigned long long)(base + 4u * kWave), (long long)lds_max);
    // as many individuals per CU as the table allows; the rest of their
    // share of the CU's LDS holds tabu pairs
    const int64_t res = std::max<int64_t>(1, std::min<int64_t>(32, lds_cu / (int64_t)(base + 4u * kWave)));
    const int64_t budget = std::min<int64_t>(lds_max, lds_cu / res) & ~15ll;
    P.acap = (int32_t)std::min<int64_t>(16384, ((budget - (int64_t)base) / 4) & ~63ll);
    P.table = DLM_TABLE_WAVE8;
    P.block = 64;
    P.lds = w8_layout(n, k, P.acap).bytes;
    if (pop > 0) {
      P.slot_bytes = tab_entries(n, k) * TabGlobal16::kGlobalBytes;
      int64_t slots = std::min<int64_t>(pop, 2 * (int64_t)device_cu_count());
      P.slots = std::max<int64_t>(1, std::min<int64_t>(slots, (int64_t)((1ull << 30) / std::max<uint64_t>(P.slot_bytes, 1))));
      P.lds_rr = tabu_layout(n, k, 256 / kWave, TabGlobal16::kLdsBytes).bytes;
      P.start_bytes = sizeof(int16_t) * (uint64_t)pop * (uint64_t)n;
    }
    P.ws_bytes = align256(P.start_bytes) + align256(P.slot_bytes * (uint64_t)P.slots);
    return DLM_OK;
  }
  int block = p->block ? p->block : 256;
  if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
    return set_error(DLM_E_INVAL, "%s: block=%d not in {64,128,256,512,1024}", fn, block);
  int table = p->table;
  if (table == DLM_TABLE_AUTO) {
    // the LDS tier that keeps more individuals resident per CU; byte gamma on a tie loses
    const int nw0 = block / kWave;
    const uint64_t l16 = tabu_layout(n, k, nw0, TabLds16::kLdsBytes).bytes;
    const uint64_t l8 = tabu_layout(n, k, nw0, TabSplit8::kLdsBytes).bytes;
    const int o16 = l16 <= (uint64_t)lds_max ? resident<TabLds16>(block, l16) : 0;
    const int o8 = l8 <= (uint64_t)lds_max ? resident<TabSplit8>(block, l8) : 0;
    table = o8 > o16 ? DLM_TABLE_SPLIT8 : (o16 > 0 ? DLM_TABLE_LDS16 : DLM_TABLE_GLOBAL16);
    // automatic block: when a single LDS-resident individual fills a CU, 512
    // threads hide more of the per-move latency than 256
    if (p->block == 0 && std::max(o16, o8) == 1 && block == 256) block = 512;
  }
  const int nw = block / kWave;
  int eb = 0, gb = 0;
  switch (table) {
    case DLM_TABLE_LDS16: eb = TabLds16::kLdsBytes; break;
    case DLM_TABLE_LDS32: eb = TabLds32::kLdsBytes; break;
    case DLM_TABLE_GLOBAL16: eb = 0; gb = TabGlobal16::kGlobalBytes; break;
    case DLM_TABLE_SPLIT16: eb = TabSplit16::kLdsBytes; gb = TabSplit16::kGlobalBytes; break;
    case DLM_TABLE_SPLIT8: eb = TabSplit8::kLdsBytes; gb = TabSplit8::kGlobalBytes; break;
    default: return set_error(DLM_E_INVAL, "%s: unknown table %d", fn, table);
  }
  P.table = table;
  P.block = block;
  P.lds = tabu_layout(n, k, nw, eb).bytes;
  if (P.lds > (uint64_t)lds_max)
    return set_error(DLM_E_UNSUPPORTED, "%s: %llu bytes of LDS needed, %lld available", fn,
                     (unsigned long long)P.lds, (long long)lds_max);
  P.gtab_bytes = (uint64_t)pop * tab_entries(n, k) * (uint64_t)gb;
  if (table == DLM_TABLE_SPLIT8 && pop > 0) {
    // rerun slots: a few per CU, at most 1 GiB of packed tables
    P.slot_bytes = tab_entries(n, k) * TabGlobal16::kGlobalBytes;
    int64_t slots = std::min<int64_t>(pop, 2 * (int64_t)device_cu_count());
    P.slots = std::max<int64_t>(1, std::min<int64_t>(slots, (int64_t)((1ull << 30) / std::max<uint64_t>(P.slot_bytes, 1))));
    P.lds_rr = tabu_layout(n, k, nw, TabGlobal16::kLdsBytes).bytes;
    P.start_bytes = sizeof(int16_t) * (uint64_t)pop * (uint64_t)n;
  }
  P.ws_bytes = align256(P.gtab_bytes) + align256(P.start_bytes) + align256(P.slot_bytes * (uint64_t)P.slots);
  return DLM_OK;
}

// The search itself, after the caller's arguments passed tabu_check: plan,
// workspace checks, launches.  Shared by both entry points.
static int tabu_run(const char* fn, const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                    int16_t* colors, int32_t* f_best, int32_t* iters, int64_t* stats, uint64_t* hash,
                    int32_t* trace, void* workspace, size_t workspace_bytes, hipStream_t s,
                    uint64_t ws_limit) {
  if (p->trace_cap > 0 && !trace)
    return set_error(DLM_E_INVAL, "%s: trace_cap=%d needs a trace buffer", fn, p->trace_cap);
  if (pop == 0) return DLM_OK;
  if (!colors || !f_best || !iters) return set_error(DLM_E_INVAL, "%s: null output buffer", fn);
  TabuPlan P;
  int rc;
  if ((rc = tabu_plan(fn, g, p, pop, P)) != DLM_OK) return rc;
  if (P.ws_bytes > ws_limit)
    return set_error(DLM_E_UNSUPPORTED, "%s: %llu bytes of workspace needed, the fixed scratch holds %llu", fn,
                     (unsigned long long)P.ws_bytes, (unsigned long long)ws_limit);
  if (P.ws_bytes > 0 && (!workspace || workspace_bytes < P.ws_bytes))
    return set_error(DLM_E_INVAL, "%s: workspace of %zu bytes at %p, %llu needed (dlm_tabu_workspace_bytes)", fn,
                     workspace_bytes, workspace, (unsigned long long)P.ws_bytes);
  if (P.ws_bytes > 0 && (reinterpret_cast<uintptr_t>(workspace) & 255u))
    return set_error(DLM_E_INVAL, "%s: workspace must be 256-byte aligned", fn);
  const int n = g->n, k = p->k;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  TabuArgs a{g->row_ptr, g->col_idx, g->erow, colors, f_best, iters, stats, hash, trace, nullptr,
             make_key(p->seed), n, k, p->max_iters, p->ten_num, p->ten_den, p->ten_rand,
             p->ind_base, p->trace_cap};
  if (P.gtab_bytes > 0) a.gtab = ws;
  switch (P.table) {
    case DLM_TABLE_WAVE8: {
      int16_t* start = reinterpret_cast<int16_t*>(ws);
      unsigned char* slot_mem = ws + align256(P.start_bytes);
      const int64_t cells = (int64_t)pop * n;
      hipLaunchKernelGGL(copy_i16_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, colors, start,
                         cells);
      DLM_HIP(hipGetLastError());
      if ((rc = launch_w8(a, pop, P.acap, P.lds, s)) != DLM_OK) return rc;
      const Rerun rr{start, slot_mem, (int32_t)P.slots};
      return launch_tab<TabGlobal16>(a, pop, 256, P.lds_rr, s, &rr);
    }
    case DLM_TABLE_SPLIT8: {
      int16_t* start = reinterpret_cast<int16_t*>(ws + align256(P.gtab_bytes));
      unsigned char* slot_mem = ws + align256(P.gtab_bytes) + align256(P.start_bytes);
      const int64_t cells = (int64_t)pop * n;
      hipLaunchKernelGGL(copy_i16_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, colors, start,
                         cells);
      DLM_HIP(hipGetLastError());
      if ((rc = launch_tab<TabSplit8>(a, pop, P.block, P.lds, s)) != DLM_OK) return rc;
      const Rerun rr{start, slot_mem, (int32_t)P.slots};
      return launch_tab<TabGlobal16>(a, pop, P.block, P.lds_rr, s, &rr);
    }
    case DLM_TABLE_SPLIT16: return launch_tab<TabSplit16>(a, pop, P.block, P.lds, s);
    case DLM_TABLE_GLOBAL16: return launch_tab<TabGlobal16>(a, pop, P.block, P.lds, s);
    case DLM_TABLE_LDS32: return launch_tab<TabLds32>(a, pop, P.block, P.lds, s);
    default: return launch_tab<TabLds16>(a, pop, P.block, P.lds, s);
  }
}

// Fixed device scratch of the allocation-free entry point.  In host code the
// array's name is only a stand-in: its device address, one per GPU, comes
// from hipGetSymbolAddress on the first call on that device and is the only
// form host code hands to kernels.  Every call on a device shares the array.
constexpr uint64_t kStaticScratchBytes = DLM_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int static_scratch(const char* fn, void** out) {
  int dev = -1;
  DLM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(DLM_E_UNSUPPORTED, "%s: device %d >= %d", fn, dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_error(DLM_E_HIP, "%s: hipGetSymbolAddress gave a null scratch address", fn);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DLM_OK;
}

}  // namespace dlm

using namespace dlm;

extern "C" int dlm_tabu_workspace_bytes(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                                        size_t* bytes) {
  if (!bytes) return set_error(DLM_E_INVAL, "dlm_tabu_workspace_bytes: bytes is NULL");
  *bytes = 0;
  int rc = tabu_check("dlm_tabu_workspace_bytes", g, p, pop);
  if (rc != DLM_OK) return rc;
  TabuPlan P;
  if ((rc = tabu_plan("dlm_tabu_workspace_bytes", g, p, pop, P)) != DLM_OK) return rc;
  *bytes = (size_t)P.ws_bytes;
  return DLM_OK;
}

extern "C" int dlm_tabu_batch(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                              int16_t* colors, int32_t* f_best, int32_t* iters, int64_t* stats,
                              uint64_t* hash, int32_t* trace, void* workspace, size_t workspace_bytes,
                              void* stream) {
  const int rc = tabu_check("dlm_tabu_batch", g, p, pop);
  if (rc != DLM_OK) return rc;
  return tabu_run("dlm_tabu_batch", g, p, pop, colors, f_best, iters, stats, hash, trace, workspace,
                  workspace_bytes, (hipStream_t)stream, ~0ull);
}

extern "C" int dlm_tabu_batch_static(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                                     int16_t* colors, int32_t* f_best, int32_t* iters, int64_t* stats,
                                     uint64_t* hash, int32_t* trace, void* stream) {
  const char* fn = "dlm_tabu_batch_static";
  int rc = tabu_check(fn, g, p, pop);
  if (rc != DLM_OK) return rc;
  if (pop == 0) return DLM_OK;
  void* ws = nullptr;
  if ((rc = static_scratch(fn, &ws)) != DLM_OK) return rc;
  return tabu_run(fn, g, p, pop, colors, f_best, iters, stats, hash, trace, ws, (size_t)kStaticScratchBytes,
                  (hipStream_t)stream, kStaticScratchBytes);
}
