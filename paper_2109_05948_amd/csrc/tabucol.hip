// Population TabuCol for k-COL (Section 2.7 of the paper: TabuCol with the
// gamma table of its efficient implementation), one workgroup per individual.
//
// Per individual, in LDS (or device memory for tables too large for LDS):
//   tab[v*k + c]  gamma[v][c] (neighbours of v coloured c) and the tabu
//                 expiry of (v, c); LDS16 packs both into one 32-bit word
//                 (gamma low 16 bits, expiry relative to a rebased origin
//                 high 16 bits), LDS32 keeps two 32-bit words (absolute
//                 expiry)
//   cg[v]         colour of v (low 16) | gamma[v][col v] (high 16)
//   cmask         one bit per vertex: v is in conflict (gamma[v][col v] > 0)
//   conf[]        the conflicting vertices, rebuilt from cmask after a move
//
// One iteration:
//   scan      every thread takes candidates j = i*k + c (i-th conflicting
//             vertex, colour c) strided by the block size and keeps its best
//             admissible (delta, v, c) and how many tie with it;
//   reduce    DPP wave minimum, cross-wave minimum through LDS; if several
//             admissible moves share the minimum delta, the holders of those
//             moves hash them (Philox of (ind, t, v, c)) and a second
//             reduction picks the smallest (hash, v, c);
//   apply     wave 0 updates the colour, tabu expiry, the gamma rows of the
//             neighbours (CSR row of v* streamed from device memory), the
//             conflict mask and list, f and the lazily kept best colouring.
#include <algorithm>

#include "dlm_common.h"

namespace dlm {

constexpr int kBias = 32768;          // delta + kBias >= 0 for |delta| < 2^15
constexpr int kRebaseEvery = 16384;   // LDS16: expiry origin moves every 2^14 iterations

// ---------------------------------------------------------------------------
// Table storage policies.
struct TabLds16 {
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 4;
  uint32_t* w;
  __device__ static TabLds16 make(unsigned char* lds, uint32_t*, size_t) {
    return TabLds16{reinterpret_cast<uint32_t*>(lds)};
  }
  __device__ __forceinline__ void zero(int i) { w[i] = 0u; }
  __device__ __forceinline__ void add(int i, int d) { atomicAdd(&w[i], (uint32_t)d); }
  __device__ __forceinline__ uint32_t gamma(int i) const { return w[i] & 0xffffu; }
  __device__ __forceinline__ void read(int i, uint32_t& g, uint32_t& ex) const {
    const uint32_t x = w[i];
    g = x & 0xffffu;
    ex = x >> 16;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) {
    reinterpret_cast<uint16_t*>(w)[2 * i + 1] = (uint16_t)ex;
  }
  __device__ __forceinline__ void rebase(int i) {
    const uint32_t x = w[i];
    const uint32_t e = x >> 16;
    w[i] = (x & 0xffffu) | ((e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u) << 16);
  }
  __device__ __forceinline__ void sync() {}
};

struct TabLds32 {
  static constexpr bool kRebase = false;
  static constexpr int kLdsBytes = 8;
  uint32_t* w;  // w[2i] = gamma, w[2i+1] = absolute expiry
  __device__ static TabLds32 make(unsigned char* lds, uint32_t*, size_t) {
    return TabLds32{reinterpret_cast<uint32_t*>(lds)};
  }
  __device__ __forceinline__ void zero(int i) {
    w[2 * i] = 0u;
    w[2 * i + 1] = 0u;
  }
  __device__ __forceinline__ void add(int i, int d) { atomicAdd(&w[2 * i], (uint32_t)d); }
  __device__ __forceinline__ uint32_t gamma(int i) const { return w[2 * i]; }
  __device__ __forceinline__ void read(int i, uint32_t& g, uint32_t& ex) const {
    const uint2 x = reinterpret_cast<const uint2*>(w)[i];
    g = x.x;
    ex = x.y;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) { w[2 * i + 1] = ex; }
  __device__ __forceinline__ void rebase(int) {}
  __device__ __forceinline__ void sync() {}
};

// Packed 16-bit words in device memory.  Reads are device-coherent loads so
// that a wave sees the atomic updates made by another wave of its workgroup.
struct TabGlobal16 {
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 0;
  uint32_t* w;
  __device__ static TabGlobal16 make(unsigned char*, uint32_t* g, size_t off) {
    return TabGlobal16{g + off};
  }
  __device__ __forceinline__ uint32_t ld(int i) const {
    return __hip_atomic_load(&w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void zero(int i) {
    __hip_atomic_store(&w[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void add(int i, int d) {
    __hip_atomic_fetch_add(&w[i], (uint32_t)d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ uint32_t gamma(int i) const { return ld(i) & 0xffffu; }
  __device__ __forceinline__ void read(int i, uint32_t& g, uint32_t& ex) const {
    const uint32_t x = ld(i);
    g = x & 0xffffu;
    ex = x >> 16;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) {
    // only the high half changes; the low half of row v* is not touched by this move
    const uint32_t x = ld(i);
    __hip_atomic_store(&w[i], (x & 0xffffu) | (ex << 16), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void rebase(int i) {
    const uint32_t x = ld(i);
    const uint32_t e = x >> 16;
    __hip_atomic_store(&w[i], (x & 0xffffu) | ((e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u) << 16),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // complete this wave's table updates before the next workgroup barrier
  __device__ __forceinline__ void sync() { __threadfence(); }
};

// ---------------------------------------------------------------------------
struct TabuArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* erow;
  int16_t* colors;
  int32_t* f_best;
  int32_t* iters;
  int64_t* stats;
  uint64_t* hash;
  int32_t* trace;
  uint32_t* gtab;
  Key key;
  int32_t n, k, T, ten_num, ten_den, ten_rand, ind_base, trace_cap;
};

struct TabuLayout {
  uint64_t tab, cg, conf, cmask, red, redc, red2, sc, bytes;
};

__host__ __device__ inline TabuLayout tabu_layout(int n, int k, int nw, int entry_bytes) {
  TabuLayout L;
  uint64_t o = 0;
  L.tab = o;
  o += (((uint64_t)n * k * entry_bytes) + 15u) & ~15ull;
  L.cg = o;
  o += align16(4u * n);
  L.conf = o;
  o += align16(2u * n);
  L.cmask = o;
  o += align16(4u * ((n + 31) / 32));
  L.red = o;
  o += 16u * nw;
  L.redc = o;
  o += align16(8u * nw);
  L.red2 = o;
  o += 16u * nw;
  L.sc = o;
  o += 16;
  L.bytes = o;
  return L;
}

// Wave 0 rebuilds the list of conflicting vertices from the mask.  The order
// of the list is irrelevant: the chosen move is a total-order minimum.
__device__ __forceinline__ void build_conflict_list(const uint32_t* cmask, uint16_t* conf,
                                                    int32_t* count, int nwords, int lane) {
  if (lane == 0) *count = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int w = lane; w < nwords; w += kWave) {
    uint32_t m = cmask[w];
    if (m) {
      int pos = atomicAdd(count, __popc(m));
      while (m) {
        const int b = __ffs(m) - 1;
        m &= m - 1;
        conf[pos++] = (uint16_t)(w * 32 + b);
      }
    }
  }
}

template <int BLOCK, class Tab>
__global__ __launch_bounds__(BLOCK) void tabucol_kernel(TabuArgs a) {
  constexpr int NW = BLOCK / kWave;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int li = blockIdx.x;
  const uint32_t ind = (uint32_t)(a.ind_base + li);
  const int n = a.n, k = a.k, nk = n * k;
  const int nwords = (n + 31) >> 5;
  const TabuLayout L = tabu_layout(n, k, NW, Tab::kLdsBytes);
  Tab tab = Tab::make(smem + L.tab, a.gtab, (size_t)li * (size_t)nk);
  uint32_t* cg = reinterpret_cast<uint32_t*>(smem + L.cg);
  uint16_t* conf = reinterpret_cast<uint16_t*>(smem + L.conf);
  uint32_t* cmask = reinterpret_cast<uint32_t*>(smem + L.cmask);
  uint64_t* red = reinterpret_cast<uint64_t*>(smem + L.red);
  uint32_t* redc = reinterpret_cast<uint32_t*>(smem + L.redc);
  uint64_t* red2 = reinterpret_cast<uint64_t*>(smem + L.red2);
  int32_t* sc = reinterpret_cast<int32_t*>(smem + L.sc);
  int16_t* gcol = a.colors + (size_t)li * n;

  // 1. start colouring (rejected whole if a colour is outside [0, k)), empty table and mask
  int bad = 0;
  for (int v = tid; v < n; v += BLOCK) {
    const int c = gcol[v];
    bad |= (c < 0) | (c >= k);
    cg[v] = (uint32_t)(c & 0xffff);
  }
  if (__syncthreads_or(bad)) {
    if (tid == 0) {
      a.f_best[li] = -1;
      a.iters[li] = -1;
    }
    return;
  }
  for (int i = tid; i < nk; i += BLOCK) tab.zero(i);
  for (int w = tid; w < nwords; w += BLOCK) cmask[w] = 0u;
  tab.sync();
  __syncthreads();
  // 2. gamma from the CSR entries
  const int nnz = a.row_ptr[n];
  for (int e = tid; e < nnz; e += BLOCK) tab.add(a.erow[e] * k + (int)(cg[a.col_idx[e]] & 0xffffu), 1);
  tab.sync();
  __syncthreads();
  // 3. gamma of the current colour, conflict mask, f = sum / 2
  uint32_t fs = 0;
  for (int v = tid; v < n; v += BLOCK) {
    const uint32_t cv = cg[v];
    const uint32_t g = tab.gamma(v * k + (int)cv);
    cg[v] = cv | (g << 16);
    if (g) atomicOr(&cmask[v >> 5], 1u << (v & 31));
    fs += g;
  }
  fs = wave_sum_u32(fs);
  if (lane == 0) redc[wid] = fs;
  __syncthreads();
  int f = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) f += (int)redc[w];
  f >>= 1;
  if (wid == 0) build_conflict_list(cmask, conf, sc, nwords, lane);
  __syncthreads();
  int C = sc[0];

  int t = 0, f_best = f, base = 0;
  bool best_cur = true;
  // statistics and fingerprint live in wave 0
  uint64_t st_moves = 0, st_noops = 0, st_conf = 0, st_deg = 0, st_ties = 0, st_cap = 0;
  uint64_t fp = kFnvOffset;
  uint32_t Lreg = 0;
  const int i0 = tid / k, c0 = tid - (tid / k) * k, di = BLOCK / k, dc = BLOCK - (BLOCK / k) * k;

  while (t < a.T && f > 0) {
    if (Tab::kRebase && t - base == kRebaseEvery) {
      for (int i = tid; i < nk; i += BLOCK) tab.rebase(i);
      base += kRebaseEvery;
      tab.sync();
      __syncthreads();
    }
    const uint32_t trel = Tab::kRebase ? (uint32_t)(t - base) : (uint32_t)t;
    const int asp = f_best - f - 1;  // aspiration: delta <= asp  <=>  f + delta < f_best
    const int par = (t & 1) * NW;
    if (wid == 0 && (t & 63) == 0)
      Lreg = lemire(philox_w0(ind, (uint32_t)(t + lane), 0u, kDomTenure, a.key), (uint32_t)a.ten_rand);

    // ---- scan
    uint32_t bd = 0xffffffffu, bidx = 0xffffffffu, bcnt = 0, s0 = 0, s1 = 0;
    {
      int i = i0, c = c0;
      const int total = C * k;
      for (int j = tid; j < total; j += BLOCK) {
        const int v = conf[i];
        const uint32_t x = cg[v];
        if (c != (int)(x & 0xffffu)) {
          uint32_t g, ex;
          tab.read(v * k + c, g, ex);
          const int d = (int)g - (int)(x >> 16);
          if (ex <= trel || d <= asp) {
            const uint32_t bdv = (uint32_t)(d + kBias);
            const uint32_t idx = ((uint32_t)v << 16) | (uint32_t)c;
            if (bdv < bd) {
              bd = bdv;
              bidx = idx;
              bcnt = 1;
              s0 = idx;
            } else if (bdv == bd) {
              bidx = min(bidx, idx);
              if (bcnt == 1) s1 = idx;
              ++bcnt;
            }
          }
        }
        c += dc;
        i += di;
        if (c >= k) {
          c -= k;
          ++i;
        }
      }
    }
    // ---- reduce: minimum (delta, v, c) and the number of moves at that delta
    {
      const uint64_t wk = wave_min_u64(((uint64_t)bd << 32) | bidx);
      const uint32_t wcnt = wave_sum_u32(bd == (uint32_t)(wk >> 32) ? bcnt : 0u);
      if (lane == 0) {
        red[par + wid] = wk;
        redc[par + wid] = wcnt;
      }
    }
    __syncthreads();
    uint64_t gk = red[par];
#pragma unroll
    for (int w = 1; w < NW; ++w) gk = umin64(gk, red[par + w]);
    const uint32_t gbd = (uint32_t)(gk >> 32);
    uint32_t gcnt = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
      if ((uint32_t)(red[par + w] >> 32) == gbd) gcnt += redc[par + w];

    if (gbd == 0xffffffffu) {  // nothing admissible: no-op iteration
      if (wid == 0) {
        ++st_noops;
        st_conf += (uint64_t)C;
        fp = fnv_step(fp, 0xffffu, 0xffffu, f);
        if (lane == 0 && a.trace && t < a.trace_cap) {
          int32_t* tr = a.trace + ((size_t)li * a.trace_cap + t) * 2;
          tr[0] = -1;
          tr[1] = f;
        }
      }
      ++t;
      continue;
    }

    uint32_t win;
    if (gcnt == 1) {
      win = (uint32_t)gk;
    } else {
      // ties on delta: smallest (Philox word, v, c) among the tied moves
      uint64_t hk = ~0ull;
      if (bd == gbd) {
        auto hkey = [&](uint32_t idx) -> uint64_t {
          const uint32_t h = philox_w0(ind, (uint32_t)t, idx >> 16, idx & 0xffffu, a.key);
          return ((uint64_t)h << 32) | idx;
        };
        if (bcnt <= 2) {
          hk = hkey(s0);
          if (bcnt == 2) hk = umin64(hk, hkey(s1));
        } else {
          int i = i0, c = c0;
          const int total = C * k;
          const int dmin = (int)gbd - kBias;
          for (int j = tid; j < total; j += BLOCK) {
            const int v = conf[i];
            const uint32_t x = cg[v];
            if (c != (int)(x & 0xffffu)) {
              uint32_t g, ex;
              tab.read(v * k + c, g, ex);
              const int d = (int)g - (int)(x >> 16);
              if (d == dmin && (ex <= trel || d <= asp))
                hk = umin64(hk, hkey(((uint32_t)v << 16) | (uint32_t)c));
            }
            c += dc;
            i += di;
            if (c >= k) {
              c -= k;
              ++i;
            }
          }
        }
      }
      hk = wave_min_u64(hk);
      if (lane == 0) red2[par + wid] = hk;
      __syncthreads();
      uint64_t gh = red2[par];
#pragma unroll
      for (int w = 1; w < NW; ++w) gh = umin64(gh, red2[par + w]);
      win = (uint32_t)gh;
    }

    // ---- apply (wave 0)
    const int vs = (int)(win >> 16), cs = (int)(win & 0xffffu);
    const int fnew = f + ((int)gbd - kBias);
    const bool snap = best_cur && fnew >= f_best;  // leaving the best state: keep a copy
    if (wid == 0) {
      if (snap)
        for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffffu);
      const int old = (int)(cg[vs] & 0xffffu);
      const uint32_t Lt = readlane(Lreg, t & 63);
      int64_t ttf = (int64_t)a.ten_num * fnew / a.ten_den;
      const bool capped = ttf > kTenureCap;
      if (capped) ttf = kTenureCap;
      const int rs = a.row_ptr[vs], re = a.row_ptr[vs + 1];
      for (int e = rs + lane; e < re; e += kWave) {
        const int u = a.col_idx[e];
        const uint32_t xu = cg[u];
        const int cu = (int)(xu & 0xffffu);
        tab.add(u * k + old, -1);
        tab.add(u * k + cs, +1);
        if (cu == old) {
          cg[u] = xu - 0x10000u;
          if ((xu >> 16) == 1u) atomicAnd(&cmask[u >> 5], ~(1u << (u & 31)));
        } else if (cu == cs) {
          cg[u] = xu + 0x10000u;
          if ((xu >> 16) == 0u) atomicOr(&cmask[u >> 5], 1u << (u & 31));
        }
      }
      if (lane == 0) {
        tab.set_tabu(vs * k + old, trel + Lt + (uint32_t)ttf);
        const uint32_t gnew = tab.gamma(vs * k + cs);
        cg[vs] = (uint32_t)cs | (gnew << 16);
        if (gnew == 0u) atomicAnd(&cmask[vs >> 5], ~(1u << (vs & 31)));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      build_conflict_list(cmask, conf, sc, nwords, lane);
      ++st_moves;
      st_conf += (uint64_t)C;
      st_deg += (uint64_t)(re - rs);
      st_ties += gcnt > 1;
      st_cap += capped;
      fp = fnv_step(fp, (uint32_t)vs, (uint32_t)cs, fnew);
      if (lane == 0 && a.trace && t < a.trace_cap) {
        int32_t* tr = a.trace + ((size_t)li * a.trace_cap + t) * 2;
        tr[0] = vs | (cs << 16);
        tr[1] = fnew;
      }
      tab.sync();
    }
    f = fnew;
    if (f < f_best) {
      f_best = f;
      best_cur = true;
    } else if (snap) {
      best_cur = false;
    }
    ++t;
    __syncthreads();
    C = sc[0];
  }

  if (wid == 0) {
    if (best_cur)
      for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffffu);
    if (lane == 0) {
      a.f_best[li] = f_best;
      a.iters[li] = t;
      if (a.stats) {
        int64_t* s = a.stats + (size_t)li * DLM_NSTATS;
        s[0] = (int64_t)st_moves;
        s[1] = (int64_t)st_noops;
        s[2] = (int64_t)st_conf;
        s[3] = (int64_t)st_deg;
        s[4] = (int64_t)st_ties;
        s[5] = (int64_t)st_cap;
        s[6] = 0;
        s[7] = 0;
      }
      if (a.hash) a.hash[li] = fp;
    }
  }
}

template <int BLOCK, class Tab>
static int launch_block(const TabuArgs& a, int pop, size_t lds, hipStream_t s) {
  auto kern = tabucol_kernel<BLOCK, Tab>;
  DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(pop), dim3(BLOCK), lds, s, a);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

template <class Tab>
static int launch_tab(const TabuArgs& a, int pop, int block, size_t lds, hipStream_t s) {
  switch (block) {
    case 64: return launch_block<64, Tab>(a, pop, lds, s);
    case 128: return launch_block<128, Tab>(a, pop, lds, s);
    case 256: return launch_block<256, Tab>(a, pop, lds, s);
    case 512: return launch_block<512, Tab>(a, pop, lds, s);
    case 1024: return launch_block<1024, Tab>(a, pop, lds, s);
  }
  return set_error(DLM_E_INVAL, "dlm_tabu_batch: block=%d not in {64,128,256,512,1024}", block);
}

}  // namespace dlm

using namespace dlm;

extern "C" int dlm_tabu_batch(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                              int16_t* colors, int32_t* f_best, int32_t* iters, int64_t* stats,
                              uint64_t* hash, int32_t* trace, void* stream) {
  if (!g || !p) return set_error(DLM_E_INVAL, "dlm_tabu_batch: graph or params is NULL");
  if (pop < 0) return set_error(DLM_E_INVAL, "dlm_tabu_batch: pop < 0");
  if (p->k < 1 || p->k > 32767) return set_error(DLM_E_INVAL, "dlm_tabu_batch: k=%d outside [1, 32767]", p->k);
  if (p->max_iters < 0 || p->max_iters > (1 << 30))
    return set_error(DLM_E_INVAL, "dlm_tabu_batch: max_iters=%d outside [0, 2^30]", p->max_iters);
  if (p->ten_den <= 0 || p->ten_num < 0 || p->ten_num > 32767)
    return set_error(DLM_E_INVAL, "dlm_tabu_batch: tenure slope %d/%d invalid", p->ten_num, p->ten_den);
  if (p->ten_rand < 1 || p->ten_rand > 1024)
    return set_error(DLM_E_INVAL, "dlm_tabu_batch: ten_rand=%d outside [1, 1024]", p->ten_rand);
  if (p->ind_base < 0 || (int64_t)p->ind_base + pop > 0x7fffffffll)
    return set_error(DLM_E_INVAL, "dlm_tabu_batch: ind_base + pop exceeds 2^31");
  if (p->trace_cap < 0 || (p->trace_cap > 0 && !trace))
    return set_error(DLM_E_INVAL, "dlm_tabu_batch: trace_cap=%d needs a trace buffer", p->trace_cap);
  if (p->reserved != 0) return set_error(DLM_E_INVAL, "dlm_tabu_batch: reserved must be 0");
  if (pop == 0) return DLM_OK;
  if (!colors || !f_best || !iters) return set_error(DLM_E_INVAL, "dlm_tabu_batch: null output buffer");
  const int block = p->block ? p->block : 256;
  const int nw = block / kWave;
  const int n = g->n, k = p->k;
  const int64_t lds_max = device_lds_limit();
  int table = p->table;
  if (table == DLM_TABLE_AUTO)
    table = tabu_layout(n, k, nw, TabLds16::kLdsBytes).bytes <= (uint64_t)lds_max ? DLM_TABLE_LDS16
                                                                                  : DLM_TABLE_GLOBAL16;
  int eb = 0;
  switch (table) {
    case DLM_TABLE_LDS16: eb = TabLds16::kLdsBytes; break;
    case DLM_TABLE_LDS32: eb = TabLds32::kLdsBytes; break;
    case DLM_TABLE_GLOBAL16: eb = 0; break;
    default: return set_error(DLM_E_INVAL, "dlm_tabu_batch: unknown table %d", table);
  }
  const uint64_t lds = tabu_layout(n, k, nw, eb).bytes;
  if (lds > (uint64_t)lds_max)
    return set_error(DLM_E_UNSUPPORTED, "dlm_tabu_batch: %llu bytes of LDS needed, %lld available",
                     (unsigned long long)lds, (long long)lds_max);
  TabuArgs a{g->row_ptr, g->col_idx, g->erow, colors, f_best, iters, stats, hash, trace, nullptr,
             make_key(p->seed), n, k, p->max_iters, p->ten_num, p->ten_den, p->ten_rand,
             p->ind_base, p->trace_cap};
  hipStream_t s = (hipStream_t)stream;
  if (table == DLM_TABLE_GLOBAL16) {
    const size_t bytes = (size_t)pop * n * k * sizeof(uint32_t);
    DLM_HIP(hipMallocAsync((void**)&a.gtab, bytes, s));
    int rc = launch_tab<TabGlobal16>(a, pop, block, lds, s);
    hipError_t e = hipFreeAsync(a.gtab, s);
    if (rc != DLM_OK) return rc;
    DLM_HIP(e);
    return DLM_OK;
  }
  if (table == DLM_TABLE_LDS32) return launch_tab<TabLds32>(a, pop, block, lds, s);
  return launch_tab<TabLds16>(a, pop, block, lds, s);
}
