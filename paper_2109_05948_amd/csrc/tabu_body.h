// TabuCol search of one individual by one workgroup, shared by the
// single-graph batch kernel and the persistent multi-graph kernel.
#pragma once

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
  static constexpr int kGlobalBytes = 0;
  __device__ static TabLds16 make(unsigned char* lds, unsigned char*) {
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
  // four consecutive entries (i a multiple of 4: one 16-byte LDS read)
  __device__ __forceinline__ void read4(int i, uint32_t g[4], uint32_t ex[4]) const {
    const uint4 x = *reinterpret_cast<const uint4*>(w + i);
    g[0] = x.x & 0xffffu; ex[0] = x.x >> 16;
    g[1] = x.y & 0xffffu; ex[1] = x.y >> 16;
    g[2] = x.z & 0xffffu; ex[2] = x.z >> 16;
    g[3] = x.w & 0xffffu; ex[3] = x.w >> 16;
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
  static constexpr int kGlobalBytes = 0;
  __device__ static TabLds32 make(unsigned char* lds, unsigned char*) {
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
  __device__ __forceinline__ void read4(int i, uint32_t g[4], uint32_t ex[4]) const {
    const uint4 x = *reinterpret_cast<const uint4*>(w + 2 * i);
    const uint4 y = *reinterpret_cast<const uint4*>(w + 2 * i + 4);
    g[0] = x.x; ex[0] = x.y; g[1] = x.z; ex[1] = x.w;
    g[2] = y.x; ex[2] = y.y; g[3] = y.z; ex[3] = y.w;
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
  static constexpr int kGlobalBytes = 4;
  __device__ static TabGlobal16 make(unsigned char*, unsigned char* g) {
    return TabGlobal16{reinterpret_cast<uint32_t*>(g)};
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
  __device__ __forceinline__ void read4(int i, uint32_t g[4], uint32_t ex[4]) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t x = ld(i + q);
      g[q] = x & 0xffffu;
      ex[q] = x >> 16;
    }
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

// Split storage: gamma (16 bits) in LDS, tabu expiries (16 bits, relative
// to the rebased origin) in device memory.  Half the LDS of LDS16, so twice
// as many individuals fit on a CU; the expiry rows of the resident
// individuals stay in L2.  Expiries are read with device-coherent loads.
struct TabSplit16 {
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 2;
  static constexpr int kGlobalBytes = 2;
  uint16_t* g;   // LDS gamma
  uint16_t* tb;  // device tabu expiries
  __device__ static TabSplit16 make(unsigned char* lds, unsigned char* gm) {
    return TabSplit16{reinterpret_cast<uint16_t*>(lds), reinterpret_cast<uint16_t*>(gm)};
  }
  __device__ __forceinline__ void zero(int i) {
    g[i] = 0;
    tb[i] = 0;
  }
  __device__ __forceinline__ void add(int i, int d) {
    // 16-bit add inside the containing 32-bit LDS word; a decrement only
    // happens on a positive count, so no borrow crosses the halves
    const uint32_t inc = d > 0 ? 1u : 0xffffu;
    atomicAdd(reinterpret_cast<uint32_t*>(g) + (i >> 1), (i & 1) ? (inc << 16) : (d > 0 ? 1u : 0xffffffffu));
  }
  __device__ __forceinline__ uint32_t gamma(int i) const { return g[i]; }
  __device__ __forceinline__ uint32_t ldt(int i) const {
    const uint32_t w = __hip_atomic_load(reinterpret_cast<const uint32_t*>(tb) + (i >> 1), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return (i & 1) ? (w >> 16) : (w & 0xffffu);
  }
  __device__ __forceinline__ void read4(int i, uint32_t gg[4], uint32_t ex[4]) const {
    const uint2 x = *reinterpret_cast<const uint2*>(g + i);
    const uint64_t t = __hip_atomic_load(reinterpret_cast<const uint64_t*>(tb + i), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    gg[0] = x.x & 0xffffu; gg[1] = x.x >> 16; gg[2] = x.y & 0xffffu; gg[3] = x.y >> 16;
    ex[0] = (uint32_t)t & 0xffffu; ex[1] = (uint32_t)(t >> 16) & 0xffffu;
    ex[2] = (uint32_t)(t >> 32) & 0xffffu; ex[3] = (uint32_t)(t >> 48);
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) { tb[i] = (uint16_t)ex; }
  __device__ __forceinline__ void rebase(int i) {
    const uint32_t e = ldt(i);
    tb[i] = (uint16_t)(e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u);
  }
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
  unsigned char* gtab;  // device-memory table storage (global and split tiers)
  Key key;
  int32_t n, k, T, ten_num, ten_den, ten_rand, ind_base, trace_cap;
};

struct TabuLayout {
  uint64_t tab, cg, conf, cmask, rp, red, redc, red2, sc, bytes;
};

// Table rows are padded to a multiple of 4 colours so that a quad of
// candidates is one aligned 16-byte read.
__host__ __device__ constexpr int tab_stride(int k) { return (k + 3) & ~3; }

__host__ __device__ inline TabuLayout tabu_layout(int n, int k, int nw, int entry_bytes) {
  TabuLayout L;
  uint64_t o = 0;
  L.tab = o;
  o += (((uint64_t)n * tab_stride(k) * entry_bytes) + 15u) & ~15ull;
  L.cg = o;
  o += align16(4u * n);
  L.conf = o;
  o += align16(2u * n);
  L.cmask = o;
  o += align16(4u * ((n + 31) / 32));
  L.rp = o;
  o += align16(4u * (n + 1));
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

// One individual (row li of a.colors) searched by the calling workgroup.
// gtab: the device-memory part of this workgroup's table (global and split tiers).
template <int BLOCK, class Tab>
__device__ __forceinline__ void tabu_individual(const TabuArgs& a, int li, unsigned char* gtab,
                                                unsigned char* smem) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const uint32_t ind = (uint32_t)(a.ind_base + li);
  const int n = a.n, k = a.k, kp = tab_stride(k), nk = n * kp;
  const int nwords = (n + 31) >> 5;
  const TabuLayout L = tabu_layout(n, k, NW, Tab::kLdsBytes);
  Tab tab = Tab::make(smem + L.tab, gtab);
  uint32_t* cg = reinterpret_cast<uint32_t*>(smem + L.cg);
  uint16_t* conf = reinterpret_cast<uint16_t*>(smem + L.conf);
  uint32_t* cmask = reinterpret_cast<uint32_t*>(smem + L.cmask);
  uint64_t* red = reinterpret_cast<uint64_t*>(smem + L.red);
  uint32_t* redc = reinterpret_cast<uint32_t*>(smem + L.redc);
  uint64_t* red2 = reinterpret_cast<uint64_t*>(smem + L.red2);
  int32_t* sc = reinterpret_cast<int32_t*>(smem + L.sc);
  int32_t* rp = reinterpret_cast<int32_t*>(smem + L.rp);  // CSR row offsets, cached
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
  for (int v = tid; v <= n; v += BLOCK) rp[v] = a.row_ptr[v];
  tab.sync();
  __syncthreads();
  // 2. gamma from the CSR entries
  const int nnz = a.row_ptr[n];
  for (int e = tid; e < nnz; e += BLOCK) tab.add(a.erow[e] * kp + (int)(cg[a.col_idx[e]] & 0xffffu), 1);
  tab.sync();
  __syncthreads();
  // 3. gamma of the current colour, conflict mask, f = sum / 2
  uint32_t fs = 0;
  for (int v = tid; v < n; v += BLOCK) {
    const uint32_t cv = cg[v];
    const uint32_t g = tab.gamma(v * kp + (int)cv);
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
  // quads (i, q): the i-th conflicting vertex, colours 4q..4q+3; thread tid takes quads tid + s*BLOCK
  const int kq = kp >> 2;
  const int i0 = tid / kq, q0 = tid - (tid / kq) * kq, di = BLOCK / kq, dq = BLOCK - (BLOCK / kq) * kq;

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
    auto consider = [&](int v, int c, uint32_t x, uint32_t g, uint32_t ex) {
      const int d = (int)g - (int)(x >> 16);
      if (c < k && c != (int)(x & 0xffffu) && (ex <= trel || d <= asp)) {
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
    };
    auto step = [&](int& i, int& q) {
      q += dq;
      i += di;
      if (q >= kq) {
        q -= kq;
        ++i;
      }
    };
    {
      const int totq = C * kq;
      int i = i0, q = q0, j = tid;
      // two quads per round: their loads are independent and issue together
      for (; j + BLOCK < totq; j += 2 * BLOCK) {
        const int ia = i, qa = q;
        step(i, q);
        const int ib = i, qb = q;
        step(i, q);
        const int va = conf[ia], vb = conf[ib];
        const uint32_t xa = cg[va], xb = cg[vb];
        uint32_t ga[4], ea[4], gb[4], eb[4];
        tab.read4(va * kp + 4 * qa, ga, ea);
        tab.read4(vb * kp + 4 * qb, gb, eb);
#pragma unroll
        for (int r = 0; r < 4; ++r) consider(va, 4 * qa + r, xa, ga[r], ea[r]);
#pragma unroll
        for (int r = 0; r < 4; ++r) consider(vb, 4 * qb + r, xb, gb[r], eb[r]);
      }
      if (j < totq) {
        const int v = conf[i];
        const uint32_t x = cg[v];
        uint32_t g4[4], e4[4];
        tab.read4(v * kp + 4 * q, g4, e4);
#pragma unroll
        for (int r = 0; r < 4; ++r) consider(v, 4 * q + r, x, g4[r], e4[r]);
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
          const int totq = C * kq;
          const int dmin = (int)gbd - kBias;
          int i = i0, q = q0;
          for (int j = tid; j < totq; j += BLOCK) {
            const int v = conf[i];
            const uint32_t x = cg[v];
            uint32_t g4[4], e4[4];
            tab.read4(v * kp + 4 * q, g4, e4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int c = 4 * q + r;
              const int d = (int)g4[r] - (int)(x >> 16);
              if (c < k && c != (int)(x & 0xffffu) && d == dmin && (e4[r] <= trel || d <= asp))
                hk = umin64(hk, hkey(((uint32_t)v << 16) | (uint32_t)c));
            }
            step(i, q);
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
      const int rs = rp[vs], re = rp[vs + 1];
      auto update = [&](int u) {
        const uint32_t xu = cg[u];
        const int cu = (int)(xu & 0xffffu);
        tab.add(u * kp + old, -1);
        tab.add(u * kp + cs, +1);
        if (cu == old) {
          cg[u] = xu - 0x10000u;
          if ((xu >> 16) == 1u) atomicAnd(&cmask[u >> 5], ~(1u << (u & 31)));
        } else if (cu == cs) {
          cg[u] = xu + 0x10000u;
          if ((xu >> 16) == 0u) atomicOr(&cmask[u >> 5], 1u << (u & 31));
        }
      };
      // the first 8 x 64 neighbours: all loads issued before any is used
      constexpr int kPre = 8;
      int nb[kPre];
#pragma unroll
      for (int r = 0; r < kPre; ++r) {
        const int e = rs + lane + r * kWave;
        nb[r] = e < re ? a.col_idx[e] : -1;
      }
#pragma unroll
      for (int r = 0; r < kPre; ++r)
        if (nb[r] >= 0) update(nb[r]);
      for (int e = rs + kPre * kWave + lane; e < re; e += kWave) update(a.col_idx[e]);
      if (lane == 0) {
        tab.set_tabu(vs * kp + old, trel + Lt + (uint32_t)ttf);
        const uint32_t gnew = tab.gamma(vs * kp + cs);
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


}  // namespace dlm
