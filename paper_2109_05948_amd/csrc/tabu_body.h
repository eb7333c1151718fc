// TabuCol search of one individual by one workgroup, shared by the
// single-graph batch kernel and the persistent multi-graph kernel.
#pragma once

#include <algorithm>

#include "dlm_common.h"

namespace dlm {

constexpr int kBias = 32768;             // delta + kBias >= 0 for |delta| < 2^15
constexpr int kRebaseEvery = 16384;      // 16-bit expiries: the origin moves every 2^14 iterations
constexpr uint32_t kPadGamma = 0x7fffu;  // gamma stored in the padding colours k .. kp-1
constexpr uint32_t kNone = 0xffffffffu;  // no admissible candidate
constexpr int kStage = 64;               // tied moves a wave hashes in one staged pass
constexpr int kKeyRounds = 16384;        // rounds per lane that 16-bit candidate numbers cover

// Table encoding, common to every storage policy:
//  * the entry (v, col v) of a vertex's current colour holds the expiry
//    kInf, which no iteration reaches, so it is never admissible by tenure;
//    its delta is 0 and the aspiration needs f + delta < f_best <= f, so it
//    is never admissible at all;
//  * the padding colours c in [k, kp) hold a large gamma (kPadGamma, or
//    255 for byte gamma) and expiry kInf: delta >= 1, never admissible
//    either.
// The scan therefore needs no test on the colour of a candidate.  A vertex's
// old colour gets its real expiry when the vertex leaves it, the new colour
// gets kInf; the expiry an entry held while it was the current colour is
// never read (the move rule excludes c = col v).

// ---------------------------------------------------------------------------
// Table storage policies.  load4(i) fetches the four entries i..i+3 (i a
// multiple of 4) and eval4(raw, thr, g, fr) reports their gamma and "not
// tabu" (expiry <= trel, with thr = free_thr(trel)); the two halves are
// separate so that a thread can have several quads in flight.
struct TabLds16 {
  static constexpr bool kBounded = false;
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 4;
  static constexpr int kGlobalBytes = 0;
  static constexpr uint32_t kInf = 0xffffu;
  uint32_t* w;  // gamma low 16 bits, expiry (relative to the rebased origin) high 16 bits
  __device__ static TabLds16 make(unsigned char* lds, unsigned char*) {
    return TabLds16{reinterpret_cast<uint32_t*>(lds)};
  }
  __device__ __forceinline__ void init(int i, bool pad) { w[i] = pad ? (kPadGamma | (kInf << 16)) : 0u; }
  __device__ __forceinline__ void add(int i, int d) { atomicAdd(&w[i], (uint32_t)d); }
  __device__ __forceinline__ uint32_t gamma(int i) const { return w[i] & 0xffffu; }
  // expiry <= trel  <=>  the packed word <= (trel << 16) | 0xffff
  __device__ static __forceinline__ uint32_t free_thr(uint32_t trel) { return (trel << 16) | 0xffffu; }
  using Raw = uint4;
  __device__ __forceinline__ Raw load4(int i) const { return *reinterpret_cast<const uint4*>(w + i); }
  __device__ static __forceinline__ void eval4(const Raw& x, uint32_t thr, uint32_t g[4], bool fr[4]) {
    g[0] = x.x & 0xffffu; fr[0] = x.x <= thr;
    g[1] = x.y & 0xffffu; fr[1] = x.y <= thr;
    g[2] = x.z & 0xffffu; fr[2] = x.z <= thr;
    g[3] = x.w & 0xffffu; fr[3] = x.w <= thr;
  }
  __device__ static __forceinline__ void eval4h(const Raw& x, uint32_t thr, uint32_t gh[4], bool fr[4]) {
    gh[0] = x.x << 16; fr[0] = x.x <= thr;
    gh[1] = x.y << 16; fr[1] = x.y <= thr;
    gh[2] = x.z << 16; fr[2] = x.z <= thr;
    gh[3] = x.w << 16; fr[3] = x.w <= thr;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) {
    reinterpret_cast<uint16_t*>(w)[2 * i + 1] = (uint16_t)ex;
  }
  __device__ __forceinline__ void rebase(int i) {
    const uint32_t x = w[i];
    uint32_t e = x >> 16;
    if (e != kInf) e = e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u;
    w[i] = (x & 0xffffu) | (e << 16);
  }
};

struct TabLds32 {
  static constexpr bool kBounded = false;
  static constexpr bool kRebase = false;
  static constexpr int kLdsBytes = 8;
  static constexpr int kGlobalBytes = 0;
  static constexpr uint32_t kInf = 0xffffffffu;
  uint32_t* w;  // w[2i] = gamma, w[2i+1] = absolute expiry
  __device__ static TabLds32 make(unsigned char* lds, unsigned char*) {
    return TabLds32{reinterpret_cast<uint32_t*>(lds)};
  }
  __device__ __forceinline__ void init(int i, bool pad) {
    w[2 * i] = pad ? kPadGamma : 0u;
    w[2 * i + 1] = pad ? kInf : 0u;
  }
  __device__ __forceinline__ void add(int i, int d) { atomicAdd(&w[2 * i], (uint32_t)d); }
  __device__ __forceinline__ uint32_t gamma(int i) const { return w[2 * i]; }
  __device__ static __forceinline__ uint32_t free_thr(uint32_t trel) { return trel; }
  struct Raw {
    uint4 x, y;
  };
  __device__ __forceinline__ Raw load4(int i) const {
    return Raw{*reinterpret_cast<const uint4*>(w + 2 * i), *reinterpret_cast<const uint4*>(w + 2 * i + 4)};
  }
  __device__ static __forceinline__ void eval4(const Raw& r, uint32_t thr, uint32_t g[4], bool fr[4]) {
    g[0] = r.x.x; fr[0] = r.x.y <= thr; g[1] = r.x.z; fr[1] = r.x.w <= thr;
    g[2] = r.y.x; fr[2] = r.y.y <= thr; g[3] = r.y.z; fr[3] = r.y.w <= thr;
  }
  __device__ static __forceinline__ void eval4h(const Raw& r, uint32_t thr, uint32_t gh[4], bool fr[4]) {
    gh[0] = r.x.x << 16; fr[0] = r.x.y <= thr; gh[1] = r.x.z << 16; fr[1] = r.x.w <= thr;
    gh[2] = r.y.x << 16; fr[2] = r.y.y <= thr; gh[3] = r.y.z << 16; fr[3] = r.y.w <= thr;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) { w[2 * i + 1] = ex; }
  __device__ __forceinline__ void rebase(int) {}
};

// Packed 16-bit words in device memory.  Only the waves of one workgroup
// touch a table, and every read of an entry written by another wave comes
// after a workgroup barrier, so plain loads and stores and workgroup-scope
// atomics are enough (no device-scope fence, which would write back and
// invalidate L2).
struct TabGlobal16 {
  static constexpr bool kBounded = false;
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 0;
  static constexpr int kGlobalBytes = 4;
  static constexpr uint32_t kInf = 0xffffu;
  uint32_t* w;
  __device__ static TabGlobal16 make(unsigned char*, unsigned char* g) {
    return TabGlobal16{reinterpret_cast<uint32_t*>(g)};
  }
  __device__ __forceinline__ uint32_t ld(int i) const { return w[i]; }
  __device__ __forceinline__ void st(int i, uint32_t x) { w[i] = x; }
  __device__ __forceinline__ void init(int i, bool pad) { st(i, pad ? (kPadGamma | (kInf << 16)) : 0u); }
  __device__ __forceinline__ void add(int i, int d) {
    __hip_atomic_fetch_add(&w[i], (uint32_t)d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ __forceinline__ uint32_t gamma(int i) const { return ld(i) & 0xffffu; }
  __device__ static __forceinline__ uint32_t free_thr(uint32_t trel) { return (trel << 16) | 0xffffu; }
  using Raw = uint4;
  __device__ __forceinline__ Raw load4(int i) const { return *reinterpret_cast<const uint4*>(w + i); }
  __device__ static __forceinline__ void eval4(const Raw& x, uint32_t thr, uint32_t g[4], bool fr[4]) {
    g[0] = x.x & 0xffffu; fr[0] = x.x <= thr;
    g[1] = x.y & 0xffffu; fr[1] = x.y <= thr;
    g[2] = x.z & 0xffffu; fr[2] = x.z <= thr;
    g[3] = x.w & 0xffffu; fr[3] = x.w <= thr;
  }
  __device__ static __forceinline__ void eval4h(const Raw& x, uint32_t thr, uint32_t gh[4], bool fr[4]) {
    gh[0] = x.x << 16; fr[0] = x.x <= thr;
    gh[1] = x.y << 16; fr[1] = x.y <= thr;
    gh[2] = x.z << 16; fr[2] = x.z <= thr;
    gh[3] = x.w << 16; fr[3] = x.w <= thr;
  }
  // only the high half changes; the low half of row v* is not touched by this move
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) { st(i, (ld(i) & 0xffffu) | (ex << 16)); }
  __device__ __forceinline__ void rebase(int i) {
    const uint32_t x = ld(i);
    uint32_t e = x >> 16;
    if (e != kInf) e = e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u;
    st(i, (x & 0xffffu) | (e << 16));
  }
};

// Split storage: gamma (16 bits) in LDS, tabu expiries (16 bits, relative
// to the rebased origin) in device memory.  Half the LDS of LDS16, so twice
// as many individuals fit on a CU; the expiry rows of the resident
// individuals stay in L2.  As for the device table, plain accesses ordered by
// workgroup barriers suffice.
struct TabSplit16 {
  static constexpr bool kBounded = false;
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 2;
  static constexpr int kGlobalBytes = 2;
  static constexpr uint32_t kInf = 0xffffu;
  uint16_t* g;   // LDS gamma
  uint16_t* tb;  // device tabu expiries
  __device__ static TabSplit16 make(unsigned char* lds, unsigned char* gm) {
    return TabSplit16{reinterpret_cast<uint16_t*>(lds), reinterpret_cast<uint16_t*>(gm)};
  }
  __device__ __forceinline__ void init(int i, bool pad) {
    g[i] = (uint16_t)(pad ? kPadGamma : 0u);
    tb[i] = (uint16_t)(pad ? kInf : 0u);
  }
  __device__ __forceinline__ void add(int i, int d) {
    // 16-bit add inside the containing 32-bit LDS word; a decrement only
    // happens on a positive count, so no borrow crosses the halves
    const uint32_t inc = d > 0 ? 1u : 0xffffu;
    atomicAdd(reinterpret_cast<uint32_t*>(g) + (i >> 1), (i & 1) ? (inc << 16) : (d > 0 ? 1u : 0xffffffffu));
  }
  __device__ __forceinline__ uint32_t gamma(int i) const { return g[i]; }
  __device__ __forceinline__ uint32_t ldt(int i) const { return tb[i]; }
  __device__ static __forceinline__ uint32_t free_thr(uint32_t trel) { return trel; }
  struct Raw {
    uint2 x;
    uint64_t t;
  };
  __device__ __forceinline__ Raw load4(int i) const {
    return Raw{*reinterpret_cast<const uint2*>(g + i), *reinterpret_cast<const uint64_t*>(tb + i)};
  }
  __device__ static __forceinline__ void eval4(const Raw& r, uint32_t thr, uint32_t gg[4], bool fr[4]) {
    const uint2 x = r.x;
    const uint64_t t = r.t;
    gg[0] = x.x & 0xffffu; gg[1] = x.x >> 16; gg[2] = x.y & 0xffffu; gg[3] = x.y >> 16;
    fr[0] = ((uint32_t)t & 0xffffu) <= thr;
    fr[1] = ((uint32_t)(t >> 16) & 0xffffu) <= thr;
    fr[2] = ((uint32_t)(t >> 32) & 0xffffu) <= thr;
    fr[3] = (uint32_t)(t >> 48) <= thr;
  }
  __device__ static __forceinline__ void eval4h(const Raw& r, uint32_t thr, uint32_t gh[4], bool fr[4]) {
    const uint2 x = r.x;
    const uint64_t t = r.t;
    gh[0] = x.x << 16; gh[1] = x.x & 0xffff0000u; gh[2] = x.y << 16; gh[3] = x.y & 0xffff0000u;
    fr[0] = ((uint32_t)t & 0xffffu) <= thr;
    fr[1] = ((uint32_t)(t >> 16) & 0xffffu) <= thr;
    fr[2] = ((uint32_t)(t >> 32) & 0xffffu) <= thr;
    fr[3] = (uint32_t)(t >> 48) <= thr;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) { tb[i] = (uint16_t)ex; }
  __device__ __forceinline__ void rebase(int i) {
    uint32_t e = ldt(i);
    if (e == kInf) return;
    tb[i] = (uint16_t)(e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u);
  }
};


// Byte gamma in LDS, tabu expiries (16 bits) in device memory: a quarter of
// the LDS of LDS16.  Exact while every colour class has at most 255
// vertices (gamma[v][c] never exceeds the size of class c); the search body
// keeps the class sizes and gives up on an individual (iters = -2) before a
// move would break the bound, and the caller reruns it from its start
// colouring with 16-bit gamma.
struct TabSplit8 {
  static constexpr bool kBounded = true;
  static constexpr bool kRebase = true;
  static constexpr int kLdsBytes = 1;
  static constexpr int kGlobalBytes = 2;
  static constexpr uint32_t kInf = 0xffffu;
  static constexpr uint32_t kPad = 0xffu;  // padding gamma: delta >= 1, never admissible
  uint8_t* g;    // LDS gamma
  uint16_t* tb;  // device tabu expiries
  __device__ static TabSplit8 make(unsigned char* lds, unsigned char* gm) {
    return TabSplit8{reinterpret_cast<uint8_t*>(lds), reinterpret_cast<uint16_t*>(gm)};
  }
  __device__ __forceinline__ void init(int i, bool pad) {
    g[i] = (uint8_t)(pad ? kPad : 0u);
    tb[i] = (uint16_t)(pad ? kInf : 0u);
  }
  __device__ __forceinline__ void add(int i, int d) {
    // byte add inside the containing 32-bit word: a decrement only happens on
    // a positive count and an increment never reaches 256, so no carry or
    // borrow leaves the byte
    const uint32_t one = 1u << (8 * (i & 3));
    atomicAdd(reinterpret_cast<uint32_t*>(g) + (i >> 2), d > 0 ? one : 0u - one);
  }
  __device__ __forceinline__ uint32_t gamma(int i) const { return g[i]; }
  __device__ static __forceinline__ uint32_t free_thr(uint32_t trel) { return trel; }
  struct Raw {
    uint32_t x;
    uint64_t t;
  };
  __device__ __forceinline__ Raw load4(int i) const {
    return Raw{*reinterpret_cast<const uint32_t*>(g + i), *reinterpret_cast<const uint64_t*>(tb + i)};
  }
  __device__ static __forceinline__ void eval4(const Raw& r, uint32_t thr, uint32_t gg[4], bool fr[4]) {
    const uint32_t x = r.x;
    const uint64_t t = r.t;
    gg[0] = x & 0xffu; gg[1] = (x >> 8) & 0xffu; gg[2] = (x >> 16) & 0xffu; gg[3] = x >> 24;
    fr[0] = ((uint32_t)t & 0xffffu) <= thr;
    fr[1] = ((uint32_t)(t >> 16) & 0xffffu) <= thr;
    fr[2] = ((uint32_t)(t >> 32) & 0xffffu) <= thr;
    fr[3] = (uint32_t)(t >> 48) <= thr;
  }
  __device__ static __forceinline__ void eval4h(const Raw& r, uint32_t thr, uint32_t gh[4], bool fr[4]) {
    const uint32_t x = r.x;
    const uint64_t t = r.t;
    // byte c of x into bits 16..23, zeros elsewhere (selector byte 0x0c reads as 0): one v_perm_b32 each
#pragma unroll
    for (int c = 0; c < 4; ++c) gh[c] = __builtin_amdgcn_perm(x, x, 0x0c000c0cu | ((uint32_t)c << 16));
    fr[0] = ((uint32_t)t & 0xffffu) <= thr;
    fr[1] = ((uint32_t)(t >> 16) & 0xffffu) <= thr;
    fr[2] = ((uint32_t)(t >> 32) & 0xffffu) <= thr;
    fr[3] = (uint32_t)(t >> 48) <= thr;
  }
  __device__ __forceinline__ void set_tabu(int i, uint32_t ex) { tb[i] = (uint16_t)ex; }
  __device__ __forceinline__ void rebase(int i) {
    const uint32_t e = tb[i];
    if (e == kInf) return;
    tb[i] = (uint16_t)(e > (uint32_t)kRebaseEvery ? e - kRebaseEvery : 0u);
  }
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
  uint64_t tab, cg, list, pos, red, stage, csize, sc, bytes;
  int32_t cap;      // conflict-list capacity (entries)
  int32_t len_max;  // longest list a move may start from (rebuilt beyond it)
};

// Table rows are padded to a multiple of 4 colours so that a quad of
// candidates is one aligned 16-byte read.  Row n is all padding: conflict
// list entries that no longer name a conflicting vertex point at it.
__host__ __device__ constexpr int tab_stride(int k) { return (k + 3) & ~3; }
__host__ __device__ constexpr uint64_t tab_entries(int n, int k) { return (uint64_t)(n + 1) * tab_stride(k); }

__host__ __device__ inline TabuLayout tabu_layout(int n, int k, int nw, int entry_bytes) {
  TabuLayout L;
  uint64_t o = 0;
  L.tab = o;
  o += ((tab_entries(n, k) * entry_bytes) + 15u) & ~15ull;
  L.cg = o;
  o += align16(4u * (n + 1));  // cg[n] = 0 belongs to the all-padding row
  // a move appends at most the members of one colour class: at most 255 of
  // them with byte gamma (the class bound), at most n otherwise
  const int max_insert = entry_bytes == 1 ? (n < 255 ? n : 255) : n;
  L.cap = n + 32 + max_insert < 65535 ? n + 32 + max_insert : 65535;  // 16-bit positions
  L.len_max = L.cap - max_insert;
  L.list = o;
  o += align16(2u * L.cap);
  L.pos = o;
  o += align16(2u * n);
  L.red = o;
  o += 2u * 16u * nw;
  L.stage = o;
  o += (uint64_t)nw * 4u * (kStage + 4);
  L.csize = o;
  o += align16(4u * tab_stride(k));
  L.sc = o;
  o += 16;
  L.bytes = o;
  return L;
}

constexpr uint16_t kNoPos = 0xffffu;

// Wave 0 rebuilds the conflict list from cg (cg[v] = col v | gamma[v][col v] << 16):
// the conflicting vertices in vertex order, pos[v] = index of v in the list
// or kNoPos.  Returns the list length.
__device__ __forceinline__ int build_conflict_list(const uint32_t* cg, uint16_t* list, uint16_t* pos, int n,
                                                   int lane) {
  int base = 0;
  for (int v0 = 0; v0 < n; v0 += 4 * kWave) {
    uint32_t x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = v0 + r * kWave + lane;
      x[r] = v < n ? cg[v] : 0u;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = v0 + r * kWave + lane;
      const bool cf = x[r] >= 0x10000u;
      const uint64_t m = __ballot(cf);
      const int p = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      if (cf) list[p] = (uint16_t)v;
      if (v < n) pos[v] = cf ? (uint16_t)p : kNoPos;
      base += __popcll(m);
    }
  }
  return base;
}

// Slots for the active lanes of a wave whose pred is true: one LDS atomic
// per wave on *counter; returns counter's old value + the lane's rank.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred, int lane) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0;
  const int leader = __builtin_ctzll(m);
  uint32_t b = 0;
  if (lane == leader) b = atomicAdd(counter, (uint32_t)__popcll(m));
  b = readlane(b, leader);
  return b + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A copy of a uniform device-memory pointer in scalar registers of its own,
// so that the argument block it came from (loaded as one 16-register tuple)
// can die; typed as a global-address-space pointer so accesses stay global
// (not flat) instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> own_sgpr(T* p) {
  uint64_t x = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(x));
  return (gptr<T>)x;
}

// One individual (row li of a.colors) searched by the calling workgroup.
// gtab: the device-memory part of this workgroup's table (global and split tiers).
//
// The conflict list holds one live entry (the vertex) per conflicting vertex
// and tombstones (n, the all-padding row, whose cg word is 0) for vertices
// that stopped conflicting; a move tombstones and appends in place, and the
// list is rebuilt when tombstones pass a quarter of it.  The chosen move is a
// minimum over a set, so list order is free.
template <int BLOCK, class Tab>
__device__ __forceinline__ void tabu_individual(const TabuArgs& a, int li, unsigned char* gtab,
                                                unsigned char* smem) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const uint32_t ind = (uint32_t)(a.ind_base + li);
  const int n = a.n, k = a.k, kp = tab_stride(k), nk = (int)tab_entries(n, k);
  // the fields the iteration loop needs, as separate values (the argument
  // block as a whole would otherwise be kept in, and spilled from, scalar registers)
  const gptr<const int32_t> col_idx = own_sgpr(a.col_idx);
  const gptr<int32_t> trace = own_sgpr(a.trace);
  const int trace_cap = a.trace_cap, T = a.T;
  const Key key = a.key;
  const uint32_t ten_num = (uint32_t)a.ten_num, ten_den = (uint32_t)a.ten_den, ten_rand = (uint32_t)a.ten_rand;
  const uint32_t den_inv = 0xffffffffu / ten_den;
  const TabuLayout L = tabu_layout(n, k, NW, Tab::kLdsBytes);
  Tab tab = Tab::make(smem + L.tab, gtab);
  uint32_t* cg = reinterpret_cast<uint32_t*>(smem + L.cg);
  uint16_t* list = reinterpret_cast<uint16_t*>(smem + L.list);
  uint16_t* pos = reinterpret_cast<uint16_t*>(smem + L.pos);
  uint4* red = reinterpret_cast<uint4*>(smem + L.red);
  uint32_t* stage = reinterpret_cast<uint32_t*>(smem + L.stage);  // per wave: kStage tied moves + a counter
  uint32_t* csize = reinterpret_cast<uint32_t*>(smem + L.csize);  // class sizes (byte gamma only)
  uint32_t* sc = reinterpret_cast<uint32_t*>(smem + L.sc);  // [0] list length, [1] tombstones, [2..3] best delta
                                                            // published so far (by iteration parity)
  int16_t* gcol = a.colors + (size_t)li * n;
  const uint16_t kTomb = (uint16_t)n;
  // CSR row offsets through the scalar cache (read-only for the whole launch)
  const __attribute__((address_space(4))) int32_t* row_c =
      (const __attribute__((address_space(4))) int32_t*)a.row_ptr;

  auto rebuild = [&]() {
    if (wid == 0) {
      const int c = build_conflict_list(cg, list, pos, n, lane);
      if (lane == 0) {
        sc[0] = (uint32_t)c;
        sc[1] = 0u;
      }
    }
    __syncthreads();
  };

  // 1. start colouring (rejected whole if a colour is outside [0, k)), empty table
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
  for (int i = tid; i < nk; i += BLOCK) tab.init(i, i >= n * kp || i - (i / kp) * kp >= k);
  if (tid == 0) {
    cg[n] = 0u;
    sc[2] = kNone;
    sc[3] = kNone;
  }
  if (Tab::kBounded)
    for (int c = tid; c < kp; c += BLOCK) csize[c] = 0u;
  __syncthreads();
  // 2. gamma from the CSR entries (and the class sizes)
  const int nnz = a.row_ptr[n];
  if (Tab::kBounded) {
    for (int v = tid; v < n; v += BLOCK) atomicAdd(&csize[cg[v] & 0xffffu], 1u);
    __syncthreads();
    int big = 0;
    for (int c = tid; c < k; c += BLOCK) big |= csize[c] > 255u;
    if (__syncthreads_or(big)) {  // a class too large for byte gamma: left to the 16-bit rerun
      if (tid == 0) a.iters[li] = -2;
      return;
    }
  }
  for (int e = tid; e < nnz; e += BLOCK) tab.add(a.erow[e] * kp + (int)(cg[a.col_idx[e]] & 0xffffu), 1);
  __syncthreads();
  // 3. gamma of the current colour, its expiry kInf, f = sum / 2
  uint32_t fs = 0;
  for (int v = tid; v < n; v += BLOCK) {
    const uint32_t cv = cg[v];
    const uint32_t g = tab.gamma(v * kp + (int)cv);
    tab.set_tabu(v * kp + (int)cv, Tab::kInf);
    cg[v] = cv | (g << 16);
    fs += g;
  }
  fs = wave_sum_u32(fs);
  if (lane == 0) red[wid].x = fs;
  __syncthreads();
  int f = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) f += (int)red[w].x;
  f >>= 1;
  rebuild();  // its barrier also retires the reads of red above

  int t = 0, f_best = f, base = 0;
  bool best_cur = true;
  // statistics and fingerprint live in lane 0 of wave 0 (vector registers:
  // the scalar file is the scarce one); moves = t - no-ops
  uint64_t st_conf = 0, st_deg = 0, fp = kFnvOffset;
  uint32_t st_noops = 0, st_ties = 0, st_cap = 0;
  uint32_t Lreg = 0;
  // quads (i, q): list entry i, colours 4q..4q+3; thread tid takes quads tid + s*BLOCK
  const int kq = kp >> 2;
  const int i0 = tid / kq, q0 = tid - (tid / kq) * kq, di = BLOCK / kq, dq = BLOCK - (BLOCK / kq) * kq;
  const uint32_t kq_inv = 0xffffffffu / (uint32_t)kq;  // quotient by kq: one __umulhi and one correction
  auto step = [&](int& i, int& q) {
    q += dq;
    i += di;
    if (q >= kq) {
      q -= kq;
      ++i;
    }
  };

  while (t < T && f > 0) {
    int len = (int)sc[0], dead = (int)sc[1];
    if (4 * dead > len || len > L.len_max) {  // compact (every thread read sc before this barrier)
      __syncthreads();
      rebuild();
      len = (int)sc[0];
      dead = 0;
    }
    const int C = len - dead;  // conflicting vertices
    if (Tab::kRebase && t - base == kRebaseEvery) {
      for (int i = tid; i < nk; i += BLOCK) tab.rebase(i);
      base += kRebaseEvery;
      __syncthreads();
    }
    const uint32_t trel = Tab::kRebase ? (uint32_t)(t - base) : (uint32_t)t;
    const uint32_t thr = Tab::free_thr(trel);
    // aspiration: f + delta < f_best  <=>  delta + kBias <= f_best - f - 1 + kBias
    const int aspb = f_best - f - 1 + kBias;
    const int par = (t & 1) * NW;
    if (wid == 0 && (t & 63) == 0)
      Lreg = lemire(philox_w0(ind, (uint32_t)(t + lane), 0u, kDomTenure, key), ten_rand);

    // ---- scan.  Quad j (list entry j / kq, colours 4 (j % kq) .. +3) belongs
    // to thread j % BLOCK, which reaches it in its round j / BLOCK.
    const int totq = len * kq;
    uint32_t wbd;
    bool live;
    uint64_t hk = ~0ull;
    uint32_t wcnt = 0u;  // moves of this wave at its best delta
    uint32_t* stg = stage + wid * (kStage + 4);
    // publish the wave's best delta; a wave beaten by an earlier one cannot
    // hold the chosen move and skips the hashing
    auto publish = [&](uint32_t w) {
      bool lv = w != kNone;
      if (lv) {
        uint32_t prev = 0u;
        if (lane == 0) prev = atomicMin(&sc[2 + (t & 1)], w);
        lv = readlane(prev, 0) >= w;
      }
      return lv;
    };
    auto hkey = [&](uint32_t idx) -> uint64_t {
      const uint32_t h = philox_w0(ind, (uint32_t)t, idx >> 16, idx & 0xffffu, key);
      return ((uint64_t)h << 32) | idx;
    };
    // The moves tied at the wave's best delta are hashed before the
    // cross-wave step, so one barrier settles the iteration.  They are first
    // gathered in LDS so that one Philox evaluation per lane covers up to
    // kStage of them.
    auto hash_staged = [&](uint32_t total) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (uint32_t c0 = 0; c0 < total; c0 += kWave)
        if (c0 + lane < total) hk = umin64(hk, hkey(stg[c0 + lane]));
    };
    if (totq <= kKeyRounds * BLOCK) {
      // Candidate keys: biased delta << 16 | (4 * round + r), r the colour
      // within the quad.  A key names one candidate of the lane and orders
      // the candidates by delta; each lane keeps its three smallest
      // admissible keys (a v_min and two v_med3 per candidate).
      const uint32_t aspk = aspb >= 0 ? ((uint32_t)aspb + 1u) << 16 : 0u;  // key < aspk <=> biased delta <= aspb
      uint32_t m1 = kNone, m2 = kNone, m3 = kNone;
      auto keys = [&](const typename Tab::Raw& raw, uint32_t e, uint32_t r4, auto&& fn) {
        uint32_t g4[4];
        bool f4[4];
        Tab::eval4h(raw, thr, g4, f4);
        uint32_t x = (((uint32_t)kBias - (e >> 16)) << 16) + r4;
        asm("" : "+v"(x));  // one offset per quad: each key is then a single v_add3_u32
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t kk = g4[r] + x + (uint32_t)r;
          fn(r, kk, f4[r] | (kk < aspk));
        }
      };
      auto keep = [&](int, uint32_t kk, bool adm) {
        const uint32_t y = adm ? kk : kNone;
        m3 = umed3(m2, y, m3);
        m2 = umed3(m1, y, m2);
        m1 = min(m1, y);
      };
      {
        int i = i0, q = q0, j = tid;
        uint32_t r4 = 0;
        // two quads per round: their loads are independent and issue together
        for (; j + BLOCK < totq; j += 2 * BLOCK, r4 += 8) {
          const int ia = i, qa = q;
          step(i, q);
          const int ib = i, qb = q;
          step(i, q);
          const uint32_t va = list[ia], vb = list[ib];
          const typename Tab::Raw ra = tab.load4((int)__umul24(va, (uint32_t)kp) + 4 * qa);
          const typename Tab::Raw rb = tab.load4((int)__umul24(vb, (uint32_t)kp) + 4 * qb);
          const uint32_t ea = cg[va], eb = cg[vb];
          keys(ra, ea, r4, keep);
          keys(rb, eb, r4 + 4, keep);
        }
        if (j < totq) {
          const uint32_t v = list[i];
          keys(tab.load4((int)__umul24(v, (uint32_t)kp) + 4 * q), cg[v], r4, keep);
        }
      }
      const uint32_t wmin = wave_min_u32(m1);
      wbd = wmin == kNone ? kNone : wmin >> 16;
      live = publish(wbd);
      if (live) {
        // a lane with one or two ties names them from its keys; a lane with
        // three or more lists all of its ties by a rescan of its quads
        auto move_of = [&](uint32_t kk) {  // key of this lane -> move (v << 16) | c
          const uint32_t jj = (uint32_t)tid + ((kk & 0xffffu) >> 2) * (uint32_t)BLOCK;
          uint32_t ii = __umulhi(jj, kq_inv), qq = jj - ii * (uint32_t)kq;
          if (qq >= (uint32_t)kq) {
            qq -= (uint32_t)kq;
            ++ii;
          }
          return ((uint32_t)list[ii] << 16) | (4u * qq + (kk & 3u));
        };
        const bool R = (m3 >> 16) == wbd;
        const bool A = !R && (m1 >> 16) == wbd, B = !R && (m2 >> 16) == wbd;
        const uint32_t xa = A ? move_of(m1) : 0u, xb = B ? move_of(m2) : 0u;
        const uint64_t mA = __ballot(A), mB = __ballot(B), mR = __ballot(R);
        const uint32_t nA = (uint32_t)__popcll(mA);
        uint32_t total = nA + (uint32_t)__popcll(mB);
        if (A) stg[lane_rank(mA)] = xa;
        if (B && nA + lane_rank(mB) < (uint32_t)kStage) stg[nA + lane_rank(mB)] = xb;
        // every tie of the lanes in R, round by round over the wave's quads
        auto rescan = [&](auto&& fn) {
          int i = i0, q = q0;
          for (int j0 = wid * kWave; j0 < totq; j0 += BLOCK) {  // uniform over the wave
            bool tie[4] = {false, false, false, false};
            uint32_t mv = 0u;
            if (R && j0 + lane < totq) {
              const uint32_t v = list[i];
              mv = (v << 16) | (uint32_t)(4 * q);
              keys(tab.load4((int)__umul24(v, (uint32_t)kp) + 4 * q), cg[v], 0u,
                   [&](int r, uint32_t kk, bool adm) { tie[r] = adm && (kk >> 16) == wbd; });
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) fn(tie[r], mv + (uint32_t)r);
            step(i, q);
          }
        };
        if (mR != 0)
          rescan([&](bool tie, uint32_t mv) {
            const uint64_t m = __ballot(tie);
            const uint32_t p = total + lane_rank(m);
            if (tie && p < (uint32_t)kStage) stg[p] = mv;
            total += (uint32_t)__popcll(m);
          });
        wcnt = total;
        if (total <= (uint32_t)kStage) {
          hash_staged(total);
        } else {
          // too many ties to stage: every lane hashes its own
          if (A) hk = hkey(xa);
          if (B) hk = umin64(hk, hkey(xb));
          if (mR != 0)
            rescan([&](bool tie, uint32_t mv) {
              if (tie) hk = umin64(hk, hkey(mv));
            });
        }
      }
    } else {
      // More rounds than 16-bit candidate numbers cover: each lane keeps its
      // best biased delta, the count of candidates at it and the first two
      // (move index (v << 16) | c).
      uint32_t bd = kNone, cnt = 0, s0 = 0, s1 = 0;
      auto consider = [&](uint32_t idx, uint32_t g, bool fr, uint32_t boff) {
        const uint32_t bdv = g + boff;  // gamma[v][c] - gamma[v][col v] + kBias
        const uint32_t b = (fr || (int)bdv <= aspb) ? bdv : kNone;
        const bool lt = b < bd, eq = b == bd;
        s1 = (eq && cnt == 1u) ? idx : s1;
        cnt = lt ? 1u : cnt + (eq ? 1u : 0u);
        s0 = lt ? idx : s0;
        bd = lt ? b : bd;
      };
      auto do_quad = [&](int i, int q, auto&& fn) {
        const uint32_t v = list[i];
        uint32_t g4[4];
        bool f4[4];
        Tab::eval4(tab.load4((int)__umul24(v, (uint32_t)kp) + 4 * q), thr, g4, f4);
        const uint32_t boff = (uint32_t)kBias - (cg[v] >> 16);
        const uint32_t idx = (v << 16) | (uint32_t)(4 * q);
#pragma unroll
        for (int r = 0; r < 4; ++r) fn(idx + r, g4[r], f4[r], boff);
      };
      {
        int i = i0, q = q0;
        for (int j = tid; j < totq; j += BLOCK) {
          do_quad(i, q, consider);
          step(i, q);
        }
      }
      wbd = wave_min_u32(bd);
      live = publish(wbd);
      if (live) {
        auto is_tie = [&](uint32_t g, bool fr, uint32_t boff) {
          const uint32_t bdv = g + boff;
          return (fr || (int)bdv <= aspb) && bdv == wbd;
        };
        const bool tie = bd == wbd;
        const bool A = tie && cnt <= 2u, B = tie && cnt == 2u, R = tie && cnt > 2u;
        const uint64_t mA = __ballot(A), mB = __ballot(B);
        const uint32_t nR = wave_sum_u32(R ? cnt : 0u);
        const uint32_t nA = (uint32_t)__popcll(mA), nB = (uint32_t)__popcll(mB);
        const uint32_t total = nA + nB + nR;
        wcnt = total;
        if (total <= (uint32_t)kStage) {
          uint32_t* rctr = stg + kStage;
          if (lane == 0) *rctr = nA + nB;
          if (A) stg[lane_rank(mA)] = s0;
          if (B) stg[nA + lane_rank(mB)] = s1;
          if (R) {
            uint32_t p = atomicAdd(rctr, cnt);
            int i = i0, q = q0;
            for (int j = tid; j < totq; j += BLOCK) {
              do_quad(i, q, [&](uint32_t idx, uint32_t g, bool fr, uint32_t boff) {
                if (is_tie(g, fr, boff)) stg[p++] = idx;
              });
              step(i, q);
            }
          }
          hash_staged(total);
        } else {
          // too many ties to stage: every lane hashes its own
          if (A) hk = hkey(s0);
          if (B) hk = umin64(hk, hkey(s1));
          if (R) {
            int i = i0, q = q0;
            for (int j = tid; j < totq; j += BLOCK) {
              do_quad(i, q, [&](uint32_t idx, uint32_t g, bool fr, uint32_t boff) {
                if (is_tie(g, fr, boff)) hk = umin64(hk, hkey(idx));
              });
              step(i, q);
            }
          }
        }
      }
    }
    {
      const uint64_t whk = live ? wave_min_u64(hk) : ~0ull;
      // colour of this wave's chosen vertex, read while no wave writes cg,
      // and (byte gamma) whether the move would grow a class past 255
      const uint32_t wold = live ? (cg[(uint32_t)whk >> 16] & 0xffffu) : 0u;
      const uint32_t ovf = Tab::kBounded && live && csize[(uint32_t)whk & 0xffffu] >= 255u ? 1u : 0u;
      if (lane == 0)
        red[par + wid] = make_uint4((wbd & 0xffffu) | (wold << 16) | (ovf << 31), wcnt, (uint32_t)whk,
                                    (uint32_t)(whk >> 32));
    }
    __syncthreads();
    // every wave has published: the slot is free again for iteration t + 2
    if (tid == 0) sc[2 + (t & 1)] = kNone;
    // cross-wave: smallest (delta, hash, v, c); tie count over the waves at
    // that delta.  The slots are uniform: fold them in scalar registers.
    auto rfl = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); };
    uint32_t bx, bz, bw, gcnt;
    {
      const uint4 e0 = red[par];
      bx = rfl(e0.x); gcnt = rfl(e0.y); bz = rfl(e0.z); bw = rfl(e0.w);
    }
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const uint4 e = red[par + w];
      const uint32_t ex = rfl(e.x), ey = rfl(e.y), ez = rfl(e.z), ew = rfl(e.w);
      const uint32_t eb = ex & 0xffffu, bb = bx & 0xffffu;
      const bool hless = ew < bw || (ew == bw && ez < bz);
      gcnt = eb < bb ? ey : (eb == bb ? gcnt + ey : gcnt);
      const bool take = eb < bb || (eb == bb && hless);
      bx = take ? ex : bx;
      bz = take ? ez : bz;
      bw = take ? ew : bw;
    }
    const uint32_t gbd = bx & 0xffffu;

    if (gbd == 0xffffu) {  // nothing admissible: no-op iteration
      if (wid == 0 && lane == 0) {
        ++st_noops;
        st_conf += (uint64_t)C;
        fp = fnv_step(fp, 0xffffu, 0xffffu, f);
        if (trace && t < trace_cap) {
          gptr<int32_t> tr = trace + ((size_t)li * trace_cap + t) * 2;
          tr[0] = -1;
          tr[1] = f;
        }
      }
      ++t;
      continue;
    }

    if (Tab::kBounded && (bx >> 31)) {  // left to the 16-bit rerun
      if (tid == 0) a.iters[li] = -2;
      return;
    }
    // ---- apply: every thread takes a share of the neighbours of v*
    const uint32_t win = bz;
    const int vs = (int)(win >> 16), cs = (int)(win & 0xffffu), old = (int)((bx >> 16) & 0x7fffu);
    const int fnew = f + ((int)gbd - kBias);
    const bool snap = best_cur && fnew >= f_best;  // leaving the best state: keep a copy
    const int rs = row_c[vs], re = row_c[vs + 1];
    if (wid == 0 && snap)
      for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffffu);
    {
      // neighbour u: gamma[u][old] - 1, gamma[u][c*] + 1; if u has colour old
      // or c*, its own gamma and its conflict-list entry follow
      auto update = [&](int u, bool live) {
        uint32_t xu = 0, gu = 0;
        bool lo = false, hi = false;
        if (live) {
          xu = cg[u];
          const uint32_t cu = xu & 0xffffu;
          gu = xu >> 16;
          tab.add(u * kp + old, -1);
          tab.add(u * kp + cs, +1);
          lo = cu == (uint32_t)old;
          hi = cu == (uint32_t)cs;
          cg[u] = xu - (lo ? 0x10000u : 0u) + (hi ? 0x10000u : 0u);
          if (lo && gu == 1u) {
            list[pos[u]] = kTomb;
            pos[u] = kNoPos;
          }
        }
        const bool ins = hi && gu == 0u;
        const uint32_t p = wave_append(&sc[0], ins, lane);
        if (ins) {
          list[p] = (uint16_t)u;
          pos[u] = (uint16_t)p;
        }
        (void)wave_append(&sc[1], lo && gu == 1u, lane);
      };
      // the first kPre * BLOCK neighbours: all loads issued before any is used
      constexpr int kPre = BLOCK >= 256 ? 2 : 4;
      int nb[kPre];
#pragma unroll
      for (int r = 0; r < kPre; ++r) {
        const int e = rs + tid + r * BLOCK;
        nb[r] = e < re ? col_idx[e] : -1;
      }
      // v*'s own state, by wave 0 while the row loads are in flight.  None of
      // it touches what the neighbour updates touch: they change rows u != v*
      // of the table, cg[u], pos[u] and other list slots (the shared
      // tombstone count is an atomic); the snapshot above was taken first.
      if (wid == 0) {
        const uint32_t Lt = readlane(Lreg, t & 63);
        if (lane == 0) {
          // tenure term floor(num * f / den), capped; the product fits 32 bits in
          // practice, and then the quotient is a multiply by the reciprocal
          // 0xffffffff / den (low by at most 2) and two corrections
          const uint64_t prod = (uint64_t)ten_num * (uint32_t)fnew;
          uint32_t ttf;
          if (prod <= 0xffffffffull) {
            const uint32_t x = (uint32_t)prod;
            ttf = __umulhi(x, den_inv);
            uint32_t rem = x - ttf * ten_den;
            if (rem >= ten_den) {
              rem -= ten_den;
              ++ttf;
            }
            if (rem >= ten_den) ++ttf;
          } else {
            ttf = (uint32_t)std::min<uint64_t>(prod / ten_den, kTenureCap + 1);
          }
          const bool capped = ttf > (uint32_t)kTenureCap;
          if (capped) ttf = kTenureCap;
          tab.set_tabu(vs * kp + old, trel + Lt + ttf);
          tab.set_tabu(vs * kp + cs, Tab::kInf);
          const uint32_t gnew = tab.gamma(vs * kp + cs);
          cg[vs] = (uint32_t)cs | (gnew << 16);
          if (Tab::kBounded) {
            csize[old] -= 1u;
            csize[cs] += 1u;
          }
          if (gnew == 0u) {
            list[pos[vs]] = kTomb;
            pos[vs] = kNoPos;
            atomicAdd(&sc[1], 1u);
          }
          if (trace && t < trace_cap) {
            gptr<int32_t> tr = trace + ((size_t)li * trace_cap + t) * 2;
            tr[0] = vs | (cs << 16);
            tr[1] = fnew;
          }
          st_conf += (uint64_t)C;
          st_deg += (uint64_t)(re - rs);
          st_ties += gcnt > 1u;
          st_cap += capped;
          fp = fnv_step(fp, (uint32_t)vs, (uint32_t)cs, fnew);
        }
      }
#pragma unroll
      for (int r = 0; r < kPre; ++r)
        if (rs + r * BLOCK < re) update(nb[r], nb[r] >= 0);  // uniform per round: ballots see the whole wave
      for (int e0 = rs + kPre * BLOCK; e0 < re; e0 += BLOCK) {
        const int e = e0 + tid;
        update(e < re ? col_idx[e] : 0, e < re);
      }
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
  }

  if (wid == 0) {
    if (best_cur)
      for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffffu);
    if (lane == 0) {
      a.f_best[li] = f_best;
      a.iters[li] = t;
      if (a.stats) {
        int64_t* s = a.stats + (size_t)li * DLM_NSTATS;
        s[0] = (int64_t)(t - (int)st_noops);
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
