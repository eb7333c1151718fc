// TabuCol with one wavefront per individual (the WAVE8 table tier).
//
// Per individual, all in LDS:
//   tab[v*kp + c]  one byte: gamma[v][c] in bits 0..6, a flag in bit 7.  The
//                  flag is set exactly when c is v's current colour, c is a
//                  padding colour (c >= k), or the pair (v, c) is tabu.  A
//                  byte without the flag is therefore a move that no tenure
//                  forbids, and the smallest such byte of a row is the row's
//                  best non-tabu move.
//   act[]          the tabu pairs: ((v*kp + c) << 15) | (expiry mod 2^15).
//                  Only about 0.6 f + 5 of them are live at a time, so they
//                  are walked one by one after every move: an entry whose
//                  expiry arrives clears its flag, the others are checked
//                  for aspiration (f + delta < f_best).
//   cg[v]          colour (bits 0..7) | gamma[v][col v] (bits 8..14) |
//                  "listed" (bit 15)
//   list           the listed vertices: every conflicting vertex once, plus
//                  vertices that stopped conflicting ("stale", rebuilt away
//                  when they cost a scan round)
//   rowkey[i]      best biased delta of list entry i (scans of several rounds)
//   stage          tied moves waiting for their Philox hash
//   csize          colour class sizes (gamma <= class size <= 127 keeps bit 7
//                  free; a run that would pass it gives up with iters = -2
//                  and is rerun with the 16-bit device table)
//
// One iteration, with no workgroup barrier (the wave owns the individual):
//   scan   lane i takes list entry i (64 per round) and reads its row: the
//          smallest non-flagged byte in three VALU per four colours (two
//          packed 16-bit minima over the byte pairs);
//   min    DPP minimum of the rows' and the aspiring tabu pairs' biased
//          deltas;
//   ties   the rows at the minimum are read again, 64 / W rows at a time
//          (W lanes per row), and their bytes equal to the target value
//          staged; tabu pairs at the minimum come from the list;
//   hash   one Philox evaluation per lane over the staged moves, DPP
//          minimum of (hash, v, c);
//   apply  the CSR row of v* from device memory, one neighbour per lane:
//          two byte adds in its row, its cg word, list membership; v*'s flag,
//          class sizes, the new tabu pair;
//   list   expiries of the next iteration and its aspiration candidates.
#pragma once

#include "tabu_body.h"

namespace dlm {

constexpr uint32_t kW8Flag = 0x80u;
constexpr uint32_t kW8ClassMax = 127u;
constexpr uint32_t kW8None = 255u;        // biased delta (delta + 128) of "no admissible move"
constexpr int kW8Stage = 320;             // staged ties: < 64 left over + at most 256 from one pass
constexpr uint32_t kW8ExpMask = 0x7fffu;  // expiries are kept modulo 2^15
constexpr uint32_t kW8NoKey = 0xffffffffu;

struct W8Layout {
  uint32_t tab, cg, list, rowkey, stage, csize, sink, act, bytes;
};

// LDS of one individual with room for acap tabu pairs.  A row read covers
// up to KQ dwords; reads past the last row land in the arrays that follow
// the table (the stage alone is larger than any such overrun).
__host__ __device__ inline W8Layout w8_layout(int n, int k, int acap) {
  const uint32_t kp = (uint32_t)tab_stride(k);
  W8Layout L;
  uint32_t o = 0;
  L.tab = o;
  o += align16((uint32_t)(n + 1) * kp);
  L.cg = o;
  o += align16(2u * (uint32_t)(n + 1));
  L.list = o;
  o += align16(2u * (uint32_t)n);
  L.rowkey = o;
  o += align16((uint32_t)n);
  L.stage = o;
  o += 4u * kW8Stage;
  L.csize = o;
  o += align16(2u * kp);
  L.sink = o;  // lanes with nothing to store or add aim here (no branch around them)
  o += 16;
  L.act = o;
  o += 4u * (uint32_t)acap;
  L.bytes = o;
  return L;
}

// dwords per row bucket of the scan (rows of 9 to 15 and 17 to 23 dwords
// are launched at their exact width)
__host__ __device__ constexpr int w8_bucket(int k) {
  const int kq = tab_stride(k) >> 2;
  return kq <= 8 ? 8 : kq <= 16 ? 16 : kq <= 24 ? 24 : kq <= 32 ? 32 : kq <= 64 ? 64 : 0;
}

typedef unsigned short w8_u16x2 __attribute__((ext_vector_type(2)));

// per 16-bit half minimum (one v_pk_min_u16)
__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b) {
  const w8_u16x2 x = __builtin_bit_cast(w8_u16x2, a), y = __builtin_bit_cast(w8_u16x2, b);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(x, y));
}

// Orders the wave's LDS accesses around it in the compiler's view; the LDS
// itself serves one wave's instructions in issue order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a uniform 32-bit value in a scalar register of its own (see own_sgpr)
__device__ __forceinline__ uint32_t own_u32(uint32_t x) {
  asm volatile("" : "+s"(x));
  return x;
}

// The twenty Philox4x32-10 round keys (the seed's two words bumped by the
// Weyl constants), computed once and held in vector registers: in scalar
// registers, the scarce file here, they would spill, and recomputing them
// per call costs twenty scalar adds.
struct W8RoundKeys {
  uint32_t k[20];
};

__device__ __forceinline__ uint32_t to_vgpr(uint32_t x) {
  uint32_t y;
  asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
  return y;
}

__device__ __forceinline__ W8RoundKeys w8_round_keys(Key key) {
  W8RoundKeys rk;
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    rk.k[2 * r] = to_vgpr(k0);
    rk.k[2 * r + 1] = to_vgpr(k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return rk;
}

// Philox4x32-10 word 0 (the same function as philox_w0) from precomputed round keys
__device__ __forceinline__ uint32_t philox_w0_rk(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                 const W8RoundKeys& rk) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ rk.k[2 * r], y2 = (uint32_t)(p0 >> 32) ^ x3 ^ rk.k[2 * r + 1];
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
  }
  return x0;
}

__device__ __forceinline__ uint32_t rfl(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// The conflicting vertices in vertex order; sets "listed" on exactly those.
// Returns the list length.
__device__ __forceinline__ int w8_build_list(uint16_t* cg, uint16_t* list, int n, int lane) {
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
      const bool cf = ((x[r] >> 8) & 0x7fu) != 0u;
      const uint64_t m = __ballot(cf);
      if (v < n) {
        const uint32_t y = (x[r] & 0x7fffu) | (cf ? 0x8000u : 0u);
        if (y != x[r]) cg[v] = (uint16_t)y;
      }
      if (cf) list[base + (int)lane_rank(m)] = (uint16_t)v;
      base += __popcll(m);
    }
  }
  return base;
}

// Drops the stale entries (vertices no longer conflicting) from the list in
// place and clears their "listed" bit.  Returns the new length.
__device__ __forceinline__ int w8_compact_list(uint16_t* cg, uint16_t* list, int len, int lane) {
  int base = 0;
  for (int i0 = 0; i0 < len; i0 += kWave) {
    const int i = i0 + lane;
    const uint32_t v = i < len ? (uint32_t)list[i] : 0u;
    const uint32_t x = i < len ? (uint32_t)cg[v] : 0u;
    const bool keep = ((x >> 8) & 0x7fu) != 0u;
    if (i < len && !keep) cg[v] = (uint16_t)(x & 0x7fffu);
    const uint64_t m = __ballot(keep);
    if (keep) list[base + (int)lane_rank(m)] = (uint16_t)v;  // base <= i0: entries are read before they are overwritten
    base += __popcll(m);
  }
  return base;
}

// One individual (row li of a.colors) searched by the calling wavefront.
// KQ: dwords read per row, kp / 4 <= KQ (the exact width for rows of 9 to 15
// and 17 to 23 dwords, else the bucket of w8_bucket); acap: tabu pairs the
// LDS holds.
template <int KQ>
__device__ __forceinline__ void tabu_w8_individual(const TabuArgs& a, int li, int acap, unsigned char* smem) {
  // a bucket (8, 16, 24, 32, 64 dwords) masks what it reads past the row; any
  // other KQ is the exact row width (kq == KQ): nothing to mask
  constexpr bool bucket = KQ == 8 || KQ == 16 || KQ == 24 || KQ == 32 || KQ == 64;
  constexpr int KQ_LO = !bucket ? KQ : KQ == 8 ? 0 : KQ == 16 ? 8 : KQ == 24 ? 16 : KQ == 32 ? 24 : 32;
  const int lane = threadIdx.x;
  // every field the search needs, as a value of its own: the argument block
  // as a whole (about 30 scalar registers) would otherwise stay live in, and
  // spill from, scalar registers
  const uint32_t ind = own_u32((uint32_t)(a.ind_base + li));
  const int n = (int)own_u32((uint32_t)a.n), k = (int)own_u32((uint32_t)a.k);
  const uint32_t kp = (uint32_t)tab_stride(k), kq = kp >> 2;
  const gptr<const int32_t> col_idx = own_sgpr(a.col_idx);
  const gptr<int32_t> trace = own_sgpr(a.trace);
  const gptr<int32_t> iters_out = own_sgpr(a.iters + li);
  const gptr<int32_t> f_best_out = own_sgpr(a.f_best + li);
  const gptr<int64_t> stats_out = own_sgpr(a.stats ? a.stats + (size_t)li * DLM_NSTATS : nullptr);
  const gptr<uint64_t> hash_out = own_sgpr(a.hash ? a.hash + li : nullptr);
  const int trace_cap = (int)own_u32((uint32_t)a.trace_cap), T = (int)own_u32((uint32_t)a.T);
  const Key key{own_u32(a.key.k0), own_u32(a.key.k1)};
  const uint32_t ten_num = own_u32((uint32_t)a.ten_num), ten_den = own_u32((uint32_t)a.ten_den);
  const uint32_t ten_rand = own_u32((uint32_t)a.ten_rand);
  const uint32_t den_inv = 0xffffffffu / ten_den;
  // ceil(2^32 / kp): v = umulhi(v*kp + c, kp_inv) is exact for v*kp + c < 2^17
  const uint32_t kp_inv = (uint32_t)((0x100000000ull + kp - 1u) / kp);
  const W8Layout L = w8_layout(n, k, acap);
  uint8_t* tab = smem + L.tab;
  uint32_t* tabw = reinterpret_cast<uint32_t*>(smem + L.tab);
  uint16_t* cg = reinterpret_cast<uint16_t*>(smem + L.cg);
  uint16_t* list = reinterpret_cast<uint16_t*>(smem + L.list);
  uint8_t* rowkey = smem + L.rowkey;
  uint32_t* stage = reinterpret_cast<uint32_t*>(smem + L.stage);
  uint32_t* csw = reinterpret_cast<uint32_t*>(smem + L.csize);  // class sizes, two 16-bit counts per word
  uint32_t* act = reinterpret_cast<uint32_t*>(smem + L.act);
  uint32_t* sink = reinterpret_cast<uint32_t*>(smem + L.sink);
  const gptr<int16_t> gcol = own_sgpr(a.colors + (size_t)li * n);
  const gptr<const int32_t> erow = own_sgpr(a.erow);
  const __attribute__((address_space(4))) int32_t* row_c =
      (const __attribute__((address_space(4))) int32_t*)(const int32_t*)own_sgpr(a.row_ptr);
  // tie pass: LPR lanes per row (two dwords each), rpp rows per pass; this
  // lane's row within a pass and its dword pair
  const int lpr = (int)((kq + 1u) >> 1), rpp = kWave / lpr;
  const int lrow = lane / lpr, lj = lane - lrow * lpr;
  auto csize = [&](uint32_t c) { return (csw[c >> 1] >> (16u * (c & 1u))) & 0xffffu; };
  auto give_up = [&]() {
    if (lane == 0) *iters_out = -2;
  };

  // 1. start colouring (rejected whole if a colour is outside [0, k)), padded table, class sizes
  int bad = 0;
  for (int v = lane; v < n; v += kWave) {
    const int c = gcol[v];
    bad |= (c < 0) | (c >= k);
    cg[v] = (uint16_t)(c & 0xff);
  }
  if (__ballot(bad)) {
    if (lane == 0) {
      *f_best_out = -1;
      *iters_out = -1;
    }
    return;
  }
  for (int i = lane; i < (int)(kp >> 1); i += kWave) csw[i] = 0u;
  {
    const int words = (n + 1) * (int)kq;
    for (int i = lane; i < words; i += kWave) {
      const int v = i / (int)kq, q = i - v * (int)kq;
      uint32_t w = 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (v == n || 4 * q + b >= k) w |= 0xffu << (8 * b);
      tabw[i] = w;
    }
  }
  if (lane == 0) cg[n] = 0;
  wave_sync();
  for (int v = lane; v < n; v += kWave) {
    const uint32_t c = cg[v];
    atomicAdd(&csw[c >> 1], 1u << (16u * (c & 1u)));
  }
  wave_sync();
  {
    int big = 0;
    for (int c = lane; c < k; c += kWave) big |= csize((uint32_t)c) > kW8ClassMax;
    if (__ballot(big)) {
      give_up();
      return;
    }
  }
  // 2. gamma from the CSR entries
  const int nnz = row_c[n];
  for (int e = lane; e < nnz; e += kWave) {
    const uint32_t u = (uint32_t)col_idx[e], v = (uint32_t)erow[e];
    const uint32_t c = cg[u];
    atomicAdd(&tabw[v * kq + (c >> 2)], 1u << (8u * (c & 3u)));
  }
  wave_sync();
  // 3. the current colour's gamma into cg, its flag set; f = sum / 2
  uint32_t fs = 0;
  for (int v = lane; v < n; v += kWave) {
    const uint32_t c = cg[v];
    const uint32_t g = tab[(uint32_t)v * kp + c];
    atomicOr(&tabw[(uint32_t)v * kq + (c >> 2)], kW8Flag << (8u * (c & 3u)));
    cg[v] = (uint16_t)(c | (g << 8));
    fs += g;
  }
  int f = (int)(wave_sum_u32(fs) >> 1);
  wave_sync();
  int len = w8_build_list(cg, list, n, lane);
  int C = len;  // conflicting vertices, as the last scan counted them

  int t = 0, f_best = f, A = 0;
  bool best_cur = true;
  uint32_t asp = kW8None;  // this lane's best biased delta among aspiring tabu pairs
  // statistics and fingerprint accumulate in lane 0 (vector registers, by
  // select rather than branch: the scalar file is the scarce one); moves = t - no-ops
  uint64_t st_conf = 0, st_deg = 0, fp = kFnvOffset;
  uint32_t st_noops = 0, st_ties = 0, st_cap = 0;
  const bool l0 = lane == 0;
  uint32_t Lreg = 0;
  uint16_t* sink16 = reinterpret_cast<uint16_t*>(sink);
  const W8RoundKeys rk = w8_round_keys(key);

  while (t < T && f > 0) {
    if (((len + 63) >> 6) > ((C + 64) >> 6)) {  // stale entries cost a scan round: compact
      wave_sync();
      len = w8_compact_list(cg, list, len, lane);
      wave_sync();
    }
    if ((t & 63) == 0) Lreg = lemire(philox_w0_rk(ind, (uint32_t)(t + lane), 0u, kDomTenure, rk), ten_rand);

    // ---- scan: list entry (r << 6) + lane in round r
    const int rounds = (len + 63) >> 6;
    uint32_t best = kW8None, dlast = kW8None, vlast = (uint32_t)n, glast = 0u;
    C = 0;
    for (int r = 0; r < rounds; ++r) {
      const int i = (r << 6) + lane;
      const uint32_t v = i < len ? (uint32_t)list[i] : (uint32_t)n;
      const uint32_t g = ((uint32_t)cg[v] >> 8) & 0x7fu;
      C += __popcll(__ballot(g != 0u));
      const uint32_t* row = tabw + __umul24(v, kq);
      uint32_t w[KQ];
#pragma unroll
      for (int q = 0; q < KQ; ++q) w[q] = row[q];
      // bytes 0, 2 of each dword as the high bytes of the 16-bit halves of
      // w << 8, bytes 1, 3 as those of w itself: the packed minima's high
      // bytes are the smallest bytes
      uint32_t ml = 0xffffffffu, mh = 0xffffffffu;
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const uint32_t x = (q >= KQ_LO && q >= (int)kq) ? 0xffffffffu : w[q];
        ml = pk_min_u16(ml, x << 8);
        mh = pk_min_u16(mh, x);
      }
      const uint32_t m = min(min(ml & 0xffffu, ml >> 16), min(mh & 0xffffu, mh >> 16)) >> 8;
      const uint32_t d = (g != 0u && m < kW8Flag) ? m + 128u - g : kW8None;
      if (rounds > 1) *(i < len ? rowkey + i : reinterpret_cast<uint8_t*>(sink)) = (uint8_t)d;
      best = min(best, d);
      dlast = d;
      vlast = v;
      glast = g;
    }
    const uint32_t dstar = wave_min_u32(min(best, asp));
    uint32_t key_star = kW8NoKey;  // the tabu pair a move onto a tabu colour consumes

    if (dstar == kW8None) {  // nothing admissible: no-op iteration
      st_noops += l0 ? 1u : 0u;
      st_conf += l0 ? (uint64_t)C : 0ull;
      fp = l0 ? fnv_step(fp, 0xffffu, 0xffffu, f) : fp;
      if (trace && t < trace_cap && lane == 0) {
        gptr<int32_t> tr = trace + ((size_t)li * trace_cap + t) * 2;
        tr[0] = -1;
        tr[1] = f;
      }
    } else {
      // ---- every admissible move at dstar, hashed where it is found
      // The rows at dstar are gathered into slots ((v << 8) | the byte value
      // their best move has) and read again LPR lanes per row, two dwords
      // per lane; tabu pairs at dstar come from the list.  Each lane hashes
      // its own tied moves (Philox of (ind, t, v, c)) and keeps the smallest
      // (hash, v, c).
      uint64_t hk = ~0ull;
      uint32_t seen = 0;  // tied moves met so far, counted up to 2
      // mask: bit 8 b + 7 set for a tie at colour c0 + b
      auto hash_in = [&](uint64_t mask, uint32_t v, uint32_t c0) {
        const uint64_t any = __ballot(mask != 0ull);
        seen += (uint32_t)__popcll(any) + (__ballot(__popcll(mask) > 1) != 0ull ? 1u : 0u);
        if (any == 0ull) return;
        while (__ballot(mask != 0ull)) {
          if (mask) {
            const uint32_t c = c0 + ((uint32_t)__builtin_ctzll(mask) >> 3);
            mask &= mask - 1ull;
            hk = umin64(hk, ((uint64_t)philox_w0_rk(ind, (uint32_t)t, v, c, rk) << 32) | (v << 16) | c);
          }
        }
      };
      auto scan_slots = [&](int cnt) {
        for (int p0 = 0; p0 < cnt; p0 += rpp) {
          const int ri = p0 + lrow;
          const bool ok = lrow < rpp && ri < cnt;
          const uint32_t e0 = stage[ri];  // past cnt: harmless, replaced below
          const uint32_t e = ok ? e0 : ((uint32_t)n << 8);  // row n: all padding, matches nothing
          const uint32_t v = e >> 8, tv = (e & 0xffu) * 0x01010101u;
          const uint32_t* rw = tabw + v * kq + 2u * (uint32_t)lj;
          const uint32_t x0 = rw[0];
          const uint32_t x1 = 2 * lj + 1 < (int)kq ? rw[1] : 0xffffffffu;
          // bit 7 of byte b set iff byte b equals the target (a target is
          // below 128, so flagged and padding bytes never match)
          const uint32_t y0 = x0 ^ tv, y1 = x1 ^ tv;
          const uint32_t z0 = ~(((y0 & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y0) & 0x80808080u;
          const uint32_t z1 = ~(((y1 & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y1) & 0x80808080u;
          hash_in((uint64_t)z0 | ((uint64_t)z1 << 32), v, 8u * (uint32_t)lj);
        }
      };
      {
        int nrows = 0;
        for (int r = 0; r < rounds; ++r) {
          const bool lastr = r == rounds - 1;
          const int i = (r << 6) + lane;
          uint32_t vr = vlast, gr = glast, dr = dlast;
          if (!lastr) {
            dr = i < len ? (uint32_t)rowkey[i] : kW8None;
            vr = i < len ? (uint32_t)list[i] : (uint32_t)n;
            gr = ((uint32_t)cg[vr] >> 8) & 0x7fu;
          }
          const bool tied = dr == dstar;
          const uint64_t M = __ballot(tied);
          *(tied ? stage + nrows + (int)lane_rank(M) : sink) = (vr << 8) | (dstar + gr - 128u);
          nrows += __popcll(M);
          if (nrows > kW8Stage - kWave || lastr) {
            wave_sync();
            scan_slots(nrows);
            nrows = 0;
            wave_sync();
          }
        }
      }
      if (__ballot(asp == dstar)) {
        // tabu pairs at dstar: all of them aspire (the test depends on delta only)
        for (int i0 = 0; i0 < A; i0 += kWave) {
          const int i = i0 + lane;
          const uint32_t kk = i < A ? act[i] >> 15 : 0u;
          const uint32_t v = __umulhi(kk, kp_inv), c = kk - v * kp;
          const uint32_t g = ((uint32_t)cg[v] >> 8) & 0x7fu;
          const bool hit = i < A && g != 0u && (uint32_t)(tab[kk] & 0x7fu) + 128u - g == dstar;
          hash_in(hit ? 0x80ull : 0ull, v, c);
        }
      }
      const uint32_t win = (uint32_t)wave_min_u64(hk);

      // ---- apply (v*, c*)
      const uint32_t vs = win >> 16, cs = win & 0xffffu;
      const uint32_t xv = rfl((uint32_t)cg[vs]);
      const uint32_t bnew = rfl((uint32_t)tab[vs * kp + cs]);
      const uint32_t csz = rfl(csize(cs));
      const uint32_t old = xv & 0xffu;
      const int fnew = f + (int)dstar - 128;
      if (csz >= kW8ClassMax) {  // left to the 16-bit rerun
        give_up();
        return;
      }
      const bool snap = best_cur && fnew >= f_best;  // leaving the best state: keep a copy
      if (snap)
        for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffu);
      const int rs = row_c[vs], re = row_c[vs + 1];
      const uint32_t dec = 0u - (1u << (8u * (old & 3u))), inc = 1u << (8u * (cs & 3u));
      const uint32_t wo = old >> 2, wn = cs >> 2;
      // neighbour u: gamma[u][old] - 1, gamma[u][c*] + 1; if u has colour old
      // or c*, its own gamma and list membership follow.  Up to 256
      // neighbours at a time: every CSR load issued before any is used, then
      // every table add and cg read, then the cg updates; lanes past the row
      // aim at the sink.
      constexpr int kPre = 4;
      for (int e0 = rs; e0 < re; e0 += kPre * kWave) {
        uint32_t nb[kPre], xs[kPre];
#pragma unroll
        for (int r = 0; r < kPre; ++r)  // past the row: a copy of its last entry (valid, redirected below)
          nb[r] = (uint32_t)col_idx[min(e0 + lane + r * kWave, re - 1)];
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
          const bool live = e0 + lane + r * kWave < re;
          uint32_t* ru = tabw + __umul24(nb[r], kq);
          atomicAdd(live ? ru + wo : sink, dec);
          atomicAdd(live ? ru + wn : sink, inc);
          xs[r] = cg[nb[r]];
        }
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
          if (e0 + r * kWave >= re) break;  // uniform: ballots see the whole wave
          const bool live = e0 + lane + r * kWave < re;
          const uint32_t x = xs[r], cu = x & 0xffu;
          const bool lo = cu == old, hi = cu == cs;
          // a neighbour that starts to conflict and is not listed yet is appended
          const bool ins = live && hi && (x & 0xff00u) == 0u;
          const uint32_t nx = x + (hi ? 0x100u : 0u) - (lo ? 0x100u : 0u) + (ins ? 0x8000u : 0u);
          *(live ? &cg[nb[r]] : sink16) = (uint16_t)nx;
          const uint64_t mi = __ballot(ins);
          *(ins ? &list[len + (int)lane_rank(mi)] : sink16) = (uint16_t)nb[r];
          len += __popcll(mi);
        }
      }
      // v*: its new colour flagged, its state, class sizes, the new tabu pair
      const uint32_t gnew = bnew & 0x7fu;
      if (bnew & kW8Flag) key_star = vs * kp + cs;  // a move onto a tabu colour: that pair is consumed
      // tenure term floor(num * f / den), capped (as in the block kernel)
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
      const uint32_t expiry = (uint32_t)t + readlane(Lreg, t & 63) + ttf;
      const bool tabu_next = expiry > (uint32_t)t + 1u;  // tabu from iteration t + 1 on
      if (tabu_next && A >= acap) {
        give_up();
        return;
      }
      if (lane == 0) {
        atomicOr(&tabw[vs * kq + wn], kW8Flag << (8u * (cs & 3u)));
        cg[vs] = (uint16_t)(cs | (gnew << 8) | 0x8000u);
        atomicAdd(&csw[old >> 1], 0u - (1u << (16u * (old & 1u))));
        atomicAdd(&csw[cs >> 1], 1u << (16u * (cs & 1u)));
        if (tabu_next)
          act[A] = ((vs * kp + old) << 15) | (expiry & kW8ExpMask);
        else  // a tenure of 0 or 1 never forbids anything
          atomicAnd(&tabw[vs * kq + wo], ~(kW8Flag << (8u * (old & 3u))));
      }
      if (tabu_next) ++A;
      if (trace && t < trace_cap && lane == 0) {
        gptr<int32_t> tr = trace + ((size_t)li * trace_cap + t) * 2;
        tr[0] = (int32_t)(vs | (cs << 16));
        tr[1] = fnew;
      }
      st_conf += l0 ? (uint64_t)C : 0ull;
      st_deg += l0 ? (uint64_t)(re - rs) : 0ull;
      st_ties += l0 && seen > 1u ? 1u : 0u;
      st_cap += l0 && capped ? 1u : 0u;
      fp = l0 ? fnv_step(fp, vs, cs, fnew) : fp;
      f = fnew;
      if (f < f_best) {
        f_best = f;
        best_cur = true;
      } else if (snap) {
        best_cur = false;
      }
    }
    ++t;

    // ---- tabu pairs for iteration t: expiries, the consumed pair, aspiration
    wave_sync();
    {
      const int aspd = f_best - f - 1;  // admissible by aspiration iff delta <= aspd
      asp = kW8None;
      int base = 0;
      for (int i0 = 0; i0 < A; i0 += kWave) {
        const int i = i0 + lane;
        const bool alive = i < A;
        const uint32_t e = act[alive ? i : 0];
        const uint32_t kk = e >> 15;
        const bool expired = alive && (e & kW8ExpMask) == ((uint32_t)t & kW8ExpMask);
        const bool drop = alive && kk == key_star;
        atomicAnd(expired && !drop ? &tabw[kk >> 2] : sink, ~(kW8Flag << (8u * (kk & 3u))));
        const bool keep = alive && !expired && !drop;
        const uint32_t v = __umulhi(kk, kp_inv);
        const int g = (int)(((uint32_t)cg[v] >> 8) & 0x7fu);
        const int d = (int)(tab[kk] & 0x7fu) - g;
        if (keep && g != 0 && d <= aspd) asp = min(asp, (uint32_t)(d + 128));
        const uint64_t mk = __ballot(keep);
        *(keep ? &act[base + (int)lane_rank(mk)] : sink) = e;
        base += __popcll(mk);
      }
      A = base;
    }
    wave_sync();
  }

  if (best_cur)
    for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffu);
  if (lane == 0) {
    *f_best_out = f_best;
    *iters_out = t;
    if (stats_out) {
      gptr<int64_t> s = stats_out;
      s[0] = (int64_t)(t - (int)st_noops);
      s[1] = (int64_t)st_noops;
      s[2] = (int64_t)st_conf;
      s[3] = (int64_t)st_deg;
      s[4] = (int64_t)st_ties;
      s[5] = (int64_t)st_cap;
      s[6] = 0;
      s[7] = 0;
    }
    if (hash_out) *hash_out = fp;
  }
}

}  // namespace dlm
