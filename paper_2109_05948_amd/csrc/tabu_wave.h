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
  uint32_t tab, cg, list, rowkey, stage, csize, act, bytes;
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
  L.act = o;
  o += 4u * (uint32_t)acap;
  L.bytes = o;
  return L;
}

// dwords per row bucket of the scan (template argument of the kernel)
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

// One individual (row li of a.colors) searched by the calling wavefront.
// KQ: dword bucket of the rows (kp / 4 <= KQ); acap: tabu pairs the LDS holds.
template <int KQ>
__device__ __forceinline__ void tabu_w8_individual(const TabuArgs& a, int li, int acap, unsigned char* smem) {
  constexpr int KQ_LO = KQ == 8 ? 0 : (KQ == 16 ? 8 : (KQ == 24 ? 16 : (KQ == 32 ? 24 : 32)));
  constexpr int W = KQ <= 8 ? 8 : (KQ <= 16 ? 16 : (KQ <= 32 ? 32 : 64));  // lanes per row, tie pass
  constexpr int P = kWave / W;                                              // rows per tie pass
  const int lane = threadIdx.x;
  const uint32_t ind = (uint32_t)(a.ind_base + li);
  const int n = a.n, k = a.k;
  const uint32_t kp = (uint32_t)tab_stride(k), kq = kp >> 2;
  const gptr<const int32_t> col_idx = own_sgpr(a.col_idx);
  const gptr<int32_t> trace = own_sgpr(a.trace);
  const int trace_cap = a.trace_cap, T = a.T;
  const Key key = a.key;
  const uint32_t ten_num = (uint32_t)a.ten_num, ten_den = (uint32_t)a.ten_den, ten_rand = (uint32_t)a.ten_rand;
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
  int16_t* gcol = a.colors + (size_t)li * n;
  const __attribute__((address_space(4))) int32_t* row_c =
      (const __attribute__((address_space(4))) int32_t*)a.row_ptr;
  auto csize = [&](uint32_t c) { return (csw[c >> 1] >> (16u * (c & 1u))) & 0xffffu; };
  auto give_up = [&]() {
    if (lane == 0) a.iters[li] = -2;
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
      a.f_best[li] = -1;
      a.iters[li] = -1;
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
  const int nnz = a.row_ptr[n];
  for (int e = lane; e < nnz; e += kWave) {
    const uint32_t u = (uint32_t)col_idx[e], v = (uint32_t)a.erow[e];
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
  int stale = 0;

  int t = 0, f_best = f, A = 0;
  bool best_cur = true;
  uint32_t asp = kW8None;  // this lane's best biased delta among aspiring tabu pairs
  // statistics and fingerprint live in lane 0; moves = t - no-ops
  uint64_t st_conf = 0, st_deg = 0, fp = kFnvOffset;
  uint32_t st_noops = 0, st_ties = 0, st_cap = 0;
  uint32_t Lreg = 0;

  while (t < T && f > 0) {
    if (((len + 63) >> 6) > ((len - stale + 63) >> 6)) {  // stale entries cost a scan round: rebuild
      wave_sync();
      len = w8_build_list(cg, list, n, lane);
      stale = 0;
      wave_sync();
    }
    const int C = len - stale;  // conflicting vertices
    if ((t & 63) == 0) Lreg = lemire(philox_w0(ind, (uint32_t)(t + lane), 0u, kDomTenure, key), ten_rand);

    // ---- scan: list entry (r << 6) + lane in round r
    const int rounds = (len + 63) >> 6;
    uint32_t best = kW8None, dlast = kW8None, vlast = (uint32_t)n, glast = 0u;
    for (int r = 0; r < rounds; ++r) {
      const int i = (r << 6) + lane;
      const uint32_t v = i < len ? (uint32_t)list[i] : (uint32_t)n;
      const uint32_t g = ((uint32_t)cg[v] >> 8) & 0x7fu;
      const uint32_t* row = tabw + v * kq;
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
      if (i < len) rowkey[i] = (uint8_t)d;
      best = min(best, d);
      dlast = d;
      vlast = v;
      glast = g;
    }
    const uint32_t dstar = wave_min_u32(min(best, asp));
    uint32_t key_star = kW8NoKey;  // the tabu pair a move onto a tabu colour consumes

    if (dstar == kW8None) {  // nothing admissible: no-op iteration
      if (lane == 0) {
        ++st_noops;
        st_conf += (uint64_t)C;
        fp = fnv_step(fp, 0xffffu, 0xffffu, f);
        if (trace && t < trace_cap) {
          gptr<int32_t> tr = trace + ((size_t)li * trace_cap + t) * 2;
          tr[0] = -1;
          tr[1] = f;
        }
      }
    } else {
      // ---- every admissible move at dstar: staged, hashed 64 at a time
      int cnt = 0, total = 0;
      uint64_t hk = ~0ull;
      auto flush64 = [&]() {
        wave_sync();
        const uint32_t e = stage[cnt - 64 + lane];
        hk = umin64(hk, ((uint64_t)philox_w0(ind, (uint32_t)t, e >> 16, e & 0xffffu, key) << 32) | e);
        cnt -= 64;
        wave_sync();
      };
      auto put = [&](bool hit, uint32_t mv) {
        const uint64_t mb = __ballot(hit);
        if (hit) stage[cnt + (int)lane_rank(mb)] = mv;
        cnt += __popcll(mb);
        total += __popcll(mb);
      };
      const int jl = lane & (W - 1), pl = lane / W;
      for (int r = 0; r < rounds; ++r) {
        const bool lastr = r == rounds - 1;
        const int i = (r << 6) + lane;
        const uint32_t dr = lastr ? dlast : (i < len ? (uint32_t)rowkey[i] : kW8None);
        uint64_t M = __ballot(dr == dstar);
        while (M) {
          // the next P tied rows: lane group pl takes row pl
          uint32_t vsel = (uint32_t)n, tsel = 0u;
#pragma unroll
          for (int pp = 0; pp < P; ++pp) {
            if (M) {
              const int ln = __builtin_ctzll(M);
              M &= M - 1;
              uint32_t vr, gr;
              if (lastr) {
                vr = readlane(vlast, ln);
                gr = readlane(glast, ln);
              } else {
                vr = rfl((uint32_t)list[(r << 6) + ln]);
                gr = rfl(((uint32_t)cg[vr] >> 8) & 0x7fu);
              }
              if (pl == pp) {
                vsel = vr;
                tsel = dstar + gr - 128u;  // the row's smallest byte
              }
            }
          }
          const uint32_t x = jl < (int)kq ? tabw[vsel * kq + (uint32_t)jl] : 0xffffffffu;
          const uint32_t y = x ^ (tsel * 0x01010101u);
          // bit 7 of byte b set iff byte b of x equals tsel (tsel < 128, so
          // flagged and padding bytes never match)
          const uint32_t z = ~(((y & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y) & 0x80808080u;
#pragma unroll
          for (int b = 0; b < 4; ++b)
            put(((z >> (8 * b + 7)) & 1u) != 0u, (vsel << 16) | (uint32_t)(4 * jl + b));
          while (cnt >= 64) flush64();
        }
      }
      if (__ballot(asp == dstar)) {
        // tabu pairs at dstar: all of them aspire (the test depends on delta only)
        for (int i0 = 0; i0 < A; i0 += kWave) {
          const int i = i0 + lane;
          bool hit = false;
          uint32_t mv = 0u;
          if (i < A) {
            const uint32_t kk = act[i] >> 15;
            const uint32_t v = __umulhi(kk, kp_inv), c = kk - v * kp;
            const uint32_t g = ((uint32_t)cg[v] >> 8) & 0x7fu;
            hit = g != 0u && (uint32_t)(tab[kk] & 0x7fu) + 128u - g == dstar;
            mv = (v << 16) | c;
          }
          put(hit, mv);
          while (cnt >= 64) flush64();
        }
      }
      wave_sync();
      uint32_t win;
      if (total == 1) {
        win = rfl(stage[0]);
      } else {
        if (lane < cnt) {
          const uint32_t e = stage[lane];
          hk = umin64(hk, ((uint64_t)philox_w0(ind, (uint32_t)t, e >> 16, e & 0xffffu, key) << 32) | e);
        }
        win = (uint32_t)wave_min_u64(hk);
      }

      // ---- apply (v*, c*)
      const uint32_t vs = win >> 16, cs = win & 0xffffu;
      const uint32_t xv = rfl((uint32_t)cg[vs]);
      const uint32_t old = xv & 0xffu;
      const uint32_t bnew = rfl((uint32_t)tab[vs * kp + cs]);
      const int fnew = f + (int)dstar - 128;
      if (rfl(csize(cs)) >= kW8ClassMax) {  // left to the 16-bit rerun
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
      // or c*, its own gamma and list membership follow
      auto update = [&](uint32_t u, bool live) {
        bool to_stale = false, from_stale = false, ins = false;
        if (live) {
          atomicAdd(&tabw[u * kq + wo], dec);
          atomicAdd(&tabw[u * kq + wn], inc);
          const uint32_t x = cg[u];
          const uint32_t cu = x & 0xffu, g = (x >> 8) & 0x7fu;
          if (cu == old) {
            cg[u] = (uint16_t)(x - 0x100u);
            to_stale = g == 1u;
          } else if (cu == cs) {
            if (g == 0u) {
              from_stale = (x >> 15) != 0u;
              ins = !from_stale;
            }
            cg[u] = (uint16_t)((x + 0x100u) | (ins ? 0x8000u : 0u));
          }
        }
        const uint64_t mi = __ballot(ins);
        if (ins) list[len + (int)lane_rank(mi)] = (uint16_t)u;
        len += __popcll(mi);
        stale += __popcll(__ballot(to_stale)) - __popcll(__ballot(from_stale));
      };
      constexpr int kPre = 4;  // the first 256 neighbours: every load issued before any is used
      int nb[kPre];
#pragma unroll
      for (int r = 0; r < kPre; ++r) {
        const int e = rs + lane + r * kWave;
        nb[r] = e < re ? col_idx[e] : -1;
      }
#pragma unroll
      for (int r = 0; r < kPre; ++r)
        if (rs + r * kWave < re) update((uint32_t)nb[r], nb[r] >= 0);
      for (int e0 = rs + kPre * kWave; e0 < re; e0 += kWave) {
        const int e = e0 + lane;
        update(e < re ? (uint32_t)col_idx[e] : 0u, e < re);
      }
      // v*: its new colour flagged, its state, class sizes
      const uint32_t gnew = bnew & 0x7fu;
      if (bnew & kW8Flag) key_star = vs * kp + cs;  // a move onto a tabu colour: that pair is consumed
      if (lane == 0) {
        atomicOr(&tabw[vs * kq + wn], kW8Flag << (8u * (cs & 3u)));
        cg[vs] = (uint16_t)(cs | (gnew << 8) | 0x8000u);
        atomicAdd(&csw[old >> 1], 0u - (1u << (16u * (old & 1u))));
        atomicAdd(&csw[cs >> 1], 1u << (16u * (cs & 1u)));
      }
      if (gnew == 0u) ++stale;
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
      if (expiry > (uint32_t)t + 1u) {  // tabu from iteration t + 1 on
        if (A >= acap) {
          give_up();
          return;
        }
        if (lane == 0) act[A] = ((vs * kp + old) << 15) | (expiry & kW8ExpMask);
        ++A;
      } else if (lane == 0) {  // a tenure of 0 or 1 never forbids anything
        atomicAnd(&tabw[vs * kq + wo], ~(kW8Flag << (8u * (old & 3u))));
      }
      if (lane == 0) {
        if (trace && t < trace_cap) {
          gptr<int32_t> tr = trace + ((size_t)li * trace_cap + t) * 2;
          tr[0] = (int32_t)(vs | (cs << 16));
          tr[1] = fnew;
        }
        st_conf += (uint64_t)C;
        st_deg += (uint64_t)(re - rs);
        st_ties += total > 1 ? 1u : 0u;
        st_cap += capped ? 1u : 0u;
        fp = fnv_step(fp, vs, cs, fnew);
      }
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
        const uint32_t e = alive ? act[i] : 0u;
        const uint32_t kk = e >> 15;
        const bool expired = alive && (e & kW8ExpMask) == ((uint32_t)t & kW8ExpMask);
        const bool drop = alive && kk == key_star;
        if (expired && !drop) atomicAnd(&tabw[kk >> 2], ~(kW8Flag << (8u * (kk & 3u))));
        const bool keep = alive && !expired && !drop;
        if (keep && aspd >= -127) {
          const uint32_t v = __umulhi(kk, kp_inv);
          const int g = (int)(((uint32_t)cg[v] >> 8) & 0x7fu);
          const int d = (int)(tab[kk] & 0x7fu) - g;
          if (g != 0 && d <= aspd) asp = min(asp, (uint32_t)(d + 128));
        }
        const uint64_t mk = __ballot(keep);
        if (keep) act[base + (int)lane_rank(mk)] = e;
        base += __popcll(mk);
      }
      A = base;
    }
    wave_sync();
  }

  if (best_cur)
    for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffu);
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

}  // namespace dlm
