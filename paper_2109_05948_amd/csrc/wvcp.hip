// Weighted vertex colouring: the iterated feasible/infeasible tabu search of
// Section 2.2 and Algorithm 2, one workgroup per individual.
//
// Round r minimises g = (f_w << S) + phi * c (eq. (AFISA_score) in fixed
// point with S fractional bits of phi), f_w = sum over classes of the
// largest weight (eq. (score_WVCP)), c = conflicting edges.  Moves are the
// one-moves of every vertex; a moved vertex is frozen for
// L + floor(frz_num * n / frz_den) iterations (Section 2.2); a frozen move is
// allowed when it improves the best g of the round (aspiration).  phi_0 =
// floor(k * max_w * 2^S / (2 n)); after a round whose best-g state is legal
// phi is halved, otherwise doubled (capped at 2^30); the last round uses
// phi = 2 * max_w.  Each round restarts from the previous round's best-g
// state with a fresh freeze list; the iteration counter t runs on across
// rounds.  The result is the best legal colouring met anywhere.
//
// One iteration: a branch-free scan of every (v, c) one-move, a quad of
// colours at a time with the per-vertex terms computed once per quad; each
// wave hashes the moves tied at its best key before one barrier picks the
// (key, hash, v, c) minimum; every thread takes a share of v*'s neighbours;
// the class c* gains v* in O(1) and the class it left is rescanned only when
// v* carried its largest weight alone or its second largest weight.
//
// LDS per individual: gamma[v][c] (u16, rows padded to 4 colours), per
// vertex {colour | gamma of own colour, weight, frozen-until}, per class
// (largest weight, its multiplicity, second largest weight), the best-g
// colouring.
#include "dlm_common.h"

namespace dlm {

constexpr uint64_t kGBias = 1ull << 62;
constexpr int kWStage = 128;  // tied moves a wave hashes in one staged pass

struct WvcpArgs {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* erow;
  const int32_t* weights;
  int16_t* colors;
  int32_t* best_legal;
  int64_t* stats;
  uint64_t* hash;
  Key key;
  int32_t n, k, T, R, ten_rand, frz, shift, ind_base, max_w, max_deg;
};

// gamma rows are padded to kp = k rounded up to 4 colours (one 8-byte read
// per quad of candidates); per vertex {colour | gamma(own colour) << 16,
// weight, frozen-until, 0}; per class {largest weight, its multiplicity,
// second largest, 0} and the largest weights again as a dense vector.
struct WvcpLayout {
  uint32_t gam, vinfo, cls, m1v, bestg, red, stage, pub, bytes;
};

__host__ __device__ constexpr int wvcp_stride(int k) { return (k + 3) & ~3; }

__host__ __device__ inline WvcpLayout wvcp_layout(int n, int k, int nw) {
  WvcpLayout L;
  const uint32_t kp = (uint32_t)wvcp_stride(k);
  uint32_t o = 0;
  L.gam = o;
  o += align16(2u * n * kp);
  L.vinfo = o;
  o += 16u * n;
  L.cls = o;
  o += 16u * kp;
  L.m1v = o;
  o += align16(4u * kp);
  L.bestg = o;
  o += align16(2u * n);
  L.red = o;
  o += 2u * 32u * nw;  // two parity buffers of 8 words per wave
  L.stage = o;
  o += nw * 4u * (kWStage + 4);
  L.pub = o;  // best key published so far, by iteration parity
  o += 16u;
  L.bytes = o;
  return L;
}

// (largest, multiplicity, second largest) of a set of weights; associative
struct Cls {
  uint32_t m1, c1, m2;
};
__device__ __forceinline__ Cls cls_join(Cls a, Cls b) {
  if (a.m1 > b.m1) return Cls{a.m1, a.c1, max(a.m2, b.m1)};
  if (a.m1 < b.m1) return Cls{b.m1, b.c1, max(b.m2, a.m1)};
  return Cls{a.m1, a.c1 + b.c1, max(a.m2, b.m2)};
}
template <int CTRL>
__device__ __forceinline__ Cls cls_dpp(Cls x) {
  return Cls{dpp_mov<CTRL>(x.m1), dpp_mov<CTRL>(x.c1), dpp_mov<CTRL>(x.m2)};
}
__device__ __forceinline__ Cls cls_readlane(Cls x, int l) {
  return Cls{readlane(x.m1, l), readlane(x.c1, l), readlane(x.m2, l)};
}
__device__ __forceinline__ Cls wave_cls(Cls x) {
  x = cls_join(x, cls_dpp<dpp::kXor1>(x));
  x = cls_join(x, cls_dpp<dpp::kXor2>(x));
  x = cls_join(x, cls_dpp<dpp::kHalfMirror>(x));
  x = cls_join(x, cls_dpp<dpp::kMirror>(x));
  return cls_join(cls_join(cls_readlane(x, 0), cls_readlane(x, 16)),
                  cls_join(cls_readlane(x, 32), cls_readlane(x, 48)));
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void wvcp_kernel(WvcpArgs a) {
  constexpr int NW = BLOCK / kWave;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int li = blockIdx.x;
  const uint32_t ind = (uint32_t)(a.ind_base + li);
  const int n = a.n, k = a.k, kp = wvcp_stride(k), kq = kp >> 2, S = a.shift;
  const WvcpLayout L = wvcp_layout(n, k, NW);
  uint16_t* gam = reinterpret_cast<uint16_t*>(smem + L.gam);
  uint4* vinfo = reinterpret_cast<uint4*>(smem + L.vinfo);  // {cg, weight, frozen, 0}
  uint4* cls = reinterpret_cast<uint4*>(smem + L.cls);      // {m1, c1, m2, 0}
  uint32_t* m1v = reinterpret_cast<uint32_t*>(smem + L.m1v);
  int16_t* bestg = reinterpret_cast<int16_t*>(smem + L.bestg);
  uint32_t* red = reinterpret_cast<uint32_t*>(smem + L.red);  // [2][NW][8]
  uint32_t* stage = reinterpret_cast<uint32_t*>(smem + L.stage);
  unsigned long long* pub = reinterpret_cast<unsigned long long*>(smem + L.pub);
  int16_t* gcol = a.colors + (size_t)li * n;
  const Key key = a.key;
  const int32_t* __restrict__ col_idx = a.col_idx;
  __shared__ int32_t s_red[2 * NW];

  int bad = 0;
  if (tid == 0) {
    pub[0] = ~0ull;
    pub[1] = ~0ull;
  }
  for (int v = tid; v < n; v += BLOCK) {
    const int c = gcol[v];
    bad |= (c < 0) | (c >= k);
    bestg[v] = (int16_t)c;
  }
  if (__syncthreads_or(bad)) {
    if (tid == 0) a.best_legal[li] = -1;
    return;
  }

  const int64_t phi_max = 1ll << 30;
  int64_t phi = ((int64_t)k * a.max_w << S) / (2 * (int64_t)n);
  int64_t best_legal = INT64_MAX;
  int t = 0;
  // statistics and fingerprint live in lane 0 of wave 0; moves = t - no-ops
  uint64_t st_deg = 0, fp = kFnvOffset;
  uint32_t st_noops = 0, st_ties = 0, st_legal_rounds = 0;
  uint32_t Lreg = 0;
  const int i0 = tid / kq, q0 = tid - (tid / kq) * kq, di = BLOCK / kq, dq = BLOCK - (BLOCK / kq) * kq;
  const int totq = n * kq;
  auto step = [&](int& i, int& q) {
    q += dq;
    i += di;
    if (q >= kq) {
      q -= kq;
      ++i;
    }
  };

  for (int r = 0; r < a.R; ++r) {
    if (r == a.R - 1) phi = (int64_t)(2 * a.max_w) << S;
    const int32_t phi32 = (int32_t)phi;  // phi <= 2^30
    // |dg| <= (max_w << S) + phi * max_deg: 32-bit keys when that stays below 2^31 - 1
    const bool k32_round = ((int64_t)a.max_w << S) + phi * (int64_t)a.max_deg < (int64_t)INT32_MAX - 1;
    // ---- fresh round state from the best-g colouring of the previous round
    for (int i = tid; i < n * kp / 2; i += BLOCK) reinterpret_cast<uint32_t*>(gam)[i] = 0u;
    for (int v = tid; v < n; v += BLOCK)
      vinfo[v] = make_uint4((uint32_t)(uint16_t)bestg[v], (uint32_t)a.weights[v], 0u, 0u);
    for (int c = tid; c < kp; c += BLOCK) {
      cls[c] = make_uint4(0u, 0u, 0u, 0u);
      m1v[c] = 0u;
    }
    __syncthreads();
    const int nnz = a.row_ptr[n];
    for (int e = tid; e < nnz; e += BLOCK) {
      const int ix = a.erow[e] * kp + (int)(vinfo[col_idx[e]].x & 0xffffu);
      atomicAdd(reinterpret_cast<uint32_t*>(gam) + (ix >> 1), (ix & 1) ? 0x10000u : 1u);
    }
    for (int v = tid; v < n; v += BLOCK) atomicMax(&cls[vinfo[v].x & 0xffffu].x, vinfo[v].y);
    __syncthreads();
    uint32_t cs2 = 0;
    for (int v = tid; v < n; v += BLOCK) {
      const uint32_t c = vinfo[v].x & 0xffffu, wv = vinfo[v].y;
      const uint32_t g = gam[v * kp + (int)c];
      vinfo[v].x = c | (g << 16);
      cs2 += g;
      if (wv == cls[c].x) atomicAdd(&cls[c].y, 1u);
      else atomicMax(&cls[c].z, wv);
    }
    cs2 = wave_sum_u32(cs2);
    uint32_t fwp = 0;
    for (int c = tid; c < k; c += BLOCK) {
      fwp += cls[c].x;
      m1v[c] = cls[c].x;
    }
    fwp = wave_sum_u32(fwp);
    if (lane == 0) {
      s_red[wid] = (int32_t)cs2;
      s_red[NW + wid] = (int32_t)fwp;
    }
    __syncthreads();
    int64_t conf = 0, fw = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      conf += s_red[q];
      fw += s_red[NW + q];
    }
    conf >>= 1;
    int64_t G = (fw << S) + phi * conf, G_best = G, conf_best = conf;
    if (conf == 0 && fw < best_legal) {
      best_legal = fw;
      if (wid == 0)
        for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(vinfo[v].x & 0xffffu);
    }
    __syncthreads();  // s_red is reused by the next round

    for (int it = 0; it < a.T; ++it, ++t) {
      const int par = (t & 1) * NW;
      if (wid == 0 && (t & 63) == 0)
        Lreg = lemire(philox_w0(ind, (uint32_t)(t + lane), 0u, kDomTenure, key), (uint32_t)a.ten_rand);
      const int64_t asp = G_best - G - 1;  // aspiration: G + dg < G_best

      // ---- scan every one-move (v, c), c != col v, one quad of colours at a time.
      // Keys are dg + bias in 32 bits when the round's bound allows it, else 64.
      auto pick = [&](auto key_zero) {
      using KT = decltype(key_zero);
      constexpr bool k32 = sizeof(KT) == 4;
      constexpr KT kNoKey = (KT)~(KT)0;
      const int32_t asp32 = (int32_t)max<int64_t>(min<int64_t>(asp, INT32_MAX), INT32_MIN);
      KT bd = kNoKey;
      uint32_t cnt = 0, s0 = 0, s1 = 0;
      auto eval_quad = [&](int v, int q, auto&& fn) {
        const uint4 vi = vinfo[v];
        const uint32_t cv = vi.x & 0xffffu, gcur = vi.x >> 16, wv = vi.y;
        const bool fr = (int)vi.z <= t;
        const uint4 ca = cls[cv];
        const int32_t base_fw = (int32_t)((wv < ca.x || ca.y > 1u) ? ca.x : ca.z) - (int32_t)ca.x;
        const uint4 m4 = *reinterpret_cast<const uint4*>(m1v + 4 * q);
        const uint2 g2 = *reinterpret_cast<const uint2*>(gam + v * kp + 4 * q);
        const uint32_t gq[4] = {g2.x & 0xffffu, g2.x >> 16, g2.y & 0xffffu, g2.y >> 16};
        const uint32_t mq[4] = {m4.x, m4.y, m4.z, m4.w};
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int c = 4 * q + rr;
          const int32_t dfw = (int32_t)(max(mq[rr], wv) - mq[rr]) + base_fw;
          const int32_t dcf = (int32_t)gq[rr] - (int32_t)gcur;
          if constexpr (k32) {
            const int32_t dg = dfw * (int32_t)(1 << S) + phi32 * dcf;  // |dg| < 2^31 - 1 this round
            const bool adm = c < k && (uint32_t)c != cv && (fr || dg <= asp32);
            fn(((uint32_t)v << 16) | (uint32_t)c, adm ? (KT)((uint32_t)dg + 0x80000000u) : kNoKey);
          } else {
            const int64_t dg = (int64_t)dfw * ((int64_t)1 << S) + (int64_t)phi32 * dcf;
            const bool adm = c < k && (uint32_t)c != cv && (fr || dg <= asp);
            fn(((uint32_t)v << 16) | (uint32_t)c, adm ? (KT)((uint64_t)dg + kGBias) : kNoKey);
          }
        }
      };
      auto consider = [&](uint32_t idx, KT b) {
        const bool lt = b < bd, eq = b == bd;
        s1 = (eq && cnt == 1u) ? idx : s1;
        cnt = lt ? 1u : cnt + (eq ? 1u : 0u);
        s0 = lt ? idx : s0;
        bd = lt ? b : bd;
      };
      {
        int i = i0, q = q0;
        for (int j = tid; j < totq; j += BLOCK) {
          eval_quad(i, q, consider);
          step(i, q);
        }
      }

      // ---- wave result: smallest (key, Philox word, v, c); the moves tied at
      // the wave's best key are staged in LDS and hashed in one pass
      KT wbd;
      if constexpr (k32) wbd = wave_min_u32(bd);
      else wbd = wave_min_u64(bd);
      // the wave's best key as dg + 2^62, whichever width the scan used
      uint64_t wk64 = ~0ull;
      if constexpr (k32) {
        if (wbd != kNoKey) wk64 = (uint64_t)(int64_t)(int32_t)((uint32_t)wbd - 0x80000000u) + kGBias;
      } else {
        wk64 = wbd;
      }
      // publish it; a wave beaten by an earlier one cannot hold the chosen
      // move and skips the hashing
      bool live = wbd != kNoKey;
      if (live) {
        unsigned long long prev = 0ull;
        if (lane == 0) prev = atomicMin(&pub[t & 1], (unsigned long long)wk64);
        const uint64_t p64 = ((uint64_t)readlane((uint32_t)(prev >> 32), 0) << 32) | readlane((uint32_t)prev, 0);
        live = p64 >= wk64;
      }
      uint64_t hk = ~0ull;
      uint32_t wcnt = 0u;
      if (live) {
        auto hkey = [&](uint32_t idx) -> uint64_t {
          return ((uint64_t)philox_w0(ind, (uint32_t)t, idx >> 16, idx & 0xffffu, key) << 32) | idx;
        };
        const bool tie = bd == wbd;
        const bool A = tie && cnt <= 2u, B = tie && cnt == 2u, Rr = tie && cnt > 2u;
        const uint64_t mA = __ballot(A), mB = __ballot(B);
        const uint32_t nR = wave_sum_u32(Rr ? cnt : 0u);
        const uint32_t nA = (uint32_t)__popcll(mA), nB = (uint32_t)__popcll(mB);
        const uint32_t total = nA + nB + nR;
        wcnt = total;
        auto rescan = [&](auto&& sink) {
          int i = i0, q = q0;
          for (int j = tid; j < totq; j += BLOCK) {
            eval_quad(i, q, [&](uint32_t idx, KT b) {
              if (b == wbd) sink(idx);
            });
            step(i, q);
          }
        };
        if (total <= (uint32_t)kWStage) {
          uint32_t* stg = stage + wid * (kWStage + 4);
          uint32_t* rctr = stg + kWStage;
          if (lane == 0) *rctr = nA + nB;
          if (A) stg[__builtin_amdgcn_mbcnt_hi((uint32_t)(mA >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mA, 0u))] = s0;
          if (B) stg[nA + __builtin_amdgcn_mbcnt_hi((uint32_t)(mB >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mB, 0u))] = s1;
          if (Rr) {
            uint32_t p = atomicAdd(rctr, cnt);
            rescan([&](uint32_t idx) { stg[p++] = idx; });
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          for (uint32_t c0 = 0; c0 < total; c0 += kWave)
            if (c0 + lane < total) hk = umin64(hk, hkey(stg[c0 + lane]));
        } else {
          if (A) hk = hkey(s0);
          if (B) hk = umin64(hk, hkey(s1));
          if (Rr) rescan([&](uint32_t idx) { hk = umin64(hk, hkey(idx)); });
        }
      }
      {
        const uint64_t whk = live ? wave_min_u64(hk) : ~0ull;
        // the chosen vertex's colour and gamma, read while no wave writes them
        uint32_t wold = 0, wdcf = 0;
        if (live) {
          const uint32_t v = (uint32_t)whk >> 16, c = (uint32_t)whk & 0xffffu;
          const uint32_t x = vinfo[v].x;
          wold = x & 0xffffu;
          wdcf = (uint32_t)((int32_t)gam[v * kp + (int)c] - (int32_t)(x >> 16));
        }
        if (lane == 0) {
          uint32_t* e = red + (par + wid) * 8;
          *reinterpret_cast<uint4*>(e) = make_uint4((uint32_t)wk64, (uint32_t)(wk64 >> 32), wcnt, (uint32_t)whk);
          *reinterpret_cast<uint4*>(e + 4) = make_uint4((uint32_t)(whk >> 32), wold, wdcf, 0u);
        }
      }
      };
      if (k32_round) pick(0u);
      else pick(0ull);
      __syncthreads();
      // every wave has published: the slot is free again for iteration t + 2
      if (tid == 0) pub[t & 1] = ~0ull;
      // cross-wave: smallest (key, hash, v, c), folded in scalar registers
      auto rfl = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); };
      uint64_t gk, gh;
      uint32_t gcnt, gold, gdcf;
      {
        const uint4 e0 = *reinterpret_cast<const uint4*>(red + par * 8);
        const uint4 e1 = *reinterpret_cast<const uint4*>(red + par * 8 + 4);
        gk = ((uint64_t)rfl(e0.y) << 32) | rfl(e0.x);
        gcnt = rfl(e0.z);
        gh = ((uint64_t)rfl(e1.x) << 32) | rfl(e0.w);
        gold = rfl(e1.y);
        gdcf = rfl(e1.z);
      }
#pragma unroll
      for (int q = 1; q < NW; ++q) {
        const uint4 e0 = *reinterpret_cast<const uint4*>(red + (par + q) * 8);
        const uint4 e1 = *reinterpret_cast<const uint4*>(red + (par + q) * 8 + 4);
        const uint64_t ek = ((uint64_t)rfl(e0.y) << 32) | rfl(e0.x);
        const uint64_t eh = ((uint64_t)rfl(e1.x) << 32) | rfl(e0.w);
        const uint32_t ec = rfl(e0.z), eo = rfl(e1.y), ed = rfl(e1.z);
        gcnt = ek < gk ? ec : (ek == gk ? gcnt + ec : gcnt);
        const bool take = ek < gk || (ek == gk && eh < gh);
        gk = take ? ek : gk;
        gh = take ? eh : gh;
        gold = take ? eo : gold;
        gdcf = take ? ed : gdcf;
      }
      if (gk == ~0ull) {  // nothing admissible
        if (wid == 0 && lane == 0) {
          ++st_noops;
          fp = fnv_step(fp, 0xffffu, 0xffffu, (int32_t)(G >> S));
        }
        continue;
      }
      const uint32_t win = (uint32_t)gh;
      const int vs = (int)(win >> 16), cs = (int)(win & 0xffffu), old = (int)gold;
      const int64_t dg = (int64_t)(gk - kGBias);
      const int rs = a.row_ptr[vs], re = a.row_ptr[vs + 1];

      // ---- apply: every thread takes a share of the neighbours of v*
      {
        auto update = [&](int u) {
          const int io = u * kp + old, ic = u * kp + cs;
          atomicAdd(reinterpret_cast<uint32_t*>(gam) + (io >> 1), (io & 1) ? 0xffff0000u : 0xffffffffu);
          atomicAdd(reinterpret_cast<uint32_t*>(gam) + (ic >> 1), (ic & 1) ? 0x10000u : 1u);
          const uint32_t xu = vinfo[u].x;
          const uint32_t cu = xu & 0xffffu;
          vinfo[u].x = xu - (cu == (uint32_t)old ? 0x10000u : 0u) + (cu == (uint32_t)cs ? 0x10000u : 0u);
        };
        constexpr int kPre = BLOCK >= 256 ? 2 : 4;
        int nb[kPre];
#pragma unroll
        for (int q = 0; q < kPre; ++q) {
          const int e = rs + tid + q * BLOCK;
          nb[q] = e < re ? col_idx[e] : -1;
        }
#pragma unroll
        for (int q = 0; q < kPre; ++q)
          if (nb[q] >= 0) update(nb[q]);
        for (int e = rs + kPre * BLOCK + tid; e < re; e += BLOCK) update(col_idx[e]);
      }
      if (wid == 0) {
        const uint32_t Lt = readlane(Lreg, t & 63);
        const uint32_t wv = vinfo[vs].y;
        if (lane == 0) {
          vinfo[vs].x = (uint32_t)cs | ((uint32_t)gam[vs * kp + cs] << 16);
          vinfo[vs].z = (uint32_t)(t + (int)Lt + a.frz);
          // class c* gains v*
          const uint4 cb = cls[cs];
          const uint32_t nm1 = max(cb.x, wv);
          const uint32_t nc1 = wv > cb.x ? 1u : (wv == cb.x ? cb.y + 1u : cb.y);
          const uint32_t nm2 = wv > cb.x ? cb.x : (wv == cb.x ? cb.z : max(cb.z, wv));
          cls[cs] = make_uint4(nm1, nc1, nm2, 0u);
          m1v[cs] = nm1;
        }
        // class old loses v*: its triple changes without a rescan unless v*
        // carried its largest weight alone or its second largest
        const uint4 ca = cls[old];
        if (wv == ca.x && ca.y > 1u) {
          if (lane == 0) cls[old].y = ca.y - 1u;
        } else if (wv == ca.x || wv == ca.z) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          Cls acc{0, 0, 0};
          for (int v = lane; v < n; v += kWave) {
            const uint4 vi = vinfo[v];
            if ((vi.x & 0xffffu) == (uint32_t)old) acc = cls_join(acc, Cls{vi.y, 1u, 0u});
          }
          acc = wave_cls(acc);
          if (lane == 0) {
            cls[old] = make_uint4(acc.m1, acc.c1, acc.m2, 0u);
            m1v[old] = acc.m1;
          }
        }
        if (lane == 0) {
          st_deg += (uint64_t)(re - rs);
          st_ties += gcnt > 1u;
        }
      }
      __syncthreads();
      conf += (int32_t)gdcf;
      G += dg;
      fw = (G - phi * conf) >> S;
      if (wid == 0 && lane == 0) fp = fnv_step(fp, (uint32_t)vs, (uint32_t)cs, (int32_t)(G >> S));
      if (G < G_best) {
        G_best = G;
        conf_best = conf;
        for (int v = tid; v < n; v += BLOCK) bestg[v] = (int16_t)(vinfo[v].x & 0xffffu);
      }
      if (conf == 0 && fw < best_legal) {
        best_legal = fw;
        if (wid == 0)
          for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(vinfo[v].x & 0xffffu);
      }
    }
    // next round starts from bestg (already in LDS); adapt phi
    const bool legal = conf_best == 0;
    if (wid == 0 && lane == 0) st_legal_rounds += legal;
    if (r < a.R - 1) phi = legal ? (phi >> 1) : min(phi << 1, phi_max);
    __syncthreads();
  }
  if (wid == 0) {
    if (best_legal == INT64_MAX)
      for (int v = lane; v < n; v += kWave) gcol[v] = bestg[v];
    if (lane == 0) {
      a.best_legal[li] = best_legal == INT64_MAX ? 0x7fffffff : (int32_t)best_legal;
      if (a.stats) {
        int64_t* s = a.stats + (size_t)li * DLM_NSTATS;
        s[0] = (int64_t)(t - (int)st_noops);
        s[1] = (int64_t)st_noops;
        s[2] = (int64_t)st_deg;
        s[3] = (int64_t)st_ties;
        s[4] = (int64_t)st_legal_rounds;
        s[5] = phi;
        s[6] = 0;
        s[7] = 0;
      }
      if (a.hash) a.hash[li] = fp;
    }
  }
}

template <int BLOCK>
static int launch_wvcp(const WvcpArgs& a, int pop, size_t lds, hipStream_t s) {
  auto kern = wvcp_kernel<BLOCK>;
  DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(pop), dim3(BLOCK), lds, s, a);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

}  // namespace dlm

using namespace dlm;

extern "C" int dlm_wvcp_batch(const dlm_graph* g, const dlm_wvcp_params* p, int32_t pop,
                              int16_t* colors, int32_t* best_legal, int64_t* stats, uint64_t* hash,
                              void* stream) {
  if (!g || !p) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: graph or params is NULL");
  if (!g->weights) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: the graph has no vertex weights");
  if (pop < 0) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: pop < 0");
  if (p->k < 1 || p->k > 32767) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: k=%d outside [1, 32767]", p->k);
  if (p->iters_per_round < 0 || p->rounds < 0 || (int64_t)p->iters_per_round * p->rounds > (1ll << 30))
    return set_error(DLM_E_INVAL, "dlm_wvcp_batch: rounds x iterations must be in [0, 2^30]");
  if (p->ten_rand < 1 || p->ten_rand > 1024)
    return set_error(DLM_E_INVAL, "dlm_wvcp_batch: ten_rand=%d outside [1, 1024]", p->ten_rand);
  if (p->frz_den <= 0 || p->frz_num < 0 || p->frz_num > 1024)
    return set_error(DLM_E_INVAL, "dlm_wvcp_batch: freeze slope %d/%d invalid", p->frz_num, p->frz_den);
  if (p->shift < 0 || p->shift > 16) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: shift=%d outside [0, 16]", p->shift);
  if (((int64_t)2 * g->max_w << p->shift) > (1ll << 30))
    return set_error(DLM_E_UNSUPPORTED, "dlm_wvcp_batch: 2 * max weight (%d) << shift (%d) exceeds 2^30", g->max_w,
                     p->shift);
  if (p->ind_base < 0 || (int64_t)p->ind_base + pop > 0x7fffffffll)
    return set_error(DLM_E_INVAL, "dlm_wvcp_batch: ind_base + pop exceeds 2^31");
  if (p->reserved != 0) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: reserved must be 0");
  if (pop == 0) return DLM_OK;
  if (!colors || !best_legal) return set_error(DLM_E_INVAL, "dlm_wvcp_batch: null output buffer");
  const int block = p->block ? p->block : 256;
  if (block != 64 && block != 128 && block != 256 && block != 512)
    return set_error(DLM_E_INVAL, "dlm_wvcp_batch: block=%d not in {64,128,256,512}", block);
  const size_t lds = wvcp_layout(g->n, p->k, block / kWave).bytes;
  if ((int64_t)lds > device_lds_limit())
    return set_error(DLM_E_UNSUPPORTED, "dlm_wvcp_batch: %zu bytes of LDS needed", lds);
  WvcpArgs a{g->row_ptr, g->col_idx, g->erow, g->weights, colors, best_legal, stats, hash,
             make_key(p->seed), g->n, p->k, p->iters_per_round, p->rounds, p->ten_rand,
             (int32_t)((int64_t)p->frz_num * g->n / p->frz_den), p->shift, p->ind_base, g->max_w, g->max_deg};
  hipStream_t s = (hipStream_t)stream;
  switch (block) {
    case 64: return launch_wvcp<64>(a, pop, lds, s);
    case 128: return launch_wvcp<128>(a, pop, lds, s);
    case 256: return launch_wvcp<256>(a, pop, lds, s);
    default: return launch_wvcp<512>(a, pop, lds, s);
  }
}
