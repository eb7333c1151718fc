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
// LDS per individual: gamma[v][c] (u16), colour|gamma-of-own-colour per
// vertex, weights, freeze expiries, best-g colouring, per-class (largest
// weight, its multiplicity, second largest weight).
#include "dlm_common.h"

namespace dlm {

constexpr uint64_t kGBias = 1ull << 62;

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
  int32_t n, k, T, R, ten_rand, frz, shift, ind_base, max_w;
};

struct WvcpLayout {
  uint32_t gam, cg, w, frozen, bestg, m1, c1, m2, red, bytes;
};

__host__ __device__ inline WvcpLayout wvcp_layout(int n, int k, int nw) {
  WvcpLayout L;
  uint32_t o = 0;
  L.gam = o;
  o += align16(2u * n * k);
  L.cg = o;
  o += align16(4u * n);
  L.w = o;
  o += align16(4u * n);
  L.frozen = o;
  o += align16(4u * n);
  L.bestg = o;
  o += align16(2u * n);
  L.m1 = o;
  o += align16(4u * k);
  L.c1 = o;
  o += align16(4u * k);
  L.m2 = o;
  o += align16(4u * k);
  L.red = o;
  o += 2u * 8u * 4u * nw;  // two parity buffers of {key, idx|cnt, hash} per wave
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
  const int n = a.n, k = a.k, nk = n * k, S = a.shift;
  const WvcpLayout L = wvcp_layout(n, k, NW);
  uint16_t* gam = reinterpret_cast<uint16_t*>(smem + L.gam);
  uint32_t* cg = reinterpret_cast<uint32_t*>(smem + L.cg);
  int32_t* w = reinterpret_cast<int32_t*>(smem + L.w);
  int32_t* frozen = reinterpret_cast<int32_t*>(smem + L.frozen);
  int16_t* bestg = reinterpret_cast<int16_t*>(smem + L.bestg);
  uint32_t* m1 = reinterpret_cast<uint32_t*>(smem + L.m1);
  uint32_t* c1 = reinterpret_cast<uint32_t*>(smem + L.c1);
  uint32_t* m2 = reinterpret_cast<uint32_t*>(smem + L.m2);
  uint64_t* rkey = reinterpret_cast<uint64_t*>(smem + L.red);  // [2][NW]
  uint64_t* rhash = rkey + 2 * NW;                              // [2][NW]
  uint32_t* ridx = reinterpret_cast<uint32_t*>(rhash + 2 * NW); // [2][NW]
  uint32_t* rcnt = ridx + 2 * NW;                               // [2][NW]
  int16_t* gcol = a.colors + (size_t)li * n;

  int bad = 0;
  for (int v = tid; v < n; v += BLOCK) {
    const int c = gcol[v];
    bad |= (c < 0) | (c >= k);
    bestg[v] = (int16_t)c;
    w[v] = a.weights[v];
  }
  if (__syncthreads_or(bad)) {
    if (tid == 0) a.best_legal[li] = -1;
    return;
  }

  const int64_t phi_max = 1ll << 30;
  int64_t phi = ((int64_t)k * a.max_w << S) / (2 * (int64_t)n);
  int64_t best_legal = INT64_MAX;
  int t = 0;
  uint64_t st_moves = 0, st_noops = 0, st_deg = 0, st_ties = 0, st_legal_rounds = 0;
  uint64_t fp = kFnvOffset;
  uint32_t Lreg = 0;
  int Lbase = -64;
  const int i0 = tid / k, c0 = tid - (tid / k) * k, di = BLOCK / k, dc = BLOCK - (BLOCK / k) * k;
  __shared__ int32_t s_red[2 * NW];
  __shared__ int32_t s_dcs;

  for (int r = 0; r < a.R; ++r) {
    if (r == a.R - 1) phi = (int64_t)(2 * a.max_w) << S;
    // ---- fresh round state from the best-g colouring of the previous round
    for (int i = tid; i < nk; i += BLOCK) gam[i] = 0;
    for (int v = tid; v < n; v += BLOCK) {
      cg[v] = (uint32_t)(uint16_t)bestg[v];
      frozen[v] = 0;
    }
    for (int c = tid; c < k; c += BLOCK) {
      m1[c] = 0;
      c1[c] = 0;
      m2[c] = 0;
    }
    __syncthreads();
    const int nnz = a.row_ptr[n];
    for (int e = tid; e < nnz; e += BLOCK)
      atomicAdd(reinterpret_cast<uint32_t*>(gam) + ((a.erow[e] * k + (int)(cg[a.col_idx[e]] & 0xffffu)) >> 1),
                (a.erow[e] * k + (int)(cg[a.col_idx[e]] & 0xffffu)) & 1 ? 0x10000u : 1u);
    for (int v = tid; v < n; v += BLOCK) atomicMax(&m1[cg[v] & 0xffffu], (uint32_t)w[v]);
    __syncthreads();
    uint32_t cs2 = 0;
    for (int v = tid; v < n; v += BLOCK) {
      const uint32_t c = cg[v] & 0xffffu;
      const uint32_t g = gam[v * k + (int)c];
      cg[v] = c | (g << 16);
      cs2 += g;
      if ((uint32_t)w[v] == m1[c]) atomicAdd(&c1[c], 1u);
      else atomicMax(&m2[c], (uint32_t)w[v]);
    }
    cs2 = wave_sum_u32(cs2);
    uint32_t fwp = 0;
    for (int c = tid; c < k; c += BLOCK) fwp += m1[c];
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
        for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffffu);
    }

    for (int it = 0; it < a.T; ++it, ++t) {
      const int par = (t & 1) * NW;
      if (wid == 0 && t - Lbase >= 64) {
        Lbase = t;
        Lreg = lemire(philox_w0(ind, (uint32_t)(t + lane), 0u, kDomTenure, a.key), (uint32_t)a.ten_rand);
      }
      const int64_t asp = G_best - G - 1;
      // ---- scan every one-move (v, c), c != col v
      uint64_t bd = ~0ull;
      uint32_t bidx = 0xffffffffu, bcnt = 0, s0 = 0, s1 = 0;
      {
        int i = i0, c = c0;
        for (int j = tid; j < nk; j += BLOCK) {
          const int v = i;
          const uint32_t x = cg[v];
          const int cv = (int)(x & 0xffffu);
          if (c != cv) {
            const uint32_t wv = (uint32_t)w[v];
            const uint32_t am1 = m1[cv];
            const uint32_t m_after = (wv < am1 || c1[cv] > 1u) ? am1 : m2[cv];
            const uint32_t bm1 = m1[c];
            const int64_t dfw = (int64_t)(max(bm1, wv) - bm1) + ((int64_t)m_after - (int64_t)am1);
            const int64_t dcf = (int64_t)gam[v * k + c] - (int64_t)(x >> 16);
            const int64_t dg = (dfw << S) + phi * dcf;
            if (frozen[v] <= t || dg <= asp) {
              const uint64_t key = (uint64_t)dg + kGBias;
              const uint32_t idx = ((uint32_t)v << 16) | (uint32_t)c;
              if (key < bd) {
                bd = key;
                bidx = idx;
                bcnt = 1;
                s0 = idx;
              } else if (key == bd) {
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
      {
        const uint64_t wk = wave_min_u64(bd);
        const uint64_t wi = wave_min_u64(bd == wk ? (uint64_t)bidx : ~0ull);
        const uint32_t wc = wave_sum_u32(bd == wk ? bcnt : 0u);
        if (lane == 0) {
          rkey[par + wid] = wk;
          ridx[par + wid] = (uint32_t)wi;
          rcnt[par + wid] = wc;
        }
      }
      __syncthreads();
      uint64_t gk = rkey[par];
#pragma unroll
      for (int q = 1; q < NW; ++q) gk = umin64(gk, rkey[par + q]);
      uint32_t gcnt = 0, gidx = 0xffffffffu;
#pragma unroll
      for (int q = 0; q < NW; ++q)
        if (rkey[par + q] == gk) {
          gcnt += rcnt[par + q];
          gidx = min(gidx, ridx[par + q]);
        }
      if (gk == ~0ull) {  // nothing admissible
        if (wid == 0) {
          ++st_noops;
          fp = fnv_step(fp, 0xffffu, 0xffffu, (int32_t)(G >> S));
        }
        continue;
      }
      uint32_t win = gidx;
      if (gcnt > 1) {
        uint64_t hk = ~0ull;
        if (bd == gk) {
          auto hkey = [&](uint32_t idx) -> uint64_t {
            return ((uint64_t)philox_w0(ind, (uint32_t)t, idx >> 16, idx & 0xffffu, a.key) << 32) | idx;
          };
          if (bcnt <= 2) {
            hk = hkey(s0);
            if (bcnt == 2) hk = umin64(hk, hkey(s1));
          } else {
            int i = i0, c = c0;
            for (int j = tid; j < nk; j += BLOCK) {
              const int v = i;
              const uint32_t x = cg[v];
              const int cv = (int)(x & 0xffffu);
              if (c != cv) {
                const uint32_t wv = (uint32_t)w[v];
                const uint32_t am1 = m1[cv];
                const uint32_t m_after = (wv < am1 || c1[cv] > 1u) ? am1 : m2[cv];
                const uint32_t bm1 = m1[c];
                const int64_t dfw = (int64_t)(max(bm1, wv) - bm1) + ((int64_t)m_after - (int64_t)am1);
                const int64_t dcf = (int64_t)gam[v * k + c] - (int64_t)(x >> 16);
                const int64_t dg = (dfw << S) + phi * dcf;
                if ((uint64_t)dg + kGBias == gk && (frozen[v] <= t || dg <= asp))
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
        if (lane == 0) rhash[par + wid] = hk;
        __syncthreads();
        uint64_t gh = rhash[par];
#pragma unroll
        for (int q = 1; q < NW; ++q) gh = umin64(gh, rhash[par + q]);
        win = (uint32_t)gh;
      }
      // ---- apply (wave 0)
      const int vs = (int)(win >> 16), cs = (int)(win & 0xffffu);
      const int64_t dg = (int64_t)(gk - kGBias);
      if (wid == 0) {
        const uint32_t xs = cg[vs];
        const int old = (int)(xs & 0xffffu);
        const int64_t dcs = (int64_t)gam[vs * k + cs] - (int64_t)(xs >> 16);
        const int rs = a.row_ptr[vs], re = a.row_ptr[vs + 1];
        for (int e = rs + lane; e < re; e += kWave) {
          const int u = a.col_idx[e];
          const int io = u * k + old, ic = u * k + cs;
          atomicAdd(reinterpret_cast<uint32_t*>(gam) + (io >> 1), (io & 1) ? 0xffff0000u : 0xffffffffu);
          atomicAdd(reinterpret_cast<uint32_t*>(gam) + (ic >> 1), (ic & 1) ? 0x10000u : 1u);
          const uint32_t xu = cg[u];
          const int cu = (int)(xu & 0xffffu);
          if (cu == old) cg[u] = xu - 0x10000u;
          else if (cu == cs) cg[u] = xu + 0x10000u;
        }
        if (lane == 0) {
          cg[vs] = (uint32_t)cs | ((uint32_t)gam[vs * k + cs] << 16);
          frozen[vs] = t + (int)readlane(Lreg, t - Lbase) + a.frz;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // class statistics of the two classes touched
        Cls ca{0, 0, 0}, cb{0, 0, 0};
        for (int v = lane; v < n; v += kWave) {
          const int c = (int)(cg[v] & 0xffffu);
          const Cls one{(uint32_t)w[v], 1u, 0u};
          if (c == old) ca = cls_join(ca, one);
          else if (c == cs) cb = cls_join(cb, one);
        }
        ca = wave_cls(ca);
        cb = wave_cls(cb);
        if (lane == 0) {
          m1[old] = ca.m1;
          c1[old] = ca.c1;
          m2[old] = ca.m2;
          m1[cs] = cb.m1;
          c1[cs] = cb.c1;
          m2[cs] = cb.m2;
        }
        if (lane == 0) s_dcs = (int32_t)dcs;
        ++st_moves;
        st_deg += (uint64_t)(re - rs);
        st_ties += gcnt > 1;
      }
      __syncthreads();
      conf += s_dcs;
      G += dg;
      fw = (G - phi * conf) >> S;
      if (wid == 0) fp = fnv_step(fp, (uint32_t)vs, (uint32_t)cs, (int32_t)(G >> S));
      const bool new_best_g = G < G_best;
      const bool new_legal = conf == 0 && fw < best_legal;
      if (new_best_g) {
        G_best = G;
        conf_best = conf;
        for (int v = tid; v < n; v += BLOCK) bestg[v] = (int16_t)(cg[v] & 0xffffu);
      }
      if (new_legal) {
        best_legal = fw;
        if (wid == 0)
          for (int v = lane; v < n; v += kWave) gcol[v] = (int16_t)(cg[v] & 0xffffu);
      }
    }
    // next round starts from bestg (already in LDS); adapt phi
    const bool legal = conf_best == 0;
    st_legal_rounds += legal;
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
        s[0] = (int64_t)st_moves;
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
             (int32_t)((int64_t)p->frz_num * g->n / p->frz_den), p->shift, p->ind_base, g->max_w};
  hipStream_t s = (hipStream_t)stream;
  switch (block) {
    case 64: return launch_wvcp<64>(a, pop, lds, s);
    case 128: return launch_wvcp<128>(a, pop, lds, s);
    case 256: return launch_wvcp<256>(a, pop, lds, s);
    default: return launch_wvcp<512>(a, pop, lds, s);
  }
}
