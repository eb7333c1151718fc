// Distance-based population management (Sections 2.4 to 2.6 of the paper):
// the approximate set-theoretic partition distance between colourings, the
// quality-ordered population update under a minimum spacing, and the K
// nearest neighbours used for parent matching.
//
// Partition distance.  For colourings A and B of the same n vertices,
// M[c][d] = |A_c & B_d|.  One greedy pass takes the classes of A by
// decreasing size (ties by index) and gives each the free class of B with
// the largest positive overlap (ties by index); a second pass swaps the
// roles; D~ = n - the larger matched total.  Both passes are matchings, so
// D~ is an upper bound of the exact distance (n - a maximum matching), and
// it is exact on close partitions.
//
// One wave per pair: the k x k overlap counts are 16-bit halves of 32-bit
// LDS words (k^2 / 2 words per wave), filled by one LDS atomic per vertex.
// A greedy step is one LDS read per owned column (lane c owns classes c,
// c + 64, ...) and a DPP wave maximum of (overlap << 16 | 0xffff - class);
// the two passes run interleaved, as two independent chains.  The class
// orders are computed once per colouring by a small kernel first.
#include "dlm_common.h"

namespace dlm {

constexpr int kMaxDistK = 256;

// rec[r] = int16[k + 2]: the classes of row r by decreasing size (ties by
// index), then the number of non-empty classes, or -1 there when a colour
// of the row lies outside [0, k).
__global__ __launch_bounds__(64) void class_order_kernel(const int16_t* __restrict__ rows, int32_t n, int32_t k,
                                                         int16_t* __restrict__ rec) {
  __shared__ uint32_t size[kMaxDistK];
  const int lane = threadIdx.x;
  const int16_t* row = rows + (size_t)blockIdx.x * n;
  for (int c = lane; c < k; c += kWave) size[c] = 0u;
  __syncthreads();
  uint32_t bad = 0u;
  for (int v = lane; v < n; v += kWave) {
    const int c = row[v];
    if (c < 0 || c >= k)
      bad = 1u;
    else
      atomicAdd(&size[c], 1u);
  }
  __syncthreads();
  int16_t* out = rec + (size_t)blockIdx.x * (k + 2);
  uint32_t nonempty = 0u;
  for (int c = lane; c < k; c += kWave) {
    const uint32_t sc = size[c];
    uint32_t rank = 0u;
    for (int d = 0; d < k; ++d) {
      const uint32_t sd = size[d];
      rank += (sd > sc) || (sd == sc && d < c);
    }
    out[rank] = (int16_t)c;
    nonempty += sc > 0u;
  }
  nonempty = wave_sum_u32(nonempty);
  bad = wave_max_u32(bad);
  if (lane == 0) {
    out[k] = bad ? (int16_t)-1 : (int16_t)nonempty;
    out[k + 1] = 0;
  }
}

// wave maxima of two values at once: four in-row DPP steps, then
// row_bcast:15 and row_bcast:31 carry the row maxima up to lane 63 (one
// readlane instead of four).  The two chains alternate, so each one's DPP
// steps fill the other's wait states.
__device__ __forceinline__ void wave_max2(uint32_t& a, uint32_t& b) {
  a = max(a, dpp_mov<dpp::kXor1>(a));
  b = max(b, dpp_mov<dpp::kXor1>(b));
  a = max(a, dpp_mov<dpp::kXor2>(a));
  b = max(b, dpp_mov<dpp::kXor2>(b));
  a = max(a, dpp_mov<dpp::kHalfMirror>(a));
  b = max(b, dpp_mov<dpp::kHalfMirror>(b));
  a = max(a, dpp_mov<dpp::kMirror>(a));
  b = max(b, dpp_mov<dpp::kMirror>(b));
  // rows 1 and 3 take lane 15 of the row below, then rows 2 and 3 take lane
  // 31; lanes outside the row mask keep the old operand, 0, which max ignores
  a = max(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x142, 0xa, 0xf, false));
  b = max(b, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)b, 0x142, 0xa, 0xf, false));
  a = max(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x143, 0xc, 0xf, false));
  b = max(b, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)b, 0x143, 0xc, 0xf, false));
  a = readlane(a, 63);
  b = readlane(b, 63);
}

// words of one wave's overlap table, a multiple of 4 (cleared with 16-byte stores)
__host__ __device__ inline uint32_t hist_words(int k) { return (((uint32_t)(k * k) + 1u) / 2u + 3u) & ~3u; }

template <int KW>
__global__ __launch_bounds__(256) void distance_kernel(const int16_t* __restrict__ A, const int16_t* __restrict__ B,
                                                       const int16_t* __restrict__ recA,
                                                       const int16_t* __restrict__ recB, int32_t nb, int32_t m_tri,
                                                       int32_t n, int32_t k, int64_t npairs, int32_t wpb,
                                                       int32_t* __restrict__ out, int64_t ld) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t words = hist_words(k);
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem) + (size_t)wid * words;
  const uint16_t* h16 = reinterpret_cast<const uint16_t*>(hist);
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  for (int64_t q = (int64_t)blockIdx.x * wpb + wid; q < npairs; q += nwaves) {
    // the triangle form walks the full square in the block form's order and
    // skips j <= i: consecutive workgroups (spread over the XCDs in turn)
    // then keep taking the same residues of j, so each XCD's L2 holds a
    // fixed share of the rows
    const int i = (int)(q / nb);
    const int j = (int)(q - (int64_t)i * nb);
    if (m_tri > 0 && j <= i) continue;
    const int16_t* ra = recA + (size_t)i * (k + 2);
    const int16_t* rb = recB + (size_t)j * (k + 2);
    const int nea = ra[k], neb = rb[k];
    int32_t d = -1;
    if (nea >= 0 && neb >= 0) {
      for (uint32_t w = (uint32_t)lane; w < words / 4u; w += kWave)
        reinterpret_cast<uint4*>(hist)[w] = make_uint4(0u, 0u, 0u, 0u);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int16_t* a = A + (size_t)i * n;
      const int16_t* b = B + (size_t)j * n;
      for (int v = lane; v < n; v += kWave) {
        const uint32_t e = (uint32_t)a[v] * (uint32_t)k + (uint32_t)b[v];
        atomicAdd(&hist[e >> 1], (e & 1u) ? 0x10000u : 1u);  // a count stays below 2^15: no carry
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // class orders in registers: lane holds entries lane, lane + 64, ...
      int oa[KW], ob[KW];
      // per owned class c = lane + 64 w: 0xffff - c while the class is free in
      // that pass (all ones then), 0 once matched or when c >= k
      // per owned class c = lane + 64 w: lowc = 0xffff - c, and a byte
      // selector that builds the key (overlap << 16 | lowc) in one v_perm_b32
      // while the class is free in that pass, or 0 once matched or for c >= k
      constexpr uint32_t kSelKey = 0x05040100u, kSelZero = 0x0c0c0c0cu;
      uint32_t lowc[KW], selB[KW], selA[KW];
#pragma unroll
      for (int w = 0; w < KW; ++w) {
        const int t = lane + kWave * w;
        oa[w] = t < k ? ra[t] : 0;
        ob[w] = t < k ? rb[t] : 0;
        lowc[w] = 0xffffu - (uint32_t)t;
        selB[w] = selA[w] = t < k ? kSelKey : kSelZero;
      }
      // every lane loaded the same counts: make that visible to the compiler
      const int na_ = __builtin_amdgcn_readfirstlane(nea), nb_ = __builtin_amdgcn_readfirstlane(neb);
      uint32_t sab = 0u, sba = 0u;
      auto order_at = [&](const int (&o)[KW], int t) {
        uint32_t x = 0u;
#pragma unroll
        for (int w = 0; w < KW; ++w)
          if (w == t / kWave) x = readlane((uint32_t)o[w], t % kWave);
        return x;
      };
      // pass over A: row ro of M, lanes own the columns (classes of B); pass
      // over B: column co of M, lanes own the rows (classes of A).  A key with
      // overlap 0 never beats one with a positive overlap, so a zero maximum
      // overlap means "no match".
      auto key_a = [&](uint32_t ro) {
        uint32_t ka = 0u;
#pragma unroll
        for (int w = 0; w < KW; ++w) {
          const int c0 = lane + kWave * w;
          const uint32_t c = (uint32_t)(c0 < k ? c0 : k - 1);  // in-table address; the selector drops the value
          ka = max(ka, __builtin_amdgcn_perm((uint32_t)h16[ro * (uint32_t)k + c], lowc[w], selB[w]));
        }
        return ka;
      };
      auto key_b = [&](uint32_t co) {
        uint32_t kb = 0u;
#pragma unroll
        for (int w = 0; w < KW; ++w) {
          const int c0 = lane + kWave * w;
          const uint32_t c = (uint32_t)(c0 < k ? c0 : k - 1);
          kb = max(kb, __builtin_amdgcn_perm((uint32_t)h16[c * (uint32_t)k + co], lowc[w], selA[w]));
        }
        return kb;
      };
      auto take = [&](uint32_t m, uint32_t& sum, uint32_t (&sel)[KW]) {
        if (m >> 16) {
          sum += m >> 16;
          const uint32_t c = 0xffffu - (m & 0xffffu);
#pragma unroll
          for (int w = 0; w < KW; ++w)
            if (c == (uint32_t)(lane + kWave * w)) sel[w] = kSelZero;
        }
      };
      const int both = na_ < nb_ ? na_ : nb_;
      int t = 0;
      for (; t < both; ++t) {  // both passes, their maxima interleaved
        uint32_t ka = key_a(order_at(oa, t)), kb = key_b(order_at(ob, t));
        wave_max2(ka, kb);
        take(ka, sab, selB);
        take(kb, sba, selA);
      }
      for (; t < na_; ++t) {  // the longer pass alone
        uint32_t ka = key_a(order_at(oa, t)), kz = 0u;
        wave_max2(ka, kz);
        take(ka, sab, selB);
      }
      for (; t < nb_; ++t) {
        uint32_t kb = key_b(order_at(ob, t)), kz = 0u;
        wave_max2(kb, kz);
        take(kb, sba, selA);
      }
      d = n - (int32_t)(sab > sba ? sab : sba);
    }
    if (lane == 0) out[(size_t)i * ld + j] = d;
  }
}

__global__ __launch_bounds__(256) void diag_zero_kernel(int32_t m, int32_t* __restrict__ out, int64_t ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[(size_t)i * ld + i] = 0;
}

// out[i][j] = out[j][i] for i > j: 32 x 32 tiles of the strict upper
// triangle read by rows into LDS and written transposed by rows, so both
// sides stay coalesced
__global__ __launch_bounds__(256) void mirror_kernel(int32_t m, int32_t* __restrict__ out, int64_t ld) {
  __shared__ int32_t tile[32][33];
  const int ti = blockIdx.y, tj = blockIdx.x;  // destination tile (ti, tj), ti >= tj
  if (ti < tj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int r = ty; r < 32; r += 8) {  // source tile (tj, ti): rows tj*32 + r, columns ti*32 + tx
    const int si = tj * 32 + r, sj = ti * 32 + tx;
    tile[r][tx] = (si < m && sj < m && si < sj) ? out[(size_t)si * ld + sj] : 0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {  // destination rows ti*32 + r, columns tj*32 + tx
    const int di = ti * 32 + r, dj = tj * 32 + tx;
    if (di < m && dj < m && di > dj) out[(size_t)di * ld + dj] = tile[tx][r];
  }
}

// ---------------------------------------------------------------------------
// population update: the pool's quality order (f ascending, index ascending)
// by counting, then one workgroup takes it greedily
__global__ __launch_bounds__(256) void pool_rank_kernel(const int32_t* __restrict__ fa, int32_t na,
                                                        const int32_t* __restrict__ fb, int32_t nb,
                                                        int32_t* __restrict__ order) {
  __shared__ uint64_t tile[1024];
  const int total = na + nb;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  auto key = [&](int x) {
    const int32_t f = x < na ? fa[x] : fb[x - na];
    return ((uint64_t)((uint32_t)f ^ 0x80000000u) << 32) | (uint32_t)x;  // signed order of f, then index
  };
  const uint64_t mine = i < total ? key(i) : ~0ull;
  uint32_t rank = 0u;
  for (int base = 0; base < total; base += 1024) {
    const int cnt = min(1024, total - base);
    __syncthreads();
    for (int x = threadIdx.x; x < cnt; x += blockDim.x) tile[x] = key(base + x);
    __syncthreads();
    for (int x = 0; x < cnt; ++x) rank += tile[x] < mine;
  }
  if (i < total) order[rank] = i;
}

constexpr int kMaxPool = 1 << 16;

// The update under a minimum spacing goes through the quality order in
// chunks of kChunk members.  Many workgroups screen a chunk's members
// against the members taken in earlier chunks; then one workgroup settles
// the chunk's survivors among themselves, in order, from a conflict bit
// matrix in LDS.  A member joins exactly when it would in the one-at-a-time
// walk: it is too close to no member taken before it.  order[r] keeps the
// pool index in its low bits, kBlocked on a member too close to an earlier
// chunk's member, kTaken on a member that joined.  n_spaced holds the running
// count between the launches.
constexpr int kChunk = 512;
constexpr int32_t kIndexMask = 0x1ffff, kBlocked = 1 << 29, kTaken = 1 << 30;

__device__ inline int32_t pool_dist(const int32_t* __restrict__ dist, int64_t ld, int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return dist[(size_t)lo * ld + hi];  // the upper triangle holds the pool's distances
}

// one workgroup per member r0 + blockIdx.x, against pick[0 .. count)
__global__ __launch_bounds__(256) void spacing_screen_kernel(int32_t* __restrict__ order, int32_t r0,
                                                             const int32_t* __restrict__ dist, int64_t ld,
                                                             int32_t keep, int32_t spacing,
                                                             const int32_t* __restrict__ pick,
                                                             const int32_t* __restrict__ n_spaced) {
  const int count = *n_spaced;
  if (count >= keep) return;
  const int r = r0 + blockIdx.x;
  const int c = order[r] & kIndexMask;
  int hit = 0;
#pragma unroll 4
  for (int s = threadIdx.x; s < count; s += blockDim.x) hit |= pool_dist(dist, ld, c, pick[s]) <= spacing;
  if (__syncthreads_or(hit) && threadIdx.x == 0) order[r] = c | kBlocked;
}

// the chunk [r0, r0 + cnt): its unblocked members in order, each joining
// unless too close to one of them that joined before it, until keep
__global__ __launch_bounds__(1024) void spacing_resolve_kernel(int32_t* __restrict__ order, int32_t r0, int32_t cnt,
                                                               const int32_t* __restrict__ dist, int64_t ld,
                                                               int32_t keep, int32_t spacing, int32_t first,
                                                               int32_t* __restrict__ pick,
                                                               int32_t* __restrict__ n_spaced) {
  __shared__ uint32_t conf[kChunk][kChunk / 32];  // row b, bit a < b: survivors a and b too close
  __shared__ int32_t surv[kChunk];                // pool index of each survivor, in order
  __shared__ int16_t spos[kChunk];                // its position in the chunk
  __shared__ int32_t wave_total[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int count0 = first ? 0 : *n_spaced;
  if (count0 >= keep) {
    if (first && tid == 0) *n_spaced = 0;
    return;
  }
  const int32_t v = tid < cnt ? order[r0 + tid] : kBlocked;
  const bool alive = !(v & kBlocked);
  const uint64_t m = __ballot(alive);
  if (lane == 0) wave_total[wave] = __popcll(m);
  __syncthreads();
  int before = 0, S = 0;
  for (int w = 0; w < 16; ++w) {
    const int t = wave_total[w];
    before += w < wave ? t : 0;
    S += t;
  }
  if (alive) {
    const int at = before + __popcll(m & ((1ull << lane) - 1ull));
    surv[at] = v & kIndexMask;
    spos[at] = (int16_t)tid;
  }
  __syncthreads();
  const int W = (S + 31) / 32;
  for (int task = tid; task < S * W; task += blockDim.x) {
    const int b = task / W, w = task % W;
    uint32_t word = 0u;
    if (32 * w < b) {
      // all 32 loads are issued before the first result is needed: a >= b
      // reads the pair (surv[0], surv[b]) and is masked off
      const int cb = surv[b];
      int32_t d[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        const int a = 32 * w + j;
        d[j] = pool_dist(dist, ld, surv[a < b ? a : 0], cb);
      }
#pragma unroll
      for (int j = 0; j < 32; ++j) word |= (uint32_t)(32 * w + j < b && d[j] <= spacing) << j;
    }
    conf[b][w] = word;
  }
  __syncthreads();
  if (wave == 0) {
    uint32_t acc = 0u;  // lane w < W: word w of the survivors that joined
    int count = count0;
    for (int b = 0; b < S && count < keep; ++b) {
      const uint32_t row = lane < W ? conf[b][lane] : 0u;
      if (__ballot((row & acc) != 0u) == 0ull) {
        if (lane == (b >> 5)) acc |= 1u << (b & 31);
        if (lane == 0) {
          pick[count] = surv[b];
          order[r0 + spos[b]] = surv[b] | kTaken;
        }
        ++count;
      }
    }
    if (lane == 0) *n_spaced = count;
  }
}

// places left after the spacing walk: the best members not taken, in order
__global__ __launch_bounds__(1024) void spacing_fill_kernel(const int32_t* __restrict__ order, int32_t total,
                                                            int32_t keep, int32_t first, int32_t* __restrict__ pick,
                                                            int32_t* __restrict__ n_spaced) {
  __shared__ int32_t wave_total[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int count = first ? 0 : *n_spaced;
  if (first && tid == 0) *n_spaced = 0;
  for (int base = 0; base < total && count < keep; base += blockDim.x) {
    const int r = base + tid;
    const int32_t v = r < total ? order[r] : kTaken;
    const bool want = !(v & kTaken);
    const uint64_t m = __ballot(want);
    if (lane == 0) wave_total[wave] = __popcll(m);
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
      const int t = wave_total[w];
      before += w < wave ? t : 0;
      all += t;
    }
    if (want) {
      const int at = count + before + __popcll(m & ((1ull << lane) - 1ull));
      if (at < keep) pick[at] = v & kIndexMask;
    }
    count += all;
    __syncthreads();  // wave_total is written again
  }
}

// out[a][b] = dist[min(pa, pb)][max(pa, pb)] for a != b, 0 on the diagonal
__global__ __launch_bounds__(256) void gather_dist_kernel(const int32_t* __restrict__ dist, int64_t ld,
                                                          const int32_t* __restrict__ idx, int32_t count,
                                                          int32_t* __restrict__ out, int64_t ld_out) {
  const int a = blockIdx.x;
  const int pa = idx[a];
  for (int b = threadIdx.x; b < count; b += blockDim.x) {
    const int pb = idx[b];
    const int lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
    out[(size_t)a * ld_out + b] = a == b ? 0 : dist[(size_t)lo * ld + hi];
  }
}

// row r of out = pool member pick[r] (a row of ra for indices below na, else
// of rb); an index outside the pool gives a row of -1 and score -1
__global__ __launch_bounds__(256) void gather_pool_kernel(const int16_t* __restrict__ ra, const int32_t* __restrict__ fa,
                                                          int32_t na, const int16_t* __restrict__ rb,
                                                          const int32_t* __restrict__ fb, int32_t nb, int32_t n,
                                                          const int32_t* __restrict__ pick, int16_t* __restrict__ out,
                                                          int32_t* __restrict__ fout) {
  const int64_t r = blockIdx.x;
  const int s = pick[r];
  const bool ok = s >= 0 && s < na + nb;
  const int16_t* src = !ok ? nullptr : (s < na ? ra + (size_t)s * n : rb + (size_t)(s - na) * n);
  for (int v = threadIdx.x; v < n; v += blockDim.x) out[(size_t)r * n + v] = ok ? src[v] : (int16_t)-1;
  if (threadIdx.x == 0) fout[r] = !ok ? -1 : (s < na ? fa[s] : fb[s - na]);
}

// K nearest of row i: K extractions of the smallest key dist << 16 | j
// above the last one taken (keys are distinct: j is part of them)
__global__ __launch_bounds__(256) void nearest_kernel(const int32_t* __restrict__ dist, int64_t ld, int32_t p,
                                                      int32_t K, int32_t* __restrict__ nn) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= p) return;  // whole waves leave together
  const int32_t* row = dist + (size_t)i * ld;
  uint32_t last = 0u;
  bool first = true;
  for (int t = 0; t < K; ++t) {
    uint32_t best = 0xffffffffu;
    for (int j = lane; j < p; j += kWave) {
      const uint32_t key = ((uint32_t)row[j] << 16) | (uint32_t)j;
      if (j != i && (first || key > last)) best = min(best, key);
    }
    last = wave_min_u32(best);
    first = false;
    if (lane == 0) nn[(size_t)i * K + t] = (int32_t)(last & 0xffffu);
  }
}

}  // namespace dlm

using namespace dlm;

static int distance_pairs(const int16_t* a, const int16_t* b, const int16_t* recA, const int16_t* recB, int32_t na,
                          int32_t nb, int32_t tri, int32_t n, int32_t k, int64_t npairs, int32_t* out, int64_t ld,
                          hipStream_t s);

extern "C" {

int dlm_partition_distance(int32_t n, int32_t k, const int16_t* a, int32_t na, const int16_t* b, int32_t nb,
                           int32_t tri, int32_t* out, int64_t ld, void* workspace, void* stream) {
  if (n < 1 || n > 32767 || k < 1 || k > kMaxDistK || na < 0 || nb < 0 || tri < 0 || tri > 2)
    return set_error(DLM_E_INVAL, "dlm_partition_distance: n=%d k=%d na=%d nb=%d tri=%d", n, k, na, nb, tri);
  if (tri && (a != b || na != nb))
    return set_error(DLM_E_INVAL, "dlm_partition_distance: tri needs the same rows on both sides");
  if (ld < nb) return set_error(DLM_E_INVAL, "dlm_partition_distance: ld=%lld < nb=%d", (long long)ld, nb);
  if (na == 0 || nb == 0) return DLM_OK;
  if (!a || !b || !out || !workspace) return set_error(DLM_E_INVAL, "dlm_partition_distance: null buffer");
  hipStream_t s = (hipStream_t)stream;
  int16_t* recA = (int16_t*)workspace;
  int16_t* recB = tri ? recA : recA + (size_t)na * (k + 2);
  hipLaunchKernelGGL(class_order_kernel, dim3(na), dim3(kWave), 0, s, a, n, k, recA);
  DLM_HIP(hipGetLastError());
  if (!tri) {
    hipLaunchKernelGGL(class_order_kernel, dim3(nb), dim3(kWave), 0, s, b, n, k, recB);
    DLM_HIP(hipGetLastError());
  }
  const int64_t npairs = tri ? (na > 1 ? (int64_t)na * na : 0) : (int64_t)na * nb;  // triangle: slots of the square
  if (tri) {
    hipLaunchKernelGGL(diag_zero_kernel, dim3((na + 255) / 256), dim3(256), 0, s, na, out, ld);
    DLM_HIP(hipGetLastError());
  }
  if (npairs == 0) return DLM_OK;
  const int rc = distance_pairs(a, b, recA, recB, na, nb, tri, n, k, npairs, out, ld, s);
  if (rc != DLM_OK || tri != 1) return rc;
  const unsigned tiles = (unsigned)((na + 31) / 32);
  hipLaunchKernelGGL(mirror_kernel, dim3(tiles, tiles), dim3(256), 0, s, na, out, ld);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

static int distance_pairs(const int16_t* a, const int16_t* b, const int16_t* recA, const int16_t* recB, int32_t na,
                          int32_t nb, int32_t tri, int32_t n, int32_t k, int64_t npairs, int32_t* out, int64_t ld,
                          hipStream_t s) {
  const uint32_t wave_bytes = 4u * hist_words(k);
  int wpb = (int)(65536u / wave_bytes);  // up to 4 waves and 64 KB of LDS per workgroup
  wpb = wpb < 1 ? 1 : (wpb > 4 ? 4 : wpb);
  const size_t lds = (size_t)wpb * wave_bytes;
  const int64_t blocks_needed = (npairs + wpb - 1) / wpb;
  const int64_t cap = (int64_t)device_cu_count() * 64;
  const unsigned grid = (unsigned)(blocks_needed < cap ? blocks_needed : cap);
  const int kw = (k + kWave - 1) / kWave;
  auto launch = [&](auto kern) -> int {
    DLM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * wpb), lds, s, a, b, recA, recB, nb, tri ? na : 0, n, k,
                       npairs, wpb, out, ld);
    DLM_HIP(hipGetLastError());
    return DLM_OK;
  };
  switch (kw) {
    case 1: return launch(distance_kernel<1>);
    case 2: return launch(distance_kernel<2>);
    case 3: return launch(distance_kernel<3>);
    default: return launch(distance_kernel<4>);
  }
}

int dlm_spacing_update(const int32_t* fa, int32_t na, const int32_t* fb, int32_t nb, const int32_t* dist, int64_t ld,
                       int32_t keep, int32_t spacing, int32_t* pick, int32_t* n_spaced, void* workspace,
                       void* stream) {
  const int64_t total = (int64_t)na + nb;
  if (na < 0 || nb < 0 || total > kMaxPool || keep < 0 || keep > total || ld < total)
    return set_error(DLM_E_INVAL, "dlm_spacing_update: na=%d nb=%d keep=%d ld=%lld", na, nb, keep, (long long)ld);
  if ((keep > 0 && !pick) || !n_spaced || (total > 0 && (!dist || !workspace)) || (na > 0 && !fa) || (nb > 0 && !fb))
    return set_error(DLM_E_INVAL, "dlm_spacing_update: null buffer");
  hipStream_t s = (hipStream_t)stream;
  int32_t* order = (int32_t*)workspace;
  if (total == 0) {
    hipLaunchKernelGGL(spacing_fill_kernel, dim3(1), dim3(1024), 0, s, order, 0, keep, 1, pick, n_spaced);
    DLM_HIP(hipGetLastError());
    return DLM_OK;
  }
  hipLaunchKernelGGL(pool_rank_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, fa, na, fb, nb, order);
  DLM_HIP(hipGetLastError());
  for (int32_t r0 = 0; r0 < total; r0 += kChunk) {
    const int32_t cnt = (int32_t)std::min<int64_t>(kChunk, total - r0);
    if (r0 > 0)
      hipLaunchKernelGGL(spacing_screen_kernel, dim3((unsigned)cnt), dim3(256), 0, s, order, r0, dist, ld, keep,
                         spacing, pick, n_spaced);
    hipLaunchKernelGGL(spacing_resolve_kernel, dim3(1), dim3(1024), 0, s, order, r0, cnt, dist, ld, keep, spacing,
                       (int32_t)(r0 == 0), pick, n_spaced);
  }
  hipLaunchKernelGGL(spacing_fill_kernel, dim3(1), dim3(1024), 0, s, order, (int32_t)total, keep, 0, pick, n_spaced);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_gather_distances(const int32_t* dist, int64_t ld, const int32_t* idx, int32_t count, int32_t* out,
                         int64_t ld_out, void* stream) {
  if (count < 0 || ld_out < count) return set_error(DLM_E_INVAL, "dlm_gather_distances: count=%d", count);
  if (count == 0) return DLM_OK;
  if (!dist || !idx || !out) return set_error(DLM_E_INVAL, "dlm_gather_distances: null buffer");
  hipLaunchKernelGGL(gather_dist_kernel, dim3(count), dim3(256), 0, (hipStream_t)stream, dist, ld, idx, count, out,
                     ld_out);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_gather_pool(const int16_t* ra, const int32_t* fa, int32_t na, const int16_t* rb, const int32_t* fb,
                    int32_t nb, int32_t n, const int32_t* pick, int32_t count, int16_t* out, int32_t* fout,
                    void* stream) {
  if (na < 0 || nb < 0 || n < 1 || count < 0)
    return set_error(DLM_E_INVAL, "dlm_gather_pool: na=%d nb=%d n=%d count=%d", na, nb, n, count);
  if (count == 0) return DLM_OK;
  if (!pick || !out || !fout || (na > 0 && (!ra || !fa)) || (nb > 0 && (!rb || !fb)))
    return set_error(DLM_E_INVAL, "dlm_gather_pool: null buffer");
  hipLaunchKernelGGL(gather_pool_kernel, dim3(count), dim3(256), 0, (hipStream_t)stream, ra, fa, na, rb, fb, nb, n,
                     pick, out, fout);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

int dlm_nearest(const int32_t* dist, int64_t ld, int32_t p, int32_t K, int32_t* nn, void* stream) {
  if (p < 0 || p > kMaxPool || K < 0 || (p > 0 && K > p - 1) || ld < p)
    return set_error(DLM_E_INVAL, "dlm_nearest: p=%d K=%d ld=%lld", p, K, (long long)ld);
  if (p == 0 || K == 0) return DLM_OK;
  if (!dist || !nn) return set_error(DLM_E_INVAL, "dlm_nearest: null buffer");
  hipLaunchKernelGGL(nearest_kernel, dim3((p + 3) / 4), dim3(256), 0, (hipStream_t)stream, dist, ld, p, K, nn);
  DLM_HIP(hipGetLastError());
  return DLM_OK;
}

}  // extern "C"
