// BF16 x BF16 -> FP32 products for the colour-invariant network (the
// per-layer products of Section 2.3: Z = X Lambda, U = R Gamma, their weight
// gradients and their input gradients), on gfx950's 32x32x16 BF16 MFMA.
//
//   C[m][n] = sum_k A(m, k) B(k, n)      (C row-major FP32, pitch ldc; beta = 0)
//
// A(m, k) is A[m * sa + k] when AK (K contiguous) else A[k * sa + m];
// B(k, n) is B[n * sb + k] when BK (K contiguous) else B[k * sb + n].
// The network's three forms:
//   rows:  C = X W        A = X [rows][inner] (AK), B = W [inner][cols] (!BK)
//   at:    C = X^T D      A = X [rows][inner] (!AK, K = rows), B = D [rows][cols] (!BK)
//   wt:    C = D W^T      A = D [rows][cols] (AK), B = W [inner][cols] (BK)
//
// A workgroup of four waves computes a T x T tile of C (T = 64 TM, TM = 1,
// 2 or 4); wave w owns the quarter (w / 2, w % 2), TM x TM MFMA tiles of
// 32 x 32, with the accumulators in registers for the whole K loop.  Per K
// step of 64 both operand tiles are staged in LDS K-contiguous ([row][k],
// rows padded to 72 values so that the 16-byte operand reads of 16 lanes fall
// on distinct banks); each MFMA operand is one 16-byte LDS read per lane.  A
// K-contiguous source is copied in VEC-value pieces; an M- or N-contiguous
// one is read along its contiguous dimension (VEC values at each of 4
// consecutive k) and transposed in registers into 8-byte LDS writes.
//
// Pipeline: the global reads of step s + 2 are issued at the start of step
// s into one of two register sets, the MFMAs of step s run from LDS buffer
// s % 2 (operand fragments read one 16-deep slice ahead), and the other
// register set (step s + 1, read during step s - 1) is written to the other
// buffer at the end of the step; one barrier per step.  A read thus has two
// steps of MFMAs to arrive.  Scheduling groups
// interleave the global reads and the LDS writes with the MFMAs so that the
// matrix unit keeps issuing.  Every step is the same branch-free code: reads
// are clamped into the operand (rows past the edge of A or B read the last
// valid row, whose products only reach rows or columns of C that are not
// stored; k past K reads a valid k), and values at k >= K are zeroed in
// both operands when they are written to LDS.  VEC (4, 2 or 1 values per
// global read) divides both pitches, both contiguous extents and both
// pointers' alignment.
//
// Split K: when the tile grid is too small to fill the device and K is long
// (the weight gradients X^T dZ, K = the batch's class rows), the K range is
// cut into S chunks of whole steps; chunk s writes its partial product to
// W[s][M][N] and a second kernel sums the S partials in order s = 0 .. S-1.
// Results therefore depend only on (M, N, K, tile, S): repeated calls agree
// bit for bit.
#include "gemm.h"

namespace dlm {

namespace gemm {

constexpr int BKT = 64, PITCH = BKT + 8, THREADS = 256, KS = BKT / 16;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

// VEC consecutive BF16 values read from global memory, kept as raw words
template <int VEC>
struct Piece;
template <>
struct Piece<4> {
  uint2 w;
  __device__ __forceinline__ void load(const uint16_t* p) { w = *reinterpret_cast<const uint2*>(p); }
  __device__ __forceinline__ uint32_t get(int e) const { return ((e >> 1 ? w.y : w.x) >> (16 * (e & 1))) & 0xffffu; }
  __device__ __forceinline__ void store(uint16_t* s) const { *reinterpret_cast<uint2*>(s) = w; }
  __device__ __forceinline__ void mask(uint32_t m) { w.x &= m; w.y &= m; }
};
template <>
struct Piece<2> {
  uint32_t w;
  __device__ __forceinline__ void load(const uint16_t* p) { w = *reinterpret_cast<const uint32_t*>(p); }
  __device__ __forceinline__ uint32_t get(int e) const { return (w >> (16 * e)) & 0xffffu; }
  __device__ __forceinline__ void store(uint16_t* s) const { *reinterpret_cast<uint32_t*>(s) = w; }
  __device__ __forceinline__ void mask(uint32_t m) { w &= m; }
};
template <>
struct Piece<1> {
  uint32_t w;
  __device__ __forceinline__ void load(const uint16_t* p) { w = *p; }
  __device__ __forceinline__ uint32_t get(int) const { return w; }
  __device__ __forceinline__ void store(uint16_t* s) const { *s = (uint16_t)w; }
  __device__ __forceinline__ void mask(uint32_t m) { w &= m; }
};

// One operand's share of a K step: the [R rows] x [BKT k] tile of X(r, k)
// (KC: X[r * pitch + k], else X[k * pitch + r]) whose LDS image is s[r][k].
//   KC:  a unit is VEC values along k of one row: lane tid holds column
//        piece tid % PR of row tid / PR + RPI i for i < NU.
//   !KC: a unit is VEC rows at 4 consecutive k, k = 4 kg .. 4 kg + 3 with
//        kg = kq + 4 kh; 16 neighbouring lanes take neighbouring row pieces
//        rc of one k row (every group of 4 lanes reads one 32-byte run, 16
//        lanes one 128-byte line), then kq, then the remaining rc and kh.
// WIN (windowed): every read lies inside the operand because the caller
// places the window (rows r0 .. r0 + R - 1, k from kb) inside it; each read
// is a base shared by the workgroup plus one loop-invariant 32-bit lane
// offset.  Otherwise (clamped) rows past the edge read the last row, k past
// K reads a valid k, and keep bits zero the k >= K at store.
template <bool KC, int R, int VEC, bool WIN>
struct Stage {
  static constexpr int PR = BKT / VEC, RPI = THREADS / PR;  // KC: pieces per row, rows per unit index
  static constexpr int RC = R / VEC;                         // !KC: row pieces
  static constexpr int NU = KC ? R / RPI : RC / 16;
  static_assert(KC ? R % RPI == 0 : RC % 16 == 0, "whole units per thread");
  static constexpr int PER = KC ? 1 : 4;
  static constexpr int LOADS = NU * PER;
  static constexpr int STORES = KC ? NU : NU * VEC;
  Piece<VEC> p[NU][PER];
  uint32_t keep;  // clamped: bit i * PER + q keeps the piece (its k lies below K)

  // !KC unit i of lane tid: 16 neighbouring lanes read neighbouring row
  // pieces of one k row; lane bits 4-5 pick kq, the rest row pieces and kh
  static constexpr int G = RC / 16;  // 1, 2, 4 or 8
  __device__ static __forceinline__ int kq_lane(int tid) { return (tid >> 4) & 3; }
  __device__ static __forceinline__ int rc_lane(int tid) {
    return (tid & 15) + 16 * (G <= 4 ? (tid >> 6) % G : (tid >> 6));
  }
  __device__ static __forceinline__ int kh_lane(int tid) { return G <= 4 ? (tid >> 6) / G : 0; }
  __device__ static __forceinline__ int rc_unif(int i) { return G <= 4 ? 0 : 64 * (i % (G / 4)); }
  __device__ static __forceinline__ int kh_unif(int i) { return G <= 4 ? (4 / G) * i : i / (G / 4); }

  // windowed: rows r0 .. r0 + R - 1 and k kb .. kb + BKT - 1 all inside X
  __device__ __forceinline__ void load_win(const uint16_t* __restrict__ X, int64_t pitch, int r0, int kb, int tid) {
    const int ip = (int)pitch;
    if (KC) {
      const uint16_t* base = X + (int64_t)r0 * pitch + kb;
      const uint32_t lo = (uint32_t)((tid / PR) * ip + VEC * (tid % PR));
#pragma unroll
      for (int i = 0; i < NU; ++i) p[i][0].load(base + (int64_t)(RPI * i) * pitch + lo);
    } else {
      const uint16_t* base = X + (int64_t)kb * pitch + r0;
      const uint32_t lo = (uint32_t)((4 * kq_lane(tid) + 16 * kh_lane(tid)) * ip + VEC * rc_lane(tid));
#pragma unroll
      for (int i = 0; i < NU; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          p[i][q].load(base + ((int64_t)(16 * kh_unif(i) + q) * pitch + VEC * rc_unif(i)) + lo);
    }
  }

  // clamped: any shape; the step starts at k0 (past K: everything dropped)
  __device__ __forceinline__ void load_clamp(const uint16_t* __restrict__ X, int64_t pitch, int rows, int K, int r0,
                                             int k0, int tid) {
    const int ip = (int)pitch;
    const int kb = min(k0, ((K - 1) / BKT) * BKT);  // a step that holds valid k
    keep = 0u;
    if (KC) {
      const uint16_t* base = X + (int64_t)r0 * pitch + kb;
      const int kc = tid % PR, rl = tid / PR, last = rows - 1 - r0;
      const int kl = min(VEC * kc, K - VEC - kb);
      const bool ok = k0 + VEC * kc < K;
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        p[i][0].load(base + (uint32_t)(min(rl + RPI * i, last) * ip + kl));
        keep |= ok ? 1u << i : 0u;
      }
    } else {
      const uint16_t* base = X + (int64_t)kb * pitch + r0;
      const int last = rows - VEC - r0;
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        const int r = min(VEC * (rc_lane(tid) + rc_unif(i)), last);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int kk = 4 * kq_lane(tid) + 16 * (kh_lane(tid) + kh_unif(i)) + q;
          p[i][q].load(base + (uint32_t)(min(kk, K - 1 - kb) * ip + r));
          keep |= k0 + kk < K ? 1u << (4 * i + q) : 0u;
        }
      }
    }
  }

  // write the step to LDS; MASKED: keep only the pieces whose k (relative to
  // the window) lies in [lo, BKT) (windowed) or whose keep bit is set (clamped)
  template <bool MASKED>
  __device__ __forceinline__ void store(uint16_t* s, int tid, int lo) const {
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      if (KC) {
        const int kc = tid % PR, r = tid / PR + RPI * i;
        Piece<VEC> v = p[i][0];
        if (MASKED) v.mask(WIN ? (VEC * kc >= lo ? 0xffffffffu : 0u) : ((keep >> i) & 1u ? 0xffffffffu : 0u));
        v.store(s + r * PITCH + VEC * kc);
      } else {
        const int r = VEC * (rc_lane(tid) + rc_unif(i));
        const int kg4 = 4 * kq_lane(tid) + 16 * (kh_lane(tid) + kh_unif(i));
        uint32_t m[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          m[q] = !MASKED ? 0xffffu
                         : (WIN ? (kg4 + q >= lo ? 0xffffu : 0u) : ((keep >> (4 * i + q)) & 1u ? 0xffffu : 0u));
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const uint32_t w0 = (p[i][0].get(e) & m[0]) | ((p[i][1].get(e) & m[1]) << 16);
          const uint32_t w1 = (p[i][2].get(e) & m[2]) | ((p[i][3].get(e) & m[3]) << 16);
          *reinterpret_cast<uint2*>(s + (r + e) * PITCH + kg4) = make_uint2(w0, w1);
        }
      }
    }
  }
};

// Workgroup w of the launch runs on XCD w % 8; give each XCD a contiguous
// range of tiles (row-major over the tile grid), so that the tiles sharing
// rows of A are resident in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = nb / 8, rem = nb % 8, x = b % 8, i = b / 8;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// the MFMAs of one K step from LDS (fragments of slice ks + 1 read while
// the MFMAs of slice ks issue)
template <int TM>
__device__ __forceinline__ void mma_step(const uint16_t* sA, const uint16_t* sB, int wm, int wn, int lr, int lk,
                                         f16v (&acc)[TM][TM]) {
  bf8 a[2][TM], b[2][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    a[0][i] = *reinterpret_cast<const bf8*>(sA + (wm + 32 * i + lr) * PITCH + lk);
    b[0][i] = *reinterpret_cast<const bf8*>(sB + (wn + 32 * i + lr) * PITCH + lk);
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int c = ks & 1;
    if (ks + 1 < KS) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        a[c ^ 1][i] = *reinterpret_cast<const bf8*>(sA + (wm + 32 * i + lr) * PITCH + 16 * (ks + 1) + lk);
        b[c ^ 1][i] = *reinterpret_cast<const bf8*>(sB + (wn + 32 * i + lr) * PITCH + 16 * (ks + 1) + lk);
      }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TM; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
  }
}

// Scheduling groups for one steady step: the first slice's fragment reads,
// then the MFMAs with the next step's global reads spread over the first
// half, the later fragment reads one per two MFMAs, and the LDS writes of
// the next step spread over the second half.
template <int NM, int NV, int NR, int NW>
__device__ __forceinline__ void interleave() {
  constexpr int H = NM / 2;
  __builtin_amdgcn_sched_group_barrier(0x100, NR / (KS - 1), 0);  // the first slice's fragments
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
    if (i < H) {
      const int nv = (i + 1) * NV / H - i * NV / H;
#pragma unroll
      for (int j = 0; j < nv; ++j) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // global read
    } else {
      const int ii = i - H;
      const int nw = (ii + 1) * NW / H - ii * NW / H;
#pragma unroll
      for (int j = 0; j < nw; ++j) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
    }
    const int nr = (i + 1) * NR / NM - i * NR / NM;
#pragma unroll
    for (int j = 0; j < nr; ++j) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
  }
}

// Store a workgroup's tile: tile (i, j) value r of lane l is row
// 32 i + 8 (r / 4) + 4 (l / 32) + r % 4, column 32 j + l % 32 of the wave's
// quarter; rows below m0 and columns below n0 (a windowed edge tile's
// overlap with its neighbour) and past M, N are not stored.  EV: the
// evaluation epilogue (GemmEval) writes BF16 activations instead of C.
template <int TM, bool EV>
__device__ __forceinline__ void store_tile(const f16v (&acc)[TM][TM], int mr, int m0, int nr, int n0, int wm, int wn,
                                           int lane, int M, int N, float* __restrict__ C, int64_t ldc,
                                           const GemmEval& ev) {
  const int lr = lane & 31, l4 = 4 * (lane >> 5);
  constexpr int T = 64 * TM;
  // an interior tile (the usual case) stores every value: no per-value tests
  const bool interior = m0 == mr && n0 == nr && mr + T <= M && nr + T <= N;
  if (!EV && interior) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TM; ++j) {
        float* c = C + (int64_t)(mr + wm + 32 * i + l4) * ldc + (nr + wn + 32 * j + lr);
#pragma unroll
        for (int r = 0; r < 16; ++r) c[(int64_t)(8 * (r >> 2) + (r & 3)) * ldc] = acc[i][j][r];
      }
    return;
  }
  if (!EV) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TM; ++j) {
        const int n = nr + wn + 32 * j + lr;
        if (n < N && n >= n0) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int m = mr + wm + 32 * i + 8 * (r >> 2) + l4 + (r & 3);
            if (m < M && m >= m0) C[(int64_t)m * ldc + n] = acc[i][j][r];
          }
        }
      }
    return;
  }
  // evaluation epilogue: row m belongs to colouring m / k; a 32-row group
  // starting at mi spans colouring c0 = mi / k and (k >= 32, checked on the
  // host) at most c0 + 1.  Every parameter and U value the tile needs is
  // read first (addresses clamped inside the arrays; values for columns or
  // rows that are not stored go unused), so that the stores wait on nothing.
  const int k = ev.k, cmax = (M - 1) / k;
  float bb[TM], mm[TM], rs[TM], g[TM], sf[TM], u0[TM][TM], u1[TM][TM];
  int c0[TM], r0[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int mi = mr + wm + 32 * i;
    c0[i] = mi / k;
    r0[i] = mi - c0[i] * k;
  }
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    const int n = min(nr + wn + 32 * j + lr, N - 1);
    bb[j] = ev.beta[n];
    mm[j] = ev.mean[n];
    rs[j] = ev.var[n];
    g[j] = ev.gamma[n];
    sf[j] = ev.mu[n];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      u0[i][j] = ev.u[(int64_t)min(c0[i], cmax) * N + n];
      u1[i][j] = ev.u[(int64_t)min(c0[i] + 1, cmax) * N + n];
    }
  }
  // y = ((acc + u + beta) - mean) * rs * gamma + mu = acc * sc + off, with
  // sc per column and off per (colouring, column): one FMA per value, then
  // LReLU and the hardware BF16 conversion (round to nearest even)
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    const float sc = g[j] / sqrtf(rs[j] + ev.eps);
    g[j] = sc;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      u0[i][j] = ((u0[i][j] + bb[j]) - mm[j]) * sc + sf[j];
      u1[i][j] = ((u1[i][j] + bb[j]) - mm[j]) * sc + sf[j];
    }
  }
  if (interior) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TM; ++j) {
        uint16_t* x = ev.x + (int64_t)(mr + wm + 32 * i + l4) * N + (nr + wn + 32 * j + lr);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int d = 8 * (r >> 2) + l4 + (r & 3);
          const float yy = fmaf(acc[i][j][r], g[j], r0[i] + d >= k ? u1[i][j] : u0[i][j]);
          const __bf16 o = (__bf16)(yy > 0.f ? yy : ev.slope * yy);
          x[(int64_t)(8 * (r >> 2) + (r & 3)) * N] = __builtin_bit_cast(uint16_t, o);
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int mi = mr + wm + 32 * i;
#pragma unroll
    for (int j = 0; j < TM; ++j) {
      const int n = nr + wn + 32 * j + lr;
      if (n < N && n >= n0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int d = 8 * (r >> 2) + l4 + (r & 3), m = mi + d;
          if (m < M && m >= m0) {
            const float yy = fmaf(acc[i][j][r], g[j], r0[i] + d >= k ? u1[i][j] : u0[i][j]);
            const __bf16 o = (__bf16)(yy > 0.f ? yy : ev.slope * yy);
            ev.x[(int64_t)m * N + n] = __builtin_bit_cast(uint16_t, o);
          }
        }
      }
    }
  }
}

template <int TM, bool AK, bool BK, int VEC, bool WIN, bool EV>
__global__ __launch_bounds__(THREADS) void gemm_bf16_kernel(const uint16_t* __restrict__ A, int64_t sa,
                                                            const uint16_t* __restrict__ B, int64_t sb,
                                                            float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                            int tiles_n, int kchunk, float* __restrict__ W,
                                                            GemmEval ev) {
  constexpr int T = 64 * TM;
  __shared__ __align__(16) uint16_t sA[2][T * PITCH];
  __shared__ __align__(16) uint16_t sB[2][T * PITCH];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int m0 = (t / tiles_n) * T, n0 = (t % tiles_n) * T;
  // windowed: an edge tile reads the last T rows (columns) instead, and
  // stores only its own
  const int mr = WIN ? min(m0, M - T) : m0, nr = WIN ? min(n0, N - T) : n0;
  const int wm = (wid >> 1) * 32 * TM, wn = (wid & 1) * 32 * TM;
  const int lr = lane & 31, lk = 8 * (lane >> 5);
  // this workgroup's K chunk (the whole K without a split)
  const int kbeg = (int)blockIdx.y * kchunk;
  const int Kl = min(K - kbeg, kchunk);
  A += AK ? (int64_t)kbeg : (int64_t)kbeg * sa;
  B += BK ? (int64_t)kbeg : (int64_t)kbeg * sb;
  if (gridDim.y > 1) {
    C = W + (int64_t)blockIdx.y * M * N;
    ldc = N;
  }
  f16v acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = f16v{};

  // two register sets per operand: the reads of step s + 2 are issued while
  // step s runs, and the set holding step s + 1 is written to LDS after it
  using SA = Stage<AK, T, VEC, WIN>;
  using SB = Stage<BK, T, VEC, WIN>;
  SA ga0, ga1;
  SB gb0, gb1;
  const int nk = (Kl + BKT - 1) / BKT;
  // Windowed steps read k from min(k0, Kl - BKT) (inside the operand since
  // K >= BKT, and at or past kbeg - BKT + 1); lo = k0 - that start masks the
  // k already summed (everything, for a step past the end).  The loop runs
  // an even number of steps; an odd count gets one step past the end, which
  // adds zeros.
#define DLM_GEMM_ISSUE(LA, LB, STEP)                                 \
  do {                                                               \
    const int k0_ = (STEP) * BKT;                                    \
    if (WIN) {                                                       \
      const int kb_ = min(k0_, Kl - BKT);                            \
      LA.load_win(A, sa, mr, kb_, tid);                              \
      LB.load_win(B, sb, nr, kb_, tid);                              \
    } else {                                                         \
      LA.load_clamp(A, sa, M, Kl, m0, k0_, tid);                     \
      LB.load_clamp(B, sb, N, Kl, n0, k0_, tid);                     \
    }                                                                \
  } while (0)
#define DLM_GEMM_PUT(LA, LB, BUF)                                    \
  do {                                                               \
    LA.template store<!WIN>(sA[BUF], tid, 0);                        \
    LB.template store<!WIN>(sB[BUF], tid, 0);                        \
  } while (0)
#define DLM_GEMM_FIX(LA, LB, STEP, BUF)                              \
  do {                                                               \
    if (WIN) {                                                       \
      const int k0_ = (STEP) * BKT, kb_ = min(k0_, Kl - BKT);        \
      if (k0_ > kb_) {                                               \
        LA.template store<true>(sA[BUF], tid, k0_ - kb_);            \
        LB.template store<true>(sB[BUF], tid, k0_ - kb_);            \
      }                                                              \
    }                                                                \
  } while (0)
  if (nk > 0) {
    DLM_GEMM_ISSUE(ga0, gb0, 0);
    DLM_GEMM_ISSUE(ga1, gb1, 1);
    DLM_GEMM_PUT(ga0, gb0, 0);
    DLM_GEMM_FIX(ga0, gb0, 0, 0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    DLM_GEMM_ISSUE(ga0, gb0, kt + 2);
    mma_step<TM>(sA[0], sB[0], wm, wn, lr, lk, acc);
    DLM_GEMM_PUT(ga1, gb1, 1);
    interleave<KS * TM * TM, SA::LOADS + SB::LOADS, (KS - 1) * 2 * TM, SA::STORES + SB::STORES>();
    DLM_GEMM_FIX(ga1, gb1, kt + 1, 1);
    __syncthreads();
    DLM_GEMM_ISSUE(ga1, gb1, kt + 3);
    mma_step<TM>(sA[1], sB[1], wm, wn, lr, lk, acc);
    DLM_GEMM_PUT(ga0, gb0, 0);
    interleave<KS * TM * TM, SA::LOADS + SB::LOADS, (KS - 1) * 2 * TM, SA::STORES + SB::STORES>();
    DLM_GEMM_FIX(ga0, gb0, kt + 2, 0);
    __syncthreads();
  }
#undef DLM_GEMM_ISSUE
#undef DLM_GEMM_PUT
#undef DLM_GEMM_FIX
  store_tile<TM, EV>(acc, mr, m0, nr, n0, wm, wn, lane, M, N, C, ldc, ev);
}

// 16 bytes per lane from global memory straight into LDS (lane l writes LDS
// bytes [16 l, 16 l + 16) past L).  The builtin only exists for the device;
// the host pass, which only needs the kernel's launch stub, sees nothing.
#if defined(__HIP_DEVICE_COMPILE__)
#define DLM_LDS_DIRECT16(G, L) __builtin_amdgcn_global_load_lds((G), (L), 16, 0, 0)
#else
#define DLM_LDS_DIRECT16(G, L) ((void)(G), (void)(L))
#endif

// One step of the direct kernel from its swizzled LDS image.  Fragments
// live in two register sets (fa, fb)[2] that persist across steps: slices
// alternate between them, so a step ends with its last slice in set 1,
// whose MFMAs run at the start of the next step and cover the latency of
// that step's first fragment reads (set 0) across the barrier between the
// steps.  NV direct reads of the next step, issued just before the call,
// are spread over the first MFMAs.
template <int TM, int NV>
__device__ __forceinline__ void mma_direct(const uint16_t* sA, const uint16_t* sB, int wm, int wn, int lr, int lh,
                                           f16v (&acc)[TM][TM], bf8 (&fa)[2][TM], bf8 (&fb)[2][TM]) {
  static_assert(KS % 2 == 0, "the last slice of a step lands in set 1");
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int ra = wm + 32 * i + lr, rb = wn + 32 * i + lr;
    fa[0][i] = *reinterpret_cast<const bf8*>(sA + ra * BKT + 8 * (lh ^ (ra & 7)));
    fb[0][i] = *reinterpret_cast<const bf8*>(sB + rb * BKT + 8 * (lh ^ (rb & 7)));
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1][i], fb[1][j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int c = ks & 1;
    if (ks + 1 < KS) {
      const int ch = 2 * (ks + 1) + lh;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int ra = wm + 32 * i + lr, rb = wn + 32 * i + lr;
        fa[c ^ 1][i] = *reinterpret_cast<const bf8*>(sA + ra * BKT + 8 * (ch ^ (ra & 7)));
        fb[c ^ 1][i] = *reinterpret_cast<const bf8*>(sB + rb * BKT + 8 * (ch ^ (rb & 7)));
      }
    }
    if (ks + 1 < KS) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TM; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[c][i], fb[c][j], acc[i][j], 0, 0, 0);
    }
  }
  // schedule: this step's first fragment reads; the carried slice's MFMAs
  // with the NV direct reads spread over them; then each slice's MFMAs with
  // the next slice's reads spread over them
  constexpr int NMS = TM * TM, NRS = 2 * TM;  // MFMAs and fragment reads per slice
  __builtin_amdgcn_sched_group_barrier(0x100, NRS, 0);
#pragma unroll
  for (int m = 0; m < NMS; ++m) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    const int nv = (m + 1) * NV / NMS - m * NV / NMS;
#pragma unroll
    for (int j = 0; j < nv; ++j) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
  }
#pragma unroll
  for (int ks = 0; ks + 1 < KS; ++ks)
#pragma unroll
    for (int m = 0; m < NMS; ++m) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      const int nr = (m + 1) * NRS / NMS - m * NRS / NMS;
#pragma unroll
      for (int j = 0; j < nr; ++j) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
}

// Both operands K-contiguous with 16-byte aligned rows: the reads go from
// global memory straight to LDS (16 bytes per lane, no registers, no LDS
// write instructions).  One such read fills 1 KB of LDS in lane order, 8
// rows of 64 k; each row is 8 chunks of 16 bytes stored at chunk c ^ (row % 8),
// so that the 16-byte operand reads of 8 neighbouring rows hit distinct
// banks.  Step s + 1 is read into the other buffer while step s runs (four
// separate LDS arrays, the loop unrolled by two, so that the compiler sees
// the reads and the buffer being written apart); a wait and a barrier end
// each step.  Windowed only (the reads stay inside the operands); where a
// step's window overlaps k already summed, those chunks are zeroed in LDS
// before the barrier.  An odd step count runs one step past the end, which
// is all zeros.
template <int TM, bool EV>
__global__ __launch_bounds__(THREADS) void gemm_direct_kernel(const uint16_t* __restrict__ A, int64_t sa,
                                                              const uint16_t* __restrict__ B, int64_t sb,
                                                              float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                              int tiles_n, int kchunk, float* __restrict__ W,
                                                              GemmEval ev) {
  constexpr int T = 64 * TM;
  __shared__ __align__(16) uint16_t sA0[T * BKT];
  __shared__ __align__(16) uint16_t sA1[T * BKT];
  __shared__ __align__(16) uint16_t sB0[T * BKT];
  __shared__ __align__(16) uint16_t sB1[T * BKT];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int m0 = (t / tiles_n) * T, n0 = (t % tiles_n) * T;
  const int mr = min(m0, M - T), nr = min(n0, N - T);
  const int wm = (wid >> 1) * 32 * TM, wn = (wid & 1) * 32 * TM;
  const int lr = lane & 31, lh = lane >> 5;
  const int kbeg = (int)blockIdx.y * kchunk;
  const int Kl = min(K - kbeg, kchunk);
  A += kbeg;
  B += kbeg;
  if (gridDim.y > 1) {
    C = W + (int64_t)blockIdx.y * M * N;
    ldc = N;
  }
  f16v acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = f16v{};
  // lane's place in a 1 KB group: row lane / 8, LDS chunk lane % 8, which
  // holds source chunk (lane % 8) ^ (row % 8)
  const int grow = lane >> 3, gch = (lane & 7) ^ (grow & 7);
  const uint16_t* pa = A + (int64_t)(mr + grow) * sa + 8 * gch;
  const uint16_t* pb = B + (int64_t)(nr + grow) * sb + 8 * gch;
  constexpr int GPW = T / 32;  // 8-row groups per wave and operand
  const int nk = (Kl + BKT - 1) / BKT;
#define DLM_DIRECT_ISSUE(SA_, SB_, STEP)                                                                   \
  do {                                                                                                     \
    const int kb_ = min((STEP) * BKT, Kl - BKT);                                                           \
    _Pragma("unroll") for (int g = 0; g < GPW; ++g) {                                                      \
      const int grp = wid + 4 * g;                                                                          \
      DLM_LDS_DIRECT16(pa + (int64_t)(8 * grp) * sa + kb_, SA_ + grp * 8 * BKT);                    \
      DLM_LDS_DIRECT16(pb + (int64_t)(8 * grp) * sb + kb_, SB_ + grp * 8 * BKT);                    \
    }                                                                                                      \
  } while (0)
  // after the step's reads have landed in every wave: zero the chunks below
  // lo (k already summed, everything past the end) of both operands
#define DLM_DIRECT_MASK(SA_, SB_, STEP)                                                   \
  do {                                                                                   \
    const int k0_ = (STEP) * BKT, kb_ = min(k0_, Kl - BKT);                              \
    if (k0_ > kb_) {                                                                     \
      __syncthreads(); /* every wave's reads have landed before any chunk is zeroed */   \
      const int nch_ = min((k0_ - kb_) / 8, 8);                                          \
      for (int e_ = tid; e_ < T * nch_; e_ += THREADS) {                                 \
        const int r_ = e_ / nch_, c_ = e_ % nch_;                                        \
        const int off_ = r_ * BKT + 8 * (c_ ^ (r_ & 7));                                 \
        *reinterpret_cast<uint4*>(SA_ + off_) = make_uint4(0u, 0u, 0u, 0u);              \
        *reinterpret_cast<uint4*>(SB_ + off_) = make_uint4(0u, 0u, 0u, 0u);              \
      }                                                                                  \
    }                                                                                    \
  } while (0)
  if (nk > 0) {
    DLM_DIRECT_ISSUE(sA0, sB0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    DLM_DIRECT_MASK(sA0, sB0, 0);
  }
  __syncthreads();
  // fragment sets; set 1 (the carried last slice) starts as zeros, whose
  // MFMAs add nothing
  bf8 fa[2][TM], fb[2][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    fa[1][i] = bf8{};
    fb[1][i] = bf8{};
  }
  for (int kt = 0; kt < nk; kt += 2) {
    DLM_DIRECT_ISSUE(sA1, sB1, kt + 1);
    mma_direct<TM, 2 * GPW>(sA0, sB0, wm, wn, lr, lh, acc, fa, fb);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's reads of the next step have landed
    DLM_DIRECT_MASK(sA1, sB1, kt + 1);
    __syncthreads();
    DLM_DIRECT_ISSUE(sA0, sB0, kt + 2);
    mma_direct<TM, 2 * GPW>(sA1, sB1, wm, wn, lr, lh, acc, fa, fb);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    DLM_DIRECT_MASK(sA0, sB0, kt + 2);
    __syncthreads();
  }
  // the last step's last slice
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1][i], fb[1][j], acc[i][j], 0, 0, 0);
#undef DLM_DIRECT_ISSUE
#undef DLM_DIRECT_MASK
  store_tile<TM, EV>(acc, mr, m0, nr, n0, wm, wn, lane, M, N, C, ldc, ev);
}

// C[m][n] = sum over s = 0 .. S-1 (in that order) of W[s][m][n]
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const float* __restrict__ W, int S, int M, int N,
                                                          float* __restrict__ C, int64_t ldc) {
  const int64_t MN = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < MN; e += (int64_t)gridDim.x * 256) {
    float v = W[e];
    for (int s = 1; s < S; ++s) v += W[s * MN + e];
    C[(e / N) * ldc + e % N] = v;
  }
}

// the widest piece (4, 2 or 1 values) that divides the pitch, the
// contiguous extent and the pointer's alignment
int piece_width(const uint16_t* p, int64_t pitch, int64_t extent) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  for (int v : {4, 2})
    if (a % (2u * v) == 0 && pitch % v == 0 && extent % v == 0) return v;
  return 1;
}

int64_t tiles(int64_t M, int64_t N, int t) { return ((M + t - 1) / t) * ((N + t - 1) / t); }

template <int TM, int VEC, bool WIN, bool EV>
void launch_vec(bool ak, bool bk, dim3 grid, hipStream_t s, const uint16_t* A, int64_t sa, const uint16_t* B,
                int64_t sb, float* C, int64_t ldc, int M, int N, int K, int tn, int kchunk, float* W,
                const GemmEval& ev) {
  if (EV || (ak && bk))  // the evaluation epilogue comes with K-contiguous operands only
    hipLaunchKernelGGL((gemm_bf16_kernel<TM, true, true, VEC, WIN, EV>), grid, dim3(THREADS), 0, s, A, sa, B, sb, C,
                       ldc, M, N, K, tn, kchunk, W, ev);
  else if (ak && !bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<TM, true, false, VEC, WIN, false>), grid, dim3(THREADS), 0, s, A, sa, B, sb,
                       C, ldc, M, N, K, tn, kchunk, W, ev);
  else if (!ak && !bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<TM, false, false, VEC, WIN, false>), grid, dim3(THREADS), 0, s, A, sa, B, sb,
                       C, ldc, M, N, K, tn, kchunk, W, ev);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<TM, false, true, VEC, WIN, false>), grid, dim3(THREADS), 0, s, A, sa, B, sb,
                       C, ldc, M, N, K, tn, kchunk, W, ev);
}

template <bool EV>
void launch_direct(int tile, dim3 grid, hipStream_t s, const uint16_t* A, int64_t sa, const uint16_t* B, int64_t sb,
                   float* C, int64_t ldc, int M, int N, int K, int tn, int kchunk, float* W, const GemmEval& ev) {
  if (tile == 256)
    hipLaunchKernelGGL((gemm_direct_kernel<4, EV>), grid, dim3(THREADS), 0, s, A, sa, B, sb, C, ldc, M, N, K, tn,
                       kchunk, W, ev);
  else if (tile == 128)
    hipLaunchKernelGGL((gemm_direct_kernel<2, EV>), grid, dim3(THREADS), 0, s, A, sa, B, sb, C, ldc, M, N, K, tn,
                       kchunk, W, ev);
  else
    hipLaunchKernelGGL((gemm_direct_kernel<1, EV>), grid, dim3(THREADS), 0, s, A, sa, B, sb, C, ldc, M, N, K, tn,
                       kchunk, W, ev);
}

// the windowed kernels need 2- or 4-value pieces, a whole tile of rows in
// both operands and at least one whole K step
bool windowed(int M, int N, int K, int vec, int T) { return vec >= 2 && M >= T && N >= T && K >= BKT; }

int cu_count_cached() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return device_cu_count();
  if (!cus[dev]) cus[dev] = device_cu_count();
  return cus[dev];
}

}  // namespace gemm

// Tile and split for a product.  Model: a workgroup of tile T runs one K
// step in time T^2 / eff(T) (eff: 1, 0.75, 0.45 for T = 256, 128, 64, from
// the MFMA density per LDS byte), CUs hold occ(T) = 1, 2, 4 workgroups, the
// grid runs in ceil(workgroups / (CUs occ)) rounds, and a split adds the
// reduction's (S + 1) M N 4 bytes at about 2 KB per cycle over the device.
GemmPlan gemm_plan(int M, int N, int K, int vec, int64_t ws_bytes, int tile, int splits) {
  const int cus = gemm::cu_count_cached();
  const int steps = (K + gemm::BKT - 1) / gemm::BKT;
  GemmPlan best{64, 1};
  double best_cost = 1e300;
  for (int T : {256, 128, 64}) {
    if (tile && T != tile) continue;
    if (T > 64 && !gemm::windowed(M, N, K, vec, T)) continue;  // larger tiles are windowed only
    const double eff = T == 256 ? 1.0 : T == 128 ? 0.75 : 0.45;
    const int occ = T == 256 ? 1 : T == 128 ? 2 : 4;
    const int64_t nt = gemm::tiles(M, N, T);
    const int smax = std::max(1, std::min(16, steps / 4));
    for (int S = 1; S <= smax; ++S) {
      if (splits && S != splits) continue;
      if (S > 1 && (int64_t)S * M * N * 4 > ws_bytes) break;
      const int per = (steps + S - 1) / S;  // steps per chunk
      const int64_t rounds = (nt * S + (int64_t)cus * occ - 1) / ((int64_t)cus * occ);
      // cycles: one step of a T tile is T^2 * 64 * 2 flops over 4 SIMDs x 1024 flops/cycle
      double cost = (double)rounds * per * ((double)T * T * gemm::BKT * 2.0 / 4096.0) / eff * occ;
      if (S > 1) cost += (double)(S + 1) * M * N * 4 / 2048.0;
      if (cost < best_cost) {
        best_cost = cost;
        best = {T, S};
      }
    }
  }
  if (best_cost == 1e300) best = {64, splits > 1 ? splits : 1};
  return best;
}

// Host launch: C[M][N] (pitch ldc) = A(m, k) B(k, n) as described above.
// tile / splits: 0 chooses from the shape, else forced (a split needs
// splits M N 4 bytes of workspace; a tile the shape cannot take falls back
// to 64).  eval: write the evaluation epilogue's BF16 activations instead
// of C (both operands K-contiguous, no split; C unused).
int gemm_bf16(bool a_kcontig, const uint16_t* A, int64_t sa, bool b_kcontig, const uint16_t* B, int64_t sb, float* C,
              int64_t ldc, int M, int N, int K, int tile, int splits, void* ws, int64_t ws_bytes, hipStream_t s,
              const GemmEval* eval) {
  if (M < 0 || N < 0 || K < 0 || ldc < N || splits < 0 || splits > 64 || ws_bytes < 0)
    return set_error(DLM_E_INVAL, "gemm_bf16: M=%d N=%d K=%d ldc=%lld splits=%d", M, N, K, (long long)ldc, splits);
  if (tile != 0 && tile != 64 && tile != 128 && tile != 256)
    return set_error(DLM_E_INVAL, "gemm_bf16: tile %d (need 0, 64, 128 or 256)", tile);
  if (M == 0 || N == 0) return DLM_OK;
  if (!A || !B || (!C && !eval)) return set_error(DLM_E_INVAL, "gemm_bf16: null operand");
  if ((a_kcontig ? sa < K : sa < M) || (b_kcontig ? sb < K : sb < N))
    return set_error(DLM_E_INVAL, "gemm_bf16: pitch smaller than the contiguous extent");
  if (sa > (1 << 22) || sb > (1 << 22))  // lane offsets within one step stay below 2^31 values
    return set_error(DLM_E_INVAL, "gemm_bf16: pitch above 2^22 values");
  if (eval && (!a_kcontig || !b_kcontig || splits > 1 || eval->k < 32 || !eval->x || !eval->u))
    return set_error(DLM_E_INVAL, "gemm_bf16: the evaluation epilogue needs K-contiguous operands, no split, k >= 32");
  if (splits > 1 && (!ws || (int64_t)splits * M * N * 4 > ws_bytes))
    return set_error(DLM_E_INVAL, "gemm_bf16: %d splits need %lld bytes of workspace", splits,
                     (long long)splits * M * N * 4);
  // K == 0 is an empty sum: the kernel skips its K loop and stores zeros
  const int va = gemm::piece_width(A, sa, a_kcontig ? K : M), vb = gemm::piece_width(B, sb, b_kcontig ? K : N);
  const int vec = va < vb ? va : vb;
  if (tile > 64 && !gemm::windowed(M, N, K, vec, tile)) tile = 64;
  const GemmPlan p = gemm_plan(M, N, K, vec, (ws && !eval) ? ws_bytes : 0, tile, eval ? 1 : splits);
  const int S = p.splits;
  const int steps = (K + gemm::BKT - 1) / gemm::BKT;
  const int kchunk = S > 1 ? ((steps + S - 1) / S) * gemm::BKT : std::max(K, 1);
  const int Sg = S > 1 ? (K + kchunk - 1) / kchunk : 1;  // chunks that hold some k
  const int tn = (N + p.tile - 1) / p.tile;
  const int64_t nt = gemm::tiles(M, N, p.tile);
  if (nt > 0x7fffffff) return set_error(DLM_E_INVAL, "gemm_bf16: %lld tiles", (long long)nt);
  const dim3 grid((unsigned)nt, (unsigned)Sg);
  float* W = (float*)ws;
  const GemmEval ev = eval ? *eval : GemmEval{};
  const bool win = gemm::windowed(M, N, K, vec, p.tile);
  // both operands K-contiguous with 16-byte aligned rows and K steps: the
  // direct-to-LDS kernel
  const bool direct = win && a_kcontig && b_kcontig && K % 8 == 0 && sa % 8 == 0 && sb % 8 == 0 &&
                      reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(B) % 16 == 0;
  if (direct) {
    if (eval)
      gemm::launch_direct<true>(p.tile, grid, s, A, sa, B, sb, C, ldc, M, N, K, tn, kchunk, W, ev);
    else
      gemm::launch_direct<false>(p.tile, grid, s, A, sa, B, sb, C, ldc, M, N, K, tn, kchunk, W, ev);
  } else {
#define DLM_GEMM_LAUNCH(TM, V, WIN)                                                                              \
  do {                                                                                                           \
    if (eval)                                                                                                    \
      gemm::launch_vec<TM, V, WIN, true>(a_kcontig, b_kcontig, grid, s, A, sa, B, sb, C, ldc, M, N, K, tn, kchunk, \
                                         W, ev);                                                                 \
    else                                                                                                         \
      gemm::launch_vec<TM, V, WIN, false>(a_kcontig, b_kcontig, grid, s, A, sa, B, sb, C, ldc, M, N, K, tn,     \
                                          kchunk, W, ev);                                                        \
  } while (0)
    if (p.tile == 256) {
      if (vec == 4)
        DLM_GEMM_LAUNCH(4, 4, true);
      else
        DLM_GEMM_LAUNCH(4, 2, true);
    } else if (p.tile == 128) {
      if (vec == 4)
        DLM_GEMM_LAUNCH(2, 4, true);
      else
        DLM_GEMM_LAUNCH(2, 2, true);
    } else if (win) {
      if (vec == 4)
        DLM_GEMM_LAUNCH(1, 4, true);
      else
        DLM_GEMM_LAUNCH(1, 2, true);
    } else {
      if (vec == 4)
        DLM_GEMM_LAUNCH(1, 4, false);
      else if (vec == 2)
        DLM_GEMM_LAUNCH(1, 2, false);
      else
        DLM_GEMM_LAUNCH(1, 1, false);
    }
#undef DLM_GEMM_LAUNCH
  }
  DLM_HIP(hipGetLastError());
  if (Sg > 1) {
    const int64_t MN = (int64_t)M * N;
    const unsigned blocks = (unsigned)std::min<int64_t>((MN + 255) / 256, 8192);
    hipLaunchKernelGGL(gemm::gemm_reduce_kernel, dim3(blocks), dim3(256), 0, s, W, Sg, M, N, C, ldc);
    DLM_HIP(hipGetLastError());
  }
  return DLM_OK;
}

int64_t gemm_workspace_bytes(int M, int N, int K) {
  const GemmPlan p = gemm_plan(M, N, K, 4, INT64_MAX / 4, 0, 0);
  return p.splits > 1 ? (int64_t)p.splits * M * N * 4 : 0;
}

}  // namespace dlm

extern "C" int dlm_gemm_bf16(int32_t a_kcontig, const uint16_t* A, int64_t sa, int32_t b_kcontig, const uint16_t* B,
                             int64_t sb, float* C, int64_t ldc, int32_t M, int32_t N, int32_t K, int32_t tile,
                             int32_t splits, void* workspace, int64_t workspace_bytes, void* stream) {
  return dlm::gemm_bf16(a_kcontig != 0, A, sa, b_kcontig != 0, B, sb, C, ldc, M, N, K, tile, splits, workspace,
                        workspace_bytes, (hipStream_t)stream);
}
