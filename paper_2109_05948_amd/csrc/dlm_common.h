// Shared host/device helpers of the gfx950 colouring library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/dlmcol.h"

namespace dlm {

constexpr int kWave = 64;
constexpr uint32_t kDomTenure = 0x80000001u;
constexpr uint32_t kDomInit = 0x80000002u;
constexpr uint32_t kDomGpxFill = 0x80000003u;
constexpr uint32_t kDomSelect = 0x80000006u;
constexpr uint32_t kDomGpxTie = 0x80000007u;
constexpr uint32_t kDomGreedy = 0x80000008u;
constexpr int kTenureCap = 32757;  // cap of the floor(num * f / den) tenure term

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications; key (k0, k1) = (low, high word of the seed),
// bumped by the Weyl constants after every round.  Returns word 0 only
// unless all four are asked for.
struct Key {
  uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed) {
  return Key{static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
}

__device__ __forceinline__ uint4 philox4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                         Key key) {
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit multiply per product (hi and lo halves together)
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(x0, x1, x2, x3);
}

__device__ __forceinline__ uint32_t philox_w0(uint32_t x0, uint32_t x1, uint32_t x2,
                                              uint32_t x3, Key key) {
  return philox4(x0, x1, x2, x3, key).x;
}

// uniform integer in [0, K) from a 32-bit word: floor(x * K / 2^32)
__host__ __device__ __forceinline__ uint32_t lemire(uint32_t x, uint32_t K) {
  return static_cast<uint32_t>((static_cast<uint64_t>(x) * K) >> 32);
}

// ---------------------------------------------------------------------------
// Wave64 reductions on DPP lane moves.  Every lane of the wave must be active.
// After quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and
// row_mirror each lane holds the reduction of its 16-lane row; the four row
// results are combined on the scalar unit.  The result is wave-uniform.
namespace dpp {
constexpr int kXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141; // row_half_mirror
constexpr int kMirror = 0x140;     // row_mirror
}  // namespace dpp

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t x) {
  // every control used here permutes lanes within a row, so no lane reads out
  // of bounds; bound_ctrl lets the compiler fold the move into the consumer
  // (one v_min_u32_dpp / v_add_u32_dpp per step)
  return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ uint32_t readlane(uint32_t x, int lane) {
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), lane));
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// median of three (one v_med3_u32)
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

// number of lanes below the calling lane whose bit is set in m
__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  x = min(x, dpp_mov<dpp::kXor1>(x));
  x = min(x, dpp_mov<dpp::kXor2>(x));
  x = min(x, dpp_mov<dpp::kHalfMirror>(x));
  x = min(x, dpp_mov<dpp::kMirror>(x));
  return min(min(readlane(x, 0), readlane(x, 16)), min(readlane(x, 32), readlane(x, 48)));
}

// smallest 64-bit key (hi, lo): the minimum of hi, then the minimum of lo
// over the lanes holding that hi
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
  const uint32_t hi = static_cast<uint32_t>(x >> 32);
  const uint32_t mh = wave_min_u32(hi);
  const uint32_t ml = wave_min_u32(hi == mh ? static_cast<uint32_t>(x) : 0xffffffffu);
  return (static_cast<uint64_t>(mh) << 32) | ml;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  x += dpp_mov<dpp::kXor1>(x);
  x += dpp_mov<dpp::kXor2>(x);
  x += dpp_mov<dpp::kHalfMirror>(x);
  x += dpp_mov<dpp::kMirror>(x);
  return readlane(x, 0) + readlane(x, 16) + readlane(x, 32) + readlane(x, 48);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = max(x, dpp_mov<dpp::kXor1>(x));
  x = max(x, dpp_mov<dpp::kXor2>(x));
  x = max(x, dpp_mov<dpp::kHalfMirror>(x));
  x = max(x, dpp_mov<dpp::kMirror>(x));
  return max(max(readlane(x, 0), readlane(x, 16)), max(readlane(x, 32), readlane(x, 48)));
}

__host__ __device__ constexpr uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

// FNV-1a over 64-bit move records
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;
__device__ __forceinline__ uint64_t fnv_step(uint64_t h, uint32_t v, uint32_t c, int32_t f) {
  const uint64_t x = static_cast<uint64_t>(v & 0xffffu) | (static_cast<uint64_t>(c & 0xffffu) << 16) |
                     (static_cast<uint64_t>(static_cast<uint32_t>(f)) << 32);
  return (h ^ x) * kFnvPrime;
}

// ---------------------------------------------------------------------------
// Host-side error plumbing.
int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int device_lds_limit();  // max dynamic LDS bytes per workgroup on the current device
int device_cu_count();
int device_lds_per_cu();  // LDS bytes of one CU on the current device

#define DLM_HIP(call)                                    \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::dlm::hip_fail(e_, #call); \
  } while (0)

}  // namespace dlm

struct dlm_graph {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t max_deg = 0;
  int32_t max_w = 0;
  int device = 0;
  int32_t* row_ptr = nullptr;  // device int32[n+1]
  int32_t* col_idx = nullptr;  // device int32[nnz]
  int32_t* erow = nullptr;     // device int32[nnz]: source vertex of each CSR entry
  int32_t* weights = nullptr;  // device int32[n] or null
  int32_t* order = nullptr;    // device int32[n]: greedy WVCP vertex order (weighted graphs only)
};
