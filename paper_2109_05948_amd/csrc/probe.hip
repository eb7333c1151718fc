// Measurement helper: sustained LDS read bandwidth of the whole device, the
// denominator of the TabuCol kernel's LDS roofline.  Every workgroup fills a
// 64 KiB LDS buffer and streams 16-byte reads over it (consecutive lanes on
// consecutive 16-byte words, no bank conflicts); a data-dependent XOR keeps
// the reads live.
#include <algorithm>

#include "dlm_common.h"

namespace dlm {

constexpr int kProbeWords = 64 * 1024 / 16;  // uint4 words in the buffer

__global__ __launch_bounds__(256) void lds_probe_kernel(int32_t rounds, uint32_t* __restrict__ sink) {
  __shared__ uint4 buf[kProbeWords];
  for (int i = threadIdx.x; i < kProbeWords; i += 256) buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
  __syncthreads();
  uint4 acc = make_uint4(0, 0, 0, 0);
  int idx = threadIdx.x;
  for (int r = 0; r < rounds; ++r) {
#pragma unroll 8
    for (int s = 0; s < kProbeWords / 256; ++s) {
      const uint4 x = buf[(idx + s * 256) & (kProbeWords - 1)];
      acc.x ^= x.x;
      acc.y ^= x.y;
      acc.z ^= x.z;
      acc.w ^= x.w;
    }
    idx = (idx + (int)(acc.x & 1u)) & (kProbeWords - 1);
  }
  if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9e3779b9u) sink[blockIdx.x] = acc.x;  // practically never
}

}  // namespace dlm

using namespace dlm;

extern "C" int dlm_probe_lds_bandwidth(int32_t rounds, double* bytes_per_s, void* stream) {
  if (rounds < 1 || !bytes_per_s) return set_error(DLM_E_INVAL, "dlm_probe_lds_bandwidth: bad arguments");
  int per_cu = 0;
  DLM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lds_probe_kernel, 256, 0));
  const int grid = std::max(1, per_cu) * device_cu_count();
  hipStream_t s = (hipStream_t)stream;
  uint32_t* sink = nullptr;
  DLM_HIP(hipMallocAsync((void**)&sink, sizeof(uint32_t) * grid, s));
  hipEvent_t e0, e1;
  DLM_HIP(hipEventCreate(&e0));
  DLM_HIP(hipEventCreate(&e1));
  hipLaunchKernelGGL(lds_probe_kernel, dim3(grid), dim3(256), 0, s, 1, sink);  // warm-up
  DLM_HIP(hipEventRecord(e0, s));
  hipLaunchKernelGGL(lds_probe_kernel, dim3(grid), dim3(256), 0, s, rounds, sink);
  DLM_HIP(hipEventRecord(e1, s));
  DLM_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  DLM_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  DLM_HIP(hipFreeAsync(sink, s));
  *bytes_per_s = (double)grid * rounds * (double)(kProbeWords * 16) / (ms * 1e-3);
  return DLM_OK;
}
