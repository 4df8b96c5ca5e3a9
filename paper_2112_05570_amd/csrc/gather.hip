// Gather roofline: how many dependent, random 16-byte loads per second the GPU sustains when a
// buffer of a given size is chased, with the walk's launch shape (persistent waves, one chain of
// dependent loads per lane, one 16-byte load per step). This is the memory pattern of a walk step
// without its arithmetic: the walk's steps/s divided by this rate, at the same working-set size,
// is the fraction of the gather roofline it reaches.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ccsp_walk.h"

namespace ccsp {

namespace {

constexpr uint64_t kMul = 6364136223846793005ull;  // a = 1 (mod 4) and c odd: a full-period
constexpr uint64_t kAdd = 1442695040888963407ull;  // linear congruential cycle modulo 2^k

__global__ void chase_init(int4* rec, uint64_t mask) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > mask) return;
  const uint64_t next = (i * kMul + kAdd) & mask;
  rec[i] = make_int4((int)next, (int)(i * 3u), (int)(i * 5u), (int)(i * 7u));
}

__global__ void __launch_bounds__(256)
chase(const int4* __restrict__ rec, uint64_t mask, int64_t steps, int* __restrict__ sink) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t idx = (uint32_t)(((g + 1) * 0x9E3779B97F4A7C15ull >> 17) & mask);
  int acc = 0;
  for (int64_t s = 0; s < steps; ++s) {
    const int4 r = rec[idx];
    __asm__ volatile("" ::"v"(r.x), "v"(r.y), "v"(r.z), "v"(r.w));  // one 16-byte load
    acc ^= r.y ^ r.z ^ r.w;
    idx = (uint32_t)r.x;
  }
  if (acc == 0x7fffffff && idx == 0xffffffffu) sink[0] = acc;  // never true; keeps the loads
}

}  // namespace

}  // namespace ccsp

using namespace ccsp;

extern "C" int gather_roofline(int64_t working_set_bytes, int32_t waves_per_cu,
                               int64_t steps_per_lane, double* out_loads_per_s, void* stream) {
  if (!out_loads_per_s || working_set_bytes < 4096 || working_set_bytes > (int64_t(1) << 36) ||
      waves_per_cu < 1 || waves_per_cu > 64 || steps_per_lane < 1)
    return CCSP_E_ARG;
  uint64_t n = 1;
  while (n * 2 * sizeof(int4) <= (uint64_t)working_set_bytes) n *= 2;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return CCSP_E_HIP;
  int4* rec = nullptr;
  int* sink = nullptr;
  if (hipMalloc(&rec, n * sizeof(int4)) != hipSuccess) return CCSP_E_OOM;
  if (hipMalloc(&sink, sizeof(int)) != hipSuccess) {
    (void)hipFree(rec);
    return CCSP_E_OOM;
  }
  hipEvent_t a = nullptr, b = nullptr;
  int rc = CCSP_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = CCSP_E_HIP;
  if (rc == CCSP_OK) {
    const uint64_t mask = n - 1;
    hipLaunchKernelGGL(chase_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rec, mask);
    const unsigned grid = (unsigned)(cus * waves_per_cu / 4);
    hipLaunchKernelGGL(chase, dim3(grid), dim3(256), 0, st, rec, mask, steps_per_lane / 4 + 1, sink);
    (void)hipEventRecord(a, st);
    hipLaunchKernelGGL(chase, dim3(grid), dim3(256), 0, st, rec, mask, steps_per_lane, sink);
    (void)hipEventRecord(b, st);
    float ms = 0.f;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess || ms <= 0.f) {
      rc = CCSP_E_HIP;
    } else {
      *out_loads_per_s = (double)grid * 256.0 * (double)steps_per_lane / (ms * 1e-3);
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(rec);
  (void)hipFree(sink);
  return rc;
}
