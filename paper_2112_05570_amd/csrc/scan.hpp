// Exclusive prefix sum of 32-bit counts on the device, for the binning passes: out[i] = in[0] +
// ... + in[i - 1]. Three launches: per-block totals of 2,048 counts, one workgroup scanning the
// totals in place (2,048 at a time, with a running carry), then each block's counts scanned and
// offset by its block's prefix. Integer arithmetic, so the result does not depend on the order of
// the additions. The caller keeps the sums below 2^32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ccsp {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;                             // consecutive counts per thread
constexpr int kScanBlock = kScanThreads * kScanPer;     // counts per block

// Exclusive scan of one value per thread over the workgroup (every thread calls it); *total
// receives the workgroup's sum.
__device__ __forceinline__ uint32_t scan_block_exclusive(uint32_t x, uint32_t* sh,
                                                         uint32_t* total) {
  const int t = threadIdx.x;
  sh[t] = x;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t y = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += y;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - x;
}

__global__ void __launch_bounds__(kScanThreads)
scan_totals(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t total;
  (void)scan_block_exclusive(s, sh, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One workgroup: sums[0..nb) replaced by their exclusive prefix.
__global__ void __launch_bounds__(kScanThreads)
scan_sums(uint32_t* __restrict__ sums, int64_t nb) {
  __shared__ uint32_t sh[kScanThreads];
  uint32_t carry = 0;
  for (int64_t tile = 0; tile < nb; tile += kScanBlock) {
    const int64_t base = tile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = base + k < nb ? sums[base + k] : 0u;
      s += v[k];
    }
    uint32_t total;
    uint32_t run = carry + scan_block_exclusive(s, sh, &total);
    for (int k = 0; k < kScanPer; ++k) {
      if (base + k < nb) sums[base + k] = run;
      run += v[k];
    }
    carry += total;
  }
}

__global__ void __launch_bounds__(kScanThreads)
scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ sums,
           uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = sums[blockIdx.x] + scan_block_exclusive(s, sh, &total);
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// Scratch of launch_exclusive_scan for n counts, in bytes.
inline size_t exclusive_scan_bytes(int64_t n) {
  return sizeof(uint32_t) * (size_t)((n + kScanBlock - 1) / kScanBlock + 1);
}

// out[0..n) = exclusive prefix sums of in[0..n) on `stream`; sums: exclusive_scan_bytes(n) of
// device scratch. in and out may not overlap.
inline hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n,
                                        uint32_t* sums, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(scan_totals, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, in, n, sums);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanThreads), 0, stream, sums, nb);
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, in, n, sums,
                     out);
  return hipGetLastError();
}

}  // namespace
}  // namespace ccsp
