// Spatial binning of rays before the walk.
//
// Rays arrive in any order; walked in that order, the lanes resident on the GPU touch triangles
// all over the scene and every step misses the caches. Triangles are stored in Hilbert order of
// their centroids, so a range of internal triangle ids is a compact region of the plane. Sorting
// the rays by the internal id of their start triangle (a radix sort over its bits) makes the
// rays in flight at any moment start in one or two such regions, whose triangles then stay in
// the L2 of every XCD while they are walked. The sorted keys are the internal start ids, which
// the walk then reads in order instead of gathering them through the id map.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "walk.hpp"

namespace ccsp {

__global__ void bin_keys(const int32_t* __restrict__ start, const int32_t* __restrict__ perm,
                         int32_t ntri, int64_t n, uint32_t* __restrict__ key,
                         int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t s = start[i];
  key[i] = (s >= 0 && s < ntri) ? (uint32_t)perm[s] : (uint32_t)ntri;  // ntri: out of range
  idx[i] = (int32_t)i;
}

static int key_bits(int32_t ntri) {
  int b = 1;
  while ((1ll << b) <= (long long)ntri) ++b;
  return b;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static size_t cub_temp_bytes(int64_t n) {
  size_t temp = 0;
  hipcub::DoubleBuffer<uint32_t> k(nullptr, nullptr);
  hipcub::DoubleBuffer<int32_t> v(nullptr, nullptr);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, k, v, (int)n, 0, 30);
  return temp;
}

size_t bin_workspace_bytes(int64_t n) {
  return 4 * align256(sizeof(uint32_t) * (size_t)n) + align256(cub_temp_bytes(n));
}

hipError_t launch_bin_rays(const SceneDev& sc, const int32_t* start, int64_t n, void* workspace,
                           size_t ws_bytes, const int32_t** order_out,
                           const int32_t** order_start_out, hipStream_t stream) {
  if (bin_workspace_bytes(n) > ws_bytes) return hipErrorInvalidValue;
  auto* p = static_cast<unsigned char*>(workspace);
  const size_t a = align256(sizeof(uint32_t) * (size_t)n);
  uint32_t* k0 = reinterpret_cast<uint32_t*>(p);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(p + a);
  int32_t* v0 = reinterpret_cast<int32_t*>(p + 2 * a);
  int32_t* v1 = reinterpret_cast<int32_t*>(p + 3 * a);
  void* temp = p + 4 * a;
  size_t temp_bytes = ws_bytes - 4 * a;
  const int bs = 256;
  hipLaunchKernelGGL(bin_keys, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, stream, start,
                     sc.perm, sc.ntri, n, k0, v0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipcub::DoubleBuffer<uint32_t> keys(k0, k1);
  hipcub::DoubleBuffer<int32_t> vals(v0, v1);
  e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, vals, (int)n, 0,
                                         key_bits(sc.ntri), stream);
  if (e != hipSuccess) return e;
  *order_out = vals.Current();
  *order_start_out = reinterpret_cast<const int32_t*>(keys.Current());
  return hipSuccess;
}

}  // namespace ccsp
