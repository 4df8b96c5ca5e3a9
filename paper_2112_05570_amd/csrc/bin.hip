// Binning of rays before the walk, for cache reuse.
//
// Rays arrive in any order; walked in that order, the lanes resident on the GPU touch triangles
// all over the scene and nearly every step misses the caches. The rays are therefore walked in
// the order of a key, by a radix sort of (key, index) pairs; the walk reads each ray through the
// sorted index. Two keys:
//  * kKeyStart (default): the internal id of the start triangle. Triangles are numbered along a
//    Hilbert curve, so consecutive rays start close together and an L2-sized region of the scene
//    is in use at any moment. The sorted keys double as the rays' internal start ids.
//  * kKeyCoherent: [ Hilbert cell of the origin on a G x G grid | direction sector (16) |
//    sub-cell (4x4) ], G chosen for about a thousand rays per cell, so that the lanes of a wave
//    also share a direction. Needs no gather, but the walk then maps start ids itself.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "walk.hpp"

namespace ccsp {

namespace {

constexpr int kSectorBits = 4;
constexpr int kSubBits = 2;  // sub-cell grid 2^kSubBits x 2^kSubBits inside a cell

__device__ __forceinline__ uint32_t hilbert(uint32_t x, uint32_t y, int bits) {
  const uint32_t n = 1u << bits;
  uint32_t d = 0;
  for (uint32_t s = n >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = n - 1 - x;
        y = n - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

struct KeyGeom {
  double x0, y0, sx, sy;  // fine grid coordinate = (p - p0) * s, in [0, 2^(bits+kSubBits))
  int bits;               // log2 of the cell grid size G
};

__global__ void ray_keys(const double2* __restrict__ o, const double2* __restrict__ d, int64_t n,
                         KeyGeom g, uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 oi = o[i], di = d[i];
  const double hi = (double)((1u << (g.bits + kSubBits)) - 1);
  // NaN coordinates compare false and land in cell 0; the walk itself deals with such rays.
  const uint32_t fx = (uint32_t)fmin(fmax((oi.x - g.x0) * g.sx, 0.0), hi);
  const uint32_t fy = (uint32_t)fmin(fmax((oi.y - g.y0) * g.sy, 0.0), hi);
  const uint32_t cell = hilbert(fx >> kSubBits, fy >> kSubBits, g.bits);
  const uint32_t sub = hilbert(fx & ((1u << kSubBits) - 1), fy & ((1u << kSubBits) - 1), kSubBits);
  const float a = atan2f((float)di.y, (float)di.x);  // (-pi, pi]
  uint32_t sector = (uint32_t)((a + 3.14159265f) * (float)(1 << kSectorBits) / 6.2831854f);
  sector = min(sector, (1u << kSectorBits) - 1);
  key[i] = (((cell << kSectorBits) | sector) << (2 * kSubBits)) | sub;
  idx[i] = (int32_t)i;
}

__global__ void start_keys(const int32_t* __restrict__ start, const int32_t* __restrict__ perm,
                           int32_t ntri, int64_t n, uint32_t* __restrict__ key,
                           int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t s = start[i];
  key[i] = (s >= 0 && s < ntri) ? (uint32_t)perm[s] : (uint32_t)ntri;  // ntri: out of range
  idx[i] = (int32_t)i;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int bits_for(int64_t v) {  // smallest b with v < 2^b
  int b = 1;
  while (b < 31 && (int64_t(1) << b) <= v) ++b;
  return b;
}

int grid_bits(int64_t n) {  // about 1024 rays per cell, cells from 16 x 16 to 4096 x 4096
  int b = 4;
  while (b < 12 && (int64_t(1) << (2 * (b + 1))) * 1024 <= n) ++b;
  return b;
}

int key_bits(int64_t n) { return 2 * grid_bits(n) + kSectorBits + 2 * kSubBits; }

size_t sort_temp_bytes(int64_t n) {
  size_t temp = 0;
  hipcub::DoubleBuffer<uint32_t> k(nullptr, nullptr);
  hipcub::DoubleBuffer<int32_t> v(nullptr, nullptr);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, k, v, (int)n, 0, 32);
  return temp;
}

}  // namespace

size_t bin_workspace_bytes(int64_t n) {
  return 4 * align256(sizeof(uint32_t) * (size_t)n) + align256(sort_temp_bytes(n));
}

hipError_t launch_bin_rays(const SceneDev& sc, const RaysDev& in, int key_kind, void* workspace,
                           size_t ws_bytes, RaysDev* out, hipStream_t stream) {
  const int64_t n = in.n;
  if (n <= 0 || n >= INT32_MAX || bin_workspace_bytes(n) > ws_bytes) return hipErrorInvalidValue;
  auto* p = static_cast<unsigned char*>(workspace);
  const size_t a = align256(sizeof(uint32_t) * (size_t)n);
  uint32_t* k0 = reinterpret_cast<uint32_t*>(p);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(p + a);
  int32_t* v0 = reinterpret_cast<int32_t*>(p + 2 * a);
  int32_t* v1 = reinterpret_cast<int32_t*>(p + 3 * a);
  void* temp = p + 4 * a;
  size_t temp_bytes = ws_bytes - 4 * a;
  KeyGeom g;
  g.bits = grid_bits(n);
  const double fine = (double)(1u << (g.bits + kSubBits));
  g.x0 = sc.box_x0;
  g.y0 = sc.box_y0;
  g.sx = sc.box_x1 > sc.box_x0 ? fine / (sc.box_x1 - sc.box_x0) : 0.0;
  g.sy = sc.box_y1 > sc.box_y0 ? fine / (sc.box_y1 - sc.box_y0) : 0.0;
  const int bs = 256;
  const dim3 grid((unsigned)((n + bs - 1) / bs));
  int end_bit;
  if (key_kind == kKeyCoherent) {
    hipLaunchKernelGGL(ray_keys, grid, dim3(bs), 0, stream, in.o, in.d, n, g, k0, v0);
    end_bit = key_bits(n);
  } else {
    hipLaunchKernelGGL(start_keys, grid, dim3(bs), 0, stream, in.start, sc.perm, sc.ntri, n, k0, v0);
    end_bit = bits_for(sc.ntri);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipcub::DoubleBuffer<uint32_t> keys(k0, k1);
  hipcub::DoubleBuffer<int32_t> vals(v0, v1);
  e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, vals, (int)n, 0, end_bit, stream);
  if (e != hipSuccess) return e;
  *out = in;
  out->order = vals.Current();
  out->order_start = key_kind == kKeyCoherent ? nullptr : reinterpret_cast<const int32_t*>(keys.Current());
  return hipSuccess;
}

}  // namespace ccsp
