// Binning of rays before the walk, for cache reuse.
//
// Rays arrive in any order; walked in that order, the lanes resident on the GPU touch triangles
// all over the scene and nearly every step misses the caches (the walk then runs at the random
// gather rate of a scene-sized working set). Binning puts rays that start close together next to
// each other, so that the rays in flight on one XCD start in one compact region whose triangles
// (stored in Hilbert order) fit its L2.
//
// Default (kBinBuckets): one counting-sort pass into kBuckets buckets = cells of a 16 x 16 grid
// over the scene numbered along a Hilbert curve. A counting kernel histograms the buckets per
// chunk of rays, a scan turns the counts into destinations, and a scatter kernel stages each
// chunk in LDS sorted by bucket and writes it out as 48-byte records (origin, direction, exit slot
// of the first triangle, caller's index) in runs, so that both its reads and writes are coalesced
// and the walk then reads its rays contiguously, with no gather through a permutation. The scatter
// also decides each ray's first triangle (three candidate edges, Sec. 7.2) from the caller-ordered
// first-triangle record, which it has to gather anyway for the start triangle's internal id; the
// walk then starts every binned ray with its first step.
// Alternative (kBinRadix): a radix sort of (internal start triangle, index) pairs; the walk then
// gathers each ray through the sorted index.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "decide.hpp"
#include "scan.hpp"
#include "walk.hpp"

namespace ccsp {

namespace {

constexpr int kGridBits = 4;
constexpr int kBuckets = 1 << (2 * kGridBits);
constexpr int kChunk = 1024;  // rays per scatter workgroup (LDS staging: 48 KiB)
constexpr int kThreads = 256;
constexpr int kPerThread = kChunk / kThreads;

struct BinGeom {
  double x0, y0, sx, sy;  // cell = floor((p - p0) * s), clamped to the grid
};

__device__ __forceinline__ uint32_t hilbert_cell(uint32_t x, uint32_t y) {
  constexpr uint32_t n = 1u << kGridBits;
  uint32_t d = 0;
#pragma unroll
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

__device__ __forceinline__ uint32_t bucket_of(const double2 o, const BinGeom& g) {
  constexpr double hi = (double)((1 << kGridBits) - 1);
  // NaN coordinates compare false and land in cell 0; the walk itself deals with such rays.
  const double fx = fmin(fmax((o.x - g.x0) * g.sx, 0.0), hi);
  const double fy = fmin(fmax((o.y - g.y0) * g.sy, 0.0), hi);
  return hilbert_cell((uint32_t)fx, (uint32_t)fy);
}

__global__ void __launch_bounds__(kThreads)
bucket_count(const double2* __restrict__ o, int64_t n, BinGeom g, uint32_t* __restrict__ H,
             int nchunks) {
  __shared__ uint32_t h[kBuckets];
  for (int b = threadIdx.x; b < kBuckets; b += kThreads) h[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + threadIdx.x + q * kThreads;
    if (i < n) atomicAdd(&h[bucket_of(o[i], g)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBuckets; b += kThreads) H[(size_t)b * nchunks + blockIdx.x] = h[b];
}

template <bool COUNT>
__global__ void __launch_bounds__(kThreads)
bucket_scatter(const double2* __restrict__ o, const double2* __restrict__ d,
               const int32_t* __restrict__ start, SceneDev sc, int64_t n, BinGeom g,
               const uint32_t* __restrict__ Hoff, int nchunks, RayRec* __restrict__ out,
               unsigned long long* __restrict__ stats) {
  __shared__ uint32_t off[kBuckets], cnt[kBuckets], pre[kBuckets];
  __shared__ RayRec stage[kChunk];
  __shared__ uint16_t stage_bucket[kChunk];
  for (int b = threadIdx.x; b < kBuckets; b += kThreads) {
    off[b] = Hoff[(size_t)b * nchunks + blockIdx.x];
    cnt[b] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  const int len = (int)min((int64_t)kChunk, n - base);
  RayRec r[kPerThread];
  uint32_t bk[kPerThread], rank[kPerThread];
  int32_t s[kPerThread];
  TriFirst f[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int j = threadIdx.x + q * kThreads;
    if (j < len) {
      const int64_t i = base + j;
      r[q].o = o[i];
      r[q].d = d[i];
      s[q] = start[i];
      r[q].idx = (int32_t)i;
      r[q].pad[0] = r[q].pad[1] = 0;
    }
  }
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {  // every gather issued before any is used
    const int j = threadIdx.x + q * kThreads;
    if (j < len && s[q] >= 0 && s[q] < sc.ntri) f[q] = sc.first[s[q]];
  }
  unsigned fb32 = 0, fb64 = 0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int j = threadIdx.x + q * kThreads;
    if (j < len) {
      const double2 ro = r[q].o, rd = r[q].d;
      r[q].start = -1;  // start triangle out of range
      if (s[q] >= 0 && s[q] < sc.ntri)
        r[q].start = first_exit_slot<COUNT>(ray32(ro.x, ro.y, rd.x, rd.y, sc.org_x, sc.org_y), ro,
                                            rd, f[q].x[0], f[q].x[1], f[q].x[2], f[q].y[0],
                                            f[q].y[1], f[q].y[2], f[q].tri, sc, fb32, fb64);
      bk[q] = bucket_of(ro, g);
      rank[q] = atomicAdd(&cnt[bk[q]], 1u);
    }
  }
  if (COUNT) {
    if (fb32) atomicAdd(&stats[1], (unsigned long long)fb32);
    if (fb64) atomicAdd(&stats[2], (unsigned long long)fb64);
  }
  __syncthreads();
  // exclusive scan of the chunk's bucket counts (kBuckets == kThreads: one bucket per thread)
  {
    const int b = threadIdx.x;
    const uint32_t v = cnt[b];
    pre[b] = v;
    __syncthreads();
    for (int s = 1; s < kBuckets; s <<= 1) {
      const uint32_t add = b >= s ? pre[b - s] : 0u;
      __syncthreads();
      pre[b] += add;
      __syncthreads();
    }
    pre[b] -= v;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int j = threadIdx.x + q * kThreads;
    if (j < len) {
      const uint32_t p = pre[bk[q]] + rank[q];
      stage[p] = r[q];
      stage_bucket[p] = (uint16_t)bk[q];
    }
  }
  __syncthreads();
  // consecutive staged records of one bucket go to consecutive destinations
  for (int j = threadIdx.x; j < len; j += kThreads) {
    const uint32_t b = stage_bucket[j];
    out[off[b] + (j - pre[b])] = stage[j];
  }
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

int n_chunks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

size_t scan_temp_bytes(size_t items) { return exclusive_scan_bytes((int64_t)items); }

size_t sort_temp_bytes(int64_t n) {
  size_t temp = 0;
  hipcub::DoubleBuffer<uint32_t> k(nullptr, nullptr);
  hipcub::DoubleBuffer<int32_t> v(nullptr, nullptr);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, k, v, (int)n, 0, 32);
  return temp;
}

}  // namespace

static_assert(kBuckets == kThreads, "the chunk scan assigns one bucket per thread");
static_assert(sizeof(RayRec) == 48, "ray record layout");

size_t bin_workspace_bytes(int64_t n) {
  const size_t items = (size_t)kBuckets * n_chunks(n);
  const size_t bucket = align256(sizeof(RayRec) * (size_t)n) + 2 * align256(sizeof(uint32_t) * items) +
                        align256(scan_temp_bytes(items));
  const size_t radix = 4 * align256(sizeof(uint32_t) * (size_t)n) + align256(sort_temp_bytes(n));
  // plus the parked results (16 B per ray, at the start)
  return align256(16 * (size_t)n) + (bucket > radix ? bucket : radix);
}

hipError_t launch_bin_rays(const SceneDev& sc, const RaysDev& in, int kind, void* workspace,
                           size_t ws_bytes, RaysDev* out, unsigned long long* stats,
                           hipStream_t stream) {
  const int64_t n = in.n;
  if (n <= 0 || n >= INT32_MAX || bin_workspace_bytes(n) > ws_bytes) return hipErrorInvalidValue;
  auto* p = static_cast<unsigned char*>(workspace);
  *out = in;
  out->park = reinterpret_cast<double2*>(p);
  p += align256(16 * (size_t)n);
  ws_bytes -= align256(16 * (size_t)n);
  hipError_t e;
  if (kind == kBinRadix) {
    const size_t a = align256(sizeof(uint32_t) * (size_t)n);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(p);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(p + a);
    int32_t* v0 = reinterpret_cast<int32_t*>(p + 2 * a);
    int32_t* v1 = reinterpret_cast<int32_t*>(p + 3 * a);
    size_t temp_bytes = ws_bytes - 4 * a;
    const int bs = 256;
    hipLaunchKernelGGL(start_keys, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, stream,
                       in.start, sc.perm, sc.ntri, n, k0, v0);
    // the walk reads each ray (and its caller's start triangle) through the sorted index
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipcub::DoubleBuffer<uint32_t> keys(k0, k1);
    hipcub::DoubleBuffer<int32_t> vals(v0, v1);
    e = hipcub::DeviceRadixSort::SortPairs(p + 4 * a, temp_bytes, keys, vals, (int)n, 0,
                                           bits_for(sc.ntri), stream);
    if (e != hipSuccess) return e;
    out->order = vals.Current();
    return hipSuccess;
  }
  const int nch = n_chunks(n);
  const size_t items = (size_t)kBuckets * nch;
  RayRec* recs = reinterpret_cast<RayRec*>(p);
  p += align256(sizeof(RayRec) * (size_t)n);
  uint32_t* H = reinterpret_cast<uint32_t*>(p);
  p += align256(sizeof(uint32_t) * items);
  uint32_t* Hoff = reinterpret_cast<uint32_t*>(p);
  p += align256(sizeof(uint32_t) * items);
  BinGeom g;
  const double cells = (double)(1 << kGridBits);
  g.x0 = sc.box_x0;
  g.y0 = sc.box_y0;
  g.sx = sc.box_x1 > sc.box_x0 ? cells / (sc.box_x1 - sc.box_x0) : 0.0;
  g.sy = sc.box_y1 > sc.box_y0 ? cells / (sc.box_y1 - sc.box_y0) : 0.0;
  hipLaunchKernelGGL(bucket_count, dim3(nch), dim3(kThreads), 0, stream, in.o, n, g, H, nch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan(H, Hoff, (int64_t)items, reinterpret_cast<uint32_t*>(p), stream);
  if (e != hipSuccess) return e;
  if (stats)
    hipLaunchKernelGGL(bucket_scatter<true>, dim3(nch), dim3(kThreads), 0, stream, in.o, in.d,
                       in.start, sc, n, g, Hoff, nch, recs, stats);
  else
    hipLaunchKernelGGL(bucket_scatter<false>, dim3(nch), dim3(kThreads), 0, stream, in.o, in.d,
                       in.start, sc, n, g, Hoff, nch, recs, stats);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  out->recs = recs;
  return hipSuccess;
}

}  // namespace ccsp
