// Exact sign of small sums of products of binary64 numbers, for host and device.
//
// Each product a*b is split without error into hi + lo with an FMA (the TwoProduct transform of
// Dekker 1971, FMA form), and the terms are accumulated with Knuth's TwoSum into a nonoverlapping
// expansion (Shewchuk 1997, Grow-Expansion without zero elimination, so that the expansion length
// is static and the compiler can keep it in registers). The largest nonzero component carries the
// sign of the exact sum. Valid while no product underflows, which the walk's inputs (finite
// coordinates of magnitude < 2^64) guarantee for every case the filters hand over.
//
// Translation units must be compiled with -ffp-contract=off: TwoSum relies on every addition being
// rounded on its own.
#pragma once
#include <hip/hip_runtime.h>

namespace ccsp {

#define CCSP_HD __host__ __device__ __forceinline__

CCSP_HD void two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  const double bv = x - a;
  const double av = x - bv;
  y = (a - av) + (b - bv);
}

CCSP_HD void two_product(double a, double b, double& x, double& y) {
  x = a * b;
  y = fma(a, b, -x);
}

// h[0..m-1] += b, keeping the expansion nonoverlapping; the length grows by one.
template <int M>
CCSP_HD void grow(double (&h)[M], int m, double b) {
  double q = b;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    if (i < m) {
      double s, t;
      two_sum(q, h[i], s, t);
      h[i] = t;
      q = s;
    }
  }
  h[m] = q;
}

// sign( sum_k sg[k] * a[k] * b[k] ) exactly, for N products.
template <int N>
CCSP_HD int exact_sum_of_products_sign(const double (&a)[N], const double (&b)[N], const int (&sg)[N]) {
  double h[2 * N];
#pragma unroll
  for (int i = 0; i < 2 * N; ++i) h[i] = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double hi, lo;
    two_product(a[k], b[k], hi, lo);
    if (sg[k] < 0) {
      hi = -hi;
      lo = -lo;
    }
    grow(h, 2 * k, lo);
    grow(h, 2 * k + 1, hi);
  }
  int s = 0;
#pragma unroll
  for (int i = 0; i < 2 * N; ++i)
    if (h[i] != 0.0) s = h[i] > 0.0 ? 1 : -1;  // the last nonzero component is the largest
  return s;
}

// sign of D(v) = dx*(vy-oy) - dy*(vx-ox) = dx*vy - dx*oy - dy*vx + dy*ox
CCSP_HD int side_exact(double ox, double oy, double dx, double dy, double vx, double vy) {
  const double a[4] = {dx, dx, dy, dy};
  const double b[4] = {vy, oy, vx, ox};
  const int sg[4] = {+1, -1, -1, +1};
  return exact_sum_of_products_sign(a, b, sg);
}

// sign of (b-a) x (c-a) = bx*cy - bx*ay - ax*cy - by*cx + by*ax + ay*cx
CCSP_HD int orient_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  const double p[6] = {bx, bx, ax, by, by, ay};
  const double q[6] = {cy, ay, cy, cx, ax, cx};
  const int sg[6] = {+1, -1, -1, -1, +1, +1};
  return exact_sum_of_products_sign(p, q, sg);
}

// Binary64 filter for D(v): the rounded evaluation (two differences, two products, one
// difference) has error below 2u*M + u|D| with M = |dx(vy-oy)| + |dy(vx-ox)|, u = 2^-53; the
// threshold 3u*M_computed + 2^-1000 covers it with margin, including subnormal results.
CCSP_HD int side_fp64_filtered(double ox, double oy, double dx, double dy, double vx, double vy,
                               bool& certain) {
  const double p = dx * (vy - oy);
  const double q = dy * (vx - ox);
  const double D = p - q;
  const double M = fabs(p) + fabs(q);
  certain = fabs(D) > 0x1.8p-52 * M + 0x1p-1000;
  return D > 0.0 ? 1 : (D < 0.0 ? -1 : 0);
}

}  // namespace ccsp
