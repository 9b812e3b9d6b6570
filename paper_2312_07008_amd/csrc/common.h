// Internal helpers shared by the HIP translation units of libdfpt2.so.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace dfpt2 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// Error-free transformations for double-double accumulation (Knuth two-sum).
__host__ __device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += x
__host__ __device__ inline void dd_add(double& hi, double& lo, double x) {
  double s, e;
  two_sum(hi, x, s, e);
  lo += e;
  two_sum(s, lo, hi, lo);
}

// (hi, lo) += (bh, bl)
__host__ __device__ inline void dd_add_dd(double& hi, double& lo, double bh, double bl) {
  double s, e;
  two_sum(hi, bh, s, e);
  e += lo + bl;
  two_sum(s, e, hi, lo);
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Compensated wave reduction of a (hi, lo) pair.
__device__ inline void wave_sum_dd(double& hi, double& lo) {
  for (int off = 32; off > 0; off >>= 1) {
    double oh = __shfl_xor(hi, off, 64);
    double ol = __shfl_xor(lo, off, 64);
    dd_add_dd(hi, lo, oh, ol);
  }
}

// Tile pair index tp -> (I, J) with I <= J over an nt x nt upper triangle,
// enumerated row by row: (0,0) (0,1) .. (0,nt-1) (1,1) ..
__host__ __device__ inline void tile_pair(int tp, int nt, int& I, int& J) {
  int i = 0, rem = tp;
  while (rem >= nt - i) { rem -= nt - i; ++i; }
  I = i;
  J = i + rem;
}

}  // namespace dfpt2
