// Operand splitting for the mixed-precision path (row a1 of the pass): every
// FP64 row x (one virtual of one hole slab, all auxiliary functions) becomes a
// sum of BF16 slices with round-to-nearest-even:
//     m = max_Q |x_Q| = f 2^E (f in [1/2, 1)),   y = x 2^-E   (|y| < 1)
//     s_1 = rint(y 2^8),  r_1 = y 2^8 - s_1              (|s_1| <= 256, |r_1| <= 1/2)
//     s_t = rint(r_{t-1} 2^9), r_t = r_{t-1} 2^9 - s_t   (|s_t| <= 256)
//     slice_t = s_t 2^(E - 8 - 9 (t-1))                    (exact in BF16: 8-bit integers
//                                                          times a power of two)
// so x = sum_t slice_t + O(2^(E - 8 - 9 k)).  Every slice of a row is an integer
// multiple of that row's unit 2^(E - 8 - 9(t-1)); products of slices from two
// rows are integer multiples of one common unit, which is what makes the FP32
// MFMA sums of the leading levels exact (see pair_bf16_v.hip).
// Range: the deepest kept level of two rows with exponent E is a multiple of
// 2^(2(E - 8) - 9(k - 1)), which must stay a normal FP32 number (>= 2^-126) for
// the sums to keep their bits; rows with 0 < max|x| < 2^(E_min - 1),
// E_min = bf16_min_row_exponent(k), set *range_flag and the pass reports the
// input as unsupported for BF16 slicing (FP64 and INT8 digits have no such
// limit).  E_min is -41 at k = 4, i.e. rows below ~2e-13.
// Slices are written true-scale, so a dot product of slices needs no rescaling.
//
// The kernel also returns every row's squared norm in FP64.  The pair kernel uses
// it for the diagonal V^{ii}_{aa} = ||B_ia||^2: there the dropped slice products
// (t, t) are sums of squares and would bias the energy instead of averaging out.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace dfpt2 {

// X: [nb][rows][ncols] FP64 (row stride ldx, matrix stride rows*ldx).
// out: BF16 in chunk-interleaved order [nb][rows_pad][ncols_pad/16][ns][16]: the
// ns slices of one 16-wide contraction chunk of a row are 32 ns contiguous bytes
// (one 128-byte line for ns = 4), which is what the pair kernel streams per
// chunk.  Rows >= rows and columns >= ncols are zeros.  One wave per row;
// blockIdx.y is the matrix index.  norm2 [nb][rows] gets the squared row norms.
__global__ __launch_bounds__(256) void split_rows_bf16_kernel(const double* X, long long ldx, int rows,
                                                              int rows_pad, int ncols, int ncols_pad, int ns,
                                                              __bf16* out, double* norm2, int* range_flag) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y, nb = gridDim.y;
  if (row >= rows_pad) return;
  (void)nb;
  __bf16* orow = out + ((size_t)b * rows_pad + row) * ncols_pad * ns;
  auto at = [&](int c, int t) -> __bf16& { return orow[((c >> 4) * ns + t) * 16 + (c & 15)]; };
  X += (size_t)b * rows * ldx;
  if (row >= rows) {
    for (int c = lane; c < ncols_pad; c += 64)
      for (int t = 0; t < ns; ++t) at(c, t) = (__bf16)0.0f;
    return;
  }
  const double* x = X + (size_t)row * ldx;
  double m = 0.0, q = 0.0;
  for (int c = lane; c < ncols; c += 64) {
    m = fmax(m, fabs(x[c]));
    q += x[c] * x[c];
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  q = wave_sum(q);
  if (norm2 && lane == 0) norm2[(size_t)b * rows + row] = q;
  int E = 0;
  if (m > 0.0) frexp(m, &E);
  if (range_flag && lane == 0 && m > 0.0 && E < bf16_min_row_exponent(ns)) atomicOr(range_flag, 1);
  for (int c = lane; c < ncols_pad; c += 64) {
    double r = (c < ncols && m > 0.0) ? ldexp(x[c], -E) * 256.0 : 0.0;
    int sh = E - 8;
    for (int t = 0; t < ns; ++t) {
      const double s = rint(r);
      r = (r - s) * 512.0;
      at(c, t) = (__bf16)(float)ldexp(s, sh);
      sh -= 9;
    }
  }
}

hipError_t launch_split_rows_bf16(const double* X, long long ldx, int nb, int rows, int rows_pad, int ncols,
                                  int ncols_pad, int ns, __bf16* out, double* norm2, int* range_flag,
                                  hipStream_t st) {
  if (rows_pad <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_rows_bf16_kernel, dim3((rows_pad + 3) / 4, nb), dim3(256), 0, st, X, ldx, rows,
                     rows_pad, ncols, ncols_pad, ns, out, norm2, range_flag);
  return hipGetLastError();
}


// ------------------------------------------------------------------ FP8 slices
// FP8 (OCP e4m3) operands with per-block power-of-two scales: every 32-wide block
// of a row (32 consecutive auxiliary functions of one virtual of one hole) is
// split on its own, relative to the block's largest magnitude m = f 2^E:
//     y = x 2^(4 - E)               (|y| < 16)
//     s_1 = rint(y),  r_1 = y - s_1            (|s_1| <= 16, |r_1| <= 1/2)
//     s_t = rint(32 r_{t-1}), r_t = 32 r_{t-1} - s_t   (|s_t| <= 16)
// Integers of magnitude <= 16 are exact in e4m3; slice t of the block carries the
// E8M0 scale 2^(E - 4 - 5 (t - 1)), applied by the scaled MFMA.  So x = sum_t
// s_t 2^(E - 4 - 5(t-1)) + O(2^(E - 5 k)) per element: about 5 bits per slice.
//
// Layout, chosen for the lane layout of the 32x32x64 scaled MFMA (a lane of half
// h holds the 16-element groups h and 2 + h of a 64-wide chunk, and the scale of
// K-block h comes from that half):
//   out:    [nb][rows_pad][ncols_pad/64][ns][64] bytes; within one slice of one
//           chunk, element kk (0..63) sits at 32 ((kk % 32) / 16) + (kk % 16) + 16 (kk / 32)
//   scales: [nb][rows_pad][ncols_pad/64][2] words; byte t of word h is the E8M0
//           scale of slice t of K-block h (ns <= 4)
// Blocks whose largest magnitude is below 2^-100 (E8M0 underflow of trailing
// slices) keep only the slices whose scale is representable.
namespace {
__device__ inline uint32_t e4m3_of_int(int n) {  // |n| <= 16, exact
  if (n == 0) return 0u;
  const uint32_t sgn = n < 0 ? 0x80u : 0u;
  const int m = n < 0 ? -n : n;
  const int k = 31 - __clz(m);                  // floor(log2 m), 0..4
  const int mant = ((m - (1 << k)) << 3) >> k;  // 3 mantissa bits, exact for m <= 16
  return sgn | (uint32_t)((k + 7) << 3) | (uint32_t)mant;
}
}  // namespace

__global__ __launch_bounds__(256) void split_rows_fp8_kernel(const double* X, long long ldx, int rows, int rows_pad,
                                                             int ncols, int ncols_pad, int ns, uint8_t* out,
                                                             uint32_t* scales, double* norm2) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y;
  if (row >= rows_pad) return;
  const int nch = ncols_pad >> 6;
  uint8_t* orow = out + ((size_t)b * rows_pad + row) * (size_t)ncols_pad * ns;
  uint32_t* srow = scales + ((size_t)b * rows_pad + row) * (size_t)nch * 2;
  const int h = (lane & 31) >> 4, e = (lane & 15) + 16 * (lane >> 5);
  const double* x = X + ((size_t)b * rows + (row < rows ? row : 0)) * ldx;
  double q = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    const int c = ch * 64 + lane;
    const double v = (row < rows && c < ncols) ? x[c] : 0.0;
    q += v * v;
    double m = fabs(v);
    for (int off = 16; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));  // within the 32-lane block
    int E = 0;
    if (m > 0.0) frexp(m, &E);
    double r = (m > 0.0) ? ldexp(v, 4 - E) : 0.0;
    uint32_t word = 0u;
    for (int t = 0; t < ns; ++t) {
      const double s = rint(r);
      r = (r - s) * 32.0;
      int sb = 127 + E - 4 - 5 * t;
      int si = (int)s;
      if (sb < 0) {  // scale not representable: drop this slice
        sb = 0;
        si = 0;
      }
      orow[((size_t)ch * ns + t) * 64 + 32 * h + e] = (uint8_t)e4m3_of_int(si);
      word |= (uint32_t)sb << (8 * t);
    }
    if ((lane & 31) == 0) srow[ch * 2 + (lane >> 5)] = word;
  }
  q = wave_sum(q);
  if (norm2 && lane == 0 && row < rows) norm2[(size_t)b * rows + row] = q;
}

hipError_t launch_split_rows_fp8(const double* X, long long ldx, int nb, int rows, int rows_pad, int ncols,
                                 int ncols_pad, int ns, uint8_t* out, uint32_t* scales, double* norm2,
                                 hipStream_t st) {
  if (rows_pad <= 0 || nb <= 0) return hipSuccess;
  if (ncols_pad % 64 != 0 || ns < 1 || ns > 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_rows_fp8_kernel, dim3((rows_pad + 3) / 4, nb), dim3(256), 0, st, X, ldx, rows, rows_pad,
                     ncols, ncols_pad, ns, out, scales, norm2);
  return hipGetLastError();
}


// ------------------------------------------------------------------ INT8 digits
// Integer slicing for the INT8 MFMA path: every row x (largest magnitude
// m = f 2^E, f in [1/2, 1)) is rounded once to the integer
//     Z = rint(x 2^(6 + 8 (ns-1) - E))          (|Z| <= 2^(6 + 8 (ns-1)))
// and Z is written in balanced base 256: Z = sum_t d_t 256^(ns-1-t) with
// d_t in [-128, 127] for t >= 1 and |d_0| <= 64 (the carries of the lower digits
// add at most 1/2 to the top one).  So x = 2^(E - 6) sum_t d_t 2^(-8t) up to
// 2^(E - 7 - 8(ns-1)), and products of two rows' digits are exact integers: the
// pair kernel sums them in INT32 (pair_i8.hip) and applies the row scales
// 2^(E_a - 6) 2^(E_b - 6) once, in FP64.  Unlike BF16 slices, digits have no
// exponent of their own, so no row is too small to split.
//
// Layout (chunk-major, for the pair kernel's direct loads):
//   out:  [nb][ncols_pad/32][rows_pad][ns][32] bytes: one 32-wide contraction chunk
//         of 64 consecutive rows is 64 x 32 ns contiguous bytes
//   rexp: [nb][rows_pad] the row exponent E - 6 (0 for zero and padding rows)
// One wave per row; lane l handles four consecutive columns per 256-wide stretch.
__global__ __launch_bounds__(256) void split_rows_i8_kernel(const double* X, long long ldx, int rows, int rows_pad,
                                                            int ncols, int ncols_pad, int ns, int8_t* out, int* rexp,
                                                            double* norm2) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y;
  if (row >= rows_pad) return;
  const int nch = ncols_pad >> 5;
  const double* x = X + ((size_t)b * rows + (row < rows ? row : 0)) * ldx;
  double m = 0.0, q = 0.0;
  if (row < rows) {
    for (int c = lane; c < ncols; c += 64) {
      m = fmax(m, fabs(x[c]));
      q += x[c] * x[c];
    }
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  q = wave_sum(q);
  int E = 0;
  if (m > 0.0) frexp(m, &E);
  if (lane == 0) {
    if (norm2 && row < rows) norm2[(size_t)b * rows + row] = q;
    rexp[(size_t)b * rows_pad + row] = m > 0.0 ? E - 6 : 0;
  }
  const int sh = 6 + 8 * (ns - 1) - E;
  for (int c0 = 4 * lane; c0 < ncols_pad; c0 += 256) {
    uint32_t word[8];  // ns <= 8
    for (int t = 0; t < ns; ++t) word[t] = 0u;
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      long long Z = (row < rows && c < ncols && m > 0.0) ? (long long)rint(ldexp(x[c], sh)) : 0;
      for (int t = ns - 1; t >= 1; --t) {
        const long long d = ((Z + 128) & 255) - 128;
        Z = (Z - d) >> 8;
        word[t] |= ((uint32_t)d & 0xffu) << (8 * e);
      }
      word[0] |= ((uint32_t)Z & 0xffu) << (8 * e);
    }
    const int ch = c0 >> 5, kk = c0 & 31;
    int8_t* dst = out + (((size_t)b * nch + ch) * rows_pad + row) * (size_t)(32 * ns) + kk;
    for (int t = 0; t < ns; ++t) *reinterpret_cast<uint32_t*>(dst + 32 * t) = word[t];
  }
}

hipError_t launch_split_rows_i8(const double* X, long long ldx, int nb, int rows, int rows_pad, int ncols,
                                int ncols_pad, int ns, int8_t* out, int* rexp, double* norm2, hipStream_t st) {
  if (rows_pad <= 0 || nb <= 0) return hipSuccess;
  if (ncols_pad % 32 != 0 || ns < 1 || ns > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_rows_i8_kernel, dim3((rows_pad + 3) / 4, nb), dim3(256), 0, st, X, ldx, rows, rows_pad,
                     ncols, ncols_pad, ns, out, rexp, norm2);
  return hipGetLastError();
}

}  // namespace dfpt2
