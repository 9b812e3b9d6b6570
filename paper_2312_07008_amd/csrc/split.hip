// Operand splitting for the mixed-precision path (row a1 of the pass): every
// FP64 row x (one virtual of one hole slab, all auxiliary functions) becomes a
// sum of BF16 slices with round-to-nearest-even:
//     m = max_Q |x_Q| = f 2^E (f in [1/2, 1)),   y = x 2^-E   (|y| < 1)
//     s_1 = rint(y 2^8),  r_1 = y 2^8 - s_1              (|s_1| <= 256, |r_1| <= 1/2)
//     s_t = rint(r_{t-1} 2^9), r_t = r_{t-1} 2^9 - s_t   (|s_t| <= 256)
//     slice_t = s_t 2^(E - 8 - 9 (t-1))                    (exact in BF16: 8-bit integers
//                                                          times a power of two)
// so x = sum_t slice_t + O(2^(E - 8 - 9 k)).  (Rows whose largest magnitude is
// below 2^-90 would push trailing slices into BF16's subnormal range and lose
// bits.)  Every slice of a row is an integer multiple of that row's unit 2^(E - 8 - 9(t-1)); products of slices from two
// rows are integer multiples of one common unit, which is what makes the FP32
// MFMA sums of the leading levels exact (see pair_bf16.hip).
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
                                                              __bf16* out, double* norm2) {
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
                                  int ncols_pad, int ns, __bf16* out, double* norm2, hipStream_t st) {
  if (rows_pad <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_rows_bf16_kernel, dim3((rows_pad + 3) / 4, nb), dim3(256), 0, st, X, ldx, rows,
                     rows_pad, ncols, ncols_pad, ns, out, norm2);
  return hipGetLastError();
}

}  // namespace dfpt2
