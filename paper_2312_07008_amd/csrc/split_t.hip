// Amplitude splitting for the split-BF16 density product (row a4 of the pass).
//
// For one unordered pair {i <= j} with amplitude matrix T = T^{ij} (n_v x n_v),
// the two ordered pairs contribute X1 Y1^T + X2 Y2^T to D (Eq. A9 with zero
// cumulants, see density_f64.hip), with, for a virtual c along the contraction,
//     m = 0:  X1[a][c] = T[a][c]
//     m = 1:  X2[a][c] = T[c][a]
//     m = 2:  Y1[b][c] = 2 T[b][c] - T[c][b]
//     m = 3:  Y2[b][c] = 2 T[c][b] - T[b][c]
// BF16 slices (split_t_bf16_kernel): every row of the four matrices is split
// per 64-column block, from the largest magnitude of the row within the block
// (amp_tile.h), into ns true-scale BF16 slices whose integer digits satisfy
// sum_t s_t 512^(ns-1-t) = rint(x 2^(8 + 9(ns-1) - E)), so the density kernel can
// sum the slice products of one pair and one block exactly in FP32.  The kernel
// takes the block maxima itself: every workgroup holds whole 64-column blocks of
// its rows.  Output per pair q: [q][m][rows_pad][n_v_pad/16][ns][16] (rows and
// columns n_v .. n_v_pad - 1 are zeros), the chunk-interleaved layout of B's
// slices.  The matrix stride rows_pad >= n_v_pad lets the density kernel load
// 128-row panels; rows n_v_pad .. rows_pad - 1 are not written (the density
// kernel's waves that load them form no products from them).  The main pass
// forms the same slices in the pair epilogue (epi_split_bf16.hip); this kernel
// serves amplitude matrices already in memory (the active blocks).
//
// The diagonal of the pair's contribution, w_q sum_c (X1 Y1 + X2 Y2)[a][c] =
// w_q sum_c 2 (x^2 - x y + y^2) with x = T[a][c], y = T[c][a], is summed in
// FP64, one partial per (row, 64-column block) in dgp, and accumulated in a
// fixed order by diag_accumulate_kernel: on the diagonal the rows of X and Y
// carry the same amplitudes, so the slice products the density kernel drops
// would not average out there, and the diagonal carries the trace of D.  The
// density kernel leaves the diagonal out.
//
// INT8 digits (split_t_i8_kernel) keep one exponent per row: the four row maxima
// and the diagonal partial sums come from the pair kernel's epilogue
// (pair_epilogue.h) or from pair_row_stats_kernel.
#include <cmath>

#include "amp_tile.h"
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

using amp::LD;
using amp::TB;
using amp::u4;

// ---------------------------------------------------------------- slices
// Workgroup = (row block A, column block C, pair q): rows A x columns C of the
// four matrices.  x = T[a][c] comes straight from global memory, y = T[c][a]
// from the mirror tile T[C, A] staged in LDS (amp::load_tile).  The thread's 16
// columns are exactly one 16-wide chunk of the output row; the slices of each
// matrix go through the LDS tile to whole-row stores (amp::split_block_rows).
template <int NS, bool VEC>
__global__ __launch_bounds__(256) void split_t_bf16_kernel(const double* T, const int* slot, int n_v, int n_v_pad,
                                                           int rows_pad, int nt, double* dgp, __bf16* out) {
  // T[C-block row][A-block col], then the staged slices
  __shared__ __attribute__((aligned(16))) double tm[TB][LD];
  const int A = blockIdx.x / nt, C = blockIdx.x - (blockIdx.x / nt) * nt, q = blockIdx.y;
  const double* Tp = T + (size_t)(slot ? slot[q] : q) * n_v * n_v;
  const int tid = threadIdx.x;
  const int r = tid >> 2, k4 = tid & 3;
  const int row = A * TB + r;
  double x[16];
  amp::load_tile<VEC>(Tp, n_v, A, C, tm, x, true);
  double y[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) y[j] = tm[k4 * 16 + j][r];
  const size_t row_elems = (size_t)n_v_pad * NS, mat_elems = (size_t)rows_pad * row_elems;
  __bf16* base = out + (size_t)q * 4 * mat_elems + (size_t)(A * TB) * row_elems + (size_t)(C * 4) * (NS * 16);
  const double dg = amp::split_block_rows<NS>(x, y, reinterpret_cast<u4*>(&tm[0][0]), base, mat_elems, row_elems);
  if (k4 == 0 && row < n_v) dgp[((size_t)q * nt + C) * n_v_pad + row] = dg;
}

// ---------------------------------------------------------------- INT8 digits
// The same four matrices as balanced base-256 digits for the INT8 density kernel
// (density_i8.hip): per row, Z = rint(v 2^(6 + 8 (NS-1) - E)) with 2^E above the
// row's largest magnitude (tmax), digits d_t in [-128, 127] (|d_0| <= 64), row
// value 2^(E - 6) sum_t d_t 2^(-8t).  Layout, chunk-major as for B (split.hip):
// [q][m][n_v_pad/32][n_v_pad][NS][32] bytes, and the row exponents E - 6 in
// rexp[q][m][n_v_pad] (0 for zero rows).  Thread (row r, quarter k4) holds 16
// consecutive columns, i.e. one half of a 32-wide chunk: one 16-byte piece per
// digit.  The workgroup's part of a matrix is two contiguous runs (its two
// chunks, 64 rows of 32 NS bytes each), so the pieces go through the LDS tile
// and every store of a wave writes 1 KB contiguous.
template <int NS, bool VEC>
__global__ __launch_bounds__(256) void split_t_i8_kernel(const double* T, const int* slot, int n_v, int n_v_pad,
                                                         int nt, const unsigned long long* tmax, int8_t* out,
                                                         int* rexp) {
  // T[C-block row][A-block col], then the staged digits
  __shared__ __attribute__((aligned(16))) double tm[TB][LD];
  const int A = blockIdx.x / nt, C = blockIdx.x - (blockIdx.x / nt) * nt, q = blockIdx.y;
  const double* Tp = T + (size_t)(slot ? slot[q] : q) * n_v * n_v;
  const int tid = threadIdx.x;
  const int r = tid >> 2, k4 = tid & 3;
  const int row = A * TB + r;
  double x[16];
  amp::load_tile<VEC>(Tp, n_v, A, C, tm, x, true);
  double y[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) y[j] = tm[k4 * 16 + j][r];

  const int nck = n_v_pad >> 5;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double mx = __longlong_as_double((long long)tmax[((size_t)q * 4 + m) * n_v_pad + row]);
    int E = 0;
    if (mx > 0.0) frexp(mx, &E);
    if (C == 0 && k4 == 0) rexp[((size_t)q * 4 + m) * n_v_pad + row] = mx > 0.0 ? E - 6 : 0;
    uint32_t word[NS][4];
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) word[t][u] = 0u;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double v = m == 0 ? x[j] : m == 1 ? y[j] : m == 2 ? 2.0 * x[j] - y[j] : 2.0 * y[j] - x[j];
      long long Z = (mx > 0.0) ? (long long)rint(ldexp(v, 6 + 8 * (NS - 1) - E)) : 0;
#pragma unroll
      for (int t = NS - 1; t >= 1; --t) {
        const long long d = ((Z + 128) & 255) - 128;
        Z = (Z - d) >> 8;
        word[t][j >> 2] |= ((uint32_t)d & 0xffu) << (8 * (j & 3));
      }
      word[0][j >> 2] |= ((uint32_t)Z & 0xffu) << (8 * (j & 3));
    }
    // staged as [2 chunks][64 rows][2 NS pieces of 16 bytes]: 256 NS pieces
    u4* stg = reinterpret_cast<u4*>(&tm[0][0]);
    __syncthreads();  // every earlier read of tm is done
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      u4 v4;
      v4[0] = word[t][0];
      v4[1] = word[t][1];
      v4[2] = word[t][2];
      v4[3] = word[t][3];
      stg[(k4 >> 1) * (128 * NS) + r * (2 * NS) + 2 * t + (k4 & 1)] = v4;
    }
    __syncthreads();
    int8_t* mb = out + (((size_t)q * 4 + m) * nck + 2 * C) * n_v_pad * (size_t)(32 * NS);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int P = i * 256 + tid, c2 = P / (128 * NS), off = P - c2 * (128 * NS);
      *reinterpret_cast<u4*>(mb + ((size_t)c2 * n_v_pad + (size_t)A * TB) * (32 * NS) + (size_t)off * 16) = stg[P];
    }
  }
}

// ---------------------------------------------------------------- row data
// The row data the split kernels read, for amplitude matrices that did not pass
// through a pair-kernel epilogue (the amplitudes of the active blocks, rotated to
// the natural orbitals of Gamma_act): for matrix T = T + slot[q] n_v^2, the
// largest magnitudes of the rows of T, T^T, 2T - T^T and 2T^T - T (atomic max on
// the bit patterns of non-negative doubles, so independent of order) and the
// diagonal partial sums 2 (x^2 - x y + y^2) per (row a, 64-column block C), as
// pair_epilogue.h records them.  Workgroup (A, C, q) as in the split kernels.
template <bool VEC>
__global__ __launch_bounds__(256) void pair_row_stats_kernel(const double* T, const int* slot, int n_v, int n_v_pad,
                                                             int nt, unsigned long long* tmax, double* dgp) {
  __shared__ double tm[TB][LD];
  const int A = blockIdx.x / nt, C = blockIdx.x - (blockIdx.x / nt) * nt, q = blockIdx.y;
  const double* Tp = T + (size_t)(slot ? slot[q] : q) * n_v * n_v;
  const int tid = threadIdx.x;
  const int r = tid >> 2, k4 = tid & 3;
  const int row = A * TB + r;
  double x[16];
  amp::load_tile<VEC>(Tp, n_v, A, C, tm, x, true);
  double mx[4] = {0.0, 0.0, 0.0, 0.0}, dg = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double xv = x[j], yv = tm[k4 * 16 + j][r];
    mx[0] = fmax(mx[0], fabs(xv));
    mx[1] = fmax(mx[1], fabs(yv));
    mx[2] = fmax(mx[2], fabs(2.0 * xv - yv));
    mx[3] = fmax(mx[3], fabs(2.0 * yv - xv));
    dg += 2.0 * (xv * xv - xv * yv + yv * yv);
  }
  // over the row's quad (the four 16-column quarters), in a fixed pattern
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    mx[m] = fmax(mx[m], amp::quad_xor<0xB1>(mx[m]));
    mx[m] = fmax(mx[m], amp::quad_xor<0x4E>(mx[m]));
  }
  dg += amp::quad_xor<0xB1>(dg);
  dg += amp::quad_xor<0x4E>(dg);
  if (k4 == 0 && row < n_v) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
      atomicMax(tmax + ((size_t)q * 4 + m) * n_v_pad + row, (unsigned long long)__double_as_longlong(mx[m]));
    dgp[((size_t)q * nt + C) * n_v_pad + row] = dg;
  }
}

hipError_t launch_pair_row_stats(const double* T, const int* slot, int n_pairs, int n_v, int n_v_pad,
                                 unsigned long long* tmax, double* dgp, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (n_v_pad % TB != 0 || n_v_pad < n_v) return hipErrorInvalidValue;
  const int nt = n_v_pad / TB;
  dim3 grid(nt * nt, n_pairs), block(256);
  if (n_v % 2 == 0)
    hipLaunchKernelGGL(pair_row_stats_kernel<true>, grid, block, 0, st, T, slot, n_v, n_v_pad, nt, tmax, dgp);
  else
    hipLaunchKernelGGL(pair_row_stats_kernel<false>, grid, block, 0, st, T, slot, n_v, n_v_pad, nt, tmax, dgp);
  return hipGetLastError();
}

// diag[a] += sum over pairs q and column blocks of w_q dgp[q][blk][a], in a fixed
// order (strided per thread, then a fixed tree), so the result is reproducible
__global__ __launch_bounds__(256) void diag_accumulate_kernel(const double* dgp, const int2* pairs, const double* pw,
                                                              double w, int n_pairs, int nt, int n_v_pad,
                                                              double* diag) {
  __shared__ double red[256];
  const int a = blockIdx.x, t = threadIdx.x;
  double v = 0.0;
  for (int i = t; i < n_pairs * nt; i += 256) {
    const int q = i / nt;
    const int2 pr = pairs[q];
    double wq = w * (pr.x == pr.y ? 0.5 : 1.0);
    if (pw) wq *= pw[q];
    v += wq * dgp[(size_t)i * n_v_pad + a];
  }
  red[t] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) diag[a] += red[0];
}

hipError_t launch_diag_accumulate(const double* dgp, const int2* pairs, const double* pw, double w, int n_pairs,
                                  int n_v, int n_v_pad, double* diag, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (n_v_pad % TB != 0 || n_v_pad < n_v) return hipErrorInvalidValue;
  hipLaunchKernelGGL(diag_accumulate_kernel, dim3(n_v), dim3(256), 0, st, dgp, pairs, pw, w, n_pairs, n_v_pad / TB,
                     n_v_pad, diag);
  return hipGetLastError();
}

hipError_t launch_split_t_bf16(const double* T, const int* slot, const int2* pairs, const double* pw, double w,
                               int n_pairs, int n_v, int n_v_pad, int rows_pad, int ns, double* dgp, __bf16* out,
                               double* diag, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (n_v_pad % TB != 0 || n_v_pad < n_v || rows_pad % TB != 0 || rows_pad < n_v_pad) return hipErrorInvalidValue;
  const int nt = n_v_pad / TB;
  hipError_t e;
  dim3 grid(nt * nt, n_pairs), block(256);
  const bool vec = (n_v % 2) == 0;
#define SPLIT_T_BF16(NS_)                                                                                          \
  do {                                                                                                             \
    if (vec)                                                                                                       \
      hipLaunchKernelGGL((split_t_bf16_kernel<NS_, true>), grid, block, 0, st, T, slot, n_v, n_v_pad, rows_pad, nt, \
                         dgp, out);                                                                                \
    else                                                                                                           \
      hipLaunchKernelGGL((split_t_bf16_kernel<NS_, false>), grid, block, 0, st, T, slot, n_v, n_v_pad, rows_pad,    \
                         nt, dgp, out);                                                                            \
  } while (0)
  switch (ns) {
    case 2: SPLIT_T_BF16(2); break;
    case 3: SPLIT_T_BF16(3); break;
    case 4: SPLIT_T_BF16(4); break;
    default: return hipErrorInvalidValue;
  }
#undef SPLIT_T_BF16
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_diag_accumulate(dgp, pairs, pw, w, n_pairs, n_v, n_v_pad, diag, st);
}

hipError_t launch_split_t_i8(const double* T, const int* slot, const int2* pairs, const double* pw, double w,
                             int n_pairs, int n_v, int n_v_pad, int ns, const unsigned long long* tmax,
                             const double* dgp, int8_t* out, int* rexp, double* diag, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (n_v_pad % TB != 0 || n_v_pad < n_v) return hipErrorInvalidValue;
  const int nt = n_v_pad / TB;
  hipError_t e;
  dim3 grid(nt * nt, n_pairs), block(256);
  const bool vec = (n_v % 2) == 0;
#define SPLIT_T_I8(NS_)                                                                                         \
  do {                                                                                                          \
    if (vec)                                                                                                    \
      hipLaunchKernelGGL((split_t_i8_kernel<NS_, true>), grid, block, 0, st, T, slot, n_v, n_v_pad, nt, tmax, out, \
                         rexp);                                                                                 \
    else                                                                                                        \
      hipLaunchKernelGGL((split_t_i8_kernel<NS_, false>), grid, block, 0, st, T, slot, n_v, n_v_pad, nt, tmax,   \
                         out, rexp);                                                                            \
  } while (0)
  switch (ns) {
    case 2: SPLIT_T_I8(2); break;
    case 3: SPLIT_T_I8(3); break;
    case 4: SPLIT_T_I8(4); break;
    case 5: SPLIT_T_I8(5); break;
    default: return hipErrorInvalidValue;
  }
#undef SPLIT_T_I8
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(diag_accumulate_kernel, dim3(n_v), dim3(256), 0, st, dgp, pairs, pw, w, n_pairs, nt, n_v_pad,
                     diag);
  return hipGetLastError();
}

}  // namespace dfpt2
