// Kernel launch interfaces used by the host library (internal).
#pragma once
#include "common.h"

namespace dfpt2 {

// ---------------------------------------------------------------- pair kernel
struct PairKernelArgs {
  const double* B;      // [n_h][n_v][n_aux]
  const double* eps_h;  // [n_h]
  const double* eps_v;  // [n_v]
  const int2* pairs;    // [n_pairs] unordered (i <= j)
  double* T;            // [n_pairs][n_v][n_v] amplitudes out, or null
  double* Vr;           // [n_pairs][n_v][n_v] renormalized integrals out, or null
  double* epart;        // [n_pairs][nTP] energy partial per tile pair, or null
  double* tpart;        // [n_pairs][nTP] ||T||^2 partial per tile pair, or null
  unsigned long long* tmax;  // INT8 digits only, or null: row maxima for the density digits (PairSlicedArgs)
  double* dgp;               // with tmax: diagonal partial sums
  int n_v, n_aux, nt, nTP;
  double s;
  double e_weight;      // energy weight of one ordered pair
};
hipError_t launch_pair_gemm_f64(const PairKernelArgs& a, int n_pairs, hipStream_t st);

// ------------------------------------------------ sliced (BF16 / FP8) pair kernels
struct PairSlicedArgs {
  const void* Bs;       // BF16: [n_h][n_v_pad][n_aux_pad/16][ns][16] slices (split.hip)
                        // FP8:  [n_h][n_v_pad][n_aux_pad/64][ns][64] e4m3 slices (split.hip)
                        // INT8: [n_h][n_aux_pad/32][n_v_pad][ns][32] balanced base-256 digits (split.hip)
  const uint32_t* scales;  // FP8 only: [n_h][n_v_pad][n_aux_pad/64][2] E8M0 scale words
  const int* rexp;      // INT8 only: [n_h][n_v_pad] row exponents (row value = 2^rexp sum_t d_t 2^-8t)
  const double* norm2;  // [n_h][n_v] ||B_ia||^2 in FP64: exact diagonal of V^{ii}
  const double* eps_h;
  const double* eps_v;
  const int2* pairs;
  double* T;            // [n_pairs][n_v][n_v] FP64 amplitudes out, or null
  double* Vr;           // [n_pairs][n_v][n_v] renormalized integrals out, or null
  double* epart;
  double* tpart;
  unsigned long long* tmax;  // INT8 only, or null: [n_pairs][4][n_v_pad] row maxima for the density digits
  double* dgp;               // with tmax: [n_pairs][nt][n_v_pad] diagonal partial sums (split_t.hip)
  int n_v, n_v_pad, n_aux_pad, nt, nTP;  // n_v_pad: slab rows of Bs; nt: 64-wide tiles of n_v;
                                        // nTP: workgroup tiles per pair
  int n_v_pad_d;        // row stride of tmax / dgp (64-multiple)
  int n_blk_pairs;      // pairs of this launch (set by the launcher)
  double s;
  double e_weight;
};
// the same pass as two kernels (pair_bf16_v.hip): the product V into a.T (slabs of a
// multiple of 128 rows), then the epilogue, which overwrites V in a.T with T
// (store) or only forms the energy partials (!store)
hipError_t launch_pair_v_bf16(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st);
hipError_t launch_pair_epi_bf16(const PairSlicedArgs& a, int n_pairs, bool store, hipStream_t st);
// the epilogue of the split-BF16 density pass (epi_split_bf16.hip): from the V in
// a.T, the energy and norm partials as above, and instead of T the ns2 BF16 slices
// of the four density operands (layout of launch_split_t_bf16, matrices rows_pad
// rows apart) in Ts and the diagonal partials in dgp ([n_pairs][nt][n_v_pad_d])
hipError_t launch_pair_epi_split_bf16(const PairSlicedArgs& a, int n_pairs, int ns2, int rows_pad, __bf16* Ts,
                                      double* dgp, hipStream_t st);
hipError_t launch_pair_gemm_fp8(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st);
hipError_t launch_pair_gemm_i8(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st);
// the INT8-digit product alone (pair_i8_v.hip): V into a.T (slabs of a multiple of
// 128 rows), for pair_epi_bf16's epilogue
hipError_t launch_pair_v_i8(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st);
// largest n_aux_pad for which the INT8 level sums stay exact with ns digits
int pair_i8_max_aux_pad(int ns);
// FP64 rows -> BF16 / FP8 slices, see split.hip.  BF16: rows whose largest
// magnitude lies below 2^(bf16_min_row_exponent(ns) - 1) set *range_flag (if non-null)
__host__ __device__ constexpr int bf16_min_row_exponent(int ns) { return 8 - (126 - 9 * (ns - 1)) / 2; }
hipError_t launch_split_rows_bf16(const double* X, long long ldx, int nb, int rows, int rows_pad, int ncols,
                                  int ncols_pad, int ns, __bf16* out, double* norm2, int* range_flag,
                                  hipStream_t st);
hipError_t launch_split_rows_fp8(const double* X, long long ldx, int nb, int rows, int rows_pad, int ncols,
                                 int ncols_pad, int ns, uint8_t* out, uint32_t* scales, double* norm2,
                                 hipStream_t st);
hipError_t launch_split_rows_i8(const double* X, long long ldx, int nb, int rows, int rows_pad, int ncols,
                                int ncols_pad, int ns, int8_t* out, int* rexp, double* norm2, hipStream_t st);

// ------------------------------------------------------------- density kernel
struct DensityKernelArgs {
  const double* T;      // [n_pairs][n_v][n_v] full amplitude matrices of unordered pairs
  const double* pw;     // [n_pairs] per-pair weight, or null (then w for every pair)
  const int2* pairs;    // [n_pairs]
  const int* slot;      // [n_pairs] matrix index of pair p in T, or null (p)
  double* Dpart;        // [nsplit][n_v][n_v]
  int n_v, nt, nTP, n_pairs, nsplit;
  double w;             // weight of one ordered pair (closed shell, spin-summed: 2)
  int accumulate;       // add into Dpart instead of overwriting
};
hipError_t launch_density_f64(const DensityKernelArgs& a, hipStream_t st);

// split-BF16 density: amplitude slices (split_t.hip) and the sliced product
struct DensitySlicedArgs {
  const __bf16* Ts;     // [n_pairs][4][rows_pad][n_v_pad/16][ns][16] (split_t.hip)
  const double* pw;     // [n_pairs] per-pair weight, or null
  const int2* pairs;    // [n_pairs]
  double* Dpart;        // [nsplit][n_v][n_v]
  int n_v, n_v_pad, nt, nTP, n_pairs, nsplit;  // nTP = density_bf16_tiles(nt)
  int rows_pad;         // rows per operand matrix: a multiple of 128, >= 128 ceil(nt / 2)
  double w;             // weight of one ordered pair
  int accumulate;
};
// workgroup tiles (128 x 64, on or above the diagonal) of the split-BF16 density kernel
int density_bf16_tiles(int nt);
// slices of the four density operands of every pair of a batch (T: [n_pairs][n_v][n_v]),
// one exponent per (row, 64-column block) taken from the block itself, plus the
// exact FP64 diagonal partials dgp ([n_pairs][n_v_pad/64][n_v_pad]) and diag[a] +=
// their weighted sum; the operand matrices are rows_pad rows apart (a multiple of
// 64, >= n_v_pad); rows n_v .. n_v_pad - 1 are written as zeros, rows
// n_v_pad .. rows_pad - 1 are not written (slot: matrix q is T + slot[q] n_v^2, or
// T + q n_v^2 when slot is null)
hipError_t launch_split_t_bf16(const double* T, const int* slot, const int2* pairs, const double* pw, double w,
                               int n_pairs, int n_v, int n_v_pad, int rows_pad, int ns, double* dgp, __bf16* out,
                               double* diag, hipStream_t st);
// diag[a] += sum over the pairs q and 64-column blocks of w_q dgp[q][blk][a]
// (w_q = w pw[q], halved for i == j), in a fixed order
hipError_t launch_diag_accumulate(const double* dgp, const int2* pairs, const double* pw, double w, int n_pairs,
                                  int n_v, int n_v_pad, double* diag, hipStream_t st);
// row maxima of the four density operands (tmax, atomic max: zero it first) and the
// diagonal partials (dgp) of amplitude matrices T + slot[q] n_v^2 that did not come
// out of a pair-kernel epilogue, for the INT8-digit split
hipError_t launch_pair_row_stats(const double* T, const int* slot, int n_pairs, int n_v, int n_v_pad,
                                 unsigned long long* tmax, double* dgp, hipStream_t st);
hipError_t launch_density_bf16(const DensitySlicedArgs& a, int ns, hipStream_t st);

// INT8-digit density: digits of the four operands (split_t.hip) and the digit product
struct DensityDigitArgs {
  const int8_t* Ts;     // [n_pairs][4][n_v_pad/32][n_v_pad][ns][32] (split_t.hip)
  const int* rexp;      // [n_pairs][4][n_v_pad] row exponents
  const double* pw;     // [n_pairs] per-pair weight, or null
  const int2* pairs;    // [n_pairs]
  double* Dpart;        // [nsplit][n_v][n_v]
  int n_v, n_v_pad, nt, nTP, n_pairs, nsplit;
  double w;             // weight of one ordered pair
  int accumulate;
};
hipError_t launch_split_t_i8(const double* T, const int* slot, const int2* pairs, const double* pw, double w,
                             int n_pairs, int n_v, int n_v_pad, int ns, const unsigned long long* tmax,
                             const double* dgp, int8_t* out, int* rexp, double* diag, hipStream_t st);
hipError_t launch_density_i8(const DensityDigitArgs& a, int ns, hipStream_t st);
// D = sum of the split slices (+ diag on the diagonal if non-null), both triangles
hipError_t launch_density_reduce(const double* Dpart, int nsplit, int n_v, const double* diag, double* D,
                                 hipStream_t st);

// ------------------------------------------------------------ small kernels
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);
hipError_t launch_build_pairs(const uint8_t* mask, int n_core, int n_h, int2* pairs, int* count,
                              hipStream_t st);
// per-pair reduction of tile partials into double-double pair energies and ||T||^2
hipError_t launch_pair_reduce(const double* epart, const double* tpart, int nTP, int n_pairs,
                              double* pe /*[n][2]*/, double* tn2 /*[n]*/, hipStream_t st);
// sum of pair energies (double-double) -> e[2]; optional scatter to n_h x n_h outputs
hipError_t launch_energy_finalize(const double* pe, const double* tn2, const int2* pairs,
                                  const int* count, int max_pairs, int n_h, double* e_out,
                                  double* pair_energy, float* pair_tnorm, hipStream_t st);

// ------------------------------------------------------------ active holes
hipError_t launch_kron_uu(const double* U, int na, double* W, hipStream_t st);
// out[b][k][e] = sum_u U[u][k] in[b][u][e] for e < n, k, u < na, b < batch
// (stacks of na matrices of n elements; na <= 32)
hipError_t launch_rotate_stack(const double* U, int na, const double* in, double* out, long long n, int batch,
                               hipStream_t st);
hipError_t launch_build_active_pairs(int kind, int m0, int ncore, int n_core, int na, int2* pairs, int* slots,
                                     hipStream_t st);
hipError_t launch_active_weights(int kind, int n, int n_core, int na, const int2* pairs, const double* occ,
                                 double scale_d, double* wd, double* we, hipStream_t st);
hipError_t launch_rotated_energy(const double* T, const double* Vr, const int* slot, int n_pairs, int n_v,
                                 double* part, hipStream_t st);
hipError_t launch_weighted_pair_reduce(const double* part, int ntile, int n_pairs, const double* we, double* pe,
                                       hipStream_t st);
hipError_t launch_energy_finalize_active(const double* pe, const int* count, const double* pe_act, int n_act_pairs,
                                         double* e_out, hipStream_t st);
hipError_t launch_scatter_active_pair_info(const int2* pairs, const double* tn2, int n, int n_h, double* pair_energy,
                                           float* pair_tnorm, hipStream_t st);

}  // namespace dfpt2
