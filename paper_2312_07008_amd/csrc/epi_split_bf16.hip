// Epilogue of the split-BF16 density pass: the DSRG amplitudes of one pair
// (paper App. A, Eq. A7), its energy and norm partials, and the BF16 slices of
// the four density operands of the core-core term of Eq. A9, formed from the
// FP64 V^{ij} = B_i B_j^T that pair_v_bf16_kernel wrote, without storing the
// FP64 amplitudes.
//
// Workgroup = one 64 x 64 tile pair (I <= J) of one pair.  Thread (row r = t / 4,
// quarter k4 = t % 4) holds the 16 consecutive columns 16 k4 .. + 15 of row
// a = 64 I + r (amp_tile.h): P = V[a][b] for b in tile J straight from global
// memory, Q = V^{ji}_{ab} = V[b][a] from the mirror tile V[J, I] staged in LDS.
// With Delta = eps_i + eps_j - eps_a - eps_b (the same for (a, b) and (b, a)),
//   T[a][b] = P (1 - e^{-s Delta^2}) / Delta,   T[b][a] = Q (1 - e^{-s Delta^2}) / Delta,
// and the energy partial (1 + e^{-s Delta^2}) (1 - e^{-s Delta^2}) / Delta
// (2 P^2 + 2 Q^2 - 2 P Q) as in the other pair kernels (pair_epilogue.h).  For
// i == j, V^{ii} is symmetric and the product kernel leaves its tiles below the
// diagonal unwritten, so Q = P, and the diagonal V^{ii}_{aa} is the exact FP64
// norm ||B_ia||^2.
//
// The thread's values then give the slices of rows a (columns of J) of the four
// operands T, T^T, 2T - T^T, 2T^T - T with one exponent per (row, 64-column
// block) (amp::split_block_rows: the block is whole in the workgroup), and the
// diagonal partial of row a for block J.  For I < J the amplitudes go through
// LDS once more, so that every thread also holds 16 columns (of I) of a row of J
// and writes those slices and that partial: each amplitude is read once, as V,
// and its slices are written once.
#include "amp_tile.h"
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
using amp::LD;
using amp::TB;

// 1-D launch -> (pair, tile pair), every XCD taking a contiguous range (as the
// product kernel, so that the V it reads back was written through its own L2)
__device__ inline int xcd_block_e(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}
}  // namespace

template <int NS, bool VEC>
__global__ __launch_bounds__(256, 3) void pair_epi_split_bf16_kernel(PairSlicedArgs a, int rows_pad, __bf16* Ts,
                                                                     double* dgp) {
  // V[J, I] (the mirror), then in turn T[b][a] and T[a][b] at [a - 64 I][b - 64 J]:
  // one tile of LDS, so that three workgroups fit on a CU
  __shared__ __attribute__((aligned(16))) double sq[TB][LD];
  __shared__ double red[8];
  const int L = xcd_block_e(blockIdx.x, a.nTP * a.n_blk_pairs);
  const int p = L / a.nTP, tp = L - p * a.nTP;
  int I, J;
  tile_pair(tp, a.nt, I, J);
  const int2 pr = a.pairs[p];
  const bool same = pr.x == pr.y, offdiag = I < J;
  const int n_v = a.n_v, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = tid >> 2, k4 = tid & 3;
  const double* Vp = a.T + (size_t)p * n_v * n_v;

  double x[16], y[16];
  amp::load_tile<VEC>(Vp, n_v, I, J, sq, x, !same);
  const int ra = I * TB + r;  // row a
  const double eij = a.eps_h[pr.x] + a.eps_h[pr.y];
  const double ea = ra < n_v ? a.eps_v[ra] : 0.0;
  const double s = a.s;
  double esum = 0.0, tsum = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int cb = J * TB + 16 * k4 + j;  // column b
    double vp = x[j], vq = same ? x[j] : sq[16 * k4 + j][r];
    double tp_ = 0.0, tq_ = 0.0;
    if (ra < n_v && cb < n_v) {
      const double dl = eij - ea - a.eps_v[cb];
      const double ex = exp(-s * dl * dl);
      const double g1 = (dl != 0.0) ? (1.0 - ex) / dl : 0.0;
      if (same && ra == cb) vp = vq = a.norm2[(size_t)pr.x * n_v + ra];  // exact ||B_ia||^2
      tp_ = vp * g1;
      tq_ = vq * g1;
      esum += (1.0 + ex) * g1 * (2.0 * vp * vp + 2.0 * vq * vq - 2.0 * vp * vq);
      tsum += tp_ * tp_ + (offdiag ? tq_ * tq_ : 0.0);
    }
    x[j] = tp_;  // T[a][b]
    y[j] = tq_;  // T[b][a]
  }

  const int n_v_pad = a.n_v_pad_d;
  const size_t row_elems = (size_t)n_v_pad * NS, mat_elems = (size_t)rows_pad * row_elems;
  __bf16* Tq = Ts + (size_t)p * 4 * mat_elems;
  amp::u4* stg = reinterpret_cast<amp::u4*>(&sq[0][0]);  // 33 KB: the 32 KB of a block of slices fit
  {  // rows a of I, columns of J
    __bf16* base = Tq + (size_t)(I * TB) * row_elems + (size_t)(J * 4) * (NS * 16);
    const double dg = amp::split_block_rows<NS>(x, y, stg, base, mat_elems, row_elems);
    if (k4 == 0 && ra < n_v) dgp[((size_t)p * a.nt + J) * n_v_pad + ra] = dg;
  }
  if (offdiag) {  // workgroup-uniform
    // rows b = 64 J + r of J, columns a = 64 I + 16 k4 + j: T[b][a] and T[a][b],
    // transposed through the one LDS tile
    __syncthreads();  // every read of the staged slices in sq is done
#pragma unroll
    for (int j = 0; j < 16; ++j) sq[r][16 * k4 + j] = y[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = sq[16 * k4 + j][r];  // T[b][a]
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) sq[r][16 * k4 + j] = x[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = sq[16 * k4 + j][r];  // T[a][b]
    // the operands of row b: x = T[b][a], y = T[a][b]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double t = x[j];
      x[j] = y[j];
      y[j] = t;
    }
    const int rb = J * TB + r;
    __bf16* base = Tq + (size_t)(J * TB) * row_elems + (size_t)(I * 4) * (NS * 16);
    const double dg = amp::split_block_rows<NS>(x, y, stg, base, mat_elems, row_elems);
    if (k4 == 0 && rb < n_v) dgp[((size_t)p * a.nt + I) * n_v_pad + rb] = dg;
  }

  const double blk_w = (offdiag ? 2.0 : 1.0) * (same ? 0.5 : 1.0) * a.e_weight;
  esum = wave_sum(esum);
  tsum = wave_sum(tsum);
  if (lane == 0) {
    red[w] = esum;
    red[4 + w] = tsum;
  }
  __syncthreads();
  if (tid == 0) {
    const size_t o = (size_t)p * a.nTP + tp;
    if (a.epart) a.epart[o] = blk_w * ((red[0] + red[1]) + (red[2] + red[3]));
    if (a.tpart) a.tpart[o] = (red[4] + red[5]) + (red[6] + red[7]);
  }
}

hipError_t launch_pair_epi_split_bf16(const PairSlicedArgs& a, int n_pairs, int ns2, int rows_pad, __bf16* Ts,
                                      double* dgp, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (!a.T || !Ts || !dgp || a.n_v_pad_d != TB * a.nt || a.n_v_pad_d < a.n_v || rows_pad < a.n_v_pad_d ||
      a.nTP != a.nt * (a.nt + 1) / 2 || (long long)a.nTP * n_pairs > 0x7fffffffLL)
    return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  const dim3 grid(a.nTP * n_pairs), block(256);
  const bool vec = (a.n_v % 2) == 0;
#define EPI_SPLIT(NS_)                                                                                            \
  do {                                                                                                            \
    if (vec) hipLaunchKernelGGL((pair_epi_split_bf16_kernel<NS_, true>), grid, block, 0, st, b, rows_pad, Ts, dgp); \
    else hipLaunchKernelGGL((pair_epi_split_bf16_kernel<NS_, false>), grid, block, 0, st, b, rows_pad, Ts, dgp);    \
  } while (0)
  switch (ns2) {
    case 2: EPI_SPLIT(2); break;
    case 3: EPI_SPLIT(3); break;
    case 4: EPI_SPLIT(4); break;
    default: return hipErrorInvalidValue;
  }
#undef EPI_SPLIT
  return hipGetLastError();
}

}  // namespace dfpt2
