// Epilogue shared by the sliced pair kernels (the epilogue kernel of
// pair_bf16_v.hip after the BF16 or INT8 product, the fused INT8 kernel of
// pair_i8.hip): once a workgroup holds P = V^{ij}[I,J] and Q = V^{ji}[I,J] of its
// tile pair in FP64, the DSRG regularizer, amplitudes and energy partials follow
// the paper's App. A (Eq. A7), exactly as in the FP64 pair kernel, plus the row
// data of the INT8-digit density.
//
// Register layout (any 32x32 MFMA accumulator): register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4 and column l % 32 of the wave's 32 x 32 block;
// wave w = 2 wr + wc owns rows wr*32.. of tile I and columns wc*32.. of tile J.
#pragma once
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

// Row information the INT8-digit density needs, from the amplitudes of one tile
// pair (x = T[a][b] for a in I, b in J, y = T[b][a]; split_t.hip):
//   the largest magnitudes of the rows of T, T^T, 2T - T^T and 2T^T - T
//   (quantities |x|, |y|, |2x - y|, |2y - x| over b for rows a of I; with the
//   roles of x and y swapped over a for rows b of J when I < J), merged with an
//   atomic max of the bit patterns of non-negative doubles (order independent);
//   and the partial sums 2 (x^2 - x y + y^2) of the exact diagonal of the pair's
//   density contribution, one slot per (row, other tile) in dgp.
// Row values are reduced over the 32 lanes of a half-wave (recursive halving,
// 16 exchanges for 16 registers), column values over the 16 registers and the
// two halves; the two waves sharing rows (columns) are combined through LDS.
// Called by all threads of the workgroup.
__device__ inline void density_row_info(const PairSlicedArgs& a, int p, int I, int J, const double* tpv,
                                        const double* tqv, double* xs) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1, r32 = lane & 31, hq = lane >> 5;
  double* xl = xs;        // [4 waves][32 rows] row partials
  double* xc = xs + 128;  // [4 waves][32 columns] column partials
  for (int m = 0; m < 5; ++m) {
    double v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const double x = tpv[r], y = tqv[r];
      v[r] = m == 0 ? fabs(x) : m == 1 ? fabs(y) : m == 2 ? fabs(2.0 * x - y) : m == 3 ? fabs(2.0 * y - x)
                                                                               : 2.0 * (x * x - x * y + y * y);
    }
    // column value: over the 16 registers, then the two halves
    double cv = v[0];
#pragma unroll
    for (int r = 1; r < 16; ++r) cv = m < 4 ? fmax(cv, v[r]) : cv + v[r];
    {
      const double o = __shfl_xor(cv, 32, 64);
      cv = m < 4 ? fmax(cv, o) : cv + o;
    }
    // row values: over the 32 lanes of the half, by recursive halving: at each
    // level a lane keeps half of its registers and adds its partner's copy of
    // them, so after offsets 16, 8, 4, 2 (and a final 1) lane l holds the full
    // sum (or maximum) of register (l >> 1) & 15
#pragma unroll
    for (int o = 16, n = 16; o >= 2; o >>= 1, n >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < n / 2; ++i) {
        const double mine = up ? v[n / 2 + i] : v[i];
        const double give = up ? v[i] : v[n / 2 + i];
        const double got = __shfl_xor(give, o, 64);
        v[i] = m < 4 ? fmax(mine, got) : mine + got;
      }
    }
    double rv = v[0];
    {
      const double o = __shfl_xor(rv, 1, 64);
      rv = m < 4 ? fmax(rv, o) : rv + o;
    }
    __syncthreads();
    if ((r32 & 1) == 0) xl[w * 32 + hq * 16 + (r32 >> 1)] = rv;
    if (hq == 0) xc[w * 32 + r32] = cv;
    __syncthreads();
    if (tid < 64) {  // rows of I: waves (wr, 0) and (wr, 1)
      const int rw = tid >> 5, k = tid & 31, h = k >> 4, r = k & 15;
      const double u0 = xl[(rw * 2 + 0) * 32 + k], u1 = xl[(rw * 2 + 1) * 32 + k];
      const double val = m < 4 ? fmax(u0, u1) : u0 + u1;
      const int row = I * 64 + rw * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      if (row < a.n_v) {
        if (m < 4)
          atomicMax(a.tmax + ((size_t)p * 4 + m) * a.n_v_pad_d + row, (unsigned long long)__double_as_longlong(val));
        else
          a.dgp[((size_t)p * a.nt + J) * a.n_v_pad_d + row] = val;
      }
    } else if (tid < 128 && I < J) {  // rows of J: waves (0, wc) and (1, wc), roles of x and y swapped
      const int cw = (tid - 64) >> 5, c = tid & 31;
      const double u0 = xc[(0 * 2 + cw) * 32 + c], u1 = xc[(1 * 2 + cw) * 32 + c];
      const double val = m < 4 ? fmax(u0, u1) : u0 + u1;
      const int row = J * 64 + cw * 32 + c;
      if (row < a.n_v) {
        if (m < 4) {
          const int mm = m ^ 1;  // |x| <-> |y|, |2x - y| <-> |2y - x|
          atomicMax(a.tmax + ((size_t)p * 4 + mm) * a.n_v_pad_d + row, (unsigned long long)__double_as_longlong(val));
        } else {
          a.dgp[((size_t)p * a.nt + I) * a.n_v_pad_d + row] = val;
        }
      }
    }
  }
  __syncthreads();
}

// dP / dQ: the wave's values of P and Q (dQ == dP when i == j); for i == j the
// diagonal V^{ii}_{aa} is replaced by the exact FP64 norm.  scratch: at least
// 264 doubles of LDS the main loop no longer reads (all threads call this after
// a barrier that retired the last LDS reads).
template <bool STORE>
__device__ inline void sliced_pair_epilogue(const PairSlicedArgs& a, int p, int tp, int I, int J, int hi_i, int hi_j,
                                            const double* dP, const double* dQ, double* scratch) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1, r32 = lane & 31, hq = lane >> 5;
  const bool same = (hi_i == hi_j);
  const int n_v = a.n_v;
  double* red = scratch + 256;
  const double eij = a.eps_h[hi_i] + a.eps_h[hi_j];
  const double s = a.s;
  const bool offdiag = (I < J);
  const double blk_w = (offdiag ? 2.0 : 1.0) * (same ? 0.5 : 1.0) * a.e_weight;
  double* Tp = (STORE && a.T) ? a.T + (size_t)p * n_v * n_v : nullptr;
  double* Vp = (STORE && a.Vr) ? a.Vr + (size_t)p * n_v * n_v : nullptr;
  double esum = 0.0, tsum = 0.0;
  double tpv[16], tqv[16];  // amplitudes T[ga][gb], T[gb][ga] (0 outside n_v)
  const int gb = J * 64 + wc * 32 + r32;
  const bool vb = gb < n_v;
  const double eb = vb ? a.eps_v[gb] : 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ga = I * 64 + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
    tpv[r] = 0.0;
    tqv[r] = 0.0;
    if (!(vb && ga < n_v)) continue;
    const double dl = eij - a.eps_v[ga] - eb;
    const double x = exp(-s * dl * dl);
    const double g1 = (dl != 0.0) ? (1.0 - x) / dl : 0.0;
    double vp = dP[r], vq = dQ[r];
    if (same && ga == gb) vp = vq = a.norm2[(size_t)hi_i * n_v + ga];  // exact ||B_ia||^2
    const double tp_ = vp * g1, tq_ = vq * g1;
    tpv[r] = tp_;
    tqv[r] = tq_;
    esum += (1.0 + x) * g1 * (2.0 * vp * vp + 2.0 * vq * vq - 2.0 * vp * vq);
    tsum += tp_ * tp_ + (offdiag ? tq_ * tq_ : 0.0);
    if (STORE && Tp) {
      Tp[(size_t)ga * n_v + gb] = tp_;
      if (offdiag) Tp[(size_t)gb * n_v + ga] = tq_;
    }
    if (STORE && Vp) {
      Vp[(size_t)ga * n_v + gb] = vp * (1.0 + x);
      if (offdiag) Vp[(size_t)gb * n_v + ga] = vq * (1.0 + x);
    }
  }
  if (STORE && a.tmax) density_row_info(a, p, I, J, tpv, tqv, scratch);
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


}  // namespace dfpt2
