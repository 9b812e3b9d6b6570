// Tile helpers for the amplitude operands of the split-BF16 density product,
// shared by the stand-alone amplitude split (split_t.hip) and the epilogue that
// splits the amplitudes as it forms them (epi_split_bf16.hip).
//
// Thread layout of a 64 x 64 tile: thread t owns row t / 4 and the 16 consecutive
// columns 16 (t % 4) .. + 15, so the four threads of a row form a DPP quad and
// one thread's columns are exactly one 16-wide chunk of the density operands.
#pragma once
#include "common.h"

namespace dfpt2 {
namespace amp {

constexpr int TB = 64;      // tile edge
constexpr int LD = TB + 1;  // LDS row stride (doubles) of a staged tile
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// value of the lane k ^ 1 (CTRL = 0xB1, quad_perm [1,0,3,2]) or k ^ 2 (0x4E,
// [2,3,0,1]) of the lane's quad, by DPP moves of the two halves
template <int CTRL>
__device__ inline double quad_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// maximum / sum over the quad, the same pattern in every lane (reproducible)
__device__ inline double quad_max(double v) {
  v = fmax(v, quad_xor<0xB1>(v));
  return fmax(v, quad_xor<0x4E>(v));
}
__device__ inline double quad_sum(double v) {
  v += quad_xor<0xB1>(v);
  return v + quad_xor<0x4E>(v);
}

// Tile (row block A, column block C) of the n_v x n_v matrix M: the mirror tile
// tm[r][c] = M[C*64 + r][A*64 + c] (whole-row loads; skipped when !mirror) and,
// for thread (row r = tid / 4, quarter k4 = tid % 4), x[j] = M[A*64 + r][C*64 +
// 16 k4 + j]; zeros outside n_v.  VEC (n_v even): rows start 16-byte aligned and
// columns come in pairs below n_v, so both are read with 16-byte loads (these
// kernels are bound by the vector-load data path).  Ends with a barrier.
template <bool VEC>
__device__ inline void load_tile(const double* M, int n_v, int A, int C, double (*tm)[LD], double* x, bool mirror) {
  const int tid = threadIdx.x;
  if (mirror) {
    if (VEC) {
      for (int e = tid; e < TB * TB / 2; e += 256) {
        const int r = e >> 5, c = 2 * (e & 31);
        const int hr = C * TB + r, hc = A * TB + c;
        const double2 v = (hr < n_v && hc < n_v) ? *reinterpret_cast<const double2*>(M + (size_t)hr * n_v + hc)
                                                 : make_double2(0.0, 0.0);
        tm[r][c] = v.x;
        tm[r][c + 1] = v.y;
      }
    } else {
      for (int e = tid; e < TB * TB; e += 256) {
        const int r = e >> 6, c = e & 63;
        const int hr = C * TB + r, hc = A * TB + c;
        tm[r][c] = (hr < n_v && hc < n_v) ? M[(size_t)hr * n_v + hc] : 0.0;
      }
    }
  }
  const int row = A * TB + (tid >> 2), k4 = tid & 3;
  if (VEC) {
    // lane k4 of the row's quad reads 16-byte piece 4 j + k4 of the row's 64
    // columns, so the quad reads 64 contiguous bytes per load; the quad then
    // transposes the pieces (exchange rounds with partners k4 ^ 1 and k4 ^ 2) so
    // that lane k4 holds pieces 8 k4 .. 8 k4 + 7, i.e. columns 16 k4 .. + 15
    const double* src = M + (size_t)row * n_v + C * TB;
    double2 pc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c0 = 2 * (4 * j + k4);
      pc[j] = (row < n_v && C * TB + c0 < n_v) ? *reinterpret_cast<const double2*>(src + c0) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double2 m[4] = {pc[h], pc[2 + h], pc[4 + h], pc[6 + h]};  // lane k4: pieces 8 t + 4 h + k4
#pragma unroll
      for (int k = 1; k <= 2; k <<= 1) {
        const bool hi = (k4 & k) != 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (t & k) continue;
          const double2 snd = hi ? m[t] : m[t | k];
          double2 rcv;
          rcv.x = k == 1 ? quad_xor<0xB1>(snd.x) : quad_xor<0x4E>(snd.x);
          rcv.y = k == 1 ? quad_xor<0xB1>(snd.y) : quad_xor<0x4E>(snd.y);
          if (hi) m[t] = rcv;
          else m[t | k] = rcv;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {  // now piece 8 k4 + 4 h + t
        x[2 * (4 * h + t)] = m[t].x;
        x[2 * (4 * h + t) + 1] = m[t].y;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int gc = C * TB + k4 * 16 + j;
      x[j] = (row < n_v && gc < n_v) ? M[(size_t)row * n_v + gc] : 0.0;
    }
  }
  __syncthreads();
}

// The four density operands of one unordered pair, for a row a and the 16
// columns c of one thread (x[j] = T[a][c], y[j] = T[c][a]):
//   m = 0: T[a][c]   m = 1: T[c][a]   m = 2: 2 T[a][c] - T[c][a]   m = 3: 2 T[c][a] - T[a][c]
// Each matrix's row is split per 64-column block: 2^E from the largest magnitude
// of the row within the block (over the thread's quad), then ns true-scale BF16
// slices s_t 2^(E - 8 - 9t) by successive rounding to the nearest integer:
// u_0 = v 2^(8 - E) (|u_0| < 256), s_t = rint(u_t), u_{t+1} = 512 (u_t - s_t), every
// step exact in FP64, so |s_t| <= 256 (exact in BF16) and
// sum_t s_t 512^(ns-1-t) = rint(v 2^(8 + 9(ns-1) - E)).
// Within a block every product of a row of X and a row of Y is an integer
// multiple of one unit, so the density kernel's FP32 level sums over a block are
// exact.
//
// The workgroup (256 threads, thread t on row t / 4 of the 64-row tile, columns
// 16 (t % 4) .. + 15 of the 64-column block) writes the block of the four
// matrices: base is row 0 of the tile at the block's first column in matrix 0,
// matrix m at base + m mat_elems, rows row_elems apart; a row of the block is
// [4 chunks][ns][16] bf16, 128 ns contiguous bytes.  Each matrix's slices go
// through the LDS buffer stg (at least 64 x 8 ns 16-byte pieces, the caller's
// tile, free on entry up to the first barrier) so that every store of a wave
// covers whole rows of the block: two 512-byte runs at ns = 4 instead of
// sixteen lanes' 16-byte pieces in as many rows (the density pass's epilogue,
// 512-pair launches at 1200 virtuals: 8.8 ms with per-thread stores, 7.2 with
// the pieces exchanged within each row's four threads, 6.4 staged this way).  In LDS the piece p of
// row r sits at slot (p + r) mod 8 ns, so that the writes and the reads of a
// wave spread over all banks.  Returns the row's diagonal partial
// sum_c 2 (x^2 - x y + y^2) over the block (quad sum).  Every thread of the
// workgroup must call this: it holds barriers.
template <int NS>
__device__ inline double split_block_rows(const double* x, const double* y, u4* stg, __bf16* base,
                                          size_t mat_elems, size_t row_elems) {
  constexpr int SL = 8 * NS;  // 16-byte pieces per row of the block
  const int tid = threadIdx.x, r = tid >> 2, k4 = tid & 3;
  double dg = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) dg += 2.0 * (x[j] * x[j] - x[j] * y[j] + y[j] * y[j]);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double v[16];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      v[j] = m == 0 ? x[j] : m == 1 ? y[j] : m == 2 ? 2.0 * x[j] - y[j] : 2.0 * y[j] - x[j];
      mx = fmax(mx, fabs(v[j]));
    }
    mx = quad_max(mx);
    int E = 0;
    if (mx > 0.0) frexp(mx, &E);  // mx < 2^E
    __syncthreads();  // every earlier read of stg is done
    // columns 8 h .. 8 h + 7 form piece (t, h) of every slice t: staged half a chunk
    // at a time, so that only NS pieces are held
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf8v sl[NS];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int j = 8 * h + jj;
        double u = ldexp(v[j], 8 - E);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const double d = rint(u);
          sl[t][jj] = (__bf16)ldexpf((float)d, E - 8 - 9 * t);
          if (t + 1 < NS) u = (u - d) * 512.0;
        }
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) stg[r * SL + (k4 * 2 * NS + 2 * t + h + r) % SL] = __builtin_bit_cast(u4, sl[t]);
    }
    __syncthreads();
    char* mb = reinterpret_cast<char*>(base + m * mat_elems);
#pragma unroll
    for (int i = 0; i < SL / 4; ++i) {  // 64 SL pieces over 256 threads
      const int P = i * 256 + tid, row = P / SL, sp = P - row * SL;
      *reinterpret_cast<u4*>(mb + (size_t)row * row_elems * 2 + sp * 16) = stg[row * SL + (sp + row) % SL];
    }
  }
  return quad_sum(dg);
}

}  // namespace amp
}  // namespace dfpt2
