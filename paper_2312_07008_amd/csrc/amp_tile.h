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
template <int CTRL>
__device__ inline u4 quad_xor_u4(u4 v) {  // CTRL 0xB1: partner k ^ 1, 0x4E: partner k ^ 2
  u4 r;
  r.x = (uint32_t)__builtin_amdgcn_mov_dpp((int)v.x, CTRL, 0xf, 0xf, false);
  r.y = (uint32_t)__builtin_amdgcn_mov_dpp((int)v.y, CTRL, 0xf, 0xf, false);
  r.z = (uint32_t)__builtin_amdgcn_mov_dpp((int)v.z, CTRL, 0xf, 0xf, false);
  r.w = (uint32_t)__builtin_amdgcn_mov_dpp((int)v.w, CTRL, 0xf, 0xf, false);
  return r;
}
// one butterfly round of a quad transpose between items a and b (b = a + k of the
// partner k4 ^ k): the lane with bit k of k4 set sends a and takes the partner's b
// into a, the other sends b and takes the partner's a into b
template <int CTRL>
__device__ inline void quad_swap(u4& a, u4& b, bool hi) {
  const u4 rcv = quad_xor_u4<CTRL>(hi ? a : b);
  if (hi) a = rcv;
  else b = rcv;
}
// 4 x 4 transpose over the quad: item t of lane k becomes item k of lane t
__device__ inline void quad_transpose(u4& m0, u4& m1, u4& m2, u4& m3, int k4) {
  const bool h1 = (k4 & 1) != 0, h2 = (k4 & 2) != 0;
  quad_swap<0xB1>(m0, m1, h1);
  quad_swap<0xB1>(m2, m3, h1);
  quad_swap<0x4E>(m0, m2, h2);
  quad_swap<0x4E>(m1, m3, h2);
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
// exact.  dst[m] points at the thread's 16-column chunk of row a of matrix m:
// [ns][16] bf16, 32 ns contiguous bytes, the quad's four chunks contiguous.  For
// even ns the quad exchanges its 16-byte pieces first (quad_transpose), so that
// in each store the four lanes write 64 contiguous bytes instead of 16 bytes in
// each of four 128-byte lines (the density pass's epilogue: 8.8 -> 7.2 ms per
// 512-pair launch at 1200 virtuals).
// Returns the row's diagonal partial sum_c 2 (x^2 - x y + y^2) over the block
// (quad sum).  All four lanes of every quad must call this, with no lane
// inactive.
template <int NS>
__device__ inline double split_block_row(const double* x, const double* y, __bf16* const* dst) {
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
    bf8v sl[NS][2];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      double u = ldexp(v[j], 8 - E);
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const double d = rint(u);
        sl[t][j >> 3][j & 7] = (__bf16)ldexpf((float)d, E - 8 - 9 * t);
        if (t + 1 < NS) u = (u - d) * 512.0;
      }
    }
    u4* o = reinterpret_cast<u4*>(dst[m]);
    if constexpr (NS % 2 == 0) {
      // piece q = 2t + h of lane c sits at u4 2 NS c + q of the quad's region; store i
      // of lane k4 writes u4 4 i + k4, i.e. piece 4 (i % G) + k4 of lane i / G (G = NS / 2)
      constexpr int G = NS / 2;
      const int k4 = threadIdx.x & 3;
      u4* oq = o - 2 * NS * k4;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        u4 p0 = __builtin_bit_cast(u4, sl[2 * g][0]), p1 = __builtin_bit_cast(u4, sl[2 * g][1]);
        u4 p2 = __builtin_bit_cast(u4, sl[2 * g + 1][0]), p3 = __builtin_bit_cast(u4, sl[2 * g + 1][1]);
        quad_transpose(p0, p1, p2, p3, k4);  // p_c = piece 4 g + k4 of lane c
        oq[4 * g + k4] = p0;
        oq[4 * (G + g) + k4] = p1;
        oq[4 * (2 * G + g) + k4] = p2;
        oq[4 * (3 * G + g) + k4] = p3;
      }
    } else {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        o[2 * t] = __builtin_bit_cast(u4, sl[t][0]);
        o[2 * t + 1] = __builtin_bit_cast(u4, sl[t][1]);
      }
    }
  }
  return quad_sum(dg);
}

}  // namespace amp
}  // namespace dfpt2
