// Split-BF16 density kernel: the virtual block of the second-order 1-RDM
// (Eq. A9 with zero cumulants) accumulated over hole pairs from BF16 slices of
// the amplitudes, on the 32x32x16 BF16 MFMA.
//
// Per unordered pair the contribution is X1 Y1^T + X2 Y2^T (split_t.hip gives
// the slices of the rows of X1 = T, X2 = T^T, Y1 = 2T - T^T, Y2 = 2T^T - T).
// As in the pair kernel, the slice products of level s + t - 1 <= NS are kept.
// The operands carry one exponent per (row, 64-column block), so within one
// block of one product of one pair every product of a row a of X and a row b of
// Y is an integer multiple of one unit (the two rows' block scales): the level-1
// and level-2 sums are exact in FP32 over the block's 64 contraction steps and
// are added into FP64 at the end of every block (with the pair's weight);
// levels >= 3 are summed in FP32 per product.  The two products carry different
// units, so the contraction runs over X1 / Y1 first and X2 / Y2 after it, with
// one set of accumulators.  D is symmetric: only
// tiles on or above the diagonal are formed.  Diagonal elements are left out:
// split_t.hip sums them exactly in FP64 (the rows of X and Y there carry the
// same amplitudes, so the dropped slice products would not average out).
//
// Workgroup = (128 x 64 tile (I, J) of D with J >= 2I in 64-wide units, split s):
// split s owns a contiguous range of pairs and accumulates into its own slice
// Dpart[s]; the slices are summed in a fixed order afterwards
// (density_reduce_kernel), so results are bitwise reproducible.  A 128 x 64
// tile moves 192 rows per contraction chunk for 8192 outputs (a 64 x 64 tile
// pair of both products at once: 256 rows for 8192), 25% fewer bytes per flop.
// Four waves, wave (wr, wc) owns rows 64 wr .. + 63 (two 32 x 32 MFMA blocks)
// and columns 32 wc .. + 31; on a diagonal tile (J = 2I) rows 64 .. 127 lie
// below the diagonal and their two waves only help with the loads.  Rows of X
// beyond n_v_pad (the last row tile when n_v_pad / 64 is odd) are loaded only
// there: the operand matrices are rows_pad rows apart, and those rows are never
// written or used.  Staging as in pair_bf16_v.hip: 16-wide chunks of the 128-row
// X panel and the 64-row Y panel go from global memory straight into LDS
// (XOR-swizzled 128-byte rows), double buffered, 24 KB per buffer, two
// workgroups per CU; each step issues the next chunk's loads before its fragment
// reads and waits for them before its closing barrier.  The 1-D launch is
// remapped so that every XCD walks a contiguous range of (split, tile):
// workgroups resident on one XCD read the same pairs' slices.
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TX = 128;  // rows of D per tile (X panel)
constexpr int TY = 64;   // columns of D per tile (Y panel)
constexpr int KC = 16;
constexpr int SLOTS = 8;
constexpr int KB_X = TX / 8, KB_Y = TY / 8;  // kilobytes of the two panels per chunk
constexpr int KB_W = (KB_X + KB_Y) / 4;      // kilobytes per wave per chunk
constexpr int PY = KB_X * 64;                // u4 offset of the Y panel in a buffer
constexpr int FLUSH_CHUNKS = 64 / KC;  // one exponent block of the operands
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int swz8(int r) { return (r ^ (r >> 3)) & 7; }

__device__ inline int xcd_block_d(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

// tile td of the row-major list of (I, J), J = 2I .. nt - 1
__device__ inline void density_tile(int td, int nt, int& I, int& J) {
  int i = 0, rem = td;
  while (rem >= nt - 2 * i) {
    rem -= nt - 2 * i;
    ++i;
  }
  I = i;
  J = 2 * i + rem;
}
}  // namespace

template <int NS>
__global__ __launch_bounds__(256, 2) void density_bf16_kernel(DensitySlicedArgs a) {
  static_assert(2 * NS <= SLOTS, "slices per LDS row");
  static_assert(KB_W * 4 == KB_X + KB_Y, "whole kilobytes per wave");
  __shared__ u4 lds0[(KB_X + KB_Y) * 64];
  __shared__ u4 lds1[(KB_X + KB_Y) * 64];
  const int L = xcd_block_d(blockIdx.x, a.nTP * a.nsplit);
  const int split = L / a.nTP, td = L - split * a.nTP;
  int I, J;
  density_tile(td, a.nt, I, J);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const bool below = (J == 2 * I) && wr == 1;  // wave-uniform
  const int n_v = a.n_v;
  const int p0 = (int)((long long)split * a.n_pairs / a.nsplit);  // balanced pair ranges
  const int p1 = (int)((long long)(split + 1) * a.n_pairs / a.nsplit);
  const int ncc = a.n_v_pad / KC;  // chunks per product
  const int per_pair = 2 * ncc;
  const int total = (p1 > p0) ? (p1 - p0) * per_pair : 0;

  // kilobyte kb < KB_X of a chunk is rows 8 kb .. + 7 of the X panel (rows of
  // tile I), kilobyte KB_X + kb rows 8 kb .. + 7 of the Y panel (rows of tile J);
  // wave w moves kilobytes KB_W w .. + KB_W - 1; lane l fills physical slot l % 8
  // of row l / 8
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int row_bytes = a.n_v_pad * NS * 2;
  const size_t mat_bytes = (size_t)a.rows_pad * row_bytes;
  const char* Ts = reinterpret_cast<const char*>(a.Ts);
  const int l3 = lane >> 3, l7 = lane & 7;
  auto src_off = [&](int kb) -> uint32_t {  // kb within its panel
    const int row = 8 * kb + l3;
    const int sl = l7 ^ swz8(row);
    const int t = sl >> 1, h = sl & 1;
    return (uint32_t)(row * row_bytes + (t < NS ? t * 32 + h * 16 : 0));
  };
  // step idx: pair p0 + idx / per_pair, product h (0: X1 Y1^T, 1: X2 Y2^T), chunk ch
  auto load_chunk = [&](int idx, u4* buf) {
    const int pi = idx / per_pair, rem = idx - pi * per_pair;
    const int h = rem >= ncc ? 1 : 0, ch = rem - h * ncc;
    const char* pb = Ts + (size_t)(p0 + pi) * 4 * mat_bytes + (size_t)ch * (KC * NS * 2);
    const char* pX = pb + (size_t)h * mat_bytes + (size_t)I * TX * row_bytes;
    const char* pY = pb + (size_t)(2 + h) * mat_bytes + (size_t)J * TY * row_bytes;
#pragma unroll
    for (int m = 0; m < KB_W; ++m) {
      const int kb = KB_W * q_w + m;  // wave-uniform
      const char* src = kb < KB_X ? pX + src_off(kb) : pY + src_off(kb - KB_X);
      __builtin_amdgcn_global_load_lds((gbl_void*)src, (lds_void*)(buf + kb * 64), 16, 0, 0);
    }
  };

  f16v acc[2][3];
  double dD[2][16];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][l][r] = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) dD[b][r] = 0.0;
  }

  const int r32 = lane & 31, hq = lane >> 5;
  const int rowY = wc * 32 + r32, fY = swz8(rowY);
  auto compute = [&](const u4* buf) {
    if (below) return;
    bf8v fb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) fb[s] = __builtin_bit_cast(bf8v, buf[PY + rowY * SLOTS + ((2 * s + hq) ^ fY)]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int rowX = wr * 64 + b * 32 + r32, fX = swz8(rowX);
      bf8v fa[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) fa[s] = __builtin_bit_cast(bf8v, buf[rowX * SLOTS + ((2 * s + hq) ^ fX)]);
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int u = 0; u + s < NS; ++u) {
          const int lv = (s + u) < 2 ? (s + u) : 2;
          acc[b][lv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[u], acc[b][lv], 0, 0, 0);
        }
    }
  };
  // after chunk ch of the current product (weight wp)
  auto flush = [&](int ch, bool prod_end, double wp) {
    if ((ch + 1) % FLUSH_CHUNKS == 0 || prod_end) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          dD[b][r] += wp * ((double)acc[b][0][r] + (double)acc[b][1][r]);
          acc[b][0][r] = 0.f;
          acc[b][1][r] = 0.f;
        }
    }
    if (prod_end) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          dD[b][r] += wp * (double)acc[b][2][r];
          acc[b][2][r] = 0.f;
        }
    }
  };
  // pair weight: one ordered pair w, halved for i == j (both orders are the same)
  auto weight = [&](int p) {
    const int2 pr = a.pairs[p];
    double wp = a.w * (pr.x == pr.y ? 0.5 : 1.0);
    if (a.pw) wp *= a.pw[p];
    return wp;
  };
  int cp = p0, cch = 0, half = 0;  // pair, chunk and product of the step being computed
  double wp = (total > 0) ? weight(p0) : 0.0;
  // step idx: the loads of step idx + 1 go out first and overlap the products of
  // step idx; all have landed at the closing barrier (buffers swapped through
  // pointers, as in pair_bf16_v.hip)
  auto step = [&](int idx, u4* cur, u4* nxt) {
    if (idx + 1 < total) load_chunk(idx + 1, nxt);
    compute(cur);
    const bool prod_end = (cch + 1 == ncc);
    flush(cch, prod_end, wp);
    if (prod_end) {
      cch = 0;
      if (half) {
        half = 0;
        ++cp;
        if (cp < p1) wp = weight(cp);
      } else {
        half = 1;
      }
    } else {
      ++cch;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  if (total > 0) {
    load_chunk(0, lds0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    u4 *cur = lds0, *nxt = lds1;  // steps idx, idx + 1
    for (int idx = 0; idx < total; ++idx) {
      step(idx, cur, nxt);
      u4* t = cur;
      cur = nxt;
      nxt = t;
    }
  }

  // D tile (32x32 layout: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32)
  if (below) return;
  double* Dp = a.Dpart + (size_t)split * n_v * n_v;
  const int gb = J * TY + wc * 32 + r32;
  if (gb < n_v) {
    // all reads of the old tile first (rows beyond n_v read row n_v - 1 and are
    // not written back), so that they are in flight together
    if (a.accumulate) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int ga = I * TX + wr * 64 + b * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
          dD[b][r] += Dp[(size_t)min(ga, n_v - 1) * n_v + gb];
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ga = I * TX + wr * 64 + b * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
        // the diagonal comes from the exact FP64 sum of the amplitude split
        if (ga < n_v && ga != gb) Dp[(size_t)ga * n_v + gb] = dD[b][r];
      }
  }
}

int density_bf16_tiles(int nt) {
  int n = 0;
  for (int i = 0; 2 * i < nt; ++i) n += nt - 2 * i;
  return n;
}

hipError_t launch_density_bf16(const DensitySlicedArgs& a, int ns, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  // the X panels of the last row tile reach row 128 ceil(nt / 2) - 1
  if (a.n_v_pad != 64 * a.nt || a.rows_pad % TX != 0 || a.rows_pad < TX * ((a.nt + 1) / 2) ||
      a.nTP != density_bf16_tiles(a.nt) || (long long)a.nTP * a.nsplit > 0x7fffffffLL)
    return hipErrorInvalidValue;
  dim3 grid(a.nTP * a.nsplit), block(256);
  switch (ns) {
    case 2: hipLaunchKernelGGL(density_bf16_kernel<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(density_bf16_kernel<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(density_bf16_kernel<4>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dfpt2
