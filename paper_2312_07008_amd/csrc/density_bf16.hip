// Split-BF16 density kernel: the virtual block of the second-order 1-RDM
// (Eq. A9 with zero cumulants) accumulated over hole pairs from BF16 slices of
// the amplitudes, on the 32x32x16 BF16 MFMA.
//
// Per unordered pair the contribution is X1 Y1^T + X2 Y2^T (split_t.hip gives
// the slices of the rows of X1 = T, X2 = T^T, Y1 = 2T - T^T, Y2 = 2T^T - T).
// As in the pair kernel, the slice products of level s + t - 1 <= NS are kept;
// within one pair every product of a row a of X and a row b of Y is an integer
// multiple of one unit, so the level-1 and level-2 sums are exact in FP32 over
// 128 contraction steps and are added into FP64 every 128 steps and at the end
// of every pair (with the pair's weight); levels >= 3 are summed in FP32 per pair.
// D is symmetric: only tiles (A <= B) are formed.  Diagonal elements are left
// out: split_t.hip sums them exactly in FP64 (the rows of X and Y there carry the
// same amplitudes, so the dropped slice products would not average out).
//
// Workgroup = (tile pair (A, B), split s): split s owns a contiguous range of
// pairs and accumulates into its own slice Dpart[s]; the slices are summed in a
// fixed order afterwards (density_reduce_kernel), so results are bitwise
// reproducible.  Staging as in pair_bf16.hip: four 64-row panels per 16-wide
// chunk (X1[A], Y1[B], X2[A], Y2[B]) go from global memory straight into LDS,
// double buffered, in XOR-swizzled 128-byte rows; every wave owns one 32 x 32
// block of the tile and sums both products into it.  The 1-D launch is
// remapped so that every XCD walks a contiguous range of (split, tile pair):
// workgroups resident on one XCD read the same pairs' slices.
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 16;
constexpr int SLOTS = 8;
constexpr int PANEL_U4 = TM * SLOTS;
constexpr int FLUSH_CHUNKS = 128 / KC;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int swz8(int r) { return (r ^ (r >> 3)) & 7; }

__device__ inline int xcd_block_d(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}
}  // namespace

template <int NS>
__global__ __launch_bounds__(256, 2) void density_bf16_kernel(DensitySlicedArgs a) {
  static_assert(2 * NS <= SLOTS, "slices per LDS row");
  __shared__ u4 lds0[4 * PANEL_U4];
  __shared__ u4 lds1[4 * PANEL_U4];
  const int L = xcd_block_d(blockIdx.x, a.nTP * a.nsplit);
  const int split = L / a.nTP, tp = L - split * a.nTP;
  int A, Bt;
  tile_pair(tp, a.nt, A, Bt);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int n_v = a.n_v;
  const int p0 = (int)((long long)split * a.n_pairs / a.nsplit);  // balanced pair ranges
  const int p1 = (int)((long long)(split + 1) * a.n_pairs / a.nsplit);
  const int ncc = a.n_v_pad / KC;
  const int total = (p1 > p0) ? (p1 - p0) * ncc : 0;

  // direct loads: wave w fills panel w (X1 rows A, Y1 rows B, X2 rows A, Y2 rows B)
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int mat_w = (q_w == 0) ? 0 : (q_w == 1) ? 2 : (q_w == 2) ? 1 : 3;
  const int tile_w = (q_w == 0 || q_w == 2) ? A : Bt;
  const int row_bytes = a.n_v_pad * NS * 2;
  const size_t pair_bytes = (size_t)4 * a.n_v_pad * row_bytes;
  const char* panel0 = reinterpret_cast<const char*>(a.Ts) + ((size_t)mat_w * a.n_v_pad + tile_w * TM) * row_bytes;
  const int l3 = lane >> 3, l7 = lane & 7;
  auto src_off = [&](int m) -> uint32_t {
    const int sl = l7 ^ l3 ^ m;
    const int t = sl >> 1, h = sl & 1;
    return (uint32_t)((8 * m + l3) * row_bytes + (t < NS ? t * 32 + h * 16 : 0));
  };
  auto load_chunk = [&](int idx, u4* buf) {
    const int p = p0 + idx / ncc, ch = idx - (idx / ncc) * ncc;
    const char* base = panel0 + (size_t)p * pair_bytes + (size_t)ch * (KC * NS * 2);
#pragma unroll
    for (int m = 0; m < 8; ++m)
      __builtin_amdgcn_global_load_lds((gbl_void*)(base + src_off(m)), (lds_void*)(buf + q_w * PANEL_U4 + m * 64),
                                       16, 0, 0);
  };

  f16v accP[3], accQ[3];
  double dD[16];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accP[l][r] = 0.f;
      accQ[l][r] = 0.f;
    }
#pragma unroll
  for (int r = 0; r < 16; ++r) dD[r] = 0.0;

  const int r32 = lane & 31, hq = lane >> 5;
  const int rowA = wr * 32 + r32, rowB = wc * 32 + r32;
  const int fA = swz8(rowA), fB = swz8(rowB);

  auto compute = [&](const u4* buf) {
    bf8v fa[NS], fb[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      fa[t] = __builtin_bit_cast(bf8v, buf[0 * PANEL_U4 + rowA * SLOTS + ((2 * t + hq) ^ fA)]);
      fb[t] = __builtin_bit_cast(bf8v, buf[1 * PANEL_U4 + rowB * SLOTS + ((2 * t + hq) ^ fB)]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int t = 0; t + s < NS; ++t) {
        const int lv = (s + t) < 2 ? (s + t) : 2;
        accP[lv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[t], accP[lv], 0, 0, 0);
      }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      fa[t] = __builtin_bit_cast(bf8v, buf[2 * PANEL_U4 + rowA * SLOTS + ((2 * t + hq) ^ fA)]);
      fb[t] = __builtin_bit_cast(bf8v, buf[3 * PANEL_U4 + rowB * SLOTS + ((2 * t + hq) ^ fB)]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int t = 0; t + s < NS; ++t) {
        const int lv = (s + t) < 2 ? (s + t) : 2;
        accQ[lv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[t], accQ[lv], 0, 0, 0);
      }
  };
  // flush after chunk ch of the current pair (weight wp)
  auto flush = [&](int ch, double wp) {
    const bool pair_end = (ch + 1 == ncc);
    if ((ch + 1) % FLUSH_CHUNKS == 0 || pair_end) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        dD[r] += wp * (((double)accP[0][r] + (double)accP[1][r]) + ((double)accQ[0][r] + (double)accQ[1][r]));
        accP[0][r] = 0.f;
        accP[1][r] = 0.f;
        accQ[0][r] = 0.f;
        accQ[1][r] = 0.f;
      }
    }
    if (pair_end) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        dD[r] += wp * ((double)accP[2][r] + (double)accQ[2][r]);
        accP[2][r] = 0.f;
        accQ[2][r] = 0.f;
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
  int cp = p0, cch = 0;  // pair and chunk of the step being computed
  double wp = (total > 0) ? weight(p0) : 0.0;
  auto step = [&](int idx, u4* cur, u4* nxt) {
    if (idx + 1 < total) load_chunk(idx + 1, nxt);
    compute(cur);
    flush(cch, wp);
    if (++cch == ncc) {
      cch = 0;
      ++cp;
      if (cp < p1) wp = weight(cp);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  if (total > 0) {
    load_chunk(0, lds0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    int idx = 0;
    for (; idx + 1 < total; idx += 2) {
      step(idx, lds0, lds1);
      step(idx + 1, lds1, lds0);
    }
    if (idx < total) step(idx, lds0, lds1);
  }

  // epilogue (32x32 layout: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32)
  double* Dp = a.Dpart + (size_t)split * n_v * n_v;
  const int gb = Bt * TM + wc * 32 + r32;
  if (gb < n_v) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ga = A * TM + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
      if (ga >= n_v || ga == gb) continue;  // the diagonal comes from the exact FP64 sum (split_t.hip)
      double* dst = Dp + (size_t)ga * n_v + gb;
      *dst = a.accumulate ? *dst + dD[r] : dD[r];
    }
  }
}

hipError_t launch_density_bf16(const DensitySlicedArgs& a, int ns, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (a.n_v_pad % TM != 0 || (long long)a.nTP * a.nsplit > 0x7fffffffLL) return hipErrorInvalidValue;
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
