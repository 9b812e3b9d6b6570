// Split-BF16 pair kernel: V = B_i B_j^T from BF16 slices on the 32x32x16 BF16
// MFMA, with the same fused DSRG regularizer/energy epilogue as the FP64
// kernel (paper App. A, Eq. A7).  Launched for energy-only passes (the kept-space
// energy); passes that store the amplitudes run the product over larger tiles and
// the epilogue as a second kernel (pair_bf16_v.hip).
//
// Operands come from split.hip: each FP64 row of B is sum_t slice_t with
// slice_t an 8-bit integer times 2^(E - 8 - 9(t-1)).  The product of two rows
// is sum_{s,t} slice_s(a) . slice_t(b); terms with s + t - 1 = L form level L,
// of magnitude 2^-9(L-1) relative to level 1.  With NS slices the kernel keeps
// the levels L <= NS (NS (NS+1)/2 products; NS = 4 leaves a relative error near
// 2^-34 per element).
//
// Accumulation: level-1 and level-2 products are integer multiples of one unit
// per output element, at most 2^16 units each, so FP32 MFMA sums of 128
// contraction steps (one product per step at level 1, two at level 2) stay at or
// below 2^24 units and are exact.  These two accumulators are added into FP64
// every 128 steps.  Levels >= 3 carry 2^-18 of the value or less and are summed
// in FP32 over the whole contraction; their rounding stays far below the
// slicing error.
//
// For i == j the diagonal V^{ii}_{aa} = ||B_ia||^2 is taken from an FP64 norm
// computed while splitting: the dropped slice products (t, t) there are sums of
// squares, i.e. biased, and the diagonal carries a large share of E.
//
// Tiling as in pair_f64.hip: one workgroup = unordered pair {i <= j} x tile pair
// (I <= J) of 64 x 64; every wave owns the same 32 x 32 block of P = V^{ij}[I,J]
// and of Q = V^{ji}[I,J], so the exchange partner of P_ab is lane-local.
//
// Staging: panels go from global memory straight into LDS (global_load_lds,
// 16 bytes per lane, no register round trip), in 16-wide contraction chunks,
// double buffered.  One LDS row holds the chunk of one virtual: 8 slots of 16
// bytes (slice t, half h -> slot 2t + h; slots >= 2 NS are padding).  Slots are
// XOR-swizzled by f(r) = (r ^ (r >> 3)) & 7 so that the fragment reads (eight or
// sixteen consecutive rows, one logical slot) hit distinct banks, and each
// direct load fills one contiguous kilobyte (8 rows x 8 slots) with no conflict.
//
// Block order: the hardware deals consecutive workgroups round-robin to the 8
// XCDs, each with its own L2.  The launch is 1-D and the block index is remapped
// so that every XCD walks a contiguous range of (pair, tile pair) in order: the
// workgroups resident on one XCD then belong to one or two pairs and share the
// same slabs B_i, B_j through that XCD's L2.
#include "common.h"
#include "kernels.h"
#include "pair_epilogue.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 16;
constexpr int SLOTS = 8;               // 16-byte slots per LDS row
constexpr int PANEL_U4 = TM * SLOTS;   // u4 per panel
constexpr int FLUSH_CHUNKS = 128 / KC;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int swz(int r) { return (r ^ (r >> 3)) & 7; }

// XCD-aware block order: hardware block h runs on XCD h % 8; give XCD x the
// contiguous logical range [x q + min(x, rem), ...) of the nblk blocks.
__device__ inline int xcd_block(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}
}  // namespace

template <int NS, bool STORE>
__global__ __launch_bounds__(256, 2) void pair_gemm_bf16_kernel(PairSlicedArgs a) {
  static_assert(2 * NS <= SLOTS, "slices per LDS row");
  __shared__ u4 lds0[4 * PANEL_U4];
  __shared__ u4 lds1[4 * PANEL_U4];
  const int L = xcd_block(blockIdx.x, a.nTP * a.n_blk_pairs);
  const int p = L / a.nTP, tp = L - p * a.nTP;
  int I, J;
  tile_pair(tp, a.nt, I, J);
  const int2 pr = a.pairs[p];
  const int hi_i = pr.x, hi_j = pr.y;
  const bool same = (hi_i == hi_j);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int npanel = same ? 2 : 4;

  // Direct loads: wave w fills kilobytes kb = 8 w + m (m < 8) of the 32 per chunk;
  // kilobyte kb is panel kb / 8, rows 8 (kb % 8) .. + 7.  Lane l writes physical
  // slot l % 8 of row l / 8, i.e. logical slot (l % 8) ^ f(row).
  const int q_w = __builtin_amdgcn_readfirstlane(w);  // kilobytes 8 w .. 8 w + 7 are panel w
  const int hole_w = (q_w == 0 || q_w == 3) ? hi_i : hi_j;
  const int tile_w = (q_w == 0 || q_w == 2) ? I : J;
  const bool load_w = q_w < npanel;
  const int row_bytes = a.n_aux_pad * NS * 2;
  const char* panel = static_cast<const char*>(a.Bs) + ((size_t)hole_w * a.n_v_pad + tile_w * TM) * row_bytes;
  // row 8 m + l/8 of the panel, logical slot (l % 8) ^ f(row) = (l % 8) ^ (l / 8) ^ m
  const int l3 = lane >> 3, l7 = lane & 7;
  auto src_off = [&](int m) -> uint32_t {
    const int sl = l7 ^ l3 ^ m;
    const int t = sl >> 1, h = sl & 1;
    return (uint32_t)((8 * m + l3) * row_bytes + (t < NS ? t * 32 + h * 16 : 0));
  };
  auto load_chunk = [&](int chunk, u4* buf) {
    if (!load_w) return;
    const char* base = panel + (size_t)chunk * (KC * NS * 2);
#pragma unroll
    for (int m = 0; m < 8; ++m)
      __builtin_amdgcn_global_load_lds((gbl_void*)(base + src_off(m)), (lds_void*)(buf + q_w * PANEL_U4 + m * 64),
                                       16, 0, 0);
  };

  f16v accP[3], accQ[3];
  double dP[16], dQ[16];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accP[l][r] = 0.f;
      accQ[l][r] = 0.f;
    }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    dP[r] = 0.0;
    dQ[r] = 0.0;
  }

  const int nchunk = a.n_aux_pad / KC;
  const int r32 = lane & 31, hq = lane >> 5;
  const int rowA = wr * 32 + r32, rowB = wc * 32 + r32;
  const int fA = swz(rowA), fB = swz(rowB);

  // one chunk from LDS buffer `buf`: NS (NS+1)/2 slice products for P, then for Q
  auto compute = [&](const u4* buf, int c) {
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
    if (!same) {
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
    }
    if ((c + 1) % FLUSH_CHUNKS == 0 || c + 1 == nchunk) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        dP[r] += (double)accP[0][r] + (double)accP[1][r];
        dQ[r] += (double)accQ[0][r] + (double)accQ[1][r];
        accP[0][r] = 0.f;
        accP[1][r] = 0.f;
        accQ[0][r] = 0.f;
        accQ[1][r] = 0.f;
      }
    }
  };
  // chunk c + 1 streams into one buffer while chunk c is multiplied out of the
  // other; the wait + barrier publishes it and retires the reads of the old one
  auto step = [&](int c, u4* cur, u4* nxt) {
    if (c + 1 < nchunk) load_chunk(c + 1, nxt);
    compute(cur, c);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  load_chunk(0, lds0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  int c = 0;
  for (; c + 1 < nchunk; c += 2) {
    step(c, lds0, lds1);
    step(c + 1, lds1, lds0);
  }
  if (c < nchunk) step(c, lds0, lds1);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    dP[r] += (double)accP[2][r];
    dQ[r] += (double)accQ[2][r];
  }
  if (same) {
#pragma unroll
    for (int r = 0; r < 16; ++r) dQ[r] = dP[r];
  }

  // the last step ended with a barrier: LDS is free for the epilogue's scratch
  sliced_pair_epilogue<STORE>(a, p, tp, I, J, hi_i, hi_j, dP, dQ, reinterpret_cast<double*>(lds0));
}

hipError_t launch_pair_gemm_bf16(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if ((long long)a.nTP * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  // energy only: passes that store amplitudes run the product and the epilogue
  // as two kernels (pair_bf16_v.hip)
  if (a.T || a.Vr) return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  dim3 grid(a.nTP * n_pairs), block(256);
  switch (ns) {
    case 2: hipLaunchKernelGGL((pair_gemm_bf16_kernel<2, false>), grid, block, 0, st, b); break;
    case 3: hipLaunchKernelGGL((pair_gemm_bf16_kernel<3, false>), grid, block, 0, st, b); break;
    case 4: hipLaunchKernelGGL((pair_gemm_bf16_kernel<4, false>), grid, block, 0, st, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dfpt2
