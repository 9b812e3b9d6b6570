// INT8 pair kernel: V = B_i B_j^T from the balanced base-256 digits of split.hip
// on the 32x32x32 INT8 MFMA, with the fused DSRG regularizer/energy epilogue of
// the other pair kernels (paper App. A, Eq. A7; pair_epilogue.h).
//
// With NS digits per row, x_a = 2^e_a sum_s d_s(a) 2^(-8s), the product of two
// rows is
//     2^(e_a + e_b) sum_L 2^(-8L) sum_{s + t = L} sum_k d_s(a)_k d_t(b)_k.
// The kernel keeps the levels L <= NS - 1 (NS (NS+1)/2 digit products; 15 at
// NS = 5, which leaves a relative error near 2^-38 per element) and sums every
// level in its own INT32 accumulator.  A digit product is at most 2^14 in
// magnitude and a level holds at most NS products per contraction index, so the
// level sums are exact integers for n_aux_pad NS 2^14 < 2^31 (n_aux <= 26208 at
// NS = 5; the launcher refuses more).  The levels are combined and scaled by
// 2^(e_a + e_b) in FP64 once, after the contraction: no periodic flushes, and
// 5 bytes per element instead of the 8 of four BF16 slices.
//
// For i == j the diagonal V^{ii}_{aa} = ||B_ia||^2 comes from the FP64 norm
// computed while splitting (the dropped digit products there are biased).
//
// Tiling as in pair_f64.hip, order as in pair_bf16_v.hip: one workgroup = unordered pair {i <= j}
// x tile pair (I <= J) of 64 x 64, every wave owns the same 32 x 32 block of
// P = V^{ij}[I,J] and Q = V^{ji}[I,J]; the 1-D launch is remapped so that every
// XCD walks a contiguous range of (pair, tile pair).
//
// Staging: one 32-wide contraction chunk of a 64-row panel is 64 x 32 NS
// contiguous bytes (chunk-major digits), moved by 2 NS direct loads
// (global_load_lds, 16 bytes per lane) into LDS, double buffered.  An LDS row
// holds 2 NS slots of 16 bytes (digit t, half h -> logical slot 2t + h); the
// physical slot is XOR-swizzled (NS = 4: 128-byte rows) or rotated by
// NS ((r >> 2) ^ (r >> 3)) & 1 (NS = 3, 5) so that the fragment reads of 8 or 16
// consecutive rows at one logical slot hit distinct banks.  The direct load of
// lane l of load m fills LDS unit 64 m + l and fetches whatever logical slot
// lands there: the fetches of one load stay inside ~7 consecutive rows.
#include "common.h"
#include "i8_layout.h"
#include "kernels.h"
#include "pair_epilogue.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 32;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int xcd_block_i8(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}
}  // namespace

template <int NS, bool STORE>
__global__ __launch_bounds__(256, 2) void pair_gemm_i8_kernel(PairSlicedArgs a) {
  constexpr int SLOTS = 2 * NS;         // 16-byte slots per LDS row
  constexpr int PANEL_U4 = TM * SLOTS;  // u4 per panel
  constexpr int ROWB = 32 * NS;         // bytes of one row of one chunk
  __shared__ u4 lds[2][4 * PANEL_U4];
  const int L = xcd_block_i8(blockIdx.x, a.nTP * a.n_blk_pairs);
  const int p = L / a.nTP, tp = L - p * a.nTP;
  int I, J;
  tile_pair(tp, a.nt, I, J);
  const int2 pr = a.pairs[p];
  const int hi_i = pr.x, hi_j = pr.y;
  const bool same = (hi_i == hi_j);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int npanel = same ? 2 : 4;

  // wave w fills panel w: 0 = B_i[I], 1 = B_j[J], 2 = B_j[I], 3 = B_i[J]
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int hole_w = (q_w == 0 || q_w == 3) ? hi_i : hi_j;
  const int tile_w = (q_w == 0 || q_w == 2) ? I : J;
  const bool load_w = q_w < npanel;
  const size_t chunk_stride = (size_t)a.n_v_pad * ROWB;
  const char* panel = static_cast<const char*>(a.Bs) + (size_t)hole_w * (a.n_aux_pad / KC) * chunk_stride +
                      (size_t)tile_w * TM * ROWB;
  // byte offset, inside one panel chunk, of what lane l fetches in load m
  // (recomputed per load: a few integer operations instead of 2 NS live registers)
  auto src_off = [&](int m) -> uint32_t {
    const int u = 64 * m + lane, r = u / SLOTS, ps = u - r * SLOTS;
    return (uint32_t)(r * ROWB + 16 * i8l::logical_slot<NS>(r, ps));
  };
  auto load_chunk = [&](int chunk, u4* buf) {
    if (!load_w) return;
    const char* base = panel + (size_t)chunk * chunk_stride;
#pragma unroll
    for (int m = 0; m < SLOTS; ++m)
      __builtin_amdgcn_global_load_lds((gbl_void*)(base + src_off(m)), (lds_void*)(buf + q_w * PANEL_U4 + m * 64),
                                       16, 0, 0);
  };

  v16i accP[NS], accQ[NS];
#pragma unroll
  for (int l = 0; l < NS; ++l)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accP[l][r] = 0;
      accQ[l][r] = 0;
    }

  const int nchunk = a.n_aux_pad / KC;
  const int r32 = lane & 31, hq = lane >> 5;
  const int rowA = wr * 32 + r32, rowB = wc * 32 + r32;
  auto offA = [&](int t) { return rowA * SLOTS + i8l::phys_slot<NS>(rowA, 2 * t + hq); };
  auto offB = [&](int t) { return rowB * SLOTS + i8l::phys_slot<NS>(rowB, 2 * t + hq); };

  // one chunk: the NS (NS+1)/2 digit products of levels < NS for P, then for Q
  auto compute = [&](const u4* buf) {
    v4i fa[NS], fb[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      fa[t] = __builtin_bit_cast(v4i, buf[0 * PANEL_U4 + offA(t)]);
      fb[t] = __builtin_bit_cast(v4i, buf[1 * PANEL_U4 + offB(t)]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int t = 0; t + s < NS; ++t)
        accP[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[s], fb[t], accP[s + t], 0, 0, 0);
    if (!same) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        fa[t] = __builtin_bit_cast(v4i, buf[2 * PANEL_U4 + offA(t)]);
        fb[t] = __builtin_bit_cast(v4i, buf[3 * PANEL_U4 + offB(t)]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t + s < NS; ++t)
          accQ[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[s], fb[t], accQ[s + t], 0, 0, 0);
    }
  };
  // chunk c + 1 streams into one buffer while chunk c is multiplied out of the
  // other; the wait + barrier publishes it and retires the reads of the old one
  auto step = [&](int c, u4* cur, u4* nxt) {
    if (c + 1 < nchunk) load_chunk(c + 1, nxt);
    compute(cur);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  load_chunk(0, lds[0]);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  int c = 0;
  for (; c + 1 < nchunk; c += 2) {
    step(c, lds[0], lds[1]);
    step(c + 1, lds[1], lds[0]);
  }
  if (c < nchunk) step(c, lds[0], lds[1]);

  // levels -> FP64 (Horner in 2^-8, exact up to the final rounding), times the
  // row scales; P pairs rows of B_i with rows of B_j, Q rows of B_j with B_i
  double dP[16], dQ[16];
  const int* ei = a.rexp + (size_t)hi_i * a.n_v_pad;
  const int* ej = a.rexp + (size_t)hi_j * a.n_v_pad;
  const int gb = J * TM + wc * 32 + r32;
  const int ebP = ej[gb], ebQ = ei[gb];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ga = I * TM + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
    double vp = (double)accP[NS - 1][r], vq = (double)accQ[NS - 1][r];
#pragma unroll
    for (int l = NS - 2; l >= 0; --l) {
      vp = vp * 0.00390625 + (double)accP[l][r];
      vq = vq * 0.00390625 + (double)accQ[l][r];
    }
    dP[r] = ldexp(vp, ei[ga] + ebP);
    dQ[r] = same ? dP[r] : ldexp(vq, ej[ga] + ebQ);
  }
  // the last step ended with a barrier: LDS is free for the epilogue's scratch
  sliced_pair_epilogue<STORE>(a, p, tp, I, J, hi_i, hi_j, dP, dQ, reinterpret_cast<double*>(&lds[0][0]));
}

int pair_i8_max_aux_pad(int ns) {
  // every level sum stays below 2^31: ns products of at most 2^14 per contraction index
  return ns >= 1 ? (int)((0x7fffffffLL / ((long long)ns << 14)) / KC * KC) : 0;
}

hipError_t launch_pair_gemm_i8(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if ((long long)a.nTP * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.n_aux_pad % KC != 0 || a.n_aux_pad > pair_i8_max_aux_pad(ns) || a.n_v_pad % TM != 0 || !a.rexp)
    return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  dim3 grid(a.nTP * n_pairs), block(256);
  const bool store = a.T != nullptr || a.Vr != nullptr;
#define DFPT2_LAUNCH(NS_)                                                                          \
  if (store)                                                                                       \
    hipLaunchKernelGGL((pair_gemm_i8_kernel<NS_, true>), grid, block, 0, st, b);                    \
  else                                                                                             \
    hipLaunchKernelGGL((pair_gemm_i8_kernel<NS_, false>), grid, block, 0, st, b);
  switch (ns) {
    case 3: DFPT2_LAUNCH(3) break;
    case 4: DFPT2_LAUNCH(4) break;
    case 5: DFPT2_LAUNCH(5) break;
    default: return hipErrorInvalidValue;
  }
#undef DFPT2_LAUNCH
  return hipGetLastError();
}

}  // namespace dfpt2
