// INT8-digit pair product V = B_i B_j^T on its own (the form of pair_bf16_v.hip
// for the digits of split.hip): 128 x 128 tiles of the full V^{ij}, written in
// FP64 into a buffer of one batch, after which pair_epi_bf16_kernel runs the
// DSRG epilogue (paper App. A, Eq. A7) on it, as for the BF16 slices.
//
// With NS digits per row, x_a = 2^e_a sum_s d_s(a) 2^(-8s), the product of two
// rows is 2^(e_a + e_b) sum_L 2^(-8L) sum_{s + t = L} sum_k d_s(a)_k d_t(b)_k.  The
// kernel keeps the levels L <= NS - 1 (15 digit products at NS = 5) and sums each
// in its own INT32 accumulator, exact for n_aux_pad NS 2^14 < 2^31 (the launcher
// refuses more), then combines the levels by Horner in 2^-8 and scales them by
// 2^(e_a + e_b) in FP64 once, after the contraction.  For i == j the epilogue
// replaces the diagonal by the FP64 norm ||B_ia||^2, and the tiles wholly below
// the diagonal of the symmetric V^{ii} are not formed (the epilogue reads Q where
// P is).
//
// Tile: 8 waves, one workgroup per CU, wave (wr, wc) owns rows 64 wr .. + 63 (two
// 32 x 32 blocks of the 32x32x32 INT8 MFMA) and columns 32 wc .. + 31: 5 INT32
// registers per output element and no periodic flushes.  Against the fused INT8
// kernel (64 x 64 tile pairs, four 64-row panels per chunk) the tile moves half
// the bytes per output.  Staging: one 32-wide contraction chunk of a 128-row
// panel is 128 x 32 NS contiguous bytes (chunk-major digits), moved by direct
// loads (global_load_lds, 16 bytes per lane) into LDS rows laid out as in
// i8_layout.h, through a ring of NBUF slots: step c issues the loads of chunk
// c + NBUF - 1, runs the products of chunk c, waits for its own loads of chunk
// c + 1 only and closes with a barrier that carries no memory fence.  Block
// order: every XCD walks a contiguous range of (pair, tile), the tiles of one
// pair in bands of 6 tile rows, as in the BF16 kernel.
#include <type_traits>

#include "common.h"
#include "i8_layout.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TV = 128;  // V tile edge
constexpr int KC = 32;   // contraction chunk (INT8 MFMA K)
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int xcd_block_vi(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

// s_waitcnt immediate (gfx9 encoding): wait until at most n vector-memory
// operations of this wave are outstanding, other counters untouched
constexpr int vm_wait_imm(int n) { return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4) | (15 << 8); }
}  // namespace

template <int NS, int NBUF>
__global__ __launch_bounds__(512, 1) void pair_v_i8_kernel(PairSlicedArgs a, int nti, int ntj) {
  static_assert(NBUF == 3, "ring of 3 slots");
  constexpr int SLOTS = 2 * NS;         // 16-byte slots per LDS row
  constexpr int PANEL_U4 = TV * SLOTS;  // u4 per 128-row panel
  constexpr int ROWB = 32 * NS;         // bytes of one row of one chunk
  constexpr int LOADS = PANEL_U4 / 64;  // 1 KB direct loads per panel and chunk
  constexpr int LPW = 2 * LOADS / 8;    // loads per wave per chunk
  static_assert(LPW * 8 == 2 * LOADS, "whole loads per wave");
  // distinct arrays per ring slot and panel, so that the compiler's alias scopes
  // tell the slots apart (a read of one slot does not wait for loads into another)
  __shared__ u4 la0[PANEL_U4], la1[PANEL_U4], la2[PANEL_U4];
  __shared__ u4 lb0[PANEL_U4], lb1[PANEL_U4], lb2[PANEL_U4];
  auto slot_a = [&](auto K) __attribute__((always_inline)) -> u4* {
    if constexpr (K() == 0) return la0;
    else if constexpr (K() == 1) return la1;
    else return la2;
  };
  auto slot_b = [&](auto K) __attribute__((always_inline)) -> u4* {
    if constexpr (K() == 0) return lb0;
    else if constexpr (K() == 1) return lb1;
    else return lb2;
  };
  const int per_pair = nti * ntj;
  const int L = xcd_block_vi(blockIdx.x, per_pair * a.n_blk_pairs);
  const int p = L / per_pair, t = L - p * per_pair;
  constexpr int HB = 6;
  const int band = t / (HB * ntj), h = min(HB, nti - band * HB), r = t - band * HB * ntj;
  const int J = r / h, I = band * HB + (r - (r / h) * h);
  const int2 pr = a.pairs[p];
  // V^{ii} is symmetric and its epilogue takes Q from P: the tiles wholly below
  // the diagonal are never read (the whole workgroup leaves before any barrier)
  if (pr.x == pr.y && I > J) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3;

  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const size_t chunk_stride = (size_t)a.n_v_pad * ROWB;
  const char* Bs = static_cast<const char*>(a.Bs);
  const char* panelA = Bs + (size_t)pr.x * (a.n_aux_pad / KC) * chunk_stride + (size_t)I * TV * ROWB;
  const char* panelB = Bs + (size_t)pr.y * (a.n_aux_pad / KC) * chunk_stride + (size_t)J * TV * ROWB;
  // LDS unit u of a panel chunk is row u / SLOTS, physical slot u % SLOTS; lane l of
  // load g fills unit 64 g + l with the logical slot that lands there
  auto src_off = [&](int g) __attribute__((always_inline)) -> uint32_t {
    const int u = 64 * g + lane, rr = u / SLOTS, ps = u - rr * SLOTS;
    return (uint32_t)(rr * ROWB + 16 * i8l::logical_slot<NS>(rr, ps));
  };
  const int nchunk = a.n_aux_pad / KC;
  auto load_chunk = [&](int chunk, auto K) __attribute__((always_inline)) {  // chunk < nchunk; into slot K
    const size_t coff = (size_t)chunk * chunk_stride;
#pragma unroll
    for (int m = 0; m < LPW; ++m) {
      const int g = LPW * q_w + m;  // wave-uniform
      if (g < LOADS)
        __builtin_amdgcn_global_load_lds((gbl_void*)(panelA + coff + src_off(g)), (lds_void*)(slot_a(K) + 64 * g), 16,
                                         0, 0);
      else
        __builtin_amdgcn_global_load_lds((gbl_void*)(panelB + coff + src_off(g - LOADS)),
                                         (lds_void*)(slot_b(K) + 64 * (g - LOADS)), 16, 0, 0);
    }
  };

  v16i acc[2][NS];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int l = 0; l < NS; ++l)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[b][l][e] = 0;

  const int r32 = lane & 31, hq = lane >> 5;
  // per-lane u4 index of every fragment within a slot; passed through an empty asm
  // in every step, so that the compiler forms each slot's addresses at the read
  int offB[NS], offA[2][NS];
  {
    const int rowB = wc * 32 + r32;
#pragma unroll
    for (int s = 0; s < NS; ++s) offB[s] = rowB * SLOTS + i8l::phys_slot<NS>(rowB, 2 * s + hq);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int rowA = wr * 64 + b * 32 + r32;
#pragma unroll
      for (int s = 0; s < NS; ++s) offA[b][s] = rowA * SLOTS + i8l::phys_slot<NS>(rowA, 2 * s + hq);
    }
  }
  auto compute = [&](auto K) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      asm volatile("" : "+v"(offB[s]));
      asm volatile("" : "+v"(offA[0][s]));
      asm volatile("" : "+v"(offA[1][s]));
    }
    v4i fb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) fb[s] = __builtin_bit_cast(v4i, slot_b(K)[offB[s]]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      v4i fa[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) fa[s] = __builtin_bit_cast(v4i, slot_a(K)[offA[b][s]]);
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int u = 0; u + s < NS; ++u)
          acc[b][s + u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[s], fb[u], acc[b][s + u], 0, 0, 0);
    }
  };
  // the workgroup barrier without the memory fence of __syncthreads; the empty
  // asm keeps the compiler from moving memory accesses across it
  auto barrier = []() __attribute__((always_inline)) {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // step c: the loads of chunk c + 2 go into the slot chunk c - 1 was read from,
  // the products of chunk c follow, then each wave waits for its own loads of
  // chunk c + 1 (those of chunk c + 2 stay in flight) and the barrier makes every
  // wave's part of chunk c + 1 visible; no branch around a load or a wait in the
  // steady state, the last steps run as tail steps that wait for everything
  auto step = [&](int c, auto cur, auto nxt) __attribute__((always_inline)) {
    load_chunk(c + NBUF - 1, nxt);
    compute(cur);
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(LPW * (NBUF - 2)));
    barrier();
  };
  auto tail_step = [&](int c, auto cur, auto nxt) __attribute__((always_inline)) {
    if (c >= nchunk) return;  // uniform
    if (c + NBUF - 1 < nchunk) load_chunk(c + NBUF - 1, nxt);
    compute(cur);
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));
    barrier();
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  auto ring = [&](int c, auto&& f) __attribute__((always_inline)) {
    f(c, S0{}, S2{});
    f(c + 1, S1{}, S0{});
    f(c + 2, S2{}, S1{});
  };

  if (nchunk >= 2 * NBUF - 1) {
    load_chunk(0, S0{});
    load_chunk(1, S1{});
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(LPW * (NBUF - 2)));  // chunk 0 has landed
  } else {
    if (nchunk > 0) load_chunk(0, S0{});
    if (nchunk > 1) load_chunk(1, S1{});
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));
  }
  barrier();
  int c = 0;
  // steady state: every step of a revolution loads a chunk that exists
  for (; c + 2 * NBUF - 2 < nchunk; c += NBUF) ring(c, step);
  ring(c, tail_step);
  if (c + NBUF < nchunk) ring(c + NBUF, tail_step);

  // levels -> FP64 (Horner in 2^-8, exact up to the final rounding), times the row
  // scales; register e of lane l of a 32 x 32 block is row 8(e/4) + 4(l/32) + e%4,
  // column l%32
  const int n_v = a.n_v;
  double* Vp = a.T + (size_t)p * n_v * n_v;
  const int* ei = a.rexp + (size_t)pr.x * a.n_v_pad;
  const int* ej = a.rexp + (size_t)pr.y * a.n_v_pad;
  const int gb = J * TV + wc * 32 + r32;
  if (gb < n_v) {
    const int eb = ej[gb];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int ga = I * TV + wr * 64 + b * 32 + 8 * (e >> 2) + 4 * hq + (e & 3);
        if (ga >= n_v) continue;
        double v = (double)acc[b][NS - 1][e];
#pragma unroll
        for (int l = NS - 2; l >= 0; --l) v = v * 0.00390625 + (double)acc[b][l][e];
        Vp[(size_t)ga * n_v + gb] = ldexp(v, ei[ga] + eb);
      }
  }
}

hipError_t launch_pair_v_i8(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (!a.T || !a.rexp || a.n_v_pad % TV != 0 || a.n_aux_pad % KC != 0 || a.n_aux_pad > pair_i8_max_aux_pad(ns))
    return hipErrorInvalidValue;
  const int nti = (a.n_v + TV - 1) / TV, ntj = nti;
  if ((long long)nti * ntj * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  const dim3 grid(nti * ntj * n_pairs), block(512);
  switch (ns) {
    case 3: hipLaunchKernelGGL((pair_v_i8_kernel<3, 3>), grid, block, 0, st, b, nti, ntj); break;
    case 4: hipLaunchKernelGGL((pair_v_i8_kernel<4, 3>), grid, block, 0, st, b, nti, ntj); break;
    case 5: hipLaunchKernelGGL((pair_v_i8_kernel<5, 3>), grid, block, 0, st, b, nti, ntj); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dfpt2
