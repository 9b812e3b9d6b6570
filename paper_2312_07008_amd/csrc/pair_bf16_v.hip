// Split-BF16 pair product V = B_i B_j^T and the DSRG epilogue (paper App. A,
// Eq. A7), in two kernels:
//
//   pair_v_bf16_kernel    V^{ij} = B_i B_j^T over 128 x 128 tiles of the full
//                         n_v x n_v matrix, written in FP64 into a buffer of one
//                         batch (the amplitude buffer T[p] when the pass stores
//                         amplitudes);
//   pair_epi_bf16_kernel  per 64 x 64 tile pair (I <= J), V[I,J] and V[J,I]^T
//                         read back into the MFMA register layout, then the
//                         regularizer / energy / density-row epilogue of
//                         pair_epilogue.h, which (STORE) overwrites V with T in
//                         place, or (energy-only passes) only forms the energy
//                         and norm partials.  It also serves the INT8-digit
//                         product (pair_i8_v.hip).  The D_vv pass with the
//                         split-BF16 density runs epi_split_bf16.hip instead,
//                         which writes the density operands' slices.
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
// slicing error.  For i == j the epilogue replaces the diagonal V^{ii}_{aa} by
// ||B_ia||^2 from an FP64 norm computed while splitting: the dropped slice
// products (t, t) there are sums of squares, i.e. biased, and the diagonal
// carries a large share of E.
//
// Why two kernels: a fused kernel (the FP64, FP8 and INT8 pair kernels) computes
// V^{ij}[I,J] and V^{ji}[I,J] in one workgroup so that the exchange partner of
// every element is lane-local, which fixes its tile at 64 x 64 per product.  The
// time of these kernels is set by the bytes the direct loads request (L2 hits and
// misses), so here the product runs on its own with a 128 x 128 tile, half the
// bytes per flop, at the cost of one FP64 write and two FP64 reads of V per
// element (a few ms per batch).  Measured on the 80-core, 1200-virtual,
// 4000-auxiliary workload, ms per batch of 512 pairs for both kernels: fused BF16
// kernel (which this replaced) 62.6; with the chunk loads placed late in each step
// (two fixed LDS buffers, below the fragment reads where the compiler scheduled
// them) 128 x 64 tiles (4 waves, two workgroups per CU) 58.6, 128 x 128 tiles
// (8 waves, one per CU) 59.9, 128 x 32 tiles 80.1; with the loads first in the
// step, on one box, 128 x 64 53.1 and 128 x 128 51.1.
//
// Tile of the V kernel: 8 waves, wave (wr, wc) owns rows 64 wr .. 64 wr + 63
// (two 32 x 32 MFMA blocks) and columns 32 wc .. 32 wc + 31; one workgroup per
// CU.  Staging: 16-wide contraction chunks of two 128-row panels go from global
// memory straight into LDS (global_load_lds, 16 bytes per lane, no register
// round trip) through a ring of four 32 KB slots; every wave moves 4 of the 32
// kilobytes of a chunk.  Step c issues the loads of chunk c + 3, runs the
// products of chunk c, waits for its own loads of chunk c + 1 only and closes
// with a barrier that carries no memory fence, so two chunks stay in flight
// across it.  (The fence of __syncthreads waits for every outstanding load; the
// ring slots are distinct LDS arrays so that the compiler's alias scopes keep it
// from waiting for all loads before a fragment read.)  Same results bit for bit
// as the two-buffer form with one chunk in flight, and 1% faster (53.8 -> 53.1 ms
// per batch of 512 pairs at 1200 virtuals and 4000 auxiliary functions).
// Measured on that workload, ms per batch, with variants compiled from this
// kernel: the same products with constant fragments instead of the LDS reads
// 39.6, only the chunk loads and barriers (no products, no reads) 32.5, ring of
// three 54.0, s_setprio raised around the products 53.9, 128 x 64 tiles with two
// workgroups per CU 53.3, slabs stored chunk-major (each step reads two
// contiguous 16 KB blocks) 53.7.  The direct loads deliver about 21 bytes per
// clock per CU, so the loads alone take 60% of the kernel, and the fragment reads
// of all eight waves, issued together after each barrier, cost another 14 ms
// that the products do not hide.
// One LDS row holds the chunk of one virtual: 8 slots of 16 bytes
// (slice t, half h -> slot 2t + h; slots >= 2 NS are padding), XOR-swizzled by
// f(r) = (r ^ (r >> 3)) & 7 so that the fragment reads (eight or sixteen
// consecutive rows, one logical slot) hit distinct banks and each direct load
// fills one contiguous kilobyte (8 rows x 8 slots) with no conflict.  The slabs
// must have a multiple of 128 rows.
//
// Block order: the hardware deals consecutive workgroups round-robin to the 8
// XCDs, each with its own L2.  The launch is 1-D and the block index is remapped
// so that every XCD walks a contiguous range of (pair, tile) in order: the
// workgroups resident on one XCD then belong to one or two pairs and share the
// same slabs B_i, B_j through that XCD's L2.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "pair_epilogue.h"

namespace dfpt2 {

namespace {
constexpr int TV = 128;               // V tile edge
constexpr int KC = 16;
constexpr int SLOTS = 8;
constexpr int kVWaveCols = 4;         // column waves: 128 x 128 tiles, 8 waves, one workgroup per CU
constexpr int kVRing = 4;             // LDS ring slots: loads run three chunks ahead
constexpr int FLUSH_CHUNKS = 128 / KC;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int swz_v(int r) { return (r ^ (r >> 3)) & 7; }

__device__ inline int xcd_block_v(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}
}  // namespace

// s_waitcnt immediate (gfx9 encoding) that waits until at most n vector-memory
// operations of this wave are outstanding and leaves the other counters alone.
// Issued through the builtin, not inline asm, so that the compiler's own wait
// insertion sees it and does not add a vmcnt(0) before the LDS reads.
constexpr int vm_wait_imm(int n) { return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4) | (15 << 8); }

// WC column waves: tile 128 x (32 WC) of V, 2 WC waves, wave (wr, wc) owns rows
// 64 wr .. + 63 and columns 32 wc .. + 31.  NBUF LDS buffers form a ring: the
// loads run NBUF - 1 chunks ahead of the products.
template <int NS, int WC, int NBUF>
__global__ __launch_bounds__(128 * WC, 4 / WC) void pair_v_bf16_kernel(PairSlicedArgs a, int nti, int ntj) {
  static_assert(2 * NS <= SLOTS, "slices per LDS row");
  static_assert(NBUF >= 2 && NBUF <= 4, "ring of 2 to 4 buffers");
  constexpr int TJ = 32 * WC;                     // V tile columns
  constexpr int KB_A = TV / 8, KB_B = TJ / 8;     // kilobytes of the two panels per chunk
  constexpr int KB_W = (KB_A + KB_B) / (2 * WC);  // kilobytes per wave per chunk
  static_assert(KB_W * 2 * WC == KB_A + KB_B, "whole kilobytes per wave");
  // distinct arrays per ring slot and panel: the compiler's alias scopes then
  // tell the slots apart, so a read of one slot does not wait for the loads into
  // another; the panel-A slots (and the panel-B slots) lie within the 64 KB reach
  // of one ds_read offset, so one address register serves a fragment in every slot
  __shared__ u4 la0[KB_A * 64], la1[KB_A * 64], la2[NBUF > 2 ? KB_A * 64 : 1], la3[NBUF > 3 ? KB_A * 64 : 1];
  __shared__ u4 lb0[KB_B * 64], lb1[KB_B * 64], lb2[NBUF > 2 ? KB_B * 64 : 1], lb3[NBUF > 3 ? KB_B * 64 : 1];
  // ring slot K as a compile-time index (no pointer to a slot is ever stored)
  auto slot_a = [&](auto K) -> u4* {
    if constexpr (K() == 0) return la0;
    else if constexpr (K() == 1) return la1;
    else if constexpr (K() == 2) return la2;
    else return la3;
  };
  auto slot_b = [&](auto K) -> u4* {
    if constexpr (K() == 0) return lb0;
    else if constexpr (K() == 1) return lb1;
    else if constexpr (K() == 2) return lb2;
    else return lb3;
  };
  const int per_pair = nti * ntj;
  const int L = xcd_block_v(blockIdx.x, per_pair * a.n_blk_pairs);
  const int p = L / per_pair, t = L - p * per_pair;
  // tiles of one pair in bands of HB tile rows, taken column by column within a
  // band: the ~32 workgroups resident on one XCD then read about 6 + 5 panels
  // instead of the 14 of 3-4 whole tile rows (1% faster than row order)
  constexpr int HB = 6;
  const int band = t / (HB * ntj), h = min(HB, nti - band * HB), r = t - band * HB * ntj;
  const int J = r / h, I = band * HB + (r - (r / h) * h);
  const int2 pr = a.pairs[p];
  // V^{ii} is symmetric and its epilogue takes Q from P: the tiles wholly below
  // the diagonal are never read (the whole workgroup leaves before any barrier)
  if (pr.x == pr.y && I * TV >= (J + 1) * TJ) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w / WC, wc = w - (w / WC) * WC;

  // kilobyte kb < KB_A of a chunk is rows 8 kb .. + 7 of panel A (B_i rows of tile I),
  // kilobyte KB_A + kb rows 8 kb .. + 7 of panel B (B_j rows of tile J); wave w moves
  // kilobytes KB_W w .. + KB_W - 1; lane l fills physical slot l % 8 of row l / 8
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int row_bytes = a.n_aux_pad * NS * 2;
  const char* panelA = static_cast<const char*>(a.Bs) + ((size_t)pr.x * a.n_v_pad + (size_t)I * TV) * row_bytes;
  const char* panelB = static_cast<const char*>(a.Bs) + ((size_t)pr.y * a.n_v_pad + (size_t)J * TJ) * row_bytes;
  const int l3 = lane >> 3, l7 = lane & 7;
  auto src_off = [&](int kb) -> uint32_t {  // kb within its panel
    const int row = 8 * kb + l3;
    const int sl = l7 ^ swz_v(row);
    const int ts = sl >> 1, h = sl & 1;
    return (uint32_t)(row * row_bytes + (ts < NS ? ts * 32 + h * 16 : 0));
  };
  const int nchunk = a.n_aux_pad / KC;
  auto load_chunk = [&](int chunk, auto K) {  // chunk < nchunk; into slot K
    const size_t coff = (size_t)chunk * (KC * NS * 2);
#pragma unroll
    for (int m = 0; m < KB_W; ++m) {
      const int kb = KB_W * q_w + m;  // wave-uniform
      if (kb < KB_A)
        __builtin_amdgcn_global_load_lds((gbl_void*)(panelA + coff + src_off(kb)), (lds_void*)(slot_a(K) + kb * 64), 16,
                                         0, 0);
      else
        __builtin_amdgcn_global_load_lds((gbl_void*)(panelB + coff + src_off(kb - KB_A)),
                                         (lds_void*)(slot_b(K) + (kb - KB_A) * 64), 16, 0, 0);
    }
  };

  f16v acc[2][3];
  double dV[2][16];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][l][r] = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) dV[b][r] = 0.0;
  }

  const int r32 = lane & 31, hq = lane >> 5;
  // per-lane u4 index of every fragment within a slot (row, swizzled logical slot);
  // passed through an empty asm in every step, so that the compiler forms each
  // slot's addresses at the read instead of holding NBUF x 3 NS of them in registers
  int offB[NS], offA[2][NS];
  {
    const int rowB = wc * 32 + r32, fB = swz_v(rowB);
#pragma unroll
    for (int s = 0; s < NS; ++s) offB[s] = rowB * SLOTS + ((2 * s + hq) ^ fB);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int rowA = wr * 64 + b * 32 + r32, fA = swz_v(rowA);
#pragma unroll
      for (int s = 0; s < NS; ++s) offA[b][s] = rowA * SLOTS + ((2 * s + hq) ^ fA);
    }
  }

  auto compute = [&](auto K, int c) {  // chunk c from slot K
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      asm volatile("" : "+v"(offB[s]));
      asm volatile("" : "+v"(offA[0][s]));
      asm volatile("" : "+v"(offA[1][s]));
    }
    bf8v fb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) fb[s] = __builtin_bit_cast(bf8v, slot_b(K)[offB[s]]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      bf8v fa[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) fa[s] = __builtin_bit_cast(bf8v, slot_a(K)[offA[b][s]]);
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int u = 0; u + s < NS; ++u) {
          const int lv = (s + u) < 2 ? (s + u) : 2;
          acc[b][lv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[u], acc[b][lv], 0, 0, 0);
        }
    }
    if ((c + 1) % FLUSH_CHUNKS == 0 || c + 1 == nchunk) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          dV[b][r] += (double)acc[b][0][r] + (double)acc[b][1][r];
          acc[b][0][r] = 0.f;
          acc[b][1][r] = 0.f;
        }
    }
  };
  // the workgroup barrier without the memory fence of __syncthreads (whose
  // release waits for every outstanding load, vmcnt(0)); the empty asm keeps the
  // compiler from moving memory accesses across it
  auto barrier = [] {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // step c: the loads of chunk c + NBUF - 1 go into the slot chunk c - 1 was read
  // from (every wave finished those reads before the last barrier), the products
  // of chunk c follow, then each wave waits for its own loads of chunk c + 1 --
  // the KB_W (NBUF - 2) loads issued after them may stay in flight -- and the
  // barrier makes every wave's part of chunk c + 1 visible.  The steady-state loop
  // has no branch around a load or a wait (a merge of paths with different
  // outstanding loads makes the compiler wait for all of them); the last
  // 2 NBUF - 2 or fewer steps run in a tail that checks each load and waits for
  // everything.
  auto step = [&](int c, auto cur, auto nxt) {
    load_chunk(c + NBUF - 1, nxt);
    compute(cur, c);
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(KB_W * (NBUF - 2)));
    barrier();
  };
  auto tail_step = [&](int c, auto cur, auto nxt) {
    if (c >= nchunk) return;  // uniform
    if (c + NBUF - 1 < nchunk) load_chunk(c + NBUF - 1, nxt);
    compute(cur, c);
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));
    barrier();
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  auto ring = [&](int c, auto&& f) {
    if constexpr (NBUF == 2) {
      f(c, S0{}, S1{});
      f(c + 1, S1{}, S0{});
    } else if constexpr (NBUF == 3) {
      f(c, S0{}, S2{});
      f(c + 1, S1{}, S0{});
      f(c + 2, S2{}, S1{});
    } else {
      f(c, S0{}, S3{});
      f(c + 1, S1{}, S0{});
      f(c + 2, S2{}, S1{});
      f(c + 3, S3{}, S2{});
    }
  };

  // chunks 0 .. NBUF - 2 before the first step (chunk k lives in slot k % NBUF)
  if (nchunk >= 2 * NBUF - 1) {
    load_chunk(0, S0{});
    if constexpr (NBUF > 2) load_chunk(1, S1{});
    if constexpr (NBUF > 3) load_chunk(2, S2{});
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(KB_W * (NBUF - 2)));  // chunk 0 has landed
  } else {
    if (nchunk > 0) load_chunk(0, S0{});
    if (NBUF > 2 && nchunk > 1) load_chunk(1, S1{});
    if (NBUF > 3 && nchunk > 2) load_chunk(2, S2{});
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));
  }
  barrier();
  int c = 0;
  // steady state: every step of a revolution loads a chunk that exists
  for (; c + 2 * NBUF - 2 < nchunk; c += NBUF) ring(c, step);
  ring(c, tail_step);
  if (c + NBUF < nchunk) ring(c + NBUF, tail_step);

  // V^{ij}[ga][gb] in FP64 (register r of lane l: row 8(r/4) + 4(l/32) + r%4, column l%32)
  const int n_v = a.n_v;
  double* Vp = a.T + (size_t)p * n_v * n_v;
  const int gb = J * TJ + wc * 32 + r32;
  if (gb < n_v) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ga = I * TV + wr * 64 + b * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
        if (ga < n_v) Vp[(size_t)ga * n_v + gb] = dV[b][r] + (double)acc[b][2][r];
      }
  }
}

// Epilogue pass over 64 x 64 tile pairs (I <= J) of the V written above; without
// STORE (energy-only passes) only the energy and norm partials are formed.
template <bool STORE>
__global__ __launch_bounds__(256) void pair_epi_bf16_kernel(PairSlicedArgs a) {
  __shared__ double scratch[272];
  const int L = xcd_block_v(blockIdx.x, a.nTP * a.n_blk_pairs);
  const int p = L / a.nTP, tp = L - p * a.nTP;
  int I, J;
  tile_pair(tp, a.nt, I, J);
  const int2 pr = a.pairs[p];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1, r32 = lane & 31, hq = lane >> 5;
  const int n_v = a.n_v;
  const double* Vp = a.T + (size_t)p * n_v * n_v;
  const int gb = J * 64 + wc * 32 + r32;
  const bool same = pr.x == pr.y;
  double dP[16], dQ[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ga = I * 64 + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
    const bool ok = ga < n_v && gb < n_v;
    // V^{ji}_{ab} = V^{ij}_{ba}; for i == j, V^{ii} is symmetric and the product
    // kernel leaves its tiles below the diagonal unwritten, so Q is read where P is
    const size_t pa = (size_t)ga * n_v + gb, qa = same ? pa : (size_t)gb * n_v + ga;
    dP[r] = ok ? Vp[pa] : 0.0;  // V^{ij}_{ab}
    dQ[r] = ok ? Vp[qa] : 0.0;
  }
  __syncthreads();  // every read of this tile pair's V precedes the T written over it
  sliced_pair_epilogue<STORE>(a, p, tp, I, J, pr.x, pr.y, dP, dQ, scratch);
}

hipError_t launch_pair_v_bf16(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (!a.T || a.n_v_pad % TV != 0) return hipErrorInvalidValue;
  constexpr int WC = kVWaveCols;
  const int nti = (a.n_v + TV - 1) / TV, ntj = (a.n_v + 32 * WC - 1) / (32 * WC);
  if ((long long)nti * ntj * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  dim3 gv(nti * ntj * n_pairs), bv(128 * WC);
  switch (ns) {
    case 2: hipLaunchKernelGGL((pair_v_bf16_kernel<2, WC, kVRing>), gv, bv, 0, st, b, nti, ntj); break;
    case 3: hipLaunchKernelGGL((pair_v_bf16_kernel<3, WC, kVRing>), gv, bv, 0, st, b, nti, ntj); break;
    case 4: hipLaunchKernelGGL((pair_v_bf16_kernel<4, WC, kVRing>), gv, bv, 0, st, b, nti, ntj); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pair_epi_bf16(const PairSlicedArgs& a, int n_pairs, bool store, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (!a.T || (long long)a.nTP * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  if (store) hipLaunchKernelGGL(pair_epi_bf16_kernel<true>, dim3(a.nTP * n_pairs), dim3(256), 0, st, b);
  else hipLaunchKernelGGL(pair_epi_bf16_kernel<false>, dim3(a.nTP * n_pairs), dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace dfpt2
