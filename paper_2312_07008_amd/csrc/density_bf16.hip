// Split-BF16 density kernel: the virtual block of the second-order 1-RDM
// (Eq. A9 with zero cumulants) accumulated over hole pairs from BF16 slices of
// the amplitudes, on the 32x32x16 BF16 MFMA.
//
// Per unordered pair the contribution is X1 Y1^T + X2 Y2^T (the slices of the
// rows of X1 = T, X2 = T^T, Y1 = 2T - T^T, Y2 = 2T^T - T come from
// epi_split_bf16.hip or split_t.hip).  As in the pair kernel, the slice products
// of level s + t - 1 <= NS are kept.  The operands carry one exponent per (row,
// 64-column block), so within one block of one product of one pair every
// product of a row a of X and a row b of Y is an integer multiple of one unit
// (the two rows' block scales): the level-1 and level-2 sums are exact in FP32
// over the block's 64 contraction steps and are added into FP64 at the end of
// every block (with the pair's weight); levels >= 3 are summed in FP32 per
// product.  The two products carry different units, so the contraction runs over
// X1 / Y1 first and X2 / Y2 after it, with one set of accumulators.  D is
// symmetric: only tiles on or above the diagonal are formed, and of a tile on
// the diagonal only the elements above it are written.  Diagonal elements are
// left out: the amplitude split sums them exactly in FP64 (the rows of X and Y
// there carry the same amplitudes, so the dropped slice products would not
// average out).
//
// Workgroup = (128 x 128 tile (I, J) of D, I <= J, split s): split s owns a
// contiguous range of pairs and accumulates into its own slice Dpart[s]; the
// slices are summed in a fixed order afterwards (density_reduce_kernel), so
// results are bitwise reproducible.  Eight waves, one workgroup per CU, as the
// pair product kernel (pair_bf16_v.hip): wave (wr, wc) owns rows 64 wr .. + 63
// (two 32 x 32 MFMA blocks) and columns 32 wc .. + 31; on a diagonal tile the
// two waves wholly below the diagonal only help with the loads.  A 128 x 128
// tile moves 256 rows per contraction chunk for 16384 outputs, a third fewer
// bytes per output than 128 x 64 tiles (192 rows for 8192).  Rows beyond n_v_pad
// (the last tile row when n_v_pad / 64 is odd) are loaded only there: the
// operand matrices are rows_pad rows apart, and the outputs those rows feed are
// never written.  Staging as in the pair kernel: 16-wide chunks of the two
// 128-row panels go from global memory straight into LDS (XOR-swizzled 128-byte
// rows) through a ring of four 32 KB slots; step c issues the loads of chunk
// c + 3, runs the products of chunk c, waits for its own loads of chunk c + 1
// only and closes with a barrier that carries no memory fence.  Exponent blocks
// (four chunks) line up with the ring's revolutions, so the flushes sit at fixed
// steps.  The 1-D launch is remapped so that every XCD walks a contiguous range
// of (split, tile): workgroups resident on one XCD read the same pairs' slices.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TD = 128;  // tile edge
constexpr int KC = 16;
constexpr int SLOTS = 8;
constexpr int NBUF = 4;                  // ring slots
constexpr int KB_P = TD / 8;             // kilobytes of one panel per chunk
constexpr int KB_W = 2 * KB_P / 8;       // kilobytes per wave per chunk
constexpr int BLK_CHUNKS = 64 / KC;      // chunks per exponent block of the operands
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int swz8(int r) { return (r ^ (r >> 3)) & 7; }

__device__ inline int xcd_block_d(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

// s_waitcnt immediate (gfx9 encoding): wait until at most n vector-memory
// operations of this wave are outstanding, other counters untouched
constexpr int vm_wait_imm(int n) { return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4) | (15 << 8); }
}  // namespace

template <int NS>
__global__ __launch_bounds__(512, 1) void density_bf16_kernel(DensitySlicedArgs a) {
  static_assert(2 * NS <= SLOTS, "slices per LDS row");
  static_assert(NBUF == BLK_CHUNKS, "a ring revolution is one exponent block");
  // distinct arrays per ring slot and panel, so that the compiler's alias scopes
  // tell the slots apart (a read of one slot does not wait for loads into another)
  __shared__ u4 lx0[KB_P * 64], lx1[KB_P * 64], lx2[KB_P * 64], lx3[KB_P * 64];
  __shared__ u4 ly0[KB_P * 64], ly1[KB_P * 64], ly2[KB_P * 64], ly3[KB_P * 64];
  auto slot_x = [&](auto K) __attribute__((always_inline)) -> u4* {
    if constexpr (K() == 0) return lx0;
    else if constexpr (K() == 1) return lx1;
    else if constexpr (K() == 2) return lx2;
    else return lx3;
  };
  auto slot_y = [&](auto K) __attribute__((always_inline)) -> u4* {
    if constexpr (K() == 0) return ly0;
    else if constexpr (K() == 1) return ly1;
    else if constexpr (K() == 2) return ly2;
    else return ly3;
  };
  const int nt2 = (a.nt + 1) / 2;  // 128-row tiles
  const int L = xcd_block_d(blockIdx.x, a.nTP * a.nsplit);
  const int split = L / a.nTP, td = L - split * a.nTP;
  int I, J;
  tile_pair(td, nt2, I, J);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 2, wc = w & 3;
  const bool idle = (I == J) && wr == 1 && wc < 2;  // wave-uniform: wholly below the diagonal
  const int n_v = a.n_v;
  const int p0 = (int)((long long)split * a.n_pairs / a.nsplit);  // balanced pair ranges
  const int p1 = (int)((long long)(split + 1) * a.n_pairs / a.nsplit);
  const int nblk = a.nt;              // 64-column exponent blocks per product
  const int ncc = BLK_CHUNKS * nblk;  // chunks per product
  const int total = (p1 > p0) ? (p1 - p0) * 2 * ncc : 0;  // a multiple of 8

  // kilobyte kb < KB_P of a chunk is rows 8 kb .. + 7 of the X panel (rows of
  // tile I), kilobyte KB_P + kb rows 8 kb .. + 7 of the Y panel (rows of tile J);
  // wave w moves kilobytes KB_W w .. + KB_W - 1; lane l fills physical slot l % 8
  // of row l / 8
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int row_bytes = a.n_v_pad * NS * 2;
  const size_t mat_bytes = (size_t)a.rows_pad * row_bytes;
  const char* Ts = reinterpret_cast<const char*>(a.Ts);
  const int l3 = lane >> 3, l7 = lane & 7;
  auto src_off = [&](int kb) __attribute__((always_inline)) -> uint32_t {  // kb within its panel
    const int row = 8 * kb + l3;
    const int sl = l7 ^ swz8(row);
    const int t = sl >> 1, h = sl & 1;
    return (uint32_t)(row * row_bytes + (t < NS ? t * 32 + h * 16 : 0));
  };
  // load cursor: pair lq, product lh (0: X1 Y1^T, 1: X2 Y2^T), chunk lch
  int lq = p0, lh = 0, lch = 0;
  auto load_next = [&](auto K) __attribute__((always_inline)) {  // chunk at the cursor into slot K; cursor moves on
    const char* pb = Ts + (size_t)lq * 4 * mat_bytes + (size_t)lch * (KC * NS * 2);
    const char* pX = pb + (size_t)lh * mat_bytes + (size_t)I * TD * row_bytes;
    const char* pY = pb + (size_t)(2 + lh) * mat_bytes + (size_t)J * TD * row_bytes;
#pragma unroll
    for (int m = 0; m < KB_W; ++m) {
      const int kb = KB_W * q_w + m;  // wave-uniform
      if (kb < KB_P)
        __builtin_amdgcn_global_load_lds((gbl_void*)(pX + src_off(kb)), (lds_void*)(slot_x(K) + kb * 64), 16, 0, 0);
      else
        __builtin_amdgcn_global_load_lds((gbl_void*)(pY + src_off(kb - KB_P)),
                                         (lds_void*)(slot_y(K) + (kb - KB_P) * 64), 16, 0, 0);
    }
    if (++lch == ncc) {
      lch = 0;
      lh ^= 1;
      if (lh == 0) ++lq;
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
  // per-lane u4 index of every fragment within a slot; passed through an empty asm
  // in every step, so that the compiler forms each slot's addresses at the read
  int offY[NS], offX[2][NS];
  {
    const int rowY = wc * 32 + r32, fY = swz8(rowY);
#pragma unroll
    for (int s = 0; s < NS; ++s) offY[s] = rowY * SLOTS + ((2 * s + hq) ^ fY);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int rowX = wr * 64 + b * 32 + r32, fX = swz8(rowX);
#pragma unroll
      for (int s = 0; s < NS; ++s) offX[b][s] = rowX * SLOTS + ((2 * s + hq) ^ fX);
    }
  }
  auto compute = [&](auto K) __attribute__((always_inline)) {
    if (idle) return;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      asm volatile("" : "+v"(offY[s]));
      asm volatile("" : "+v"(offX[0][s]));
      asm volatile("" : "+v"(offX[1][s]));
    }
    bf8v fb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) fb[s] = __builtin_bit_cast(bf8v, slot_y(K)[offY[s]]);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      bf8v fa[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) fa[s] = __builtin_bit_cast(bf8v, slot_x(K)[offX[b][s]]);
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int u = 0; u + s < NS; ++u) {
          const int lv = (s + u) < 2 ? (s + u) : 2;
          acc[b][lv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[u], acc[b][lv], 0, 0, 0);
        }
    }
  };
  // pair weight: one ordered pair w, halved for i == j (both orders are the same);
  // read through the constant address space, so the loads are scalar and never
  // count among the vector loads the steps wait for
  typedef __attribute__((address_space(4))) const int c_int;
  typedef __attribute__((address_space(4))) const double c_double;
  auto weight = [&](int p) __attribute__((always_inline)) {
    const c_int* pr = (const c_int*)a.pairs + 2 * (size_t)p;
    double wp = a.w * (pr[0] == pr[1] ? 0.5 : 1.0);
    if (a.pw) wp *= ((const c_double*)a.pw)[p];
    return wp;
  };
  // compute cursor: pair cq, product chalf, exponent block cblk of the chunks being computed
  int cq = p0, chalf = 0, cblk = 0;
  double wp = (total > 0) ? weight(p0) : 0.0;
  // after the last chunk of an exponent block: the exact level-1 and level-2 sums
  // go into FP64; at the end of a product also level 3+, and the cursor moves on
  auto end_block = [&]() __attribute__((always_inline)) {
    if (!idle) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          dD[b][r] += wp * ((double)acc[b][0][r] + (double)acc[b][1][r]);
          acc[b][0][r] = 0.f;
          acc[b][1][r] = 0.f;
        }
    }
    if (++cblk == nblk) {  // uniform
      cblk = 0;
      if (!idle) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            dD[b][r] += wp * (double)acc[b][2][r];
            acc[b][2][r] = 0.f;
          }
      }
      chalf ^= 1;
      if (chalf == 0) {
        ++cq;
        if (cq < p1) wp = weight(cq);
      }
    }
  };
  // the workgroup barrier without the memory fence of __syncthreads (whose
  // release waits for every outstanding load); the empty asm keeps the compiler
  // from moving memory accesses across it
  auto barrier = []() __attribute__((always_inline)) {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // step of chunk c (slot K): the loads of chunk c + 3 go into slot KL, which
  // chunk c - 1 was read from (every wave finished those reads before the last
  // barrier); the products of chunk c follow (and the flush at the end of an
  // exponent block); then each wave waits for its own loads of chunk c + 1 -- the
  // loads of chunks c + 2 and c + 3 may stay in flight -- and the barrier makes
  // every wave's part of chunk c + 1 visible.  The steady-state steps have no
  // branch around a load or a wait; the last steps run as tail steps that check
  // each load and wait for everything.
  auto step = [&](int, auto K, auto KL, auto E) __attribute__((always_inline)) {
    load_next(KL);
    compute(K);
    if constexpr (E()) end_block();
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(KB_W * (NBUF - 2)));
    barrier();
  };
  auto tail_step = [&](int c, auto K, auto KL, auto E) __attribute__((always_inline)) {
    if (c >= total) return;  // uniform
    if (c + NBUF - 1 < total) load_next(KL);
    compute(K);
    if constexpr (E()) end_block();
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));
    barrier();
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  using F = std::false_type;
  using T = std::true_type;
  // 4 steps from chunk c (c a multiple of 4): slot c % 4, one exponent block
  auto ring = [&](int c, auto&& f) __attribute__((always_inline)) {
    f(c, S0{}, S3{}, F{});
    f(c + 1, S1{}, S0{}, F{});
    f(c + 2, S2{}, S1{}, F{});
    f(c + 3, S3{}, S2{}, T{});
  };

  if (total > 0) {
    // chunks 0 .. 2 into slots 0 .. 2
    load_next(S0{});
    load_next(S1{});
    load_next(S2{});
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(KB_W * (NBUF - 2)));  // chunk 0 has landed
    barrier();
    int c = 0;
    // steady state: every step loads a chunk that exists (up to chunk c + 6)
    for (; c + 2 * NBUF - 2 < total; c += NBUF) ring(c, step);
    ring(c, tail_step);
    if (c + NBUF < total) ring(c + NBUF, tail_step);
  }

  // D tile (32x32 layout: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column
  // l%32); only elements above the diagonal are written (the reduction reads that
  // triangle; the diagonal comes from the exact FP64 sum of the amplitude split)
  if (idle) return;
  double* Dp = a.Dpart + (size_t)split * n_v * n_v;
  const int gb = J * TD + wc * 32 + r32;
  if (gb < n_v) {
    // all reads of the old tile first (rows beyond n_v read row n_v - 1 and are
    // not written back), so that they are in flight together
    if (a.accumulate) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int ga = I * TD + wr * 64 + b * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
          dD[b][r] += Dp[(size_t)min(ga, n_v - 1) * n_v + gb];
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ga = I * TD + wr * 64 + b * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
        if (ga < gb) Dp[(size_t)ga * n_v + gb] = dD[b][r];
      }
  }
}

int density_bf16_tiles(int nt) {
  const int nt2 = (nt + 1) / 2;
  return nt2 * (nt2 + 1) / 2;
}

hipError_t launch_density_bf16(const DensitySlicedArgs& a, int ns, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  // the panels of the last tile reach row 128 ceil(nt / 2) - 1
  if (a.n_v_pad != 64 * a.nt || a.rows_pad % TD != 0 || a.rows_pad < TD * ((a.nt + 1) / 2) ||
      a.nTP != density_bf16_tiles(a.nt) || (long long)a.nTP * a.nsplit > 0x7fffffffLL)
    return hipErrorInvalidValue;
  dim3 grid(a.nTP * a.nsplit), block(512);
  switch (ns) {
    case 2: hipLaunchKernelGGL(density_bf16_kernel<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(density_bf16_kernel<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(density_bf16_kernel<4>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dfpt2
