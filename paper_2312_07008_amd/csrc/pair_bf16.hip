// Split-BF16 pair kernel: V = B_i B_j^T from BF16 slices on the 32x32x16 BF16
// MFMA, with the same fused DSRG regularizer/energy epilogue as the FP64
// kernel (paper App. A, Eq. A7).
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

// Row information the split-BF16 density needs, from the amplitudes of one tile
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

template <int NS, bool STORE>
__global__ __launch_bounds__(256, 2) void pair_gemm_bf16_kernel(PairSlicedArgs a) {
  static_assert(2 * NS <= SLOTS, "slices per LDS row");
  __shared__ u4 lds0[4 * PANEL_U4];
  __shared__ u4 lds1[4 * PANEL_U4];
  __shared__ double red[2][4];
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
  const int n_v = a.n_v;

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

  // ---- epilogue (32x32x16 layout: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32)
  const double eij = a.eps_h[hi_i] + a.eps_h[hi_j];
  const double s = a.s;
  const bool offdiag = (I < J);
  const double blk_w = (offdiag ? 2.0 : 1.0) * (same ? 0.5 : 1.0) * a.e_weight;
  double* Tp = (STORE && a.T) ? a.T + (size_t)p * n_v * n_v : nullptr;
  double* Vp = (STORE && a.Vr) ? a.Vr + (size_t)p * n_v * n_v : nullptr;
  double esum = 0.0, tsum = 0.0;
  double tpv[16], tqv[16];  // amplitudes T[ga][gb], T[gb][ga] (0 outside n_v)
  const int gb = J * TM + wc * 32 + r32;
  const bool vb = gb < n_v;
  const double eb = vb ? a.eps_v[gb] : 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ga = I * TM + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
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
  if (STORE && a.tmax) density_row_info(a, p, I, J, tpv, tqv, reinterpret_cast<double*>(lds0));
  esum = wave_sum(esum);
  tsum = wave_sum(tsum);
  if (lane == 0) {
    red[0][w] = esum;
    red[1][w] = tsum;
  }
  __syncthreads();
  if (tid == 0) {
    const size_t o = (size_t)p * a.nTP + tp;
    if (a.epart) a.epart[o] = blk_w * ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
    if (a.tpart) a.tpart[o] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

hipError_t launch_pair_gemm_bf16(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if ((long long)a.nTP * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  dim3 grid(a.nTP * n_pairs), block(256);
  const bool store = a.T != nullptr || a.Vr != nullptr;
#define DFPT2_LAUNCH(NS_)                                                                          \
  if (store)                                                                                       \
    hipLaunchKernelGGL((pair_gemm_bf16_kernel<NS_, true>), grid, block, 0, st, b);                  \
  else                                                                                             \
    hipLaunchKernelGGL((pair_gemm_bf16_kernel<NS_, false>), grid, block, 0, st, b);
  switch (ns) {
    case 2: DFPT2_LAUNCH(2) break;
    case 3: DFPT2_LAUNCH(3) break;
    case 4: DFPT2_LAUNCH(4) break;
    default: return hipErrorInvalidValue;
  }
#undef DFPT2_LAUNCH
  return hipGetLastError();
}

}  // namespace dfpt2
