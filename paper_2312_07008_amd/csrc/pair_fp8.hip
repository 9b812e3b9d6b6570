// Split-FP8 pair kernel: V = B_i B_j^T from e4m3 slices with per-block E8M0
// scales on the 32x32x64 scaled MFMA of gfx950, with the same fused DSRG
// regularizer/energy epilogue as the FP64 kernel (paper App. A, Eq. A7).
//
// Operands come from split.hip: every 32-wide block of a row is a sum of slices
// s_t 2^(E - 4 - 5(t-1)) with |s_t| <= 16, so each slice carries about 5 bits.
// The scaled MFMA applies the block scales of both operands to every 32-wide
// K-block and sums into one FP32 accumulator per output element; the kernel keeps
// the slice products of level s + t - 1 <= NS.  Unlike the BF16 kernel the sum is
// not exact: products of differently scaled blocks meet in FP32, so V carries
// FP32 rounding (relative 2^-24 per accumulation step) on top of the slicing
// error (relative 2^-(5 NS - 1) of the block maxima).
//
// Tiling as in pair_f64.hip: one workgroup = unordered pair {i <= j} x tile pair
// (I <= J) of 64 x 64; every wave owns the same 32 x 32 block of P = V^{ij}[I,J]
// and of Q = V^{ji}[I,J].  One contraction chunk is 64 wide; an LDS row holds the
// chunk of one virtual: 16 slots of 16 bytes (slice t, lane half h, quarter q ->
// slot 4t + 2h + q), XOR-swizzled by the row's low four bits.  Panels stream from
// global memory into LDS with direct loads, double buffered (128 KB of LDS, one
// workgroup per CU).  Scale words go to registers one chunk ahead.
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 64;
constexpr int SLOTS = 16;
constexpr int PANEL_U4 = TM * SLOTS;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

__device__ inline int xcd_block8(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

__device__ inline i8v frag(const u4* buf, int panel, int row, int slot0, int f) {
  const u4 lo = buf[panel * PANEL_U4 + row * SLOTS + (slot0 ^ f)];
  const u4 hi = buf[panel * PANEL_U4 + row * SLOTS + ((slot0 + 1) ^ f)];
  i8v v;
  v[0] = (int)lo[0];
  v[1] = (int)lo[1];
  v[2] = (int)lo[2];
  v[3] = (int)lo[3];
  v[4] = (int)hi[0];
  v[5] = (int)hi[1];
  v[6] = (int)hi[2];
  v[7] = (int)hi[3];
  return v;
}
}  // namespace

template <int NS, bool STORE>
__global__ __launch_bounds__(256, 1) void pair_gemm_fp8_kernel(PairSlicedArgs a) {
  static_assert(NS >= 1 && NS <= 4, "slices per LDS row");
  __shared__ u4 lds0[4 * PANEL_U4];
  __shared__ u4 lds1[4 * PANEL_U4];
  __shared__ double red[2][4];
  const int L = xcd_block8(blockIdx.x, a.nTP * a.n_blk_pairs);
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
  const int nch = a.n_aux_pad / KC;

  // direct loads: wave w fills panel w, 16 KB per chunk = 16 loads of 4 rows x 16 slots
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int hole_w = (q_w == 0 || q_w == 3) ? hi_i : hi_j;
  const int tile_w = (q_w == 0 || q_w == 2) ? I : J;
  const bool load_w = q_w < npanel;
  const int row_bytes = a.n_aux_pad * NS;
  const char* panel = static_cast<const char*>(a.Bs) + ((size_t)hole_w * a.n_v_pad + tile_w * TM) * row_bytes;
  const int l4 = lane >> 4, l15 = lane & 15;
  auto src_off = [&](int m) -> uint32_t {
    const int r = 4 * m + l4;
    const int sl = l15 ^ (r & 15);
    const int t = sl >> 2, hq = sl & 3;
    return (uint32_t)(r * row_bytes + (t < NS ? t * 64 + hq * 16 : 0));
  };
  auto load_chunk = [&](int chunk, u4* buf) {
    if (!load_w) return;
    const char* base = panel + (size_t)chunk * (KC * NS);
#pragma unroll
    for (int m = 0; m < 16; ++m)
      __builtin_amdgcn_global_load_lds((gbl_void*)(base + src_off(m)), (lds_void*)(buf + q_w * PANEL_U4 + m * 64),
                                       16, 0, 0);
  };

  // fragment rows and scale words: A side rows of tile I (P: hole i, Q: hole j),
  // B side rows of tile J (P: hole j, Q: hole i)
  const int r32 = lane & 31, h = lane >> 5;
  const int rowA = wr * 32 + r32, rowB = wc * 32 + r32;
  const int fA = rowA & 15, fB = rowB & 15;
  auto sc_ptr = [&](int hole, int tile, int row) {
    return a.scales + ((size_t)hole * a.n_v_pad + tile * TM + row) * (size_t)nch * 2 + h;
  };
  const uint32_t* scAP = sc_ptr(hi_i, I, rowA);
  const uint32_t* scBP = sc_ptr(hi_j, J, rowB);
  const uint32_t* scAQ = sc_ptr(hi_j, I, rowA);
  const uint32_t* scBQ = sc_ptr(hi_i, J, rowB);

  f16v accP, accQ;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accP[r] = 0.f;
    accQ[r] = 0.f;
  }

  auto compute = [&](const u4* buf, uint32_t sAP, uint32_t sBP, uint32_t sAQ, uint32_t sBQ) {
    i8v fa[NS], fb[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      fa[t] = frag(buf, 0, rowA, 4 * t + 2 * h, fA);
      fb[t] = frag(buf, 1, rowB, 4 * t + 2 * h, fB);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int t = 0; t + s < NS; ++t)
        accP = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[s], fb[t], accP, 0, 0, 0, (int)((sAP >> (8 * s)) & 255u),
                                                               0, (int)((sBP >> (8 * t)) & 255u));
    if (!same) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        fa[t] = frag(buf, 2, rowA, 4 * t + 2 * h, fA);
        fb[t] = frag(buf, 3, rowB, 4 * t + 2 * h, fB);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t + s < NS; ++t)
          accQ = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[s], fb[t], accQ, 0, 0, 0,
                                                                 (int)((sAQ >> (8 * s)) & 255u), 0,
                                                                 (int)((sBQ >> (8 * t)) & 255u));
    }
  };

  uint32_t sAP = scAP[0], sBP = scBP[0], sAQ = same ? 0u : scAQ[0], sBQ = same ? 0u : scBQ[0];
  load_chunk(0, lds0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  auto step = [&](int c, u4* cur, u4* nxt) {
    uint32_t nAP = 0u, nBP = 0u, nAQ = 0u, nBQ = 0u;
    if (c + 1 < nch) {
      load_chunk(c + 1, nxt);
      nAP = scAP[2 * (c + 1)];
      nBP = scBP[2 * (c + 1)];
      if (!same) {
        nAQ = scAQ[2 * (c + 1)];
        nBQ = scBQ[2 * (c + 1)];
      }
    }
    compute(cur, sAP, sBP, sAQ, sBQ);
    sAP = nAP;
    sBP = nBP;
    sAQ = nAQ;
    sBQ = nBQ;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  int c = 0;
  for (; c + 1 < nch; c += 2) {
    step(c, lds0, lds1);
    step(c + 1, lds1, lds0);
  }
  if (c < nch) step(c, lds0, lds1);

  double dP[16], dQ[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    dP[r] = (double)accP[r];
    dQ[r] = same ? dP[r] : (double)accQ[r];
  }

  // ---- epilogue (32x32 layout: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32)
  const double eij = a.eps_h[hi_i] + a.eps_h[hi_j];
  const double s = a.s;
  const bool offdiag = (I < J);
  const double blk_wt = (offdiag ? 2.0 : 1.0) * (same ? 0.5 : 1.0) * a.e_weight;
  double* Tp = (STORE && a.T) ? a.T + (size_t)p * n_v * n_v : nullptr;
  double* Vp = (STORE && a.Vr) ? a.Vr + (size_t)p * n_v * n_v : nullptr;
  double esum = 0.0, tsum = 0.0;
  const int gb = J * TM + wc * 32 + r32;
  const bool vb = gb < n_v;
  const double eb = vb ? a.eps_v[gb] : 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ga = I * TM + wr * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
    if (!(vb && ga < n_v)) continue;
    const double dl = eij - a.eps_v[ga] - eb;
    const double x = exp(-s * dl * dl);
    const double g1 = (dl != 0.0) ? (1.0 - x) / dl : 0.0;
    double vp = dP[r], vq = dQ[r];
    if (same && ga == gb) vp = vq = a.norm2[(size_t)hi_i * n_v + ga];  // exact ||B_ia||^2
    const double tp_ = vp * g1, tq_ = vq * g1;
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
  esum = wave_sum(esum);
  tsum = wave_sum(tsum);
  if (lane == 0) {
    red[0][w] = esum;
    red[1][w] = tsum;
  }
  __syncthreads();
  if (tid == 0) {
    const size_t o = (size_t)p * a.nTP + tp;
    if (a.epart) a.epart[o] = blk_wt * ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
    if (a.tpart) a.tpart[o] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

hipError_t launch_pair_gemm_fp8(const PairSlicedArgs& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if ((long long)a.nTP * n_pairs > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.n_aux_pad % KC != 0 || a.n_v_pad % TM != 0) return hipErrorInvalidValue;
  PairSlicedArgs b = a;
  b.n_blk_pairs = n_pairs;
  dim3 grid(a.nTP * n_pairs), block(256);
  const bool store = a.T != nullptr || a.Vr != nullptr;
#define DFPT2_LAUNCH(NS_)                                                                          \
  if (store)                                                                                       \
    hipLaunchKernelGGL((pair_gemm_fp8_kernel<NS_, true>), grid, block, 0, st, b);                  \
  else                                                                                             \
    hipLaunchKernelGGL((pair_gemm_fp8_kernel<NS_, false>), grid, block, 0, st, b);
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
