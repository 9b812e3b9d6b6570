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
// Panels are staged in LDS in 16-wide contraction chunks, double buffered;
// the two 8-element halves of each row are XOR-swizzled by bit 2 of the row
// so that 128-bit fragment reads of eight consecutive rows hit distinct banks.
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 16;
constexpr int FLUSH_CHUNKS = 128 / KC;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__device__ inline int swz(int row, int half) { return half ^ ((row >> 2) & 1); }
}  // namespace

template <int NS, bool STORE>
__global__ __launch_bounds__(256, 2) void pair_gemm_bf16_kernel(PairBf16Args a) {
  __shared__ u4 lds[2][4][NS][TM][2];
  __shared__ double red[2][4];
  const int tp = blockIdx.x;
  const int p = blockIdx.y;
  int I, J;
  tile_pair(tp, a.nt, I, J);
  const int2 pr = a.pairs[p];
  const int hi_i = pr.x, hi_j = pr.y;
  const bool same = (hi_i == hi_j);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int n_v = a.n_v, ldk = a.n_aux_pad;
  const int npanel = same ? 2 : 4;
  const int hole_of[4] = {hi_i, hi_j, hi_j, hi_i};
  const int blk_of[4] = {I, J, I, J};

  // staging: units u = tid + 256 m, m < 2 NS; unit -> (panel q, row r, slice t, half h)
  // with (t, h) fastest, so 2 NS consecutive lanes read one row's contiguous chunk
  // of 32 NS bytes (chunk-interleaved slice layout, see split.hip).
  u4 stage[2 * NS];
  const size_t row_stride = (size_t)ldk * NS;  // bf16 elements per row
  auto load_chunk = [&](int chunk) {
#pragma unroll
    for (int m = 0; m < 2 * NS; ++m) {
      const int u = tid + 256 * m;
      const int th = u % (2 * NS), rq = u / (2 * NS);
      const int r = rq & 63, q = rq >> 6;
      if (q < npanel) {
        const __bf16* src = a.Bs + ((size_t)hole_of[q] * a.n_v_pad + blk_of[q] * TM + r) * row_stride +
                            (size_t)chunk * (KC * NS) + th * 8;
        stage[m] = *reinterpret_cast<const u4*>(src);
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int m = 0; m < 2 * NS; ++m) {
      const int u = tid + 256 * m;
      const int th = u % (2 * NS), rq = u / (2 * NS);
      const int r = rq & 63, q = rq >> 6;
      const int t = th >> 1, h = th & 1;
      if (q < npanel) lds[buf][q][t][r][swz(r, h)] = stage[m];
    }
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

  const int nchunk = ldk / KC;
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  const int r32 = lane & 31, hq = lane >> 5;
  const int rowA = wr * 32 + r32, rowB = wc * 32 + r32;
  const int hA = swz(rowA, hq), hB = swz(rowB, hq);
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) load_chunk(c + 1);
    bf8v fa[NS], fb[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      fa[t] = __builtin_bit_cast(bf8v, lds[buf][0][t][rowA][hA]);
      fb[t] = __builtin_bit_cast(bf8v, lds[buf][1][t][rowB][hB]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int t = 0; t + s < NS; ++t) {
        const int L = (s + t) < 2 ? (s + t) : 2;
        accP[L] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[t], accP[L], 0, 0, 0);
      }
    if (!same) {
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        fa[t] = __builtin_bit_cast(bf8v, lds[buf][2][t][rowA][hA]);
        fb[t] = __builtin_bit_cast(bf8v, lds[buf][3][t][rowB][hB]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t + s < NS; ++t) {
          const int L = (s + t) < 2 ? (s + t) : 2;
          accQ[L] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[t], accQ[L], 0, 0, 0);
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
    if (c + 1 < nchunk) store_chunk(buf ^ 1);
    __syncthreads();
  }
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
  const int gb = J * TM + wc * 32 + r32;
  const bool vb = gb < n_v;
  const double eb = vb ? a.eps_v[gb] : 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ga = I * TM + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
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
    if (a.epart) a.epart[o] = blk_w * ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
    if (a.tpart) a.tpart[o] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

hipError_t launch_pair_gemm_bf16(const PairBf16Args& a, int ns, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  dim3 grid(a.nTP, n_pairs), block(256);
  const bool store = a.T != nullptr || a.Vr != nullptr;
#define DFPT2_LAUNCH(NS_)                                                                          \
  if (store)                                                                                       \
    hipLaunchKernelGGL((pair_gemm_bf16_kernel<NS_, true>), grid, block, 0, st, a);                 \
  else                                                                                             \
    hipLaunchKernelGGL((pair_gemm_bf16_kernel<NS_, false>), grid, block, 0, st, a);
  switch (ns) {
    case 2: DFPT2_LAUNCH(2) break;
    case 3: DFPT2_LAUNCH(3) break;
    case 4: DFPT2_LAUNCH(4) break;
    case 5: DFPT2_LAUNCH(5) break;
    default: return hipErrorInvalidValue;
  }
#undef DFPT2_LAUNCH
  return hipGetLastError();
}

}  // namespace dfpt2
