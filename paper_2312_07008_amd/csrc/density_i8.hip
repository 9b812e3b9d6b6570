// INT8-digit density kernel: the virtual block of the second-order 1-RDM
// (Eq. A9 with zero cumulants) accumulated over hole pairs from balanced
// base-256 digits of the amplitudes (split_t.hip) on the 32x32x32 INT8 MFMA.
//
// Per unordered pair the contribution is X1 Y1^T + X2 Y2^T (X1 = T, X2 = T^T,
// Y1 = 2T - T^T, Y2 = 2T^T - T; density_bf16.hip).  With NS digits per row the
// kernel keeps the digit products of levels s + t < NS and sums each level of
// each of the two products in its own INT32 accumulator over the pair's whole
// contraction (a level has at most NS - 1 products of 2^14 and two of 2^13 per
// index, so the sums are exact for (NS - 1) 2^14 n_v_pad < 2^31).  At the end
// of every pair the levels are combined in FP64 (Horner in 2^-8), scaled by the
// two rows' exponents and the pair's weight, and added to the workgroup's tile of
// its split's FP64 partial sum in memory (register layout of a 32x32 MFMA
// accumulator: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32).
// Diagonal elements are left out: split_t.hip sums them exactly in FP64.
//
// Workgroup = (tile pair (A <= B), split s) over a contiguous range of pairs, as
// in density_bf16.hip; staging as in pair_i8.hip (chunk-major digits, 2 NS direct
// 16-byte loads per 64-row panel and chunk, rotated or XOR-swizzled LDS rows,
// double buffered).
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 32;
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void gbl_void;

template <int NS>
__device__ inline int phys_slot_d(int r, int j) {
  if constexpr (NS == 4) {
    return j ^ ((r ^ (r >> 3)) & 7);
  } else {
    const int p = j + NS * (((r >> 2) ^ (r >> 3)) & 1);
    return p >= 2 * NS ? p - 2 * NS : p;
  }
}
template <int NS>
__device__ inline int logical_slot_d(int r, int p) {
  if constexpr (NS == 4) {
    return p ^ ((r ^ (r >> 3)) & 7);
  } else {
    const int j = p - NS * (((r >> 2) ^ (r >> 3)) & 1);
    return j < 0 ? j + 2 * NS : j;
  }
}

__device__ inline int xcd_block_di(int h, int nblk) {
  const int x = h & 7, k = h >> 3, q = nblk >> 3, rem = nblk & 7;
  return (x < rem) ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}
}  // namespace

template <int NS>
__global__ __launch_bounds__(256, 2) void density_i8_kernel(DensityDigitArgs a) {
  constexpr int SLOTS = 2 * NS;
  constexpr int PANEL_U4 = TM * SLOTS;
  constexpr int ROWB = 32 * NS;
  __shared__ u4 lds[2][4 * PANEL_U4];
  const int L = xcd_block_di(blockIdx.x, a.nTP * a.nsplit);
  const int split = L / a.nTP, tp = L - split * a.nTP;
  int A, Bt;
  tile_pair(tp, a.nt, A, Bt);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int n_v = a.n_v, n_v_pad = a.n_v_pad;
  const int p0 = (int)((long long)split * a.n_pairs / a.nsplit);
  const int p1 = (int)((long long)(split + 1) * a.n_pairs / a.nsplit);
  const int nck = n_v_pad / KC;
  const int total = (p1 > p0) ? (p1 - p0) * nck : 0;

  // wave w fills panel w: 0 = X1 rows A, 1 = Y1 rows B, 2 = X2 rows A, 3 = Y2 rows B
  const int q_w = __builtin_amdgcn_readfirstlane(w);
  const int mat_w = (q_w == 0) ? 0 : (q_w == 1) ? 2 : (q_w == 2) ? 1 : 3;
  const int tile_w = (q_w == 0 || q_w == 2) ? A : Bt;
  const size_t chunk_stride = (size_t)n_v_pad * ROWB;
  auto src_off = [&](int m) -> uint32_t {
    const int u = 64 * m + lane, r = u / SLOTS, ps = u - r * SLOTS;
    return (uint32_t)(r * ROWB + 16 * logical_slot_d<NS>(r, ps));
  };
  auto load_chunk = [&](int idx, u4* buf) {
    const int p = p0 + idx / nck, ch = idx - (idx / nck) * nck;
    const char* base = reinterpret_cast<const char*>(a.Ts) +
                       (((size_t)p * 4 + mat_w) * nck + ch) * chunk_stride + (size_t)tile_w * TM * ROWB;
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
  // the FP64 tile sum lives in this split's slice of Dpart (owned by this
  // workgroup): added to once per pair, which frees 32 registers per lane
  double* Dp = a.Dpart + (size_t)split * n_v * n_v;
  bool first = !a.accumulate;

  const int r32 = lane & 31, hq = lane >> 5;
  const int rowA = wr * 32 + r32, rowB = wc * 32 + r32;
  auto offA = [&](int t) { return rowA * SLOTS + phys_slot_d<NS>(rowA, 2 * t + hq); };
  auto offB = [&](int t) { return rowB * SLOTS + phys_slot_d<NS>(rowB, 2 * t + hq); };

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
  };
  // end of pair p: levels -> FP64, row scales of X1/Y1 and X2/Y2, pair weight;
  // the diagonal is left out (the exact FP64 sum of split_t.hip)
  const int gb = Bt * TM + wc * 32 + r32;
  auto flush = [&](int p) {
    // row stride taken through an opaque move, so that the sixteen destination
    // addresses are formed here rather than kept live (spilled) across the loop
    int nvs;
    asm volatile("s_mov_b32 %0, %1" : "=s"(nvs) : "s"(n_v));
    const int2 pr = a.pairs[p];
    double wp = a.w * (pr.x == pr.y ? 0.5 : 1.0);
    if (a.pw) wp *= a.pw[p];
    const int* ex = a.rexp + (size_t)p * 4 * n_v_pad;
    const int eY1 = ex[2 * n_v_pad + gb], eY2 = ex[3 * n_v_pad + gb];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ga = A * TM + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
      double vp = (double)accP[NS - 1][r], vq = (double)accQ[NS - 1][r];
#pragma unroll
      for (int l = NS - 2; l >= 0; --l) {
        vp = vp * 0.00390625 + (double)accP[l][r];
        vq = vq * 0.00390625 + (double)accQ[l][r];
      }
      const double v = wp * (ldexp(vp, ex[ga] + eY1) + ldexp(vq, ex[n_v_pad + ga] + eY2));
      if (gb < nvs && ga < nvs && ga != gb) {
        double* dst = Dp + (size_t)ga * nvs + gb;
        *dst = first ? v : *dst + v;
      }
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        accP[l][r] = 0;
        accQ[l][r] = 0;
      }
    }
    first = false;
  };
  // chunk idx + 1 (possibly the next pair's first) streams into one buffer while
  // chunk idx is multiplied out of the other; the pair's sums are flushed after
  // its last chunk
  int cp = p0, cch = 0;
  auto step = [&](int idx, u4* cur, u4* nxt) {
    if (idx + 1 < total) load_chunk(idx + 1, nxt);
    compute(cur);
    if (++cch == nck) {
      flush(cp);
      cch = 0;
      ++cp;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  if (total > 0) {
    load_chunk(0, lds[0]);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    int idx = 0;
    for (; idx + 1 < total; idx += 2) {
      step(idx, lds[0], lds[1]);
      step(idx + 1, lds[1], lds[0]);
    }
    if (idx < total) step(idx, lds[0], lds[1]);
  }

  // a split without pairs still owns its tile (overwrite mode: zeros)
  if (total == 0 && first && gb < n_v) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ga = A * TM + wr * 32 + 8 * (r >> 2) + 4 * hq + (r & 3);
      if (ga < n_v && ga != gb) Dp[(size_t)ga * n_v + gb] = 0.0;
    }
  }
}

hipError_t launch_density_i8(const DensityDigitArgs& a, int ns, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  // exact INT32 level sums: at most (ns - 1) 2^14 per contraction index
  if (a.n_v_pad % TM != 0 || (long long)(ns - 1) * 16384 * a.n_v_pad >= 0x7fffffffLL ||
      (long long)a.nTP * a.nsplit > 0x7fffffffLL || !a.rexp)
    return hipErrorInvalidValue;
  dim3 grid(a.nTP * a.nsplit), block(256);
  switch (ns) {
    case 2: hipLaunchKernelGGL(density_i8_kernel<2>, grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL(density_i8_kernel<3>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(density_i8_kernel<4>, grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL(density_i8_kernel<5>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dfpt2
