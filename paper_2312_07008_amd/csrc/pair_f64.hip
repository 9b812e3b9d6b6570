// FP64 pair kernel: V = B_i B_j^T on FP64 MFMA with the DSRG regularizer and
// the PT2 energy fused into the epilogue (paper App. A, Eq. A7).
//
// One workgroup owns an unordered hole pair {i <= j} and a 64 x 64 tile pair
// (I <= J) of virtual row/column blocks.  It computes, in the same register
// layout,
//     P = V^{ij}[I, J] = B_i[I] B_j[J]^T      and     Q = V^{ji}[I, J] = B_j[I] B_i[J]^T,
// so that element (a, b) of Q is V^{ij}_{ba}: the exchange partner needed by
// 2 t^{ij}_{ab} - t^{ij}_{ba} sits in the same lane and register as P_ab.
// For i == j the integrals are symmetric, Q = P and the second product is skipped.
//
// Epilogue, per element (a in I, b in J):
//   Delta = eps_i + eps_j - eps_a - eps_b,  x = exp(-s Delta^2)
//   T_P = P (1 - x)/Delta,  T_Q = Q (1 - x)/Delta             (Eq. A7)
//   energy  += w (1 - x^2)/Delta (2 P^2 + 2 Q^2 - 2 P Q)       (both ordered pairs)
//   ||T||^2 += T_P^2 (+ T_Q^2 off the diagonal tile)
// and the amplitudes of the unordered pair are stored as the full matrix
// T^{ij}: T_P at [a][b] and, for I < J, T_Q at the mirrored position [b][a]
// (T^{ij}_{ba} = T^{ji}_{ab}).  Optionally the renormalized integrals
// Vr = V (1 + x) are stored the same way (used when active holes are rotated).
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;        // tile edge
constexpr int KC = 16;        // aux chunk per pipeline stage
constexpr int LDK = KC + 1;   // padded LDS row (doubles)
}

// STORE = false: energy-only variant (kept-space pass) that writes no amplitudes.
template <bool VEC, bool STORE>
__global__ __launch_bounds__(256, 2) void pair_gemm_f64_kernel(PairKernelArgs a) {
  __shared__ double lds[2][4][TM][LDK];
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
  const int n_v = a.n_v, n_aux = a.n_aux;

  // panel sources: 0 = B_i rows I, 1 = B_j rows J, 2 = B_j rows I, 3 = B_i rows J
  const int hole_of[4] = {hi_i, hi_j, hi_j, hi_i};
  const int blk_of[4] = {I, J, I, J};
  const int npanel = same ? 2 : 4;

  // register staging of the next chunk: 4 panels x 2 double2 per thread
  double2 stage[4][2];

  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q >= npanel) break;
      const double* base = a.B + (size_t)hole_of[q] * n_v * n_aux;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = tid + 256 * h;  // 0..511
        const int row = e >> 3;
        const int kk = (e & 7) * 2;
        const int grow = blk_of[q] * TM + row;
        const int gk = k0 + kk;
        double2 v = make_double2(0.0, 0.0);
        if (grow < n_v) {
          const double* src = base + (size_t)grow * n_aux + gk;
          if (VEC) {
            if (gk + 1 < n_aux) v = *reinterpret_cast<const double2*>(src);
            else if (gk < n_aux) v.x = src[0];
          } else {
            if (gk < n_aux) v.x = src[0];
            if (gk + 1 < n_aux) v.y = src[1];
          }
        }
        stage[q][h] = v;
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q >= npanel) break;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = tid + 256 * h;
        const int row = e >> 3;
        const int kk = (e & 7) * 2;
        lds[buf][q][row][kk] = stage[q][h].x;
        lds[buf][q][row][kk + 1] = stage[q][h].y;
      }
    }
  };

  d4 P[2][2], Q[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      P[x][y] = (d4){0.0, 0.0, 0.0, 0.0};
      Q[x][y] = (d4){0.0, 0.0, 0.0, 0.0};
    }

  const int nchunk = (n_aux + KC - 1) / KC;
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  const int r16 = lane & 15, kq = lane >> 4;
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) load_chunk((c + 1) * KC);
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const int k = k4 * 4 + kq;
      const double a0 = lds[buf][0][wr * 32 + r16][k];
      const double a1 = lds[buf][0][wr * 32 + 16 + r16][k];
      const double b0 = lds[buf][1][wc * 32 + r16][k];
      const double b1 = lds[buf][1][wc * 32 + 16 + r16][k];
      P[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, P[0][0], 0, 0, 0);
      P[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, P[0][1], 0, 0, 0);
      P[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, P[1][0], 0, 0, 0);
      P[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, P[1][1], 0, 0, 0);
      if (!same) {
        const double c0 = lds[buf][2][wr * 32 + r16][k];
        const double c1 = lds[buf][2][wr * 32 + 16 + r16][k];
        const double d0 = lds[buf][3][wc * 32 + r16][k];
        const double d1 = lds[buf][3][wc * 32 + 16 + r16][k];
        Q[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(c0, d0, Q[0][0], 0, 0, 0);
        Q[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(c0, d1, Q[0][1], 0, 0, 0);
        Q[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(c1, d0, Q[1][0], 0, 0, 0);
        Q[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(c1, d1, Q[1][1], 0, 0, 0);
      }
    }
    if (c + 1 < nchunk) store_chunk(buf ^ 1);
    __syncthreads();
  }
  if (same) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) Q[x][y] = P[x][y];
  }

  // ---- epilogue
  const double ei = a.eps_h[hi_i], ej = a.eps_h[hi_j];
  const double eij = ei + ej;
  const double s = a.s;
  const bool offdiag = (I < J);
  const double blk_w = (offdiag ? 2.0 : 1.0) * (same ? 0.5 : 1.0) * a.e_weight;
  double* Tp = (STORE && a.T) ? a.T + (size_t)p * n_v * n_v : nullptr;
  double* Vp = (STORE && a.Vr) ? a.Vr + (size_t)p * n_v * n_v : nullptr;
  double esum = 0.0, tsum = 0.0;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ga = I * TM + wr * 32 + bi * 16 + kq + 4 * r;
      const bool va = ga < n_v;
      const double ea = va ? a.eps_v[ga] : 0.0;
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int gb = J * TM + wc * 32 + bj * 16 + r16;
        const bool vb = gb < n_v;
        if (!(va && vb)) continue;
        const double eb = a.eps_v[gb];
        const double dl = eij - ea - eb;
        const double x = exp(-s * dl * dl);
        const double g1 = (dl != 0.0) ? (1.0 - x) / dl : 0.0;
        const double vp = P[bi][bj][r], vq = Q[bi][bj][r];
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

hipError_t launch_pair_gemm_f64(const PairKernelArgs& a, int n_pairs, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  dim3 grid(a.nTP, n_pairs), block(256);
  const bool vec = (a.n_aux % 2) == 0;
  const bool store = (a.T != nullptr) || (a.Vr != nullptr);
  if (vec && store)
    hipLaunchKernelGGL((pair_gemm_f64_kernel<true, true>), grid, block, 0, st, a);
  else if (vec)
    hipLaunchKernelGGL((pair_gemm_f64_kernel<true, false>), grid, block, 0, st, a);
  else if (store)
    hipLaunchKernelGGL((pair_gemm_f64_kernel<false, true>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((pair_gemm_f64_kernel<false, false>), grid, block, 0, st, a);
  return hipGetLastError();
}

}  // namespace dfpt2
