// FP64 density kernel: the virtual block of the second-order 1-RDM (Eq. A9)
// accumulated over hole pairs on FP64 MFMA.
//
// For an unordered pair {i < j} with amplitude matrix T = T^{ij} the two
// ordered pairs contribute
//     T (2T - T^T)^T + T^T (2T - T^T)   =   X1 Y1^T + X2 Y2^T
// with, for a virtual c running along the contraction,
//     X1[a][c] = T[a][c],  Y1[b][c] = 2 T[b][c] - T[c][b],
//     X2[a][c] = T[c][a],  Y2[b][c] = 2 T[c][b] - T[b][c].
// For i == j (T symmetric) the same expression is twice T T^T and gets half the
// weight.  The result is symmetric, so only tiles (A <= B) of D are formed.
//
// Workgroup = (tile pair (A, B), split s).  Split s owns a contiguous range of
// pairs and accumulates into its own slice Dpart[s]; slices are summed in a
// fixed order afterwards, so results are bitwise reproducible.  The four
// operand panels per chunk (two row panels, two column panels of T) are staged
// through LDS with a register double buffer; the Y operands are formed while
// reading fragments.
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

namespace {
constexpr int TM = 64;
constexpr int KC = 16;
constexpr int LDR = KC + 1;  // row panel stride
constexpr int LDC = TM + 1;  // column panel stride
}

template <bool VEC>
__global__ __launch_bounds__(256, 2) void density_f64_kernel(DensityKernelArgs a) {
  __shared__ double rp[2][2][TM][LDR];  // T[A, c..], T[B, c..]
  __shared__ double cp[2][2][KC][LDC];  // T[c.., A], T[c.., B]
  const int tp = blockIdx.x, split = blockIdx.y;
  int A, Bt;
  tile_pair(tp, a.nt, A, Bt);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int n_v = a.n_v;
  const int per = (a.n_pairs + a.nsplit - 1) / a.nsplit;
  const int p0 = split * per;
  const int p1 = min(a.n_pairs, p0 + per);
  const int ncc = (n_v + KC - 1) / KC;
  const int total = (p1 > p0) ? (p1 - p0) * ncc : 0;
  const int blk[2] = {A, Bt};

  double2 sr[2][2], sc[2][2];
  auto load_chunk = [&](int idx) {
    const int p = p0 + idx / ncc;
    const int c0 = (idx % ncc) * KC;
    const double* Tp = a.T + (size_t)(a.slot ? a.slot[p] : p) * n_v * n_v;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = tid + 256 * h;
        // row panel: rows blk*TM + (e>>3), columns c0 + 2*(e&7)
        {
          const int row = blk[q] * TM + (e >> 3);
          const int col = c0 + (e & 7) * 2;
          double2 v = make_double2(0.0, 0.0);
          if (row < n_v) {
            const double* src = Tp + (size_t)row * n_v + col;
            if (VEC) {
              if (col + 1 < n_v) v = *reinterpret_cast<const double2*>(src);
              else if (col < n_v) v.x = src[0];
            } else {
              if (col < n_v) v.x = src[0];
              if (col + 1 < n_v) v.y = src[1];
            }
          }
          sr[q][h] = v;
        }
        // column panel: rows c0 + (e>>5), columns blk*TM + 2*(e&31)
        {
          const int row = c0 + (e >> 5);
          const int col = blk[q] * TM + (e & 31) * 2;
          double2 v = make_double2(0.0, 0.0);
          if (row < n_v) {
            const double* src = Tp + (size_t)row * n_v + col;
            if (VEC) {
              if (col + 1 < n_v) v = *reinterpret_cast<const double2*>(src);
              else if (col < n_v) v.x = src[0];
            } else {
              if (col < n_v) v.x = src[0];
              if (col + 1 < n_v) v.y = src[1];
            }
          }
          sc[q][h] = v;
        }
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = tid + 256 * h;
        const int r = e >> 3, k = (e & 7) * 2;
        rp[buf][q][r][k] = sr[q][h].x;
        rp[buf][q][r][k + 1] = sr[q][h].y;
        const int kr = e >> 5, cc = (e & 31) * 2;
        cp[buf][q][kr][cc] = sc[q][h].x;
        cp[buf][q][kr][cc + 1] = sc[q][h].y;
      }
    }
  };

  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (d4){0.0, 0.0, 0.0, 0.0};

  const int r16 = lane & 15, kq = lane >> 4;
  if (total > 0) {
    load_chunk(0);
    store_chunk(0);
  }
  __syncthreads();
  for (int idx = 0; idx < total; ++idx) {
    const int buf = idx & 1;
    const int p = p0 + idx / ncc;
    const int2 pr = a.pairs[p];
    double wp = a.w * (pr.x == pr.y ? 0.5 : 1.0);
    if (a.pw) wp *= a.pw[p];
    const double wp2 = 2.0 * wp;
    if (idx + 1 < total) load_chunk(idx + 1);
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const int k = k4 * 4 + kq;
      const int ra0 = wr * 32 + r16, ra1 = ra0 + 16;
      const int rb0 = wc * 32 + r16, rb1 = rb0 + 16;
      const double x10 = rp[buf][0][ra0][k], x11 = rp[buf][0][ra1][k];
      const double y10 = wp2 * rp[buf][1][rb0][k] - wp * cp[buf][1][k][rb0];
      const double y11 = wp2 * rp[buf][1][rb1][k] - wp * cp[buf][1][k][rb1];
      const double x20 = cp[buf][0][k][ra0], x21 = cp[buf][0][k][ra1];
      const double y20 = wp2 * cp[buf][1][k][rb0] - wp * rp[buf][1][rb0][k];
      const double y21 = wp2 * cp[buf][1][k][rb1] - wp * rp[buf][1][rb1][k];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x10, y10, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x10, y11, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x11, y10, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x11, y11, acc[1][1], 0, 0, 0);
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x20, y20, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x20, y21, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x21, y20, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x21, y21, acc[1][1], 0, 0, 0);
    }
    if (idx + 1 < total) store_chunk(buf ^ 1);
    __syncthreads();
  }

  double* Dp = a.Dpart + (size_t)split * n_v * n_v;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ga = A * TM + wr * 32 + bi * 16 + kq + 4 * r;
      if (ga >= n_v) continue;
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int gb = Bt * TM + wc * 32 + bj * 16 + r16;
        if (gb >= n_v) continue;
        double* dst = Dp + (size_t)ga * n_v + gb;
        *dst = a.accumulate ? *dst + acc[bi][bj][r] : acc[bi][bj][r];
      }
    }
}

__global__ void density_reduce_kernel(const double* Dpart, int nsplit, int n_v, const double* diag, double* D) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (b >= n_v || a > b) return;
  const size_t off = (size_t)a * n_v + b;
  const size_t stride = (size_t)n_v * n_v;
  double v = 0.0;
  for (int s = 0; s < nsplit; ++s) v += Dpart[off + s * stride];
  if (diag && a == b) v += diag[a];
  D[off] = v;
  D[(size_t)b * n_v + a] = v;
}

hipError_t launch_density_f64(const DensityKernelArgs& a, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  dim3 grid(a.nTP, a.nsplit), block(256);
  if ((a.n_v % 2) == 0)
    hipLaunchKernelGGL(density_f64_kernel<true>, grid, block, 0, st, a);
  else
    hipLaunchKernelGGL(density_f64_kernel<false>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_density_reduce(const double* Dpart, int nsplit, int n_v, const double* diag, double* D,
                                 hipStream_t st) {
  dim3 block(256), grid((n_v + 255) / 256, n_v);
  hipLaunchKernelGGL(density_reduce_kernel, grid, block, 0, st, Dpart, nsplit, n_v, diag, D);
  return hipGetLastError();
}

}  // namespace dfpt2
