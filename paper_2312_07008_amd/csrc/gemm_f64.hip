// Batched FP64 GEMM on the 16x16x4 FP64 MFMA, used by the NO transform and
// recanonicalization (Sec. 2), the natural auxiliary functions, the
// particle-particle ladder and the active-particle density terms:
//     C[b] = alpha op(A[b]) op(B[b]) + beta C[b],   op(A) M x K, op(B) K x N.
//
// One workgroup computes a 128 x 128 tile of C; its four waves own 64 x 64
// quadrants, 4 x 4 MFMA blocks of 16 x 16 (64 FP64 accumulators per lane), so
// each 16-deep contraction chunk is 64 MFMAs per wave (~4000 cycles) against
// 2 x 16 KB of operands.  The next chunk is fetched into registers (eight
// doubles of each operand per thread, consecutive lanes on consecutive
// addresses of the contiguous dimension) while the current one is multiplied
// out of LDS, then written to the other LDS buffer: one barrier per chunk, and
// the global-load latency hides behind the MFMA work of the chunk.  LDS holds
// both operands k-major ([k][m] and [k][n]) with rows padded to 144 doubles,
// so the 16 lanes of one k row and the 16 of the next read disjoint banks.
// Out-of-range rows, columns and contraction indices read as zero.
#include "common.h"
#include "host.h"

namespace dfpt2 {

namespace {

struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int lda, ldb, ldc;
  long long sA, sB, sC;
  double alpha, beta;
};

constexpr int GT = 128;       // tile edge (M and N)
constexpr int GK = 16;        // contraction chunk
constexpr int LDP = GT + 16;  // padded LDS row (doubles)
constexpr int PER = GT * GK / 256;  // staged doubles per thread and operand

// element r of this thread's share of a chunk: (row of the tile, k of the chunk)
template <bool KCONTIG>
__device__ inline void stage_index(int e, int& row, int& k) {
  if (KCONTIG) {  // the operand's k runs contiguously in memory: lanes along k
    row = e / GK;
    k = e - row * GK;
  } else {  // the tile's rows run contiguously: lanes along the rows
    k = e / GT;
    row = e - k * GT;
  }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmArgs g) {
  __shared__ double As[2][GK][LDP];
  __shared__ double Bs[2][GK][LDP];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const double* A = g.A + b * g.sA;
  const double* Bm = g.B + b * g.sB;
  double* C = g.C + b * g.sC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1, r16 = lane & 15, kq = lane >> 4;

  // A: op(A)[m][k] is A[m][k] (k contiguous) or, transposed, A[k][m] (m contiguous)
  // B: op(B)[k][n] is B[k][n] (n contiguous) or, transposed, B[n][k] (k contiguous)
  double ra[PER], rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      int row, k;
      stage_index<!TA>(tid + 256 * r, row, k);
      const int gm = m0 + row, gk = k0 + k;
      ra[r] = (gm < g.M && gk < g.K) ? (TA ? A[(size_t)gk * g.lda + gm] : A[(size_t)gm * g.lda + gk]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      int col, k;
      stage_index<TB>(tid + 256 * r, col, k);
      const int gn = n0 + col, gk = k0 + k;
      rb[r] = (gn < g.N && gk < g.K) ? (TB ? Bm[(size_t)gn * g.ldb + gk] : Bm[(size_t)gk * g.ldb + gn]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      int row, k;
      stage_index<!TA>(tid + 256 * r, row, k);
      As[buf][k][row] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      int col, k;
      stage_index<TB>(tid + 256 * r, col, k);
      Bs[buf][k][col] = rb[r];
    }
  };

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    const bool more = k0 + GK < g.K;
    if (more) load(k0 + GK);
#pragma unroll
    for (int k4 = 0; k4 < GK / 4; ++k4) {
      const int k = k4 * 4 + kq;
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][k][wr * 64 + i * 16 + r16];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[buf][k][wc * 64 + j * 16 + r16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // register r of lane l holds row l / 16 + 4 r and column l % 16 of a 16 x 16 block
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wr * 64 + i * 16 + kq + 4 * r;
      if (gm >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gn = n0 + wc * 64 + j * 16 + r16;
        if (gn >= g.N) continue;
        double* dst = C + (size_t)gm * g.ldc + gn;
        const double v = g.alpha * acc[i][j][r];
        *dst = (g.beta != 0.0) ? v + g.beta * *dst : v;
      }
    }
}

}  // namespace

hipError_t gemm_f64(const double* A, int lda, long long sA, int transA, const double* B, int ldb, long long sB,
                    int transB, double* C, int ldc, long long sC, int M, int N, int K, int batch, double alpha,
                    double beta, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535 || (M + GT - 1) / GT > 65535) return hipErrorInvalidValue;
  GemmArgs g{A, B, C, M, N, K, lda, ldb, ldc, sA, sB, sC, alpha, beta};
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch);  // K <= 0 leaves C = beta C
  if (transA) {
    if (transB) hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, dim3(256), 0, st, g);
    else hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, dim3(256), 0, st, g);
  } else {
    if (transB) hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, dim3(256), 0, st, g);
    else hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, dim3(256), 0, st, g);
  }
  return hipGetLastError();
}

}  // namespace dfpt2
