// Natural orbitals, truncation, recanonicalization and the additive PT2
// correction (paper Sec. 2: Eqs. 8-11), plus a batched FP64 MFMA GEMM for the
// basis transformations.
#include <cmath>
#include <cfloat>

#include "../../include/dfpt2.h"
#include "common.h"
#include "eigh.h"
#include "host.h"
#include "kernels.h"

namespace dfpt2 {

namespace {

// ------------------------------------------------------------- truncation
// Single thread: cumulative-occupation threshold of Eq. 10 on descending
// occupations, margins, and the anchored near-degeneracy widening.
// N' from the descending occupations by one of the truncation rules (include/dfpt2.h,
// dfpt2_trunc_rule), then the optional near-degeneracy widening (Sec. 2, after
// Eq. 10, anchored at the smallest kept occupation).  Margins: for the cumulative
// rule (p_o - c(N'-1), c(N') - p_o) as fractions of the total occupation; for the
// cutoff rule (n[N'-1] - n_kappa, n_kappa - n[N']); otherwise the occupations
// either side of the cut, (n[N'-1], n[N']).  Missing neighbours give +inf.
__global__ void rule_threshold_kernel(const double* occ, int n, int rule, double param, double degen,
                                      int64_t* n_kept, double* margins, int* flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int bad = 0;
  double total = 0.0;
  for (int k = 0; k < n; ++k) {
    if (!isfinite(occ[k])) bad = 1;
    total += occ[k];
  }
  const double inf = __builtin_huge_val();
  int kept = n;
  if (rule == DFPT2_TRUNC_CUMULATIVE) {
    const double target = param * total;
    double c = 0.0, cprev = 0.0;
    int idx = n - 1;
    for (int k = 0; k < n; ++k) {
      cprev = c;
      c += occ[k];
      if (c >= target) {
        idx = k;
        break;
      }
    }
    kept = idx + 1;
    margins[0] = param - (idx >= 1 ? cprev / total : 0.0);
    margins[1] = c / total - param;
  } else {
    if (rule == DFPT2_TRUNC_FRACTION) {
      kept = (int)ceil(param * n - 1e-9);
      if (kept > n) kept = n;
    } else if (rule == DFPT2_TRUNC_CUTOFF) {
      kept = 0;
      while (kept < n && occ[kept] >= param) ++kept;
    } else {
      kept = (int)param;
    }
    const double lo = kept >= 1 ? occ[kept - 1] : inf, hi = kept < n ? occ[kept] : inf;
    margins[0] = rule == DFPT2_TRUNC_CUTOFF ? (kept >= 1 ? lo - param : inf) : lo;
    margins[1] = rule == DFPT2_TRUNC_CUTOFF ? (kept < n ? param - hi : inf) : hi;
  }
  if (degen > 0.0 && kept >= 1) {
    const double last = occ[kept - 1];
    while (kept < n && (last - occ[kept]) < degen * last) ++kept;
  }
  *n_kept = kept;
  *flag = bad;
}

// ------------------------------------------------------------- batched GEMM
// C[b] = alpha * op(A[b]) op(B[b]) (+ beta C[b]); op(A) is M x K, op(B) is K x N.
struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int lda, ldb, ldc;
  long long sA, sB, sC;
  int transA, transB;
  double alpha, beta;
};

constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
  __shared__ double As[GT][GK + 1];
  __shared__ double Bs[GK][GT + 1];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const double* A = g.A + b * g.sA;
  const double* Bm = g.B + b * g.sB;
  double* C = g.C + b * g.sC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1, r16 = lane & 15, kq = lane >> 4;
  d4 acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc[x][y] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      int mm, kk;
      if (g.transA) {  // A stored K x M: read along m
        kk = e / GT;
        mm = e % GT;
      } else {
        mm = e / GK;
        kk = e % GK;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < g.M && gk < g.K) v = g.transA ? A[(size_t)gk * g.lda + gm] : A[(size_t)gm * g.lda + gk];
      As[mm][kk] = v;
    }
    for (int e = tid; e < GT * GK; e += 256) {
      int nn, kk;
      if (g.transB) {  // B stored N x K: read along k
        nn = e / GK;
        kk = e % GK;
      } else {
        kk = e / GT;
        nn = e % GT;
      }
      const int gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < g.N && gk < g.K) v = g.transB ? Bm[(size_t)gn * g.ldb + gk] : Bm[(size_t)gk * g.ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < GK / 4; ++k4) {
      const int k = k4 * 4 + kq;
      const double a0 = As[wr * 32 + r16][k], a1 = As[wr * 32 + 16 + r16][k];
      const double b0 = Bs[k][wc * 32 + r16], b1 = Bs[k][wc * 32 + 16 + r16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int bi = 0; bi < 2; ++bi)
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wr * 32 + bi * 16 + kq + 4 * r;
      if (gm >= g.M) continue;
      for (int bj = 0; bj < 2; ++bj) {
        const int gn = n0 + wc * 32 + bj * 16 + r16;
        if (gn >= g.N) continue;
        double* dst = C + (size_t)gm * g.ldc + gn;
        const double v = g.alpha * acc[bi][bj][r];
        *dst = (g.beta != 0.0) ? v + g.beta * *dst : v;
      }
    }
}

}  // namespace

hipError_t gemm_f64(const double* A, int lda, long long sA, int transA, const double* B, int ldb, long long sB,
                    int transB, double* C, int ldc, long long sC, int M, int N, int K, int batch, double alpha,
                    double beta, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  GemmArgs g{A, B, C, M, N, K, lda, ldb, ldc, sA, sB, sC, transA, transB, alpha, beta};
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int fno_truncate_workspace_size(int64_t n_vir, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  if (n_vir < 1 || n_vir > kEighMaxN) return fail(DFPT2_ERR_INVALID_ARG, "n_vir outside [1, %d]", kEighMaxN);
  *bytes = eigh_workspace_bytes((int)n_vir) + 512;
  return DFPT2_OK;
}

int dfpt2_eigh_sym(const double* A, int64_t n, double* w, double* Z, void* workspace, size_t ws_bytes,
                   dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!A || !w || !Z || !workspace) return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (n < 1 || n > kEighMaxN) return fail(DFPT2_ERR_INVALID_ARG, "n outside [1, %d]", kEighMaxN);
  if (ws_bytes < eigh_workspace_bytes((int)n))
    return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, eigh_workspace_bytes((int)n));
  return eigh_run(A, (int)n, w, Z, static_cast<char*>(workspace), ws_bytes, reinterpret_cast<hipStream_t>(stream), 0);
}

static int truncate_impl(const double* D_vv, int64_t n_vir, int rule, double param, double degen_rel_tol,
                         double* occ, double* no_vecs, int64_t* n_kept, double* margins, void* workspace,
                         size_t ws_bytes, dfpt2_stream_t stream) {
  if (!D_vv || !occ || !no_vecs || !n_kept || !workspace) return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (n_vir < 1 || n_vir > kEighMaxN) return fail(DFPT2_ERR_INVALID_ARG, "n_vir outside [1, %d]", kEighMaxN);
  if (!std::isfinite(param)) return fail(DFPT2_ERR_INVALID_ARG, "rule parameter must be finite");
  switch (rule) {
    case DFPT2_TRUNC_CUMULATIVE:
      if (!(param > 0.0 && param <= 1.0)) return fail(DFPT2_ERR_INVALID_ARG, "p_o must lie in (0, 1]");
      break;
    case DFPT2_TRUNC_FRACTION:
      if (!(param > 0.0 && param <= 1.0)) return fail(DFPT2_ERR_INVALID_ARG, "p_v must lie in (0, 1]");
      break;
    case DFPT2_TRUNC_CUTOFF:
      break;
    case DFPT2_TRUNC_FIXED:
      if (param != std::floor(param) || param < 1.0 || param > (double)n_vir)
        return fail(DFPT2_ERR_INVALID_ARG, "fixed N' must be an integer in [1, n_vir]");
      break;
    default:
      return fail(DFPT2_ERR_INVALID_ARG, "unknown truncation rule %d", rule);
  }
  if (!(degen_rel_tol >= 0.0) || !std::isfinite(degen_rel_tol))
    return fail(DFPT2_ERR_INVALID_ARG, "degen_rel_tol must be finite and >= 0");
  const size_t need = eigh_workspace_bytes((int)n_vir) + 512;
  if (ws_bytes < need) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  char* tail = ws + eigh_workspace_bytes((int)n_vir);
  int st_ = eigh_run(D_vv, (int)n_vir, occ, no_vecs, ws, need - 512, st, 1);
  if (st_ != DFPT2_OK) return st_;
  int64_t* d_kept = reinterpret_cast<int64_t*>(tail);
  double* d_marg = reinterpret_cast<double*>(tail + 64);
  int* d_flag = reinterpret_cast<int*>(tail + 128);
  ProfScope ps_thr(DFPT2_STAGE_REDUCE, st);
  hipLaunchKernelGGL(rule_threshold_kernel, dim3(1), dim3(64), 0, st, occ, (int)n_vir, rule, param, degen_rel_tol,
                     d_kept, d_marg, d_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "threshold kernel");
  ps_thr.close();
  struct {
    int64_t kept;
    double marg[2];
    int flag;
  } h{};
  if ((e = hipMemcpyAsync(&h.kept, d_kept, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipMemcpyAsync(h.marg, d_marg, 16, hipMemcpyDeviceToHost, st)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipMemcpyAsync(&h.flag, d_flag, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "sync");
  prof_flush();
  if (h.flag) return fail(DFPT2_ERR_NONFINITE, "non-finite occupation number");
  *n_kept = h.kept;
  if (margins) {
    margins[0] = h.marg[0];
    margins[1] = h.marg[1];
  }
  return DFPT2_OK;
}

int fno_truncate(const double* D_vv, int64_t n_vir, double p_o, double degen_rel_tol, double* occ,
                 double* no_vecs, int64_t* n_kept, double* margins, void* workspace, size_t ws_bytes,
                 dfpt2_stream_t stream) {
  g_last_error.clear();
  return truncate_impl(D_vv, n_vir, DFPT2_TRUNC_CUMULATIVE, p_o, degen_rel_tol, occ, no_vecs, n_kept, margins,
                       workspace, ws_bytes, stream);
}

int fno_truncate_rule(const double* D_vv, int64_t n_vir, int rule, double param, double degen_rel_tol, double* occ,
                      double* no_vecs, int64_t* n_kept, double* margins, void* workspace, size_t ws_bytes,
                      dfpt2_stream_t stream) {
  g_last_error.clear();
  return truncate_impl(D_vv, n_vir, rule, param, degen_rel_tol, occ, no_vecs, n_kept, margins, workspace, ws_bytes,
                       stream);
}

}  // extern "C"
