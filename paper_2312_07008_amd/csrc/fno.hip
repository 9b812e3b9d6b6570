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

}  // namespace


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
