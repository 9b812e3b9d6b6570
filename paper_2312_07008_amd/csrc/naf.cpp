// Natural auxiliary functions for the pass's density-fitted integrals (the
// compression of the auxiliary basis proposed in the paper's conclusions).
// With J[(i,a), P] = B^P_ia over every hole i and virtual a:
//   W = J^T J (FP64 MFMA GEMM, contraction over n_h n_vir), W = U diag(sigma) U^T
//   with the library's eigensolver (sigma descending), keep the n_naf functions
//   with sigma_k > eps max|sigma| = eps sigma_0 (eps <= 0 keeps all), B~ = J U[:, :n_naf].
// Eigenvectors are formed only for the kept functions: dropped ones often form a
// large cluster near zero (redundant auxiliary sets), which inverse iteration
// would otherwise orthogonalize serially.
// B~ is laid out like B with n_aux replaced by n_naf, so it can be passed to
// dfpt2_build_vv_density and pt2_energy_correction as is.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/dfpt2.h"
#include "eigh.h"
#include "host.h"

using namespace dfpt2;

namespace {
struct NafPlan {
  int n_aux;
  long long rows;  // n_h n_vir
  size_t off_W, off_U, off_eig, eig_bytes, total;
};

int plan_naf(const dfpt2_opts* o, NafPlan* p) {
  if (!o) return fail(DFPT2_ERR_INVALID_ARG, "opts is null");
  if (o->n_core < 0 || o->n_act < 0 || o->n_core + o->n_act <= 0 || o->n_vir <= 0 || o->n_aux <= 0)
    return fail(DFPT2_ERR_INVALID_ARG, "sizes must satisfy n_core, n_act >= 0, n_h > 0, n_vir > 0, n_aux > 0");
  if (o->n_aux > kEighMaxN) return fail(DFPT2_ERR_INVALID_ARG, "n_aux must be <= %d for the eigensolver", kEighMaxN);
  const long long rows = (o->n_core + o->n_act) * o->n_vir;
  if (rows > 0x7fffffffLL) return fail(DFPT2_ERR_INVALID_ARG, "n_h * n_vir too large");
  p->n_aux = (int)o->n_aux;
  p->rows = rows;
  const size_t nn = (size_t)p->n_aux * p->n_aux;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t r = off;
    off = align_up(off + b, 256);
    return r;
  };
  p->off_W = take(nn * sizeof(double));
  p->off_U = take(nn * sizeof(double));
  p->eig_bytes = eigh_workspace_bytes(p->n_aux);
  p->off_eig = take(p->eig_bytes);
  p->total = off;
  return DFPT2_OK;
}
}  // namespace

extern "C" {

int naf_compress_workspace_size(const dfpt2_opts* opts, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  NafPlan p;
  int st = plan_naf(opts, &p);
  if (st != DFPT2_OK) return st;
  *bytes = p.total;
  return DFPT2_OK;
}

int naf_compress(const dfpt2_opts* opts, const double* B, double eps, double* B_naf, double* sigma,
                 int64_t* n_naf, void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  NafPlan p;
  int st = plan_naf(opts, &p);
  if (st != DFPT2_OK) return st;
  if (!B || !B_naf || !sigma || !n_naf || !workspace) return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (!std::isfinite(eps)) return fail(DFPT2_ERR_INVALID_ARG, "eps must be finite");
  if (ws_bytes < p.total) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* W = reinterpret_cast<double*>(ws + p.off_W);
  double* U = reinterpret_cast<double*>(ws + p.off_U);
  const int na = p.n_aux;
  hipError_t e;
  {
    ProfScope ps(DFPT2_STAGE_TRANSFORM, s);
    // W = J^T J: op(A) = J^T (A stored rows x n_aux), op(B) = J
    if ((e = gemm_f64(B, na, 0, 1, B, na, 0, 0, W, na, 0, na, na, (int)p.rows, 1, 1.0, 0.0, s)) != hipSuccess)
      return hip_fail(e, "NAF metric GEMM");
  }
  st = eigh_run(W, na, sigma, U, ws + p.off_eig, p.eig_bytes, s, 1, eps > 0.0 ? eps : -1.0);
  if (st != DFPT2_OK) return st;
  std::vector<double> h(na);
  if ((e = hipMemcpyAsync(h.data(), sigma, sizeof(double) * na, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "sigma copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  int keep = na;
  if (eps > 0.0) {
    keep = 0;
    // the eigensolver forms vectors above eps max|sigma| (= eps sigma_0 for the PSD metric)
    const double thr = eps * std::max(std::fabs(h[0]), std::fabs(h[na - 1]));
    while (keep < na && h[keep] > thr) ++keep;
  }
  for (int k = 0; k < na; ++k)
    if (!std::isfinite(h[k])) return fail(DFPT2_ERR_NONFINITE, "non-finite NAF eigenvalue");
  if (keep == 0) return fail(DFPT2_ERR_INVALID_ARG, "eps %g removes every auxiliary function", eps);
  {
    ProfScope ps(DFPT2_STAGE_TRANSFORM, s);
    // B~ = J U[:, :keep]  (U row-major n_aux x n_aux, column k = NAF k)
    if ((e = gemm_f64(B, na, 0, 0, U, na, 0, 0, B_naf, keep, 0, (int)p.rows, keep, na, 1, 1.0, 0.0, s)) !=
        hipSuccess)
      return hip_fail(e, "NAF transform GEMM");
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  prof_flush();
  *n_naf = keep;
  return DFPT2_OK;
}

}  // extern "C"
