// Additive PT2 correction for a truncated virtual space (paper Sec. 2: rebuild
// in the kept NOs and recanonicalize; Eq. 11, scalar part).
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/dfpt2.h"
#include "eigh.h"
#include "host.h"
#include "kernels.h"

namespace dfpt2 {

namespace {

struct CorrPlan {
  int n_h, n_core, n_v, n_aux, nk;
  PassPlan kp;      // the kept-space pass (energy only)
  dfpt2_opts ko;    // its options
  size_t off_Y, off_F, off_et, off_W, off_U, off_Bt, off_eig, off_kp, off_tmp;
  size_t eig_bytes, total;
};

int plan_corr(const dfpt2_opts* o, int64_t n_kept, CorrPlan* cp) {
  PassPlan pl;
  int st = plan_pass(o, &pl);
  if (st != DFPT2_OK) return st;
  if (n_kept < 1 || n_kept > o->n_vir) return fail(DFPT2_ERR_INVALID_ARG, "n_kept must lie in [1, n_vir]");
  CorrPlan& c = *cp;
  c.n_h = pl.n_h;
  c.n_core = pl.n_core;
  c.n_v = pl.n_v;
  c.n_aux = pl.n_aux;
  c.nk = (int)n_kept;
  c.ko = *o;
  c.ko.n_vir = n_kept;
  c.ko.pair_batch = 0;
  st = plan_pass(&c.ko, &c.kp, true);
  if (st != DFPT2_OK) return st;
  const size_t nk = c.nk, nv = c.n_v;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o_ = off;
    off = align_up(off + b, 256);
    return o_;
  };
  c.off_Y = take(nv * nk * 8);
  c.off_F = take(nk * nk * 8);
  c.off_et = take(nk * 8);
  c.off_W = take(nk * nk * 8);
  c.off_U = take(nv * nk * 8);
  c.off_Bt = take((size_t)c.n_h * nk * c.n_aux * 8);
  c.eig_bytes = eigh_workspace_bytes(c.nk);
  c.off_eig = take(c.eig_bytes);
  c.off_kp = take(c.kp.ws_bytes);
  c.off_tmp = take(64);
  c.total = off;
  return DFPT2_OK;
}

__global__ void scale_rows_kernel(const double* V, int ldv, const double* eps, int n, int nk, double* Y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (k >= nk || a >= n) return;
  Y[(size_t)a * nk + k] = eps[a] * V[(size_t)a * ldv + k];
}

__global__ void symmetrize_kernel(double* F, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || i >= j) return;
  const double v = 0.5 * (F[(size_t)i * n + j] + F[(size_t)j * n + i]);
  F[(size_t)i * n + j] = v;
  F[(size_t)j * n + i] = v;
}

__global__ void dd_sub_kernel(const double* a, const double* b, double* out) {
  if (threadIdx.x != 0) return;
  double h = a[0], l = a[1];
  dd_add_dd(h, l, -b[0], -b[1]);
  out[0] = h;
  out[1] = l;
}

}  // namespace

}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int pt2_correction_workspace_size(const dfpt2_opts* opts, int64_t n_kept, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  CorrPlan cp;
  int st = plan_corr(opts, n_kept, &cp);
  if (st != DFPT2_OK) return st;
  *bytes = cp.total;
  return DFPT2_OK;
}

int pt2_energy_correction(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                          const double* gamma_act, const double* B, const double* no_vecs, int64_t n_kept,
                          const double* e_full, double* e_kept, double* correction, void* workspace,
                          size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  CorrPlan cp;
  int st = plan_corr(opts, n_kept, &cp);
  if (st != DFPT2_OK) return st;
  if (!eps_hole || !eps_vir || !B || !no_vecs || !e_full || !e_kept || !correction || !workspace)
    return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (opts->n_act > 0 && !gamma_act) return fail(DFPT2_ERR_INVALID_ARG, "gamma_act is null but n_act > 0");
  if (ws_bytes < cp.total) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, cp.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* Y = (double*)(ws + cp.off_Y);
  double* F = (double*)(ws + cp.off_F);
  double* et = (double*)(ws + cp.off_et);
  double* W = (double*)(ws + cp.off_W);
  double* U = (double*)(ws + cp.off_U);
  double* Bt = (double*)(ws + cp.off_Bt);
  const int nv = cp.n_v, nk = cp.nk;
  hipError_t e;
  // F' = V_k^T diag(eps) V_k
  ProfScope ps_f(DFPT2_STAGE_TRANSFORM, s);
  hipLaunchKernelGGL(scale_rows_kernel, dim3((nk + 255) / 256, nv), dim3(256), 0, s, no_vecs, nv, eps_vir, nv, nk, Y);
  if ((e = gemm_f64(no_vecs, nv, 0, 1, Y, nk, 0, 0, F, nk, 0, nk, nk, nv, 1, 1.0, 0.0, s)) != hipSuccess)
    return hip_fail(e, "gemm F");
  hipLaunchKernelGGL(symmetrize_kernel, dim3((nk + 255) / 256, nk), dim3(256), 0, s, F, nk);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "symmetrize");
  ps_f.close();
  st = eigh_run(F, nk, et, W, ws + cp.off_eig, cp.eig_bytes, s, 0);
  if (st != DFPT2_OK) return st;
  // U = V_k W ; B~_i = U^T B_i
  ProfScope ps_u(DFPT2_STAGE_TRANSFORM, s);
  if ((e = gemm_f64(no_vecs, nv, 0, 0, W, nk, 0, 0, U, nk, 0, nv, nk, nk, 1, 1.0, 0.0, s)) != hipSuccess)
    return hip_fail(e, "gemm U");
  if ((e = gemm_f64(U, nk, 0, 1, B, cp.n_aux, (long long)nv * cp.n_aux, 0, Bt, cp.n_aux, (long long)nk * cp.n_aux,
                    nk, cp.n_aux, nv, cp.n_h, 1.0, 0.0, s)) != hipSuccess)
    return hip_fail(e, "gemm Bt");
  ps_u.close();
  // kept-space pass (energy only) in the recanonicalized basis (eps~, B~)
  st = run_pass(cp.kp, cp.ko, eps_hole, et, gamma_act, Bt, nullptr, nullptr, e_kept, nullptr, nullptr,
                ws + cp.off_kp, s);
  if (st != DFPT2_OK) return st;
  ProfScope ps_sub(DFPT2_STAGE_REDUCE, s);
  hipLaunchKernelGGL(dd_sub_kernel, dim3(1), dim3(64), 0, s, e_full, e_kept, correction);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "dd_sub");
  ps_sub.close();
  double h[2];
  if ((e = hipMemcpyAsync(h, e_kept, 16, hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  prof_flush();
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(DFPT2_ERR_NONFINITE, "kept-space energy is not finite");
  return DFPT2_OK;
}

}  // extern "C"
