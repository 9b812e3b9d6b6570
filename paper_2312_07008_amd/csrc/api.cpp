// C ABI of libdfpt2.so: argument validation, workspace layout and the
// orchestration of the kernels of the DF-DSRG-PT2 virtual natural-orbital pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/dfpt2.h"
#include "host.h"
#include "kernels.h"

namespace dfpt2 {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(DFPT2_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ----------------------------------------------------------- pass planning
int plan_pass(const dfpt2_opts* o, PassPlan* pl) {
  if (!o) return fail(DFPT2_ERR_INVALID_ARG, "opts is null");
  if (o->n_core < 0 || o->n_act < 0 || o->n_vir <= 0 || o->n_aux <= 0)
    return fail(DFPT2_ERR_INVALID_ARG, "sizes must satisfy n_core >= 0, n_act >= 0, n_vir > 0, n_aux > 0");
  if (o->n_core + o->n_act <= 0) return fail(DFPT2_ERR_INVALID_ARG, "no holes (n_core + n_act == 0)");
  if (o->n_core > 1024 || o->n_act > 64)
    return fail(DFPT2_ERR_INVALID_ARG, "n_core must be <= 1024 and n_act <= 64");
  if (o->n_vir > 32768 || o->n_aux > (int64_t)1 << 30)
    return fail(DFPT2_ERR_INVALID_ARG, "n_vir must be <= 32768");
  if (!(o->s > 0.0) || !std::isfinite(o->s)) return fail(DFPT2_ERR_INVALID_ARG, "s must be finite and > 0");
  if (o->density_convention != 0 && o->density_convention != 1)
    return fail(DFPT2_ERR_INVALID_ARG, "density_convention must be 0 or 1");
  if (o->precision != DFPT2_FP64 && o->precision != DFPT2_BF16_SLICED && o->precision != DFPT2_FP8_SLICED)
    return fail(DFPT2_ERR_INVALID_ARG, "unknown precision %d", o->precision);
  if (o->slices_gemm1 < 0 || o->slices_gemm1 > 8 || o->slices_gemm2 < 0 || o->slices_gemm2 > 8)
    return fail(DFPT2_ERR_INVALID_ARG, "slice counts must lie in [0, 8]");
  if (o->pair_batch < 0) return fail(DFPT2_ERR_INVALID_ARG, "pair_batch must be >= 0");

  PassPlan& p = *pl;
  p = PassPlan{};
  p.n_core = (int)o->n_core;
  p.n_act = (int)o->n_act;
  p.n_h = p.n_core + p.n_act;
  p.n_v = (int)o->n_vir;
  p.n_aux = (int)o->n_aux;
  p.nt = (p.n_v + 63) / 64;
  p.nTP = p.nt * (p.nt + 1) / 2;
  p.n_up = p.n_core * (p.n_core + 1) / 2;
  const size_t mat = (size_t)p.n_v * p.n_v;
  int64_t batch = o->pair_batch;
  if (batch == 0) {
    const double cap_bytes = 8.0e9;
    batch = (int64_t)(cap_bytes / (double)(mat * sizeof(double)));
    if (batch > 512) batch = 512;
    if (batch < 8) batch = 8;
  }
  if (batch > 65535) batch = 65535;
  if (p.n_up > 0 && batch > p.n_up) batch = p.n_up;
  if (batch < 1) batch = 1;
  p.batch = (int)batch;
  int nsplit = (2048 + p.nTP - 1) / p.nTP;
  if (nsplit > 64) nsplit = 64;
  if (nsplit > p.batch) nsplit = p.batch;
  if (nsplit < 1) nsplit = 1;
  p.nsplit = nsplit;
  p.w_density = (o->density_convention == 0) ? 2.0 : 1.0;
  p.precision = o->precision;
  p.ns1 = o->slices_gemm1 ? o->slices_gemm1 : default_slices_gemm1(o->precision);
  p.n_v_pad = (p.n_v + 63) / 64 * 64;
  p.n_aux_pad = (p.n_aux + 15) / 16 * 16;
  if (p.precision == DFPT2_BF16_SLICED && (p.ns1 < 2 || p.ns1 > 5))
    return fail(DFPT2_ERR_INVALID_ARG, "slices_gemm1 must lie in [2, 5] for BF16 slicing");

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o_ = off;
    off = align_up(off + bytes, 256);
    return o_;
  };
  p.off_pairs = take(sizeof(int2) * (size_t)(p.n_up > 0 ? p.n_up : 1));
  p.off_count = take(sizeof(int) * 4);
  p.off_T = take(sizeof(double) * mat * p.batch);
  p.off_epart = take(sizeof(double) * (size_t)p.batch * p.nTP);
  p.off_tpart = take(sizeof(double) * (size_t)p.batch * p.nTP);
  p.off_pe = take(sizeof(double) * 2 * (size_t)(p.n_up > 0 ? p.n_up : 1));
  p.off_tn2 = take(sizeof(double) * (size_t)(p.n_up > 0 ? p.n_up : 1));
  p.off_Dpart = take(sizeof(double) * mat * p.nsplit);
  p.off_Bs = take(p.precision == DFPT2_BF16_SLICED
                      ? (size_t)p.ns1 * p.n_h * p.n_v_pad * p.n_aux_pad * sizeof(__bf16)
                      : 0);
  p.off_norm2 = take(p.precision == DFPT2_BF16_SLICED ? sizeof(double) * (size_t)p.n_h * p.n_v : 0);
  p.ws_bytes = off;
  return DFPT2_OK;
}

}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

const char* dfpt2_last_error(void) { return g_last_error.c_str(); }

const char* dfpt2_status_string(int status) {
  switch (status) {
    case DFPT2_OK: return "ok";
    case DFPT2_ERR_INVALID_ARG: return "invalid argument";
    case DFPT2_ERR_WORKSPACE: return "workspace too small";
    case DFPT2_ERR_HIP: return "HIP runtime error";
    case DFPT2_ERR_NOT_CONVERGED: return "eigensolver did not converge";
    case DFPT2_ERR_NONFINITE: return "non-finite result";
    case DFPT2_ERR_UNSUPPORTED: return "unsupported option combination";
    default: return "unknown status";
  }
}

const char* dfpt2_version(void) { return "dfpt2 0.1 (gfx950)"; }

int dfpt2_workspace_size(const dfpt2_opts* opts, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  PassPlan pl;
  int st = plan_pass(opts, &pl);
  if (st != DFPT2_OK) return st;
  *bytes = pl.ws_bytes;
  return DFPT2_OK;
}

int dfpt2_build_vv_density(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                           const double* gamma_act, const double* B, const uint8_t* pair_mask,
                           double* D_vv, double* e_pt2, double* pair_energy, float* pair_tnorm,
                           void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  PassPlan pl;
  int st = plan_pass(opts, &pl);
  if (st != DFPT2_OK) return st;
  if (!eps_hole || !eps_vir || !B || !D_vv || !e_pt2)
    return fail(DFPT2_ERR_INVALID_ARG, "eps_hole, eps_vir, B, D_vv and e_pt2 must be non-null");
  if (pl.n_act > 0 && !gamma_act) return fail(DFPT2_ERR_INVALID_ARG, "gamma_act is null but n_act > 0");
  if (!workspace && pl.ws_bytes) return fail(DFPT2_ERR_INVALID_ARG, "workspace is null");
  if (ws_bytes < pl.ws_bytes)
    return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, pl.ws_bytes);
  if (pl.n_act > 0) return fail(DFPT2_ERR_UNSUPPORTED, "active holes are not supported by this build");
  if (opts->precision == DFPT2_FP8_SLICED)
    return fail(DFPT2_ERR_UNSUPPORTED, "precision %d is not supported by this build", opts->precision);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run_pass(pl, *opts, eps_hole, eps_vir, B, pair_mask, D_vv, e_pt2, pair_energy, pair_tnorm,
                       static_cast<char*>(workspace), s);
}

}  // extern "C"

namespace dfpt2 {

int default_slices_gemm1(int precision) { return precision == DFPT2_BF16_SLICED ? 4 : 1; }

hipError_t launch_pair(const PairLaunch& L, const PairKernelArgs& a, int n_pairs, hipStream_t st) {
  if (L.precision == DFPT2_FP64) return launch_pair_gemm_f64(a, n_pairs, st);
  PairBf16Args b{};
  b.Bs = L.Bs;
  b.slice_stride = L.slice_stride;
  b.norm2 = L.norm2;
  b.eps_h = a.eps_h;
  b.eps_v = a.eps_v;
  b.pairs = a.pairs;
  b.T = a.T;
  b.epart = a.epart;
  b.tpart = a.tpart;
  b.n_v = a.n_v;
  b.n_v_pad = L.n_v_pad;
  b.n_aux_pad = L.n_aux_pad;
  b.nt = a.nt;
  b.nTP = a.nTP;
  b.s = a.s;
  b.e_weight = a.e_weight;
  return launch_pair_gemm_bf16(b, L.ns, n_pairs, st);
}

int run_pass(const PassPlan& pl, const dfpt2_opts& o, const double* eps_h, const double* eps_v,
             const double* B, const uint8_t* mask, double* D, double* e_out, double* pair_energy,
             float* pair_tnorm, char* ws, hipStream_t s) {
  hipError_t e;
  int2* pairs = reinterpret_cast<int2*>(ws + pl.off_pairs);
  int* d_count = reinterpret_cast<int*>(ws + pl.off_count);
  double* T = reinterpret_cast<double*>(ws + pl.off_T);
  double* epart = reinterpret_cast<double*>(ws + pl.off_epart);
  double* tpart = reinterpret_cast<double*>(ws + pl.off_tpart);
  double* pe = reinterpret_cast<double*>(ws + pl.off_pe);
  double* tn2 = reinterpret_cast<double*>(ws + pl.off_tn2);
  double* Dpart = reinterpret_cast<double*>(ws + pl.off_Dpart);
  const size_t mat = (size_t)pl.n_v * pl.n_v;

  PairLaunch L{pl.precision, pl.ns1, B, nullptr, 0, pl.n_v_pad, pl.n_aux_pad, nullptr};
  if (pl.precision == DFPT2_BF16_SLICED) {
    ProfScope ps(DFPT2_STAGE_SPLIT, s);
    __bf16* Bs = reinterpret_cast<__bf16*>(ws + pl.off_Bs);
    L.Bs = Bs;
    L.slice_stride = (long long)pl.n_h * pl.n_v_pad * pl.n_aux_pad;
    double* nrm = reinterpret_cast<double*>(ws + pl.off_norm2);
    L.norm2 = nrm;
    if ((e = launch_split_rows_bf16(B, pl.n_aux, pl.n_h, pl.n_v, pl.n_v_pad, pl.n_aux, pl.n_aux_pad, pl.ns1, Bs,
                                    nrm, s)) != hipSuccess)
      return hip_fail(e, "split");
  }
  {
    ProfScope ps(DFPT2_STAGE_REDUCE, s);
    if ((e = launch_build_pairs(mask, pl.n_core, pl.n_h, pairs, d_count, s)) != hipSuccess)
      return hip_fail(e, "build_pairs");
  }
  int count = 0;
  if ((e = hipMemcpyAsync(&count, d_count, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "count copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream sync");

  if (pair_energy) {
    // core-core entries start at 0 (masked pairs stay 0); pairs with an active hole are NaN
    if ((e = launch_fill(pair_energy, (size_t)pl.n_h * pl.n_h, 0.0, s)) != hipSuccess)
      return hip_fail(e, "fill");
  }
  if (pair_tnorm) {
    if ((e = launch_fill_f32(pair_tnorm, (size_t)pl.n_h * pl.n_h, 0.0f, s)) != hipSuccess)
      return hip_fail(e, "fill");
  }

  PairKernelArgs pa{};
  pa.B = B;
  pa.eps_h = eps_h;
  pa.eps_v = eps_v;
  pa.n_v = pl.n_v;
  pa.n_aux = pl.n_aux;
  pa.nt = pl.nt;
  pa.nTP = pl.nTP;
  pa.s = o.s;
  pa.e_weight = 1.0;  // 1/4 gamma_ii gamma_jj with gamma = 2 for core holes
  pa.T = T;
  pa.epart = epart;
  pa.tpart = tpart;

  DensityKernelArgs da{};
  da.T = T;
  da.n_v = pl.n_v;
  da.nt = pl.nt;
  da.nTP = pl.nTP;
  da.w = pl.w_density;

  for (int p0 = 0, b = 0; p0 < count; p0 += pl.batch, ++b) {
    const int np = (count - p0 < pl.batch) ? count - p0 : pl.batch;
    pa.pairs = pairs + p0;
    {
      ProfScope ps(DFPT2_STAGE_PAIR, s);
      if ((e = launch_pair(L, pa, np, s)) != hipSuccess) return hip_fail(e, "pair kernel");
    }
    {
      ProfScope ps(DFPT2_STAGE_REDUCE, s);
      if ((e = launch_pair_reduce(epart, tpart, pl.nTP, np, pe + 2 * (size_t)p0, tn2 + p0, s)) != hipSuccess)
        return hip_fail(e, "pair reduce");
    }
    da.pairs = pairs + p0;
    da.n_pairs = np;
    da.nsplit = pl.nsplit < np ? pl.nsplit : np;
    da.Dpart = Dpart;
    da.accumulate = (b > 0) ? 1 : 0;
    // every split slice that exists must be written on the first batch
    if (b == 0 && da.nsplit < pl.nsplit) {
      if ((e = launch_fill(Dpart, mat * pl.nsplit, 0.0, s)) != hipSuccess) return hip_fail(e, "fill");
      da.accumulate = 1;
    }
    {
      ProfScope ps(DFPT2_STAGE_DENSITY, s);
      if ((e = launch_density_f64(da, s)) != hipSuccess) return hip_fail(e, "density kernel");
    }
  }
  {
    ProfScope ps_tail(DFPT2_STAGE_REDUCE, s);
    if (count == 0) {
      if ((e = launch_fill(D, mat, 0.0, s)) != hipSuccess) return hip_fail(e, "fill");
    } else {
      if ((e = launch_density_reduce(Dpart, pl.nsplit, pl.n_v, D, s)) != hipSuccess)
        return hip_fail(e, "density reduce");
    }
    if ((e = launch_energy_finalize(pe, tn2, pairs, d_count, pl.n_up, pl.n_h, e_out, pair_energy, pair_tnorm,
                                    s)) != hipSuccess)
      return hip_fail(e, "energy finalize");
  }
  double eh[2];
  if ((e = hipMemcpyAsync(eh, e_out, sizeof(eh), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "energy copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream sync");
  prof_flush();
  if (!std::isfinite(eh[0]) || !std::isfinite(eh[1])) return fail(DFPT2_ERR_NONFINITE, "PT2 energy is not finite");
  return DFPT2_OK;
}

}  // namespace dfpt2
