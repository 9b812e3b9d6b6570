// C ABI of libdfpt2.so: argument validation, workspace layout and the
// orchestration of the kernels of the DF-DSRG-PT2 virtual natural-orbital pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/dfpt2.h"
#include "eigh.h"
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
int plan_pass(const dfpt2_opts* o, PassPlan* pl, bool energy_only) {
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
  if (o->precision != DFPT2_FP64 && o->precision != DFPT2_BF16_SLICED && o->precision != DFPT2_FP8_SLICED &&
      o->precision != DFPT2_INT8_SLICED)
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
  // energy-only passes store no amplitudes: one batch of every pair, except with
  // BF16 slices or INT8 digits, whose product writes V to a buffer of one batch
  // for the epilogue kernel
  const bool v_buffer =
      energy_only && (o->precision == DFPT2_BF16_SLICED || o->precision == DFPT2_INT8_SLICED);
  if (energy_only && !v_buffer) batch = 65535;
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
  p.energy_only = energy_only;
  p.precision = o->precision;
  p.ns1 = o->slices_gemm1 ? o->slices_gemm1 : default_slices_gemm1(o->precision);
  p.n_v_pad_d = (p.n_v + 63) / 64 * 64;
  // slab rows of the sliced operands and rows of the density operands: 128-multiples
  // for BF16 and INT8 digits (the 128-row tiles of the product kernels) and for the
  // BF16 density kernel
  p.n_v_pad = (p.precision == DFPT2_BF16_SLICED || p.precision == DFPT2_INT8_SLICED) ? (p.n_v + 127) / 128 * 128
                                                                                      : p.n_v_pad_d;
  p.n_v_rows_t = p.precision == DFPT2_BF16_SLICED ? (p.n_v + 127) / 128 * 128 : p.n_v_pad_d;
  p.nTD = density_bf16_tiles(p.nt);
  p.nTP1 = p.nTP;
  p.n_aux_pad = p.precision == DFPT2_FP8_SLICED ? (p.n_aux + 63) / 64 * 64 : (p.n_aux + 31) / 32 * 32;
  if ((p.precision == DFPT2_BF16_SLICED || p.precision == DFPT2_FP8_SLICED) && (p.ns1 < 2 || p.ns1 > 4))
    return fail(DFPT2_ERR_INVALID_ARG, "slices_gemm1 must lie in [2, 4] for BF16 and FP8 slicing");
  if (p.precision == DFPT2_INT8_SLICED) {
    if (p.ns1 < 3 || p.ns1 > 5) return fail(DFPT2_ERR_INVALID_ARG, "slices_gemm1 must lie in [3, 5] for INT8 digits");
    if (p.n_aux_pad > pair_i8_max_aux_pad(p.ns1))
      return fail(DFPT2_ERR_INVALID_ARG, "n_aux=%d too large for exact INT8 level sums with %d digits (max %d)",
                  p.n_aux, p.ns1, pair_i8_max_aux_pad(p.ns1));
  }
  const bool sliced_density = p.precision == DFPT2_BF16_SLICED || p.precision == DFPT2_INT8_SLICED;
  const int ns2_max = p.precision == DFPT2_INT8_SLICED ? 5 : 4;
  p.ns2 = o->slices_gemm2 ? o->slices_gemm2 : (p.precision == DFPT2_INT8_SLICED ? 5 : sliced_density ? 4 : 1);
  if (p.ns2 > ns2_max || (p.ns2 > 1 && !sliced_density))
    return fail(DFPT2_ERR_INVALID_ARG,
                "slices_gemm2 must be 1 (FP64 density) or 2..4 BF16 slices (BF16) or 2..5 INT8 digits (INT8)");
  if (p.precision == DFPT2_INT8_SLICED && p.ns2 >= 2 && (long long)(p.ns2 - 1) * 16384 * p.n_v_pad_d >= 0x7fffffffLL)
    return fail(DFPT2_ERR_INVALID_ARG, "n_vir too large for exact INT8 density sums with %d digits", p.ns2);
  if (energy_only) p.ns2 = 1;
  // sliced density: splits of the pair range chosen so that workgroup tiles x splits
  // fill whole rounds on 256 CUs (one BF16 workgroup per CU, two INT8 ones), with
  // at least four rounds and the batch's pairs dealt evenly to the splits
  p.nsplit2 = 1;
  if (p.ns2 >= 2) {
    double best = 1e30;
    const int cap = p.batch < 64 ? p.batch : 64;
    const int tiles = p.precision == DFPT2_BF16_SLICED ? p.nTD : p.nTP;
    const double slots = p.precision == DFPT2_BF16_SLICED ? 256.0 : 512.0;
    for (int k = 1; k <= cap; ++k) {
      const double w = (double)tiles * k;
      const double rounds = std::ceil(w / slots);
      const double per = (double)p.batch / k;
      const double waste = (rounds * slots - w) / w + (std::ceil(per) - per) / per + (w < 4.0 * slots ? 1.0 : 0.0);
      if (waste < best - 1e-12) {
        best = waste;
        p.nsplit2 = k;
      }
    }
  }
  p.nsplit_all = p.nsplit > p.nsplit2 ? p.nsplit : p.nsplit2;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o_ = off;
    off = align_up(off + bytes, 256);
    return o_;
  };
  p.off_pairs = take(sizeof(int2) * (size_t)(p.n_up > 0 ? p.n_up : 1));
  p.off_count = take(sizeof(int) * 4);
  p.off_T = take(energy_only && !v_buffer ? 0 : sizeof(double) * mat * p.batch);  // T, or V of an energy-only pass
  p.off_epart = take(sizeof(double) * (size_t)p.batch * p.nTP1);
  p.off_tpart = take(sizeof(double) * (size_t)p.batch * p.nTP1);
  p.off_pe = take(sizeof(double) * 2 * (size_t)(p.n_up > 0 ? p.n_up : 1));
  p.off_tn2 = take(sizeof(double) * (size_t)(p.n_up > 0 ? p.n_up : 1));
  p.off_Dpart = take(energy_only ? 0 : sizeof(double) * mat * p.nsplit_all);
  const size_t slice_bytes = p.precision == DFPT2_BF16_SLICED                                        ? sizeof(__bf16)
                             : (p.precision == DFPT2_FP8_SLICED || p.precision == DFPT2_INT8_SLICED) ? 1
                                                                                                    : 0;
  p.off_Bs = take(slice_bytes * p.ns1 * p.n_h * p.n_v_pad * p.n_aux_pad);
  p.off_scales = take(p.precision == DFPT2_FP8_SLICED ? sizeof(uint32_t) * 2 * (size_t)p.n_h * p.n_v_pad * (p.n_aux_pad / 64)
                                                      : 0);
  p.off_norm2 = take(p.precision != DFPT2_FP64 ? sizeof(double) * (size_t)p.n_h * p.n_v : 0);
  p.off_rexp = take(p.precision == DFPT2_INT8_SLICED ? sizeof(int) * (size_t)p.n_h * p.n_v_pad : 0);
  // active holes: core batches of the core-active block (cpb cores x n_act pairs each)
  p.n_ca = p.n_core * p.n_act;
  p.n_aa_un = p.n_act * (p.n_act + 1) / 2;
  if (p.n_act > 0) {
    const double budget = 16.0e9;
    int cap = (int)(budget / (4.0 * (double)mat * sizeof(double)));
    int cpb = cap / p.n_act;
    if (cpb < 1) cpb = 1;
    if (cpb > p.n_core) cpb = p.n_core > 0 ? p.n_core : 1;
    p.cpb = cpb;
    p.act_cap = p.n_act * p.n_act > p.n_act * cpb ? p.n_act * p.n_act : p.n_act * cpb;
  }
  // density operands: BF16 slices, or INT8 digits (+ row exponents) with INT8 precision,
  // for a batch of core pairs or of the active blocks' rotated amplitudes
  int nb_t = p.batch;
  if (p.n_act > 0 && !energy_only) {
    const int act_np = p.n_act * p.cpb > p.n_aa_un ? p.n_act * p.cpb : p.n_aa_un;
    if (act_np > nb_t) nb_t = act_np;
  }
  const size_t t_bytes = p.precision == DFPT2_INT8_SLICED ? 1 : sizeof(__bf16);
  p.off_Ts = take(p.ns2 >= 2 ? t_bytes * 4 * (size_t)nb_t * p.n_v_rows_t * p.n_v_pad_d * p.ns2 : 0);
  p.off_Texp = take(p.ns2 >= 2 && p.precision == DFPT2_INT8_SLICED ? sizeof(int) * 4 * (size_t)nb_t * p.n_v_pad_d
                                                                    : 0);
  p.off_dg = take(p.ns2 >= 2 ? sizeof(double) * (size_t)nb_t * (p.n_v_pad_d / 64) * p.n_v_pad_d : 0);
  // row maxima: INT8 digits only (the BF16 slices take one exponent per 64-column block from the block)
  p.off_tmax = take(p.ns2 >= 2 && p.precision == DFPT2_INT8_SLICED
                        ? sizeof(unsigned long long) * 4 * (size_t)nb_t * p.n_v_pad_d
                        : 0);
  p.off_diag = take(p.ns2 >= 2 ? sizeof(double) * (size_t)p.n_v : 0);
  // active holes: stacked amplitude/integral matrices before and after the rotation
  if (p.n_act > 0) {
    const size_t ac = (size_t)p.act_cap;
    p.off_act_T = take(sizeof(double) * mat * ac);
    p.off_act_V = take(sizeof(double) * mat * ac);
    p.off_act_Tr = take(sizeof(double) * mat * ac);
    p.off_act_Vr = take(sizeof(double) * mat * ac);
    p.off_act_pairs = take(sizeof(int2) * ac);
    p.off_act_slots = take(sizeof(int) * ac);
    p.off_act_pairs2 = take(sizeof(int2) * ac);
    p.off_act_slots2 = take(sizeof(int) * ac);
    p.off_act_wd = take(sizeof(double) * ac);
    p.off_act_we = take(sizeof(double) * ac);
    p.off_act_tpart = take(sizeof(double) * ac * p.nTP1);
    p.off_act_tn2 = take(sizeof(double) * ac);
    p.off_act_epart = take(sizeof(double) * ac * (size_t)p.nt * p.nt);
    p.off_act_pe = take(sizeof(double) * 2 * (size_t)(p.n_ca + p.n_aa_un));
    p.off_act_occ = take(sizeof(double) * p.n_act);
    p.off_act_U = take(sizeof(double) * p.n_act * p.n_act);
    p.off_act_W = take(sizeof(double) * (size_t)p.n_act * p.n_act * p.n_act * p.n_act);
    p.act_eig_bytes = eigh_workspace_bytes(p.n_act);
    p.off_act_eig = take(p.act_eig_bytes);
  }
  p.ws_bytes = off;
  return DFPT2_OK;
}

// Static device scratch of dfpt2_build_vv_density_noalloc: one copy per GPU,
// held from the first use on that GPU until the process ends.  Host code never
// passes this name to a kernel or a copy: each device's address comes from
// hipGetSymbolAddress (static_scratch below) and only that address is used.
static __device__ __align__(256) char scratch[DFPT2_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Address of the current device's copy of `scratch`, looked up once per device
// (with that device current) on the first call that needs it.
static int static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DFPT2_ERR_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(DFPT2_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
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
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run_pass(pl, *opts, eps_hole, eps_vir, gamma_act, B, pair_mask, D_vv, e_pt2, pair_energy, pair_tnorm,
                  static_cast<char*>(workspace), s);
}

int dfpt2_build_vv_density_noalloc(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                                   const double* gamma_act, const double* B, const uint8_t* pair_mask,
                                   double* D_vv, double* e_pt2, double* pair_energy, float* pair_tnorm,
                                   dfpt2_stream_t stream) {
  g_last_error.clear();
  PassPlan pl;
  int st = plan_pass(opts, &pl);
  if (st != DFPT2_OK) return st;
  if (!eps_hole || !eps_vir || !B || !D_vv || !e_pt2)
    return fail(DFPT2_ERR_INVALID_ARG, "eps_hole, eps_vir, B, D_vv and e_pt2 must be non-null");
  if (pl.n_act > 0 && !gamma_act) return fail(DFPT2_ERR_INVALID_ARG, "gamma_act is null but n_act > 0");
  if (pl.ws_bytes > (size_t)DFPT2_STATIC_SCRATCH_BYTES)
    return fail(DFPT2_ERR_WORKSPACE,
                "this pass needs %zu bytes of scratch, more than the %llu of the static scratch; use "
                "dfpt2_build_vv_density with a workspace, or a smaller pair_batch",
                pl.ws_bytes, (unsigned long long)DFPT2_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((st = static_scratch(&ws)) != DFPT2_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run_pass(pl, *opts, eps_hole, eps_vir, gamma_act, B, pair_mask, D_vv, e_pt2, pair_energy, pair_tnorm,
                  static_cast<char*>(ws), s);
}

}  // extern "C"

namespace dfpt2 {

int default_slices_gemm1(int precision) {
  return precision == DFPT2_FP64 ? 1 : precision == DFPT2_INT8_SLICED ? 5 : 4;
}

hipError_t launch_pair(const PairLaunch& L, const PairKernelArgs& a, int n_pairs, hipStream_t st,
                       ProfScope* product) {
  if (L.precision == DFPT2_FP64) return launch_pair_gemm_f64(a, n_pairs, st);
  // an epilogue kernel of its own is timed as a stage of its own after the main
  // pass's product; in the kept-space energy and the active blocks it stays in the
  // caller's stage
  const bool own_epi = product && product->stage() == DFPT2_STAGE_PAIR;
  auto epi_stage = [&] {
    if (own_epi) product->close();
    return own_epi ? DFPT2_STAGE_PAIR_EPILOGUE : -1;
  };
  PairSlicedArgs b{};
  b.Bs = L.Bs;
  b.scales = L.scales;
  b.rexp = L.rexp;
  b.norm2 = L.norm2;
  b.eps_h = a.eps_h;
  b.eps_v = a.eps_v;
  b.pairs = a.pairs;
  b.T = a.T;
  b.Vr = a.Vr;
  b.epart = a.epart;
  b.tpart = a.tpart;
  b.tmax = (L.precision == DFPT2_INT8_SLICED) ? a.tmax : nullptr;
  b.dgp = b.tmax ? a.dgp : nullptr;
  b.n_v = a.n_v;
  b.n_v_pad = L.n_v_pad;
  b.n_aux_pad = L.n_aux_pad;
  b.nt = a.nt;
  b.nTP = a.nTP;
  b.n_v_pad_d = (a.n_v + 63) / 64 * 64;
  b.s = a.s;
  b.e_weight = a.e_weight;
  if (L.precision == DFPT2_FP8_SLICED) return launch_pair_gemm_fp8(b, L.ns, n_pairs, st);
  if (L.precision == DFPT2_INT8_SLICED) {  // the product on its own, then the epilogue kernel
    const bool store = b.T || b.Vr;
    if (!store) {
      if (!L.vbuf) return launch_pair_gemm_i8(b, L.ns, n_pairs, st);  // energy only, fused
      b.T = L.vbuf;
    }
    const hipError_t e = launch_pair_v_i8(b, L.ns, n_pairs, st);
    if (e != hipSuccess) return e;
    ProfScope ps(epi_stage(), st);
    return launch_pair_epi_bf16(b, n_pairs, store, st);
  }
  if (L.ts && b.T && !b.Vr) {  // split-BF16 density: V in b.T, then the epilogue that slices the amplitudes
    const hipError_t e = launch_pair_v_bf16(b, L.ns, n_pairs, st);
    if (e != hipSuccess) return e;
    ProfScope ps(epi_stage(), st);
    return launch_pair_epi_split_bf16(b, n_pairs, L.ns2, L.rows_t, L.ts, L.dgp, st);
  }
  if (b.T || b.Vr) {  // amplitudes stored: product and epilogue as two kernels
    const hipError_t e = launch_pair_v_bf16(b, L.ns, n_pairs, st);
    if (e != hipSuccess) return e;
    ProfScope ps(epi_stage(), st);
    return launch_pair_epi_bf16(b, n_pairs, true, st);
  }
  if (L.vbuf) {  // energy only, with a V buffer: the same two kernels, nothing stored
    b.T = L.vbuf;
    const hipError_t e = launch_pair_v_bf16(b, L.ns, n_pairs, st);
    if (e != hipSuccess) return e;
    return launch_pair_epi_bf16(b, n_pairs, false, st);
  }
  return hipErrorInvalidValue;  // BF16 needs amplitudes to store or a V buffer
}

// Density of amplitude matrices already in memory (matrix p at T + slot[p] n_v^2)
// with per-pair weights pw, on the pass's sliced path: row data (maxima and
// diagonal partials), operand slices (BF16) or digits (INT8), then the sliced
// density product accumulated into Dpart and the exact diagonal into diag.  Used
// by the active blocks only, whose stage timer covers it: it opens none of its own.
static int sliced_density(const PassPlan& pl, const double* T, const int* slot, const int2* pairs, const double* pw,
                          int np, double* Dpart, char* ws, hipStream_t s) {
  hipError_t e;
  auto* tmax = reinterpret_cast<unsigned long long*>(ws + pl.off_tmax);
  double* dgp = reinterpret_cast<double*>(ws + pl.off_dg);
  double* diag = reinterpret_cast<double*>(ws + pl.off_diag);
  if (pl.precision == DFPT2_INT8_SLICED) {
    {  // one exponent per row: the row maxima first
      if ((e = launch_fill(reinterpret_cast<double*>(tmax), (size_t)np * 4 * pl.n_v_pad_d, 0.0, s)) != hipSuccess)
        return hip_fail(e, "fill");
      if ((e = launch_pair_row_stats(T, slot, np, pl.n_v, pl.n_v_pad_d, tmax, dgp, s)) != hipSuccess)
        return hip_fail(e, "amplitude row data");
    }
    int8_t* Ts = reinterpret_cast<int8_t*>(ws + pl.off_Ts);
    int* Texp = reinterpret_cast<int*>(ws + pl.off_Texp);
    {
      if ((e = launch_split_t_i8(T, slot, pairs, pw, 1.0, np, pl.n_v, pl.n_v_pad_d, pl.ns2, tmax, dgp, Ts, Texp, diag,
                                 s)) != hipSuccess)
        return hip_fail(e, "amplitude digits");
    }
    DensityDigitArgs dd{};
    dd.Ts = Ts;
    dd.rexp = Texp;
    dd.pw = pw;
    dd.pairs = pairs;
    dd.Dpart = Dpart;
    dd.n_v = pl.n_v;
    dd.n_v_pad = pl.n_v_pad_d;
    dd.nt = pl.nt;
    dd.nTP = pl.nTP;
    dd.n_pairs = np;
    dd.nsplit = pl.nsplit2 < np ? pl.nsplit2 : np;
    dd.w = 1.0;
    dd.accumulate = 1;
    if ((e = launch_density_i8(dd, pl.ns2, s)) != hipSuccess) return hip_fail(e, "density kernel (INT8)");
    return DFPT2_OK;
  }
  __bf16* Ts = reinterpret_cast<__bf16*>(ws + pl.off_Ts);
  {
    if ((e = launch_split_t_bf16(T, slot, pairs, pw, 1.0, np, pl.n_v, pl.n_v_pad_d, pl.n_v_rows_t, pl.ns2, dgp, Ts,
                                 diag, s)) != hipSuccess)
      return hip_fail(e, "amplitude split");
  }
  DensitySlicedArgs ds{};
  ds.Ts = Ts;
  ds.pw = pw;
  ds.pairs = pairs;
  ds.Dpart = Dpart;
  ds.n_v = pl.n_v;
  ds.n_v_pad = pl.n_v_pad_d;
  ds.nt = pl.nt;
  ds.nTP = pl.nTD;
  ds.rows_pad = pl.n_v_rows_t;
  ds.n_pairs = np;
  ds.nsplit = pl.nsplit2 < np ? pl.nsplit2 : np;
  ds.w = 1.0;
  ds.accumulate = 1;
  if ((e = launch_density_bf16(ds, pl.ns2, s)) != hipSuccess) return hip_fail(e, "density kernel (BF16)");
  return DFPT2_OK;
}

// Active blocks of the pass (row a6): core-active pairs in batches of cores, then
// the active-active block; amplitudes and renormalized integrals are rotated to
// the natural basis of Gamma_act and fed to the density kernel with weights.
static int run_active_blocks(const PassPlan& pl, const dfpt2_opts& o, const double* eps_h, const double* eps_v,
                             const double* gamma_act, const PairLaunch& L, double* Dpart, double* pair_energy,
                             float* pair_tnorm, char* ws, hipStream_t s) {
  hipError_t e;
  const int na = pl.n_act, nv = pl.n_v;
  const long long mat = (long long)nv * nv;
  double* Tin = reinterpret_cast<double*>(ws + pl.off_act_T);
  double* Vin = reinterpret_cast<double*>(ws + pl.off_act_V);
  double* Tout = reinterpret_cast<double*>(ws + pl.off_act_Tr);
  double* Vout = reinterpret_cast<double*>(ws + pl.off_act_Vr);
  int2* pairs = reinterpret_cast<int2*>(ws + pl.off_act_pairs);
  int* slots = reinterpret_cast<int*>(ws + pl.off_act_slots);
  int2* pairs2 = reinterpret_cast<int2*>(ws + pl.off_act_pairs2);
  int* slots2 = reinterpret_cast<int*>(ws + pl.off_act_slots2);
  double* wd = reinterpret_cast<double*>(ws + pl.off_act_wd);
  double* we = reinterpret_cast<double*>(ws + pl.off_act_we);
  double* tpart = reinterpret_cast<double*>(ws + pl.off_act_tpart);
  double* tn2 = reinterpret_cast<double*>(ws + pl.off_act_tn2);
  double* epart = reinterpret_cast<double*>(ws + pl.off_act_epart);
  double* pe_act = reinterpret_cast<double*>(ws + pl.off_act_pe);
  double* occ = reinterpret_cast<double*>(ws + pl.off_act_occ);
  double* Ua = reinterpret_cast<double*>(ws + pl.off_act_U);
  double* Wk = reinterpret_cast<double*>(ws + pl.off_act_W);
  const double scale_d = pl.w_density / 2.0;

  // natural orbitals of the active density: Gamma_act = U diag(n) U^T
  int st = eigh_run(gamma_act, na, occ, Ua, ws + pl.off_act_eig, pl.act_eig_bytes, s, 0);
  if (st != DFPT2_OK) return st;
  // the kept-space energy (energy only) times its active blocks with its core pairs
  ProfScope prof(pl.energy_only ? DFPT2_STAGE_KEPT_PAIR : DFPT2_STAGE_ACTIVE, s);
  if ((e = launch_kron_uu(Ua, na, Wk, s)) != hipSuccess) return hip_fail(e, "kron");

  PairKernelArgs pa{};
  pa.B = L.B;
  pa.eps_h = eps_h;
  pa.eps_v = eps_v;
  pa.n_v = nv;
  pa.n_aux = pl.n_aux;
  pa.nt = pl.nt;
  pa.nTP = pl.nTP1;
  pa.s = o.s;
  pa.e_weight = 1.0;
  pa.T = Tin;
  pa.Vr = Vin;
  pa.epart = nullptr;
  pa.tpart = tpart;
  pa.pairs = pairs;

  DensityKernelArgs da{};
  da.T = Tout;
  da.n_v = nv;
  da.nt = pl.nt;
  da.nTP = pl.nTP;
  da.w = 1.0;
  da.pw = wd;
  da.Dpart = Dpart;
  da.accumulate = 1;
  const int ntile = pl.nt * pl.nt;

  // core-active: T'_{mk} = sum_u U_uk T_{mu}, weight n_k
  for (int m0 = 0; m0 < pl.n_core; m0 += pl.cpb) {
    const int nc = (pl.n_core - m0 < pl.cpb) ? pl.n_core - m0 : pl.cpb;
    const int np = nc * na;
    if ((e = launch_build_active_pairs(0, m0, nc, pl.n_core, na, pairs, slots, s)) != hipSuccess)
      return hip_fail(e, "active pairs");
    if ((e = launch_pair(L, pa, np, s)) != hipSuccess) return hip_fail(e, "pair kernel (core-active)");
    if ((e = launch_pair_reduce(nullptr, tpart, pl.nTP1, np, nullptr, tn2, s)) != hipSuccess)
      return hip_fail(e, "pair reduce");
    if ((e = launch_scatter_active_pair_info(pairs, tn2, np, pl.n_h, pair_energy, pair_tnorm, s)) != hipSuccess)
      return hip_fail(e, "scatter");
    if (na <= 32) {  // streamed: each stack through HBM once
      if ((e = launch_rotate_stack(Ua, na, Tin, Tout, mat, nc, s)) != hipSuccess) return hip_fail(e, "rotate T");
      if ((e = launch_rotate_stack(Ua, na, Vin, Vout, mat, nc, s)) != hipSuccess) return hip_fail(e, "rotate V");
    } else {
      if ((e = gemm_f64(Ua, na, 0, 1, Tin, (int)mat, mat * na, 0, Tout, (int)mat, mat * na, na, (int)mat, na, nc, 1.0,
                        0.0, s)) != hipSuccess)
        return hip_fail(e, "rotate T");
      if ((e = gemm_f64(Ua, na, 0, 1, Vin, (int)mat, mat * na, 0, Vout, (int)mat, mat * na, na, (int)mat, na, nc, 1.0,
                        0.0, s)) != hipSuccess)
        return hip_fail(e, "rotate V");
    }
    if ((e = launch_active_weights(0, np, pl.n_core, na, pairs, occ, scale_d, wd, we, s)) != hipSuccess)
      return hip_fail(e, "weights");
    if ((e = launch_rotated_energy(Tout, Vout, slots, np, nv, epart, s)) != hipSuccess)
      return hip_fail(e, "rotated energy");
    if ((e = launch_weighted_pair_reduce(epart, ntile, np, we, pe_act + 2 * (size_t)m0 * na, s)) != hipSuccess)
      return hip_fail(e, "weighted reduce");
    if (pl.energy_only) continue;
    if (pl.ns2 >= 2) {  // the pass's sliced density path, with the weights n_k
      if ((st = sliced_density(pl, Tout, slots, pairs, wd, np, Dpart, ws, s)) != DFPT2_OK) return st;
      continue;
    }
    da.pairs = pairs;
    da.slot = slots;
    da.n_pairs = np;
    da.nsplit = pl.nsplit < np ? pl.nsplit : np;
    if ((e = launch_density_f64(da, s)) != hipSuccess) return hip_fail(e, "density (core-active)");
  }

  // active-active: all ordered (u, v), rotated with U (x) U, then unordered k <= l
  {
    const int np = na * na;
    if ((e = launch_build_active_pairs(1, 0, 0, pl.n_core, na, pairs, slots, s)) != hipSuccess)
      return hip_fail(e, "active pairs");
    if ((e = launch_pair(L, pa, np, s)) != hipSuccess) return hip_fail(e, "pair kernel (active-active)");
    if ((e = launch_pair_reduce(nullptr, tpart, pl.nTP1, np, nullptr, tn2, s)) != hipSuccess)
      return hip_fail(e, "pair reduce");
    if ((e = launch_scatter_active_pair_info(pairs, tn2, np, pl.n_h, pair_energy, pair_tnorm, s)) != hipSuccess)
      return hip_fail(e, "scatter");
    if ((e = gemm_f64(Wk, np, 0, 1, Tin, (int)mat, 0, 0, Tout, (int)mat, 0, np, (int)mat, np, 1, 1.0, 0.0, s)) !=
        hipSuccess)
      return hip_fail(e, "rotate T");
    if ((e = gemm_f64(Wk, np, 0, 1, Vin, (int)mat, 0, 0, Vout, (int)mat, 0, np, (int)mat, np, 1, 1.0, 0.0, s)) !=
        hipSuccess)
      return hip_fail(e, "rotate V");
    const int nu = pl.n_aa_un;
    if ((e = launch_build_active_pairs(2, 0, 0, pl.n_core, na, pairs2, slots2, s)) != hipSuccess)
      return hip_fail(e, "active pairs");
    if ((e = launch_active_weights(2, nu, pl.n_core, na, pairs2, occ, scale_d, wd, we, s)) != hipSuccess)
      return hip_fail(e, "weights");
    if ((e = launch_rotated_energy(Tout, Vout, slots2, nu, nv, epart, s)) != hipSuccess)
      return hip_fail(e, "rotated energy");
    if ((e = launch_weighted_pair_reduce(epart, ntile, nu, we, pe_act + 2 * (size_t)pl.n_ca, s)) != hipSuccess)
      return hip_fail(e, "weighted reduce");
    if (!pl.energy_only && pl.ns2 >= 2) {
      if ((st = sliced_density(pl, Tout, slots2, pairs2, wd, nu, Dpart, ws, s)) != DFPT2_OK) return st;
    } else if (!pl.energy_only) {
      da.pairs = pairs2;
      da.slot = slots2;
      da.n_pairs = nu;
      da.nsplit = pl.nsplit < nu ? pl.nsplit : nu;
      if ((e = launch_density_f64(da, s)) != hipSuccess) return hip_fail(e, "density (active-active)");
    }
  }
  return DFPT2_OK;
}

int run_pass(const PassPlan& pl, const dfpt2_opts& o, const double* eps_h, const double* eps_v,
             const double* gamma_act, const double* B, const uint8_t* mask, double* D, double* e_out,
             double* pair_energy, float* pair_tnorm, char* ws, hipStream_t s) {
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

  PairLaunch L{pl.precision, pl.ns1, B, nullptr, nullptr, nullptr, pl.n_v_pad, pl.n_aux_pad, nullptr};
  if (pl.energy_only && (pl.precision == DFPT2_BF16_SLICED || pl.precision == DFPT2_INT8_SLICED))
    L.vbuf = reinterpret_cast<double*>(ws + pl.off_T);
  if (!pl.energy_only && pl.precision == DFPT2_BF16_SLICED && pl.ns2 >= 2) {
    L.ts = reinterpret_cast<__bf16*>(ws + pl.off_Ts);
    L.dgp = reinterpret_cast<double*>(ws + pl.off_dg);
    L.ns2 = pl.ns2;
    L.rows_t = pl.n_v_rows_t;
  }
  // d_count[0]: pairs of the mask; d_count[1]: set by the BF16 split when a row of B
  // lies below the range its slices need (both read back with one copy below)
  if ((e = launch_fill(reinterpret_cast<double*>(d_count), 2, 0.0, s)) != hipSuccess) return hip_fail(e, "fill");
  if (pl.precision != DFPT2_FP64) {
    ProfScope ps(DFPT2_STAGE_SPLIT, s);
    double* nrm = reinterpret_cast<double*>(ws + pl.off_norm2);
    L.norm2 = nrm;
    L.Bs = ws + pl.off_Bs;
    if (pl.precision == DFPT2_BF16_SLICED) {
      if ((e = launch_split_rows_bf16(B, pl.n_aux, pl.n_h, pl.n_v, pl.n_v_pad, pl.n_aux, pl.n_aux_pad, pl.ns1,
                                      reinterpret_cast<__bf16*>(ws + pl.off_Bs), nrm, d_count + 1, s)) != hipSuccess)
        return hip_fail(e, "split");
    } else if (pl.precision == DFPT2_INT8_SLICED) {
      int* rexp = reinterpret_cast<int*>(ws + pl.off_rexp);
      L.rexp = rexp;
      if ((e = launch_split_rows_i8(B, pl.n_aux, pl.n_h, pl.n_v, pl.n_v_pad, pl.n_aux, pl.n_aux_pad, pl.ns1,
                                    reinterpret_cast<int8_t*>(ws + pl.off_Bs), rexp, nrm, s)) != hipSuccess)
        return hip_fail(e, "split");
    } else {
      uint32_t* sc = reinterpret_cast<uint32_t*>(ws + pl.off_scales);
      L.scales = sc;
      if ((e = launch_split_rows_fp8(B, pl.n_aux, pl.n_h, pl.n_v, pl.n_v_pad, pl.n_aux, pl.n_aux_pad, pl.ns1,
                                     reinterpret_cast<uint8_t*>(ws + pl.off_Bs), sc, nrm, s)) != hipSuccess)
        return hip_fail(e, "split");
    }
  }
  {
    ProfScope ps(DFPT2_STAGE_REDUCE, s);
    if ((e = launch_build_pairs(mask, pl.n_core, pl.n_h, pairs, d_count, s)) != hipSuccess)
      return hip_fail(e, "build_pairs");
  }
  int cnt[2] = {0, 0};
  if ((e = hipMemcpyAsync(cnt, d_count, sizeof(cnt), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "count copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream sync");
  const int count = cnt[0];
  if (cnt[1] != 0)
    return fail(DFPT2_ERR_UNSUPPORTED,
                "BF16 slicing: a row of B has max |B^Q_ia| below 2^%d, where products of its %d slices leave the "
                "normal FP32 range; rescale the integrals or use FP64 or INT8 digits",
                bf16_min_row_exponent(pl.ns1) - 1, pl.ns1);

  if (pair_energy) {
    // core-core entries start at 0 (masked pairs stay 0); pairs with an active hole are NaN
    if ((e = launch_fill(pair_energy, (size_t)pl.n_h * pl.n_h, 0.0, s)) != hipSuccess)
      return hip_fail(e, "fill");
  }
  if (pair_tnorm) {
    if ((e = launch_fill_f32(pair_tnorm, (size_t)pl.n_h * pl.n_h, 0.0f, s)) != hipSuccess)
      return hip_fail(e, "fill");
  }

  if (!pl.energy_only) {
    ProfScope ps(DFPT2_STAGE_REDUCE, s);
    if ((e = launch_fill(Dpart, mat * pl.nsplit_all, 0.0, s)) != hipSuccess) return hip_fail(e, "fill");
    if (pl.ns2 >= 2 && (e = launch_fill(reinterpret_cast<double*>(ws + pl.off_diag), pl.n_v, 0.0, s)) != hipSuccess)
      return hip_fail(e, "fill");
  }
  const int stage_pair = pl.energy_only ? DFPT2_STAGE_KEPT_PAIR : DFPT2_STAGE_PAIR;
  PairKernelArgs pa{};
  pa.B = B;
  pa.eps_h = eps_h;
  pa.eps_v = eps_v;
  pa.n_v = pl.n_v;
  pa.n_aux = pl.n_aux;
  pa.nt = pl.nt;
  pa.nTP = pl.nTP1;
  pa.s = o.s;
  pa.e_weight = 1.0;  // 1/4 gamma_ii gamma_jj with gamma = 2 for core holes
  pa.T = pl.energy_only ? nullptr : T;
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
    if (pl.ns2 >= 2 && pl.precision == DFPT2_INT8_SLICED) {  // row maxima and diagonal partials for the digits
      pa.tmax = reinterpret_cast<unsigned long long*>(ws + pl.off_tmax);
      pa.dgp = reinterpret_cast<double*>(ws + pl.off_dg);
      ProfScope ps(DFPT2_STAGE_SPLIT_T, s);
      if ((e = launch_fill(reinterpret_cast<double*>(pa.tmax), (size_t)np * 4 * pl.n_v_pad_d, 0.0, s)) != hipSuccess)
        return hip_fail(e, "fill");
    }
    {
      ProfScope ps(stage_pair, s);
      if ((e = launch_pair(L, pa, np, s, &ps)) != hipSuccess) return hip_fail(e, "pair kernel");
    }
    {
      ProfScope ps(DFPT2_STAGE_REDUCE, s);
      if ((e = launch_pair_reduce(epart, tpart, pl.nTP1, np, pe + 2 * (size_t)p0, tn2 + p0, s)) != hipSuccess)
        return hip_fail(e, "pair reduce");
    }
    if (pl.energy_only) continue;
    if (pl.ns2 >= 2 && pl.precision == DFPT2_INT8_SLICED) {
      int8_t* Ts = reinterpret_cast<int8_t*>(ws + pl.off_Ts);
      int* Texp = reinterpret_cast<int*>(ws + pl.off_Texp);
      {
        ProfScope ps(DFPT2_STAGE_SPLIT_T, s);
        if ((e = launch_split_t_i8(T, nullptr, pairs + p0, nullptr, pl.w_density, np, pl.n_v, pl.n_v_pad_d, pl.ns2, pa.tmax,
                                   pa.dgp, Ts, Texp, reinterpret_cast<double*>(ws + pl.off_diag), s)) != hipSuccess)
          return hip_fail(e, "amplitude digits");
      }
      DensityDigitArgs dd{};
      dd.Ts = Ts;
      dd.rexp = Texp;
      dd.pw = nullptr;
      dd.pairs = pairs + p0;
      dd.Dpart = Dpart;
      dd.n_v = pl.n_v;
      dd.n_v_pad = pl.n_v_pad_d;
      dd.nt = pl.nt;
      dd.nTP = pl.nTP;
      dd.n_pairs = np;
      dd.nsplit = pl.nsplit2 < np ? pl.nsplit2 : np;
      dd.w = pl.w_density;
      dd.accumulate = 1;
      ProfScope ps(DFPT2_STAGE_DENSITY, s);
      if ((e = launch_density_i8(dd, pl.ns2, s)) != hipSuccess) return hip_fail(e, "density kernel (INT8)");
      continue;
    }
    if (pl.ns2 >= 2) {  // the epilogue wrote the slices and the diagonal partials
      __bf16* Ts = L.ts;
      {
        ProfScope ps(DFPT2_STAGE_SPLIT_T, s);
        if ((e = launch_diag_accumulate(L.dgp, pairs + p0, nullptr, pl.w_density, np, pl.n_v, pl.n_v_pad_d,
                                        reinterpret_cast<double*>(ws + pl.off_diag), s)) != hipSuccess)
          return hip_fail(e, "density diagonal");
      }
      DensitySlicedArgs ds{};
      ds.Ts = Ts;
      ds.pw = nullptr;
      ds.pairs = pairs + p0;
      ds.Dpart = Dpart;
      ds.n_v = pl.n_v;
      ds.n_v_pad = pl.n_v_pad_d;
      ds.nt = pl.nt;
      ds.nTP = pl.nTD;
      ds.rows_pad = pl.n_v_rows_t;
      ds.n_pairs = np;
      ds.nsplit = pl.nsplit2 < np ? pl.nsplit2 : np;
      ds.w = pl.w_density;
      ds.accumulate = 1;
      ProfScope ps(DFPT2_STAGE_DENSITY, s);
      if ((e = launch_density_bf16(ds, pl.ns2, s)) != hipSuccess) return hip_fail(e, "density kernel (BF16)");
      continue;
    }
    da.pairs = pairs + p0;
    da.n_pairs = np;
    da.nsplit = pl.nsplit < np ? pl.nsplit : np;
    da.Dpart = Dpart;
    da.accumulate = 1;
    {
      ProfScope ps(DFPT2_STAGE_DENSITY, s);
      if ((e = launch_density_f64(da, s)) != hipSuccess) return hip_fail(e, "density kernel");
    }
  }
  if (pl.n_act > 0) {
    PairLaunch La = L;  // the active blocks store FP64 amplitudes and rotate them
    La.ts = nullptr;
    La.dgp = nullptr;
    int st = run_active_blocks(pl, o, eps_h, eps_v, gamma_act, La, Dpart, pair_energy, pair_tnorm, ws, s);
    if (st != DFPT2_OK) return st;
  }
  {
    ProfScope ps_tail(DFPT2_STAGE_REDUCE, s);
    if (!pl.energy_only) {
      const double* diag = pl.ns2 >= 2 ? reinterpret_cast<const double*>(ws + pl.off_diag) : nullptr;
      if ((e = launch_density_reduce(Dpart, pl.nsplit_all, pl.n_v, diag, D, s)) != hipSuccess)
        return hip_fail(e, "density reduce");
    }
    if ((e = launch_energy_finalize(pe, tn2, pairs, d_count, pl.n_up, pl.n_h, e_out, pair_energy, pair_tnorm,
                                    s)) != hipSuccess)
      return hip_fail(e, "energy finalize");
    if (pl.n_act > 0) {
      const double* pe_act = reinterpret_cast<const double*>(ws + pl.off_act_pe);
      if ((e = launch_energy_finalize_active(pe, d_count, pe_act, pl.n_ca + pl.n_aa_un, e_out, s)) != hipSuccess)
        return hip_fail(e, "energy finalize (active)");
    }
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
