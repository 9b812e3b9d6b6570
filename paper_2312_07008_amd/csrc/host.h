// Host-side plan of one pass and internal entry points (not exported).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/dfpt2.h"
#include "kernels.h"

namespace dfpt2 {

extern thread_local std::string g_last_error;
int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
size_t align_up(size_t x, size_t a);

struct PassPlan {
  int n_core, n_act, n_h, n_v, n_aux;
  int nt, nTP;      // 64-wide virtual tiles and upper-triangle tile pairs
  int nTP1;         // pair-kernel workgroup tiles per pair (energy partials per pair)
  int n_up;         // unordered core-core pairs
  int batch;        // unordered pairs per batch
  int nsplit;       // density split slices (FP64 density kernel)
  int nsplit2;      // density split slices (split-BF16 density kernel)
  int nsplit_all;   // slices of Dpart: max(nsplit, nsplit2)
  int ns2;          // slices per operand of the density product (1 = FP64 density)
  double w_density; // density weight of one ordered closed-shell pair
  int precision;    // dfpt2_precision
  bool energy_only; // no amplitudes stored, no density (kept-space energy)
  int ns1;          // slices per operand of the pair product (mixed precision)
  int n_v_pad, n_aux_pad;  // slab rows and columns of the sliced operands
  int n_v_pad_d;           // 64-multiple of n_v: layout of the density slices and row data
  int n_v_rows_t;          // rows per density operand matrix (128-multiple for the BF16 density kernel)
  int nTD;                 // workgroup tiles of the split-BF16 density kernel
  size_t off_pairs, off_count, off_T, off_epart, off_tpart, off_pe, off_tn2, off_Dpart, off_Bs, off_scales, off_norm2, off_rexp, off_Ts, off_Texp, off_dg, off_tmax, off_diag;
  // active holes
  int n_ca, n_aa_un, cpb, act_cap;
  size_t off_act_T, off_act_V, off_act_Tr, off_act_Vr, off_act_pairs, off_act_slots, off_act_pairs2,
      off_act_slots2, off_act_wd, off_act_we, off_act_tpart, off_act_tn2, off_act_epart, off_act_pe, off_act_occ,
      off_act_U, off_act_W, off_act_eig;
  size_t act_eig_bytes;
  size_t ws_bytes;
};

int plan_pass(const dfpt2_opts* o, PassPlan* pl, bool energy_only = false);

int run_pass(const PassPlan& pl, const dfpt2_opts& o, const double* eps_h, const double* eps_v,
             const double* gamma_act, const double* B, const uint8_t* mask, double* D, double* e_out,
             double* pair_energy, float* pair_tnorm, char* ws, hipStream_t s);

// Pair-kernel launcher shared by the pass and the kept-space energy: FP64, or
// split BF16 / FP8 / INT8 from the slices in `Bs` (and FP8 block scales in
// `scales`, INT8 row exponents in `rexp`),
// prepared by the caller.
struct PairLaunch {
  int precision, ns;
  const double* B;
  const void* Bs;
  const uint32_t* scales;
  const int* rexp;  // INT8 row exponents
  int n_v_pad, n_aux_pad;
  const double* norm2;
  double* vbuf = nullptr;  // BF16 energy-only passes: V of one batch for the epilogue kernel
  // BF16 passes with the split-BF16 density: the epilogue writes the density
  // operands' slices (ns2 per operand, matrices rows_t rows apart) to ts and the
  // diagonal partials to dgp instead of storing FP64 amplitudes
  __bf16* ts = nullptr;
  double* dgp = nullptr;
  int ns2 = 0, rows_t = 0;
};
class ProfScope;
// `product` (may be null): the caller's timer of the pair product; where the
// epilogue runs as a kernel of its own and that timer is the main pass's
// (DFPT2_STAGE_PAIR), it is closed after the product and the epilogue is timed as
// DFPT2_STAGE_PAIR_EPILOGUE; otherwise the epilogue stays in the caller's stage
hipError_t launch_pair(const PairLaunch& L, const PairKernelArgs& a, int n_pairs, hipStream_t st,
                       ProfScope* product = nullptr);
int default_slices_gemm1(int precision);

// Stage timer scope (see dfpt2_profile_enable); no-op unless profiling is on, and
// for a negative stage.
class ProfScope {
 public:
  ProfScope(int stage, hipStream_t s);
  ~ProfScope() { close(); }
  void close();  // records the end event now; later calls and the destructor do nothing
  int stage() const { return stage_; }
 private:
  int stage_;
  hipStream_t s_;
  hipEvent_t a_;
};
void prof_flush();

hipError_t gemm_f64(const double* A, int lda, long long sA, int transA, const double* B, int ldb, long long sB,
                    int transB, double* C, int ldc, long long sC, int M, int N, int K, int batch, double alpha,
                    double beta, hipStream_t st);

}  // namespace dfpt2
