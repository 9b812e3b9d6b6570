// Density-fitted particle-particle ladder (the N_C^2 N_V^4 part of the two-body
// contraction C2 = [O2, T2]_2 of the high-level step, Eq. 6), in the full or in
// the truncated virtual space, whose cost the FNO truncation cuts by
// (N_V'/N_V)^4 (Sec. 2):
//     (ac|bd) = sum_Q B^Q_ac B^Q_bd,     R^p_ab = sum_cd (ac|bd) T^p_cd.
//
// Integral-direct in blocks of the first virtual a, as two FP64 MFMA GEMMs per
// block (flops 2 N^4 n_aux + 2 N^4 n_amp in total, both proportional to N^4):
//   G[(a,c)][(d,b)] = sum_Q B[(a,c)][Q] B[(d,b)][Q]      (rows a of the block)
//   R[p][a][b]      = sum_(c,d) T[p][(c,d)] G[(a,c,d)][b]
// The first product reads the columns of (ac|bd) in (d,b) order, which is
// (b,d) order of B because density-fitted integrals are symmetric in their two
// orbital indices (B^Q_db = B^Q_bd); that lays G out as [(c,d)][b] per a, the
// operand the second product contracts over (c,d).  G of one block holds
// m_a N^3 doubles (m_a <= 32 values of a, at most ~16 GB, at least one a): the
// contraction runs as m_a batched GEMMs of n_amp x N, so m_a sets its parallelism.
//
// Truncated space: with the kept NOs X [N_V][ldx] (first N' columns) the inputs are transformed
// first, B'^Q = X^T B^Q X (over both virtual indices of B[a][c][Q]) and
// T'^p = X^T T^p X, by four more GEMMs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/dfpt2.h"
#include "common.h"
#include "host.h"

namespace dfpt2 {
namespace {

struct LadderPlan {
  int n, nk, na, np, ma;
  bool transform;
  size_t off_Y, off_Bk, off_Z, off_Tk, off_G, bytes;
};

constexpr double kGBlockBytes = 16.0e9;  // one block of (ac|bd): enough values of a to fill the GPU
constexpr int kMaxBlockRows = 32;  // values of a per block

int plan_ladder(int64_t n_vir, int64_t n_aux, int64_t n_amp, int64_t n_kept, bool transform, LadderPlan* pl) {
  if (n_vir < 1 || n_vir > 2048) return fail(DFPT2_ERR_INVALID_ARG, "n_vir must lie in [1, 2048]");
  if (n_aux < 1 || n_aux > (1 << 20)) return fail(DFPT2_ERR_INVALID_ARG, "n_aux must lie in [1, 2^20]");
  if (n_amp < 1 || n_amp > 65535) return fail(DFPT2_ERR_INVALID_ARG, "n_amp must lie in [1, 65535]");
  if (transform) {
    if (n_kept < 1 || n_kept > n_vir) return fail(DFPT2_ERR_INVALID_ARG, "n_kept must lie in [1, n_vir]");
  } else if (n_kept != 0 && n_kept != n_vir) {
    return fail(DFPT2_ERR_INVALID_ARG, "without X, n_kept must be 0 or n_vir");
  }
  LadderPlan& p = *pl;
  p = LadderPlan{};
  p.n = (int)n_vir;
  p.nk = transform ? (int)n_kept : (int)n_vir;
  p.na = (int)n_aux;
  p.np = (int)n_amp;
  p.transform = transform;
  const double n3 = (double)p.nk * p.nk * p.nk * sizeof(double);
  p.ma = std::max(1, std::min({p.nk, kMaxBlockRows, (int)(kGBlockBytes / n3)}));
  if ((double)p.nk * p.na > 2.0e9 || (double)p.nk * p.nk > 2.0e9)
    return fail(DFPT2_ERR_INVALID_ARG, "ladder operands exceed the GEMM index range");
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align_up(off + b, 256);
    return o;
  };
  const size_t d = sizeof(double);
  p.off_Y = take(transform ? d * p.n * p.nk * p.na : 0);
  p.off_Bk = take(transform ? d * p.nk * p.nk * p.na : 0);
  p.off_Z = take(transform ? d * p.np * p.n * p.nk : 0);
  p.off_Tk = take(transform ? d * p.np * p.nk * p.nk : 0);
  p.off_G = take(d * (size_t)p.ma * p.nk * p.nk * p.nk);
  p.bytes = off;
  return DFPT2_OK;
}

}  // namespace
}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int pp_ladder_workspace_size(int64_t n_vir, int64_t n_aux, int64_t n_amp, int64_t n_kept, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  LadderPlan p;
  const int st = plan_ladder(n_vir, n_aux, n_amp, n_kept, n_kept != 0, &p);
  if (st != DFPT2_OK) return st;
  *bytes = p.bytes;
  return DFPT2_OK;
}

int pp_ladder(int64_t n_vir, int64_t n_aux, int64_t n_amp, const double* B_vv, const double* T, const double* X,
              int64_t ldx, int64_t n_kept, double* R, void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!B_vv || !T || !R || !workspace) return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  LadderPlan p;
  if (!X && n_kept != 0 && n_kept != n_vir) return fail(DFPT2_ERR_INVALID_ARG, "without X, n_kept must be 0 or n_vir");
  int st = plan_ladder(n_vir, n_aux, n_amp, X ? n_kept : 0, X != nullptr, &p);
  if (st != DFPT2_OK) return st;
  if (X && (ldx < n_kept || ldx > n_vir)) return fail(DFPT2_ERR_INVALID_ARG, "ldx must lie in [n_kept, n_vir]");
  if (ws_bytes < p.bytes) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p.bytes);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  hipError_t e;
  const int n = p.n, nk = p.nk, na = p.na, np = p.np, lx = X ? (int)ldx : 0;
  const double* Bk = B_vv;
  const double* Tk = T;
  if (p.transform) {
    ProfScope ps(DFPT2_STAGE_LADDER_TRANSFORM, s);
    double* Y = reinterpret_cast<double*>(ws + p.off_Y);
    double* Bt = reinterpret_cast<double*>(ws + p.off_Bk);
    double* Z = reinterpret_cast<double*>(ws + p.off_Z);
    double* Tt = reinterpret_cast<double*>(ws + p.off_Tk);
    // Y[a] = X^T B[a]  (nk x na per a)
    if ((e = gemm_f64(X, lx, 0, 1, B_vv, na, (long long)n * na, 0, Y, na, (long long)nk * na, nk, na, n, n, 1.0, 0.0,
                      s)) != hipSuccess)
      return hip_fail(e, "ladder transform (B, first index)");
    // B'[a'][(c', Q)] = sum_a X[a][a'] Y[a][(c', Q)]
    if ((e = gemm_f64(X, lx, 0, 1, Y, nk * na, 0, 0, Bt, nk * na, 0, nk, nk * na, n, 1, 1.0, 0.0, s)) != hipSuccess)
      return hip_fail(e, "ladder transform (B, second index)");
    // Z[p] = T[p] X, T'[p] = X^T Z[p]
    if ((e = gemm_f64(T, n, (long long)n * n, 0, X, lx, 0, 0, Z, nk, (long long)n * nk, n, nk, n, np, 1.0, 0.0, s)) !=
        hipSuccess)
      return hip_fail(e, "ladder transform (T)");
    if ((e = gemm_f64(X, lx, 0, 1, Z, nk, (long long)n * nk, 0, Tt, nk, (long long)nk * nk, nk, nk, n, np, 1.0, 0.0,
                      s)) != hipSuccess)
      return hip_fail(e, "ladder transform (T)");
    Bk = Bt;
    Tk = Tt;
  }
  {
    ProfScope ps(DFPT2_STAGE_LADDER, s);
    double* G = reinterpret_cast<double*>(ws + p.off_G);
    const int N2 = nk * nk;
    for (int a0 = 0; a0 < nk; a0 += p.ma) {
      const int mb = std::min(p.ma, nk - a0);
      // G[(a,c)][(d,b)] = sum_Q B'[(a,c)][Q] B'[(d,b)][Q] for a in [a0, a0 + mb)
      if ((e = gemm_f64(Bk + (size_t)a0 * nk * na, na, 0, 0, Bk, na, 0, 1, G, N2, 0, mb * nk, N2, na, 1, 1.0, 0.0,
                        s)) != hipSuccess)
        return hip_fail(e, "ladder integrals");
      // R[p][a][b] = sum_(c,d) T'[p][(c,d)] G[a][(c,d)][b]
      if ((e = gemm_f64(Tk, N2, 0, 0, G, nk, (long long)N2 * nk, 0, R + (size_t)a0 * nk, N2, nk, np, nk, N2, mb, 1.0,
                        0.0, s)) != hipSuccess)
        return hip_fail(e, "ladder contraction");
    }
  }
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "ladder launch");
  return DFPT2_OK;
}

}  // extern "C"
