// Eq. A9 terms whose amplitudes carry an active particle index (zero density
// cumulants, no singles):
//     t^{ev}_{mn} tc^{fu}_{mn} eta^u_v
//   + 1/2 S( t^{ey}_{mu} tc^{fx}_{mv} ) Gamma^u_v eta^x_y
//   + 1/4 t^{ez}_{ux} tc^{fw}_{vy} Gamma^u_v Gamma^x_y eta^w_z
// with t^{ex}_{ij} = <ex|ij> (1 - e^{-s Delta^2}) / Delta (Eq. A7, particle
// indices e virtual and x active), tc^{ab}_{ij} = 2 t^{ab}_{ij} - t^{ab}_{ji} and
// eta = 2 - Gamma.  With w = gamma / 2 over the holes (1 on core holes, Gamma / 2
// on the active block) the three terms are one expression,
//     D_ef += sum_{ij} [ X_ij eta Z_ij^T ]_ef,   Z_ij = sum_{kl} w_ik w_jl Tc_kl,
// where X_ij[e][x] = t^{ex}_{ij}.  Every ordered hole pair and active particle
// is one column of an n_v x (n_h^2 n_act) matrix, so the work is
//   1. X[e][(i,j,x)] = sum_Q B^Q_ie B_act^Q_jx          (FP64 MFMA GEMM, batched over i)
//   2. regularizer (Eq. A7), then Tc = 2 X - X^(i<->j)    (elementwise)
//   3. Z = (w x w) Tc over the hole pair, Y = Z eta       (small kernel, GEMM batched over e)
//   4. E = X Y^T, D += (E + E^T) / 2                     (FP64 MFMA GEMM, symmetric add)
// The cost is O(n_h^2 n_act n_v (n_aux + n_v)): a few percent of the pass.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/dfpt2.h"
#include "common.h"
#include "host.h"

namespace dfpt2 {
namespace {

// X[e][i][j][x] *= (1 - exp(-s D^2)) / D,  D = eps_i + eps_j - eps_e - eps_(n_core + x)
__global__ void ap_regularize(double* X, const double* eps_h, const double* eps_v, int n_v, int n_h, int n_a,
                              int n_core, double s) {
  const size_t n = (size_t)n_v * n_h * n_h * n_a;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    size_t r = k;
    const int x = (int)(r % n_a);
    r /= n_a;
    const int j = (int)(r % n_h);
    r /= n_h;
    const int i = (int)(r % n_h);
    const int e = (int)(r / n_h);
    const double dl = eps_h[i] + eps_h[j] - eps_v[e] - eps_h[n_core + x];
    X[k] = (dl != 0.0) ? X[k] * (1.0 - exp(-s * dl * dl)) / dl : 0.0;
  }
}

// Z[e][i][j][x] = sum_{k,l} w_ik w_jl (2 X[e][k][l][x] - X[e][l][k][x]),
// w = identity on core holes and Gamma / 2 on the active block
__global__ void ap_pair_mix(const double* X, const double* gamma, double* Z, int n_v, int n_h, int n_a,
                            int n_core) {
  const size_t n = (size_t)n_v * n_h * n_h * n_a;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    size_t r = k;
    const int x = (int)(r % n_a);
    r /= n_a;
    const int j = (int)(r % n_h);
    r /= n_h;
    const int i = (int)(r % n_h);
    const size_t base = (r / n_h) * (size_t)n_h * n_h * n_a;
    const int k0 = i < n_core ? i : n_core, k1 = i < n_core ? i + 1 : n_h;
    const int l0 = j < n_core ? j : n_core, l1 = j < n_core ? j + 1 : n_h;
    double acc = 0.0;
    for (int kk = k0; kk < k1; ++kk) {
      const double wi = i < n_core ? 1.0 : 0.5 * gamma[(i - n_core) * n_a + (kk - n_core)];
      if (wi == 0.0) continue;
      double inner = 0.0;
      for (int ll = l0; ll < l1; ++ll) {
        const double wj = j < n_core ? 1.0 : 0.5 * gamma[(j - n_core) * n_a + (ll - n_core)];
        const double tc = 2.0 * X[base + ((size_t)kk * n_h + ll) * n_a + x] - X[base + ((size_t)ll * n_h + kk) * n_a + x];
        inner += wj * tc;
      }
      acc += wi * inner;
    }
    Z[k] = acc;
  }
}

__global__ void ap_eta(const double* gamma, int n_a, double* eta) {
  for (int k = threadIdx.x; k < n_a * n_a; k += blockDim.x) {
    const int u = k / n_a, v = k - u * n_a;
    eta[k] = (u == v ? 2.0 : 0.0) - gamma[k];
  }
}

// D += scale (E + E^T) / 2
__global__ void ap_sym_add(const double* E, double* D, int n_v, double scale) {
  const size_t n = (size_t)n_v * n_v;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t a = k / n_v, b = k - a * n_v;
    D[k] += 0.5 * scale * (E[k] + E[b * n_v + a]);
  }
}

struct ApPlan {
  int n_core, n_a, n_h, n_v, n_aux;
  size_t K;  // n_h^2 n_a
  size_t off_X, off_Z, off_Y, off_E, off_eta, bytes;
};

int plan_ap(const dfpt2_opts* o, ApPlan* p) {
  if (!o) return fail(DFPT2_ERR_INVALID_ARG, "opts is null");
  PassPlan pp;
  const int st = plan_pass(o, &pp);  // the same size checks as the pass
  if (st != DFPT2_OK) return st;
  *p = ApPlan{};
  p->n_core = (int)o->n_core;
  p->n_a = (int)o->n_act;
  p->n_h = p->n_core + p->n_a;
  p->n_v = (int)o->n_vir;
  p->n_aux = (int)o->n_aux;
  p->K = (size_t)p->n_h * p->n_h * p->n_a;
  if (p->K > 0x7fffffffULL || (double)p->n_h * p->n_a > 2.0e9)
    return fail(DFPT2_ERR_INVALID_ARG, "too many hole pairs x active orbitals");
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o_ = off;
    off = align_up(off + b, 256);
    return o_;
  };
  const size_t big = sizeof(double) * (size_t)p->n_v * p->K;
  p->off_X = take(big);
  p->off_Z = take(big);
  p->off_Y = take(big);
  p->off_E = take(sizeof(double) * (size_t)p->n_v * p->n_v);
  p->off_eta = take(sizeof(double) * (size_t)(p->n_a > 0 ? p->n_a * p->n_a : 1));
  p->bytes = off;
  return DFPT2_OK;
}

int grid_for(size_t n) {
  const size_t g = (n + 255) / 256;
  return (int)(g < 65535 ? (g > 0 ? g : 1) : 65535);
}

}  // namespace
}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int dfpt2_active_particle_workspace_size(const dfpt2_opts* opts, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  ApPlan p;
  const int st = plan_ap(opts, &p);
  if (st != DFPT2_OK) return st;
  *bytes = p.bytes;
  return DFPT2_OK;
}

int dfpt2_add_active_particle_density(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                                      const double* gamma_act, const double* B, const double* B_act, double* D_vv,
                                      void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  ApPlan p;
  int st = plan_ap(opts, &p);
  if (st != DFPT2_OK) return st;
  if (p.n_a == 0) return DFPT2_OK;  // no active particle index
  if (!eps_hole || !eps_vir || !gamma_act || !B || !B_act || !D_vv || !workspace)
    return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (ws_bytes < p.bytes) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p.bytes);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* X = reinterpret_cast<double*>(ws + p.off_X);
  double* Z = reinterpret_cast<double*>(ws + p.off_Z);
  double* Y = reinterpret_cast<double*>(ws + p.off_Y);
  double* E = reinterpret_cast<double*>(ws + p.off_E);
  double* eta = reinterpret_cast<double*>(ws + p.off_eta);
  const int n_v = p.n_v, n_h = p.n_h, n_a = p.n_a, na = p.n_aux;
  const int K = (int)p.K, NA = n_h * n_a;
  const size_t all = (size_t)n_v * p.K;
  hipError_t e;
  ProfScope ps(DFPT2_STAGE_ACTIVE, s);
  // 1. X[e][(i, j, x)] = sum_Q B[i][e][Q] B_act[(j, x)][Q]
  if ((e = gemm_f64(B, na, (long long)n_v * na, 0, B_act, na, 0, 1, X, K, NA, n_v, NA, na, n_h, 1.0, 0.0, s)) !=
      hipSuccess)
    return hip_fail(e, "active-particle integrals");
  // 2. amplitudes
  hipLaunchKernelGGL(ap_regularize, dim3(grid_for(all)), dim3(256), 0, s, X, eps_hole, eps_vir, n_v, n_h, n_a,
                     p.n_core, opts->s);
  // 3. Z = (w x w) Tc, Y = Z eta (batched over e: M = n_h^2, N = K = n_act)
  hipLaunchKernelGGL(ap_pair_mix, dim3(grid_for(all)), dim3(256), 0, s, X, gamma_act, Z, n_v, n_h, n_a, p.n_core);
  hipLaunchKernelGGL(ap_eta, dim3(1), dim3(256), 0, s, gamma_act, n_a, eta);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "active-particle kernels");
  if ((e = gemm_f64(Z, n_a, (long long)p.K, 0, eta, n_a, 0, 0, Y, n_a, (long long)p.K, n_h * n_h, n_a, n_a, n_v, 1.0,
                    0.0, s)) != hipSuccess)
    return hip_fail(e, "active-particle eta");
  // 4. E = X Y^T, D += (E + E^T) / 2 (per-spin convention: half)
  if ((e = gemm_f64(X, K, 0, 0, Y, K, 0, 1, E, n_v, 0, n_v, n_v, K, 1, 1.0, 0.0, s)) != hipSuccess)
    return hip_fail(e, "active-particle density");
  const double scale = opts->density_convention == 1 ? 0.5 : 1.0;
  hipLaunchKernelGGL(ap_sym_add, dim3(grid_for((size_t)n_v * n_v)), dim3(256), 0, s, E, D_vv, n_v, scale);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "active-particle add");
  return DFPT2_OK;
}

}  // extern "C"
