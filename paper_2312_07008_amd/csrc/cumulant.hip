// The first-order singles (Eq. A6) and the Eq. A9 terms that carry them or the
// two-body density cumulant lambda_uv^xy of the reference:
//     D1  2 t_e^m t_f^m + t_e^u t_f^v gamma_u^v
//     D2  (t_e^u t_fv^xy + t_ey^uv t_f^x) lambda_uv^xy
//     D3  t_ee'^uv t_fe'^xy lambda_uv^xy
//     D4  P( t_ey^mv t_fu^mx ) lambda_uv^xy
//     D5  1/2 t_ez^uv t_fw^xy eta_w^z lambda_uv^xy
//     D6  1/2 P( t_ey^wv t_fu^zx ) gamma_w^z lambda_uv^xy
// (t_ab^ij: particles a, b created, holes i, j annihilated; m core, u..z active,
// e, f, e' virtual; eta = 2 - gamma; P(t_ap^ij t_cd^kq) = 2 t_ap^ij t_cd^kq -
// t_ap^ij t_cd^qk - t_ap^ji t_cd^kq - t_aq^ji t_cd^pk) with the singles
//     t_e^i = 1/2 sum_ux (eps_x - eps_u) gamma_x^u tc_ex^iu (1 - e^{-s D^2}) / D,
//     D = eps_i - eps_e,  tc_ab^ij = 2 t_ab^ij - t_ab^ji          (Eq. A6, f = 0).
//
// Every term but D3 is a rank-K product D += L R^T over a few small index
// ranges, with L a gather of the amplitudes X[e][i][j][x] = t_ex^ij (one virtual
// and one active particle, the same array as active_particle.hip) or of the
// singles, and R a contraction of amplitudes with lambda, gamma or eta.  D4 and
// D6 are one form over every hole h with the hole weight w (1 on core holes,
// gamma / 2 on active ones, as the 1/2 and gamma_w^z of D6 and the shared core
// index of D4 make them):
//     sum_{h v y} X[e][h][v][y] (w (2 Q1 - Q2))[f][h v y]
//   - sum_{h v y} X[e][v][h][y] (w (Q1 + Q4))[f][h v y],
//     Q1[f][h v y] = sum_{u x} X[f][h][x][u] lambda_uv^xy,
//     Q2[f][h v y] = sum_{u x} X[f][x][h][u] lambda_uv^xy,
//     Q4[f][h v y] = sum_{u x} X[f][x][h][u] lambda_uv^yx.
// The K columns are [D4+D6 first half | second half | D5 | D1 | D2]; one FP64
// MFMA GEMM forms E = L R^T.  D3 needs the virtual-virtual amplitudes of the
// active hole pairs, T[e][uv][e'] (a GEMM per active hole), mixed with lambda
// over the hole pair (a GEMM batched over e) and contracted over (uv, e') into
// the same E.  Each term is symmetric in (e, f); D += (E + E^T) / 2.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/dfpt2.h"
#include "common.h"
#include "host.h"

namespace dfpt2 {
namespace {

__device__ inline size_t xidx(int e, int i, int j, int x, int n_h, int n_a) {
  return (((size_t)e * n_h + i) * n_h + j) * n_a + x;
}

// X[e][i][j][x] *= (1 - exp(-s D^2)) / D,  D = eps_i + eps_j - eps_e - eps_(n_core + x)
__global__ void cs_regularize_x(double* X, const double* eps_h, const double* eps_v, int n_v, int n_h, int n_a,
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

// T[e][u v][e'] *= (1 - exp(-s D^2)) / D,  D = eps_u + eps_v - eps_e - eps_e'
__global__ void cs_regularize_t(double* T, const double* eps_h, const double* eps_v, int n_v, int n_a, int n_core,
                                double s) {
  const size_t n = (size_t)n_v * n_a * n_a * n_v;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    size_t r = k;
    const int e2 = (int)(r % n_v);
    r /= n_v;
    const int v = (int)(r % n_a);
    r /= n_a;
    const int u = (int)(r % n_a);
    const int e = (int)(r / n_a);
    const double dl = eps_h[n_core + u] + eps_h[n_core + v] - eps_v[e] - eps_v[e2];
    T[k] = (dl != 0.0) ? T[k] * (1.0 - exp(-s * dl * dl)) / dl : 0.0;
  }
}

// singles t1[i][e] (Eq. A6 with f = 0)
__global__ void cs_singles(const double* X, const double* eps_h, const double* eps_v, const double* gamma, int n_v,
                           int n_h, int n_a, int n_core, double s, double* t1) {
  const size_t n = (size_t)n_h * n_v;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(k / n_v), e = (int)(k - (size_t)i * n_v);
    double src = 0.0;
    for (int u = 0; u < n_a; ++u)
      for (int x = 0; x < n_a; ++x) {
        const double w = (eps_h[n_core + x] - eps_h[n_core + u]) * gamma[x * n_a + u];
        if (w == 0.0) continue;
        src += w * (2.0 * X[xidx(e, i, n_core + u, x, n_h, n_a)] - X[xidx(e, n_core + u, i, x, n_h, n_a)]);
      }
    const double dl = eps_h[i] - eps_v[e];
    t1[k] = (dl != 0.0) ? 0.5 * src * (1.0 - exp(-s * dl * dl)) / dl : 0.0;
  }
}

// Qa = 2 Q1 - Q2 and Qb = -(Q1 + Q4), [f][h][v][y]
__global__ void cs_q(const double* X, const double* lam, int n_v, int n_h, int n_a, int n_core, double* Qa,
                     double* Qb) {
  const size_t n = (size_t)n_v * n_h * n_a * n_a;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    size_t r = k;
    const int y = (int)(r % n_a);
    r /= n_a;
    const int v = (int)(r % n_a);
    r /= n_a;
    const int h = (int)(r % n_h);
    const int f = (int)(r / n_h);
    double q1 = 0.0, q2 = 0.0, q4 = 0.0;
    for (int u = 0; u < n_a; ++u)
      for (int x = 0; x < n_a; ++x) {
        const double a1 = X[xidx(f, h, n_core + x, u, n_h, n_a)];
        const double a2 = X[xidx(f, n_core + x, h, u, n_h, n_a)];
        q1 += a1 * lam[((u * n_a + v) * n_a + x) * n_a + y];
        q2 += a2 * lam[((u * n_a + v) * n_a + x) * n_a + y];
        q4 += a2 * lam[((u * n_a + v) * n_a + y) * n_a + x];
      }
    Qa[k] = 2.0 * q1 - q2;
    Qb[k] = -(q1 + q4);
  }
}

// W1[f][u] = sum_{v x y} t_fv^xy lambda_uv^xy
__global__ void cs_w1(const double* X, const double* lam, int n_v, int n_h, int n_a, int n_core, double* W1) {
  const size_t n = (size_t)n_v * n_a;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int f = (int)(k / n_a), u = (int)(k - (size_t)f * n_a);
    double acc = 0.0;
    for (int v = 0; v < n_a; ++v)
      for (int x = 0; x < n_a; ++x)
        for (int y = 0; y < n_a; ++y)
          acc += X[xidx(f, n_core + x, n_core + y, v, n_h, n_a)] * lam[((u * n_a + v) * n_a + x) * n_a + y];
    W1[k] = acc;
  }
}

// R5[f][u v z] = 1/2 sum_{x y w} t_fw^xy eta_w^z lambda_uv^xy
__global__ void cs_r5(const double* X, const double* lam, const double* gamma, int n_v, int n_h, int n_a, int n_core,
                      double* R5) {
  const size_t n = (size_t)n_v * n_a * n_a * n_a;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    size_t r = k;
    const int z = (int)(r % n_a);
    r /= n_a;
    const int v = (int)(r % n_a);
    r /= n_a;
    const int u = (int)(r % n_a);
    const int f = (int)(r / n_a);
    double acc = 0.0;
    for (int x = 0; x < n_a; ++x)
      for (int y = 0; y < n_a; ++y) {
        const double l = lam[((u * n_a + v) * n_a + x) * n_a + y];
        if (l == 0.0) continue;
        double xe = 0.0;
        for (int w = 0; w < n_a; ++w)
          xe += X[xidx(f, n_core + x, n_core + y, w, n_h, n_a)] * ((w == z ? 2.0 : 0.0) - gamma[w * n_a + z]);
        acc += xe * l;
      }
    R5[k] = 0.5 * acc;
  }
}

struct CsDims {
  int n_v, n_h, n_a, n_core;
  int kA, kC, kD, kE, K;  // column ranges: A (and B) = n_h n_a^2, C = n_a^3, D = n_h, E = 2 n_a
  bool lam;
};

// L[e][k] (gathers) and R[f][k] (contractions, hole weight w on segments A/B)
__global__ void cs_build_lr(const double* X, const double* t1, const double* Qa, const double* Qb, const double* R5,
                            const double* W1, const double* gamma, CsDims d, double* L, double* R) {
  const size_t n = (size_t)d.n_v * d.K;
  const int n_h = d.n_h, n_a = d.n_a, nc = d.n_core, n_v = d.n_v;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(q / d.K);
    int k = (int)(q - (size_t)row * d.K);
    double lv = 0.0, rv = 0.0;
    if (d.lam && k < 2 * d.kA) {  // D4 + D6
      const bool second = k >= d.kA;
      if (second) k -= d.kA;
      const int y = k % n_a, v = (k / n_a) % n_a, h = k / (n_a * n_a);
      lv = second ? X[xidx(row, nc + v, h, y, n_h, n_a)] : X[xidx(row, h, nc + v, y, n_h, n_a)];
      const double* Q = second ? Qb : Qa;
      if (h < nc) {
        rv = Q[(((size_t)row * n_h + h) * n_a + v) * n_a + y];
      } else {
        const int w = h - nc;
        double acc = 0.0;
        for (int z = 0; z < n_a; ++z) acc += gamma[w * n_a + z] * Q[(((size_t)row * n_h + nc + z) * n_a + v) * n_a + y];
        rv = 0.5 * acc;
      }
    } else {
      if (d.lam) k -= 2 * d.kA;
      if (d.lam && k < d.kC) {  // D5
        const int z = k % n_a, v = (k / n_a) % n_a, u = k / (n_a * n_a);
        lv = X[xidx(row, nc + u, nc + v, z, n_h, n_a)];
        rv = R5[(size_t)row * d.kC + k];
      } else {
        if (d.lam) k -= d.kC;
        if (k < d.kD) {  // D1: k = hole i
          lv = t1[(size_t)k * n_v + row];
          if (k < nc) {
            rv = 2.0 * t1[(size_t)k * n_v + row];
          } else {
            double acc = 0.0;
            for (int v = 0; v < n_a; ++v) acc += gamma[(k - nc) * n_a + v] * t1[(size_t)(nc + v) * n_v + row];
            rv = acc;
          }
        } else {  // D2 (only with lambda): t_e^u W1[f][u], then W1[e][x] t_f^x
          k -= d.kD;
          if (k < n_a) {
            lv = t1[(size_t)(nc + k) * n_v + row];
            rv = W1[(size_t)row * n_a + k];
          } else {
            k -= n_a;
            lv = W1[(size_t)row * n_a + k];
            rv = t1[(size_t)(nc + k) * n_v + row];
          }
        }
      }
    }
    L[q] = lv;
    R[q] = rv;
  }
}

// D += scale (E + E^T) / 2
__global__ void cs_sym_add(const double* E, double* D, int n_v, double scale) {
  const size_t n = (size_t)n_v * n_v;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t a = k / n_v, b = k - a * n_v;
    D[k] += 0.5 * scale * (E[k] + E[b * n_v + a]);
  }
}

struct CsPlan {
  CsDims d;
  int n_aux;
  size_t off_X, off_t1, off_Qa, off_Qb, off_W1, off_R5, off_L, off_R, off_E, off_T, off_M, bytes;
};

int plan_cs(const dfpt2_opts* o, bool with_lambda, CsPlan* p) {
  if (!o) return fail(DFPT2_ERR_INVALID_ARG, "opts is null");
  PassPlan pp;
  const int st = plan_pass(o, &pp);  // the same size checks as the pass
  if (st != DFPT2_OK) return st;
  *p = CsPlan{};
  CsDims& d = p->d;
  d.n_core = (int)o->n_core;
  d.n_a = (int)o->n_act;
  d.n_h = d.n_core + d.n_a;
  d.n_v = (int)o->n_vir;
  d.lam = with_lambda;
  p->n_aux = (int)o->n_aux;
  const size_t n_v = d.n_v, n_h = d.n_h, n_a = d.n_a;
  d.kA = (int)(n_h * n_a * n_a);
  d.kC = (int)(n_a * n_a * n_a);
  d.kD = (int)n_h;
  d.kE = (int)(2 * n_a);
  d.K = with_lambda ? 2 * d.kA + d.kC + d.kD + d.kE : d.kD;
  const double k3 = (double)n_a * n_a * n_v;
  if ((double)n_h * n_h * n_a > 2.0e9 || k3 > 2.0e9)
    return fail(DFPT2_ERR_INVALID_ARG, "too many hole pairs x active orbitals");
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o_ = off;
    off = align_up(off + b, 256);
    return o_;
  };
  p->off_X = take(sizeof(double) * n_v * n_h * n_h * n_a);
  p->off_t1 = take(sizeof(double) * n_h * n_v);
  p->off_Qa = take(with_lambda ? sizeof(double) * n_v * n_h * n_a * n_a : 0);
  p->off_Qb = take(with_lambda ? sizeof(double) * n_v * n_h * n_a * n_a : 0);
  p->off_W1 = take(with_lambda ? sizeof(double) * n_v * n_a : 0);
  p->off_R5 = take(with_lambda ? sizeof(double) * n_v * n_a * n_a * n_a : 0);
  p->off_L = take(sizeof(double) * n_v * (size_t)d.K);
  p->off_R = take(sizeof(double) * n_v * (size_t)d.K);
  p->off_E = take(sizeof(double) * n_v * n_v);
  p->off_T = take(with_lambda ? sizeof(double) * n_v * n_a * n_a * n_v : 0);
  p->off_M = take(with_lambda ? sizeof(double) * n_v * n_a * n_a * n_v : 0);
  p->bytes = off;
  return DFPT2_OK;
}

int grid_cs(size_t n) {
  const size_t g = (n + 255) / 256;
  return (int)(g < 65535 ? (g > 0 ? g : 1) : 65535);
}

}  // namespace
}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int dfpt2_cumulant_singles_workspace_size(const dfpt2_opts* opts, int with_lambda, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  CsPlan p;
  const int st = plan_cs(opts, with_lambda != 0, &p);
  if (st != DFPT2_OK) return st;
  *bytes = p.bytes;
  return DFPT2_OK;
}

int dfpt2_add_cumulant_singles_density(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir,
                                       const double* gamma_act, const double* lambda_act, const double* B,
                                       const double* B_act, double* D_vv, double* t1_out, void* workspace,
                                       size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  CsPlan p;
  int st = plan_cs(opts, lambda_act != nullptr, &p);
  if (st != DFPT2_OK) return st;
  const CsDims& d = p.d;
  if (d.n_a == 0) return DFPT2_OK;  // no active orbitals: no singles source, no cumulant
  if (!eps_hole || !eps_vir || !gamma_act || !B || !B_act || !D_vv || !workspace)
    return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (ws_bytes < p.bytes) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, p.bytes);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* X = reinterpret_cast<double*>(ws + p.off_X);
  double* t1 = reinterpret_cast<double*>(ws + p.off_t1);
  double* Qa = reinterpret_cast<double*>(ws + p.off_Qa);
  double* Qb = reinterpret_cast<double*>(ws + p.off_Qb);
  double* W1 = reinterpret_cast<double*>(ws + p.off_W1);
  double* R5 = reinterpret_cast<double*>(ws + p.off_R5);
  double* L = reinterpret_cast<double*>(ws + p.off_L);
  double* R = reinterpret_cast<double*>(ws + p.off_R);
  double* E = reinterpret_cast<double*>(ws + p.off_E);
  double* T = reinterpret_cast<double*>(ws + p.off_T);
  double* M = reinterpret_cast<double*>(ws + p.off_M);
  const int n_v = d.n_v, n_h = d.n_h, n_a = d.n_a, nc = d.n_core, na = p.n_aux;
  const int KX = n_h * n_h * n_a, NA = n_h * n_a;
  const double sflow = opts->s;
  hipError_t e;
  ProfScope ps(DFPT2_STAGE_ACTIVE, s);
  // amplitudes with one active particle, X[e][(i, j, x)] (as active_particle.hip)
  if ((e = gemm_f64(B, na, (long long)n_v * na, 0, B_act, na, 0, 1, X, KX, NA, n_v, NA, na, n_h, 1.0, 0.0, s)) !=
      hipSuccess)
    return hip_fail(e, "active-particle integrals");
  const size_t nx = (size_t)n_v * KX;
  hipLaunchKernelGGL(cs_regularize_x, dim3(grid_cs(nx)), dim3(256), 0, s, X, eps_hole, eps_vir, n_v, n_h, n_a, nc,
                     sflow);
  hipLaunchKernelGGL(cs_singles, dim3(grid_cs((size_t)n_h * n_v)), dim3(256), 0, s, X, eps_hole, eps_vir, gamma_act,
                     n_v, n_h, n_a, nc, sflow, t1);
  if (d.lam) {
    hipLaunchKernelGGL(cs_q, dim3(grid_cs((size_t)n_v * n_h * n_a * n_a)), dim3(256), 0, s, X, lambda_act, n_v, n_h,
                       n_a, nc, Qa, Qb);
    hipLaunchKernelGGL(cs_w1, dim3(grid_cs((size_t)n_v * n_a)), dim3(256), 0, s, X, lambda_act, n_v, n_h, n_a, nc,
                       W1);
    hipLaunchKernelGGL(cs_r5, dim3(grid_cs((size_t)n_v * n_a * n_a * n_a)), dim3(256), 0, s, X, lambda_act,
                       gamma_act, n_v, n_h, n_a, nc, R5);
  }
  hipLaunchKernelGGL(cs_build_lr, dim3(grid_cs((size_t)n_v * d.K)), dim3(256), 0, s, X, t1, Qa, Qb, R5, W1,
                     gamma_act, d, L, R);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "cumulant/singles kernels");
  // E = L R^T
  if ((e = gemm_f64(L, d.K, 0, 0, R, d.K, 0, 1, E, n_v, 0, n_v, n_v, d.K, 1, 1.0, 0.0, s)) != hipSuccess)
    return hip_fail(e, "cumulant/singles density");
  if (d.lam) {
    // T[e][(u, v)][e'] = sum_Q B_ue^Q B_ve'^Q, one GEMM per active hole u batched over v
    const int K3 = n_a * n_a * n_v;
    for (int u = 0; u < n_a; ++u) {
      if ((e = gemm_f64(B + (size_t)(nc + u) * n_v * na, na, 0, 0, B + (size_t)nc * n_v * na, na, (long long)n_v * na,
                        1, T + (size_t)u * n_a * n_v, K3, n_v, n_v, n_v, na, n_a, 1.0, 0.0, s)) != hipSuccess)
        return hip_fail(e, "active-active integrals");
    }
    hipLaunchKernelGGL(cs_regularize_t, dim3(grid_cs((size_t)n_v * K3)), dim3(256), 0, s, T, eps_hole, eps_vir, n_v,
                       n_a, nc, sflow);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "active-active amplitudes");
    // M[f][(u, v)][e'] = sum_(x, y) lambda_uv^xy T[f][(x, y)][e'], batched over f
    if ((e = gemm_f64(lambda_act, n_a * n_a, 0, 0, T, n_v, (long long)K3, 0, M, n_v, (long long)K3, n_a * n_a, n_v,
                      n_a * n_a, n_v, 1.0, 0.0, s)) != hipSuccess)
      return hip_fail(e, "cumulant mixing");
    // E += T M^T over (u v, e')
    if ((e = gemm_f64(T, K3, 0, 0, M, K3, 0, 1, E, n_v, 0, n_v, n_v, K3, 1, 1.0, 1.0, s)) != hipSuccess)
      return hip_fail(e, "cumulant active-active term");
  }
  const double scale = opts->density_convention == 1 ? 0.5 : 1.0;
  hipLaunchKernelGGL(cs_sym_add, dim3(grid_cs((size_t)n_v * n_v)), dim3(256), 0, s, E, D_vv, n_v, scale);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "cumulant/singles add");
  if (t1_out && (e = hipMemcpyAsync(t1_out, t1, sizeof(double) * n_h * n_v, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "singles copy");
  return DFPT2_OK;
}

}  // extern "C"
