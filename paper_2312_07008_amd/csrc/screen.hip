// Learned pair screening (row a12; not part of the paper's method): pair
// features, a 5-64-64-1 tanh network trained in FP32 with mean squared error
// and Adam, and the mask that drops core pairs whose predicted ||t_ij||_F is
// below a threshold.
//
// Pair quantities for unordered core pairs i <= j (row-major order, the order
// of the pass's pair list):
//   q_iQ = ||B^Q_i.||_2,  U_ij = sum_Q q_iQ q_jQ >= ||V_ij||_F,
//   W_ij = (sum_Q q_iQ^2 q_jQ^2)^(1/2)  (||V_ij||_F for mutually orthogonal rank-one terms),
//   g_ij = max |1 - e^{-s D^2}| / |D| over the pair's range of denominators D (Eq. A7),
// so ||t_ij||_F <= g_ij U_ij is a rigorous screen and log(g_ij W_ij) is the scale
// the network corrects.  Features
//   x = (e_i, e_j, log(U/W), 0.1 (log W_ij - (log W_ii + log W_jj)/2), 0.1 log(g W)).
// Parameters (FP32) are packed [W1 64x5, b1, W2 64x64, b2, w3, b3] = 4609 values.
#include <cmath>
#include <cfloat>

#include "../../include/dfpt2.h"
#include "common.h"
#include "host.h"

namespace dfpt2 {

namespace {
constexpr int H = 64;
constexpr int NIN = 5;
constexpr int NP = H * NIN + H + H * H + H + H + 1;  // 4609
constexpr int OFF_W1 = 0, OFF_B1 = H * NIN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H;
constexpr int BW_SAMPLES = 128;  // samples per workgroup in the backward kernel

// q2[i][Q] = sum_a B[i][a][Q]^2 for core holes
__global__ void colnorm2_kernel(const double* B, int n_v, int n_aux, double* q2) {
  const int Q = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (Q >= n_aux) return;
  const double* Bi = B + (size_t)i * n_v * n_aux;
  double acc = 0.0;
  for (int a = 0; a < n_v; ++a) {
    const double x = Bi[(size_t)a * n_aux + Q];
    acc += x * x;
  }
  q2[(size_t)i * n_aux + Q] = acc;
}

// wdiag[i] = W_ii^2 = sum_Q q2_iQ^2
__global__ void wdiag_kernel(const double* q2, int n_aux, double* wdiag) {
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int Q = threadIdx.x; Q < n_aux; Q += 64) acc += q2[(size_t)i * n_aux + Q] * q2[(size_t)i * n_aux + Q];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) wdiag[i] = acc;
}

__device__ double reg_fun(double s, double x) { return x > 0.0 ? -expm1(-s * x * x) / x : 0.0; }

// one wave per pair
__global__ void pair_features_kernel(const double* q2, const double* wdiag, const double* eps_h, double e_vmin,
                                     double e_vmax, int n_core, int n_aux, double s, double x_star, float* feats,
                                     double* log_scale, int n_pairs) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n_pairs) return;
  int i = 0, rem = p;
  while (rem >= n_core - i) {
    rem -= n_core - i;
    ++i;
  }
  const int j = i + rem;
  double u = 0.0, w2 = 0.0;
  for (int Q = lane; Q < n_aux; Q += 64) {
    const double a = q2[(size_t)i * n_aux + Q], b = q2[(size_t)j * n_aux + Q];
    u += sqrt(a) * sqrt(b);
    w2 += a * b;
  }
  u = wave_sum(u);
  w2 = wave_sum(w2);
  if (lane != 0) return;
  const double ei = eps_h[i], ej = eps_h[j];
  double lo = fabs(ei + ej - 2.0 * e_vmin), hi = fabs(ei + ej - 2.0 * e_vmax);
  if (lo > hi) {
    const double t = lo;
    lo = hi;
    hi = t;
  }
  const double g = (lo <= x_star && x_star <= hi) ? reg_fun(s, x_star) : fmax(reg_fun(s, lo), reg_fun(s, hi));
  const double w = sqrt(w2);
  const double lw = log(w), lu = log(u);
  const double lg = log(g);
  float* f = feats + (size_t)p * NIN;
  f[0] = (float)ei;
  f[1] = (float)ej;
  f[2] = (float)(lu - lw);
  f[3] = (float)(0.1 * (lw - 0.25 * (log(wdiag[i]) + log(wdiag[j]))));
  f[4] = (float)(0.1 * (lg + lw));
  log_scale[2 * (size_t)p] = lg + lw;
  log_scale[2 * (size_t)p + 1] = lg + lu;
}

// ------------------------------------------------------------------ network
// One thread per sample; parameters in LDS (broadcast reads).
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* Wp, const float* X, int n, float* out,
                                                      float* cache) {
  __shared__ float w[NP];
  for (int k = threadIdx.x; k < NP; k += blockDim.x) w[k] = Wp[k];
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float x[NIN];
#pragma unroll
  for (int c = 0; c < NIN; ++c) x[c] = X[(size_t)t * NIN + c];
  float h1[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    float z = w[OFF_B1 + k];
#pragma unroll
    for (int c = 0; c < NIN; ++c) z = fmaf(w[OFF_W1 + k * NIN + c], x[c], z);
    h1[k] = tanhf(z);
    if (cache) cache[(size_t)t * 2 * H + k] = h1[k];
  }
  float o = w[OFF_B3];
  for (int k = 0; k < H; ++k) {
    float z = w[OFF_B2 + k];
#pragma unroll
    for (int m = 0; m < H; ++m) z = fmaf(w[OFF_W2 + k * H + m], h1[m], z);
    const float h2 = tanhf(z);
    if (cache) cache[(size_t)t * 2 * H + H + k] = h2;
    o = fmaf(w[OFF_W3 + k], h2, o);
  }
  out[t] = o;
}

// Gradient of sum_n dout_n out_n: a workgroup takes BW_SAMPLES samples, forms
// dz2 and dz1 per sample, then the parameter gradients as small reductions over
// its samples; partial[blockIdx.x][NP] is summed in a fixed order afterwards.
__global__ __launch_bounds__(256) void mlp_bwd_kernel(const float* Wp, const float* X, const float* cache,
                                                      const float* dout, int n, float* partial) {
  __shared__ float w2[H * H];
  __shared__ float sh1[BW_SAMPLES][H + 1];
  __shared__ float sdz2[BW_SAMPLES][H + 1];
  __shared__ float sdz1[BW_SAMPLES][H + 1];
  __shared__ float sx[BW_SAMPLES][NIN];
  __shared__ float sw3[H];
  for (int k = threadIdx.x; k < H * H; k += blockDim.x) w2[k] = Wp[OFF_W2 + k];
  for (int k = threadIdx.x; k < H; k += blockDim.x) sw3[k] = Wp[OFF_W3 + k];
  const int s0 = blockIdx.x * BW_SAMPLES;
  const int ns = min(BW_SAMPLES, n - s0);
  __syncthreads();
  // per-sample: dz2 = dout w3 (1 - h2^2); h1 and x staged
  for (int idx = threadIdx.x; idx < BW_SAMPLES * H; idx += blockDim.x) {
    const int r = idx / H, k = idx % H;
    float h1 = 0.f, dz2 = 0.f;
    if (r < ns) {
      const size_t base = (size_t)(s0 + r) * 2 * H;
      h1 = cache[base + k];
      const float h2 = cache[base + H + k];
      dz2 = dout[s0 + r] * sw3[k] * (1.f - h2 * h2);
    }
    sh1[r][k] = h1;
    sdz2[r][k] = dz2;
  }
  for (int idx = threadIdx.x; idx < BW_SAMPLES * NIN; idx += blockDim.x) {
    const int r = idx / NIN, c = idx % NIN;
    sx[r][c] = (r < ns) ? X[(size_t)(s0 + r) * NIN + c] : 0.f;
  }
  __syncthreads();
  // dz1[r][m] = (sum_k W2[k][m] dz2[r][k]) (1 - h1^2)
  for (int idx = threadIdx.x; idx < BW_SAMPLES * H; idx += blockDim.x) {
    const int r = idx / H, m = idx % H;
    float acc = 0.f;
    for (int k = 0; k < H; ++k) acc = fmaf(w2[k * H + m], sdz2[r][k], acc);
    const float h1 = sh1[r][m];
    sdz1[r][m] = acc * (1.f - h1 * h1);
  }
  __syncthreads();
  float* part = partial + (size_t)blockIdx.x * NP;
  // W2 gradient: sum_r dz2[r][k] h1[r][m]
  for (int idx = threadIdx.x; idx < H * H; idx += blockDim.x) {
    const int k = idx / H, m = idx % H;
    float acc = 0.f;
    for (int r = 0; r < BW_SAMPLES; ++r) acc = fmaf(sdz2[r][k], sh1[r][m], acc);
    part[OFF_W2 + idx] = acc;
  }
  // W1 gradient: sum_r dz1[r][k] x[r][c]
  for (int idx = threadIdx.x; idx < H * NIN; idx += blockDim.x) {
    const int k = idx / NIN, c = idx % NIN;
    float acc = 0.f;
    for (int r = 0; r < BW_SAMPLES; ++r) acc = fmaf(sdz1[r][k], sx[r][c], acc);
    part[OFF_W1 + idx] = acc;
  }
  // b1, b2, w3, b3
  for (int k = threadIdx.x; k < H; k += blockDim.x) {
    float a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int r = 0; r < BW_SAMPLES; ++r) {
      a1 += sdz1[r][k];
      a2 += sdz2[r][k];
      if (r < ns) a3 = fmaf(dout[s0 + r], cache[(size_t)(s0 + r) * 2 * H + H + k], a3);
    }
    part[OFF_B1 + k] = a1;
    part[OFF_B2 + k] = a2;
    part[OFF_W3 + k] = a3;
  }
  if (threadIdx.x == 0) {
    float a = 0.f;
    for (int r = 0; r < ns; ++r) a += dout[s0 + r];
    part[OFF_B3] = a;
  }
}

__global__ void sum_partials_kernel(const float* partial, int nblk, float* dW) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NP) return;
  float acc = 0.f;
  for (int b = 0; b < nblk; ++b) acc += partial[(size_t)b * NP + k];
  dW[k] = acc;
}

// dout = 2 (out - y) / n ; loss = mean (out - y)^2 (single workgroup, fixed order)
__global__ void mse_kernel(const float* out, const float* y, int n, float* dout, float* loss) {
  __shared__ float sh[16];
  float acc = 0.f;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const float r = out[t] - y[t];
    dout[t] = 2.f * r / (float)n;
    acc = fmaf(r, r, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    float t = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    *loss = t / (float)n;
  }
}

__global__ void adam_kernel(float* W, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  W[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// y[p] = log ||t_ij||_F - log(g W) for the core pairs, from the pass's pair_tnorm
__global__ void targets_kernel(const float* pair_tnorm, const double* log_scale, int n_core, int n_h, float* y,
                               int n_pairs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  int i = 0, rem = p;
  while (rem >= n_core - i) {
    rem -= n_core - i;
    ++i;
  }
  const int j = i + rem;
  y[p] = (float)(log((double)pair_tnorm[(size_t)i * n_h + j]) - log_scale[2 * (size_t)p]);
}

// mask: all ones, then core pairs whose predicted log-norm is below log(thr) set to 0.
//   mode 0: log(g W) + pred + margin;  mode 1: rigorous bound log(g U).
__global__ void mask_kernel(const float* pred, const double* log_scale, int n_core, int n_h, double log_thr,
                            double margin, int mode, uint8_t* mask, int* n_dropped, int n_pairs) {
  // phase 1 (all threads of the single workgroup): fill ones
  for (int k = threadIdx.x; k < n_h * n_h; k += blockDim.x) mask[k] = 1;
  __syncthreads();
  int dropped = 0;
  for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) {
    const double ln = (mode == 0) ? log_scale[2 * (size_t)p] + (double)pred[p] + margin : log_scale[2 * (size_t)p + 1];
    if (ln < log_thr) {
      int i = 0, rem = p;
      while (rem >= n_core - i) {
        rem -= n_core - i;
        ++i;
      }
      const int j = i + rem;
      mask[(size_t)i * n_h + j] = 0;
      mask[(size_t)j * n_h + i] = 0;
      ++dropped;
    }
  }
  for (int off = 32; off > 0; off >>= 1) dropped += __shfl_xor(dropped, off, 64);
  __shared__ int sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dropped;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    *n_dropped = t;
  }
}

// u* solving 2 u^2 e^{-u^2} = 1 - e^{-u^2} (maximum of (1 - e^{-u^2}) / u), by bisection
double regularizer_peak() {
  double lo = 0.5, hi = 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (2.0 * mid * mid * std::exp(-mid * mid) > -std::expm1(-mid * mid)) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

int train_nblk(int64_t n) { return (int)((n + BW_SAMPLES - 1) / BW_SAMPLES); }

}  // namespace

}  // namespace dfpt2

using namespace dfpt2;

extern "C" {

int pairscreen_num_params(void) { return NP; }

int pairscreen_workspace_size(const dfpt2_opts* opts, size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(DFPT2_ERR_INVALID_ARG, "bytes is null");
  PassPlan pl;
  int st = plan_pass(opts, &pl);
  if (st != DFPT2_OK) return st;
  *bytes = align_up(sizeof(double) * (size_t)(pl.n_core > 0 ? pl.n_core : 1) * pl.n_aux, 256) +
           align_up(sizeof(double) * (size_t)(pl.n_core > 0 ? pl.n_core : 1), 256) + 256;
  return DFPT2_OK;
}

int pairscreen_features(const dfpt2_opts* opts, const double* eps_hole, const double* eps_vir, const double* B,
                        float* feats, double* log_scale, void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  PassPlan pl;
  int st = plan_pass(opts, &pl);
  if (st != DFPT2_OK) return st;
  if (!eps_hole || !eps_vir || !B || !feats || !log_scale || !workspace)
    return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  size_t need = 0;
  pairscreen_workspace_size(opts, &need);
  if (ws_bytes < need) return fail(DFPT2_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  if (pl.n_core == 0) return DFPT2_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* q2 = reinterpret_cast<double*>(ws);
  double* wd = reinterpret_cast<double*>(ws + align_up(sizeof(double) * (size_t)pl.n_core * pl.n_aux, 256));
  // the virtual energies are ascending: the denominator range uses the first and last
  double ev[2];
  hipError_t e;
  if ((e = hipMemcpyAsync(&ev[0], eps_vir, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "copy");
  if ((e = hipMemcpyAsync(&ev[1], eps_vir + pl.n_v - 1, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  ProfScope ps(DFPT2_STAGE_SCREEN, s);
  hipLaunchKernelGGL(colnorm2_kernel, dim3((pl.n_aux + 255) / 256, pl.n_core), dim3(256), 0, s, B, pl.n_v, pl.n_aux,
                     q2);
  hipLaunchKernelGGL(wdiag_kernel, dim3(pl.n_core), dim3(64), 0, s, q2, pl.n_aux, wd);
  const double x_star = regularizer_peak() / std::sqrt(opts->s);
  hipLaunchKernelGGL(pair_features_kernel, dim3((pl.n_up + 3) / 4), dim3(256), 0, s, q2, wd, eps_hole, ev[0], ev[1],
                     pl.n_core, pl.n_aux, opts->s, x_star, feats, log_scale, pl.n_up);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "features");
  return DFPT2_OK;
}

int pairscreen_mlp_forward(const float* W, const float* feats, int64_t n, float* pred, float* act_cache,
                           dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!W || !feats || !pred) return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (n < 0 || n > (1ll << 30)) return fail(DFPT2_ERR_INVALID_ARG, "bad sample count");
  if (n == 0) return DFPT2_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(DFPT2_STAGE_SCREEN, s);
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, feats, (int)n, pred,
                     act_cache);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DFPT2_OK : hip_fail(e, "mlp forward");
}

int pairscreen_backward_workspace_size(int64_t n, size_t* bytes) {
  g_last_error.clear();
  if (!bytes || n < 0) return fail(DFPT2_ERR_INVALID_ARG, "bad argument");
  *bytes = sizeof(float) * (size_t)(train_nblk(n) > 0 ? train_nblk(n) : 1) * NP + 256;
  return DFPT2_OK;
}

int pairscreen_mlp_backward(const float* W, const float* feats, const float* act_cache, const float* dpred, int64_t n,
                            float* dW, void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!W || !feats || !act_cache || !dpred || !dW || !workspace)
    return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (n <= 0 || n > (1ll << 30)) return fail(DFPT2_ERR_INVALID_ARG, "bad sample count");
  size_t need = 0;
  pairscreen_backward_workspace_size(n, &need);
  if (ws_bytes < need) return fail(DFPT2_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(DFPT2_STAGE_SCREEN, s);
  const int nblk = train_nblk(n);
  float* partial = static_cast<float*>(workspace);
  hipLaunchKernelGGL(mlp_bwd_kernel, dim3(nblk), dim3(256), 0, s, W, feats, act_cache, dpred, (int)n, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, partial, nblk, dW);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DFPT2_OK : hip_fail(e, "mlp backward");
}

int pairscreen_adam_step(float* W, const float* dW, float* m, float* v, int64_t n_params, float lr, float b1, float b2,
                         float eps, int64_t step, dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!W || !dW || !m || !v) return fail(DFPT2_ERR_INVALID_ARG, "null pointer argument");
  if (n_params <= 0 || step < 1 || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(DFPT2_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(DFPT2_STAGE_SCREEN, s);
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n_params + 255) / 256)), dim3(256), 0, s, W, dW, m, v, (int)n_params,
                     lr, b1, b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DFPT2_OK : hip_fail(e, "adam");
}

int pairscreen_train_workspace_size(int64_t n, size_t* bytes) {
  g_last_error.clear();
  if (!bytes || n <= 0) return fail(DFPT2_ERR_INVALID_ARG, "bad argument");
  size_t b = 0;
  b += align_up(sizeof(float) * n, 256);          // pred
  b += align_up(sizeof(float) * n, 256);          // dpred
  b += align_up(sizeof(float) * n * 2 * H, 256);  // activations
  b += align_up(sizeof(float) * NP, 256);         // dW
  size_t bw = 0;
  pairscreen_backward_workspace_size(n, &bw);
  b += align_up(bw, 256);
  *bytes = b;
  return DFPT2_OK;
}

int pairscreen_train(float* W, float* m, float* v, const float* feats, const float* y, int64_t n, int64_t steps,
                     int64_t step0, float lr, float* losses, void* workspace, size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!W || !m || !v || !feats || !y || !losses || !workspace) return fail(DFPT2_ERR_INVALID_ARG, "null pointer");
  if (n <= 0 || steps <= 0 || step0 < 0 || !(lr > 0.f)) return fail(DFPT2_ERR_INVALID_ARG, "bad argument");
  size_t need = 0;
  pairscreen_train_workspace_size(n, &need);
  if (ws_bytes < need) return fail(DFPT2_ERR_WORKSPACE, "workspace too small");
  char* ws = static_cast<char*>(workspace);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = ws + off;
    off += align_up(b, 256);
    return p;
  };
  float* pred = (float*)take(sizeof(float) * n);
  float* dpred = (float*)take(sizeof(float) * n);
  float* act = (float*)take(sizeof(float) * n * 2 * H);
  float* dW = (float*)take(sizeof(float) * NP);
  size_t bw = 0;
  pairscreen_backward_workspace_size(n, &bw);
  char* bws = take(bw);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int64_t t = 1; t <= steps; ++t) {
    int st = pairscreen_mlp_forward(W, feats, n, pred, act, stream);
    if (st != DFPT2_OK) return st;
    {
      ProfScope ps(DFPT2_STAGE_SCREEN, s);
      hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, s, pred, y, (int)n, dpred, losses + (t - 1));
    }
    st = pairscreen_mlp_backward(W, feats, act, dpred, n, dW, bws, bw, stream);
    if (st != DFPT2_OK) return st;
    st = pairscreen_adam_step(W, dW, m, v, NP, lr, 0.9f, 0.999f, 1e-8f, step0 + t, stream);
    if (st != DFPT2_OK) return st;
  }
  hipError_t e = hipStreamSynchronize(s);
  prof_flush();
  return e == hipSuccess ? DFPT2_OK : hip_fail(e, "train sync");
}

int pairscreen_targets(const float* pair_tnorm, const double* log_scale, int64_t n_core, int64_t n_h, float* y,
                       dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!pair_tnorm || !log_scale || !y) return fail(DFPT2_ERR_INVALID_ARG, "null pointer");
  if (n_core < 0 || n_h < n_core || n_core > 1024) return fail(DFPT2_ERR_INVALID_ARG, "bad hole counts");
  const int np = (int)(n_core * (n_core + 1) / 2);
  if (np == 0) return DFPT2_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(targets_kernel, dim3((np + 255) / 256), dim3(256), 0, s, pair_tnorm, log_scale, (int)n_core,
                     (int)n_h, y, np);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? DFPT2_OK : hip_fail(e, "targets");
}

int pairscreen_build_mask(const float* pred, const double* log_scale, int64_t n_core, int64_t n_h, double threshold,
                          double margin, int mode, uint8_t* mask, int64_t* n_dropped, void* workspace,
                          size_t ws_bytes, dfpt2_stream_t stream) {
  g_last_error.clear();
  if (!log_scale || !mask || !workspace || ws_bytes < 64) return fail(DFPT2_ERR_INVALID_ARG, "null pointer");
  if (mode != 0 && mode != 1) return fail(DFPT2_ERR_INVALID_ARG, "mode must be 0 (network) or 1 (bound)");
  if (mode == 0 && !pred) return fail(DFPT2_ERR_INVALID_ARG, "pred is null in network mode");
  if (!(threshold > 0.0) || !std::isfinite(margin)) return fail(DFPT2_ERR_INVALID_ARG, "threshold must be > 0");
  if (n_core < 0 || n_h < n_core || n_core > 1024 || n_h > 1088) return fail(DFPT2_ERR_INVALID_ARG, "bad hole counts");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ProfScope ps(DFPT2_STAGE_SCREEN, s);
  int* d_drop = static_cast<int*>(workspace);
  const int np = (int)(n_core * (n_core + 1) / 2);
  hipLaunchKernelGGL(mask_kernel, dim3(1), dim3(1024), 0, s, pred, log_scale, (int)n_core, (int)n_h,
                     std::log(threshold), margin, mode, mask, d_drop, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mask");
  ps.close();
  if (n_dropped) {
    int h = 0;
    if ((e = hipMemcpyAsync(&h, d_drop, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
    prof_flush();
    *n_dropped = h;
  }
  return DFPT2_OK;
}

}  // extern "C"
