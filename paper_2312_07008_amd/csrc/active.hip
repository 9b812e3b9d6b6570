// Active-hole weighting (row a6): the hole density gamma = 2 I_core (+) Gamma_act
// of Eq. A1 enters Eq. A9 through the S(.) Gamma^u_v core-active term and the
// Gamma^{uv}_{xy} active-active term.  With Gamma_act = U diag(n) U^T and zero
// cumulant both terms become ordinary pair terms in the natural active basis:
//     T'_{mk} = sum_u U_uk T_{mu},   T'_{kl} = sum_{uv} U_uk U_vl T_{uv}
// (the same for the renormalized integrals), and
//     D += 1/2 sum_{kl} n~_k n~_l T'_kl (2T'_kl - T'_kl^T)^T,
//     E += 1/4 sum_{kl} n~_k n~_l <Vr'_kl, 2T'_kl - T'_kl^T>,   n~ = (2,...,2, n_1..n_act).
// The core-active rotations stream the stacked matrices through rotate_stack_kernel
// (n_act <= 32), the active-active one (K = n_act^2) is an FP64 GEMM (api.cpp);
// this file holds the small kernels around them.
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

// W[(u,v),(k,l)] = U[u][k] U[v][l]   (n_act^2 x n_act^2)
__global__ void kron_uu_kernel(const double* U, int na, double* W) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;  // (k,l)
  const int row = blockIdx.y;                             // (u,v)
  const int n2 = na * na;
  if (col >= n2 || row >= n2) return;
  const int u = row / na, v = row % na, k = col / na, l = col % na;
  W[(size_t)row * n2 + col] = U[u * na + k] * U[v * na + l];
}

hipError_t launch_kron_uu(const double* U, int na, double* W, hipStream_t st) {
  const int n2 = na * na;
  hipLaunchKernelGGL(kron_uu_kernel, dim3((n2 + 127) / 128, n2), dim3(128), 0, st, U, na, W);
  return hipGetLastError();
}

// Rotation of stacked n_v x n_v matrices to the natural active basis, for the
// core-active pairs: out[b][k][e] = sum_u U[u][k] in[b][u][e], e < n = n_v^2, one
// stack of na matrices per batch entry b.  Thread = two consecutive elements e of
// every matrix of its stack: it reads the na inputs once (16-byte loads,
// consecutive threads on consecutive addresses) and writes the na outputs once,
// so the kernel streams each stack through HBM once; U (na <= NAMAX) sits in LDS
// and every wave reads the same entry at a time (a broadcast).  As a GEMM of
// shape (na x na) x (na x n) on 128-row tiles it ran at under 1 TB/s.
template <int NAMAX, bool VEC>
__global__ __launch_bounds__(256) void rotate_stack_kernel(const double* U, int na, const double* in, double* out,
                                                           long long n) {
  __shared__ double su[NAMAX * NAMAX];
  for (int i = threadIdx.x; i < na * na; i += 256) su[i] = U[i];
  __syncthreads();
  const long long e = 2 * ((long long)blockIdx.x * 256 + threadIdx.x);
  if (e >= n) return;
  const size_t bo = (size_t)blockIdx.y * na * n;
  const bool two = VEC || e + 1 < n;  // VEC: n even, so both elements exist
  double2 x[NAMAX];
#pragma unroll
  for (int u = 0; u < NAMAX; ++u) {
    x[u] = make_double2(0.0, 0.0);
    if (u < na) {
      const double* src = in + bo + (size_t)u * n + e;
      if (VEC) x[u] = *reinterpret_cast<const double2*>(src);
      else x[u] = make_double2(src[0], two ? src[1] : 0.0);
    }
  }
#pragma unroll
  for (int k = 0; k < NAMAX; ++k) {
    if (k >= na) break;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < NAMAX; ++u) {
      if (u < na) {
        const double c = su[u * na + k];
        acc.x = fma(c, x[u].x, acc.x);
        acc.y = fma(c, x[u].y, acc.y);
      }
    }
    double* dst = out + bo + (size_t)k * n + e;
    if (VEC) {
      *reinterpret_cast<double2*>(dst) = acc;
    } else {
      dst[0] = acc.x;
      if (two) dst[1] = acc.y;
    }
  }
}

hipError_t launch_rotate_stack(const double* U, int na, const double* in, double* out, long long n, int batch,
                               hipStream_t st) {
  if (na <= 0 || n <= 0 || batch <= 0) return hipSuccess;
  if (na > 32 || batch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 511) / 512), batch), block(256);
  const bool vec = (n % 2) == 0;
#define ROT(NA_)                                                                                         \
  do {                                                                                                   \
    if (vec) hipLaunchKernelGGL((rotate_stack_kernel<NA_, true>), grid, block, 0, st, U, na, in, out, n);  \
    else hipLaunchKernelGGL((rotate_stack_kernel<NA_, false>), grid, block, 0, st, U, na, in, out, n);     \
  } while (0)
  if (na <= 8) ROT(8);
  else if (na <= 16) ROT(16);
  else ROT(32);
#undef ROT
  return hipGetLastError();
}

// Pair lists for the active blocks.
//   kind 0: core-active, cores m0 .. m0+ncore-1 x active u (m-major): (m, n_core + u)
//   kind 1: active-active, all ordered (u, v): (n_core + u, n_core + v)
//   kind 2: active-active unordered k <= l with slot k*na + l, for the density/energy
__global__ void build_active_pairs_kernel(int kind, int m0, int ncore, int n_core, int na, int2* pairs, int* slots) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (kind == 0) {
    if (t >= ncore * na) return;
    pairs[t] = make_int2(m0 + t / na, n_core + t % na);
    if (slots) slots[t] = t;
  } else if (kind == 1) {
    if (t >= na * na) return;
    pairs[t] = make_int2(n_core + t / na, n_core + t % na);
    if (slots) slots[t] = t;
  } else {
    if (t >= na * (na + 1) / 2) return;
    int k = 0, rem = t;
    while (rem >= na - k) {
      rem -= na - k;
      ++k;
    }
    const int l = k + rem;
    pairs[t] = make_int2(n_core + k, n_core + l);
    if (slots) slots[t] = k * na + l;
  }
}

hipError_t launch_build_active_pairs(int kind, int m0, int ncore, int n_core, int na, int2* pairs, int* slots,
                                     hipStream_t st) {
  const int n = kind == 0 ? ncore * na : (kind == 1 ? na * na : na * (na + 1) / 2);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(build_active_pairs_kernel, dim3((n + 127) / 128), dim3(128), 0, st, kind, m0, ncore, n_core, na,
                     pairs, slots);
  return hipGetLastError();
}

// Per-pair weights of the rotated pairs.  occ = natural occupations n_k of Gamma_act.
//   core-active (kind 0): density weight n_k per ordered pair, energy n_k per unordered pair
//   active-active (kind 2): density n_k n_l / 2 per ordered pair;
//                           energy n_k n_l / 2 (k < l) or n_k^2 / 4 (k = l)
__global__ void active_weights_kernel(int kind, int n, int n_core, int na, const int2* pairs, const double* occ,
                                      double scale_d, double* wd, double* we) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int2 pr = pairs[t];
  if (kind == 0) {
    const double nk = occ[pr.y - n_core];
    wd[t] = scale_d * nk;
    we[t] = nk;
  } else {
    const double nk = occ[pr.x - n_core], nl = occ[pr.y - n_core];
    wd[t] = scale_d * 0.5 * nk * nl;
    we[t] = (pr.x == pr.y) ? 0.25 * nk * nl : 0.5 * nk * nl;
  }
}

hipError_t launch_active_weights(int kind, int n, int n_core, int na, const int2* pairs, const double* occ,
                                 double scale_d, double* wd, double* we, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(active_weights_kernel, dim3((n + 127) / 128), dim3(128), 0, st, kind, n, n_core, na, pairs, occ,
                     scale_d, wd, we);
  return hipGetLastError();
}

// <Vr', 2T' - T'^T> over one 64 x 64 tile (A, B) of one rotated pair; the
// transposed tile T'[B, A] is staged through LDS so that every global read is
// row-contiguous.  part[p * nt * nt + A * nt + B].
__global__ __launch_bounds__(256) void rotated_energy_kernel(const double* T, const double* Vr, const int* slot,
                                                             int n_v, int nt, double* part) {
  __shared__ double tt[64][65];
  __shared__ double red[4];
  const int A = blockIdx.x / nt, Bb = blockIdx.x % nt;
  const int p = blockIdx.y;
  const size_t off = (size_t)slot[p] * n_v * n_v;
  const double* Tp = T + off;
  const double* Vp = Vr + off;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // stage T'[B-block rows][A-block cols] transposed: tt[x][y] = T'[B*64 + y][A*64 + x]
  for (int y = ty; y < 64; y += 4) {
    const int gr = Bb * 64 + y, gc = A * 64 + tx;
    tt[tx][y] = (gr < n_v && gc < n_v) ? Tp[(size_t)gr * n_v + gc] : 0.0;
  }
  __syncthreads();
  double acc = 0.0;
  for (int y = ty; y < 64; y += 4) {
    const int ga = A * 64 + y, gb = Bb * 64 + tx;
    if (ga < n_v && gb < n_v) {
      const size_t o = (size_t)ga * n_v + gb;
      acc += Vp[o] * (2.0 * Tp[o] - tt[y][tx]);
    }
  }
  acc = wave_sum(acc);
  if (tx == 0) red[ty] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)p * nt * nt + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_rotated_energy(const double* T, const double* Vr, const int* slot, int n_pairs, int n_v,
                                 double* part, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  const int nt = (n_v + 63) / 64;
  hipLaunchKernelGGL(rotated_energy_kernel, dim3(nt * nt, n_pairs), dim3(256), 0, st, T, Vr, slot, n_v, nt, part);
  return hipGetLastError();
}

// pe[p] (double-double) = we[p] * sum of the tile partials of pair p
__global__ void weighted_pair_reduce_kernel(const double* part, int ntile, int n_pairs, const double* we,
                                            double* pe) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n_pairs) return;
  double hi = 0.0, lo = 0.0;
  for (int k = lane; k < ntile; k += 64) dd_add(hi, lo, we[p] * part[(size_t)p * ntile + k]);
  wave_sum_dd(hi, lo);
  if (lane == 0) {
    pe[2 * (size_t)p] = hi;
    pe[2 * (size_t)p + 1] = lo;
  }
}

hipError_t launch_weighted_pair_reduce(const double* part, int ntile, int n_pairs, const double* we, double* pe,
                                       hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(weighted_pair_reduce_kernel, dim3((n_pairs + 3) / 4), dim3(256), 0, st, part, ntile, n_pairs,
                     we, pe);
  return hipGetLastError();
}

// E = sum of core-core pair energies (count on the device) + the rotated-pair
// energies pe_act[0 .. n_act_pairs), in double-double, written to e_out[2].
// Rotated pairs write their ||T||_F into pair_tnorm (semicanonical, ordered).
__global__ void energy_finalize_active_kernel(const double* pe, const int* count, const double* pe_act,
                                              int n_act_pairs, double* e_out) {
  __shared__ double sh[2][16];
  const int n = *count;
  double hi = 0.0, lo = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) dd_add_dd(hi, lo, pe[2 * p], pe[2 * p + 1]);
  for (int p = threadIdx.x; p < n_act_pairs; p += blockDim.x) dd_add_dd(hi, lo, pe_act[2 * p], pe_act[2 * p + 1]);
  wave_sum_dd(hi, lo);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    sh[0][w] = hi;
    sh[1][w] = lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double h = 0.0, l = 0.0;
    for (int k = 0; k < nw; ++k) dd_add_dd(h, l, sh[0][k], sh[1][k]);
    e_out[0] = h;
    e_out[1] = l;
  }
}

hipError_t launch_energy_finalize_active(const double* pe, const int* count, const double* pe_act, int n_act_pairs,
                                         double* e_out, hipStream_t st) {
  hipLaunchKernelGGL(energy_finalize_active_kernel, dim3(1), dim3(1024), 0, st, pe, count, pe_act, n_act_pairs, e_out);
  return hipGetLastError();
}

// pair_energy = NaN and pair_tnorm = ||T||_F for pairs with an active hole
__global__ void scatter_active_pair_info_kernel(const int2* pairs, const double* tn2, int n, int n_h,
                                                double* pair_energy, float* pair_tnorm) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int2 pr = pairs[t];
  if (pair_energy) {
    pair_energy[(size_t)pr.x * n_h + pr.y] = __builtin_nan("");
    pair_energy[(size_t)pr.y * n_h + pr.x] = __builtin_nan("");
  }
  if (pair_tnorm && tn2) {
    const float v = (float)sqrt(tn2[t]);
    pair_tnorm[(size_t)pr.x * n_h + pr.y] = v;
    pair_tnorm[(size_t)pr.y * n_h + pr.x] = v;
  }
}

hipError_t launch_scatter_active_pair_info(const int2* pairs, const double* tn2, int n, int n_h, double* pair_energy,
                                           float* pair_tnorm, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_active_pair_info_kernel, dim3((n + 127) / 128), dim3(128), 0, st, pairs, tn2, n, n_h,
                     pair_energy, pair_tnorm);
  return hipGetLastError();
}

}  // namespace dfpt2
