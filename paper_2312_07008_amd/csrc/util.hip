// Small kernels: fills, pair-list compaction and the compensated energy reductions.
#include <cmath>
#include "common.h"
#include "kernels.h"

namespace dfpt2 {

__global__ void fill_kernel(double* p, size_t n, double v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// Unordered core-core pairs (i <= j) whose mask entry is set, in row-major
// order.  One wave per row i: each lane scans a strip of j, a wave prefix sum
// places the survivors, and rows are laid out by a serial scan of row counts
// done by the first wave (n_core is at most a few hundred).
__global__ void build_pairs_kernel(const uint8_t* mask, int n_core, int n_h, int2* pairs, int* count) {
  __shared__ int row_start[1025];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // row counts
  for (int i = w; i < n_core; i += nw) {
    int c = 0;
    for (int j = i + lane; j < n_core; j += 64) c += (mask == nullptr || mask[(size_t)i * n_h + j]) ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) row_start[i + 1] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    row_start[0] = 0;
    for (int i = 0; i < n_core; ++i) row_start[i + 1] += row_start[i];
    *count = row_start[n_core];
  }
  __syncthreads();
  for (int i = w; i < n_core; i += nw) {
    int base = row_start[i];
    for (int j0 = i; j0 < n_core; j0 += 64) {
      const int j = j0 + lane;
      const int keep = (j < n_core) && (mask == nullptr || mask[(size_t)i * n_h + j]) ? 1 : 0;
      // exclusive prefix within the wave
      unsigned long long bal = __ballot(keep);
      const int before = __popcll(bal & ((1ull << lane) - 1ull));
      if (keep) pairs[base + before] = make_int2(i, j);
      base += __popcll(bal);
    }
  }
}

hipError_t launch_build_pairs(const uint8_t* mask, int n_core, int n_h, int2* pairs, int* count,
                              hipStream_t st) {
  if (n_core > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(build_pairs_kernel, dim3(1), dim3(1024), 0, st, mask, n_core, n_h, pairs, count);
  return hipGetLastError();
}

// one wave per pair: double-double sum of the tile partials
__global__ void pair_reduce_kernel(const double* epart, const double* tpart, int nTP, int n_pairs,
                                   double* pe, double* tn2) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= n_pairs) return;
  double hi = 0.0, lo = 0.0, t = 0.0;
  for (int k = lane; k < nTP; k += 64) {
    if (epart) dd_add(hi, lo, epart[(size_t)p * nTP + k]);
    if (tpart) t += tpart[(size_t)p * nTP + k];
  }
  wave_sum_dd(hi, lo);
  t = wave_sum(t);
  if (lane == 0) {
    if (pe) {
      pe[2 * (size_t)p] = hi;
      pe[2 * (size_t)p + 1] = lo;
    }
    if (tn2) tn2[p] = t;
  }
}

hipError_t launch_pair_reduce(const double* epart, const double* tpart, int nTP, int n_pairs,
                              double* pe, double* tn2, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  const int wpb = 4;
  hipLaunchKernelGGL(pair_reduce_kernel, dim3((n_pairs + wpb - 1) / wpb), dim3(64 * wpb), 0, st,
                     epart, tpart, nTP, n_pairs, pe, tn2);
  return hipGetLastError();
}

// single workgroup: E = sum of pair energies in double-double; scatter of the
// per-pair values into n_h x n_h matrices.
__global__ void energy_finalize_kernel(const double* pe, const double* tn2, const int2* pairs,
                                       const int* count, int n_h, double* e_out,
                                       double* pair_energy, float* pair_tnorm) {
  __shared__ double sh[2][1024 / 64];
  const int n = *count;
  double hi = 0.0, lo = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) dd_add_dd(hi, lo, pe[2 * p], pe[2 * p + 1]);
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
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const int2 pr = pairs[p];
    const double e = pe[2 * p] + pe[2 * p + 1];
    const double half = (pr.x == pr.y) ? e : 0.5 * e;
    if (pair_energy) {
      pair_energy[(size_t)pr.x * n_h + pr.y] = half;
      pair_energy[(size_t)pr.y * n_h + pr.x] = half;
    }
    if (pair_tnorm && tn2) {
      const float tn = (float)sqrt(tn2[p]);
      pair_tnorm[(size_t)pr.x * n_h + pr.y] = tn;
      pair_tnorm[(size_t)pr.y * n_h + pr.x] = tn;
    }
  }
}

hipError_t launch_energy_finalize(const double* pe, const double* tn2, const int2* pairs,
                                  const int* count, int max_pairs, int n_h, double* e_out,
                                  double* pair_energy, float* pair_tnorm, hipStream_t st) {
  (void)max_pairs;
  hipLaunchKernelGGL(energy_finalize_kernel, dim3(1), dim3(1024), 0, st, pe, tn2, pairs, count, n_h,
                     e_out, pair_energy, pair_tnorm);
  return hipGetLastError();
}

}  // namespace dfpt2
