// FP64 symmetric eigensolver on the GPU, for the natural-orbital problem of
// Eq. 8 (Gamma V = n V) and for the recanonicalization of the kept space.
//
//   1. Householder reduction to tridiagonal form, one column per step on the
//      full symmetric matrix: the reflector (formed redundantly in every
//      workgroup), p = tau A v and the rank-2 update A -= v w^T + w v^T with
//      w = p - (tau/2)(p.v) v.  Up to n = 2731 one launch per column applies the
//      previous column's update lazily while forming p; above, two launches.
//   2. Splitting at negligible off-diagonal entries, then every eigenvalue by
//      multisection on Sturm counts (one wave per eigenvalue, 64 points a round).
//   3. Eigenvectors of the tridiagonal matrix by inverse iteration with a
//      partially pivoted LU of T - lambda I; eigenvalues closer than a small
//      multiple of ||T|| form a group that one thread handles in order,
//      orthogonalizing every iterate against the group's earlier vectors.
//   4. Back-transformation Z <- H_0 H_1 ... H_{n-3} Z in compact-WY blocks of 8
//      reflectors, one workgroup per 4 (2, 1 for large n) columns held in LDS,
//      all blocks in one launch.
//   5. One first-order orthonormalization of all columns (two FP64 GEMMs): it
//      restores orthogonality between vectors of close eigenvalues that inverse
//      iteration did not group.
//   6. Columns sorted by eigenvalue and oriented so that the largest-magnitude
//      component is positive.
#include <cmath>
#include <cfloat>

#include "common.h"
#include "eigh.h"

namespace dfpt2 {

namespace {

__device__ inline double block_sum(double v, double* sh) {
  // 256-thread workgroup sum; sh holds >= 4 doubles; ends with a barrier
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += sh[k];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------- step a
// Reflector of column k and p = tau A22 v, rows split over the grid.
__global__ __launch_bounds__(256) void tridiag_step_a(const double* A, int n, int k, double* Vs,
                                                      double* tau, double* d, double* e, double* p) {
  extern __shared__ double vsh[];  // m doubles
  __shared__ double red[8];
  const int m = n - k - 1;
  const double* rowk = A + (size_t)k * n + (k + 1);  // x_i = A[k][k+1+i] (symmetric)
  double s2 = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += blockDim.x) s2 += rowk[i] * rowk[i];
  s2 = block_sum(s2, red);
  const double alpha = rowk[0];
  double t = 0.0, beta = alpha, scale = 0.0;
  if (s2 > 0.0) {
    const double mu = sqrt(alpha * alpha + s2);
    beta = (alpha > 0.0) ? -mu : mu;
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x) vsh[i] = (i == 0) ? 1.0 : rowk[i] * scale;
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) Vs[(size_t)k * n + i] = vsh[i];
    if (threadIdx.x == 0) {
      tau[k] = t;
      e[k] = beta;
      d[k] = A[(size_t)k * n + k];
    }
  }
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  for (int r = gw; r < m; r += nwaves) {
    const double* row = A + (size_t)(k + 1 + r) * n + (k + 1);
    double acc = 0.0;
    for (int c = lane; c < m; c += 64) acc += row[c] * vsh[c];
    acc = wave_sum(acc);
    if (lane == 0) p[r] = t * acc;
  }
}

// ---------------------------------------------------------------- step b
// A22 -= v w^T + w v^T, w = p - (tau/2)(p.v) v.  grid.x over columns, grid.y over row bands.
__global__ __launch_bounds__(256) void tridiag_step_b(double* A, int n, int k, const double* Vs,
                                                      const double* tau, const double* p) {
  __shared__ double red[8];
  const int m = n - k - 1;
  const double t = tau[k];
  if (t == 0.0) return;
  const double* v = Vs + (size_t)k * n;
  double dot = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) dot += p[i] * v[i];
  dot = block_sum(dot, red);
  const double K = 0.5 * t * dot;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const double vc = v[c];
  const double wc = p[c] - K * vc;
  const int rows_per = (m + gridDim.y - 1) / gridDim.y;
  const int r0 = blockIdx.y * rows_per;
  const int r1 = min(m, r0 + rows_per);
  for (int r = r0; r < r1; ++r) {
    const double vr = v[r];
    const double wr = p[r] - K * vr;
    double* a = A + (size_t)(k + 1 + r) * n + (k + 1 + c);
    *a -= vr * wc + wr * vc;
  }
}

// ---------------------------------------------------------------- fused step
// Column k with the rank-2 update of column k - 1 applied lazily: the update
// A -= v' w'^T + w' v'^T of column k - 1 (over indices k .. n - 1; w' = p' -
// (tau'/2)(p'.v') v' rebuilt here from p' = p of column k - 1) is applied to row k
// on the fly (it gives the reflector and d[k]) and, row by row, to the trailing
// block k + 1 .. n - 1, which is stored back and multiplied by v_k in the same
// pass: one launch per column instead of two, and each trailing row read and
// written once.  v', w' and v_k are staged in LDS ((3 m + 2) doubles, m = n - k - 1).
__global__ __launch_bounds__(256) void tridiag_step_lazy(double* A, int n, int k, double* Vs, double* tau,
                                                         double* d, double* e, const double* p_prev,
                                                         double* p_out) {
  extern __shared__ double sh[];
  const int m = n - k - 1;
  double* vsh = sh;           // v_k: m
  double* vpr = sh + m;       // v': m + 1 (index k + i)
  double* wpr = vpr + m + 1;  // w': m + 1
  __shared__ double red[8];
  if (k > 0) {  // workgroup-uniform
    const double* vp = Vs + (size_t)(k - 1) * n;
    double dot = 0.0;
    for (int i = threadIdx.x; i <= m; i += blockDim.x) dot += p_prev[i] * vp[i];
    dot = block_sum(dot, red);
    const double K = 0.5 * tau[k - 1] * dot;
    for (int i = threadIdx.x; i <= m; i += blockDim.x) {
      vpr[i] = vp[i];
      wpr[i] = p_prev[i] - K * vp[i];
    }
  } else {
    for (int i = threadIdx.x; i <= m; i += blockDim.x) vpr[i] = wpr[i] = 0.0;
  }
  __syncthreads();
  const double v0 = vpr[0], w0 = wpr[0];
  const double* rowk = A + (size_t)k * n + (k + 1);
  double s2 = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += blockDim.x) {
    const double x = rowk[i] - (v0 * wpr[1 + i] + w0 * vpr[1 + i]);
    s2 += x * x;
  }
  s2 = block_sum(s2, red);
  const double alpha = rowk[0] - (v0 * wpr[1] + w0 * vpr[1]);
  double t = 0.0, beta = alpha, scale = 0.0;
  if (s2 > 0.0) {
    const double mu = sqrt(alpha * alpha + s2);
    beta = (alpha > 0.0) ? -mu : mu;
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x)
    vsh[i] = (i == 0) ? 1.0 : (rowk[i] - (v0 * wpr[1 + i] + w0 * vpr[1 + i])) * scale;
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) Vs[(size_t)k * n + i] = vsh[i];
    if (threadIdx.x == 0) {
      tau[k] = t;
      e[k] = beta;
      d[k] = A[(size_t)k * n + k] - 2.0 * v0 * w0;
    }
  }
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  for (int r = gw; r < m; r += nwaves) {
    double* row = A + (size_t)(k + 1 + r) * n + (k + 1);
    const double vr = vpr[1 + r], wr = wpr[1 + r];
    double acc = 0.0;
    for (int c = lane; c < m; c += 64) {
      const double a = row[c] - (vr * wpr[1 + c] + wr * vpr[1 + c]);
      row[c] = a;
      acc += a * vsh[c];
    }
    acc = wave_sum(acc);
    if (lane == 0) p_out[r] = t * acc;
  }
}

// d[n-2], d[n-1], e[n-2] from the last 2 x 2 block, with the update of column n - 3
// still pending when the lazy steps were used (p_last = p of column n - 3)
__global__ void tridiag_tail_lazy(const double* A, int n, const double* Vs, const double* tau,
                                  const double* p_last, double* d, double* e) {
  if (threadIdx.x != 0) return;
  const double* v = Vs + (size_t)(n - 3) * n;  // entries 0, 1 <-> indices n - 2, n - 1
  const double K = 0.5 * tau[n - 3] * (p_last[0] * v[0] + p_last[1] * v[1]);
  const double w0 = p_last[0] - K * v[0], w1 = p_last[1] - K * v[1];
  d[n - 2] = A[(size_t)(n - 2) * n + (n - 2)] - 2.0 * v[0] * w0;
  d[n - 1] = A[(size_t)(n - 1) * n + (n - 1)] - 2.0 * v[1] * w1;
  e[n - 2] = A[(size_t)(n - 1) * n + (n - 2)] - (v[1] * w0 + w1 * v[0]);
}

__global__ void tridiag_tail(const double* A, int n, double* d, double* e) {
  if (threadIdx.x != 0) return;
  if (n >= 2) {
    d[n - 2] = A[(size_t)(n - 2) * n + (n - 2)];
    d[n - 1] = A[(size_t)(n - 1) * n + (n - 1)];
    e[n - 2] = A[(size_t)(n - 1) * n + (n - 2)];
  } else {
    d[0] = A[0];
  }
}

// ---------------------------------------------------------------- splitting
// Zero negligible off-diagonals, record unreduced blocks: blk_of[pos] = start of
// the block containing pos; blk_end[pos] = one past its end.  Also the norm.
__global__ void tridiag_split(int n, const double* d, double* e, int* blk_start, int* blk_end,
                              double* tnorm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double nrm = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    nrm = fmax(nrm, r);
  }
  *tnorm = nrm;
  const double eps = DBL_EPSILON;
  int start = 0;
  for (int i = 0; i < n; ++i) {
    bool brk = (i == n - 1);
    if (!brk) {
      const double ee = fabs(e[i]);
      if (ee <= eps * sqrt(fabs(d[i])) * sqrt(fabs(d[i + 1])) || ee <= DBL_MIN * 1e6 || ee <= 1e-300) {
        e[i] = 0.0;
        brk = true;
      }
    }
    if (brk) {
      for (int q = start; q <= i; ++q) {
        blk_start[q] = start;
        blk_end[q] = i + 1;
      }
      start = i + 1;
    }
  }
}

// Number of eigenvalues of the block [s, t) smaller than x (Sturm sequence).
__device__ int sturm_count(const double* d, const double* e, int s, int t, double x, double pivmin) {
  int cnt = 0;
  double q = d[s] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = s + 1; i < t; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Wave g (four per workgroup): the (g - start)-th eigenvalue of the block
// containing position g, by multisection: each lane takes the Sturm count at one
// of 64 interior points of the bracket, and the bracket shrinks to the interval
// between the highest point whose count is <= j and the lowest point above it
// whose count is > j (65x per round instead of 2x, so ~9 rounds of parallel
// counts instead of ~55 sequential ones).  The invariant count(lo) <= j <
// count(hi) holds whatever the rounding of the points or counts; the stopping
// rule is that of the bisection below.
__global__ __launch_bounds__(256) void tridiag_multisect(int n, const double* d, const double* e,
                                                         const int* blk_start, const int* blk_end,
                                                         const double* tnorm, double* lam) {
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (g >= n) return;  // wave-uniform
  const int s = blk_start[g], t = blk_end[g], j = g - s;
  double lo = DBL_MAX, hi = -DBL_MAX;
  for (int i = s + lane; i < t; i += 64) {
    const double r = (i > s ? fabs(e[i - 1]) : 0.0) + (i + 1 < t ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  const double nrm = fmax(*tnorm, DBL_MIN);
  const double pivmin = DBL_MIN * fmax(1.0, nrm * nrm) * 4.0;
  const double pad = 2.0 * DBL_EPSILON * nrm * (t - s) + 2.0 * pivmin;
  lo -= pad;
  hi += pad;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    const double x = fmin(fmax(lo + (double)(lane + 1) * ((hi - lo) / 65.0), lo), hi);
    const bool le = (x <= lo) ? true : (x >= hi) ? false : (sturm_count(d, e, s, t, x, pivmin) <= j);
    const unsigned long long m = __ballot(le);
    const int klo = m ? 63 - __clzll((long long)m) : -1;
    const unsigned long long above = ~m & (klo >= 63 ? 0ull : (~0ull << (klo + 1)));
    const int khi = above ? __ffsll((long long)above) - 1 : 64;
    const double nlo = klo >= 0 ? __shfl(x, klo, 64) : lo;
    const double nhi = khi < 64 ? __shfl(x, khi, 64) : hi;
    if (!(nlo > lo || nhi < hi)) break;  // the points no longer split the bracket
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[g] = 0.5 * (lo + hi);
}

// ------------------------------------------------------------ inverse iteration
struct LuCols {
  double *u1, *u2, *u3, *l, *piv;  // [pos][n] layout, column g owned by thread g
};

__device__ inline double hash_unit(unsigned a, unsigned b) {
  unsigned h = a * 2654435761u ^ (b + 0x9e3779b9u + (a << 6) + (a >> 2));
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  h ^= h >> 16;
  return ((double)(h & 0xffffff) / 16777216.0) - 0.5;
}

// Factor T_b - lam I (block [s, t)) into column g of the LU arrays.
__device__ void lu_factor(const double* d, const double* e, int s, int t, double lam, double tiny,
                          const LuCols& L, int n, int g) {
  double alpha = d[s] - lam;
  double beta = (s + 1 < t) ? e[s] : 0.0;
  for (int i = s; i < t - 1; ++i) {
    const double c = e[i];
    const double an = d[i + 1] - lam;
    const double bn = (i + 2 < t) ? e[i + 1] : 0.0;
    const size_t o = (size_t)i * n + g;
    if (fabs(alpha) >= fabs(c)) {
      double a_ = alpha;
      if (a_ == 0.0) a_ = tiny;
      const double mlt = c / a_;
      L.u1[o] = a_;
      L.u2[o] = beta;
      L.u3[o] = 0.0;
      L.l[o] = mlt;
      L.piv[o] = 0.0;
      alpha = an - mlt * beta;
      beta = bn;
    } else {
      const double mlt = alpha / c;
      L.u1[o] = c;
      L.u2[o] = an;
      L.u3[o] = bn;
      L.l[o] = mlt;
      L.piv[o] = 1.0;
      alpha = beta - mlt * an;
      beta = -mlt * bn;
    }
  }
  const size_t o = (size_t)(t - 1) * n + g;
  L.u1[o] = (alpha == 0.0) ? tiny : alpha;
  L.u2[o] = 0.0;
  L.u3[o] = 0.0;
}

// Solve in place: x (column g of X over positions [s, t)) <- (T - lam I)^{-1} (scl x);
// returns max |x| of the result.  The values each step produces for the next are
// carried in registers, so the loads of a step depend on nothing written by the
// one before.
__device__ double lu_solve(int s, int t, const LuCols& L, int n, int g, double* __restrict__ X, int xcol,
                           double scl) {
  const double* __restrict__ u1 = L.u1;
  const double* __restrict__ u2 = L.u2;
  const double* __restrict__ u3 = L.u3;
  const double* __restrict__ lm = L.l;
  const double* __restrict__ pv = L.piv;
  double yi = X[(size_t)s * n + xcol] * scl;
#pragma unroll 4
  for (int i = s; i < t - 1; ++i) {
    const size_t o = (size_t)i * n + g;
    double yn = X[(size_t)(i + 1) * n + xcol] * scl;
    if (pv[o] != 0.0) {
      const double tmp = yi;
      yi = yn;
      yn = tmp;
    }
    yn -= lm[o] * yi;
    X[(size_t)i * n + xcol] = yi;
    yi = yn;
  }
  X[(size_t)(t - 1) * n + xcol] = yi;
  double x1 = 0.0, x2 = 0.0;  // the solved X[i + 1], X[i + 2]
  double mx = 0.0;
#pragma unroll 4
  for (int i = t - 1; i >= s; --i) {
    const size_t o = (size_t)i * n + g;
    double v = X[(size_t)i * n + xcol];
    if (i + 1 < t) v -= u2[o] * x1;
    if (i + 2 < t) v -= u3[o] * x2;
    v = v / u1[o];
    X[(size_t)i * n + xcol] = v;
    mx = fmax(mx, fabs(v));
    x2 = x1;
    x1 = v;
  }
  return mx;
}

// Group leaders (first eigenvalue of a near-degenerate run inside a block) compute
// the vectors of their whole group; X is row-major n x n, column g = vector g.
// vec_floor: if non-null, eigenvectors are formed only for eigenvalues above
// *vec_floor; the other columns of X are zero (callers that drop those
// eigenpairs, such as the NAF compression, skip the cost of large clusters).
__global__ void tridiag_inverse_iteration(int n, const double* d, const double* e, const int* blk_start,
                                          const int* blk_end, const double* tnorm, const double* lam,
                                          LuCols L, double* X, int* status, const double* vec_floor) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int s = blk_start[g], t = blk_end[g];
  if (vec_floor && !(lam[g] > *vec_floor)) {
    for (int i = 0; i < n; ++i) X[(size_t)i * n + g] = 0.0;
    return;
  }
  const double nrm = (*tnorm > 0.0) ? *tnorm : 1.0;
  const double grp_tol = 1e-10 * nrm;
  if (t - s == 1) {  // a 1 x 1 block: the unit vector
    for (int i = 0; i < n; ++i) X[(size_t)i * n + g] = (i == s) ? 1.0 : 0.0;
    return;
  }
  // a leader above the floor starts its group; earlier members below the floor were zeroed
  if (vec_floor && g > s && fabs(lam[g] - lam[g - 1]) <= grp_tol && !(lam[g - 1] > *vec_floor)) {
    // lam[g - 1] was skipped: g leads what remains of the group
  } else if (g > s && fabs(lam[g] - lam[g - 1]) <= grp_tol) {
    return;
  }
  int g1 = g + 1;
  while (g1 < t && fabs(lam[g1] - lam[g1 - 1]) <= grp_tol) ++g1;
  const double tiny = DBL_EPSILON * nrm;
  for (int q = g; q < g1; ++q) {
    // zero the column outside the block, random start inside
    for (int i = 0; i < n; ++i) X[(size_t)i * n + q] = (i >= s && i < t) ? hash_unit(q, i) : 0.0;
    // eigenvalues of a group are spread by a few ulps so that the factors differ
    const double lq = lam[q] + (double)(q - g) * 4.0 * DBL_EPSILON * nrm;
    lu_factor(d, e, s, t, lq, tiny, L, n, g);
    // the solves and the orthogonalization are linear, so between iterations the
    // vector is only rescaled against overflow (by 1 / max |x|, applied as the
    // next solve loads it); it is normalized once at the end
    double scl = 1.0;
    for (int it = 0; it < 4; ++it) {
      double mx = lu_solve(s, t, L, n, g, X, q, scl);
      if (q > g) {
        // orthogonalize against earlier (unit) vectors of the group, twice for stability
        mx = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
          for (int r = g; r < q; ++r) {
            double dp = 0.0;
            for (int i = s; i < t; ++i) dp += X[(size_t)i * n + r] * X[(size_t)i * n + q];
            for (int i = s; i < t; ++i) {
              const double y = X[(size_t)i * n + q] - dp * X[(size_t)i * n + r];
              X[(size_t)i * n + q] = y;
              if (pass == 1 && r == q - 1) mx = fmax(mx, fabs(y));
            }
          }
        }
      }
      if (!(mx > 0.0) || !isfinite(mx)) {
        atomicExch(status, 1);
        return;
      }
      scl = 1.0 / mx;
    }
    double nx = 0.0;
    for (int i = s; i < t; ++i) {
      const double y = X[(size_t)i * n + q] * scl;
      nx += y * y;
    }
    const double inv = scl / sqrt(nx);
    for (int i = s; i < t; ++i) X[(size_t)i * n + q] *= inv;
  }
}

// ------------------------------------------------------------ back-transform
// Z <- H_0 H_1 ... H_{n-3} Z with H_k = I - tau_k v_k v_k^T (v_k: 1 at row k + 1,
// Vs[k][.] below it), applied in compact-WY blocks of WY_NB reflectors: for the
// block k0 .. k0 + WY_NB - 1, H_k0 ... H_{k0+WY_NB-1} = I - V T V^T with T upper
// triangular (T_cc = tau_c, T[0:c, c] = -tau_c T[0:c, 0:c] V[:, 0:c]^T v_c), and the
// blocks go from the last to the first: Z <- Z - V (T (V^T Z)).
constexpr int WY_NB = 8;

// V[i][j] of block k0 (row i of the full vector of reflector k0 + j), 0 outside
__device__ inline double wy_v(const double* Vs, int n, int k0, int nr, int i, int j) {
  const int k = k0 + j;
  return (j < nr && i > k) ? Vs[(size_t)k * n + (i - k - 1)] : 0.0;
}

// One workgroup per block: S = V^T V (upper triangle) by a pass over the rows,
// then T by the forward recurrence (one thread).  T: [nblk][WY_NB][WY_NB].
__global__ __launch_bounds__(256) void wy_build_t(int n, const double* Vs, const double* tau, double* Tout) {
  constexpr int NS = WY_NB * (WY_NB + 1) / 2;
  __shared__ double part[4][NS];
  __shared__ double S[WY_NB][WY_NB];
  const int b = blockIdx.x, k0 = b * WY_NB;
  const int nr = min(WY_NB, n - 2 - k0);  // reflectors 0 .. n - 3
  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  for (int i = k0 + 1 + threadIdx.x; i < n; i += blockDim.x) {
    double v[WY_NB];
#pragma unroll
    for (int j = 0; j < WY_NB; ++j) v[j] = wy_v(Vs, n, k0, nr, i, j);
    int q = 0;
#pragma unroll
    for (int l = 0; l < WY_NB; ++l)
#pragma unroll
      for (int c = l; c < WY_NB; ++c) acc[q++] += v[l] * v[c];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) part[w][q] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int q = 0;
    for (int l = 0; l < WY_NB; ++l)
      for (int c = l; c < WY_NB; ++c, ++q) S[l][c] = (part[0][q] + part[1][q]) + (part[2][q] + part[3][q]);
    double T[WY_NB][WY_NB];
    for (int c = 0; c < WY_NB; ++c) {
      const double tc = c < nr ? tau[k0 + c] : 0.0;
      for (int i = 0; i < WY_NB; ++i) T[i][c] = 0.0;
      T[c][c] = tc;
      for (int i = 0; i < c; ++i) {
        double sum = 0.0;
        for (int l = i; l < c; ++l) sum += T[i][l] * S[l][c];
        T[i][c] = -tc * sum;
      }
    }
    double* To = Tout + (size_t)b * WY_NB * WY_NB;
    for (int i = 0; i < WY_NB; ++i)
      for (int c = 0; c < WY_NB; ++c) To[i * WY_NB + c] = T[i][c];
  }
}

// One workgroup per WY_CW columns of Z, held in LDS; the blocks of reflectors in
// reverse order, two barriers per block.
template <int WY_CW>
__global__ __launch_bounds__(256) void tridiag_backtransform(int n, const double* Vs, const double* Tall,
                                                             double* Z) {
  extern __shared__ double zs[];  // [n][WY_CW]
  __shared__ double part[4][WY_NB * WY_CW];
  __shared__ double Wsh[WY_NB][WY_CW];
  const int c0 = blockIdx.x * WY_CW;
  const int ncol = min(WY_CW, n - c0);
  for (int idx = threadIdx.x; idx < n * WY_CW; idx += blockDim.x) {
    const int r = idx / WY_CW, c = idx % WY_CW;
    zs[idx] = (c < ncol) ? Z[(size_t)r * n + c0 + c] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nblk = (n - 2 + WY_NB - 1) / WY_NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * WY_NB, nr = min(WY_NB, n - 2 - k0);
    // P = V^T Z over the rows below k0
    double acc[WY_NB][WY_CW];
#pragma unroll
    for (int j = 0; j < WY_NB; ++j)
#pragma unroll
      for (int c = 0; c < WY_CW; ++c) acc[j][c] = 0.0;
    for (int i = k0 + 1 + threadIdx.x; i < n; i += blockDim.x) {
      const double* zr = zs + (size_t)i * WY_CW;
#pragma unroll
      for (int j = 0; j < WY_NB; ++j) {
        const double v = wy_v(Vs, n, k0, nr, i, j);
#pragma unroll
        for (int c = 0; c < WY_CW; ++c) acc[j][c] += v * zr[c];
      }
    }
#pragma unroll
    for (int j = 0; j < WY_NB; ++j)
#pragma unroll
      for (int c = 0; c < WY_CW; ++c) {
        const double t = wave_sum(acc[j][c]);
        if (lane == 0) part[w][j * WY_CW + c] = t;
      }
    __syncthreads();
    // W = T P (T upper triangular)
    if (threadIdx.x < WY_NB * WY_CW) {
      const int j = threadIdx.x / WY_CW, c = threadIdx.x % WY_CW;
      const double* T = Tall + (size_t)b * WY_NB * WY_NB;
      double sum = 0.0;
      for (int l = j; l < WY_NB; ++l) {
        const int q = l * WY_CW + c;
        sum += T[j * WY_NB + l] * ((part[0][q] + part[1][q]) + (part[2][q] + part[3][q]));
      }
      Wsh[j][c] = sum;
    }
    __syncthreads();
    // Z -= V W
    for (int i = k0 + 1 + threadIdx.x; i < n; i += blockDim.x) {
      double* zr = zs + (size_t)i * WY_CW;
      double u[WY_CW];
#pragma unroll
      for (int c = 0; c < WY_CW; ++c) u[c] = 0.0;
#pragma unroll
      for (int j = 0; j < WY_NB; ++j) {
        const double v = wy_v(Vs, n, k0, nr, i, j);
#pragma unroll
        for (int c = 0; c < WY_CW; ++c) u[c] += v * Wsh[j][c];
      }
#pragma unroll
      for (int c = 0; c < WY_CW; ++c) zr[c] -= u[c];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n * WY_CW; idx += blockDim.x) {
    const int r = idx / WY_CW, c = idx % WY_CW;
    if (c < ncol) Z[(size_t)r * n + c0 + c] = zs[idx];
  }
}

// ------------------------------------------------------------ sort + orient
// rank of eigenvalue g among all (ties by index), ascending
__global__ void eig_rank(int n, const double* lam, int* rank) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double x = lam[g];
  int r = 0;
  for (int q = 0; q < n; ++q) {
    const double y = lam[q];
    r += (y < x || (y == x && q < g)) ? 1 : 0;
  }
  rank[g] = r;
}

// out column dst(g) = sign-oriented column g; descending: dst = n-1-rank
// M = I - U with U = strictly upper part of E + diag(E) / 2, where E = Z^T Z - I
// arrives as G = Z^T Z in M (in place)
__global__ void orth_correction(int n, double* M) {
  const size_t nn = (size_t)n * n;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nn; k += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(k / n), j = (int)(k - (size_t)i * n);
    const double g = M[k];
    M[k] = i < j ? -g : i == j ? 1.0 - 0.5 * (g - 1.0) : 0.0;
  }
}

__global__ void eig_permute(int n, const double* lam, const int* rank, const double* Zin, double* w_out,
                            double* Z_out, int descending) {
  const int g = blockIdx.x;
  __shared__ double bestv[4];
  __shared__ int besti[4];
  double bv = -1.0;
  int bi = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double a = fabs(Zin[(size_t)i * n + g]);
    if (a > bv || (a == bv && i < bi)) {
      bv = a;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    bestv[w] = bv;
    besti[w] = bi;
  }
  __syncthreads();
  bv = bestv[0];
  bi = besti[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
    if (bestv[q] > bv || (bestv[q] == bv && besti[q] < bi)) {
      bv = bestv[q];
      bi = besti[q];
    }
  const double sgn = (Zin[(size_t)bi * n + g] < 0.0) ? -1.0 : 1.0;
  const int dst = descending ? (n - 1 - rank[g]) : rank[g];
  if (threadIdx.x == 0) w_out[dst] = lam[g];
  for (int i = threadIdx.x; i < n; i += blockDim.x) Z_out[(size_t)i * n + dst] = sgn * Zin[(size_t)i * n + g];
}

// *floor = rel * (largest eigenvalue magnitude)
__global__ void lam_floor(int n, const double* lam, double rel, double* floor) {
  __shared__ double m[64];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) v = fmax(v, fabs(lam[i]));
  m[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 64; ++i) v = fmax(v, m[i]);
    *floor = rel * fmax(v, m[0]);
  }
}

__global__ void zero_int(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

}  // namespace

size_t eigh_workspace_bytes(int n) {
  const size_t nn = (size_t)n * n;
  size_t b = 0;
  auto add = [&](size_t x) { b += align_up(x, 256); };
  add(nn * 8);      // A work copy
  add(nn * 8);      // reflectors
  add(nn * 8);      // X (tridiagonal eigenvectors, then back-transformed)
  add(5 * nn * 8);  // LU columns
  add((size_t)n * 8 * 5);  // tau d e p lam
  add((size_t)n * 4 * 3 + 64);  // blk_start blk_end rank status
  add(64);          // tnorm
  add((size_t)((n + WY_NB - 1) / WY_NB + 1) * WY_NB * WY_NB * 8);  // compact-WY T factors
  return b;
}

int eigh_run(const double* A_in, int n, double* w_out, double* Z_out, char* ws, size_t ws_bytes, hipStream_t st,
             int descending, double vec_floor_rel) {
  if (n < 1 || n > kEighMaxN) return fail(DFPT2_ERR_INVALID_ARG, "eigh: n=%d outside [1, %d]", n, kEighMaxN);
  if (ws_bytes < eigh_workspace_bytes(n)) return fail(DFPT2_ERR_WORKSPACE, "eigh workspace too small");
  const size_t nn = (size_t)n * n;
  size_t off = 0;
  auto take = [&](size_t x) {
    char* p = ws + off;
    off += align_up(x, 256);
    return p;
  };
  double* A = (double*)take(nn * 8);
  double* Vs = (double*)take(nn * 8);
  double* X = (double*)take(nn * 8);
  double* lu = (double*)take(5 * nn * 8);
  double* tau = (double*)take((size_t)n * 8 * 5);
  double* d = tau + n;
  double* e = d + n;
  double* p = e + n;
  double* lam = p + n;
  int* blk_start = (int*)take((size_t)n * 4 * 3 + 64);
  int* blk_end = blk_start + n;
  int* rank = blk_end + n;
  int* status = rank + n;
  double* tnorm = (double*)take(64);
  double* Tall = (double*)take((size_t)((n + WY_NB - 1) / WY_NB + 1) * WY_NB * WY_NB * 8);
  hipError_t err;
  ProfScope prof_all(DFPT2_STAGE_EIGH, st);
  if ((err = hipMemcpyAsync(A, A_in, nn * 8, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(err, "eigh copy");
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(64), 0, st, status, 1);
  // 1. tridiagonalization: one lazy-update launch per column where its LDS
  //    staging fits in 64 KB, else the two-launch form
  if (n >= 3 && (size_t)(3 * (n - 1) + 2) * 8 <= 64 * 1024) {
    double* pb[2] = {p, lam};  // p of consecutive columns alternate (lam is free until step 2)
    for (int k = 0; k + 2 < n; ++k) {
      const int m = n - k - 1;
      int ga = (m + 3) / 4;
      if (ga > 512) ga = 512;
      hipLaunchKernelGGL(tridiag_step_lazy, dim3(ga), dim3(256), (size_t)(3 * m + 2) * 8, st, A, n, k, Vs, tau, d,
                         e, pb[(k + 1) & 1], pb[k & 1]);
    }
    hipLaunchKernelGGL(tridiag_tail_lazy, dim3(1), dim3(64), 0, st, A, n, Vs, tau, pb[(n - 3) & 1], d, e);
  } else {
    for (int k = 0; k + 2 < n; ++k) {
      const int m = n - k - 1;
      int ga = (m + 3) / 4;
      if (ga > 512) ga = 512;
      hipLaunchKernelGGL(tridiag_step_a, dim3(ga), dim3(256), (size_t)m * 8, st, A, n, k, Vs, tau, d, e, p);
      int gx = (m + 255) / 256;
      int gy = (m + 15) / 16;
      if (gy > 256) gy = 256;
      hipLaunchKernelGGL(tridiag_step_b, dim3(gx, gy), dim3(256), 0, st, A, n, k, Vs, tau, p);
    }
    hipLaunchKernelGGL(tridiag_tail, dim3(1), dim3(64), 0, st, A, n, d, e);
  }
  // 2. split + bisection
  hipLaunchKernelGGL(tridiag_split, dim3(1), dim3(64), 0, st, n, d, e, blk_start, blk_end, tnorm);
  hipLaunchKernelGGL(tridiag_multisect, dim3((n + 3) / 4), dim3(256), 0, st, n, d, e, blk_start, blk_end, tnorm,
                     lam);
  // 3. inverse iteration
  LuCols L{lu, lu + nn, lu + 2 * nn, lu + 3 * nn, lu + 4 * nn};
  const double* floor_ptr = nullptr;
  if (vec_floor_rel > 0.0) {
    hipLaunchKernelGGL(lam_floor, dim3(1), dim3(64), 0, st, n, lam, vec_floor_rel, tnorm + 1);
    floor_ptr = tnorm + 1;
  }
  hipLaunchKernelGGL(tridiag_inverse_iteration, dim3((n + 63) / 64), dim3(64), 0, st, n, d, e, blk_start, blk_end,
                     tnorm, lam, L, X, status, floor_ptr);
  // 4. back-transformation (compact-WY blocks)
  if (n > 2) {
    int cw = 4;  // columns per workgroup: as many as the LDS holds, up to 4
    while (cw > 1 && (size_t)n * cw * 8 > 150 * 1024) cw >>= 1;
    if ((size_t)n * cw * 8 > 150 * 1024) return fail(DFPT2_ERR_UNSUPPORTED, "eigh: n=%d too large", n);
    const int nblk = (n - 2 + WY_NB - 1) / WY_NB;
    hipLaunchKernelGGL(wy_build_t, dim3(nblk), dim3(256), 0, st, n, Vs, tau, Tall);
    const dim3 grid((n + cw - 1) / cw), block(256);
    const size_t lds = (size_t)n * cw * 8;
    if (cw == 4) hipLaunchKernelGGL(tridiag_backtransform<4>, grid, block, lds, st, n, Vs, Tall, X);
    else if (cw == 2) hipLaunchKernelGGL(tridiag_backtransform<2>, grid, block, lds, st, n, Vs, Tall, X);
    else hipLaunchKernelGGL(tridiag_backtransform<1>, grid, block, lds, st, n, Vs, Tall, X);
  }
  // 5. one first-order orthonormalization of all columns: with G = Z^T Z = I + E
  //    and E small, Z <- Z (I - U), U = strict upper part of E + diag(E) / 2, leaves
  //    Z^T Z = I + O(E^2).  E is non-negligible only between vectors of close
  //    eigenvalues whose gap inverse iteration left unresolved (relative gaps
  //    just above the grouping tolerance), and mixing those moves the residuals
  //    by no more than their gap times E.  The LU columns are free by now.
  double* G = lu;
  double* Zo = lu + nn;
  if ((err = gemm_f64(X, n, 0, 1, X, n, 0, 0, G, n, 0, n, n, n, 1, 1.0, 0.0, st)) != hipSuccess)
    return hip_fail(err, "eigh orthonormalization");
  hipLaunchKernelGGL(orth_correction, dim3((unsigned)((nn + 255) / 256 < 65535 ? (nn + 255) / 256 : 65535)),
                     dim3(256), 0, st, n, G);
  if ((err = gemm_f64(X, n, 0, 0, G, n, 0, 0, Zo, n, 0, n, n, n, 1, 1.0, 0.0, st)) != hipSuccess)
    return hip_fail(err, "eigh orthonormalization");
  // 6. sort + orient
  hipLaunchKernelGGL(eig_rank, dim3((n + 255) / 256), dim3(256), 0, st, n, lam, rank);
  hipLaunchKernelGGL(eig_permute, dim3(n), dim3(256), 0, st, n, lam, rank, Zo, w_out, Z_out, descending);
  if ((err = hipGetLastError()) != hipSuccess) return hip_fail(err, "eigh launch");
  prof_all.close();
  int hs = 0;
  if ((err = hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(err, "eigh status copy");
  if ((err = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(err, "eigh sync");
  prof_flush();
  if (hs != 0) return fail(DFPT2_ERR_NOT_CONVERGED, "inverse iteration produced a zero or non-finite vector");
  return DFPT2_OK;
}

}  // namespace dfpt2
