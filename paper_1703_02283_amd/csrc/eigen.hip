// Eigenvalues of a dense symmetric matrix: the step after the Loewdin
// transform (Section IV-A: S^{-1/2} brings H c = e S c to the standard
// problem (S^{-1/2} H S^{-1/2}) c' = e c', whose eigenvalues are the e).
//
//  1. Householder tridiagonalisation, one reflector per column: with x the
//     part of column k below the diagonal, H = I - tau v v^T maps x to
//     beta e_1; the trailing matrix B becomes H B H = B - v w^T - w v^T with
//     p = tau B v and w = p - (tau / 2)(p . v) v. The trailing matrix is kept
//     whole (both triangles), so every access is a row access. Two launches
//     per column, the update of one column fused with the product of the
//     next (look-ahead): the first row of the updated block, and from it the
//     next reflector (one workgroup); then the other rows, each updated and
//     at once multiplied by the next reflector (one wave per row). HBM-bound:
//     one read and one write of (n - k)^2 doubles per column, 16 n^3 / 3
//     bytes in all.
//  2. Multisection on the Sturm count of the tridiagonal matrix (d, e), one
//     wave per eigenvalue index, from the Gershgorin interval down to the
//     spacing of doubles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/ipr.h"
#include "ipr_host.h"

namespace ipr {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reflector of column k of the n x n matrix T (rows k+1 .. n-1 of column k,
// read as row k: T is symmetric). Writes v (v[0] = 1) to V[0..m), d[k],
// e[k] and tau to *tau.
__global__ __launch_bounds__(NT) void reflector_kernel(const double* __restrict__ T, int n, int k,
                                                       double* __restrict__ V,
                                                       double* __restrict__ d,
                                                       double* __restrict__ e,
                                                       double* __restrict__ tau) {
  __shared__ double red[NT / 64];
  __shared__ double coef[2];
  const int m = n - k - 1;
  const double* x = T + (size_t)k * n + k + 1;
  double s = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += NT) s += x[i] * x[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double xnorm2 = (red[0] + red[1]) + (red[2] + red[3]);
    const double alpha = x[0];
    d[k] = T[(size_t)k * n + k];
    if (xnorm2 == 0.0) {  // already reduced: H = I
      e[k] = alpha;
      *tau = 0.0;
      coef[0] = 0.0;
    } else {
      const double beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      e[k] = beta;
      *tau = (beta - alpha) / beta;
      coef[0] = 1.0 / (alpha - beta);
    }
  }
  __syncthreads();
  const double c = coef[0];
  for (int i = threadIdx.x; i < m; i += NT) V[i] = i == 0 ? 1.0 : x[i] * c;
}

// P[i] = tau sum_j B[i][j] V[j] for the trailing m x m block B (rows and
// columns k+1 .. n-1 of T), one wave per row; partial[b] = sum over the
// workgroup's rows of P[i] V[i].
__global__ __launch_bounds__(NT) void trail_gemv_kernel(const double* __restrict__ T, int n, int k,
                                                        const double* __restrict__ V,
                                                        const double* __restrict__ tau,
                                                        double* __restrict__ P,
                                                        double* __restrict__ partial) {
  __shared__ double red[NT / 64];
  const int m = n - k - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * (NT / 64) + wave;
  double pv = 0.0;
  if (i < m) {
    const double* row = T + (size_t)(k + 1 + i) * n + k + 1;
    double s = 0.0;
    for (int j = lane; j < m; j += 64) s += row[j] * V[j];
    s = wave_sum(s) * *tau;
    if (lane == 0) P[i] = s;
    pv = s * V[i];
  }
  if (lane == 0) red[wave] = pv;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Look-ahead step after column k (trailing block B of order m = n - k - 1,
// reflector V, tau, P = tau B V with partials): row 0 of B (row k + 1 of T)
// is updated, B_0j -= V_0 W_j + W_0 V_j with W = P - c V, c = (tau / 2) P . V,
// and the reflector of column k + 1 is formed from it: V2, tau2, d[k + 1],
// e[k + 1]. One workgroup; each thread reads back only the row entries it
// wrote itself.
__global__ __launch_bounds__(NT) void next_reflector_kernel(
    double* __restrict__ T, int n, int k, const double* __restrict__ V,
    const double* __restrict__ P, const double* __restrict__ tau,
    const double* __restrict__ partial, int nparts, double* __restrict__ V2,
    double* __restrict__ d, double* __restrict__ e, double* __restrict__ tau2) {
  __shared__ double red[NT / 64];
  __shared__ double head[2];  // updated B_00 and B_01
  __shared__ double coef[2];
  const int m = n - k - 1;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) s += partial[b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double c = 0.5 * *tau * ((red[0] + red[1]) + (red[2] + red[3]));
  __syncthreads();  // (red is reused below)
  const double v0 = V[0], w0 = P[0] - c * V[0];
  double* row = T + (size_t)(k + 1) * n + k + 1;
  double q = 0.0;  // |x|^2 beyond its first entry, x = B_0j for j = 1 .. m-1
  for (int j = threadIdx.x; j < m; j += NT) {
    const double t = row[j] - (v0 * (P[j] - c * V[j]) + w0 * V[j]);
    row[j] = t;
    if (j < 2)
      head[j] = t;
    else
      q += t * t;
  }
  q = wave_sum(q);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double xnorm2 = (red[0] + red[1]) + (red[2] + red[3]);
    const double alpha = head[1];
    d[k + 1] = head[0];
    if (xnorm2 == 0.0) {
      e[k + 1] = alpha;
      *tau2 = 0.0;
      coef[0] = 0.0;
    } else {
      const double beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      e[k + 1] = beta;
      *tau2 = (beta - alpha) / beta;
      coef[0] = 1.0 / (alpha - beta);
    }
  }
  __syncthreads();
  const double cf = coef[0];
  for (int j = threadIdx.x; j < m; j += NT)
    if (j >= 1) V2[j - 1] = j == 1 ? 1.0 : row[j] * cf;
}

// Rows 1 .. m-1 of the trailing block B of column k, one wave per row: the
// rank-2 update of columns 1 .. m-1 (column 0 is not read again), and in the
// same pass P2[i - 1] = tau2 sum_j B_ij V2[j - 1], the next column's
// product; partial2[b] = sum over the workgroup's rows of P2 V2.
__global__ __launch_bounds__(NT) void update_gemv_kernel(
    double* __restrict__ T, int n, int k, const double* __restrict__ V,
    const double* __restrict__ P, const double* __restrict__ tau,
    const double* __restrict__ partial, int nparts, const double* __restrict__ V2,
    const double* __restrict__ tau2, double* __restrict__ P2, double* __restrict__ partial2) {
  __shared__ double red[NT / 64];
  const int m = n - k - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) s += partial[b];
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  const double c = 0.5 * *tau * ((red[0] + red[1]) + (red[2] + red[3]));
  __syncthreads();  // (red is reused below)
  const int i = 1 + blockIdx.x * (NT / 64) + wave;
  double pv = 0.0;
  if (i < m) {
    const double vi = V[i], wi = P[i] - c * V[i];
    double* row = T + (size_t)(k + 1 + i) * n + k + 1;
    double acc = 0.0;
    for (int j = 1 + lane; j < m; j += 64) {
      const double t = row[j] - (vi * (P[j] - c * V[j]) + wi * V[j]);
      row[j] = t;
      acc += t * V2[j - 1];
    }
    acc = wave_sum(acc) * *tau2;
    if (lane == 0) P2[i - 1] = acc;
    pv = acc * V2[i - 1];
  }
  if (lane == 0) red[wave] = pv;
  __syncthreads();
  if (threadIdx.x == 0) partial2[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// d[n-1] = T[n-1][n-1] (the last diagonal entry, untouched by reflectors).
__global__ void last_diag_kernel(const double* __restrict__ T, int n, double* __restrict__ d) {
  if (threadIdx.x == 0) d[n - 1] = T[(size_t)(n - 1) * n + n - 1];
}

// Eigenvalue `idx` (ascending) of the symmetric tridiagonal matrix with
// diagonal d[0..n) and off-diagonal e[0..n-1), by multisection on the
// number of eigenvalues below x (Sturm count of the LDL^T pivots): one wave
// per eigenvalue, its 64 lanes counting at 64 points that cut [lo, hi] into
// 65 parts, so that every round narrows the interval 65-fold (about ten
// rounds to the spacing of doubles, against sixty bisection steps).
// Invariant: count(lo) <= idx < count(hi).
__global__ __launch_bounds__(NT) void multisect_kernel(const double* __restrict__ d,
                                                       const double* __restrict__ e, int n,
                                                       double* __restrict__ W) {
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (idx >= n) return;  // (the whole wave: idx is uniform in it)
  double lo = d[0], hi = d[0], emax = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i + 1 < n) emax = fmax(emax, fabs(e[i]));
  }
  const double scale = fmax(fabs(lo), fabs(hi));
  const double pivmin = fmax(2.2250738585072014e-308, 2.2250738585072014e-308 * emax * emax);
  lo -= 2.0 * 2.220446049250313e-16 * scale + pivmin;
  hi += 2.0 * 2.220446049250313e-16 * scale + pivmin;
  for (int round = 0; round < 64; ++round) {
    const double x = lo + (lane + 1) * ((hi - lo) / 65.0);
    int below = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    below += q < 0.0;
    for (int i = 1; i < n; ++i) {
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      below += q < 0.0;
    }
    // the lanes whose point lies above eigenvalue idx form a suffix of the wave
    const unsigned long long above = __ballot(below > idx);
    const int j = above ? __ffsll(above) - 1 : 64;
    const double xlo = __shfl(x, j > 0 ? j - 1 : 0, 64);
    const double xhi = __shfl(x, j < 64 ? j : 63, 64);
    const double nlo = j == 0 ? lo : xlo;
    const double nhi = j == 64 ? hi : xhi;
    if (!(nlo > lo || nhi < hi)) break;  // no double left between the points
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) W[idx] = 0.5 * (lo + hi);
}

struct EigWork {
  double* T;
  double* V[2];
  double* P[2];
  double* d;
  double* e;
  double* tau[2];
  double* partial[2];
};

size_t eig_carve(int n, EigWork* w, void* base, size_t cap, bool* ok) {
  Carver c(base, cap);
  w->T = c.take<double>((size_t)n * n);
  for (int b = 0; b < 2; ++b) {
    w->V[b] = c.take<double>(n);
    w->P[b] = c.take<double>(n);
    w->tau[b] = c.take<double>(1);
    w->partial[b] = c.take<double>((n + NT / 64 - 1) / (NT / 64) + 1);
  }
  w->d = c.take<double>(n);
  w->e = c.take<double>(n);
  *ok = c.ok();
  return c.used;
}

}  // namespace
}  // namespace ipr

using namespace ipr;

extern "C" {

size_t ipr_eigvalsh_workspace(int n) {
  if (n < 1) return 0;
  EigWork w;
  bool ok;
  return eig_carve(n, &w, nullptr, (size_t)-1, &ok) + 256;
}

int ipr_eigvalsh(const double* dA, int n, double* dW, void* dWork, size_t work_bytes,
                 hipStream_t stream) {
  g_last_error.clear();
  if (!dA || !dW || !dWork || n < 1) return fail(IPR_EARG, "ipr_eigvalsh: bad argument");
  EigWork w;
  bool ok;
  eig_carve(n, &w, dWork, work_bytes, &ok);
  if (!ok)
    return fail(IPR_EARG, "ipr_eigvalsh: workspace too small (%zu bytes, need %zu)", work_bytes,
                ipr_eigvalsh_workspace(n));
  HIP_TRY(hipMemcpyAsync(w.T, dA, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice,
                         stream));
  if (n >= 2) {
    // column 0: its reflector and product; then, per column k, the update of
    // its block fused with the next column's reflector and product
    hipLaunchKernelGGL(reflector_kernel, dim3(1), dim3(NT), 0, stream, w.T, n, 0, w.V[0], w.d,
                       w.e, w.tau[0]);
    HIP_TRY(hipGetLastError());
    int nparts = (n - 1 + NT / 64 - 1) / (NT / 64);
    hipLaunchKernelGGL(trail_gemv_kernel, dim3(nparts), dim3(NT), 0, stream, w.T, n, 0, w.V[0],
                       w.tau[0], w.P[0], w.partial[0]);
    HIP_TRY(hipGetLastError());
    for (int k = 0; k + 3 <= n; ++k) {
      const int m = n - k - 1, a = k & 1, b = a ^ 1;
      hipLaunchKernelGGL(next_reflector_kernel, dim3(1), dim3(NT), 0, stream,
                         w.T, n, k, w.V[a], w.P[a], w.tau[a], w.partial[a], nparts, w.V[b], w.d,
                         w.e, w.tau[b]);
      HIP_TRY(hipGetLastError());
      const int nb = (m - 1 + NT / 64 - 1) / (NT / 64);
      hipLaunchKernelGGL(update_gemv_kernel, dim3(nb), dim3(NT), 0, stream, w.T, n, k, w.V[a],
                         w.P[a], w.tau[a], w.partial[a], nparts, w.V[b], w.tau[b], w.P[b],
                         w.partial[b]);
      HIP_TRY(hipGetLastError());
      nparts = nb;
    }
  }
  hipLaunchKernelGGL(last_diag_kernel, dim3(1), dim3(64), 0, stream, w.T, n, w.d);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(multisect_kernel, dim3((n + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, stream,
                     w.d, w.e, n, dW);
  HIP_TRY(hipGetLastError());
  return IPR_OK;
}

}  // extern "C"
