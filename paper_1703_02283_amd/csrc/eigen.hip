// Eigenvalues of a dense symmetric matrix: the step after the Loewdin
// transform (Section IV-A: S^{-1/2} brings H c = e S c to the standard
// problem (S^{-1/2} H S^{-1/2}) c' = e c', whose eigenvalues are the e).
//
//  1. Householder tridiagonalisation, one reflector per column: with x the
//     part of column k below the diagonal, H = I - tau v v^T maps x to
//     beta e_1; the trailing matrix B becomes H B H = B - v w^T - w v^T with
//     p = tau B v and w = p - (tau / 2)(p . v) v. Three launches per column:
//     the reflector (one workgroup), p = tau B v with the partial sums of
//     p . v (one wave per row), and the rank-2 update (tiles). The trailing
//     matrix is kept whole (both triangles), so every read is a row read.
//     HBM-bound: about 3 (n - k)^2 doubles per column, 8 n^3 bytes in all.
//  2. Bisection on the Sturm count of the tridiagonal matrix (d, e), one
//     thread per eigenvalue index, from the Gershgorin interval down to the
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

// B -= V W^T + W V^T with W = P - (tau / 2)(P . V) V; 64 x 64 tiles of B,
// each workgroup sums the gemv's partials itself (fixed order).
__global__ __launch_bounds__(NT) void trail_syr2_kernel(double* __restrict__ T, int n, int k,
                                                        const double* __restrict__ V,
                                                        const double* __restrict__ P,
                                                        const double* __restrict__ tau,
                                                        const double* __restrict__ partial,
                                                        int nparts) {
  __shared__ double red[NT / 64];
  __shared__ double cs;
  __shared__ double vi[64], wi[64], vj[64], wj[64];
  const int m = n - k - 1;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) s += partial[b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) cs = 0.5 * *tau * ((red[0] + red[1]) + (red[2] + red[3]));
  __syncthreads();
  const double c = cs;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  if (threadIdx.x < 64) {
    const int i = i0 + threadIdx.x;
    vi[threadIdx.x] = i < m ? V[i] : 0.0;
    wi[threadIdx.x] = i < m ? P[i] - c * V[i] : 0.0;
  } else if (threadIdx.x < 128) {
    const int j = j0 + threadIdx.x - 64;
    vj[threadIdx.x - 64] = j < m ? V[j] : 0.0;
    wj[threadIdx.x - 64] = j < m ? P[j] - c * V[j] : 0.0;
  }
  __syncthreads();
  const int tj = threadIdx.x & 63;
  const int j = j0 + tj;
  if (j >= m) return;
  for (int r = threadIdx.x >> 6; r < 64; r += NT / 64) {
    const int i = i0 + r;
    if (i >= m) break;
    double* t = T + (size_t)(k + 1 + i) * n + k + 1 + j;
    *t -= vi[r] * wj[tj] + wi[r] * vj[tj];
  }
}

// d[n-1] = T[n-1][n-1] (the last diagonal entry, untouched by reflectors).
__global__ void last_diag_kernel(const double* __restrict__ T, int n, double* __restrict__ d) {
  if (threadIdx.x == 0) d[n - 1] = T[(size_t)(n - 1) * n + n - 1];
}

// Eigenvalue `idx` (ascending) of the symmetric tridiagonal matrix with
// diagonal d[0..n) and off-diagonal e[0..n-1), by bisection on the number
// of eigenvalues below x (Sturm count of the LDL^T pivots).
__global__ __launch_bounds__(NT) void bisect_kernel(const double* __restrict__ d,
                                                    const double* __restrict__ e, int n,
                                                    double* __restrict__ W) {
  const int idx = blockIdx.x * NT + threadIdx.x;
  if (idx >= n) return;
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
  for (int it = 0; it < 200; ++it) {
    const double x = 0.5 * (lo + hi);
    if (!(x > lo && x < hi)) break;  // no double strictly between: converged
    int below = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    below += q < 0.0;
    for (int i = 1; i < n; ++i) {
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      below += q < 0.0;
    }
    if (below > idx)
      hi = x;
    else
      lo = x;
  }
  W[idx] = 0.5 * (lo + hi);
}

struct EigWork {
  double* T;
  double* V;
  double* P;
  double* d;
  double* e;
  double* tau;
  double* partial;
};

size_t eig_carve(int n, EigWork* w, void* base, size_t cap, bool* ok) {
  Carver c(base, cap);
  w->T = c.take<double>((size_t)n * n);
  w->V = c.take<double>(n);
  w->P = c.take<double>(n);
  w->d = c.take<double>(n);
  w->e = c.take<double>(n);
  w->tau = c.take<double>(1);
  w->partial = c.take<double>((n + NT / 64 - 1) / (NT / 64) + 1);
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
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - k - 1;
    hipLaunchKernelGGL(reflector_kernel, dim3(1), dim3(NT), 0, stream, w.T, n, k, w.V, w.d, w.e,
                       w.tau);
    HIP_TRY(hipGetLastError());
    const int gb = (m + NT / 64 - 1) / (NT / 64);
    hipLaunchKernelGGL(trail_gemv_kernel, dim3(gb), dim3(NT), 0, stream, w.T, n, k, w.V, w.tau,
                       w.P, w.partial);
    HIP_TRY(hipGetLastError());
    const int tt = (m + 63) / 64;
    hipLaunchKernelGGL(trail_syr2_kernel, dim3(tt, tt), dim3(NT), 0, stream, w.T, n, k, w.V,
                       w.P, w.tau, w.partial, gb);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(last_diag_kernel, dim3(1), dim3(64), 0, stream, w.T, n, w.d);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(bisect_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, stream, w.d, w.e, n,
                     dW);
  HIP_TRY(hipGetLastError());
  return IPR_OK;
}

}  // extern "C"
