// Eigenvalues of a dense symmetric matrix: the step after the Loewdin
// transform (Section IV-A: S^{-1/2} brings H c = e S c to the standard
// problem (S^{-1/2} H S^{-1/2}) c' = e c', whose eigenvalues are the e).
//
//  1. Householder tridiagonalisation, one reflector per column: with x the
//     part of column k below the diagonal, H = I - tau v v^T maps x to
//     beta e_1; the trailing matrix B becomes H B H = B - v w^T - w v^T with
//     p = tau B v and w = p - (tau / 2)(p . v) v. The trailing matrix is kept
//     whole (both triangles), so every access is a row access. One launch per
//     column, the update of one column fused with the reflector and product
//     of the next (look-ahead): one wave per row streams the row once,
//     updating it and at once multiplying it by the next reflector, which
//     every wave forms for itself from the block's first row. HBM-bound:
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

// Threads of the column step below, and the entries of each row a lane loads
// before it computes on them (so that as many loads are in flight: a row
// streams from memory at the rate its loads in flight allow).
constexpr int NTC = 512;
constexpr int UC = 8;
// Blocks of a larger order take two (four) rows per wave: the loads of row 0,
// V and P then serve several rows, and there are still enough waves to keep
// every CU streaming (measured at n = 8192: 872 ms with one row per wave,
// 772 ms with two above 2048, 713 ms with four above 4096; two rows from
// 1024 on made n = 2048 slower, 28.2 against 25.0 ms).
constexpr int kRows2 = 2048;
constexpr int kRows4 = 4096;

// w_j = P_j - c V_j, and entry (i, j) of the trailing block after the rank-2
// update, B_ij - (V_i w_j + w_i V_j). Every use goes through these two, with
// the fused multiply-adds written out, so that each workgroup forms the same
// bits for the same entry.
__device__ __forceinline__ double w_of(double pj, double vj, double c) {
  return __builtin_fma(-c, vj, pj);
}
__device__ __forceinline__ double rank2(double b, double vi, double wi, double vj, double wj) {
  return b - __builtin_fma(vi, wj, wi * vj);
}

// Column k's step (trailing block B of order m = n - k - 1 >= 2, reflector V,
// tau, P = tau B V with per-workgroup partials of P . V), with the next
// column's reflector and product folded in (look-ahead). With W = P - c V,
// c = (tau / 2) P . V, the update is B_ij -= V_i W_j + W_i V_j; the next
// reflector comes from x = row 0 of the updated block beyond its first entry
// (alpha = x_1, beta = -sign(alpha) |x|, V2 = (x - beta e_1) / (alpha - beta)).
// RW rows i = 1 .. m-1 per wave (rows w and w + 8 of the workgroup's 8 RW),
// each streamed once:
//  * it updates B_ij (column 0 is not read again) and, from row 0 (which no
//    wave writes: no later step reads row k + 1 of T), forms the updated x_j
//    on the fly, accumulating |x|^2 beyond x_1 and sum_{j >= 2} B_ij x_j;
//  * so every wave knows beta and the scale 1 / (alpha - beta) at the end of
//    its row, identically (same code, same order), and
//    P2[i - 1] = tau2 sum_j B_ij V2[j - 1] = tau2 (B_i1 + sum_{j >= 2} B_ij x_j / (alpha - beta));
//  * it stores V2[i - 1]; the wave of row 1 stores tau2, d[k + 1], e[k + 1].
// partial2[b] = sum over workgroup b's rows of P2 V2. One launch per column,
// and no wave waits for another beyond the sum of the partials.
template <int RW>
__global__ __launch_bounds__(NTC) void column_step_kernel(
    double* __restrict__ T, int n, int k, const double* __restrict__ V,
    const double* __restrict__ P, const double* __restrict__ tau,
    const double* __restrict__ partial, int nparts, double* __restrict__ V2,
    double* __restrict__ d, double* __restrict__ e, double* __restrict__ tau2,
    double* __restrict__ P2, double* __restrict__ partial2) {
  constexpr int NW = NTC / 64;
  __shared__ double red[NW];
  const int m = n - k - 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // workgroup sum in a fixed order, returned to every thread
  auto wg_sum = [&](double v) {
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += red[w];
    __syncthreads();  // (red is reused)
    return t;
  };
  double s = 0.0;
  for (int b = tid; b < nparts; b += NTC) s += partial[b];
  const double c = 0.5 * *tau * wg_sum(s);
  const double v0 = V[0], w0 = w_of(P[0], V[0], c);
  const double* row0 = T + (size_t)(k + 1) * n + k + 1;
  const int ibase = 1 + blockIdx.x * NW * RW + wave;
  double pv = 0.0;
  if (ibase < m) {
    int ii[RW];
    bool ok[RW];
    double vi[RW], wi[RW], acc[RW], b1[RW];
    double* row[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      ii[r] = ibase + r * NW;
      ok[r] = ii[r] < m;
      const int ic = ok[r] ? ii[r] : ibase;  // (a row past the block is not touched)
      vi[r] = V[ic];
      wi[r] = w_of(P[ic], vi[r], c);
      row[r] = T + (size_t)(k + 1 + ic) * n + k + 1;
      acc[r] = 0.0;
      b1[r] = 0.0;
    }
    double q = 0.0, x1 = 0.0;
    for (int j0 = 1 + lane; j0 < m; j0 += 64 * UC) {
      // all loads of UC entries first, so that they are in flight together
      double rr[RW][UC], r0[UC], vv[UC], pp[UC];
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int j = j0 + 64 * u;
        const bool in = j < m;
#pragma unroll
        for (int r = 0; r < RW; ++r) rr[r][u] = in && ok[r] ? row[r][j] : 0.0;
        r0[u] = in ? row0[j] : 0.0;
        vv[u] = in ? V[j] : 0.0;
        pp[u] = in ? P[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UC; ++u) {
        const int j = j0 + 64 * u;
        if (j < m) {
          const double wj = w_of(pp[u], vv[u], c);
          const double x = rank2(r0[u], v0, w0, vv[u], wj);
          if (j == 1) x1 = x; else q += x * x;
#pragma unroll
          for (int r = 0; r < RW; ++r) {
            if (ok[r]) {
              const double t = rank2(rr[r][u], vi[r], wi[r], vv[u], wj);
              row[r][j] = t;
              if (j == 1) b1[r] = t; else acc[r] += t * x;
            }
          }
        }
      }
    }
    // (b1 and x1 are nonzero in lane 0 only: their wave sums are exact copies)
    q = wave_sum(q);
    const double alpha = wave_sum(x1);
    double beta = alpha, t2 = 0.0, cf = 0.0;  // q == 0: already reduced, H = I
    if (q != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + q), alpha);
      t2 = (beta - alpha) / beta;
      cf = 1.0 / (alpha - beta);
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const double a = wave_sum(acc[r]);
      const double bb = wave_sum(b1[r]);
      if (ok[r]) {
        const int i = ii[r];
        const double p2 = t2 * __builtin_fma(a, cf, bb);
        const double v2i = i == 1 ? 1.0 : rank2(row0[i], v0, w0, vi[r], wi[r]) * cf;
        if (lane == 0) {
          P2[i - 1] = p2;
          V2[i - 1] = v2i;
          if (i == 1) {
            d[k + 1] = rank2(row0[0], v0, w0, v0, w0);
            e[k + 1] = beta;
            *tau2 = t2;
          }
          pv += p2 * v2i;
        }
      }
    }
  }
  const double ps = wg_sum(pv);
  if (tid == 0) partial2[blockIdx.x] = ps;
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
    // column 0: its reflector and product; then, per column k, one launch:
    // the update of its block fused with the next column's reflector and
    // product
    hipLaunchKernelGGL(reflector_kernel, dim3(1), dim3(NT), 0, stream, w.T, n, 0, w.V[0], w.d,
                       w.e, w.tau[0]);
    HIP_TRY(hipGetLastError());
    int nparts = (n - 1 + NT / 64 - 1) / (NT / 64);
    hipLaunchKernelGGL(trail_gemv_kernel, dim3(nparts), dim3(NT), 0, stream, w.T, n, 0, w.V[0],
                       w.tau[0], w.P[0], w.partial[0]);
    HIP_TRY(hipGetLastError());
    for (int k = 0; k + 3 <= n; ++k) {
      const int m = n - k - 1, a = k & 1, b = a ^ 1;
      // several rows per wave share the loads of row 0, V and P once the
      // block is large enough to keep every CU busy with fewer waves
      const int rw = m > kRows4 ? 4 : m > kRows2 ? 2 : 1;
      const int nb = (m - 1 + NTC / 64 * rw - 1) / (NTC / 64 * rw);
      if (rw == 4)
        hipLaunchKernelGGL(column_step_kernel<4>, dim3(nb), dim3(NTC), 0, stream, w.T, n, k,
                           w.V[a], w.P[a], w.tau[a], w.partial[a], nparts, w.V[b], w.d, w.e,
                           w.tau[b], w.P[b], w.partial[b]);
      else if (rw == 2)
        hipLaunchKernelGGL(column_step_kernel<2>, dim3(nb), dim3(NTC), 0, stream, w.T, n, k,
                           w.V[a], w.P[a], w.tau[a], w.partial[a], nparts, w.V[b], w.d, w.e,
                           w.tau[b], w.P[b], w.partial[b]);
      else
        hipLaunchKernelGGL(column_step_kernel<1>, dim3(nb), dim3(NTC), 0, stream, w.T, n, k,
                           w.V[a], w.P[a], w.tau[a], w.partial[a], nparts, w.V[b], w.d, w.e,
                           w.tau[b], w.P[b], w.partial[b]);
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
