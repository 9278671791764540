// The all-arithmetic regime of the paper's experiments (Section IV: custom
// floating-point and fixed-point types "for all involved calculations";
// Section IV-C, Figs. 2a and 3a): every scalar operation of the coupled
// iteration is one float64 operation followed by round_store to the type.
// The matrix cores cannot serve it (their products and sums are fused and
// accumulate at a fixed width, so no intermediate result can be rounded):
// these are plain VALU kernels, and the dot products run over k in
// increasing order, one rounded multiply and one rounded add per term.
#include <algorithm>

#include "arith.h"

#pragma clang fp contract(off)

namespace ipr {
namespace {

constexpr int TB = 64;   // output tile edge
constexpr int KB = 16;   // k rows per LDS stage
constexpr int NT = 256;  // 16 x 16 threads, 4 x 4 outputs each

// D = L^T R for the upper tiles (tile row <= tile column; tiles[] lists
// them), every element with i <= j written to (i, j) and (j, i):
// acc <- rnd(acc + rnd(L[k][i] R[k][j])), k = 0 .. n-1, from acc = 0.
__global__ __launch_bounds__(NT) void gemm_arith_kernel(const double* __restrict__ L,
                                                        const double* __restrict__ R,
                                                        double* __restrict__ D, int n,
                                                        int fmt, int bits) {
  __shared__ double sl[KB][TB];
  __shared__ double sr[KB][TB];
  // blockIdx.x enumerates the upper tiles row by row
  const int nt = (n + TB - 1) / TB;
  int ti = 0, rem = blockIdx.x;
  while (rem >= nt - ti) {
    rem -= nt - ti;
    ++ti;
  }
  const int tj = ti + rem;
  const int i0 = ti * TB, j0 = tj * TB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k0 = 0; k0 < n; k0 += KB) {
    for (int idx = threadIdx.x; idx < KB * TB; idx += NT) {
      const int kk = idx / TB, c = idx - kk * TB, k = k0 + kk;
      sl[kk][c] = (k < n && i0 + c < n) ? L[(size_t)k * n + i0 + c] : 0.0;
      sr[kk][c] = (k < n && j0 + c < n) ? R[(size_t)k * n + j0 + c] : 0.0;
    }
    __syncthreads();
    const int kend = min(KB, n - k0);
    for (int kk = 0; kk < kend; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = sl[kk][ty + 16 * u];
        b[u] = sr[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double prod = round_store(a[u] * b[v], fmt, bits);
          acc[u][v] = round_store(acc[u][v] + prod, fmt, bits);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * v;
      if (i < n && j < n && i <= j) {
        D[(size_t)i * n + j] = acc[u][v];
        D[(size_t)j * n + i] = acc[u][v];
      }
    }
}

// C = c I, M = rnd(cp rnd(A)) entry by entry.
__global__ __launch_bounds__(NT) void arith_start_kernel(const double* __restrict__ A, int n,
                                                         double c, double cp, int fmt, int bits,
                                                         double* __restrict__ C,
                                                         double* __restrict__ M) {
  const size_t nn = (size_t)n * n;
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < nn; t += (size_t)gridDim.x * NT) {
    const size_t i = t / n, j = t - i * n;
    C[t] = i == j ? c : 0.0;
    M[t] = round_store(cp * round_store(A[t], fmt, bits), fmt, bits);
  }
}

// One workgroup per row i: N = rnd(I + rnd(rnd(I - M) / p)); partial[i] =
// sum_j (delta_ij - M_ij)^2 in float64 (the measured residual).
__global__ __launch_bounds__(NT) void arith_next_kernel(const double* __restrict__ M, int n, int p,
                                                        int fmt, int bits, double* __restrict__ N,
                                                        double* __restrict__ partial) {
  __shared__ double red[NT / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) {
    const size_t t = (size_t)i * n + j;
    const double d = i == j ? 1.0 : 0.0;
    const double q = d - M[t];
    const double r = round_store(q, fmt, bits);
    N[t] = round_store(d + round_store(r / p, fmt, bits), fmt, bits);
    s += q * q;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[i] = (red[0] + red[1]) + (red[2] + red[3]);
}

// partial[i] = sum_j (X_ij - Y_ij)^2, one workgroup per row.
__global__ __launch_bounds__(NT) void diff_rows_kernel(const double* __restrict__ X,
                                                       const double* __restrict__ Y, int n,
                                                       double* __restrict__ partial) {
  __shared__ double red[NT / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) {
    const double d = X[(size_t)i * n + j] - Y[(size_t)i * n + j];
    s += d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[i] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

hipError_t gemm_arith(const double* L, const double* R, double* D, int n, int fmt, int bits,
                      hipStream_t stream) {
  if (n < 1) return hipSuccess;
  const int nt = (n + TB - 1) / TB;
  const int tiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(gemm_arith_kernel, dim3(tiles), dim3(NT), 0, stream, L, R, D, n, fmt, bits);
  return hipGetLastError();
}

hipError_t arith_start(const double* A, int n, double c, double cp, int fmt, int bits, double* C,
                       double* M, hipStream_t stream) {
  const size_t nn = (size_t)n * n;
  const int grid = (int)std::min<size_t>((nn + NT - 1) / NT, 4096);
  hipLaunchKernelGGL(arith_start_kernel, dim3(grid), dim3(NT), 0, stream, A, n, c, cp, fmt, bits,
                     C, M);
  return hipGetLastError();
}

hipError_t arith_next(const double* M, int n, int p, int fmt, int bits, double* N,
                      double* partial, hipStream_t stream) {
  hipLaunchKernelGGL(arith_next_kernel, dim3(n), dim3(NT), 0, stream, M, n, p, fmt, bits, N,
                     partial);
  return hipGetLastError();
}

hipError_t diff_rows(const double* X, const double* Y, int n, double* partial,
                     hipStream_t stream) {
  hipLaunchKernelGGL(diff_rows_kernel, dim3(n), dim3(NT), 0, stream, X, Y, n, partial);
  return hipGetLastError();
}

}  // namespace ipr
