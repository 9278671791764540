// HBM-bound helpers of the iteration: the norms of eq. (3), the scaled
// identity start, the Frobenius-norm reduction and small elementwise maps.
// All reductions run in a fixed order, so their results are bitwise
// reproducible from run to run.
#include <algorithm>

#include "ipr_internal.h"

namespace ipr {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += red[w];
  }
  return s;  // valid in thread 0
}

// Row sums of |A|: one workgroup per row.
__global__ __launch_bounds__(NT) void row_abs_sum(const double* __restrict__ A, int n,
                                                   double* __restrict__ rows) {
  __shared__ double red[NT / 64];
  const int i = blockIdx.x;
  const double* a = A + (size_t)i * n;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) s += fabs(a[j]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) rows[i] = s;
}

// Column sums of |A| over a strip of 256 rows: partial[strip][j].
constexpr int STRIP = 256;
__global__ __launch_bounds__(NT) void col_abs_partial(const double* __restrict__ A, int n,
                                                       double* __restrict__ partial) {
  const int j = blockIdx.x * NT + threadIdx.x;
  const int r0 = blockIdx.y * STRIP;
  if (j >= n) return;
  const int r1 = min(n, r0 + STRIP);
  double s = 0.0;
  for (int i = r0; i < r1; ++i) s += fabs(A[(size_t)i * n + j]);
  partial[(size_t)blockIdx.y * n + j] = s;
}

__global__ __launch_bounds__(NT) void col_abs_finish(const double* __restrict__ partial,
                                                      int n, int strips,
                                                      double* __restrict__ cols) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int t = 0; t < strips; ++t) s += partial[(size_t)t * n + j];
  cols[j] = s;
}

// out[0] = max(cols), out[1] = max(rows)
__global__ __launch_bounds__(1024) void max2(const double* __restrict__ cols,
                                              const double* __restrict__ rows, int n,
                                              double* __restrict__ out) {
  __shared__ double mc[1024], mr[1024];
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < n; j += 1024) {
    a = fmax(a, cols[j]);
    b = fmax(b, rows[j]);
  }
  mc[threadIdx.x] = a;
  mr[threadIdx.x] = b;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      mc[threadIdx.x] = fmax(mc[threadIdx.x], mc[threadIdx.x + s]);
      mr[threadIdx.x] = fmax(mr[threadIdx.x], mr[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = mc[0];
    out[1] = mr[0];
  }
}

// C = c I, M = cp A, N = ((p+1) I - M) / p; partial[i] = sum_j (I - M)_ij^2.
__global__ __launch_bounds__(NT) void init_identity_kernel(const double* __restrict__ A, int n,
                                                            int p, double c, double cp,
                                                            double* __restrict__ C,
                                                            double* __restrict__ M,
                                                            double* __restrict__ N,
                                                            double* __restrict__ partial) {
  __shared__ double red[NT / 64];
  const int i = blockIdx.x;
  const size_t base = (size_t)i * n;
  const double inv_p = 1.0 / p;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) {
    const double d = (i == j) ? 1.0 : 0.0;
    const double m = cp * A[base + j];
    const double r = d - m;
    C[base + j] = c * d;
    M[base + j] = m;
    N[base + j] = d + r * inv_p;
    s += r * r;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[i] = s;
}

// out = sqrt(sum slots): each of 1024 threads sums a fixed strided subset,
// then a fixed-shape tree.
__global__ __launch_bounds__(1024) void reduce_fro_kernel(const double* __restrict__ slots,
                                                           int count, double* __restrict__ out) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int t = threadIdx.x; t < count; t += 1024) s += slots[t];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(sh[0]);
}

__global__ __launch_bounds__(NT) void affine_kernel(const double* __restrict__ X, int n, double a,
                                                     double b, double* __restrict__ Y) {
  const size_t total = (size_t)n * n;
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < total;
       t += (size_t)gridDim.x * NT) {
    const size_t i = t / n, j = t - i * n;
    Y[t] = a * X[t] + (i == j ? b : 0.0);
  }
}

__global__ __launch_bounds__(NT) void copy_kernel(const double* __restrict__ X, size_t count,
                                                   double* __restrict__ Y) {
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < count;
       t += (size_t)gridDim.x * NT)
    Y[t] = X[t];
}

// X <- (X + X^T) / 2 in place: thread t owns the pair (i, j), i < j.
// X <- (X + X^T) / 2 in place. Block (bx, by) with bx >= by owns the tile
// pair (by, bx) / (bx, by): both 32 x 32 tiles are read as row segments into
// LDS, averaged, and written back as row segments (the diagonal tile pairs
// with itself). Blocks with bx < by have nothing to do.
__global__ __launch_bounds__(256) void symmetrize_kernel(double* __restrict__ X, int n) {
  __shared__ double u[32][33], v[32][33];
  const int bx = blockIdx.x, by = blockIdx.y;
  if (bx < by) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int r0 = by * 32, c0 = bx * 32;  // tile U = X[r0.., c0..], tile V = X[c0.., r0..]
  for (int r = ty; r < 32; r += 8) {
    const int i = r0 + r, j = c0 + tx;
    if (i < n && j < n) u[r][tx] = X[(size_t)i * n + j];
    const int i2 = c0 + r, j2 = r0 + tx;
    if (i2 < n && j2 < n) v[r][tx] = X[(size_t)i2 * n + j2];
  }
  __syncthreads();
  // U[r][c] pairs with V[c][r]
  for (int r = ty; r < 32; r += 8) {
    const int i = r0 + r, j = c0 + tx;
    if (i < n && j < n) X[(size_t)i * n + j] = 0.5 * (u[r][tx] + v[tx][r]);
    const int i2 = c0 + r, j2 = r0 + tx;
    if (i2 < n && j2 < n) X[(size_t)i2 * n + j2] = 0.5 * (v[r][tx] + u[tx][r]);
  }
}

// Y = X^T (Y must not alias X), 32 x 32 tiles through LDS so that reads and
// writes are row segments: block (bx, by) reads rows 32 by.. of columns 32 bx..
// and writes them as rows 32 bx.. of columns 32 by...
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ X, int n,
                                                        double* __restrict__ Y) {
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int r = ty; r < 32; r += 8) {
    const int i = r0 + r, j = c0 + tx;
    if (i < n && j < n) t[r][tx] = X[(size_t)i * n + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = c0 + r, j = r0 + tx;  // Y[i][j] = X[j][i]
    if (i < n && j < n) Y[(size_t)i * n + j] = t[tx][r];
  }
}

// Y = a0 I + a1 A + a2 G.
__global__ __launch_bounds__(NT) void lincomb_kernel(const double* __restrict__ A,
                                                      const double* __restrict__ G, int n,
                                                      double a0, double a1, double a2,
                                                      double* __restrict__ Y) {
  const size_t total = (size_t)n * n;
  for (size_t t = (size_t)blockIdx.x * NT + threadIdx.x; t < total;
       t += (size_t)gridDim.x * NT) {
    const size_t i = t / n, j = t - i * n;
    Y[t] = (i == j ? a0 : 0.0) + a1 * A[t] + (G ? a2 * G[t] : 0.0);
  }
}

int grid_for(size_t count) {
  size_t g = (count + NT - 1) / NT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t norms_1_inf(const double* A, int n, double* scratch, double* out, hipStream_t stream) {
  // scratch layout: rows[n], cols[n], partial[strips * n]
  double* rows = scratch;
  double* cols = scratch + n;
  double* part = scratch + 2 * (size_t)n;
  const int strips = (n + STRIP - 1) / STRIP;
  hipLaunchKernelGGL(row_abs_sum, dim3(n), dim3(NT), 0, stream, A, n, rows);
  hipLaunchKernelGGL(col_abs_partial, dim3((n + NT - 1) / NT, strips), dim3(NT), 0, stream, A, n,
                     part);
  hipLaunchKernelGGL(col_abs_finish, dim3((n + NT - 1) / NT), dim3(NT), 0, stream, part, n, strips,
                     cols);
  hipLaunchKernelGGL(max2, dim3(1), dim3(1024), 0, stream, cols, rows, n, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(NT) void round_kernel(double* __restrict__ X, size_t count, int fmt,
                                                   int bits) {
  for (size_t i = blockIdx.x * (size_t)NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT)
    X[i] = round_store(X[i], fmt, bits);
}

hipError_t round_matrix(double* X, size_t count, int fmt, int bits, hipStream_t stream) {
  const size_t blocks = std::min<size_t>((count + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(round_kernel, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(NT), 0, stream,
                     X, count, fmt, bits);
  return hipGetLastError();
}

hipError_t init_identity(const double* A, int n, int p, double c, double cp, double* C,
                         double* M, double* N, double* partial, hipStream_t stream) {
  hipLaunchKernelGGL(init_identity_kernel, dim3(n), dim3(NT), 0, stream, A, n, p, c, cp, C, M, N,
                     partial);
  return hipGetLastError();
}

hipError_t reduce_fro(const double* slots, int count, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_fro_kernel, dim3(1), dim3(1024), 0, stream, slots, count, out);
  return hipGetLastError();
}

hipError_t affine(const double* X, int n, double a, double b, double* Y, hipStream_t stream) {
  hipLaunchKernelGGL(affine_kernel, dim3(grid_for((size_t)n * n)), dim3(NT), 0, stream, X, n, a, b,
                     Y);
  return hipGetLastError();
}

hipError_t lincomb(const double* A, const double* G, int n, double a0, double a1, double a2,
                   double* Y, hipStream_t stream) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for((size_t)n * n)), dim3(NT), 0, stream, A, G, n,
                     a0, a1, a2, Y);
  return hipGetLastError();
}

hipError_t symmetrize(double* X, int n, hipStream_t stream) {
  const unsigned nb = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nb, nb), dim3(256), 0, stream, X, n);
  return hipGetLastError();
}

hipError_t transpose(const double* X, int n, double* Y, hipStream_t stream) {
  if (X == Y) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, dim3(nb, nb), dim3(256), 0, stream, X, n, Y);
  return hipGetLastError();
}

hipError_t copy(const double* X, size_t count, double* Y, hipStream_t stream) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(count)), dim3(NT), 0, stream, X, count, Y);
  return hipGetLastError();
}

}  // namespace ipr
