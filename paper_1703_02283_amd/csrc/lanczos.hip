// Vector kernels of the Lanczos estimate of lambda_min(A) used by the
// dynamically scaled iteration (ipr_solve with schedule.dynamic_scaling).
//
// The scaled iteration needs a rough lower end of the spectrum of C_0^p A.
// A few Lanczos steps on A give Ritz values inside [lambda_min, lambda_max];
// the smallest is an estimate of lambda_min from above, good enough to
// choose the scale factors (an overestimate only makes them less aggressive).
// All of it is matrix-vector work: one pass over A (8 n^2 bytes) per step.
#include "ipr_internal.h"

namespace ipr {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// y = A x, A n x n row-major: one wave per row, lanes stride the columns.
__global__ __launch_bounds__(NT) void gemv_kernel(const double* __restrict__ A, int n,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y) {
  const int row = (int)((blockIdx.x * (size_t)NT + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = A + (size_t)row * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * x[j];
  s = wave_sum(s);
  if (lane == 0) y[row] = s;
}

// h[i] = Q_i . w for the m vectors Q_i (contiguous, length n): block i.
__global__ __launch_bounds__(NT) void dots_kernel(const double* __restrict__ Q, int n,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ h) {
  __shared__ double red[NT / 64];
  const double* q = Q + (size_t)blockIdx.x * n;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) s += q[j] * w[j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += red[k];
    h[blockIdx.x] = t;
  }
}

// w -= sum_i h[i] Q_i (i < m)
__global__ __launch_bounds__(NT) void sub_kernel(const double* __restrict__ Q, int m, int n,
                                                 const double* __restrict__ h,
                                                 double* __restrict__ w) {
  const size_t j = blockIdx.x * (size_t)NT + threadIdx.x;
  if (j >= (size_t)n) return;
  double v = w[j];
  for (int i = 0; i < m; ++i) v -= h[i] * Q[(size_t)i * n + j];
  w[j] = v;
}

__global__ __launch_bounds__(NT) void scale_kernel(const double* __restrict__ w, int n, double a,
                                                   double* __restrict__ v) {
  const size_t j = blockIdx.x * (size_t)NT + threadIdx.x;
  if (j < (size_t)n) v[j] = a * w[j];
}

// A fixed start vector with entries in (-1, 1) (splitmix64 of the index).
__global__ __launch_bounds__(NT) void start_kernel(double* __restrict__ v, int n) {
  const size_t j = blockIdx.x * (size_t)NT + threadIdx.x;
  if (j >= (size_t)n) return;
  uint64_t z = (uint64_t)j + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  v[j] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

inline unsigned blocks_for(size_t count) { return (unsigned)((count + NT - 1) / NT); }

}  // namespace

hipError_t lz_gemv(const double* A, int n, const double* x, double* y, hipStream_t stream) {
  hipLaunchKernelGGL(gemv_kernel, dim3(blocks_for((size_t)n * 64)), dim3(NT), 0, stream, A, n, x,
                     y);
  return hipGetLastError();
}

hipError_t lz_dots(const double* Q, int m, int n, const double* w, double* h,
                   hipStream_t stream) {
  hipLaunchKernelGGL(dots_kernel, dim3(m), dim3(NT), 0, stream, Q, n, w, h);
  return hipGetLastError();
}

hipError_t lz_sub(const double* Q, int m, int n, const double* h, double* w, hipStream_t stream) {
  hipLaunchKernelGGL(sub_kernel, dim3(blocks_for(n)), dim3(NT), 0, stream, Q, m, n, h, w);
  return hipGetLastError();
}

hipError_t lz_scale(const double* w, int n, double a, double* v, hipStream_t stream) {
  hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n)), dim3(NT), 0, stream, w, n, a, v);
  return hipGetLastError();
}

hipError_t lz_start(double* v, int n, hipStream_t stream) {
  hipLaunchKernelGGL(start_kernel, dim3(blocks_for(n)), dim3(NT), 0, stream, v, n);
  return hipGetLastError();
}

}  // namespace ipr
