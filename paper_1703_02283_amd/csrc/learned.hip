// Learned start of the iteration: cheap matrix features, the 16-64-64-3 GELU
// network that maps them to a polynomial start C_0 = s^{-1/p} q(A/s), its
// training kernels, and the per-eigenvalue iteration counts that label the
// training data.
//
// The start must satisfy eq. (2) of Section II; the host checks the predicted
// polynomial in closed form and falls back to the scaled identity otherwise.
#include <cstdint>

#include "learned.h"

namespace ipr {
namespace {

constexpr int NT = 256;
constexpr int NI = 16, NH = 64, NO = 3;
constexpr int kFeatRowsMin = 256;  // from this order on the single-matrix features use many workgroups
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH,
              NPARAM = OFF_B3 + NO;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// Reduces one value per wave (lane 0 holds it) across the 4 waves of the block
// in a fixed order; op 0 sum, 1 max, 2 min. Result in every thread.
__device__ double block_red(double v, int op, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < NT / 64; ++w)
    r = op == 0 ? r + sh[w] : (op == 1 ? fmax(r, sh[w]) : fmin(r, sh[w]));
  __syncthreads();
  return r;
}

// Row statistics of a matrix (sums, then maxima and minima) from which the
// features follow: sum d, sum d^2, sum |d|, sum o, sum r, sum of squares, max
// off-diagonal |A_ij|, min d, max d, min (d_i - o_i) (unscaled A).
struct RowStats {
  double sd, sd2, sabsd, so, sr, sq, offmax, dmin, dmax, gmin;
};
constexpr int kRowStats = 10;

__device__ void write_features(float* f, int n, int pm, double n1, double ninf,
                               const RowStats& r) {
  const double s = sqrt(n1 * ninf);
  const double t1 = r.sd / s / n, t2 = r.sq / (s * s) / n;
  const double mean_d = r.sd / n;
  const double var_d = fmax(r.sd2 / n - mean_d * mean_d, 0.0);
  // the order enters clipped to the training sizes 64..1024: beyond them the
  // network would extrapolate, and the iteration count depends on the
  // spectrum, not on n
  f[0] = (float)(fmin(fmax(log2((double)n), 6.0), 10.0) / 10.0);
  f[1] = (float)(pm / 4.0);
  f[2] = (float)t1;
  f[3] = (float)t2;
  f[4] = (float)log10(t1);
  f[5] = (float)log10(t2);
  f[6] = (float)(t1 * t1 / t2);
  f[7] = (float)(r.dmin / s);
  f[8] = (float)(r.dmax / s);
  f[9] = (float)log10(fmax(r.dmin / s, 1e-30));
  f[10] = (float)(r.gmin / s);
  f[11] = (float)(r.sr / s / n);
  f[12] = (float)(r.so / r.sabsd);
  f[13] = (float)(n > 1 ? r.offmax / s : 0.0);
  f[14] = (float)(sqrt(var_d) / mean_d);
  f[15] = (float)log10(s);
}

// One workgroup per matrix. With s = sqrt(||A||_1 ||A||_inf), B = A / s,
// d = diag B, r_i = sum_j |B_ij|, o_i = r_i - |d_i|, t1 = trace(B)/n,
// t2 = ||B||_F^2 / n, the 16 features are
//  0 clamp(log2 n, 6, 10)/10   1 p/4   2 t1   3 t2   4 log10 t1   5 log10 t2   6 t1^2/t2
//  7 min d   8 max d   9 log10 max(min d, 1e-30)   10 min (d_i - o_i)
//  11 mean r   12 sum o / sum |d|   13 max_{i != j} |B_ij|   14 std(d)/mean(d)
//  15 log10 s.
__global__ __launch_bounds__(NT) void features_kernel(const double* __restrict__ Apack,
                                                       const int64_t* __restrict__ off,
                                                       const int* __restrict__ ns,
                                                       const int* __restrict__ ps, int n_one,
                                                       int p_one, float* __restrict__ feat) {
  __shared__ double sh[NT / 64];
  const int m = blockIdx.x;
  const int n = ns ? ns[m] : n_one;           // one matrix: n, p passed by value
  const int pm = ps ? ps[m] : p_one;
  const double* A = Apack + (off ? off[m] : 0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ||A||_1: column sums
  double cmax = 0.0;
  for (int j = tid; j < n; j += NT) {
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += fabs(A[(size_t)i * n + j]);
    cmax = fmax(cmax, cs);
  }
  const double n1 = block_red(wmax(cmax), 1, sh);
  // one wave per row: row sums, diagonal, squares, off-diagonal max
  double rmax = 0.0, sd = 0.0, sd2 = 0.0, sabsd = 0.0, so = 0.0, sr = 0.0, sq = 0.0,
         offmax = 0.0, dmin = 1e308, dmax = -1e308, gmin = 1e308;
  for (int i = wave; i < n; i += NT / 64) {
    double rs = 0.0, q2 = 0.0, om = 0.0;
    for (int j = lane; j < n; j += 64) {
      const double v = A[(size_t)i * n + j];
      rs += fabs(v);
      q2 += v * v;
      if (j != i) om = fmax(om, fabs(v));
    }
    rs = wsum(rs);
    q2 = wsum(q2);
    om = wmax(om);
    const double d = A[(size_t)i * n + i];
    const double o = rs - fabs(d);
    rmax = fmax(rmax, rs);
    sd += d;
    sd2 += d * d;
    sabsd += fabs(d);
    so += o;
    sr += rs;
    sq += q2;
    offmax = fmax(offmax, om);
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
    gmin = fmin(gmin, d - o);
  }
  const double ninf = block_red(rmax, 1, sh);
  RowStats r;
  r.sd = block_red(sd, 0, sh);
  r.sd2 = block_red(sd2, 0, sh);
  r.sabsd = block_red(sabsd, 0, sh);
  r.so = block_red(so, 0, sh);
  r.sr = block_red(sr, 0, sh);
  r.sq = block_red(sq, 0, sh);
  r.offmax = block_red(offmax, 1, sh);
  r.dmin = block_red(dmin, 2, sh);
  r.dmax = block_red(dmax, 1, sh);
  r.gmin = block_red(gmin, 2, sh);
  if (tid == 0) write_features(feat + (size_t)m * NI, n, pm, n1, ninf, r);
}

// One large matrix: block b takes rows 16 b .. 16 b + 15 (one wave per row,
// four rows per wave) and writes its RowStats (kRowStats doubles) to part.
__global__ __launch_bounds__(NT) void features_rows_kernel(const double* __restrict__ A, int n,
                                                           double* __restrict__ part) {
  __shared__ double sh[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double sd = 0.0, sd2 = 0.0, sabsd = 0.0, so = 0.0, sr = 0.0, sq = 0.0, offmax = 0.0,
         dmin = 1e308, dmax = -1e308, gmin = 1e308;
  for (int k = 0; k < 4; ++k) {
    const int i = blockIdx.x * 16 + 4 * k + wave;
    if (i >= n) break;
    double rs = 0.0, q2 = 0.0, om = 0.0;
    for (int j = lane; j < n; j += 64) {
      const double v = A[(size_t)i * n + j];
      rs += fabs(v);
      q2 += v * v;
      if (j != i) om = fmax(om, fabs(v));
    }
    rs = wsum(rs);
    q2 = wsum(q2);
    om = wmax(om);
    const double d = A[(size_t)i * n + i];
    const double o = rs - fabs(d);
    sd += d;
    sd2 += d * d;
    sabsd += fabs(d);
    so += o;
    sr += rs;
    sq += q2;
    offmax = fmax(offmax, om);
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
    gmin = fmin(gmin, d - o);
  }
  const double v[kRowStats] = {block_red(sd, 0, sh),     block_red(sd2, 0, sh),
                               block_red(sabsd, 0, sh),  block_red(so, 0, sh),
                               block_red(sr, 0, sh),     block_red(sq, 0, sh),
                               block_red(offmax, 1, sh), block_red(dmin, 2, sh),
                               block_red(dmax, 1, sh),   block_red(gmin, 2, sh)};
  if (tid == 0)
    for (int k = 0; k < kRowStats; ++k) part[(size_t)blockIdx.x * kRowStats + k] = v[k];
}

// Combines the nb blocks' RowStats (in a fixed order) with ||A||_1 and
// ||A||_inf (device, norms[0..1]) into the 16 features.
__global__ __launch_bounds__(NT) void features_finish_kernel(const double* __restrict__ part,
                                                             int nb, int n, int pm,
                                                             const double* __restrict__ norms,
                                                             float* __restrict__ feat) {
  __shared__ double sh[NT / 64];
  const int tid = threadIdx.x;
  double acc[kRowStats];
  for (int k = 0; k < kRowStats; ++k) acc[k] = k == 7 || k == 9 ? 1e308 : (k == 8 ? -1e308 : 0.0);
  for (int b = tid; b < nb; b += NT) {
    const double* q = part + (size_t)b * kRowStats;
    for (int k = 0; k < 6; ++k) acc[k] += q[k];
    acc[6] = fmax(acc[6], q[6]);
    acc[7] = fmin(acc[7], q[7]);
    acc[8] = fmax(acc[8], q[8]);
    acc[9] = fmin(acc[9], q[9]);
  }
  for (int k = 0; k < kRowStats; ++k) {
    const int op = k < 6 ? 0 : (k == 7 || k == 9 ? 2 : 1);
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double u = __shfl_xor(v, off, 64);
      v = op == 0 ? v + u : (op == 1 ? fmax(v, u) : fmin(v, u));
    }
    acc[k] = block_red(v, op, sh);
  }
  if (tid == 0) {
    RowStats r;
    r.sd = acc[0];
    r.sd2 = acc[1];
    r.sabsd = acc[2];
    r.so = acc[3];
    r.sr = acc[4];
    r.sq = acc[5];
    r.offmax = acc[6];
    r.dmin = acc[7];
    r.dmax = acc[8];
    r.gmin = acc[9];
    write_features(feat, n, pm, norms[0], norms[1], r);
  }
}

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Forward pass, one thread per sample; parameters staged in LDS. When Z1/Z2
// are given the pre-activations are kept for the backward pass.
__global__ __launch_bounds__(NT) void mlp_forward_kernel(const float* __restrict__ params,
                                                          const float* __restrict__ X, int batch,
                                                          float* __restrict__ Y,
                                                          float* __restrict__ Z1,
                                                          float* __restrict__ Z2) {
  __shared__ float w[NPARAM];
  for (int t = threadIdx.x; t < NPARAM; t += NT) w[t] = params[t];
  __syncthreads();
  const int b = blockIdx.x * NT + threadIdx.x;
  if (b >= batch) return;
  float x[NI], h1[NH], h2[NH];
#pragma unroll
  for (int i = 0; i < NI; ++i) x[i] = X[(size_t)b * NI + i];
  for (int o = 0; o < NH; ++o) {
    float z = w[OFF_B1 + o];
#pragma unroll
    for (int i = 0; i < NI; ++i) z += w[OFF_W1 + o * NI + i] * x[i];
    if (Z1) Z1[(size_t)b * NH + o] = z;
    h1[o] = gelu(z);
  }
  for (int o = 0; o < NH; ++o) {
    float z = w[OFF_B2 + o];
    for (int i = 0; i < NH; ++i) z += w[OFF_W2 + o * NH + i] * h1[i];
    if (Z2) Z2[(size_t)b * NH + o] = z;
    h2[o] = gelu(z);
  }
  for (int o = 0; o < NO; ++o) {
    float z = w[OFF_B3 + o];
    for (int i = 0; i < NH; ++i) z += w[OFF_W3 + o * NH + i] * h2[i];
    Y[(size_t)b * NO + o] = z;
  }
}

// Per-sample backward of the mean squared error: dZ1, dZ2 (pre-activation
// gradients), dY, and H1 = gelu(Z1), H2 = gelu(Z2) for the weight gradients;
// loss terms per sample.
__global__ __launch_bounds__(NT) void mlp_backward_sample_kernel(
    const float* __restrict__ params, const float* __restrict__ Y, const float* __restrict__ T,
    const float* __restrict__ Z1, const float* __restrict__ Z2, int batch,
    float* __restrict__ dY, float* __restrict__ dZ1, float* __restrict__ dZ2,
    float* __restrict__ H1, float* __restrict__ H2, float* __restrict__ lossv) {
  __shared__ float w[NPARAM];
  for (int t = threadIdx.x; t < NPARAM; t += NT) w[t] = params[t];
  __syncthreads();
  const int b = blockIdx.x * NT + threadIdx.x;
  if (b >= batch) return;
  const float scale = 2.0f / ((float)batch * NO);
  float dy[NO], l = 0.f;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const float r = Y[(size_t)b * NO + o] - T[(size_t)b * NO + o];
    dy[o] = scale * r;
    l += r * r;
    dY[(size_t)b * NO + o] = dy[o];
  }
  lossv[b] = l;
  float g2[NH];
  for (int i = 0; i < NH; ++i) {
    const float z = Z2[(size_t)b * NH + i];
    H2[(size_t)b * NH + i] = gelu(z);
    float g = 0.f;
#pragma unroll
    for (int o = 0; o < NO; ++o) g += dy[o] * w[OFF_W3 + o * NH + i];
    g2[i] = g * gelu_grad(z);
    dZ2[(size_t)b * NH + i] = g2[i];
  }
  for (int i = 0; i < NH; ++i) {
    const float z = Z1[(size_t)b * NH + i];
    H1[(size_t)b * NH + i] = gelu(z);
    float g = 0.f;
    for (int o = 0; o < NH; ++o) g += g2[o] * w[OFF_W2 + o * NH + i];
    dZ1[(size_t)b * NH + i] = g * gelu_grad(z);
  }
}

// Weight and bias gradients: one thread per parameter, summing over the
// batch in order (deterministic).
__global__ __launch_bounds__(NT) void mlp_grad_reduce_kernel(
    const float* __restrict__ X, const float* __restrict__ H1, const float* __restrict__ H2,
    const float* __restrict__ dY, const float* __restrict__ dZ1, const float* __restrict__ dZ2,
    int batch, float* __restrict__ grad) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= NPARAM) return;
  const float* g;  // upstream gradient column
  const float* a;  // input activation column (nullptr: bias)
  int gs, as, gi, ai = 0;
  if (t < OFF_B1) {
    gi = (t - OFF_W1) / NI; ai = (t - OFF_W1) % NI; g = dZ1; gs = NH; a = X; as = NI;
  } else if (t < OFF_W2) {
    gi = t - OFF_B1; g = dZ1; gs = NH; a = nullptr; as = 0;
  } else if (t < OFF_B2) {
    gi = (t - OFF_W2) / NH; ai = (t - OFF_W2) % NH; g = dZ2; gs = NH; a = H1; as = NH;
  } else if (t < OFF_W3) {
    gi = t - OFF_B2; g = dZ2; gs = NH; a = nullptr; as = 0;
  } else if (t < OFF_B3) {
    gi = (t - OFF_W3) / NH; ai = (t - OFF_W3) % NH; g = dY; gs = NO; a = H2; as = NH;
  } else {
    gi = t - OFF_B3; g = dY; gs = NO; a = nullptr; as = 0;
  }
  double s = 0.0;
  for (int b = 0; b < batch; ++b) {
    const double gv = g[(size_t)b * gs + gi];
    s += a ? gv * a[(size_t)b * as + ai] : gv;
  }
  grad[t] = (float)s;
}

__global__ __launch_bounds__(NT) void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int count, float lr, float bc1, float bc2) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= count) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mt = b1 * m[t] + (1.f - b1) * g[t];
  const float vt = b2 * v[t] + (1.f - b2) * g[t] * g[t];
  m[t] = mt;
  v[t] = vt;
  w[t] -= lr * (mt / bc1) / (sqrtf(vt / bc2) + eps);
}

// Mean of the per-sample squared errors (sum over the 3 outputs), fixed order.
__global__ __launch_bounds__(1024) void loss_kernel(const float* __restrict__ lossv, int batch,
                                                     float* __restrict__ out) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int b = threadIdx.x; b < batch; b += 1024) s += lossv[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(sh[0] / ((double)batch * NO));
}

// Iteration counts of eq. (1) per eigenvalue: for matrix m with eigenvalues
// lam[off[m] .. off[m] + n[m]), root p[m], scale s[m] and candidate start c
// (q(x) = b0 + b1 x + b2 x^2, C_0 = s^{-1/p} q(A/s)), iterate
// c_x <- c_x (p + 1 - c_x^p x) / p on the scaled values and count updates
// until sqrt(sum (1 - c_x^p x)^2) < tol. One workgroup per (matrix, candidate).
__global__ __launch_bounds__(NT) void spectral_counts_kernel(
    const double* __restrict__ lam, const int64_t* __restrict__ off, const int* __restrict__ ns,
    const int* __restrict__ ps, const double* __restrict__ scale, const double* __restrict__ cand,
    int ncand, double tol, int max_iter, int* __restrict__ counts) {
  __shared__ double sh[NT / 64];
  const int m = blockIdx.y, ci = blockIdx.x;
  const int n = ns[m], p = ps[m];
  const double s = scale[m];
  // ncand == 0: one candidate per matrix (cand[3 m ..]), else a shared list
  const double* cc = ncand ? cand + 3 * ci : cand + 3 * m;
  const double b0 = cc[0], b1 = cc[1], b2 = cc[2];
  // each thread keeps up to 8 eigenvalues (n <= 2048)
  double x[8], y[8];  // x = lambda / s, y = q(x)^p x = current eigenvalue of M
  int cnt = 0;
  for (int i = threadIdx.x; i < n && cnt < 8; i += NT) {
    const double xv = lam[off[m] + i] / s;
    const double q = b0 + b1 * xv + b2 * xv * xv;
    x[cnt] = xv;
    y[cnt] = pow(q, p) * xv;
    ++cnt;
  }
  int k = 0;
  for (; k <= max_iter; ++k) {
    double r2 = 0.0;
    for (int t = 0; t < cnt; ++t) r2 += (1.0 - y[t]) * (1.0 - y[t]);
    r2 = block_red(wsum(r2), 0, sh);
    if (!(r2 == r2) || r2 > 1e12) {  // NaN or diverging: not converged
      k = max_iter + 1;
      break;
    }
    if (sqrt(r2) < tol) break;
    for (int t = 0; t < cnt; ++t) {  // y <- y ((p + 1 - y) / p)^p  (M <- N^p M)
      const double nf = (p + 1 - y[t]) / p;
      y[t] = pow(nf, p) * y[t];
    }
  }
  if (threadIdx.x == 0) counts[(size_t)m * (ncand ? ncand : 1) + ci] = k;
  (void)x;
}

}  // namespace

int mlp_nparam() { return NPARAM; }

hipError_t features(const double* Apack, const int64_t* off, const int* ns, const int* ps,
                    int batch, float* feat, hipStream_t stream) {
  hipLaunchKernelGGL(features_kernel, dim3(batch), dim3(NT), 0, stream, Apack, off, ns, ps, 0, 0,
                     feat);
  return hipGetLastError();
}

int features_one_part(int n) { return n < kFeatRowsMin ? 0 : ((n + 15) / 16) * kRowStats; }

hipError_t features_one(const double* A, int n, int p, const double* norms, double* part,
                        float* feat, hipStream_t stream) {
  if (n < kFeatRowsMin) {
    hipLaunchKernelGGL(features_kernel, dim3(1), dim3(NT), 0, stream, A, nullptr, nullptr, nullptr,
                       n, p, feat);
    return hipGetLastError();
  }
  // one workgroup cannot stream a large matrix at HBM speed (909 ms for
  // n = 16384): rows are spread over n / 16 workgroups
  const int nb = (n + 15) / 16;
  hipLaunchKernelGGL(features_rows_kernel, dim3(nb), dim3(NT), 0, stream, A, n, part);
  hipLaunchKernelGGL(features_finish_kernel, dim3(1), dim3(NT), 0, stream, part, nb, n, p, norms,
                     feat);
  return hipGetLastError();
}

hipError_t mlp_forward(const float* params, const float* X, int batch, float* Y, float* Z1,
                       float* Z2, hipStream_t stream) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((batch + NT - 1) / NT), dim3(NT), 0, stream, params,
                     X, batch, Y, Z1, Z2);
  return hipGetLastError();
}

hipError_t mlp_train_step(float* params, float* grad, float* m, float* v, const float* X,
                          const float* T, int batch, int step, float lr, float* loss,
                          const MlpScratch& s, hipStream_t stream) {
  const dim3 g((batch + NT - 1) / NT);
  hipLaunchKernelGGL(mlp_forward_kernel, g, dim3(NT), 0, stream, params, X, batch, s.Y, s.Z1, s.Z2);
  hipLaunchKernelGGL(mlp_backward_sample_kernel, g, dim3(NT), 0, stream, params, s.Y, T, s.Z1,
                     s.Z2, batch, s.dY, s.dZ1, s.dZ2, s.H1, s.H2, s.lossv);
  hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((NPARAM + NT - 1) / NT), dim3(NT), 0, stream, X,
                     s.H1, s.H2, s.dY, s.dZ1, s.dZ2, batch, grad);
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(1024), 0, stream, s.lossv, batch, loss);
  const float bc1 = 1.f - powf(0.9f, (float)step), bc2 = 1.f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + NT - 1) / NT), dim3(NT), 0, stream, params, grad,
                     m, v, NPARAM, lr, bc1, bc2);
  return hipGetLastError();
}

hipError_t spectral_counts(const double* lam, const int64_t* off, const int* ns, const int* ps,
                           const double* scale, const double* cand, int ncand, int batch,
                           double tol, int max_iter, int* counts, hipStream_t stream) {
  hipLaunchKernelGGL(spectral_counts_kernel, dim3(ncand ? ncand : 1, batch), dim3(NT), 0, stream,
                     lam, off, ns, ps, scale, cand, ncand, tol, max_iter, counts);
  return hipGetLastError();
}

}  // namespace ipr
