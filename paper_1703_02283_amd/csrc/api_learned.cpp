// C ABI of the learned start: features, MLP inference and training steps,
// and the per-eigenvalue iteration counts used as training labels.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/ipr.h"
#include "ipr_host.h"
#include "learned.h"

using namespace ipr;

namespace {

// Host arrays describing a packed batch are staged into the workspace.
struct Staged {
  int64_t* off;
  int* n;
  int* p;
};

int stage(const int64_t* off, const int* n, const int* p, int batch, Carver& c, Staged* s,
          hipStream_t stream) {
  s->off = c.take<int64_t>(batch);
  s->n = c.take<int>(batch);
  s->p = c.take<int>(batch);
  if (!c.ok()) return fail(IPR_EARG, "workspace too small for the batch descriptors");
  HIP_TRY(hipMemcpyAsync(s->off, off, batch * sizeof(int64_t), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(s->n, n, batch * sizeof(int), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(s->p, p, batch * sizeof(int), hipMemcpyHostToDevice, stream));
  return IPR_OK;
}

}  // namespace

extern "C" {

int ipr_features(const double* dA, const int64_t* offsets, const int* n, const int* p, int batch,
                 float* dFeat, void* dWork, size_t work_bytes, hipStream_t stream) {
  g_last_error.clear();
  if (!dA || !offsets || !n || !p || !dFeat || !dWork || batch < 1)
    return fail(IPR_EARG, "ipr_features: bad argument");
  for (int i = 0; i < batch; ++i)
    if (n[i] < 1 || p[i] < 1 || offsets[i] < 0)
      return fail(IPR_EARG, "ipr_features: item %d has n=%d p=%d", i, n[i], p[i]);
  Carver c(dWork, work_bytes);
  Staged s;
  if (int rc = stage(offsets, n, p, batch, c, &s, stream)) return rc;
  HIP_TRY(features(dA, s.off, s.n, s.p, batch, dFeat, stream));
  HIP_TRY(hipStreamSynchronize(stream));  // the staged host arrays are the caller's
  return IPR_OK;
}

int ipr_mlp_forward(const float* dParams, const float* dX, float* dY, int batch,
                    hipStream_t stream) {
  g_last_error.clear();
  if (!dParams || !dX || !dY || batch < 1) return fail(IPR_EARG, "ipr_mlp_forward: bad argument");
  HIP_TRY(mlp_forward(dParams, dX, batch, dY, nullptr, nullptr, stream));
  return IPR_OK;
}

size_t ipr_mlp_workspace(int batch) {
  if (batch < 1) return 0;
  return (size_t)batch * kMlpScratchPerSample * sizeof(float) + 16 * 256;
}

int ipr_mlp_train_step(float* dParams, float* dGrad, float* dM, float* dV, const float* dX,
                       const float* dT, int batch, int step, float lr, float* dLoss, void* dWork,
                       size_t work_bytes, hipStream_t stream) {
  g_last_error.clear();
  if (!dParams || !dGrad || !dM || !dV || !dX || !dT || !dLoss || !dWork || batch < 1 ||
      step < 1 || !(lr > 0.f))
    return fail(IPR_EARG, "ipr_mlp_train_step: bad argument");
  Carver c(dWork, work_bytes);
  MlpScratch s;
  s.Y = c.take<float>((size_t)batch * 3);
  s.Z1 = c.take<float>((size_t)batch * 64);
  s.Z2 = c.take<float>((size_t)batch * 64);
  s.dY = c.take<float>((size_t)batch * 3);
  s.dZ1 = c.take<float>((size_t)batch * 64);
  s.dZ2 = c.take<float>((size_t)batch * 64);
  s.H1 = c.take<float>((size_t)batch * 64);
  s.H2 = c.take<float>((size_t)batch * 64);
  s.lossv = c.take<float>((size_t)batch);
  if (!c.ok()) return fail(IPR_EARG, "ipr_mlp_train_step: workspace too small");
  HIP_TRY(mlp_train_step(dParams, dGrad, dM, dV, dX, dT, batch, step, lr, dLoss, s, stream));
  return IPR_OK;
}

int ipr_spectral_counts(const double* dLam, const int64_t* offsets, const int* n, const int* p,
                        const double* scale, int batch, const double* cand, int ncand, double tol,
                        int max_iter, int* counts, void* dWork, size_t work_bytes,
                        hipStream_t stream) {
  g_last_error.clear();
  if (!dLam || !offsets || !n || !p || !scale || !cand || !counts || !dWork || batch < 1 ||
      ncand < 0 || !(tol > 0.0) || max_iter < 0)
    return fail(IPR_EARG, "ipr_spectral_counts: bad argument");
  for (int i = 0; i < batch; ++i)
    if (n[i] < 1 || n[i] > 2048 || p[i] < 1 || !(scale[i] > 0.0))
      return fail(IPR_EARG, "ipr_spectral_counts: item %d has n=%d p=%d", i, n[i], p[i]);
  Carver c(dWork, work_bytes);
  Staged s;
  if (int rc = stage(offsets, n, p, batch, c, &s, stream)) return rc;
  double* dScale = c.take<double>(batch);
  const size_t nc = ncand ? (size_t)ncand : (size_t)batch;  // 0: one per matrix
  const size_t ncount = ncand ? (size_t)batch * ncand : (size_t)batch;
  double* dCand = c.take<double>(3 * nc);
  int* dCounts = c.take<int>(ncount);
  if (!c.ok()) return fail(IPR_EARG, "ipr_spectral_counts: workspace too small");
  HIP_TRY(hipMemcpyAsync(dScale, scale, batch * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(dCand, cand, 3 * nc * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_TRY(spectral_counts(dLam, s.off, s.n, s.p, dScale, dCand, ncand, batch, tol, max_iter,
                          dCounts, stream));
  HIP_TRY(hipMemcpyAsync(counts, dCounts, ncount * sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return IPR_OK;
}

}  // extern "C"
