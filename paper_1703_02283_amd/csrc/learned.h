// Learned start (learned.hip): features, MLP, training, spectral labels.
#pragma once
#include <cstdint>

#include "ipr_internal.h"

namespace ipr {

int mlp_nparam();

struct MlpScratch {  // per-sample buffers of one training step (float32)
  float *Y, *Z1, *Z2, *dY, *dZ1, *dZ2, *H1, *H2, *lossv;
};
constexpr int kMlpScratchPerSample = 3 + 64 + 64 + 3 + 64 + 64 + 64 + 64 + 1;

hipError_t features(const double* Apack, const int64_t* off, const int* ns, const int* ps,
                    int batch, float* feat, hipStream_t stream);
// Features of one matrix; norms (device) holds ||A||_1, ||A||_inf, and part
// (device) features_one_part(n) doubles of scratch.
int features_one_part(int n);
hipError_t features_one(const double* A, int n, int p, const double* norms, double* part,
                        float* feat, hipStream_t stream);
hipError_t mlp_forward(const float* params, const float* X, int batch, float* Y, float* Z1,
                       float* Z2, hipStream_t stream);
hipError_t mlp_train_step(float* params, float* grad, float* m, float* v, const float* X,
                          const float* T, int batch, int step, float lr, float* loss,
                          const MlpScratch& s, hipStream_t stream);
hipError_t spectral_counts(const double* lam, const int64_t* off, const int* ns, const int* ps,
                           const double* scale, const double* cand, int ncand, int batch,
                           double tol, int max_iter, int* counts, hipStream_t stream);

}  // namespace ipr
