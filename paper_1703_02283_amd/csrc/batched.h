// Persistent batched solver (batched.hip): per-matrix work items and results.
#pragma once
#include <cstdint>

#include "ipr_internal.h"

namespace ipr {

// Resident workgroups per CU (the kernel's launch bound and the grid size).
constexpr int kBatchWgPerCu = 2;

// Elements between an item's scratch matrices: n^2 rounded up to 32, so
// that with a 256-byte aligned scratch base every scratch matrix starts on a
// 256-byte boundary (the products' 16-byte direct loads need 16).
__host__ __device__ inline size_t batch_scratch_stride(int n) {
  return ((size_t)n * n + 31) & ~(size_t)31;
}

struct BatchItem {
  int64_t a_off;   // element offset of A_i (and C_i) in the packed buffers
  int64_t s_off;   // element offset of its 7 scratch matrices (batch_scratch_stride apart)
  int n, p, tile, pad;
};

struct BatchResult {
  int status, iters_bulk, iters_fp64, fallback_used;
  double residual_proxy, residual_true, norm1, norminf;
  double init_scale, lmin_est;
  double lmin_reest;  // lower end of M_k estimated again (scaled steps), before step reest_iter
  int reest_iter, pad;
};

struct BatchArgs {
  const double* A;
  double* C;
  double* scratch;
  const BatchItem* items;
  const int* order;      // items by decreasing estimated work
  int count;             // items in order[]
  int* next;             // work counter: the next position of order[] to take (zeroed per launch)
  BatchResult* results;  // by item index
  double tol, bulk_switch, stall_ratio;
  int max_iter, bulk_bf16;
  int squarings;  // scale_squarings of the schedule (FP64 items)
  int dynamic;    // dynamic_scaling of the schedule (FP64 items, n >= 32)
  int lanczos_scale;  // scale_lanczos of the schedule (FP64 items, n >= 32)
};

hipError_t batched_launch(const BatchArgs& args, int grid, hipStream_t stream);

// Fills matrices with a deterministic SPD pattern (autotuner input):
// A_i = diag(1 + j/n) + small symmetric off-diagonal band.
hipError_t batched_fill_test(double* A, const BatchItem* items, int count, hipStream_t stream);

}  // namespace ipr
