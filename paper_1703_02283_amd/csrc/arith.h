// Kernels of the all-arithmetic regime (arith.hip): every scalar operation
// rounded with round_store (ipr_internal.h).
#pragma once
#include "ipr_internal.h"

namespace ipr {

// D = L^T R, upper triangle computed and mirrored; each term
// acc <- rnd(acc + rnd(L[k][i] R[k][j])) over k = 0 .. n-1 in order.
hipError_t gemm_arith(const double* L, const double* R, double* D, int n, int fmt, int bits,
                      hipStream_t stream);

// C = c I, M = rnd(cp rnd(A)) entry by entry.
hipError_t arith_start(const double* A, int n, double c, double cp, int fmt, int bits, double* C,
                       double* M, hipStream_t stream);

// N = rnd(I + rnd(rnd(I - M) / p)); partial[0..n) = row sums of (I - M)^2
// in float64.
hipError_t arith_next(const double* M, int n, int p, int fmt, int bits, double* N,
                      double* partial, hipStream_t stream);

// partial[0..n) = row sums of (X - Y)^2.
hipError_t diff_rows(const double* X, const double* Y, int n, double* partial,
                     hipStream_t stream);

}  // namespace ipr
