// Low-precision operand storage and products (lowp.hip).
#pragma once
#include "ipr_internal.h"

namespace ipr {

// Same codes as ipr_dtype.
enum { LP_BF16 = 1, LP_FP16 = 2, LP_FP8 = 3, LP_I8 = 4 };

int lp_padded(int n);              // n rounded up to a multiple of 256
int lp_esize(int dtype);           // bytes per code
size_t lp_bytes(int n, int dtype); // bytes of one padded code matrix
size_t lp_exp_count(int n);        // ints of one tile-exponent array
int lp_partial_slots(int n, int tri);

// Q (padded, transposed) and E (per-tile exponents) from X (n x n float64).
hipError_t quantize_t(const double* X, int n, int dtype, void* Q, int* E, hipStream_t stream);

// D = L^T R from quantized operands (fp32 accumulation) with the float64 epilogue.
hipError_t gemm_lp(const void* Lq, const int* EL, const void* Rq, const int* ER, int n,
                   int dtype, int tri, const Epilogue& e, hipStream_t stream);

// FP64-accurate products from int8 digit slices (error-free splitting,
// beta = 7 bits per digit, s digits per entry).
constexpr int kMaxSlices = 12;
size_t slice_bytes(int n);   // bytes of one digit matrix (padded, transposed)
int slice_max_n();           // largest order whose digit products fit an int32 accumulation

// s digit matrices of X^T into Q (s * slice_bytes(n) bytes), the row
// exponents of X^T into E (lp_padded(n) ints); cm: n scratch words.
hipError_t slices_split(const double* X, int n, int s, void* Q, int* E, unsigned long long* cm,
                        hipStream_t stream);

// D = L^T R from two such splits, with the float64 epilogue. P and S: n x n
// float64 scratch (a level's exact partial sum, the running sum of levels).
hipError_t gemm_slices(const void* Lq, const int* EL, const void* Rq, const int* ER, int n, int s,
                       double* P, double* S, int tri, const Epilogue& e, hipStream_t stream);

}  // namespace ipr
