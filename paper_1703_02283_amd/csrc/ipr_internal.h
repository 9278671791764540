// Internal declarations shared by the HIP translation units of libipr.
// Not part of the public C ABI (include/ipr.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ipr {

// Affine epilogue applied to each output element (i, j) of a product
// acc = L^T R:
//   out = alpha * acc + beta * X[i,j] + gamma * (i == j)
//   D[i,j] = out                                   (when D != nullptr)
//   S[i,j] = (s_init ? sa*(i==j) + sb*Y[i,j] : S[i,j]) + sc*out   (when S != nullptr)
//   partial[tile] = sum of (out - pd*(i==j))^2 over the tile (when partial != nullptr)
// With rfmt != 0, out and the S value are rounded as stored values
// (round_store) before they are written and before S and the partial sums
// use out.
// In triangle mode only tiles with row-block <= column-block are computed;
// every element with i <= j is written to (i, j) and (j, i), and the partial
// sums count off-diagonal elements twice, so they are sums over the full matrix.
struct Epilogue {
  double alpha = 1.0;
  double beta = 0.0;
  const double* X = nullptr;
  double gamma = 0.0;
  double* D = nullptr;
  double* S = nullptr;
  const double* Y = nullptr;
  double sa = 0.0, sb = 0.0, sc = 0.0;
  int s_init = 0;
  double* partial = nullptr;
  double pd = 0.0;
  int rfmt = 0;    // 0: none, 1: float with rbits stored mantissa bits, 2: fixed point, rbits fractional bits
  int rbits = 0;
};

// A value as the approximate storage of Sections III-C and IV keeps it: a
// float with `bits` stored mantissa bits and an unbounded exponent (fmt 1),
// or fixed point with `bits` fractional bits and enough integer bits (fmt 2);
// round to nearest, ties to even. Zero, Inf and NaN pass unchanged.
__host__ __device__ inline double round_store(double v, int fmt, int bits) {
  if (fmt == 1) {
    if (v == 0.0 || !(fabs(v) <= 1.79769313486231570815e308)) return v;
    const int sh = ilogb(v) - bits;  // leading bit 2^ilogb(v): weight of the last stored bit
    return ldexp(rint(ldexp(v, -sh)), sh);
  }
  if (fmt == 2) return ldexp(rint(ldexp(v, bits)), -bits);
  return v;
}

// Residual below which the FP64 phase counts stagnation toward IPR_EFLOOR.
// When ||I - M_k|| <= 1/2 every eigenvalue error e of M_k has |e| <= 1/2 and
// one exact step of eq. (1) leaves at most |e|/2 (p = 1 exactly; less for
// p >= 2), so a step that does not halve the residual there is rounding.
// Between 1/2 and 1 one small eigenvalue still in the slow phase of the
// iteration can hold the residual nearly flat for several steps.
constexpr double kFloorZone = 0.5;

// Number of per-tile partial slots a product of order n writes.
int gemm_partial_slots(int n, int tri);

// D = L^T R (n x n, row-major, leading dimension n) in FP64 on the matrix
// cores, with the epilogue above. L^T R equals L R whenever L is symmetric,
// which holds for every left operand of the iteration.
// With `scratch` (scratch_elems >= gemm_tail_scratch_elems(n) doubles,
// device), a triangle product whose tiles do not fill whole rounds of the CUs
// splits its last tiles along k among all CUs.
hipError_t gemm_f64(const double* L, const double* R, int n, int tri,
                    const Epilogue& e, hipStream_t stream, double* scratch = nullptr,
                    size_t scratch_elems = 0);
size_t gemm_tail_scratch_elems(int n);

// sqrt(sum of slots[0..count)) into *out (device), fixed summation order.
hipError_t reduce_fro(const double* slots, int count, double* out, hipStream_t stream);

// Column and row sums of |A|; writes norm1 = max column sum and
// norminf = max row sum to out[0], out[1] (device). scratch holds n doubles.
hipError_t norms_1_inf(const double* A, int n, double* scratch, double* out,
                       hipStream_t stream);

// C = c I, M = cp A and N = ((p+1) I - M) / p, with per-row partial sums of
// (I - M)^2 in partial[0..n).
hipError_t init_identity(const double* A, int n, int p, double c, double cp, double* C,
                         double* M, double* N, double* partial, hipStream_t stream);

// Y = a * X + b * I (elementwise over an n x n matrix).
hipError_t affine(const double* X, int n, double a, double b, double* Y,
                  hipStream_t stream);

hipError_t copy(const double* X, size_t count, double* Y, hipStream_t stream);

// X[i] = round_store(X[i], fmt, bits) for i < count.
hipError_t round_matrix(double* X, size_t count, int fmt, int bits, hipStream_t stream);

// Y = a0 I + a1 A + a2 G (G may be null).
hipError_t lincomb(const double* A, const double* G, int n, double a0, double a1, double a2,
                   double* Y, hipStream_t stream);

// X <- (X + X^T) / 2 in place.
hipError_t symmetrize(double* X, int n, hipStream_t stream);
// Y = X^T for n x n row-major X (Y must not alias X).
hipError_t transpose(const double* X, int n, double* Y, hipStream_t stream);

// Lanczos vector kernels (lanczos.hip)
hipError_t lz_gemv(const double* A, int n, const double* x, double* y, hipStream_t stream);
hipError_t lz_dots(const double* Q, int m, int n, const double* w, double* h, hipStream_t stream);
hipError_t lz_sub(const double* Q, int m, int n, const double* h, double* w, hipStream_t stream);
hipError_t lz_scale(const double* w, int n, double a, double* v, hipStream_t stream);
hipError_t lz_start(double* v, int n, hipStream_t stream);

}  // namespace ipr
