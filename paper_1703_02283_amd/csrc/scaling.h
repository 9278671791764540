// Scalar rules of the scaled-identity start and of the dynamically scaled
// iteration, shared by the single solve (solve.cpp) and the batched solver
// (batched.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace ipr {

// One coupled step maps an eigenvalue m of M to g(m) = m ((p + 1 - m) / p)^p.
__host__ __device__ inline double step_map(double m, int p) {
  return m * pow((p + 1.0 - m) / p, (double)p);
}

// Bounds [na, nb] on the spectrum of M after one step with scale factor mu,
// from bounds [a, b] before it (g rises on (0, 1), has its maximum 1 at 1
// and falls on (1, p + 1)).
__host__ __device__ inline void step_bounds(double a, double b, double mu, int p, double* na,
                                            double* nb) {
  const double ga = step_map(mu * a, p), gb = step_map(mu * b, p);
  *na = fmin(ga, gb);
  *nb = (mu * a <= 1.0 && 1.0 <= mu * b) ? 1.0 : fmax(ga, gb);
}

// Largest scaled top of the spectrum: below 2 (eq. (2)'s region) and, for
// p = 1, where g(m) = m (2 - m) = 1/2: a top eigenvalue pushed closer to 2
// falls near 0 after the step and climbs back with fewer correct digits (the
// p = 1 floor rose 2-3x at kappa >= 3e4 with a cap of 1.98). For p >= 2,
// g(2) >= 1/2 already.
__host__ __device__ inline double mu_cap(int p) { return p == 1 ? 1.0 + sqrt(0.5) : 1.98; }

// A squaring of the start's scale bound (one product) pays when it lowers
// the bound by more than what one product buys in the slow phase of the
// iteration, where the lower end of the spectrum grows by (1 + 1/p)^p per
// step of p + 1 products, or by mu_cap (1 + 1/p)^p with scaled steps.
// Successive squarings improve the bound by about the square root of the
// previous improvement, so squaring stops once that prediction falls below.
__host__ __device__ inline double squaring_worth(int p, bool scaled_steps) {
  const double grow = pow(1.0 + 1.0 / p, (double)p) * (scaled_steps ? mu_cap(p) : 1.0);
  return pow(grow, 1.0 / (p + 1.0));
}

// Scale factor of a step on a spectrum in [a, b]: the mu in [1, mu_cap / b]
// that maximises the lower end after the step, min(g(mu a), g(mu b)); 1 once
// a >= 1/2, where the unscaled step is already in its quadratic phase.
__host__ __device__ inline double choose_mu(double a, double b, int p) {
  if (!(a > 0.0) || !(b > 0.0) || a >= 0.5) return 1.0;
  const double hi = mu_cap(p) / b;
  if (hi <= 1.0) return 1.0;
  if (step_map(hi * a, p) - step_map(hi * b, p) <= 0.0) return hi;  // lower end binds at the cap
  if (step_map(a, p) - step_map(b, p) >= 0.0) return 1.0;
  double lo = 1.0, up = hi;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + up);
    if (step_map(mid * a, p) - step_map(mid * b, p) < 0.0)
      lo = mid;
    else
      up = mid;
  }
  return lo;
}

// Smallest eigenvalue of the symmetric tridiagonal matrix with diagonal
// al[0..m) and off-diagonal be[0..m-1), by bisection on the Sturm count.
__host__ __device__ inline double tridiag_min(const double* al, const double* be, int m) {
  double lo = al[0], hi = al[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < m ? fabs(be[i]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double x = 0.5 * (lo + hi);
    int below = 0;  // eigenvalues < x
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      d = al[i] - x - (i > 0 ? be[i - 1] * be[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      below += d < 0.0;
    }
    if (below >= 1)
      hi = x;
    else
      lo = x;
  }
  return hi;
}

}  // namespace ipr
