// Host driver of libipr: argument checks, workspace carving, the starts of
// Section II and the iteration loop of eq. (1), built from the kernels of
// gemm_f64.hip and elementwise.hip.
//
// Evaluation of eq. (1). In exact arithmetic every iterate is a polynomial in
// A, so eq. (1) can carry M_k = C_k^p A beside C_k (the coupled form):
//   N_k = I + (I - M_k) / p,  C_{k+1} = C_k N_k,  M_{k+1} = N_k^p M_k,
// and C_{k+1} equals ((p + 1) C_k - C_k^{p+1} A) / p. This ordering is stable
// (the right-multiplied order of eq. (1) amplifies rounding errors that do
// not commute with A), costs p + 1 products per iteration and yields the
// residual I - M_k for free. The last product of each iteration also writes
// N_{k+1} and the Frobenius partial sums of I - M_{k+1} in its epilogue.
// For p = 1 after a low-precision phase the Newton-Schulz order
// R_k = I - A C_k, C_{k+1} = C_k + C_k R_k is used instead: it recomputes the
// residual from A and so removes errors of any kind.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/ipr.h"
#include "ipr_host.h"
#include "scaling.h"
#include "ipr_internal.h"
#include "arith.h"
#include "learned.h"
#include "lowp.h"

namespace ipr {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

static double* pinned_scalars() {
  thread_local double* buf = nullptr;
  if (!buf) {
    if (hipHostMalloc((void**)&buf, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
      buf = nullptr;
  }
  return buf;
}

thread_local bool g_no_alloc = false;

int read_scalars(const double* d, int count, double* host, hipStream_t stream) {
  if (g_no_alloc) {
    // no pinned buffer (its first use would allocate): a copy to pageable
    // host memory, which the runtime stages itself
    HIP_TRY(hipMemcpyAsync(host, d, count * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return IPR_OK;
  }
  double* pin = pinned_scalars();
  if (!pin) return fail(IPR_EHIP, "hipHostMalloc of the scalar buffer failed");
  HIP_TRY(hipMemcpyAsync(pin, d, count * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (int i = 0; i < count; ++i) host[i] = pin[i];
  return IPR_OK;
}

void poly_guard(const double b[3], int p, double* sup_phi, int* q_pos) {
  auto q = [&](double x) { return b[0] + b[1] * x + b[2] * x * x; };
  auto phi = [&](double x) { return std::pow(q(x), p) * x; };
  // sup of q^p x on [0, 1]: at x = 1 or at a root of
  // d/dx (q^p x) / q^(p-1) = (2p+1) b2 x^2 + (p+1) b1 x + b0 in (0, 1).
  double s = phi(1.0);
  const double aa = (2.0 * p + 1.0) * b[2], bb = (p + 1.0) * b[1], cc = b[0];
  if (aa != 0.0) {
    const double disc = bb * bb - 4 * aa * cc;
    if (disc >= 0) {
      const double sq = std::sqrt(disc);
      for (double x : {(-bb + sq) / (2 * aa), (-bb - sq) / (2 * aa)})
        if (x > 0.0 && x < 1.0) s = std::max(s, phi(x));
    }
  } else if (bb != 0.0) {
    const double x = -cc / bb;
    if (x > 0.0 && x < 1.0) s = std::max(s, phi(x));
  }
  // q > 0 on (0, 1]
  int pos;
  if (b[0] == 0.0) {
    // q = x (b1 + b2 x): positive on (0, 1] iff b1 > 0 and b1 + b2 > 0 ... and
    // b1 + b2 x > 0 on (0, 1], i.e. at both ends of the linear factor
    pos = (b[1] > 0.0 && b[1] + b[2] > 0.0) ? 1 : 0;
  } else {
    double mq = std::min(q(0.0), q(1.0));
    if (b[2] != 0.0) {
      const double xv = -b[1] / (2 * b[2]);
      if (xv > 0.0 && xv < 1.0) mq = std::min(mq, q(xv));
    }
    pos = mq > 0.0 ? 1 : 0;
  }
  *sup_phi = s;
  *q_pos = pos;
}

// Least value of phi(x) = q(x)^p x over [a, 1] for q(x) = b0 + b1 x + b2 x^2
// positive there: at an end or at a root of (2p+1) b2 x^2 + (p+1) b1 x + b0
// (where d/dx phi vanishes).
double poly_min(const double b[3], int p, double a) {
  auto phi = [&](double x) { return std::pow(b[0] + b[1] * x + b[2] * x * x, p) * x; };
  double m = std::min(phi(a), phi(1.0));
  const double aa = (2.0 * p + 1.0) * b[2], bb = (p + 1.0) * b[1], cc = b[0];
  if (aa != 0.0) {
    const double disc = bb * bb - 4 * aa * cc;
    if (disc >= 0) {
      const double sq = std::sqrt(disc);
      for (double x : {(-bb + sq) / (2 * aa), (-bb - sq) / (2 * aa)})
        if (x > a && x < 1.0) m = std::min(m, phi(x));
    }
  } else if (bb != 0.0) {
    const double x = -cc / bb;
    if (x > a && x < 1.0) m = std::min(m, phi(x));
  }
  return m;
}

}  // namespace ipr

using namespace ipr;

namespace {

constexpr int NMAT = 7;     // float64 n x n work matrices
// Lower end of the scaled iteration's spectrum bound at which lambda_min(M_k)
// is estimated again (dynamic scaling)
constexpr double kReestimateAt = 0.03;
constexpr int NLP = 6;      // quantized operand slots (low-precision phase)

struct Work {
  double* m[NMAT];
  double* partial;
  double* norms_scratch;
  double* scal;
  void* lq[NLP];
  int* le[NLP];
  // int8-slice products: digit matrices of L^T and R^T in lq[0], lq[1]
  unsigned long long* cm;
  double* slP;
  double* slS;
  double* Ar;   // approximate storage: A as stored
  double* tail; // split tail of the FP64 triangle products
  size_t tail_elems;
};

// digits per operand of the int8-slice products (0 when the dtype does not use them)
int emul_digits(const ipr_schedule& s) {
  if (s.bulk_dtype != IPR_FP64_INT8_EMUL) return 0;
  return s.emul_slices ? s.emul_slices : 10;
}

int n_mats(int p) { return p == 1 ? 5 : (p == 2 ? 6 : NMAT); }

// Powers L^p by repeated squaring when p is a power of two >= 4 (fewer
// products than p - 1 successive ones).
bool binary_powers(int p) { return p >= 4 && (p & (p - 1)) == 0; }

size_t carve(int n, int p, int dtype, int slices, bool store, Work* w, void* base, size_t cap,
             bool* ok) {
  Carver c(base, cap);
  const size_t nn = (size_t)n * n;
  const int nm = n_mats(p);
  for (int i = 0; i < NMAT; ++i) w->m[i] = i < nm ? c.take<double>(nn) : nullptr;
  const size_t slots =
      std::max<size_t>(std::max(gemm_partial_slots(n, 0), gemm_partial_slots(n, 1)), n);
  w->partial = c.take<double>(slots);
  const size_t strips = (n + 255) / 256;
  w->norms_scratch = c.take<double>(2 * (size_t)n + strips * n);
  w->scal = c.take<double>(64);
  const bool emul = dtype == IPR_FP64_INT8_EMUL;
  for (int i = 0; i < NLP; ++i) {
    const bool lp = dtype != IPR_FP64 && !emul;
    const bool sl = emul && i < 2;
    w->lq[i] = lp   ? (void*)c.take<uint8_t>(lp_bytes(n, dtype))
               : sl ? (void*)c.take<uint8_t>((size_t)slices * slice_bytes(n))
                    : nullptr;
    w->le[i] = lp ? c.take<int>(lp_exp_count(n)) : sl ? c.take<int>(lp_padded(n)) : nullptr;
  }
  w->cm = emul ? c.take<unsigned long long>(n) : nullptr;
  w->slP = emul ? c.take<double>(nn) : nullptr;
  w->slS = emul ? c.take<double>(nn) : nullptr;
  w->Ar = store ? c.take<double>(nn) : nullptr;
  w->tail_elems = gemm_tail_scratch_elems(n);
  w->tail = w->tail_elems ? c.take<double>(w->tail_elems) : nullptr;
  *ok = c.ok();
  return c.used;
}

// Phase times from device events (none in the allocation-free entry point,
// where every ms_* field stays 0).
struct Timer {
  hipEvent_t ev[8] = {};
  hipStream_t s;
  bool on;
  Timer(hipStream_t st, bool enabled) : s(st), on(enabled) {
    if (on)
      for (auto& e : ev) (void)hipEventCreate(&e);
  }
  ~Timer() {
    if (on)
      for (auto& e : ev) (void)hipEventDestroy(e);
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
  double ms(int a, int b) {
    float t = 0.f;
    if (!on || hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0.0;
    return t;
  }
};

// Products of one solve. In the low-precision phase every operand is read
// through a small cache of quantized copies; a float64 matrix that a product
// or an elementwise kernel rewrites loses its cached copy.
struct Prod {
  int n;
  hipStream_t st;
  int lowp_dtype = 0;  // 0: FP64 products
  int emul = 0;        // > 0: int8-slice products with this many digits
  int rfmt = 0, rbits = 0;  // approximate storage of the iteration's products (round_store)
  Work* w;
  int gemms = 0;
  bool timing = false;
  std::vector<hipEvent_t> ev;  // start/stop pairs of timed products
  std::vector<double> flops;
  std::vector<char> is_lp;     // per timed product: low-precision kernel
  const double* src[NLP] = {};
  bool valid[NLP] = {};
  unsigned long use[NLP] = {};
  unsigned long clock = 0;

  void invalidate(const double* X) {
    for (int i = 0; i < NLP; ++i)
      if (src[i] == X) valid[i] = false;
  }
  int slot_for(const double* X, int keep, hipError_t* err) {
    for (int i = 0; i < NLP; ++i)
      if (valid[i] && src[i] == X) {
        use[i] = ++clock;
        return i;
      }
    int v = -1;  // a free slot, else the least recently used one (never `keep`)
    for (int i = 0; i < NLP && v < 0; ++i)
      if (i != keep && !valid[i]) v = i;
    if (v < 0)
      for (int i = 0; i < NLP; ++i)
        if (i != keep && (v < 0 || use[i] < use[v])) v = i;
    *err = quantize_t(X, n, lowp_dtype, w->lq[v], w->le[v], st);
    src[v] = X;
    valid[v] = true;
    use[v] = ++clock;
    return v;
  }
  ~Prod() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  // a product in FP64 whatever the phase
  hipError_t f64(const double* L, const double* R, int tri, const Epilogue& e) {
    const int keep = lowp_dtype, keep_e = emul, keep_r = rfmt;
    lowp_dtype = 0;
    emul = 0;
    rfmt = 0;
    hipError_t err = (*this)(L, R, tri, e);
    lowp_dtype = keep;
    emul = keep_e;
    rfmt = keep_r;
    return err;
  }
  hipError_t operator()(const double* L, const double* R, int tri, const Epilogue& e_in) {
    hipError_t err = hipSuccess;
    Epilogue e = e_in;
    if (rfmt && !lowp_dtype && !emul) {  // (the FP64 kernel's epilogue rounds; solve() allows
                                          // approximate storage with FP64 products only)
      e.rfmt = rfmt;
      e.rbits = rbits;
    }
    ++gemms;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto start = [&]() -> hipError_t {
      if (!timing) return hipSuccess;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return hipErrorOutOfMemory;
      ev.push_back(e0);
      ev.push_back(e1);
      flops.push_back(tri ? (double)n * n * (n + 1.0) : 2.0 * n * n * (double)n);
      is_lp.push_back(lowp_dtype != 0 || emul != 0);
      return hipEventRecord(e0, st);
    };
    if (emul) {
      // split afresh for every product (about 1% of its time): no cached
      // digits can go stale behind a kernel that rewrites an operand
      if ((err = slices_split(L, n, emul, w->lq[0], w->le[0], w->cm, st)) != hipSuccess) return err;
      const int b = R == L ? 0 : 1;
      if (b && (err = slices_split(R, n, emul, w->lq[1], w->le[1], w->cm, st)) != hipSuccess)
        return err;
      if ((err = start()) != hipSuccess) return err;
      err = gemm_slices(w->lq[0], w->le[0], w->lq[b], w->le[b], n, emul, w->slP, w->slS, tri, e,
                        st);
    } else if (!lowp_dtype) {
      if ((err = start()) != hipSuccess) return err;
      err = gemm_f64(L, R, n, tri, e, st, w->tail, w->tail_elems);
    } else {
      const int a = slot_for(L, -1, &err);
      if (err != hipSuccess) return err;
      const int b = slot_for(R, a, &err);
      if (err != hipSuccess) return err;
      if ((err = start()) != hipSuccess) return err;
      err = gemm_lp(w->lq[a], w->le[a], w->lq[b], w->le[b], n, lowp_dtype, tri, e, st);
    }
    if (e1) (void)hipEventRecord(e1, st);
    if (e.D) invalidate(e.D);
    if (e.S) invalidate(e.S);
    return err;
  }
  // partial sums written by the last product (the kernels' grids differ)
  int slots(int tri) const {
    return (lowp_dtype || emul) ? lp_partial_slots(n, tri) : gemm_partial_slots(n, tri);
  }
  // after the stream has drained
  void totals(int lp, int* count, double* ms, double* fl) const {
    *count = 0;
    *ms = *fl = 0.0;
    for (size_t i = 0; i < flops.size(); ++i) {
      if ((is_lp[i] != 0) != (lp != 0)) continue;
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) *ms += t;
      *fl += flops[i];
      ++*count;
    }
  }
};

#define TRY(expr)                       \
  do {                                  \
    hipError_t _e = (expr);             \
    if (_e != hipSuccess)               \
      return fail(IPR_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

struct Solver {
  const double* A;      // the A the iteration multiplies by (as stored)
  const double* Atrue;  // the caller's A: the final check uses it
  int n, p, tri;
  hipStream_t st;
  Work w;
  Prod prod;
  double* Cb[2];
  int ci = 0;
  double* Mb[2];
  int mi = 0;
  double* Nb[2];
  int ni = 0;
  double* X[2] = {nullptr, nullptr};
  double* Rns = nullptr;  // Newton-Schulz residual (p = 1 after a low-precision phase)
  int slots = 0;          // partial slots holding the current residual's sum of squares
  // dynamically scaled iteration: M_k enters step k as mu_cur M_k (with C_k as
  // mu_cur^{1/p} C_k); the product that forms M_{k+1} writes N_{k+1} for
  // mu_next
  double mu_cur = 1.0, mu_next = 1.0;
  // scaled Newton-Schulz step (p = 1): the step runs on mu C_k, whose
  // residual is (1 - mu) I + mu R_k, so C_{k+1} = mu (2 - mu) C_k + mu^2 C_k R_k
  double ns_mu = 1.0;

  double* C() { return Cb[ci]; }
  double* M() { return Mb[mi]; }
  double* rho_dev() { return w.scal + 8; }

  int reduce() {
    TRY(reduce_fro(w.partial, slots, rho_dev(), st));
    return IPR_OK;
  }

  // Epilogue of the product that yields M: writes M, N = ((p+1) I - M) / p and
  // the partial sums of (I - M)^2.
  Epilogue m_epilogue(double* Mout, double* Nout) {
    Epilogue e;
    e.D = Mout;
    e.S = Nout;
    e.s_init = 1;
    e.sa = (p + 1.0) / p;
    e.sc = -mu_next / p;
    e.partial = w.partial;
    e.pd = 1.0;
    return e;
  }

  // Mout = L^p alpha1 B (last product with m_epilogue), t = triangle mode.
  // For p a power of two >= 4 by binary powering: P = L^(p/2) from repeated
  // squaring, then P (P B), log2(p) + 1 products (3 instead of 4 for p = 4);
  // otherwise L (L (... (L B))), p products.
  int power_chain(const double* L, const double* B, double* Mout, double* Nout, int t,
                  double alpha1 = 1.0) {
    if (binary_powers(p)) {
      const double* P = L;
      int xb = 0;  // X[0] and X[1] alternate (both exist for p >= 3)
      for (int q = 1; 2 * q <= p / 2; q *= 2) {
        Epilogue e;  // L^(2q) = L^q L^q
        e.D = X[xb];
        TRY(prod(P, P, t, e));
        P = e.D;
        xb ^= 1;
      }
      Epilogue e;  // T = P alpha1 B
      e.D = X[xb];
      e.alpha = alpha1;
      TRY(prod(P, B, t, e));
      TRY(prod(P, e.D, t, m_epilogue(Mout, Nout)));
    } else {
      const double* src = B;
      for (int j = 1; j <= p; ++j) {
        Epilogue e;
        if (j == p)
          e = m_epilogue(Mout, Nout);
        else
          e.D = X[(j - 1) & 1];  // j < p: X[0] for j = 1, X[1] exists when p >= 3
        if (j == 1) e.alpha = alpha1;
        TRY(prod(L, src, t, e));
        src = e.D;
      }
    }
    if (!t) {
      TRY(symmetrize(Mout, n, st));
      TRY(symmetrize(Nout, n, st));
      prod.invalidate(Mout);
      prod.invalidate(Nout);
    }
    slots = prod.slots(t);
    return reduce();
  }

  // One update of eq. (1); leaves the residual's partial sums in w.partial.
  // With m_update = false only C_{k+1} is formed (M and N are then stale
  // until recompute()).
  int step(bool ns, bool m_update = true) {
    double* Cc = C();
    double* Cn = Cb[ci ^ 1];
    if (ns) {
      Epilogue e;  // C_{k+1} = C_k + C_k R_k (symmetric: C_k - C_k A C_k + C_k)
      e.alpha = ns_mu * ns_mu;
      e.beta = ns_mu * (2.0 - ns_mu);
      e.X = Cc;
      e.D = Cn;
      TRY(prod(Cc, Rns, tri, e));
      if (!tri) TRY(symmetrize(Cn, n, st));
      prod.invalidate(Cn);
      // R_{k+1} = I - A C_{k+1}, full product: mirroring it would symmetrise the
      // residual, and C + C sym(I - A C) is not self-correcting (an error E that
      // does not commute with A is multiplied by (1 - lambda_j / lambda_i) / 2).
      Epilogue e2;
      e2.alpha = -1.0;
      e2.gamma = 1.0;
      e2.D = Rns;
      e2.partial = w.partial;
      TRY(prod(A, Cn, 0, e2));
      slots = prod.slots(0);
      ci ^= 1;
      return reduce();
    }
    double* Nc = Nb[ni];
    {
      Epilogue e;  // C_{k+1} = C_k N_k (scaled: mu^{1/p} C_k N_k)
      e.alpha = mu_cur == 1.0 ? 1.0 : std::pow(mu_cur, 1.0 / p);
      e.D = Cn;
      TRY(prod(Cc, Nc, tri, e));
      if (!tri) TRY(symmetrize(Cn, n, st));
      prod.invalidate(Cn);
    }
    if (!m_update) {
      ci ^= 1;
      return IPR_OK;
    }
    // M_{k+1} = N_k (N_k (... (N_k mu M_k))), N_{k+1} from M_{k+1}
    if (int rc = power_chain(Nc, M(), Mb[mi ^ 1], Nb[ni ^ 1], tri, mu_cur)) return rc;
    ci ^= 1;
    mi ^= 1;
    ni ^= 1;
    return IPR_OK;
  }

  // Literal order of eq. (1): X = C^p A (into Nb[1]) and the partial sums of
  // (I - X)^2. The iterate is not kept symmetric, so every left operand of a
  // product (which the kernel reads as L^T) is transposed first; C^T stays in
  // Mb[0] for the update.
  int literal_x() {
    double* T = Mb[0];
    double* T2 = Nb[0];
    double* Pb[2] = {Mb[1], X[0]};
    TRY(transpose(C(), n, T, st));
    for (int j = 2; j <= p; ++j) {  // C^j = C^{j-1} C
      Epilogue e;
      e.D = Pb[j & 1];
      TRY(prod.f64(j == 2 ? T : T2, C(), 0, e));
      TRY(transpose(e.D, n, T2, st));
    }
    Epilogue e;
    e.D = Nb[1];
    e.partial = w.partial;
    e.pd = 1.0;
    TRY(prod.f64(p == 1 ? T : T2, A, 0, e));
    slots = prod.slots(0);
    return reduce();
  }

  // C_{k+1} = ((p + 1) C_k - C_k X) / p with X from literal_x().
  int literal_update() {
    Epilogue e;
    e.alpha = -1.0 / p;
    e.beta = (p + 1.0) / p;
    e.X = C();
    e.D = Cb[ci ^ 1];
    TRY(prod.f64(Mb[0], Nb[1], 0, e));
    ci ^= 1;
    return IPR_OK;
  }

  // ||I - C^p A||_F into *tau (host): the symmetric powers C^2 .. C^p as
  // triangle products (when enabled), then one full product C^p A.
  int true_residual(double* tau) {
    const double* P = C();
    if (binary_powers(p)) {
      int xb = 0;
      for (int q = 1; q < p; q *= 2) {  // C^(2q) = C^q C^q
        Epilogue e;
        e.D = X[xb];
        TRY(prod.f64(P, P, tri, e));
        if (!tri) TRY(symmetrize(e.D, n, st));
        P = e.D;
        xb ^= 1;
      }
    } else {
      for (int j = 2; j <= p; ++j) {
        Epilogue e;
        e.D = X[j & 1];  // X[0] for C^2, X[1] (p >= 3) for C^3, ...
        TRY(prod.f64(C(), P, tri, e));
        if (!tri) TRY(symmetrize(e.D, n, st));
        P = e.D;
      }
    }
    Epilogue e;
    e.alpha = -1.0;
    e.gamma = 1.0;
    e.partial = w.partial;
    TRY(prod.f64(P, Atrue, 0, e));
    TRY(reduce_fro(w.partial, gemm_partial_slots(n, 0), w.scal + 9, st));
    return read_scalars(w.scal + 9, 1, tau, st);
  }

  // Smallest Ritz value of `steps` Lanczos steps on A with full
  // reorthogonalisation: an estimate of lambda_min(A) from above. buf holds
  // (steps + 2) n + steps + 2 doubles.
  int lanczos_min(int steps, double* buf, double* theta) {
    double hi;
    return lanczos_range(A, steps, buf, theta, &hi);
  }

  // Smallest and largest Ritz values of `steps` Lanczos steps on the
  // symmetric matrix S (estimates of its extreme eigenvalues from inside).
  int lanczos_range(const double* S, int steps, double* buf, double* theta, double* theta_hi) {
    double* Q = buf;
    double* wv = buf + (size_t)(steps + 1) * n;
    double* h = wv + n;
    double hs[2];
    TRY(lz_start(Q, n, st));
    TRY(lz_dots(Q, 1, n, Q, h, st));
    if (int rc = read_scalars(h, 1, hs, st)) return rc;
    TRY(lz_scale(Q, n, 1.0 / std::sqrt(hs[0]), Q, st));
    std::vector<double> al, be;
    for (int j = 0; j < steps; ++j) {
      TRY(lz_gemv(S, n, Q + (size_t)j * n, wv, st));
      TRY(lz_dots(Q, j + 1, n, wv, h, st));  // h[j] = q_j . A q_j = alpha_j
      if (int rc = read_scalars(h + j, 1, hs, st)) return rc;
      al.push_back(hs[0]);
      TRY(lz_sub(Q, j + 1, n, h, wv, st));
      TRY(lz_dots(Q, j + 1, n, wv, h, st));  // second pass
      TRY(lz_sub(Q, j + 1, n, h, wv, st));
      TRY(lz_dots(wv, 1, n, wv, h, st));
      if (int rc = read_scalars(h, 1, hs, st)) return rc;
      const double beta = std::sqrt(hs[0]);
      if (j + 1 == steps || !(beta > 1e-10 * std::fabs(al[0]))) break;  // invariant subspace
      be.push_back(beta);
      TRY(lz_scale(wv, n, 1.0 / beta, Q + (size_t)(j + 1) * n, st));
    }
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    *theta = tridiag_min(al.data(), be.data(), (int)al.size());
    std::vector<double> neg(al.size());
    for (size_t i = 0; i < al.size(); ++i) neg[i] = -al[i];
    *theta_hi = -tridiag_min(neg.data(), be.data(), (int)neg.size());
    return IPR_OK;
  }

  // Iterate k's entries of the caller's history arrays: rho = ||I - M_k||_F
  // and, with a reference matrix, ||C_k - ref||_F (one pass over C_k).
  int record_hist(const ipr_schedule& s, int k, double rho) {
    if (k < 0 || k >= s.hist_len) return IPR_OK;
    if (s.hist_rho) s.hist_rho[k] = rho;
    if (s.hist_ref && s.hist_err) {
      TRY(diff_rows(C(), s.hist_ref, n, w.norms_scratch, st));
      TRY(reduce_fro(w.norms_scratch, n, w.scal + 10, st));
      if (int rc = read_scalars(w.scal + 10, 1, &s.hist_err[k], st)) return rc;
    }
    return IPR_OK;
  }

  // M_k = C_k^p A (and N_k) from C_k, or R_k = I - A C_k in Newton-Schulz mode.
  int recompute(bool ns) {
    if (ns) {
      Epilogue e;
      e.alpha = -1.0;
      e.gamma = 1.0;
      e.D = Rns;
      e.partial = w.partial;
      TRY(prod(A, C(), 0, e));
      slots = prod.slots(0);
      return reduce();
    }
    return power_chain(C(), A, M(), Nb[ni], 0);
  }
};

// The all-arithmetic regime (schedule.store_regime = 1): the coupled
// iteration from the scaled identity with every scalar operation rounded to
// the custom type (arith.hip). The stopping rules are the FP64 loop's; the
// final check ||I - C^p A||_F runs in FP64 against the caller's A.
int solve_arith(Solver& sv, const ipr_schedule& s, double tol, double sigma, ipr_result& res) {
  const int n = sv.n, p = sv.p, fmt = s.store_format, bits = s.store_bits;
  hipStream_t st = sv.st;
  const double c = round_store(std::pow(sigma, -1.0 / p), fmt, bits);
  const double cp = round_store(std::pow(c, (double)p), fmt, bits);
  HIP_TRY(arith_start(sv.Atrue, n, c, cp, fmt, bits, sv.C(), sv.M(), st));
  HIP_TRY(arith_next(sv.M(), n, p, fmt, bits, sv.Nb[sv.ni], sv.w.partial, st));
  sv.slots = n;
  if (int rc = sv.reduce()) return rc;
  res.init_scale = sigma;
  res.init_bound = 1.0;
  res.poly_used[0] = 1.0;
  double best = std::numeric_limits<double>::infinity(), last_tau = best, rho = 0.0;
  int stale = 0, failed_verify = 0, status = IPR_EMAXITER, k = 0, verified_at = -1;
  for (k = 0;; ++k) {
    if (int rc = read_scalars(sv.rho_dev(), 1, &rho, st)) return rc;
    res.residual_proxy = rho;
    if (int rc = sv.record_hist(s, k, rho)) return rc;
    if (!std::isfinite(rho) || rho > 1e6) {
      status = IPR_EDIVERGED;
      break;
    }
    bool floor = false;
    if (rho < tol && s.verify) {
      double tau;
      if (int rc = sv.true_residual(&tau)) return rc;
      res.residual_true = tau;
      verified_at = k;
      if (tau < tol) {
        status = IPR_OK;
        break;
      }
      floor = ++failed_verify >= 2 && !(tau < 0.5 * last_tau);
      last_tau = tau;
    } else if (rho < tol) {
      status = IPR_OK;
      break;
    }
    if (rho < kFloorZone) {
      if (rho < s.stall_ratio * best) {
        best = rho;
        stale = 0;
      } else if (++stale >= 3) {
        floor = true;
      }
    }
    if (floor) {
      status = IPR_EFLOOR;
      break;
    }
    if (k >= s.max_iter) break;
    // C_{k+1} = C_k N_k, M_{k+1} = N_k (N_k (... (N_k M_k))), N_{k+1}
    double* Nc = sv.Nb[sv.ni];
    HIP_TRY(gemm_arith(sv.C(), Nc, sv.Cb[sv.ci ^ 1], n, fmt, bits, st));
    const double* src = sv.M();
    for (int j = 1; j <= p; ++j) {
      double* dst = j == p ? sv.Mb[sv.mi ^ 1] : sv.X[(j - 1) & 1];
      HIP_TRY(gemm_arith(Nc, src, dst, n, fmt, bits, st));
      src = dst;
    }
    sv.prod.gemms += p + 1;
    sv.ci ^= 1;
    sv.mi ^= 1;
    HIP_TRY(arith_next(sv.M(), n, p, fmt, bits, Nc, sv.w.partial, st));
    sv.slots = n;
    if (int rc = sv.reduce()) return rc;
  }
  res.iters_fp64 = k;
  if (status != IPR_OK && status != IPR_EDIVERGED && s.verify && verified_at != k) {
    double tau;
    if (int rc = sv.true_residual(&tau)) return rc;
    res.residual_true = tau;
  }
  return status;
}

}  // namespace

extern "C" {

void ipr_schedule_default(ipr_schedule* s) {
  if (!s) return;
  std::memset(s, 0, sizeof *s);
  s->init = IPR_INIT_IDENTITY;
  s->bulk_dtype = IPR_FP64;
  s->max_iter = 100;
  s->triangle = 1;
  s->guard_fallback = 1;
  s->verify = 1;
  s->bulk_switch = 0.05;
  s->stall_ratio = 0.5;
  s->poly[0] = 1.0;
}

const char* ipr_last_error(void) { return g_last_error.c_str(); }

size_t ipr_workspace_size(int n_max, int p_max, int batch, const ipr_schedule* s) {
  if (n_max < 1 || p_max < 1 || batch < 1) return 0;
  Work w;
  bool ok;
  const int dt = s ? s->bulk_dtype : IPR_FP64;
  const int sl = s ? emul_digits(*s) : 0;
  const bool store = s && s->store_format != IPR_STORE_NONE;
  const size_t single = carve(n_max, p_max, dt, sl, store, &w, nullptr, (size_t)-1, &ok) + 256;
  return std::max(single, batched_workspace_bytes(n_max, batch));
}

size_t ipr_lowdin_workspace(int n, const ipr_schedule* s) {
  if (n < 1) return 0;
  return std::max(ipr_workspace_size(n, 2, 1, s), (size_t)n * n * sizeof(double) + 256);
}

int ipr_lowdin(const double* dS, const double* dH, double* dX, double* dHout, int n, double tol,
               const ipr_schedule* s, ipr_result* out, void* dWork, size_t work_bytes,
               hipStream_t stream) {
  g_last_error.clear();
  if (!dS || !dH || !dX || !dHout || !dWork || n < 1)
    return fail(IPR_EARG, "ipr_lowdin: bad argument");
  if (dHout == dS || dHout == dH || dHout == dX || dX == dH)
    return fail(IPR_EARG, "ipr_lowdin: outputs must not alias the inputs or each other");
  if (work_bytes < ipr_lowdin_workspace(n, s))
    return fail(IPR_EARG, "ipr_lowdin: workspace too small (%zu bytes, need %zu)", work_bytes,
                ipr_lowdin_workspace(n, s));
  if (int rc = ipr_solve(dS, dX, n, 2, tol, s, out, dWork, work_bytes, stream)) return rc;
  // the solve is done with its workspace: its first n^2 doubles hold H X
  Carver c(dWork, work_bytes);
  double* T = c.take<double>((size_t)n * n);
  Epilogue e1;
  e1.D = T;
  HIP_TRY(gemm_f64(dH, dX, n, 0, e1, stream));     // (H^T X = H X, H symmetric)
  Epilogue e2;
  e2.D = dHout;
  HIP_TRY(gemm_f64(T, dX, n, 1, e2, stream));      // (H X)^T X = X H X: symmetric, one triangle
  return IPR_OK;
}

int ipr_norms(const double* dA, int n, double* out, void* dWork, size_t work_bytes,
              hipStream_t stream) {
  g_last_error.clear();
  if (!dA || !out || !dWork || n < 1) return fail(IPR_EARG, "ipr_norms: bad argument");
  Carver c(dWork, work_bytes);
  const size_t strips = (n + 255) / 256;
  double* scratch = c.take<double>(2 * (size_t)n + strips * n);
  double* res = c.take<double>(2);
  if (!c.ok())
    return fail(IPR_EARG, "ipr_norms: workspace too small (%zu < %zu)", work_bytes, c.used);
  HIP_TRY(norms_1_inf(dA, n, scratch, res, stream));
  return read_scalars(res, 2, out, stream);
}

int ipr_gemm(const double* dL, const double* dR, const double* dX, double* dD, int n,
             double alpha, double beta, double gamma, int triangle, hipStream_t stream) {
  g_last_error.clear();
  if (!dL || !dR || !dD || n < 1) return fail(IPR_EARG, "ipr_gemm: bad argument");
  if (dD == dL || dD == dR) return fail(IPR_EARG, "ipr_gemm: output aliases an operand");
  Epilogue e;
  e.alpha = alpha;
  e.beta = dX ? beta : 0.0;
  e.X = dX;
  e.gamma = gamma;
  e.D = dD;
  HIP_TRY(gemm_f64(dL, dR, n, triangle ? 1 : 0, e, stream));
  return IPR_OK;
}

int ipr_solve(const double* dA, double* dC, int n, int p, double tol, const ipr_schedule* sched,
              ipr_result* out, void* dWork, size_t work_bytes, hipStream_t stream) {
  g_last_error.clear();
  ipr_schedule sd;
  ipr_schedule_default(&sd);
  const ipr_schedule& s = sched ? *sched : sd;
  ipr_result res;
  std::memset(&res, 0, sizeof res);
  res.residual_true = std::numeric_limits<double>::quiet_NaN();
  if (!dA || !dC || !dWork) return fail(IPR_EARG, "ipr_solve: null pointer");
  if ((const void*)dA == (const void*)dC) return fail(IPR_EARG, "ipr_solve: dC must not alias dA");
  if (n < 1 || p < 1 || p > 64) return fail(IPR_EARG, "ipr_solve: need n >= 1 and 1 <= p <= 64");
  if (!(tol > 0.0)) return fail(IPR_EARG, "ipr_solve: tol must be > 0");
  if (s.max_iter < 0) return fail(IPR_EARG, "ipr_solve: max_iter < 0");
  if (s.init < IPR_INIT_IDENTITY || s.init > IPR_INIT_USER)
    return fail(IPR_EARG, "ipr_solve: unknown init %d", s.init);
  if (s.evaluation < IPR_EVAL_COUPLED || s.evaluation > IPR_EVAL_NEWTON_SCHULZ)
    return fail(IPR_EARG, "ipr_solve: unknown evaluation %d", s.evaluation);
  if (s.evaluation == IPR_EVAL_NEWTON_SCHULZ && p != 1)
    return fail(IPR_EARG, "ipr_solve: the Newton-Schulz order is the p = 1 case");
  if (s.evaluation != IPR_EVAL_COUPLED && s.bulk_dtype != IPR_FP64)
    return fail(IPR_EARG, "ipr_solve: the literal and Newton-Schulz orders run in FP64 only");
  if (s.bulk_dtype < IPR_FP64 || s.bulk_dtype > IPR_FP64_INT8_EMUL)
    return fail(IPR_EARG, "ipr_solve: unknown bulk dtype %d", s.bulk_dtype);
  const int slices = emul_digits(s);
  if (s.bulk_dtype == IPR_FP64_INT8_EMUL) {
    if (slices < 1 || slices > kMaxSlices)
      return fail(IPR_EARG, "ipr_solve: emul_slices must be in 1..%d", kMaxSlices);
    if (n > slice_max_n())
      return fail(IPR_EARG, "ipr_solve: int8-slice products need n <= %d", slice_max_n());
  }
  const bool store = s.store_format != IPR_STORE_NONE;
  if (s.store_format < IPR_STORE_NONE || s.store_format > IPR_STORE_FIXED)
    return fail(IPR_EARG, "ipr_solve: unknown store_format %d", s.store_format);
  if (store) {
    if (s.store_format == IPR_STORE_FLOAT && (s.store_bits < 1 || s.store_bits > 52))
      return fail(IPR_EARG, "ipr_solve: store_bits must be 1..52 stored mantissa bits");
    // (2^bits |x| must stay finite for every stored value)
    if (s.store_format == IPR_STORE_FIXED && (s.store_bits < 1 || s.store_bits > 64))
      return fail(IPR_EARG, "ipr_solve: store_bits must be 1..64 fractional bits");
    if (s.init != IPR_INIT_IDENTITY || s.evaluation != IPR_EVAL_COUPLED ||
        s.bulk_dtype != IPR_FP64 || s.scale_squarings || s.scale_lanczos ||
        s.dynamic_scaling)
      return fail(IPR_EARG, "ipr_solve: approximate storage runs the plain coupled iteration "
                  "from the scaled identity in FP64 (no squarings, no scaled steps)");
  }
  if (s.store_regime < 0 || s.store_regime > 1)
    return fail(IPR_EARG, "ipr_solve: unknown store_regime %d", s.store_regime);
  if (s.store_regime == 1 && !store)
    return fail(IPR_EARG, "ipr_solve: the all-arithmetic regime needs a store_format");
  if (s.hist_len < 0) return fail(IPR_EARG, "ipr_solve: hist_len < 0");
  if (s.scale_squarings > 0 && s.scale_lanczos)
    return fail(IPR_EARG, "ipr_solve: scale_squarings and scale_lanczos are two ways to the "
                "same scale: choose one");
  if (s.init == IPR_INIT_LEARNED && !s.mlp_params)
    return fail(IPR_EARG, "ipr_solve: the learned start needs schedule.mlp_params");

  Solver sv;
  bool ok;
  carve(n, p, s.bulk_dtype, slices, store, &sv.w, dWork, work_bytes, &ok);
  if (!ok)
    return fail(IPR_EARG, "ipr_solve: workspace too small (%zu bytes, need %zu)", work_bytes,
                ipr_workspace_size(n, p, 1, sched));
  sv.A = dA;
  sv.Atrue = dA;
  sv.n = n;
  sv.p = p;
  sv.tri = s.triangle ? 1 : 0;
  sv.st = stream;
  sv.prod.n = n;
  sv.prod.st = stream;
  sv.prod.w = &sv.w;
  sv.prod.timing = s.timing != 0;
  sv.prod.emul = slices;
  Work& w = sv.w;
  sv.Cb[0] = dC;
  sv.Cb[1] = w.m[0];
  sv.Mb[0] = w.m[1];
  sv.Mb[1] = w.m[2];
  sv.Nb[0] = w.m[3];
  sv.Nb[1] = w.m[4];
  sv.X[0] = p >= 2 ? w.m[5] : nullptr;
  sv.X[1] = p >= 3 ? w.m[6] : nullptr;
  sv.Rns = w.m[2];  // Newton-Schulz (p = 1) does not carry M
  const size_t nn = (size_t)n * n;
  Timer tm(stream, !g_no_alloc);

  // ---- norms of eq. (3)
  tm.mark(0);
  HIP_TRY(norms_1_inf(dA, n, w.norms_scratch, w.scal, stream));
  double nrm[2];
  if (int rc = read_scalars(w.scal, 2, nrm, stream)) return rc;
  res.norm1 = nrm[0];
  res.norminf = nrm[1];
  const double s2 = nrm[0] * nrm[1];
  const double sigma = std::sqrt(s2);
  tm.mark(1);
  if (!(s2 > 0.0) || !std::isfinite(s2))
    return fail(IPR_EARG, "ipr_solve: A has zero or non-finite norm");

  if (store && s.store_regime == 1) {
    const int status = solve_arith(sv, s, tol, sigma, res);
    if (status == IPR_EHIP || status == IPR_EARG) return status;
    tm.mark(4);
    if (sv.C() != dC) HIP_TRY(copy(sv.C(), nn, dC, stream));
    tm.mark(5);
    HIP_TRY(hipStreamSynchronize(stream));
    res.ms_norms = tm.ms(0, 1);
    res.ms_refine = tm.ms(1, 4);
    res.ms_verify = tm.ms(4, 5);
    res.status = status;
    res.gemms = sv.prod.gemms;
    sv.prod.totals(0, &res.gemm_launches, &res.ms_gemm, &res.gemm_flops);
    if (out) *out = res;
    return status;
  }

  // ---- start C_0 = sc^{-1/p} q(A / sc), q(x) = b0 + b1 x + b2 x^2, with the
  // spectrum of A / sc inside (0, 1]; then M_0 = C_0^p A and N_0.
  double b[3] = {1.0, 0.0, 0.0};
  double sc = sigma;            // ||A||_2 <= sqrt(||A||_1 ||A||_inf)
  double lz_lo = 0.0;           // lambda_min estimate of a Lanczos run made for the scale
  const double* G = nullptr;    // A^2 when the learned start computed it
  int init = s.init;
  if (init == IPR_INIT_POLY) {
    for (int i = 0; i < 3; ++i) b[i] = s.poly[i];
  } else if (init == IPR_INIT_PAPER_EQ3) {
    // A / sigma^2 = sigma^{-1/p} q(A / sigma) with q(x) = sigma^{1/p - 1} x
    b[0] = 0.0;
    b[1] = std::pow(sigma, 1.0 / p - 1.0);
  } else if (init == IPR_INIT_IDENTITY && s.scale_squarings > 0) {
    // A tighter scale from repeated squaring: lambda_max(A)^(2^k) =
    // lambda_max(A^(2^k)) <= sqrt(||A^(2^k)||_1 ||A^(2^k)||_inf), a bound that
    // falls towards lambda_max as k grows. Each squaring is one triangle
    // product of S_k = (A / sigma)^(2^k) (||S_k|| <= 1: no overflow). It stops
    // once the next squaring is predicted to gain less than one product's
    // worth (squaring_worth). The
    // 1% margin covers rounding in S_k; a start with lambda_max / s in (1, 2)
    // would still satisfy eq. (2).
    const double worth = squaring_worth(p, s.dynamic_scaling != 0);
    double* Sb[2] = {sv.Mb[1], sv.Nb[1]};  // free until the first iteration
    const double* src = dA;
    double best = sigma, prev = sigma;
    for (int k = 1; k <= s.scale_squarings; ++k) {
      Epilogue e;
      e.alpha = k == 1 ? 1.0 / s2 : 1.0;  // (A / sigma)^2 = A A / sigma^2
      e.D = Sb[(k - 1) & 1];
      HIP_TRY(sv.prod.f64(src, src, 1, e));
      HIP_TRY(norms_1_inf(e.D, n, w.norms_scratch, w.scal + 2, stream));
      double g[2];
      if (int rc = read_scalars(w.scal + 2, 2, g, stream)) return rc;
      const double bk = sigma * std::pow(g[0] * g[1], 1.0 / std::ldexp(1.0, k + 1)) * 1.01;
      if (!(bk > 0.0) || !std::isfinite(bk)) break;
      best = std::min(best, bk);
      if (std::sqrt(prev / bk) < worth) break;  // the next squaring would not pay
      prev = bk;
      src = e.D;
    }
    sc = best;
    res.init_scale = sc;
  } else if (init == IPR_INIT_IDENTITY && s.scale_lanczos && n >= 32) {
    // The scale from the largest Ritz value of the Lanczos run on A that the
    // scaled steps take their lower end from (so it runs once, here): a Ritz
    // value lies inside the spectrum, and the largest one approaches
    // lambda_max from below within a fraction of a percent after 24 steps on
    // spectra that are dense near their top; the 1% margin puts s at or above
    // lambda_max in practice. No product is spent. It is not a certified
    // bound: eq. (2) holds while lambda_max / s < 2, the scaled steps keep
    // mu lambda_max / s below p + 1 unless s is off by more than 15%, and a
    // run that diverges restarts from the norm-scaled identity.
    double lo = 0.0, hi = 0.0;
    if (int rc = sv.lanczos_range(dA, std::min(24, n - 8), w.m[0], &lo, &hi)) return rc;
    if (hi > 0.0 && std::isfinite(hi)) sc = std::min(sigma, 1.01 * hi);
    if (lo > 0.0 && std::isfinite(lo)) lz_lo = lo;
    res.init_scale = sc;
  } else if (init == IPR_INIT_LEARNED) {
    // Certified scale: lambda_max(A)^2 = lambda_max(A^2) <= sqrt(||A^2||_1 ||A^2||_inf),
    // one triangle product; then the network's polynomial in units of that bound.
    double* Gm = sv.Mb[1];  // free until the first iteration
    Epilogue e;
    e.D = Gm;
    HIP_TRY(sv.prod.f64(dA, dA, 1, e));
    HIP_TRY(norms_1_inf(Gm, n, w.norms_scratch, w.scal + 2, stream));
    float* feat = reinterpret_cast<float*>(w.scal + 16);   // 16 floats
    float* yout = reinterpret_cast<float*>(w.scal + 24);   // 3 floats
    // w.partial holds max(n, tile count) doubles, more than the features need
    if ((size_t)features_one_part(n) > std::max<size_t>(n, 1))
      return fail(IPR_EARG, "ipr_solve: feature scratch too small");
    HIP_TRY(features_one(dA, n, p, w.scal, w.partial, feat, stream));
    HIP_TRY(mlp_forward(s.mlp_params, feat, 1, yout, nullptr, nullptr, stream));
    double hs[32];
    if (int rc = read_scalars(w.scal, 32, hs, stream)) return rc;
    float y[3];
    std::memcpy(y, &hs[24], sizeof y);
    // rounding of the computed A^2 is below n u relative; keep a margin of 8 n u
    const double bound = std::sqrt(std::sqrt(hs[2] * hs[3])) *
                         (1.0 + 8.0 * n * std::numeric_limits<double>::epsilon());
    if (std::isfinite(bound) && bound > 0.0) sc = std::min(sigma, bound);
    G = Gm;
    b[0] = std::exp((double)y[0]);
    b[1] = (double)y[1];
    b[2] = (double)y[2];
    if (!std::isfinite(b[0]) || !std::isfinite(b[1]) || !std::isfinite(b[2])) b[0] = -1.0;
    // polynomial terms cost p products: use them only when the network asks
    // for them (beyond 5% of b0)
    if (std::fabs(b[1]) < 0.05 * b[0] && std::fabs(b[2]) < 0.05 * b[0]) b[1] = b[2] = 0.0;
    res.init_scale = sc;
  }
  double sup_phi;
  int q_pos;
  poly_guard(b, p, &sup_phi, &q_pos);
  if (init == IPR_INIT_LEARNED && q_pos && std::isfinite(sup_phi) && sup_phi >= 2.0) {
    // A prediction beyond eq. (2): q -> t q scales q^p x by t^p, so t with
    // t^p sup = 1.98 brings it back inside (q > 0 is unchanged).
    const double t = std::pow(1.98 / sup_phi, 1.0 / p);
    for (double& v : b) v *= t;
    poly_guard(b, p, &sup_phi, &q_pos);
  }
  if (!(q_pos && sup_phi < 2.0)) {
    if (!s.guard_fallback)
      return fail(IPR_EGUARD, "ipr_solve: start violates eq. (2) (sup q^p x = %g)", sup_phi);
    res.fallback_used = 1;
    // the scaled identity at the same scale (sigma, or the learned start's
    // tighter bound on lambda_max) satisfies eq. (2)
    if (init != IPR_INIT_LEARNED) sc = sigma;
    init = IPR_INIT_IDENTITY;
    b[0] = 1.0;
    b[1] = b[2] = 0.0;
    poly_guard(b, p, &sup_phi, &q_pos);
  }
  res.init_bound = sup_phi;
  for (int i = 0; i < 3; ++i) res.poly_used[i] = b[i];
  if (res.init_scale == 0.0) res.init_scale = sc;

  // Dynamically scaled iteration: bounds [mod_a, mod_b] on the spectrum of
  // M_k are carried through the scalar map of a step; each step k multiplies
  // M_k by mu_k >= 1 (C_k by mu_k^{1/p}), chosen to lift the lower end. With
  // the start C_0 = sc^{-1/p} q(A / sc) (the scaled identity: q = 1) the
  // eigenvalues of M_0 are phi(x) = q(x)^p x at x = lambda / sc in (0, 1]:
  // the upper end is sup phi on (0, 1] (certified; with scale_lanczos, where
  // sc is an estimate, held there all the same), the lower end the least
  // phi on [theta / sc, 1], theta a Lanczos estimate of lambda_min (from
  // above: an overestimate only makes the factors smaller). mu_k mod_b < 2
  // keeps every step inside eq. (2). Once the residual is below 1 it bounds
  // both ends, and from a lower end of 1/2 on the steps are unscaled. mu_0
  // is folded into the start (q -> mu_0^{1/p} q).
  bool dyn = s.dynamic_scaling &&
             (init == IPR_INIT_IDENTITY || init == IPR_INIT_LEARNED || init == IPR_INIT_POLY) &&
             (s.bulk_dtype == IPR_FP64 || s.bulk_dtype == IPR_FP64_INT8_EMUL) &&
             s.evaluation == IPR_EVAL_COUPLED && n >= 32;
  double mod_a = 0.0, mod_b = 1.0, mu_k = 1.0;
  if (dyn) {
    double theta = lz_lo;
    if (!(theta > 0.0))
      if (int rc = sv.lanczos_min(std::min(24, n - 8), w.m[0], &theta)) return rc;
    res.lmin_est = theta;
    dyn = theta > 0.0 && std::isfinite(theta) && std::isfinite(sup_phi) && sup_phi > 0.0;
    if (dyn) {
      const double lo = poly_min(b, p, std::min(theta / sc, 1.0));
      dyn = lo > 0.0;
      if (dyn) {
        const double mu0 = choose_mu(lo, sup_phi, p);
        const double t = std::pow(mu0, 1.0 / p);
        for (double& v : b) v *= t;
        mod_a = lo * mu0;
        mod_b = sup_phi * mu0;
        res.init_bound = mod_b;  // sup of C_0^p lambda over the spectrum bound
        for (int i = 0; i < 3; ++i) res.poly_used[i] = b[i];
      }
    }
  }

  const double root = std::pow(sc, -1.0 / p);
  if (init == IPR_INIT_USER) {
    // C_0 is the caller's, already in dC (= C buffer 0); its residual below
  } else if (b[1] == 0.0 && b[2] == 0.0) {
    // scaled identity c I, c = b0 sc^{-1/p}: M_0 = c^p A elementwise
    const double c = b[0] * root;
    if (store) {
      // approximate storage (Sections III-C, IV): the iteration works on A
      // as stored, and C_0, M_0, N_0 are stored the same way
      HIP_TRY(copy(dA, nn, w.Ar, stream));
      HIP_TRY(round_matrix(w.Ar, nn, s.store_format, s.store_bits, stream));
      sv.A = w.Ar;
    }
    HIP_TRY(init_identity(sv.A, n, p, c, std::pow(b[0], (double)p) / sc, sv.C(), sv.M(),
                          sv.Nb[sv.ni], w.partial, stream));
    if (store) {
      for (double* X : {sv.C(), sv.M(), sv.Nb[sv.ni]})
        HIP_TRY(round_matrix(X, nn, s.store_format, s.store_bits, stream));
      sv.prod.rfmt = s.store_format;
      sv.prod.rbits = s.store_bits;
    }
    sv.slots = n;
    if (int rc = sv.reduce()) return rc;
  } else {
    if (b[2] != 0.0 && !G) {
      Epilogue e;  // C_0 from one product A A
      e.alpha = root * b[2] / (sc * sc);
      e.beta = root * b[1] / sc;
      e.X = dA;
      e.gamma = root * b[0];
      e.D = sv.C();
      HIP_TRY(sv.prod(dA, dA, sv.tri, e));
      if (!sv.tri) HIP_TRY(symmetrize(sv.C(), n, stream));
    } else {
      HIP_TRY(lincomb(dA, G, n, root * b[0], root * b[1] / sc, root * b[2] / (sc * sc), sv.C(),
                      stream));
    }
    // M_0 = C_0^p A: products of polynomials in A, symmetric
    if (s.evaluation == IPR_EVAL_COUPLED)
      if (int rc = sv.power_chain(sv.C(), dA, sv.M(), sv.Nb[sv.ni], sv.tri)) return rc;
  }
  tm.mark(2);

  // ---- iterations: optional low-precision bulk phase, then FP64
  // (int8-slice products are FP64-accurate: no low-precision phase)
  // A bf16 / fp16 / fp8 phase for p >= 2 would end in the FP64 restart (its
  // error does not commute with A): skipped unless forced.
  const bool lp_dtype = s.bulk_dtype != IPR_FP64 && s.bulk_dtype != IPR_FP64_INT8_EMUL;
  const bool lowp = lp_dtype && (p == 1 || s.bulk_force);
  res.bulk_skipped = lp_dtype && !lowp ? 1 : 0;
  bool lp_restart = false;
  int status = IPR_EMAXITER;
  int k = 0, kb = 0;
  double rho = 0.0;
  auto restart_identity = [&]() -> int {
    res.fallback_used = 1;
    sv.mu_cur = sv.mu_next = 1.0;
    sv.ci = sv.mi = sv.ni = 0;
    HIP_TRY(init_identity(dA, n, p, std::pow(s2, -1.0 / (2.0 * p)), 1.0 / sigma, sv.C(),
                          sv.M(), sv.Nb[sv.ni], w.partial, stream));
    sv.slots = n;
    return sv.reduce();
  };
  const bool literal = s.evaluation == IPR_EVAL_LITERAL;
  const bool ns_order = s.evaluation == IPR_EVAL_NEWTON_SCHULZ;
  // Residual of the start for the chosen order: R_0 = I - A C_0 (Newton-Schulz),
  // M_0 = C_0^p A for a caller's start (coupled; the other starts built M_0),
  // X_0 = C_0^p A (literal).
  auto start_residual = [&]() -> int {
    if (ns_order) return sv.recompute(true);
    if (literal) return sv.literal_x();
    if (init == IPR_INIT_USER) return sv.power_chain(sv.C(), dA, sv.M(), sv.Nb[sv.ni], sv.tri);
    return IPR_OK;
  };
  if (int rc = start_residual()) return rc;
  if (init == IPR_INIT_USER) {
    // Eq. (2) for the caller's start. ||I - R||_F < 1 (R = C_0^p A, or A C_0
    // in Newton-Schulz order) bounds the spectrum inside (0, 2) outright.
    // Otherwise, for the coupled and literal orders, a Lanczos estimate of
    // the extreme eigenvalues of the symmetric C_0^p A must lie in (0, 1.9)
    // (an estimate from inside the spectrum, hence the margin).
    double r0;
    if (int rc = read_scalars(sv.rho_dev(), 1, &r0, stream)) return rc;
    bool ok = r0 < 1.0;
    double lo = 1.0 - r0, hi = 1.0 + r0;
    if (!ok && !ns_order && std::isfinite(r0) && n >= 16) {  // (the Lanczos basis fits w.m[0])
      const double* M0 = literal ? sv.Nb[1] : sv.M();
      if (int rc = sv.lanczos_range(M0, std::max(1, std::min(24, n - 8)), w.m[0], &lo, &hi))
        return rc;
      ok = lo > 0.0 && hi < 1.9;
    }
    res.init_bound = hi;
    res.init_scale = 0.0;
    for (double& v : res.poly_used) v = 0.0;
    if (!ok) {
      if (!s.guard_fallback)
        return fail(IPR_EGUARD, "ipr_solve: the caller's start has residual %g >= 1", r0);
      init = IPR_INIT_IDENTITY;
      if (int rc = restart_identity()) return rc;
      res.init_bound = 1.0;
      res.init_scale = sigma;
      res.poly_used[0] = 1.0;
      if (ns_order || literal)
        if (int rc = start_residual()) return rc;
    }
  }
  if (literal) {
    // Eq. (1) as printed. X_k = C_k^p A is formed from C_k and A, so its
    // residual is the true one and no separate check is needed.
    double best = std::numeric_limits<double>::infinity();
    int stale = 0;
    tm.mark(3);
    for (k = 0;; ++k) {
      if (int rc = read_scalars(sv.rho_dev(), 1, &rho, stream)) return rc;
      res.residual_proxy = rho;
      res.residual_true = rho;
      if (!std::isfinite(rho) || rho > 1e6) {
        status = IPR_EDIVERGED;
        break;
      }
      if (rho < tol) {
        status = IPR_OK;
        break;
      }
      if (rho < kFloorZone) {
        if (rho < s.stall_ratio * best) {
          best = rho;
          stale = 0;
        } else if (++stale >= 3) {
          status = IPR_EFLOOR;
          break;
        }
      }
      if (k >= s.max_iter) break;
      if (int rc = sv.literal_update()) return rc;
      if (int rc = sv.literal_x()) return rc;
    }
    tm.mark(4);
    res.iters_fp64 = k;
    if (sv.C() != dC) HIP_TRY(copy(sv.C(), nn, dC, stream));
    tm.mark(5);
    HIP_TRY(hipStreamSynchronize(stream));
    res.ms_norms = tm.ms(0, 1);
    res.ms_init = tm.ms(1, 2);
    res.ms_refine = tm.ms(3, 4);
    res.ms_verify = tm.ms(4, 5);
    res.status = status;
    res.gemms = sv.prod.gemms;
    sv.prod.totals(0, &res.gemm_launches, &res.ms_gemm, &res.gemm_flops);
    if (out) *out = res;
    return status;
  }
  if (lowp) {
    // Scaled steps in a p = 1 bulk phase: Newton-Schulz steps on mu_k C_k,
    // mu_k from bounds [ba, bb] on the spectrum of A C_k by the FP64 rules
    // (the lower end from the Lanczos estimate of lambda_min, the top from
    // the scale; both narrowed by the residual once it is below 1). The factor
    // costs no product (it enters the update's epilogue).
    bool bulk_dyn = s.dynamic_scaling && p == 1 && init == IPR_INIT_IDENTITY && n >= 32 &&
                    s.evaluation == IPR_EVAL_COUPLED;
    double ba = 0.0, bb = 1.0;
    if (bulk_dyn) {
      double theta = lz_lo;
      if (!(theta > 0.0))
        if (int rc = sv.lanczos_min(std::min(24, n - 8), w.m[0], &theta)) return rc;
      res.lmin_est = theta;
      ba = std::min(theta / sc, 1.0);
      bb = sup_phi;
      bulk_dyn = ba > 0.0 && std::isfinite(ba) && std::isfinite(bb) && bb > 0.0;
    }
    sv.prod.lowp_dtype = s.bulk_dtype;
    if (p == 1)  // Newton-Schulz bulk: R_0 = I - A C_0
      if (int rc = sv.recompute(true)) return rc;
    double best = std::numeric_limits<double>::infinity(), top = best;
    int stale = 0, flat = 0;
    for (kb = 0; kb < s.max_iter; ++kb) {
      if (int rc = read_scalars(sv.rho_dev(), 1, &rho, stream)) return rc;
      if (!std::isfinite(rho) || rho > 1e6) break;
      if (rho < s.bulk_switch) break;
      if (bulk_dyn) {
        if (rho < 1.0) {
          ba = std::max(ba, 1.0 - rho);
          bb = std::min(bb, 1.0 + rho);
        }
        sv.ns_mu = choose_mu(ba, bb, 1);
        double na, nb;
        step_bounds(ba, bb, sv.ns_mu, 1, &na, &nb);
        ba = na;
        bb = nb;
      }
      if (rho < 1.0) {
        if (rho < s.stall_ratio * best) {
          best = rho;
          stale = 0;
        } else if (++stale >= 2) {
          break;
        }
      } else if (rho < top) {  // above 1 the residual must still fall every step
        top = rho;
        flat = 0;
      } else if (++flat >= 2) {
        break;
      }
      if (int rc = sv.step(p == 1)) return rc;
    }
    sv.prod.lowp_dtype = 0;
    sv.ns_mu = 1.0;
    res.iters_bulk = kb;
    if (!std::isfinite(rho) || rho > 1e6) {
      // the low-precision phase diverged: start again in FP64 from the scaled identity
      lp_restart = true;
      if (int rc = restart_identity()) return rc;
    } else {
      if (int rc = sv.recompute(p == 1)) return rc;
    }
  }
  tm.mark(3);
  // Newton-Schulz order for p = 1 once a low-precision phase has run, or on request
  bool ns = (lowp && p == 1 && !lp_restart) || ns_order;
  double best = std::numeric_limits<double>::infinity();
  int stale = 0, failed_verify = 0, verified_at = -1;
  bool short_failed = false, reestimated = false, div_restart = false;
  double last_tau = std::numeric_limits<double>::infinity();
  double prev = std::numeric_limits<double>::infinity();
  const int kmax = s.max_iter - res.iters_bulk;
  for (k = 0;; ++k) {
    if (int rc = read_scalars(sv.rho_dev(), 1, &rho, stream)) return rc;
    res.residual_proxy = rho;
    if (int rc = sv.record_hist(s, k, rho)) return rc;
    const bool bad = !std::isfinite(rho) || rho > 1e6;
    if (dyn && rho < 1.0) {  // ||I - M_k||_2 <= rho bounds the spectrum of M_k
      mod_a = std::max(mod_a, 1.0 - rho);
      mod_b = std::min(mod_b, 1.0 + rho);
    }
    // From a start that commutes with A the residual of the coupled form falls
    // every step until the rounding floor. After a low-precision phase the
    // iterate carries rounding errors that do not commute with A; for p >= 2
    // the FP64 steps amplify them, and a growing residual is the sign. Then
    // (once) start again in FP64 from the scaled identity.
    const bool rising = rho > 1.1 * prev && rho > 1e-6;
    prev = rho;
    bool floor = false;  // stagnation above tol (see below)
    if (!bad && rho < tol && !ns && s.verify) {
      double tau;
      if (int rc = sv.true_residual(&tau)) return rc;
      res.residual_true = tau;
      verified_at = k;
      if (tau < tol) {
        status = IPR_OK;
        break;
      }
      floor = ++failed_verify >= 2 && !(tau < 0.5 * last_tau);
      last_tau = tau;
    }
    if (!bad && rho < kFloorZone) {
      if (rho < s.stall_ratio * best) {
        best = rho;
        stale = 0;
      } else if (++stale >= 3) {
        floor = true;
      }
    }
    // (a bulk result whose FP64 residual is not below 1 is no start either)
    if (lowp && !lp_restart && (bad || rising || floor || (k == 0 && !(rho < 1.0)))) {
      lp_restart = true;
      ns = false;
      if (int rc = restart_identity()) return rc;
      best = last_tau = prev = std::numeric_limits<double>::infinity();
      stale = failed_verify = 0;
      verified_at = -1;
      --k;  // no step was taken
      continue;
    }
    if (bad && !lp_restart && !div_restart && !store) {
      // Divergence (an eq. (3) start outside eq. (2)'s region that the guard
      // let through, a caller's start, rounding): one restart from the scaled
      // identity at the norm bound, with plain steps. A second divergence
      // (e.g. an indefinite A) is reported.
      div_restart = true;
      dyn = false;
      ns = ns_order;
      if (int rc = restart_identity()) return rc;
      if (ns_order)
        if (int rc = sv.recompute(true)) return rc;
      best = last_tau = prev = std::numeric_limits<double>::infinity();
      stale = failed_verify = 0;
      verified_at = -1;
      short_failed = false;
      --k;  // no step was taken
      continue;
    }
    if (bad) {
      status = IPR_EDIVERGED;
      break;
    }
    if (rho < tol && (ns || !s.verify)) {
      if (ns) res.residual_true = rho;  // R_k = I - A C_k is the true residual
      status = IPR_OK;
      break;
    }
    if (floor) {
      status = IPR_EFLOOR;
      break;
    }
    if (k >= kmax) break;
    if (dyn && !reestimated && k >= 1 && mod_a >= kReestimateAt) {
      // Lanczos on A converges slowly to lambda_min when the small
      // eigenvalues are dense (an overestimate by 7x at kappa = 1e4 after 24
      // steps), and then every factor is smaller than it could be. Once the
      // scaled steps have lifted the lower end of M_k to kReestimateAt, M_k is
      // well conditioned and the same number of steps on it estimates its
      // lower end closely; the bound is replaced by that estimate, once.
      double th, hi;
      if (int rc = sv.lanczos_range(sv.M(), std::min(24, n - 8), sv.Cb[sv.ci ^ 1], &th, &hi))
        return rc;
      reestimated = true;
      if (th > 0.0 && std::isfinite(th)) {
        mod_a = std::min(th, mod_b);
        res.reest_iter = k;
        res.lmin_reest = th;
      }
    }
    if (dyn) {
      double na, nb;
      step_bounds(mod_a, mod_b, mu_k, p, &na, &nb);
      const double mu_n = choose_mu(na, nb, p);
      sv.mu_cur = mu_k;
      sv.mu_next = mu_n;
      mod_a = na;
      mod_b = nb;
      mu_k = mu_n;
    }
    // Last step: with unscaled steps each eigenvalue error e of M becomes at
    // most (p + 1) / (2p) e^2, so ||I - M_{k+1}||_F <= (p + 1) / (2p) rho^2.
    // When that bound is below tol, the p products of the M update would only
    // feed the convergence test, and the check of the true residual that
    // follows it anyway replaces that test. If the check fails (rounding
    // floor), M is recomputed from C_{k+1} and the iteration goes on.
    const bool clean = !ns && (!lowp || lp_restart) && !store;
    if (clean && s.verify && !short_failed && sv.mu_cur == 1.0 && rho < 0.5 &&
        (p + 1.0) / (2.0 * p) * rho * rho < tol && k < kmax) {
      if (int rc = sv.step(false, false)) return rc;
      ++k;
      if (int rc = sv.record_hist(s, k, std::numeric_limits<double>::quiet_NaN())) return rc;
      double tau;
      if (int rc = sv.true_residual(&tau)) return rc;
      res.residual_true = tau;
      verified_at = k;
      if (tau < tol) {
        status = IPR_OK;
        break;
      }
      ++failed_verify;
      last_tau = tau;
      short_failed = true;  // at the rounding floor: no second shortcut
      if (int rc = sv.recompute(false)) return rc;
      prev = std::numeric_limits<double>::infinity();
      --k;  // the loop's increment follows; the step above is counted
      continue;
    }
    if (int rc = sv.step(ns)) return rc;
  }
  tm.mark(4);
  res.iters_fp64 = k;
  if (ns && status != IPR_EDIVERGED) {
    res.residual_true = rho;  // of the returned iterate
  } else if (status != IPR_OK && s.verify && status != IPR_EDIVERGED && verified_at != k) {
    double tau;
    if (int rc = sv.true_residual(&tau)) return rc;
    res.residual_true = tau;
  }
  if (sv.C() != dC) HIP_TRY(copy(sv.C(), nn, dC, stream));
  tm.mark(5);
  HIP_TRY(hipStreamSynchronize(stream));
  res.ms_norms = tm.ms(0, 1);
  res.ms_init = tm.ms(1, 2);
  res.ms_bulk = tm.ms(2, 3);
  res.ms_refine = tm.ms(3, 4);
  res.ms_verify = tm.ms(4, 5);
  res.status = status;
  res.gemms = sv.prod.gemms;
  sv.prod.totals(0, &res.gemm_launches, &res.ms_gemm, &res.gemm_flops);
  sv.prod.totals(1, &res.lp_gemm_launches, &res.ms_lp_gemm, &res.lp_gemm_flops);
  if (out) *out = res;
  return status;
}

}  // extern "C"
