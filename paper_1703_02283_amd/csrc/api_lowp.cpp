// C ABI of the low-precision product (ipr_gemm_lowp).
#include <hip/hip_runtime.h>

#include "../../include/ipr.h"
#include "ipr_host.h"
#include "lowp.h"

using namespace ipr;

namespace {
struct LpWork {
  void* lq;
  void* rq;
  int* el;
  int* er;
};
size_t lp_work(int n, int dtype, LpWork* w, void* base, size_t cap, bool* ok) {
  Carver c(base, cap);
  w->lq = c.take<uint8_t>(lp_bytes(n, dtype));
  w->rq = c.take<uint8_t>(lp_bytes(n, dtype));
  w->el = c.take<int>(lp_exp_count(n));
  w->er = c.take<int>(lp_exp_count(n));
  *ok = c.ok();
  return c.used;
}
struct EmulWork {
  void* lq;
  void* rq;
  int* el;
  int* er;
  unsigned long long* cm;
  double* P;
  double* S;
};
size_t emul_work(int n, int s, EmulWork* w, void* base, size_t cap, bool* ok) {
  Carver c(base, cap);
  w->lq = c.take<uint8_t>((size_t)s * slice_bytes(n));
  w->rq = c.take<uint8_t>((size_t)s * slice_bytes(n));
  w->el = c.take<int>(lp_padded(n));
  w->er = c.take<int>(lp_padded(n));
  w->cm = c.take<unsigned long long>(n);
  w->P = c.take<double>((size_t)n * n);
  w->S = c.take<double>((size_t)n * n);
  *ok = c.ok();
  return c.used;
}
}  // namespace

extern "C" {

size_t ipr_gemm_lowp_workspace(int n) {
  if (n < 1) return 0;
  LpWork w;
  bool ok;
  return lp_work(n, LP_FP16, &w, nullptr, (size_t)-1, &ok) + 256;
}

int ipr_gemm_lowp(const double* dL, const double* dR, double* dD, int n, int dtype, int triangle,
                  void* dWork, size_t work_bytes, hipStream_t stream) {
  g_last_error.clear();
  if (!dL || !dR || !dD || !dWork || n < 1) return fail(IPR_EARG, "ipr_gemm_lowp: bad argument");
  if (dtype != IPR_BF16 && dtype != IPR_FP16 && dtype != IPR_FP8_E4M3)
    return fail(IPR_EARG, "ipr_gemm_lowp: dtype must be BF16, FP16 or FP8_E4M3");
  if (dD == dL || dD == dR) return fail(IPR_EARG, "ipr_gemm_lowp: output aliases an operand");
  LpWork w;
  bool ok;
  lp_work(n, dtype, &w, dWork, work_bytes, &ok);
  if (!ok) return fail(IPR_EARG, "ipr_gemm_lowp: workspace too small");
  HIP_TRY(quantize_t(dL, n, dtype, w.lq, w.el, stream));
  HIP_TRY(quantize_t(dR, n, dtype, w.rq, w.er, stream));
  Epilogue e;
  e.D = dD;
  HIP_TRY(gemm_lp(w.lq, w.el, w.rq, w.er, n, dtype, triangle ? 1 : 0, e, stream));
  return IPR_OK;
}

size_t ipr_gemm_emul_workspace(int n, int slices) {
  if (n < 1 || slices < 1 || slices > kMaxSlices) return 0;
  EmulWork w;
  bool ok;
  return emul_work(n, slices, &w, nullptr, (size_t)-1, &ok) + 256;
}

int ipr_gemm_emul(const double* dL, const double* dR, double* dD, int n, int slices, int triangle,
                  void* dWork, size_t work_bytes, hipStream_t stream) {
  g_last_error.clear();
  if (!dL || !dR || !dD || !dWork || n < 1) return fail(IPR_EARG, "ipr_gemm_emul: bad argument");
  if (slices < 1 || slices > kMaxSlices)
    return fail(IPR_EARG, "ipr_gemm_emul: slices must be in 1..%d", kMaxSlices);
  if (n > slice_max_n())
    return fail(IPR_EARG, "ipr_gemm_emul: n = %d exceeds %d, the largest order whose digit "
                "products fit an int32 accumulation", n, slice_max_n());
  if (dD == dL || dD == dR) return fail(IPR_EARG, "ipr_gemm_emul: output aliases an operand");
  EmulWork w;
  bool ok;
  emul_work(n, slices, &w, dWork, work_bytes, &ok);
  if (!ok) return fail(IPR_EARG, "ipr_gemm_emul: workspace too small");
  HIP_TRY(slices_split(dL, n, slices, w.lq, w.el, w.cm, stream));
  HIP_TRY(slices_split(dR, n, slices, w.rq, w.er, w.cm, stream));
  Epilogue e;
  e.D = dD;
  HIP_TRY(gemm_slices(w.lq, w.el, w.rq, w.er, n, slices, w.P, w.S, triangle ? 1 : 0, e, stream));
  return IPR_OK;
}

}  // extern "C"
