// Host-side helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace ipr {

extern thread_local std::string g_last_error;
int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return ::ipr::fail(IPR_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Copies `count` device doubles to host through a pinned buffer and waits.
int read_scalars(const double* d, int count, double* host, hipStream_t stream);

// Set while the allocation-free entry point runs on this thread: scalars are
// read without the pinned buffer and no events are created.
extern thread_local bool g_no_alloc;

// For q(x) = b0 + b1 x + b2 x^2: *sup_phi = sup_{x in (0,1]} q(x)^p x and
// *q_pos = 1 when q > 0 on all of (0, 1].
void poly_guard(const double b[3], int p, double* sup_phi, int* q_pos);

// Workspace of ipr_solve_batched for `batch` matrices with sum n_i^2 <= n_max^2.
size_t batched_workspace_bytes(int n_max, int batch);

// Carves 256-byte aligned pieces out of a workspace.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* b, size_t c) : base((char*)b), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~(size_t)255;
    used = off + count * sizeof(T);
    return base ? (T*)(base + off) : nullptr;
  }
  bool ok() const { return used <= cap; }
};

}  // namespace ipr
