// C ABI of the batched solver: validation, the order in which workgroups
// take the matrices (largest estimated work first), the persistent launch
// captured in a HIP graph (replayed when the same call repeats), results,
// and the tile-edge autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/ipr.h"
#include "batched.h"
#include "ipr_host.h"

using namespace ipr;

namespace {

constexpr int kBucketMax[IPR_BATCH_BUCKETS] = {48, 96, 192, 384, 768, 1024};
std::mutex g_mu;
int g_tiles[IPR_BATCH_BUCKETS] = {32, 64, 64, 64, 64, 64};

int bucket_of(int n) {
  for (int b = 0; b < IPR_BATCH_BUCKETS; ++b)
    if (n <= kBucketMax[b]) return b;
  return IPR_BATCH_BUCKETS - 1;
}

bool valid_tile(int t) { return t == 32 || t == 64; }

int grid_size(int batch) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return std::max(1, std::min(batch, kBatchWgPerCu * cus));  // all resident at once
}

struct Layout {
  double* scratch;
  BatchItem* items;
  int* order;
  int* next;
  BatchResult* results;
};

size_t layout(int batch, int grid, size_t scratch_elems, void* base, size_t cap, Layout* L,
              bool* ok) {
  Carver c(base, cap);
  L->scratch = c.take<double>(scratch_elems);
  L->items = c.take<BatchItem>(batch);
  L->order = c.take<int>(batch);
  L->next = c.take<int>(1);
  L->results = c.take<BatchResult>(batch);
  *ok = c.ok();
  return c.used;
}

// Items by decreasing estimated work: n^3 times the products of one update
// (p + 1, or log2 p + 2 by binary powering for powers of two from 4). The
// workgroups take them in this order as they become free.
std::vector<int> work_order(const std::vector<BatchItem>& items) {
  std::vector<int> idx(items.size());
  std::iota(idx.begin(), idx.end(), 0);
  auto cost = [&](int i) {
    const double n = items[i].n;
    const int p = items[i].p;
    const bool binary = p >= 4 && (p & (p - 1)) == 0;
    int lg = 0;
    while ((1 << (lg + 1)) <= p) ++lg;
    return n * n * n * (binary ? lg + 2 : p + 1);
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost(a) > cost(b); });
  return idx;
}

// One cached executable graph of the persistent launch, keyed by its arguments.
struct GraphCache {
  bool valid = false;
  BatchArgs args;
  int grid = 0;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
};
thread_local GraphCache g_graph;

bool same(const BatchArgs& a, const BatchArgs& b) { return std::memcmp(&a, &b, sizeof a) == 0; }

int launch_graph(const BatchArgs& args, int grid, hipStream_t stream) {
  GraphCache& g = g_graph;
  if (!(g.valid && g.grid == grid && g.stream == stream && same(g.args, args))) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = GraphCache();
    // Capture on a stream of the library's own (the caller's may be the null
    // stream, which cannot be captured); the graph is launched on the caller's.
    thread_local hipStream_t cap = nullptr;
    if (!cap) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = batched_launch(args, grid, cap);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cap, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(IPR_EHIP, "batched launch failed during capture: %s", hipGetErrorString(le));
    }
    HIP_TRY(ce);
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    g.valid = true;
    g.args = args;
    g.grid = grid;
    g.stream = stream;
    g.exec = exec;
    g.graph = graph;
  }
  HIP_TRY(hipGraphLaunch(g.exec, stream));
  return IPR_OK;
}

int run_batch(const double* dA, double* dC, const std::vector<BatchItem>& items, double tol,
              const ipr_schedule& s, void* dWork, size_t work_bytes, std::vector<BatchResult>* res,
              hipStream_t stream, bool use_graph) {
  const int batch = (int)items.size();
  const int grid = grid_size(batch);
  size_t scratch = 0;
  for (const auto& it : items)
    scratch = std::max<size_t>(scratch, it.s_off + 7 * batch_scratch_stride(it.n));
  Layout L;
  bool ok;
  layout(batch, grid, scratch, dWork, work_bytes, &L, &ok);
  if (!ok) return fail(IPR_EARG, "ipr_solve_batched: workspace too small (%zu bytes)", work_bytes);
  const std::vector<int> order = work_order(items);
  HIP_TRY(hipMemcpyAsync(L.items, items.data(), batch * sizeof(BatchItem), hipMemcpyHostToDevice,
                         stream));
  HIP_TRY(hipMemcpyAsync(L.order, order.data(), batch * sizeof(int), hipMemcpyHostToDevice, stream));
  BatchArgs a;
  std::memset(&a, 0, sizeof a);
  a.A = dA;
  a.C = dC;
  a.scratch = L.scratch;
  a.items = L.items;
  a.order = L.order;
  a.count = batch;
  a.next = L.next;
  a.results = L.results;
  a.tol = tol;
  a.bulk_switch = s.bulk_switch;
  a.stall_ratio = s.stall_ratio;
  a.max_iter = s.max_iter;
  a.bulk_bf16 = s.bulk_dtype == IPR_BF16 ? 1 : 0;
  a.squarings = std::max(0, s.scale_squarings);
  a.dynamic = s.dynamic_scaling ? 1 : 0;
  a.lanczos_scale = s.scale_lanczos ? 1 : 0;
  if (use_graph) {
    if (int rc = launch_graph(a, grid, stream)) return rc;
  } else {
    HIP_TRY(batched_launch(a, grid, stream));
  }
  res->resize(batch);
  HIP_TRY(hipMemcpyAsync(res->data(), L.results, batch * sizeof(BatchResult),
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return IPR_OK;
}

}  // namespace

extern "C" {

int ipr_get_batched_tiles(int* tiles) {
  if (!tiles) return fail(IPR_EARG, "ipr_get_batched_tiles: null pointer");
  std::lock_guard<std::mutex> lk(g_mu);
  std::memcpy(tiles, g_tiles, sizeof g_tiles);
  return IPR_OK;
}

int ipr_set_batched_tiles(const int* tiles) {
  if (!tiles) return fail(IPR_EARG, "ipr_set_batched_tiles: null pointer");
  for (int b = 0; b < IPR_BATCH_BUCKETS; ++b)
    if (!valid_tile(tiles[b])) return fail(IPR_EARG, "tile edges must be 32 or 64");
  std::lock_guard<std::mutex> lk(g_mu);
  std::memcpy(g_tiles, tiles, sizeof g_tiles);
  return IPR_OK;
}

int ipr_solve_batched(const double* dA, double* dC, const int64_t* offsets, const int* n,
                      const int* p, int batch, double tol, const ipr_schedule* sched,
                      ipr_result* out, void* dWork, size_t work_bytes, hipStream_t stream) {
  g_last_error.clear();
  ipr_schedule sd;
  ipr_schedule_default(&sd);
  const ipr_schedule& s = sched ? *sched : sd;
  if (!dA || !dC || !offsets || !n || !p || !dWork || batch < 1)
    return fail(IPR_EARG, "ipr_solve_batched: bad argument");
  if (!(tol > 0.0)) return fail(IPR_EARG, "ipr_solve_batched: tol must be > 0");
  if (s.init != IPR_INIT_IDENTITY)
    return fail(IPR_EARG, "ipr_solve_batched: only the scaled-identity start is supported");
  if (s.bulk_dtype != IPR_FP64 && s.bulk_dtype != IPR_BF16)
    return fail(IPR_EARG, "ipr_solve_batched: bulk dtype must be FP64 or BF16");
  if (s.evaluation != IPR_EVAL_COUPLED)
    return fail(IPR_EARG, "ipr_solve_batched: only the coupled order is supported");
  if (s.store_format != IPR_STORE_NONE)
    return fail(IPR_EARG, "ipr_solve_batched: approximate storage is an ipr_solve option");
  if (s.tile != 0 && !valid_tile(s.tile))
    return fail(IPR_EARG, "ipr_solve_batched: tile must be 0, 32 or 64");
  if (s.max_iter < 0) return fail(IPR_EARG, "ipr_solve_batched: max_iter < 0");
  if (s.scale_lanczos && s.scale_squarings > 0)
    return fail(IPR_EARG, "ipr_solve_batched: scale_squarings and scale_lanczos are two ways "
                "to the same scale: choose one");
  int tiles[IPR_BATCH_BUCKETS];
  ipr_get_batched_tiles(tiles);
  std::vector<BatchItem> items(batch);
  int64_t soff = 0;
  for (int i = 0; i < batch; ++i) {
    if (n[i] < 1 || n[i] > 1024 || p[i] < 1 || p[i] > 8 || offsets[i] < 0)
      return fail(IPR_EARG, "ipr_solve_batched: item %d has n=%d p=%d offset=%lld", i, n[i], p[i],
                  (long long)offsets[i]);
    items[i].a_off = offsets[i];
    items[i].s_off = soff;
    items[i].n = n[i];
    items[i].p = p[i];
    items[i].tile = s.tile ? s.tile : tiles[bucket_of(n[i])];
    items[i].pad = 0;
    soff += 7 * (int64_t)batch_scratch_stride(n[i]);
  }
  std::vector<BatchResult> res;
  if (int rc = run_batch(dA, dC, items, tol, s, dWork, work_bytes, &res, stream, true)) return rc;
  int status = IPR_OK;
  for (int i = 0; i < batch; ++i) {
    if (out) {
      ipr_result& r = out[i];
      std::memset(&r, 0, sizeof r);
      r.status = res[i].status;
      r.iters_bulk = res[i].iters_bulk;
      r.iters_fp64 = res[i].iters_fp64;
      r.fallback_used = res[i].fallback_used;
      r.residual_proxy = res[i].residual_proxy;
      r.residual_true = res[i].residual_true >= 0 ? res[i].residual_true
                                                   : std::numeric_limits<double>::quiet_NaN();
      r.norm1 = res[i].norm1;
      r.norminf = res[i].norminf;
      r.init_bound = 1.0;
      r.init_scale = res[i].init_scale;
      r.lmin_est = res[i].lmin_est;
      r.reest_iter = res[i].reest_iter;
      r.lmin_reest = res[i].lmin_reest;
      r.poly_used[0] = 1.0;
      // the bf16 bulk phase runs for p = 1 items only
      r.bulk_skipped = (s.bulk_dtype != IPR_FP64 && p[i] >= 2) ? 1 : 0;
    }
    if (res[i].status != IPR_OK && status == IPR_OK) status = res[i].status;
  }
  return status;
}

int ipr_tune_batched(void* dWork, size_t work_bytes, int* tiles_out, hipStream_t stream) {
  g_last_error.clear();
  if (!dWork) return fail(IPR_EARG, "ipr_tune_batched: null workspace");
  ipr_schedule s;
  ipr_schedule_default(&s);
  s.max_iter = 3;  // fixed work per matrix: the tolerance below is never met
  int table[IPR_BATCH_BUCKETS];
  ipr_get_batched_tiles(table);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = IPR_OK;
  for (int b = 0; b < IPR_BATCH_BUCKETS && rc == IPR_OK; ++b) {
    const int nb = kBucketMax[b];
    const size_t nn = (size_t)nb * nb;
    // per matrix: A, C and 7 scratch matrices, plus bookkeeping
    const size_t per = 9 * nn * sizeof(double) + 2 * sizeof(BatchItem) + sizeof(BatchResult) + 16;
    const size_t slack = 1 << 20;
    const int count = work_bytes > slack ? (int)std::min<size_t>(512, (work_bytes - slack) / per) : 0;
    if (count < 1) continue;
    Carver c(dWork, work_bytes);
    double* A = c.take<double>(count * nn);
    double* C = c.take<double>(count * nn);
    BatchItem* fill_items = c.take<BatchItem>(count);
    void* rest = c.base + ((c.used + 255) & ~(size_t)255);
    const size_t rest_bytes = work_bytes - ((c.used + 255) & ~(size_t)255);
    std::vector<BatchItem> items(count);
    for (int i = 0; i < count; ++i) {
      items[i].a_off = (int64_t)i * nn;
      items[i].s_off = (int64_t)i * 7 * (int64_t)batch_scratch_stride(nb);
      items[i].n = nb;
      items[i].p = 2;
      items[i].tile = table[b];
      items[i].pad = 0;
    }
    HIP_TRY(hipMemcpyAsync(fill_items, items.data(), count * sizeof(BatchItem),
                           hipMemcpyHostToDevice, stream));
    HIP_TRY(batched_fill_test(A, fill_items, count, stream));
    float best_ms = std::numeric_limits<float>::max();
    int best_tile = table[b];
    for (int t : {32, 64}) {
      for (auto& it : items) it.tile = t;
      std::vector<BatchResult> res;
      (void)hipEventRecord(e0, stream);
      rc = run_batch(A, C, items, 1e-300, s, rest, rest_bytes, &res, stream, false);
      (void)hipEventRecord(e1, stream);
      if (rc != IPR_OK) break;
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best_ms) {
        best_ms = ms;
        best_tile = t;
      }
    }
    table[b] = best_tile;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != IPR_OK) return rc;
  ipr_set_batched_tiles(table);
  if (tiles_out) std::memcpy(tiles_out, table, sizeof table);
  return IPR_OK;
}

}  // extern "C"

size_t ipr::batched_workspace_bytes(int n_max, int batch) {
  Layout L;
  bool ok;
  // (each item's scratch stride rounds n^2 up by at most 31 elements)
  return layout(batch, grid_size(batch), 7 * ((size_t)n_max * n_max + 32 * (size_t)batch), nullptr,
                (size_t)-1, &L, &ok) +
         256;
}

