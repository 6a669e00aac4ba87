// trsm_autotune: the block size n0 and the tile policy measured on the
// device (Sec. VIII leaves the n0 constants to experiment), kept in a
// process-wide table that trsm_plan consults when asked to choose n0;
// trsm_batch_autotune: the same for the common block size of a batch.
#include "tune.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/trsm.h"
#include "kernels.hpp"

namespace trsm {

namespace {

// A candidate replaces the best so far only when it is this much faster, so
// that timing noise between near-equal configurations does not flip the
// choice from run to run (the cost model's choice is the first incumbent).
constexpr double kTuneMargin = 0.01;

struct Choice {
  int64_t n0;
  uint32_t flags;
};

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Choice>& table() {
  static std::map<std::tuple<int, int, int>, Choice> t;
  return t;
}

int clog2(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

std::tuple<int, int, int> key_of(int64_t n, int64_t k, int prec) {
  return std::make_tuple(prec, clog2(n), clog2(k));
}

struct DeviceBuf {
  void* p = nullptr;
  ~DeviceBuf() {
    if (p) (void)hipFree(p);
  }
  bool alloc(size_t bytes) { return hipMalloc(&p, std::max<size_t>(bytes, 256)) == hipSuccess; }
};

// Median milliseconds of `reps` runs of invert + solve with one plan.
trsm_status time_config(int64_t n, int64_t k, trsm_precision prec, int64_t n0, uint32_t flags,
                        int reps, const void* L, const void* B, void* X, hipStream_t s,
                        double* ms) {
  trsm_plan_t plan = nullptr;
  trsm_status st = trsm_plan(n, k, prec, n0, flags, &plan);
  if (st != TRSM_OK) return st;
  trsm_plan_info info;
  trsm_plan_get_info(plan, &info);
  DeviceBuf linv, ws;
  if (!linv.alloc(info.linv_bytes) || !ws.alloc(info.workspace_bytes)) {
    trsm_plan_destroy(plan);
    return TRSM_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<float> t;
  st = TRSM_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = TRSM_EHIP;
  for (int r = -1; r < reps && st == TRSM_OK; ++r) {
    if (r >= 0 && hipEventRecord(e0, s) != hipSuccess) st = TRSM_EHIP;
    if (st == TRSM_OK) st = trsm_invert_diag(plan, L, n, linv.p, s);
    if (st == TRSM_OK) st = trsm_solve(plan, L, n, linv.p, B, k, X, k, ws.p, s, nullptr);
    if (st == TRSM_OK && r >= 0) {
      float e = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&e, e0, e1) != hipSuccess)
        st = TRSM_EHIP;
      t.push_back(e);
    } else if (st == TRSM_OK && hipStreamSynchronize(s) != hipSuccess) {
      st = TRSM_EHIP;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  trsm_plan_destroy(plan);
  if (st != TRSM_OK) return st;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return TRSM_OK;
}

// Batches: the common block size of a batch of systems of uneven (n, k),
// keyed by (precision, ceil(log2 count), ceil(log2 max n), ceil(log2 max k)).
std::map<std::tuple<int, int, int, int>, int64_t>& batch_table() {
  static std::map<std::tuple<int, int, int, int>, int64_t> t;
  return t;
}

std::tuple<int, int, int, int> batch_key(int32_t count, const int64_t* n, const int64_t* k,
                                         int prec) {
  int64_t mn = 1, mk = 1;
  for (int32_t i = 0; i < count; ++i) {
    mn = std::max(mn, n[i]);
    mk = std::max(mk, k[i]);
  }
  return std::make_tuple(prec, clog2(count), clog2(mn), clog2(mk));
}

// One batch of synthetic systems: L, B, X per item, and its Linv per
// candidate block size.
struct BatchData {
  std::vector<DeviceBuf> L, B, X, Linv;
  explicit BatchData(int32_t count) : L(count), B(count), X(count), Linv(count) {}
};

// Median milliseconds of `reps` graph replays of trsm_batch_run with the
// common block size n0 (the inversions are done once, outside the timing,
// as a caller that keeps factors resident does).
trsm_status time_batch(int32_t count, const int64_t* n, const int64_t* k, trsm_precision prec,
                       int64_t n0, int reps, BatchData& d, hipStream_t s, double* ms) {
  std::vector<trsm_batch_item> items(count);
  for (int32_t i = 0; i < count; ++i) {
    trsm_plan_t plan = nullptr;
    trsm_status st = trsm_plan(n[i], k[i], prec, n0, 0, &plan);
    if (st != TRSM_OK) return st;
    trsm_plan_info info;
    trsm_plan_get_info(plan, &info);
    DeviceBuf& lb = d.Linv[i];
    if (lb.p) (void)hipFree(lb.p);
    lb.p = nullptr;
    if (!lb.alloc(info.linv_bytes)) {
      trsm_plan_destroy(plan);
      return TRSM_ENOMEM;
    }
    st = trsm_invert_diag(plan, d.L[i].p, n[i], lb.p, s);
    trsm_plan_destroy(plan);
    if (st != TRSM_OK) return st;
    items[i] = trsm_batch_item{n[i], k[i], d.L[i].p, n[i], lb.p, d.B[i].p, k[i], d.X[i].p, k[i]};
  }
  trsm_batch_t b = nullptr;
  trsm_status st = trsm_batch_create(count, items.data(), prec, n0, &b);
  if (st != TRSM_OK) return st;
  size_t wsb = 0;
  trsm_batch_workspace_bytes(b, &wsb);
  DeviceBuf ws;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<float> t;
  if (!ws.alloc(wsb)) st = TRSM_ENOMEM;
  if (st == TRSM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = TRSM_EHIP;
  // the first run captures the graph; later ones replay it
  for (int r = -1; r < reps && st == TRSM_OK; ++r) {
    if (r >= 0 && hipEventRecord(e0, s) != hipSuccess) st = TRSM_EHIP;
    if (st == TRSM_OK) st = trsm_batch_run(b, ws.p, s, 1);
    if (st == TRSM_OK && r >= 0) {
      float e = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&e, e0, e1) != hipSuccess)
        st = TRSM_EHIP;
      t.push_back(e);
    } else if (st == TRSM_OK && hipStreamSynchronize(s) != hipSuccess) {
      st = TRSM_EHIP;
    }
  }
  if (st == TRSM_OK) st = trsm_batch_check(b, ws.p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  trsm_batch_destroy(b);
  if (st != TRSM_OK) return st;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return TRSM_OK;
}

}  // namespace

bool tune_lookup(int64_t n, int64_t k, int prec, int64_t* n0, uint32_t* flags) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = table().find(key_of(n, k, prec));
  if (it == table().end()) return false;
  *n0 = it->second.n0;
  *flags = it->second.flags;
  return true;
}

}  // namespace trsm

using namespace trsm;

extern "C" {

trsm_status trsm_autotune(int64_t n, int64_t k, trsm_precision prec, int32_t reps, void* stream,
                          trsm_tune_result* out) {
  if (!out || n <= 0 || k <= 0 || reps <= 0) return TRSM_EINVAL;
  if (prec != TRSM_F64 && prec != TRSM_F32) return TRSM_EINVAL;
  if (n * k > ((int64_t)1 << 31) - 1 || n > ((int64_t)1 << 17)) return TRSM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t es = prec == TRSM_F32 ? 4 : 8;
  DeviceBuf L, B, X;
  if (!L.alloc((size_t)n * n * es) || !B.alloc((size_t)n * k * es) || !X.alloc((size_t)n * k * es))
    return TRSM_ENOMEM;
  hipError_t e = prec == TRSM_F32
                     ? launch_fill_system<float>((float*)L.p, n, (float*)B.p, k, 1234u, s)
                     : launch_fill_system<double>((double*)L.p, n, (double*)B.p, k, 1234u, s);
  if (e != hipSuccess) return (trsm_status)note_hip_error(e);
  // the cost model's choice, with the default tile policy, as the reference
  int64_t model_n0 = 0;
  {
    // a plan made without a record gives the model's choice
    std::lock_guard<std::mutex> g(g_tune_mu);
    table().erase(key_of(n, k, (int)prec));
  }
  trsm_plan_t p0 = nullptr;
  trsm_status st = trsm_plan(n, k, prec, 0, 0, &p0);
  if (st != TRSM_OK) return st;
  trsm_plan_info i0;
  trsm_plan_get_info(p0, &i0);
  model_n0 = i0.n0;
  trsm_plan_destroy(p0);
  double model_ms = 0.0;
  st = time_config(n, k, prec, model_n0, 0, reps, L.p, B.p, X.p, s, &model_ms);
  if (st != TRSM_OK) return st;
  Choice best{model_n0, 0u};
  double best_ms = model_ms;
  int32_t count = 1;
  int64_t top = 1;
  while (top < n) top <<= 1;
  top = std::min<int64_t>(top, 4096);
  // blocks much smaller than n (more than 256 steps) are never competitive
  int64_t lo = 32;
  while (lo < 4096 && lo * 256 < n) lo <<= 1;
  for (int64_t n0 = std::min(lo, std::max<int64_t>(top, 32)); n0 <= std::max<int64_t>(top, 32);
       n0 <<= 1) {
    for (uint32_t fl : {0u, (uint32_t)TRSM_FLAG_LARGE_TILES}) {
      if (n0 == model_n0 && fl == 0u) continue;   // timed above
      double ms = 0.0;
      st = time_config(n, k, prec, n0, fl, reps, L.p, B.p, X.p, s, &ms);
      if (st != TRSM_OK) return st;
      ++count;
      if (ms < best_ms * (1.0 - kTuneMargin)) {
        best_ms = ms;
        best = Choice{n0, fl};
      }
    }
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    table()[key_of(n, k, (int)prec)] = best;
  }
  out->n0 = best.n0;
  out->flags = best.flags;
  out->ms = best_ms;
  out->model_n0 = model_n0;
  out->model_ms = model_ms;
  out->candidates = count;
  return TRSM_OK;
}

trsm_status trsm_autotune_lookup(int64_t n, int64_t k, trsm_precision prec, int64_t* n0,
                                 uint32_t* flags) {
  if (!n0 || !flags || n <= 0 || k <= 0) return TRSM_EINVAL;
  *n0 = 0;
  *flags = 0;
  int64_t v = 0;
  uint32_t f = 0;
  if (tune_lookup(n, k, (int)prec, &v, &f)) {
    *n0 = v;
    *flags = f;
  }
  return TRSM_OK;
}

trsm_status trsm_autotune_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  table().clear();
  batch_table().clear();
  return TRSM_OK;
}

trsm_status trsm_batch_autotune(int32_t count, const int64_t* n, const int64_t* k,
                                trsm_precision prec, int32_t reps, trsm_batch_tune_result* out) {
  if (!out || count <= 0 || !n || !k || reps <= 0) return TRSM_EINVAL;
  if (prec != TRSM_F64 && prec != TRSM_F32) return TRSM_EINVAL;
  const size_t es = prec == TRSM_F32 ? 4 : 8;
  int64_t mn = 1;
  double bytes = 0.0;
  for (int32_t i = 0; i < count; ++i) {
    if (n[i] <= 0 || k[i] <= 0 || n[i] > ((int64_t)1 << 16) || k[i] > ((int64_t)1 << 16))
      return TRSM_EINVAL;
    mn = std::max(mn, n[i]);
    bytes += (double)es * ((double)n[i] * n[i] + 2.0 * n[i] * k[i]);
  }
  if (bytes > (double)((size_t)64 << 30)) return TRSM_ENOMEM;   // the synthetic systems
  hipStream_t s = nullptr;
  if (hipStreamCreate(&s) != hipSuccess) return (trsm_status)note_hip_error(hipGetLastError());
  trsm_status st = TRSM_OK;
  {
    BatchData d(count);
    for (int32_t i = 0; i < count && st == TRSM_OK; ++i) {
      if (!d.L[i].alloc((size_t)n[i] * n[i] * es) || !d.B[i].alloc((size_t)n[i] * k[i] * es) ||
          !d.X[i].alloc((size_t)n[i] * k[i] * es)) {
        st = TRSM_ENOMEM;
        break;
      }
      const hipError_t e =
          prec == TRSM_F32
              ? launch_fill_system<float>((float*)d.L[i].p, n[i], (float*)d.B[i].p, k[i], 777u + i, s)
              : launch_fill_system<double>((double*)d.L[i].p, n[i], (double*)d.B[i].p, k[i], 777u + i, s);
      if (e != hipSuccess) st = (trsm_status)note_hip_error(e);
    }
    // incumbent: every system inverted whole (up to 4096 rows), each sweep
    // one product per system
    int64_t top = 1;
    while (top < mn) top <<= 1;
    top = std::min<int64_t>(std::max<int64_t>(top, 64), 4096);
    double best_ms = 0.0, def_ms = 0.0;
    int64_t best = top;
    int32_t cands = 0;
    if (st == TRSM_OK) st = time_batch(count, n, k, prec, top, reps, d, s, &def_ms);
    best_ms = def_ms;
    ++cands;
    for (int64_t n0 = 64; n0 < top && st == TRSM_OK; n0 <<= 1) {
      double ms = 0.0;
      st = time_batch(count, n, k, prec, n0, reps, d, s, &ms);
      if (st != TRSM_OK) break;
      ++cands;
      if (ms < best_ms * (1.0 - kTuneMargin)) {
        best_ms = ms;
        best = n0;
      }
    }
    if (st == TRSM_OK) {
      {
        std::lock_guard<std::mutex> g(g_tune_mu);
        batch_table()[batch_key(count, n, k, (int)prec)] = best;
      }
      out->n0 = best;
      out->ms = best_ms;
      out->default_n0 = top;
      out->default_ms = def_ms;
      out->candidates = cands;
    }
    (void)hipStreamSynchronize(s);
  }
  (void)hipStreamDestroy(s);
  return st;
}

trsm_status trsm_batch_autotune_lookup(int32_t count, const int64_t* n, const int64_t* k,
                                       trsm_precision prec, int64_t* n0) {
  if (!n0 || count <= 0 || !n || !k) return TRSM_EINVAL;
  *n0 = 0;
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = batch_table().find(batch_key(count, n, k, (int)prec));
  if (it != batch_table().end()) *n0 = it->second;
  return TRSM_OK;
}

}  // extern "C"
