// Continuous-batching server for triangular solves with resident factors.
//
// Each registered factor L keeps, in server-owned device memory, a binary64
// copy, a binary32 copy, and its inverted n0 x n0 diagonal blocks (Alg.
// Diagonal-Inverter, computed once).  Clients submit right-hand sides without
// blocking; a worker thread admits queued requests while the HBM budget and
// the slot count allow, groups the admitted requests by block count, and
// launches each group as one batch of grouped kernels on one of several
// streams, so that batches admitted at different times overlap on the GPU.
// Per request, the batch runs binary32 sweeps (Alg. It-Inv-TRSM) with one
// step of iterative refinement driven by a binary64 residual:
//     X0 = solve32(B);  R = B - L X0 (binary64);  X = X0 + solve32(R).
// Every request's tiles are computed identically whatever else is in its
// batch, so its result does not depend on the mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/trsm.h"
#include "batch.hpp"
#include "kernels.hpp"

using namespace trsm;

namespace {

constexpr size_t kAl = 256;
constexpr int64_t kCholMaxN0 = 512;
inline size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device block (offsets only; host bookkeeping).
class Arena {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  // Returns SIZE_MAX when no free range is large enough.
  size_t alloc(size_t bytes) {
    bytes = al(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        sizes_[off] = bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t len = s->second;
    sizes_.erase(s);
    used_ -= len;
    size_t start = off;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> sizes_;  // live allocations
};

struct Factor {
  int64_t n = 0, m = 0, n0 = 0;
  size_t off = 0, bytes = 0;
  double* L64 = nullptr;  int64_t ld64 = 0;
  float* L32 = nullptr;   int64_t ld32 = 0;
  double* Linv64 = nullptr;
  float* Linv32 = nullptr;
  // Cholesky factors (requests solve A X = B, A = L L^T): U = L^T and the
  // transposed inverse blocks
  bool chol = false;
  double* U64 = nullptr;
  float* U32 = nullptr;
  float* Uinv32 = nullptr;
};

struct Request {
  uint64_t ticket = 0;
  int32_t l_id = -1;
  int64_t k = 0, kp = 0;
  const double* B = nullptr;
  int64_t ldb = 0;
  double* X = nullptr;
  int64_t ldx = 0;
  int state = TRSM_REQ_PENDING;
  int status = TRSM_OK;
  double t_submit = 0, t_done = 0;
  size_t ws_off = SIZE_MAX, ws_bytes = 0;
};

struct Batch {
  std::vector<std::shared_ptr<Request>> reqs;
  hipEvent_t done = nullptr;
  size_t table_off = SIZE_MAX;
  size_t cnt_off = SIZE_MAX;  // counters of the persistent sweeps (n0 = kPB)
  std::vector<char> table;   // host copy kept alive until completion
  int stream = 0;
};

}  // namespace

struct trsm_server_s {
  int device = 0;
  size_t budget = 0;
  int32_t max_slots = 0;
  int64_t n0 = 128;
  char* base = nullptr;        // one device block of `budget` bytes
  Arena arena;
  std::vector<Factor> factors;
  std::vector<hipStream_t> streams;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<Batch> inflight;
  int32_t slots_used = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  int fatal = 0;

  // statistics (guarded by mu)
  uint64_t submitted = 0, completed = 0, failed = 0, batches = 0;
  std::vector<double> lat_us;
  double flops_done = 0, t_first = 0, t_last = 0;
  int32_t max_inflight_slots = 0;
};

namespace {

size_t factor_bytes(int64_t n, int64_t n0, bool chol) {
  const int64_t m = ceil_div(n, n0);
  // the binary64 inverses take a TRSM_F64 plan's whole Linv buffer (the
  // packed blocks and the inversion's status word)
  size_t b = al((size_t)n * round_up(n, 2) * 8) + al((size_t)n * round_up(n, 4) * 4) +
             al((size_t)m * n0 * n0 * 8) + al(8) + al((size_t)m * n0 * n0 * 4);
  if (chol)
    b += al((size_t)n * round_up(n, 2) * 8) + al((size_t)n * round_up(n, 4) * 4) +
         al((size_t)m * n0 * n0 * 4);
  return b;
}

// Internal buffers of a request are kp = round_up(k, 4) columns wide (zero
// padded) so that every product takes the 16-byte vector path.
size_t request_bytes(int64_t n, int64_t kp, bool chol) {
  // B, X, R (binary64), running RHS and correction (binary32); for A = L L^T
  // also the backward sweep's output (binary32) and L^T X (binary64)
  size_t b = 3 * al((size_t)n * kp * 8) + 2 * al((size_t)n * kp * 4);
  if (chol) b += al((size_t)n * kp * 4) + al((size_t)n * kp * 8);
  return b;
}

struct ReqBufs {
  double* B64; double* X64; double* R64; float* Rl; float* D;
  float* E; double* T64;   // Cholesky requests only
};

ReqBufs bufs_of(trsm_server_s* S, const Request& r, int64_t n, bool chol) {
  char* p = S->base + r.ws_off;
  ReqBufs b{};
  b.B64 = (double*)p; p += al((size_t)n * r.kp * 8);
  b.X64 = (double*)p; p += al((size_t)n * r.kp * 8);
  b.R64 = (double*)p; p += al((size_t)n * r.kp * 8);
  b.Rl = (float*)p;   p += al((size_t)n * r.kp * 4);
  b.D = (float*)p;    p += al((size_t)n * r.kp * 4);
  if (chol) {
    b.E = (float*)p;    p += al((size_t)n * r.kp * 4);
    b.T64 = (double*)p;
  }
  return b;
}

// Record the full refinement pipeline of a group of requests.  With n0 =
// kPB both binary32 sweeps are persistent launches that share the counter
// words at `counters` (each launch clears them first; same stream).
// Requests on Cholesky factors (A = L L^T) add a backward sweep with U = L^T
// after each forward sweep, and their residual B - L (U X) takes one more
// binary64 product.
void record_pipeline(trsm_server_s* S, const std::vector<std::shared_ptr<Request>>& reqs,
                     LaunchList& list, unsigned* counters) {
  std::vector<EwEntry> ew_b, ew_in, ew_x0, ew_r, ew_add, ew_out;
  std::vector<SweepItem<float>> sweep, back;
  std::vector<GemmP64> resid_u, resid;
  for (const auto& rp : reqs) {
    const Request& r = *rp;
    const Factor& f = S->factors[r.l_id];
    const ReqBufs b = bufs_of(S, r, f.n, f.chol);
    const int n = (int)f.n, k = (int)r.k, kp = (int)r.kp;
    ew_b.push_back(EwEntry{r.B, r.ldb, b.B64, kp, n, kp, 1.0, EW_F64_COPY, k});
    ew_in.push_back(EwEntry{r.B, r.ldb, b.Rl, kp, n, kp, 1.0, EW_F64_TO_F32, k});
    SweepItem<float> it{};
    it.n = f.n; it.k = kp; it.n0 = f.n0;
    it.L = f.L32; it.ldl = f.ld32;
    it.Linv = f.Linv32;
    it.B = b.Rl; it.ldb = kp;          // the running right-hand side is updated in place
    it.X = b.D; it.ldx = kp;
    it.R = b.Rl; it.ldr = kp;
    sweep.push_back(it);
    float* sol = b.D;                  // the binary32 solution of one pass
    const double* prod = b.X64;        // what L multiplies in the residual
    if (f.chol) {
      SweepItem<float> u{};
      u.n = f.n; u.k = kp; u.n0 = f.n0;
      u.L = f.U32; u.ldl = f.ld32;     // upper triangular
      u.Linv = f.Uinv32;
      u.B = b.D; u.ldb = kp;
      u.X = b.E; u.ldx = kp;
      u.R = b.Rl; u.ldr = kp;          // free again after the forward pass
      back.push_back(u);
      sol = b.E;
      auto q = gemm_params<double, double, double, float>();
      q.A = f.U64; q.lda = f.ld64;     // T = L^T X
      q.B = b.X64; q.ldb = kp;
      q.Cout = b.T64; q.ldco = kp;
      q.M = n; q.N = kp; q.K = n;
      q.flags = G_A_UPPER;
      resid_u.push_back(q);
      prod = b.T64;
    }
    ew_x0.push_back(EwEntry{sol, kp, b.X64, kp, n, kp, 1.0, EW_F32_TO_F64_SET, kp});
    auto p = gemm_params<double, double, double, float>();
    p.A = f.L64; p.lda = f.ld64;
    p.B = prod; p.ldb = kp;
    p.Cin = b.B64; p.ldci = kp;
    p.Cout = b.R64; p.ldco = kp;
    p.M = n; p.N = kp; p.K = n;
    p.alpha = -1.0; p.beta = 1.0;
    p.flags = G_A_LOWER | G_BETA;
    resid.push_back(p);
    ew_r.push_back(EwEntry{b.R64, kp, b.Rl, kp, n, kp, 1.0, EW_F64_TO_F32, kp});
    ew_add.push_back(EwEntry{sol, kp, b.X64, kp, n, kp, 1.0, EW_F32_TO_F64_ADD, kp});
    ew_out.push_back(EwEntry{b.X64, kp, r.X, r.ldx, n, k, 1.0, EW_F64_COPY, k});
  }
  const bool persist = S->n0 == kPB;
  auto sweeps = [&] {
    if (persist) record_persist<float>(list, sweep, counters);
    else record_sweep<float>(list, sweep);
    if (!back.empty()) record_sweep_back<float>(list, back);
  };
  list.clear();
  list.add_ew(ew_b);
  list.add_ew(ew_in);
  sweeps();
  list.add_ew(ew_x0);
  if (!resid_u.empty()) list.add_gemm64(resid_u);
  list.add_gemm64(resid);
  list.add_ew(ew_r);
  sweeps();
  list.add_ew(ew_add);
  list.add_ew(ew_out);
}

// Counter words of a group's persistent sweeps (0 when the server sweeps by
// phases).
size_t pipeline_counter_bytes(trsm_server_s* S, const std::vector<std::shared_ptr<Request>>& reqs) {
  if (S->n0 != kPB) return 0;
  int64_t tiles = 0;
  for (const auto& rp : reqs) tiles += ceil_div(rp->kp, kPB);
  return (size_t)(tiles + 2) * 4;
}

int bucket_of(int64_t m) {
  int b = 0;
  while ((1ll << b) < m) ++b;
  return b;
}

void complete_batch(trsm_server_s* S, Batch& b, int status) {
  const double t = now_us();
  for (auto& rp : b.reqs) {
    Request& r = *rp;
    r.state = status == TRSM_OK ? TRSM_REQ_DONE : TRSM_REQ_ERROR;
    r.status = status;
    r.t_done = t;
    if (r.ws_off != SIZE_MAX) S->arena.release(r.ws_off);
    r.ws_off = SIZE_MAX;
    S->slots_used -= 1;
    if (status == TRSM_OK) {
      S->completed += 1;
      S->lat_us.push_back(r.t_done - r.t_submit);
      const Factor& f = S->factors[r.l_id];
      const double n = (double)f.n;
      S->flops_done += (f.chol ? 2.0 : 1.0) * n * n * (double)r.k;
      S->t_last = t;
    } else {
      S->failed += 1;
    }
  }
  if (b.table_off != SIZE_MAX) S->arena.release(b.table_off);
  if (b.cnt_off != SIZE_MAX) S->arena.release(b.cnt_off);
  b.table_off = b.cnt_off = SIZE_MAX;
  if (b.done) (void)hipEventDestroy(b.done);
  b.done = nullptr;
}

// One pass of the worker: retire finished batches, then -- if a stream is
// free -- admit queued requests (arrival order, while slots and memory
// allow) and launch them.  Requests that arrive while every stream is busy
// accumulate and form a larger batch on the next free stream (continuous
// batching: admission happens as soon as capacity frees up, and batches on
// different streams run concurrently).
bool worker_tick(trsm_server_s* S) {
  std::vector<std::shared_ptr<Request>> admitted;
  std::vector<int> free_streams;
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (size_t i = 0; i < S->inflight.size();) {
      hipError_t q = hipEventQuery(S->inflight[i].done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      complete_batch(S, S->inflight[i], q == hipSuccess ? TRSM_OK : TRSM_EHIP);
      S->inflight.erase(S->inflight.begin() + i);
    }
    std::vector<bool> busy(S->streams.size(), false);
    for (const Batch& b : S->inflight) busy[b.stream] = true;
    for (size_t i = 0; i < busy.size(); ++i)
      if (!busy[i]) free_streams.push_back((int)i);
    if (free_streams.empty()) return false;
    while (!S->pending.empty() && S->slots_used < S->max_slots) {
      auto rp = S->pending.front();
      const Factor& f = S->factors[rp->l_id];
      const size_t need = request_bytes(f.n, rp->kp, f.chol);
      const size_t off = S->arena.alloc(need);
      if (off == SIZE_MAX) {
        // cannot fit now; if it can never fit (nothing else holds memory), fail it
        if (S->inflight.empty() && admitted.empty()) {
          S->pending.pop_front();
          rp->state = TRSM_REQ_ERROR;
          rp->status = TRSM_ENOMEM;
          S->failed += 1;
          continue;
        }
        break;
      }
      rp->ws_off = off;
      rp->ws_bytes = need;
      rp->state = TRSM_REQ_RUNNING;
      S->pending.pop_front();
      S->slots_used += 1;
      admitted.push_back(rp);
    }
    S->max_inflight_slots = std::max(S->max_inflight_slots, S->slots_used);
  }
  if (admitted.empty()) return false;
  // Group by block count (small systems need few sweep phases) and merge the
  // smallest groups until there is one group per free stream.
  std::map<int, std::vector<std::shared_ptr<Request>>> by_bucket;
  for (auto& rp : admitted) by_bucket[bucket_of(S->factors[rp->l_id].m)].push_back(rp);
  std::vector<std::vector<std::shared_ptr<Request>>> groups;
  for (auto& kv : by_bucket) groups.push_back(std::move(kv.second));
  while (groups.size() > free_streams.size()) {
    groups[1].insert(groups[1].end(), groups[0].begin(), groups[0].end());
    groups.erase(groups.begin());
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Batch b;
    b.reqs = std::move(groups[gi]);
    b.stream = free_streams[gi];
    LaunchList list;
    int status = TRSM_OK;
    const size_t cb = pipeline_counter_bytes(S, b.reqs);
    if (cb) {
      std::lock_guard<std::mutex> g(S->mu);
      b.cnt_off = S->arena.alloc(cb);
      if (b.cnt_off == SIZE_MAX) status = TRSM_ENOMEM;
    }
    unsigned* counters = cb && status == TRSM_OK ? (unsigned*)(S->base + b.cnt_off) : nullptr;
    record_pipeline(S, b.reqs, list, counters);
    const size_t tb = list.table_bytes();
    b.table.assign((const char*)list.host_table(), (const char*)list.host_table() + tb);
    if (status == TRSM_OK) {
      std::lock_guard<std::mutex> g(S->mu);
      b.table_off = S->arena.alloc(tb);
      if (b.table_off == SIZE_MAX) status = TRSM_ENOMEM;
    }
    hipStream_t s = S->streams[b.stream];
    if (status == TRSM_OK) {
      char* dev = S->base + b.table_off;
      hipError_t e = hipMemcpyAsync(dev, b.table.data(), tb, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = list.run(dev, s);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(b.done, s);
      if (e != hipSuccess) status = note_hip_error(e);
    }
    std::lock_guard<std::mutex> g(S->mu);
    S->batches += 1;
    if (status != TRSM_OK) {
      complete_batch(S, b, status);
    } else {
      S->inflight.push_back(std::move(b));
    }
  }
  return true;
}

void worker_main(trsm_server_s* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    bool busy = worker_tick(S);
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->stop && S->pending.empty() && S->inflight.empty()) break;
    if (!busy) {
      // wake on a new request, or poll in-flight batches every 20 us
      S->cv.wait_for(lk, std::chrono::microseconds(S->inflight.empty() ? 2000 : 20));
    }
  }
}

}  // namespace

extern "C" {

trsm_status trsm_server_create(size_t hbm_budget, int32_t max_slots, int64_t n0,
                               trsm_server_t* out) {
  if (!out) return TRSM_EINVAL;
  *out = nullptr;
  if (max_slots <= 0 || hbm_budget < (1u << 20)) return TRSM_EINVAL;
  if (n0 <= 0 || (n0 & (n0 - 1))) return TRSM_EINVAL;
  trsm_server_s* S = new (std::nothrow) trsm_server_s();
  if (!S) return TRSM_ENOMEM;
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  S->n0 = n0;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return TRSM_EHIP;
  }
  if (hipMalloc((void**)&S->base, hbm_budget) != hipSuccess) {
    delete S;
    return TRSM_ENOMEM;
  }
  S->arena.init(hbm_budget);
  for (int i = 0; i < 4; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto t : S->streams) (void)hipStreamDestroy(t);
      (void)hipFree(S->base);
      delete S;
      return TRSM_EHIP;
    }
    S->streams.push_back(s);
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return TRSM_OK;
}

}  // extern "C"

namespace {

trsm_status register_factor(trsm_server_t S, const double* L, int64_t n, int64_t ldl, bool chol,
                            int32_t* l_id) {
  if (!S || !L || !l_id || n <= 0 || ldl < n || n > (1 << 20)) return TRSM_EINVAL;
  Factor f;
  f.n = n;
  // A = L L^T has the square of L's condition number, and the single
  // refinement step must remove the binary32 error of two sweeps; fully
  // inverted blocks of more than kCholMaxN0 rows left too little margin to
  // 1e-12 (measured), so Cholesky factors use at most that block size.
  f.n0 = effective_n0(n, chol ? std::min<int64_t>(S->n0, kCholMaxN0) : S->n0);
  f.m = ceil_div(n, f.n0);
  f.chol = chol;
  f.bytes = factor_bytes(n, f.n0, chol);
  {
    std::lock_guard<std::mutex> g(S->mu);
    f.off = S->arena.alloc(f.bytes);
  }
  if (f.off == SIZE_MAX) return TRSM_ENOMEM;
  char* p = S->base + f.off;
  f.ld64 = round_up(n, 2);
  f.L64 = (double*)p; p += al((size_t)n * f.ld64 * 8);
  f.ld32 = round_up(n, 4);
  f.L32 = (float*)p; p += al((size_t)n * f.ld32 * 4);
  f.Linv64 = (double*)p; p += al((size_t)f.m * f.n0 * f.n0 * 8) + al(8);
  f.Linv32 = (float*)p; p += al((size_t)f.m * f.n0 * f.n0 * 4);
  if (chol) {
    f.U64 = (double*)p; p += al((size_t)n * f.ld64 * 8);
    f.U32 = (float*)p; p += al((size_t)n * f.ld32 * 4);
    f.Uinv32 = (float*)p;
  }
  hipStream_t s = S->streams[0];
  trsm_plan_t plan = nullptr;
  trsm_status st = trsm_plan(n, 1, TRSM_F64, f.n0, 0, &plan);   // the factor's own block size
  hipError_t e = hipSuccess;
  if (st == TRSM_OK) {
    trsm_plan_info pi;
    st = trsm_plan_get_info(plan, &pi);
    if (st == TRSM_OK && pi.linv_bytes > al((size_t)f.m * f.n0 * f.n0 * 8) + al(8)) st = TRSM_EINVAL;
  }
  if (st == TRSM_OK) {
    e = launch_copy2d<double, double>(L, ldl, f.L64, f.ld64, n, n, 1.0, s);
    if (e == hipSuccess) e = launch_copy2d<double, float>(L, ldl, f.L32, f.ld32, n, n, 1.0, s);
    if (e == hipSuccess) st = trsm_invert_diag(plan, f.L64, f.ld64, f.Linv64, s);
    if (st == TRSM_OK && e == hipSuccess)
      e = launch_convert<double, float>(f.Linv64, f.Linv32, f.m * f.n0 * f.n0, s);
    if (chol && st == TRSM_OK && e == hipSuccess) {
      // U = L^T (zeros below the diagonal) and Uinv_ii = Linv_ii^T
      e = launch_transpose<double, double>(f.L64, f.ld64, f.U64, f.ld64, n, n, 1, 0, 0, true, s);
      if (e == hipSuccess)
        e = launch_transpose<float, float>(f.L32, f.ld32, f.U32, f.ld32, n, n, 1, 0, 0, true, s);
      if (e == hipSuccess)
        e = launch_transpose<float, float>(f.Linv32, f.n0, f.Uinv32, f.n0, f.n0, f.n0, f.m,
                                           f.n0 * f.n0, f.n0 * f.n0, false, s);
    }
    if (st == TRSM_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    if (st == TRSM_OK && e == hipSuccess) {
      trsm_status le;
      int64_t idx;
      st = trsm_plan_last_error(plan, &le, &idx);
      if (st == TRSM_OK && le != TRSM_OK) st = le;
    }
    trsm_plan_destroy(plan);
  }
  if (st == TRSM_OK && e != hipSuccess) st = TRSM_EHIP;
  std::lock_guard<std::mutex> g(S->mu);
  if (st != TRSM_OK) {
    S->arena.release(f.off);
    return st;
  }
  S->factors.push_back(f);
  *l_id = (int32_t)S->factors.size() - 1;
  return TRSM_OK;
}

}  // namespace

extern "C" {

trsm_status trsm_server_register_L(trsm_server_t S, const double* L, int64_t n, int64_t ldl,
                                   int32_t* l_id) {
  return register_factor(S, L, n, ldl, false, l_id);
}

trsm_status trsm_server_register_chol(trsm_server_t S, const double* L, int64_t n, int64_t ldl,
                                      int32_t* l_id) {
  return register_factor(S, L, n, ldl, true, l_id);
}

trsm_status trsm_serve_submit(trsm_server_t S, int32_t l_id, const double* B, int64_t k,
                              int64_t ldb, double* X, int64_t ldx, uint64_t* ticket) {
  if (!S || !ticket || !B || !X || k <= 0 || ldb < k || ldx < k) return TRSM_EINVAL;
  auto r = std::make_shared<Request>();
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (l_id < 0 || l_id >= (int32_t)S->factors.size()) return TRSM_EINVAL;
    const int64_t n = S->factors[l_id].n;
    const uintptr_t b0 = (uintptr_t)B, b1 = b0 + ((size_t)(n - 1) * ldb + k) * 8;
    const uintptr_t x0 = (uintptr_t)X, x1 = x0 + ((size_t)(n - 1) * ldx + k) * 8;
    if (b0 < x1 && x0 < b1) return TRSM_EINVAL;
    r->ticket = S->next_ticket++;
    r->l_id = l_id;
    r->k = k;
    r->kp = round_up(k, 4);
    r->B = B;
    r->ldb = ldb;
    r->X = X;
    r->ldx = ldx;
    r->t_submit = now_us();
    if (S->t_first == 0) S->t_first = r->t_submit;
    S->pending.push_back(r);
    S->all[r->ticket] = r;
    S->submitted += 1;
    *ticket = r->ticket;
  }
  S->cv.notify_one();
  return TRSM_OK;
}

trsm_status trsm_serve_poll(trsm_server_t S, uint64_t ticket, trsm_req_state* state,
                            double* latency_us) {
  if (!S || !state) return TRSM_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) {
    *state = TRSM_REQ_UNKNOWN;
    return TRSM_EINVAL;
  }
  const Request& r = *it->second;
  *state = (trsm_req_state)r.state;
  if (latency_us) *latency_us = r.state == TRSM_REQ_DONE ? r.t_done - r.t_submit : -1.0;
  if (r.state == TRSM_REQ_DONE || r.state == TRSM_REQ_ERROR) {
    const trsm_status st = (trsm_status)r.status;
    S->all.erase(it);   // a finished ticket is reported once
    return st == TRSM_OK ? TRSM_OK : st;
  }
  return TRSM_OK;
}

trsm_status trsm_server_stats(trsm_server_t S, trsm_serve_stats* st) {
  if (!S || !st) return TRSM_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  memset(st, 0, sizeof(*st));
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->failed = S->failed;
  st->batches = S->batches;
  std::vector<double> v = S->lat_us;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      size_t i = (size_t)std::min<double>(v.size() - 1, std::max(0.0, std::ceil(q * v.size()) - 1));
      return v[i];
    };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
    double s = 0;
    for (double x : v) s += x;
    st->mean_us = s / v.size();
  }
  st->flops_done = S->flops_done;
  st->wall_s = (S->t_last > S->t_first) ? (S->t_last - S->t_first) * 1e-6 : 0.0;
  st->hbm_budget = S->budget;
  st->hbm_in_use = S->arena.used();
  size_t res = 0;
  for (const auto& f : S->factors) res += f.bytes;
  st->resident_bytes = res;
  st->queue_depth = (int32_t)S->pending.size();
  st->in_flight = S->slots_used;
  st->max_in_flight = S->max_inflight_slots;
  st->factors = (int32_t)S->factors.size();
  return TRSM_OK;
}

trsm_status trsm_server_reset_stats(trsm_server_t S) {
  if (!S) return TRSM_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  S->completed = S->failed = S->submitted = S->batches = 0;
  S->lat_us.clear();
  S->flops_done = 0;
  S->t_first = S->t_last = 0;
  S->max_inflight_slots = S->slots_used;
  return TRSM_OK;
}

trsm_status trsm_server_destroy(trsm_server_t S) {
  if (!S) return TRSM_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto s : S->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (S->base) (void)hipFree(S->base);
  delete S;
  return TRSM_OK;
}

}  // extern "C"
