// Continuous-batching server for triangular solves with resident factors.
//
// Each registered factor L keeps, in server-owned device memory, its
// binary64 copy (for residuals), the copy its sweeps read (binary32 or
// binary64) and its inverted n0 x n0 diagonal blocks (Alg. Diagonal-Inverter,
// computed once).  Clients submit right-hand sides without blocking.  A
// request is solved by iterative refinement around the sweep of Alg.
// It-Inv-TRSM, one "pass" at a time:
//     pass 0:  X = sweep(B);  [binary32 factors: R = B - L X;  X += sweep(R)]
//     pass j:  X += sweep(R)                    (R from the previous pass)
// and every pass ends with R = B - L X in binary64, the request's norms
// ||R||, ||X||, ||last correction|| (deterministic grouped reductions), and a
// copy of X to the caller.  The worker thread reads the norms when the
// pass's batch completes and applies the request's stopping test; a request
// that needs another correction rejoins the queue with the newest arrivals,
// so admission happens at pass granularity ("continuous batching").  Every
// request's tiles and sums are computed identically whatever else is in its
// batch, so its result does not depend on the mix.
#include <hip/hip_runtime.h>
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
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
constexpr int kStreams = 4;
constexpr int64_t kDefaultN0 = 4096;
constexpr int64_t kCholMaxN0F32 = 512;
constexpr int kDefaultMaxCorr = 10;
constexpr int kMaxCorrLimit = 50;
constexpr int kStatRow = 8;   // doubles per slot of the pinned norm table
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

// Every factor is kept padded to np = round_up(n, 4) rows and columns (zero
// off-diagonal entries, ones on the padded diagonal) and every internal
// right-hand side to np rows (zero padding), so that every product takes the
// 16-byte vector path; the padding never changes the first n rows.
struct Factor {
  int64_t n = 0, np = 0, m = 0, n0 = 0;
  int prec = TRSM_F32;     // sweep precision: TRSM_F32 or TRSM_F64
  bool chol = false;       // requests solve A X = B with A = L L^T
  size_t off = 0, bytes = 0;
  double lnorm = 0.0;      // ||L||_F (of the n x n factor)
  double* L64 = nullptr;  int64_t ld64 = 0;   // ld = np
  float* L32 = nullptr;   int64_t ld32 = 0;
  double* Linv64 = nullptr;   // binary64 sweeps
  float* Linv32 = nullptr;    // binary32 sweeps
  // Cholesky factors: U = L^T (zeros below the diagonal) and its inverted
  // blocks Uinv_ii = Linv_ii^T
  double* U64 = nullptr;
  float* U32 = nullptr;
  double* Uinv64 = nullptr;
  float* Uinv32 = nullptr;
};

struct Request {
  uint64_t ticket = 0;
  const Factor* f = nullptr;
  int64_t k = 0, kp = 0;
  const double* B = nullptr;
  int64_t ldb = 0;
  double* X = nullptr;
  int64_t ldx = 0;
  int state = TRSM_REQ_PENDING;
  int status = TRSM_OK;
  double t_submit = 0, t_done = 0;
  size_t ws_off = SIZE_MAX, ws_bytes = 0;
  int slot = -1;            // row of the pinned norm table
  int passes = 0;           // passes completed
  int corrections = 0;      // corrections applied
  double prev_corr = -1.0;  // corr of the previous correction
  trsm_info info{0, 0, -1.0, -1.0, -1.0};
};

// The batch running on one stream (at most one per stream).
struct Batch {
  std::vector<std::shared_ptr<Request>> reqs;
  size_t table_off = SIZE_MAX;
  size_t cnt_off = SIZE_MAX;   // counters of the persistent sweeps (n0 = kPB)
  bool busy = false;
};

}  // namespace

struct trsm_server_s {
  int device = 0;
  size_t budget = 0;
  int32_t max_slots = 0;
  int64_t n0 = kDefaultN0;
  double tol = 0.0;           // 0: sqrt(n) 2^-53 per factor
  int max_corr = kDefaultMaxCorr;
  char* base = nullptr;       // one device block of `budget` bytes
  Arena arena;
  std::vector<std::unique_ptr<Factor>> factors;   // pointers stay valid
  hipStream_t streams[kStreams] = {};
  hipEvent_t events[kStreams] = {};
  Batch batch[kStreams];
  // pinned staging of each stream's launch table
  char* stage[kStreams] = {};
  size_t stage_cap[kStreams] = {};
  hipStream_t reg_stream = nullptr;   // registrations
  std::mutex reg_mu;                  // one registration at a time
  // per-slot sums of squares of R, X and the last correction (each as s 4^x,
  // see FinEntry): pinned host memory written by the final reduction of
  // each pass
  double* hstat = nullptr;
  double* hstat_dev = nullptr;
  std::vector<int> free_slots;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> pending;   // not yet admitted
  std::deque<std::shared_ptr<Request>> ready;     // admitted, waiting for their next pass
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  int32_t slots_used = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;

  // statistics (guarded by mu)
  uint64_t submitted = 0, completed = 0, failed = 0, batches = 0, unconverged = 0, passes = 0;
  std::vector<double> lat_us;
  double flops_done = 0, t_first = 0, t_last = 0;
  int32_t max_inflight_slots = 0;
};

namespace {

// Device bytes a factor keeps (the binary64 inverses of a TRSM_F64 factor
// take a TRSM_F64 plan's whole Linv buffer: the packed blocks and the
// inversion's status word).
size_t factor_bytes(int64_t np, int64_t n0, bool chol, int prec) {
  const int64_t m = ceil_div(np, n0);
  const size_t l64 = al((size_t)np * np * 8);
  const size_t l32 = al((size_t)np * np * 4);
  const size_t blk64 = al((size_t)m * n0 * n0 * 8), blk32 = al((size_t)m * n0 * n0 * 4);
  if (prec == TRSM_F64) return l64 + blk64 + al(8) + (chol ? l64 + blk64 : 0);
  return l64 + l32 + blk32 + (chol ? l64 + l32 + blk32 : 0);
}

// Internal buffers of a request are np x kp, kp = round_up(k, 4) (zero
// padded) so that every product takes the 16-byte vector path.
struct ReqBufs {
  double* B64; double* X64; double* R64;
  void* D;        // the correction (binary32 or binary64)
  void* E;        // Cholesky: the forward sweep's output
  double* T64;    // Cholesky: L^T X
  float* Rl;      // binary32: the scaled running right-hand side
  double* part;   // kRedMaxParts x kPartStride partial sums
  double* sc;     // the binary32 conversion scale
  void* split;    // split-K partial products of the request's products
  int64_t split_bytes;
};

// Split-K scratch of a request: what its products would split into with
// unlimited scratch (its binary64 residual, its Cholesky product, its sweep's
// diagonal-block products), capped at max(64 np kp, 4 MiB) bytes.  A function
// of the request's own shape only, so its products split the same way in any
// batch.
int64_t split_bytes_for(const Factor& f, int64_t kp) {
  const int np = (int)f.np, N = (int)kp, b = (int)std::min(f.n0, f.np);
  const int elem = f.prec == TRSM_F64 ? 8 : 4;
  const int64_t inf = INT64_MAX / 4;
  int64_t need = grouped_split_slices(np, N, np, G_A_LOWER | G_BETA, inf, 8) * (int64_t)np * N * 8;
  if (f.chol)
    need = std::max<int64_t>(need, grouped_split_slices(np, N, np, G_A_UPPER, inf, 8) *
                                       (int64_t)np * N * 8);
  need = std::max<int64_t>(need, grouped_split_slices(b, N, b, G_A_LOWER, inf, elem) *
                                     (int64_t)b * N * elem);
  return std::min<int64_t>(need, std::max<int64_t>(64 * (int64_t)np * kp, 4 << 20));
}

size_t layout(const Factor& f, int64_t kp, char* p, ReqBufs* b) {
  const int64_t n = f.np;
  const size_t m64 = al((size_t)n * kp * 8), m32 = al((size_t)n * kp * 4);
  const size_t mw = f.prec == TRSM_F64 ? m64 : m32;
  char* q = p;
  ReqBufs r{};
  r.B64 = (double*)q; q += m64;
  r.X64 = (double*)q; q += m64;
  r.R64 = (double*)q; q += m64;
  r.D = q;            q += mw;
  if (f.prec == TRSM_F32) { r.Rl = (float*)q; q += m32; }
  if (f.chol) {
    r.E = q;          q += mw;
    r.T64 = (double*)q; q += m64;
  }
  r.part = (double*)q; q += al((size_t)kRedMaxParts * kPartStride * 8);
  r.sc = (double*)q;   q += al(8);
  r.split_bytes = split_bytes_for(f, kp);
  r.split = q;         q += al((size_t)r.split_bytes);
  if (b) *b = r;
  return (size_t)(q - p);
}

size_t request_bytes(const Factor& f, int64_t kp) { return layout(f, kp, nullptr, nullptr); }

// The lists of one pass over a group of requests, in launch order.
struct PassLists {
  std::vector<RedEntry> load, red1, norms;
  std::vector<EwEntry> conv0, x0, conv, add;
  std::vector<SweepItem<float>> f1_32, b1_32, f2_32, b2_32;
  std::vector<SweepItem<double>> f1_64, b1_64, f2_64, b2_64;
  std::vector<GemmP64> u1, r1, u2, r2;
  std::vector<FinEntry> fin;
};

template <typename T>
SweepItem<T> sweep_item(const Factor& f, bool upper, int64_t kp, const void* B, void* R, void* X,
                        const ReqBufs& b) {
  SweepItem<T> it{};
  it.n = f.np; it.k = kp; it.n0 = f.n0;
  it.part = b.split; it.part_bytes = b.split_bytes;
  if constexpr (std::is_same<T, double>::value) {
    it.L = upper ? f.U64 : f.L64; it.ldl = f.ld64;
    it.Linv = upper ? f.Uinv64 : f.Linv64;
  } else {
    it.L = upper ? f.U32 : f.L32; it.ldl = f.ld32;
    it.Linv = upper ? f.Uinv32 : f.Linv32;
  }
  it.B = (const T*)B; it.ldb = kp;
  it.R = (T*)R; it.ldr = kp;
  it.X = (T*)X; it.ldx = kp;
  return it;
}

// One sweep of a request: rhs -> out (forward with L; for A = L L^T also the
// backward sweep with U = L^T through E).  `work` is the forward sweep's
// running right-hand side (it may be rhs itself when rhs may be destroyed).
void add_sweep(PassLists& pl, bool second, const Factor& f, int64_t kp, const void* rhs,
               void* work, void* out, const ReqBufs& b) {
  void* E = b.E;
  if (f.prec == TRSM_F64) {
    auto& fw = second ? pl.f2_64 : pl.f1_64;
    auto& bw = second ? pl.b2_64 : pl.b1_64;
    if (!f.chol) {
      fw.push_back(sweep_item<double>(f, false, kp, rhs, work, out, b));
    } else {
      fw.push_back(sweep_item<double>(f, false, kp, rhs, work, E, b));
      bw.push_back(sweep_item<double>(f, true, kp, E, E, out, b));
    }
  } else {
    auto& fw = second ? pl.f2_32 : pl.f1_32;
    auto& bw = second ? pl.b2_32 : pl.b1_32;
    if (!f.chol) {
      fw.push_back(sweep_item<float>(f, false, kp, rhs, work, out, b));
    } else {
      fw.push_back(sweep_item<float>(f, false, kp, rhs, work, E, b));
      bw.push_back(sweep_item<float>(f, true, kp, E, E, out, b));
    }
  }
}

// R = B - L X (binary64); for A = L L^T first T = L^T X.
void add_residual(PassLists& pl, bool second, const Factor& f, int64_t kp, const ReqBufs& b) {
  const int n = (int)f.np;
  const double* prod = b.X64;
  if (f.chol) {
    auto q = gemm_params<double, double, double, float>();
    q.A = f.U64; q.lda = f.ld64;
    q.B = b.X64; q.ldb = kp;
    q.Cout = b.T64; q.ldco = kp;
    q.M = n; q.N = (int)kp; q.K = n;
    q.flags = G_A_UPPER;
    q.part = b.split; q.part_bytes = b.split_bytes;
    (second ? pl.u2 : pl.u1).push_back(q);
    prod = b.T64;
  }
  auto p = gemm_params<double, double, double, float>();
  p.A = f.L64; p.lda = f.ld64;
  p.B = prod; p.ldb = kp;
  p.Cin = b.B64; p.ldci = kp;
  p.Cout = b.R64; p.ldco = kp;
  p.M = n; p.N = (int)kp; p.K = n;
  p.alpha = -1.0; p.beta = 1.0;
  p.flags = G_A_LOWER | G_BETA;
  p.part = b.split; p.part_bytes = b.split_bytes;
  (second ? pl.r2 : pl.r1).push_back(p);
}

EwEntry ew(const void* src, int64_t lds, void* dst, int64_t ldd, int rows, int cols, int op,
           int valid, const double* part = nullptr, int nparts = 0, double* sc = nullptr) {
  EwEntry e{};
  e.src = src; e.lds = lds; e.dst = dst; e.ldd = ldd;
  e.rows = rows; e.cols = cols; e.scale = 1.0; e.op = op; e.valid_cols = valid;
  e.part = part; e.nparts = nparts; e.sc = sc;
  return e;
}

RedEntry red(int op, int rows, int cols, int valid_rows, int valid, const double* a, int64_t lda,
             double* part) {
  RedEntry e{};
  e.op = op; e.rows = rows; e.cols = cols; e.valid_rows = valid_rows; e.valid_cols = valid;
  e.a = a; e.lda = lda; e.part = part;
  red_split(rows, cols, &e.chunk, &e.nparts);
  return e;
}

void record_request(trsm_server_s* S, const Request& r, PassLists& pl) {
  const Factor& f = *r.f;
  ReqBufs b;
  layout(f, r.kp, S->base + r.ws_off, &b);
  const int n = (int)f.np, nv = (int)f.n, k = (int)r.k;
  const int64_t kp = r.kp;
  const bool f32 = f.prec == TRSM_F32;
  const bool first = r.passes == 0;
  int chunk, nparts;
  red_split(n, kp, &chunk, &nparts);
  if (first) {
    RedEntry e = red(RD_LOAD, n, (int)kp, nv, k, r.B, r.ldb, b.part);
    e.b = b.B64; e.ldb = kp;
    pl.load.push_back(e);
    if (f32) {
      // X_0 = sweep(s B) / s
      pl.conv0.push_back(ew(b.B64, kp, b.Rl, kp, n, (int)kp, EW_F64_TO_F32_PS, (int)kp, b.part,
                            nparts, b.sc));
      add_sweep(pl, false, f, kp, b.Rl, b.Rl, b.D, b);
      pl.x0.push_back(ew(b.D, kp, b.X64, kp, n, (int)kp, EW_F32_TO_F64_SET_SC, (int)kp, nullptr, 0,
                         b.sc));
      add_residual(pl, false, f, kp, b);
      pl.red1.push_back(red(RD_RES, n, (int)kp, n, (int)kp, b.R64, kp, b.part));
    } else {
      // X_0 = sweep(B); the sweep's running right-hand side lives in R
      add_sweep(pl, false, f, kp, b.B64, b.R64, b.X64, b);
      add_residual(pl, false, f, kp, b);
    }
  }
  const bool correct = f32 || !first;
  if (correct) {
    if (f32) {
      pl.conv.push_back(ew(b.R64, kp, b.Rl, kp, n, (int)kp, EW_F64_TO_F32_PS, (int)kp, b.part,
                           nparts, b.sc));
      add_sweep(pl, true, f, kp, b.Rl, b.Rl, b.D, b);
      pl.add.push_back(ew(b.D, kp, b.X64, kp, n, (int)kp, EW_F32_TO_F64_ADD_SC, (int)kp, nullptr, 0,
                          b.sc));
    } else {
      add_sweep(pl, true, f, kp, b.R64, b.R64, b.D, b);
      pl.add.push_back(ew(b.D, kp, b.X64, kp, n, (int)kp, EW_F64_ADD, (int)kp));
    }
    add_residual(pl, true, f, kp, b);
  }
  RedEntry e = red(RD_NORMS, n, (int)kp, nv, k, b.R64, kp, b.part);
  e.b = b.X64; e.ldb = kp;
  e.d = correct ? b.D : nullptr;
  e.ldd = kp;
  e.d_f64 = f32 ? 0 : 1;
  e.xo = r.X; e.ldxo = r.ldx;
  pl.norms.push_back(e);
  FinEntry fe{};
  fe.part = b.part;
  fe.sc = correct && f32 ? b.sc : nullptr;
  fe.out = S->hstat_dev + kStatRow * r.slot;
  fe.nparts = nparts;
  pl.fin.push_back(fe);
}

// Record one pass of every request in `reqs`.  With n0 = kPB the sweeps are
// persistent launches that share the counter words at `counters` (each
// launch clears them first; same stream).
void record_batch(trsm_server_s* S, const std::vector<std::shared_ptr<Request>>& reqs,
                  LaunchList& list, unsigned* counters) {
  PassLists pl;
  for (const auto& rp : reqs) record_request(S, *rp, pl);
  const bool persist = S->n0 == kPB;
  auto sweeps = [&](const std::vector<SweepItem<float>>& f32, const std::vector<SweepItem<double>>& f64,
                    const std::vector<SweepItem<float>>& b32, const std::vector<SweepItem<double>>& b64) {
    if (persist) {
      if (!f32.empty()) record_persist<float>(list, f32, counters);
      if (!f64.empty()) record_persist<double>(list, f64, counters);
    } else {
      record_sweep<float>(list, f32);
      record_sweep<double>(list, f64);
    }
    record_sweep_back<float>(list, b32);
    record_sweep_back<double>(list, b64);
  };
  list.clear();
  list.add_red(pl.load);
  list.add_ew(pl.conv0);
  sweeps(pl.f1_32, pl.f1_64, pl.b1_32, pl.b1_64);
  list.add_ew(pl.x0);
  list.add_gemm64(pl.u1);
  list.add_gemm64(pl.r1);
  list.add_red(pl.red1);
  list.add_ew(pl.conv);
  sweeps(pl.f2_32, pl.f2_64, pl.b2_32, pl.b2_64);
  list.add_ew(pl.add);
  list.add_gemm64(pl.u2);
  list.add_gemm64(pl.r2);
  list.add_red(pl.norms);
  list.add_fin(pl.fin);
}

// Counter words of a group's persistent sweeps (0 when the server sweeps by
// phases): enough for the largest single launch.
size_t counter_bytes(trsm_server_s* S, const std::vector<std::shared_ptr<Request>>& reqs) {
  if (S->n0 != kPB) return 0;
  int64_t tiles = 0;
  for (const auto& rp : reqs) tiles += ceil_div(rp->kp, kPB);
  return (size_t)(tiles + 2) * 4;
}

double request_flops(const Request& r) {
  const double n = (double)r.f->n;
  return (r.f->chol ? 2.0 : 1.0) * n * n * (double)r.k;
}

// Retire a request (lock held).
void finish(trsm_server_s* S, Request& r, int status, bool error) {
  r.state = error ? TRSM_REQ_ERROR : TRSM_REQ_DONE;
  r.status = status;
  r.t_done = now_us();
  if (r.ws_off != SIZE_MAX) S->arena.release(r.ws_off);
  r.ws_off = SIZE_MAX;
  if (r.slot >= 0) {
    S->free_slots.push_back(r.slot);
    S->slots_used -= 1;
  }
  r.slot = -1;
  if (error) {
    S->failed += 1;
    return;
  }
  S->completed += 1;
  if (status == TRSM_ENOTCONVERGED) S->unconverged += 1;
  S->lat_us.push_back(r.t_done - r.t_submit);
  S->flops_done += request_flops(r);
  S->t_last = r.t_done;
}

// The stopping test after a pass (lock held): finish the request or queue
// its next pass.
void after_pass(trsm_server_s* S, const std::shared_ptr<Request>& rp) {
  Request& r = *rp;
  const Factor& f = *r.f;
  const double* st = S->hstat + kStatRow * r.slot;
  // sums of squares s 4^x: log2 of the norms (-inf for a zero sum)
  auto lg = [](double s, double x) { return 0.5 * std::log2(s) + x; };
  const double lr = lg(st[0], st[1]), lx = lg(st[2], st[3]), ld = lg(st[4], st[5]);
  const bool finite = std::isfinite(st[0]) && std::isfinite(st[2]) && std::isfinite(st[4]);
  const bool corrected = !(f.prec == TRSM_F64 && r.passes == 0);
  r.passes += 1;
  S->passes += 1;
  if (corrected) r.corrections += 1;
  const double llnorm = std::log2(f.lnorm) * (f.chol ? 2.0 : 1.0);   // ||L|| (||L||^2 for L L^T)
  const bool rzero = st[0] == 0.0, xzero = st[2] == 0.0;
  const double berr = rzero ? 0.0 : xzero ? HUGE_VAL : std::exp2(lr - lx - llnorm);
  double corr = -1.0;
  if (corrected) corr = st[4] == 0.0 ? 0.0 : xzero ? HUGE_VAL : std::exp2(ld - lx);
  r.info.iterations = r.corrections;
  r.info.backward_error = berr;
  r.info.correction = corr;
  if (corrected && r.corrections == 1) r.info.unrefined_error = corr;
  if (!finite) {
    finish(S, r, TRSM_ENOTCONVERGED, false);
    return;
  }
  const double tol = S->tol > 0.0 ? S->tol : std::sqrt((double)f.n) * std::ldexp(1.0, -53);
  bool done = rzero || berr <= tol;
  if (!done && corrected) {
    done = corr <= 1e-15;
    if (!done && r.prev_corr > 0.0) {
      const double rho = corr / r.prev_corr;
      done = rho <= 0.5 && corr * rho <= 1e-14;
    }
  }
  if (corrected) r.prev_corr = corr;
  if (done) {
    r.info.converged = 1;
    finish(S, r, TRSM_OK, false);
  } else if (r.corrections >= S->max_corr) {
    finish(S, r, TRSM_ENOTCONVERGED, false);
  } else {
    S->ready.push_back(rp);
  }
}

// Split the ready requests (sorted by work) into at most g groups of about
// equal count, so that small requests share fast batches and large ones
// share slow ones.
std::vector<std::vector<std::shared_ptr<Request>>> partition(std::vector<std::shared_ptr<Request>> v,
                                                             size_t g) {
  std::stable_sort(v.begin(), v.end(), [](const std::shared_ptr<Request>& a,
                                          const std::shared_ptr<Request>& b) {
    return request_flops(*a) * (double)a->kp / (double)a->k <
           request_flops(*b) * (double)b->kp / (double)b->k;
  });
  g = std::min(g, v.size());
  std::vector<std::vector<std::shared_ptr<Request>>> out(g);
  for (size_t i = 0; i < g; ++i) {
    const size_t lo = v.size() * i / g, hi = v.size() * (i + 1) / g;
    out[i].assign(v.begin() + lo, v.begin() + hi);
  }
  return out;
}

// Release a batch's device memory (lock held).
void release_batch(trsm_server_s* S, Batch& b) {
  if (b.table_off != SIZE_MAX) S->arena.release(b.table_off);
  if (b.cnt_off != SIZE_MAX) S->arena.release(b.cnt_off);
  b.table_off = b.cnt_off = SIZE_MAX;
  b.reqs.clear();
  b.busy = false;
}

// Record, upload and launch a batch on stream i (worker thread, lock not
// held; the stream is idle).
int launch_batch(trsm_server_s* S, int i) {
  Batch& b = S->batch[i];
  LaunchList list;
  const size_t cb = counter_bytes(S, b.reqs);
  if (cb) {
    std::lock_guard<std::mutex> g(S->mu);
    b.cnt_off = S->arena.alloc(cb);
    if (b.cnt_off == SIZE_MAX) return TRSM_ENOMEM;
  }
  unsigned* counters = cb ? (unsigned*)(S->base + b.cnt_off) : nullptr;
  record_batch(S, b.reqs, list, counters);
  const size_t tb = list.table_bytes();
  {
    std::lock_guard<std::mutex> g(S->mu);
    b.table_off = S->arena.alloc(tb);
    if (b.table_off == SIZE_MAX) return TRSM_ENOMEM;
  }
  if (S->stage_cap[i] < tb) {
    if (S->stage[i]) (void)hipHostFree(S->stage[i]);
    S->stage[i] = nullptr;
    S->stage_cap[i] = 0;
    const size_t cap = std::max<size_t>(tb * 2, 1 << 16);
    hipError_t e = hipHostMalloc((void**)&S->stage[i], cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      S->stage[i] = nullptr;
      note_hip_error(e);
      return TRSM_EHIP;
    }
    S->stage_cap[i] = cap;
  }
  memcpy(S->stage[i], list.host_table(), tb);
  hipStream_t s = S->streams[i];
  char* dev = S->base + b.table_off;
  hipError_t e = hipMemcpyAsync(dev, S->stage[i], tb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = list.run(dev, s);
  if (e == hipSuccess) e = hipEventRecord(S->events[i], s);
  if (e != hipSuccess) {
    note_hip_error(e);
    return TRSM_EHIP;
  }
  return TRSM_OK;
}

// One pass of the worker: retire completed batches (stopping tests), admit
// queued requests while slots and memory allow, and launch the ready
// requests on the idle streams.
bool worker_tick(trsm_server_s* S) {
  std::vector<int> launch;
  bool progressed = false;
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (int i = 0; i < kStreams; ++i) {
      Batch& b = S->batch[i];
      if (!b.busy) continue;
      const hipError_t q = hipEventQuery(S->events[i]);
      if (q == hipErrorNotReady) continue;
      std::atomic_thread_fence(std::memory_order_acquire);
      progressed = true;
      for (auto& rp : b.reqs) {
        if (q == hipSuccess) after_pass(S, rp);
        else finish(S, *rp, note_hip_error(q), true);
      }
      release_batch(S, b);
    }
    while (!S->pending.empty() && S->slots_used < S->max_slots) {
      auto rp = S->pending.front();
      const size_t need = request_bytes(*rp->f, rp->kp);
      const size_t off = S->arena.alloc(need);
      if (off == SIZE_MAX) {
        // cannot fit now; if it can never fit (nothing else holds memory), fail it
        bool idle = S->ready.empty();
        for (int i = 0; i < kStreams; ++i) idle &= !S->batch[i].busy;
        if (idle) {
          S->pending.pop_front();
          finish(S, *rp, TRSM_ENOMEM, true);
          progressed = true;
          continue;
        }
        break;
      }
      rp->ws_off = off;
      rp->ws_bytes = need;
      rp->slot = S->free_slots.back();
      S->free_slots.pop_back();
      rp->state = TRSM_REQ_RUNNING;
      S->pending.pop_front();
      S->slots_used += 1;
      S->ready.push_back(rp);
    }
    S->max_inflight_slots = std::max(S->max_inflight_slots, S->slots_used);
    std::vector<int> idle;
    for (int i = 0; i < kStreams; ++i)
      if (!S->batch[i].busy) idle.push_back(i);
    if (idle.empty() || S->ready.empty()) return progressed;
    std::vector<std::shared_ptr<Request>> all(S->ready.begin(), S->ready.end());
    S->ready.clear();
    auto groups = partition(std::move(all), idle.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      Batch& b = S->batch[idle[gi]];
      b.reqs = std::move(groups[gi]);
      b.busy = true;
      launch.push_back(idle[gi]);
    }
    S->batches += groups.size();
  }
  bool retry = false;
  for (int i : launch) {
    const int st = launch_batch(S, i);
    if (st == TRSM_OK) continue;
    std::lock_guard<std::mutex> g(S->mu);
    Batch& b = S->batch[i];
    if (st == TRSM_ENOMEM) {
      // no room for the batch's launch table: run it once other batches
      // have released memory (fail it only if nothing else is running)
      bool others = false;
      for (int j = 0; j < kStreams; ++j) others |= j != i && S->batch[j].busy;
      if (others) {
        for (auto it = b.reqs.rbegin(); it != b.reqs.rend(); ++it) S->ready.push_front(*it);
        S->batches -= 1;
        release_batch(S, b);
        retry = true;
        continue;
      }
    } else {
      // anything already enqueued on the stream must drain before its
      // memory is reused
      (void)hipStreamSynchronize(S->streams[i]);
    }
    for (auto& rp : b.reqs) finish(S, *rp, st, true);
    release_batch(S, b);
  }
  // a deferred batch waits for a completion instead of spinning
  return !retry;
}

void worker_main(trsm_server_s* S) {
  (void)hipSetDevice(S->device);
  // short waits must stay short (the default timer slack is 50 us)
  (void)prctl(PR_SET_TIMERSLACK, 1UL, 0, 0, 0);
  for (;;) {
    const bool busy = worker_tick(S);
    std::unique_lock<std::mutex> lk(S->mu);
    bool inflight = false;
    for (int i = 0; i < kStreams; ++i) inflight |= S->batch[i].busy;
    if (S->stop && S->pending.empty() && S->ready.empty() && !inflight) break;
    if (!busy) {
      // wake on a new request, or poll in-flight batches every 10 us
      S->cv.wait_for(lk, std::chrono::microseconds(inflight ? 10 : 2000));
    }
  }
}

void destroy_resources(trsm_server_s* S) {
  for (int i = 0; i < kStreams; ++i) {
    if (S->streams[i]) {
      (void)hipStreamSynchronize(S->streams[i]);
      (void)hipStreamDestroy(S->streams[i]);
    }
    if (S->events[i]) (void)hipEventDestroy(S->events[i]);
    if (S->stage[i]) (void)hipHostFree(S->stage[i]);
  }
  if (S->reg_stream) {
    (void)hipStreamSynchronize(S->reg_stream);
    (void)hipStreamDestroy(S->reg_stream);
  }
  if (S->hstat) (void)hipHostFree(S->hstat);
  if (S->base) (void)hipFree(S->base);
}

trsm_status create_server(size_t hbm_budget, int32_t max_slots, const trsm_server_options* opt,
                          trsm_server_t* out) {
  if (!out) return TRSM_EINVAL;
  *out = nullptr;
  if (max_slots <= 0 || max_slots > (1 << 20) || hbm_budget < (1u << 20)) return TRSM_EINVAL;
  int64_t n0 = kDefaultN0;
  double tol = 0.0;
  int max_corr = kDefaultMaxCorr;
  if (opt) {
    if (opt->reserved != 0 || opt->n0 < 0 || (opt->n0 & (opt->n0 - 1)) ||
        !(opt->tolerance >= 0.0) || opt->max_corrections < 0 ||
        opt->max_corrections > kMaxCorrLimit)
      return TRSM_EINVAL;
    if (opt->n0) n0 = opt->n0;
    tol = opt->tolerance;
    if (opt->max_corrections) max_corr = opt->max_corrections;
  }
  trsm_server_s* S = new (std::nothrow) trsm_server_s();
  if (!S) return TRSM_ENOMEM;
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  S->n0 = n0;
  S->tol = tol;
  S->max_corr = max_corr;
  trsm_status st = TRSM_OK;
  if (hipGetDevice(&S->device) != hipSuccess) st = TRSM_EHIP;
  if (st == TRSM_OK && hipMalloc((void**)&S->base, hbm_budget) != hipSuccess) {
    S->base = nullptr;
    st = TRSM_ENOMEM;
  }
  if (st == TRSM_OK &&
      hipHostMalloc((void**)&S->hstat, (size_t)max_slots * kStatRow * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    S->hstat = nullptr;
    st = TRSM_ENOMEM;
  }
  if (st == TRSM_OK && hipHostGetDevicePointer((void**)&S->hstat_dev, S->hstat, 0) != hipSuccess)
    st = TRSM_EHIP;
  for (int i = 0; st == TRSM_OK && i < kStreams; ++i) {
    if (hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->events[i], hipEventDisableTiming) != hipSuccess)
      st = TRSM_EHIP;
  }
  if (st == TRSM_OK && hipStreamCreateWithFlags(&S->reg_stream, hipStreamNonBlocking) != hipSuccess)
    st = TRSM_EHIP;
  if (st != TRSM_OK) {
    destroy_resources(S);
    delete S;
    return st;
  }
  memset(S->hstat, 0, (size_t)max_slots * kStatRow * sizeof(double));
  S->arena.init(hbm_budget);
  S->free_slots.reserve(max_slots);
  for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  S->worker = std::thread(worker_main, S);
  *out = S;
  return TRSM_OK;
}

// Ones on the padded part of the diagonal: L[i][i] = 1 for n <= i < np.
__global__ void pad_identity_kernel(double* L, int64_t np, int64_t n) {
  const int64_t i = n + threadIdx.x;
  if (i < np) L[i * np + i] = 1.0;
}

trsm_status register_factor(trsm_server_t S, const double* L, int64_t n, int64_t ldl, int prec,
                            bool chol, int32_t* l_id) {
  if (!S || !L || !l_id || n <= 0 || ldl < n || n > (1 << 20)) return TRSM_EINVAL;
  if (prec != TRSM_F32 && prec != TRSM_F64) return TRSM_EINVAL;
  std::lock_guard<std::mutex> reg(S->reg_mu);
  auto fp = std::make_unique<Factor>();
  Factor& f = *fp;
  f.n = n;
  f.np = round_up(n, 4);
  const int64_t np = f.np;
  f.prec = prec;
  f.chol = chol;
  // A = L L^T has the square of L's condition number: binary32 sweeps with
  // inverted blocks of more than kCholMaxN0F32 rows lose too much of their
  // accuracy to it (each correction then gains little)
  f.n0 = effective_n0(np, chol && prec == TRSM_F32 ? std::min<int64_t>(S->n0, kCholMaxN0F32) : S->n0);
  f.m = ceil_div(np, f.n0);
  f.bytes = factor_bytes(np, f.n0, chol, prec);
  // temporaries: the binary64 inverses of a binary32 factor, and the norm's partial sums
  const size_t inv64 = al((size_t)f.m * f.n0 * f.n0 * 8) + al(8);
  const size_t tmp_bytes = (prec == TRSM_F32 ? inv64 : 0) + al(2 * kNormBlocks * 8) + al(16);
  size_t tmp_off = SIZE_MAX;
  {
    std::lock_guard<std::mutex> g(S->mu);
    f.off = S->arena.alloc(f.bytes);
    if (f.off != SIZE_MAX) {
      tmp_off = S->arena.alloc(tmp_bytes);
      if (tmp_off == SIZE_MAX) S->arena.release(f.off);
    }
  }
  if (f.off == SIZE_MAX || tmp_off == SIZE_MAX) return TRSM_ENOMEM;
  char* p = S->base + f.off;
  const size_t blk64 = al((size_t)f.m * f.n0 * f.n0 * 8), blk32 = al((size_t)f.m * f.n0 * f.n0 * 4);
  f.ld64 = np;
  f.ld32 = np;
  const size_t l64 = al((size_t)np * np * 8), l32 = al((size_t)np * np * 4);
  f.L64 = (double*)p; p += l64;
  if (prec == TRSM_F64) {
    f.Linv64 = (double*)p; p += blk64 + al(8);
    if (chol) {
      f.U64 = (double*)p; p += l64;
      f.Uinv64 = (double*)p; p += blk64;
    }
  } else {
    f.L32 = (float*)p; p += l32;
    f.Linv32 = (float*)p; p += blk32;
    if (chol) {
      f.U64 = (double*)p; p += l64;
      f.U32 = (float*)p; p += l32;
      f.Uinv32 = (float*)p; p += blk32;
    }
  }
  char* t = S->base + tmp_off;
  double* inv = prec == TRSM_F64 ? f.Linv64 : (double*)t;
  if (prec == TRSM_F32) t += inv64;
  double* npart = (double*)t;
  double* nout = (double*)(t + al(2 * kNormBlocks * 8));

  hipStream_t s = S->reg_stream;
  trsm_plan_t plan = nullptr;
  trsm_status st = trsm_plan(np, 1, TRSM_F64, f.n0, 0, &plan);   // the factor's own block size
  hipError_t e = hipSuccess;
  double lsq = 0.0;
  if (st == TRSM_OK) {
    trsm_plan_info pi;
    st = trsm_plan_get_info(plan, &pi);
    if (st == TRSM_OK && pi.linv_bytes > inv64) st = TRSM_EINVAL;
  }
  if (st == TRSM_OK) {
    // L64 = [L 0; 0 I] (np x np), L32 its binary32 copy
    e = launch_fill_u32((unsigned*)f.L64, np * np * 2, 0u, s);
    if (e == hipSuccess) e = launch_copy2d<double, double>(L, ldl, f.L64, np, n, n, 1.0, s);
    if (e == hipSuccess && np > n) {
      pad_identity_kernel<<<1, 64, 0, s>>>(f.L64, np, n);
      e = hipGetLastError();
    }
    if (e == hipSuccess && prec == TRSM_F32)
      e = launch_copy2d<double, float>(f.L64, np, f.L32, np, np, np, 1.0, s);
    if (e == hipSuccess) e = launch_sumsq_lower<double>(f.L64, np, n, npart, nout, s);
    if (e == hipSuccess) st = trsm_invert_diag(plan, f.L64, f.ld64, inv, s);
    if (st == TRSM_OK && e == hipSuccess && prec == TRSM_F32)
      e = launch_convert<double, float>(inv, f.Linv32, f.m * f.n0 * f.n0, s);
    if (chol && st == TRSM_OK && e == hipSuccess) {
      // U = L^T (zeros below the diagonal) and Uinv_ii = Linv_ii^T
      e = launch_transpose<double, double>(f.L64, np, f.U64, np, np, np, 1, 0, 0, true, s);
      if (e == hipSuccess && prec == TRSM_F32)
        e = launch_transpose<float, float>(f.L32, np, f.U32, np, np, np, 1, 0, 0, true, s);
      if (e == hipSuccess && prec == TRSM_F32)
        e = launch_transpose<float, float>(f.Linv32, f.n0, f.Uinv32, f.n0, f.n0, f.n0, f.m,
                                           f.n0 * f.n0, f.n0 * f.n0, false, s);
      if (e == hipSuccess && prec == TRSM_F64)
        e = launch_transpose<double, double>(f.Linv64, f.n0, f.Uinv64, f.n0, f.n0, f.n0, f.m,
                                             f.n0 * f.n0, f.n0 * f.n0, false, s);
    }
    if (st == TRSM_OK && e == hipSuccess)
      e = hipMemcpyAsync(&lsq, nout, sizeof(double), hipMemcpyDeviceToHost, s);
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
  // the stopping test divides by ||L||_F: its square must be a normal binary64
  if (st == TRSM_OK && !(lsq >= 2.2250738585072014e-308 && std::isfinite(lsq))) st = TRSM_EINVAL;
  if (e != hipSuccess) note_hip_error(e);
  (void)hipStreamSynchronize(s);   // nothing in flight reads the temporaries
  f.lnorm = std::sqrt(lsq);
  std::lock_guard<std::mutex> g(S->mu);
  S->arena.release(tmp_off);
  if (st != TRSM_OK) {
    S->arena.release(f.off);
    return st;
  }
  S->factors.push_back(std::move(fp));
  *l_id = (int32_t)S->factors.size() - 1;
  return TRSM_OK;
}

}  // namespace

extern "C" {

trsm_status trsm_server_create(size_t hbm_budget, int32_t max_slots, trsm_server_t* out) {
  return create_server(hbm_budget, max_slots, nullptr, out);
}

trsm_status trsm_server_create_ex(size_t hbm_budget, int32_t max_slots,
                                  const trsm_server_options* options, trsm_server_t* out) {
  if (!options) {
    if (out) *out = nullptr;
    return TRSM_EINVAL;
  }
  return create_server(hbm_budget, max_slots, options, out);
}

trsm_status trsm_server_register_L(trsm_server_t S, const double* L, int64_t n, int64_t ldl,
                                   trsm_precision prec, int32_t* l_id) {
  return register_factor(S, L, n, ldl, (int)prec, false, l_id);
}

trsm_status trsm_server_register_chol(trsm_server_t S, const double* L, int64_t n, int64_t ldl,
                                      trsm_precision prec, int32_t* l_id) {
  return register_factor(S, L, n, ldl, (int)prec, true, l_id);
}

trsm_status trsm_serve_submit(trsm_server_t S, int32_t l_id, const double* B, int64_t k,
                              int64_t ldb, double* X, int64_t ldx, uint64_t* ticket) {
  if (!S || !ticket || !B || !X || k <= 0 || k > (1 << 24) || ldb < k || ldx < k)
    return TRSM_EINVAL;
  auto r = std::make_shared<Request>();
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (l_id < 0 || l_id >= (int32_t)S->factors.size()) return TRSM_EINVAL;
    const Factor* f = S->factors[l_id].get();
    const int64_t n = f->n;
    const uintptr_t b0 = (uintptr_t)B, b1 = b0 + ((size_t)(n - 1) * ldb + k) * 8;
    const uintptr_t x0 = (uintptr_t)X, x1 = x0 + ((size_t)(n - 1) * ldx + k) * 8;
    if (b0 < x1 && x0 < b1) return TRSM_EINVAL;
    r->ticket = S->next_ticket++;
    r->f = f;
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

trsm_status trsm_serve_request_bytes(trsm_server_t S, int32_t l_id, int64_t k, size_t* bytes) {
  if (!S || !bytes || k <= 0 || k > (1 << 24)) return TRSM_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  if (l_id < 0 || l_id >= (int32_t)S->factors.size()) return TRSM_EINVAL;
  *bytes = request_bytes(*S->factors[l_id], round_up(k, 4));
  return TRSM_OK;
}

trsm_status trsm_serve_poll(trsm_server_t S, uint64_t ticket, trsm_req_state* state,
                            trsm_info* info) {
  if (!S || !state) return TRSM_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) {
    *state = TRSM_REQ_UNKNOWN;
    return TRSM_EINVAL;
  }
  const Request& r = *it->second;
  *state = (trsm_req_state)r.state;
  if (r.state == TRSM_REQ_DONE || r.state == TRSM_REQ_ERROR) {
    if (info) *info = r.info;
    const trsm_status st = (trsm_status)r.status;
    S->all.erase(it);   // a finished ticket is reported once
    return st;
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
  st->unconverged = S->unconverged;
  st->passes = S->passes;
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
  for (const auto& f : S->factors) res += f->bytes;
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
  S->completed = S->failed = S->submitted = S->batches = S->unconverged = S->passes = 0;
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
  destroy_resources(S);
  delete S;
  return TRSM_OK;
}

}  // extern "C"
