// Host runtime and C ABI of the gfx950 inversion-based triangular solver.
//
// trsm_plan        : block size n0 and buffer layout (Sec. VIII rule reported,
//                    a one-GPU cost model chooses).
// trsm_invert_diag : Alg. Diagonal-Inverter with Alg. RecTriInv per block.
// trsm_solve       : the blocked forward sweep of Alg. It-Inv-TRSM
//                    (right-looking with the deferred update of B), the
//                    recursive baseline (Alg. Rec-TRSM order), or the mixed
//                    precision sweep with iterative refinement.
// trsm_residual    : B - L X in binary64 plus deterministic norms.
#include "../../include/trsm.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "crt.hpp"
#include "gemm.hpp"
#include "kernels.hpp"
#include "lpgemm.hpp"
#include "tune.hpp"

using namespace trsm;

namespace {

thread_local int g_last_hip = 0;

inline trsm_status hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return TRSM_EHIP;
}

}  // namespace

int trsm::note_hip_error(hipError_t e) {
  g_last_hip = (int)e;
  return (int)TRSM_EHIP;
}

namespace {

#define TRSM_HIP(...)                           \
  do {                                          \
    hipError_t e_ = (__VA_ARGS__);              \
    if (e_ != hipSuccess) return hip_fail(e_);  \
  } while (0)

#define TRSM_TRY(...)                           \
  do {                                          \
    trsm_status s_ = (__VA_ARGS__);             \
    if (s_ != TRSM_OK) return s_;               \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
inline int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}
inline int64_t prev_pow2(int64_t v) {
  int64_t p = 1;
  while (p * 2 <= v) p <<= 1;
  return p;
}

inline size_t elem_size(trsm_precision p) { return p == TRSM_F32 ? 4 : 8; }
inline bool is_mixed(trsm_precision p) {
  return p == TRSM_MIXED_BF16 || p == TRSM_MIXED_F16 || p == TRSM_MIXED_FP8;
}

}  // namespace

// Optional per-plan timing of the matrix-core launches: each launch is
// bracketed by two hipEvents on its stream; the elapsed times are summed when
// the host asks for them (after synchronising).
struct LaunchTimer {
  bool enabled = false;
  std::vector<hipEvent_t> ev;   // 2 per record, reused
  std::vector<double> flops;    // algorithmic flops per record
  size_t used = 0;

  hipError_t begin(hipStream_t s) {
    if (2 * used + 2 > ev.size()) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
      }
    }
    return hipEventRecord(ev[2 * used], s);
  }
  hipError_t end(hipStream_t s, double f) {
    hipError_t r = hipEventRecord(ev[2 * used + 1], s);
    if (r != hipSuccess) return r;
    if (flops.size() <= used) flops.resize(used + 1);
    flops[used] = f;
    ++used;
    return hipSuccess;
  }
  void release() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    flops.clear();
    used = 0;
  }
};

namespace {
thread_local LaunchTimer* g_timer = nullptr;

struct TimerScope {
  LaunchTimer* prev;
  explicit TimerScope(LaunchTimer* t) : prev(g_timer) { g_timer = (t && t->enabled) ? t : nullptr; }
  ~TimerScope() { g_timer = prev; }
};

// Split-K scratch for the products launched inside one library call (the
// caller's workspace, or the plan's own buffer during the inversion).
struct SplitBuf {
  void* ptr = nullptr;
  int64_t bytes = 0;
};
thread_local SplitBuf g_split;

// Tile policy of the current call (TRSM_FLAG_LARGE_TILES: 128 x 128 only).
thread_local bool g_large_tiles = false;

struct TilePolicyScope {
  bool prev;
  explicit TilePolicyScope(bool large) : prev(g_large_tiles) { g_large_tiles = large; }
  ~TilePolicyScope() { g_large_tiles = prev; }
};

struct SplitScope {
  SplitBuf prev;
  SplitScope(void* p, int64_t b) : prev(g_split) { g_split = SplitBuf{p, b}; }
  ~SplitScope() { g_split = prev; }
};

template <typename P>
void use_split(P& p) {
  if (!p.part) {
    p.part = g_split.ptr;
    p.part_bytes = g_split.bytes;
  }
}

// Scratch for split-K partial products: up to kSplitMax slices of an
// output of `elems` elements (binary64 partials), at most 128 MiB.
constexpr size_t kSplitCap = (size_t)128 << 20;
size_t split_bytes(int64_t elems) {
  const size_t want = (size_t)kSplitMax * (size_t)std::max<int64_t>(elems, 0) * 8;
  return std::min(want, kSplitCap);
}

template <typename F>
hipError_t timed(double flops, hipStream_t s, F&& launch) {
  LaunchTimer* t = g_timer;
  if (!t) return launch();
  hipError_t e = t->begin(s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return t->end(s, flops);
}

// Algorithmic flops of one (batched) product: 2MNK, or M(M+1)N when A is
// square lower triangular, or MN(N+1) when B is.
template <typename P>
double gemm_flops(const P& p, int batch) {
  const double M = p.M, N = p.N, K = p.K;
  double f;
  if ((p.flags & (G_A_LOWER | G_A_UPPER)) && p.M == p.K) f = M * (M + 1) * N;
  else if ((p.flags & G_B_LOWER) && p.K == p.N) f = M * N * (N + 1);
  else f = 2.0 * M * N * K;
  return f * batch;
}
}  // namespace

struct trsm_plan_s {
  int64_t n = 0, k = 0, n0 = 1, m = 0, leaf = 1, n0_paper = 1;
  trsm_precision prec = TRSM_F64;
  uint32_t flags = 0;
  // mixed plans: target of the estimated relative forward error of the
  // refined X (0: refine to binary64's backward-error level)
  double tol = 0.0;
  // Linv buffer layout (byte offsets)
  size_t off_linv64 = 0, off_linv32 = 0, off_llow = 0, off_rscale = 0, off_lnorm = 0, off_lpart = 0;
  // transposed plans: U = L^T (n x ldu, upper) and the blocks Uinv_ii = Linv_ii^T
  size_t off_ut = 0, off_uinv = 0;
  int64_t ldu = 0;
  size_t linv_bytes = 0;
  // workspace layout (byte offsets)
  size_t ws_r = 0, ws_r64 = 0, ws_rl = 0, ws_d = 0, ws_xlow = 0, ws_xsc = 0, ws_part = 0,
         ws_norm = 0;
  size_t ws_split = 0, ws_split_bytes = 0;
  // mixed plans: residue planes of L's strictly lower part (Linv buffer) and
  // of the correction pieces and the products (workspace); npad = n rounded
  // up to 64, ldz = k rounded up to 16
  size_t off_crt_e = 0, off_crt_rowmax = 0, off_crt_rowpart = 0, off_crt_stats = 0,
         off_crt_a = 0, off_crt_sl = 0;
  // mixed plans: 16-bit copy of the inverted blocks with one scale per row
  // (the diagonal apply of the first, coarse sweep)
  size_t off_linv16 = 0, off_linv16_rs = 0;
  size_t ws_q = 0, ws_z = 0, ws_colmax = 0, ws_ty = 0, ws_rpart = 0, ws_dpart = 0;
  size_t ws_d1 = 0, ws_d2 = 0;   // the second and third correction pieces
  int64_t npad = 0, ldz = 0;
  size_t ws_bytes = 0;
  // first singular row: a device word inside the caller's Linv buffer (at
  // off_status), written by the last trsm_invert_diag; last_linv remembers
  // that buffer for trsm_plan_last_error
  size_t off_status = 0;
  const void* last_linv = nullptr;
  LaunchTimer timer;
  // lookahead: a second stream and the events that order the two
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> events;
};

// ---------------------------------------------------------------------------
// A0: choice of n0.
// ---------------------------------------------------------------------------
namespace {

// Sec. VIII regime rule at p = 1: n < 4k -> one large dimension, n0 = n;
// n > 4k -> two large dimensions, n0 = (n k^3)^{1/4}; n = 4k -> three large
// dimensions, n0 = min(sqrt(n k), n).
int64_t paper_rule_n0(int64_t n, int64_t k) {
  if (n <= 0) return 1;
  double v;
  if (n < 4 * k) v = (double)n;
  else if (n > 4 * k) v = pow((double)n * (double)k * (double)k * (double)k, 0.25);
  else v = fmin(sqrt((double)n * (double)k), (double)n);
  if (v < 1) v = 1;
  return (int64_t)llround(v);
}

// One-GPU reading of the alpha-beta-gamma model (Sec. II-A): the sweep's n^2 k
// flops do not depend on n0; the inversion adds n n0^2 / 3 flops, and each of
// the ceil(n/n0) dependent steps costs a fixed synchronisation time.
int64_t auto_n0(int64_t n, int64_t k, trsm_precision prec) {
  if (n <= 16) return next_pow2(n < 1 ? 1 : n);
  const double rate = (prec == TRSM_F32) ? 90e12 : 45e12;  // sustained matrix-core rate
  const double t_step = 12e-6;                             // per dependent step
  const double t_level = 10e-6;                            // per inversion level
  int64_t best = 16;
  double best_t = 1e300;
  const int64_t top = next_pow2(n);
  for (int64_t n0 = 16; n0 <= top; n0 <<= 1) {
    const double m = ceil((double)n / (double)n0);
    const double levels = n0 > 64 ? log2((double)n0 / 64.0) : 0.0;
    const double t = (double)n * n0 * n0 / 3.0 / rate + levels * t_level + m * t_step;
    (void)k;
    if (t < best_t) {
      best_t = t;
      best = n0;
    }
  }
  return best;
}

}  // namespace

// ---------------------------------------------------------------------------
// GEMM front-ends (tile shapes per element type).
// ---------------------------------------------------------------------------
namespace {

template <typename T>
struct Gemm {
  using P = GemmParams<T, T, T, float>;
  // Products that give fewer workgroups than two per compute unit with
  // 128 x 128 tiles use 64 x 64 tiles (four times as many workgroups; the
  // binary64/binary32 matrix-core rate per workgroup does not depend on the
  // tile), and split K if they are still small.
  static hipError_t run(const P& p0, int batch, hipStream_t s) {
    P p = p0;
    use_split(p);
    const bool small = !g_large_tiles &&
                       (int64_t)gemm_wgs(p.M, p.N, p.K, p.flags, 128, 128) * batch < kSplitTarget;
    return timed(gemm_flops(p, batch), s, [&] {
      return small ? launch_gemm<T, T, T, float, 64, 64, 2, 2, false>(p, batch, s)
                   : launch_gemm<T, T, T, float, 128, 128, 2, 2, false>(p, batch, s);
    });
  }
};

// C[M x N] = beta*C + alpha * op(A) * op(B), row-major, no batching.
template <typename T>
hipError_t gemm_simple(const T* A, int64_t lda, const T* B, int64_t ldb, const T* Cin,
                       int64_t ldci, T* Cout, int64_t ldco, int64_t M, int64_t N, int64_t K,
                       double alpha, double beta, uint32_t flags, hipStream_t s) {
  auto p = gemm_params<T, T, T, float>();
  p.A = A; p.lda = lda;
  p.B = B; p.ldb = ldb;
  p.Cin = Cin; p.ldci = ldci;
  p.Cout = Cout; p.ldco = ldco;
  p.M = (int)M; p.N = (int)N; p.K = (int)K;
  p.alpha = alpha; p.beta = beta;
  p.flags = flags | (Cin ? G_BETA : 0u);
  return Gemm<T>::run(p, 1, s);
}

bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + abytes, b0 = (uintptr_t)b, b1 = b0 + bbytes;
  return a0 < b1 && b0 < a1;
}

}  // namespace

// ---------------------------------------------------------------------------
// A1: Alg. Diagonal-Inverter / Alg. RecTriInv.
// ---------------------------------------------------------------------------
namespace {

// All levels of the recursive inversion, batched over every pair of every
// block.  At level h the pair [[A11, 0], [A21, A22]] (2h x 2h, A11 and A22
// already inverted) is completed with
//     T   = A22^{-1} A21          (stored in the pair's unused upper-right)
//     A21 = -T A11^{-1}
// which is Alg. RecTriInv's combine, -(Linv22 L21) Linv11, in the paper's
// association order.
hipError_t rec_tri_inv_levels(double* Linv, int64_t n0, int64_t m, int64_t nb, hipStream_t s) {
  for (int64_t h = nb; h < n0; h *= 2) {
    const int64_t ppb = n0 / (2 * h);  // pairs per block
    auto p = gemm_params<double, double, double, float>();
    p.M = p.N = p.K = (int)h;
    p.zdiv = (int)ppb;
    // GEMM 1: T = A22inv * A21
    p.A = Linv + h * n0 + h;  p.lda = n0;  p.sa_o = n0 * n0;  p.sa_i = 2 * h * (n0 + 1);
    p.B = Linv + h * n0;      p.ldb = n0;  p.sb_o = n0 * n0;  p.sb_i = 2 * h * (n0 + 1);
    p.Cout = Linv + h;        p.ldco = n0; p.sco_o = n0 * n0; p.sco_i = 2 * h * (n0 + 1);
    p.flags = G_A_LOWER;
    p.alpha = 1.0;
    hipError_t e = Gemm<double>::run(p, (int)(m * ppb), s);
    if (e != hipSuccess) return e;
    // GEMM 2: A21 = -T * A11inv
    p.A = Linv + h;           p.lda = n0;  p.sa_o = n0 * n0;  p.sa_i = 2 * h * (n0 + 1);
    p.B = Linv;               p.ldb = n0;  p.sb_o = n0 * n0;  p.sb_i = 2 * h * (n0 + 1);
    p.Cout = Linv + h * n0;   p.ldco = n0; p.sco_o = n0 * n0; p.sco_i = 2 * h * (n0 + 1);
    p.flags = G_B_LOWER;
    p.alpha = -1.0;
    e = Gemm<double>::run(p, (int)(m * ppb), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// A2/A3: the blocked sweep of Alg. It-Inv-TRSM, right-looking.
//   X(S_i)      = Linv_ii * B'(S_i)                 (solve line)
//   B'(T_{i+1}) = B'(T_{i+1}) - L(T_{i+1},S_i) X(S_i) (update lines)
// B' lives in the workspace R; the first step reads B directly (or a copy of
// B(S_0) when X is B).
// ---------------------------------------------------------------------------
namespace {

template <typename T>
trsm_status sweep_right(trsm_plan_s& P, const T* L, int64_t ldl, const T* Linv, const T* B,
                        int64_t ldb, T* X, int64_t ldx, T* R, hipStream_t s) {
  const int64_t n = P.n, k = P.k, n0 = P.n0, m = P.m;
  const bool alias = (const void*)X == (const void*)B;
  const T* src0 = B;
  int64_t ld_src0 = ldb;
  if (alias) {
    TRSM_HIP(launch_copy2d<T, T>(B, ldb, R, k, std::min(n0, n), k, 1.0, s));
    src0 = R;
    ld_src0 = k;
  }
  // Lookahead over two streams.  Stream s carries the critical chain
  //   diag apply i -> update of the next block rows S_{i+1} -> diag apply i+1,
  // stream `side` carries the update of the remaining rows T_{i+2}, which
  // therefore overlaps the next diagonal apply.  Events order the two:
  //   side waits for the diag apply i (it reads X(S_i));
  //   s waits for side's update i-1 before updating rows S_{i+1} (both
  //   update those rows, read-modify-write).
  const bool look = (P.flags & TRSM_FLAG_LOOKAHEAD) && m > 2;
  if (look) {
    if (!P.side) TRSM_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
    const size_t need = (size_t)(2 * m + 2);
    while (P.events.size() < need) {
      hipEvent_t e;
      TRSM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      P.events.push_back(e);
    }
  }
  hipEvent_t* ev_x = look ? P.events.data() : nullptr;        // diag apply i done (on s)
  hipEvent_t* ev_b = look ? P.events.data() + m : nullptr;    // side update i done
  hipEvent_t ev_start = look ? P.events[2 * m] : nullptr;
  hipEvent_t ev_end = look ? P.events[2 * m + 1] : nullptr;
  hipStream_t s2 = P.side;
  // the two streams' products may run at once: each stream splits K in its
  // own half of the split-K scratch
  char* const sp = (char*)g_split.ptr;
  const int64_t half = sp ? (g_split.bytes / 2) / 256 * 256 : 0;
  SplitScope crit_split(sp, look ? half : g_split.bytes);
  if (look) {
    TRSM_HIP(hipEventRecord(ev_start, s));
    TRSM_HIP(hipStreamWaitEvent(s2, ev_start, 0));
  }
  for (int64_t i = 0; i < m; ++i) {
    const int64_t r0 = i * n0, sz = std::min(n0, n - r0);
    const T* src = (i == 0) ? src0 + r0 * ld_src0 : R + r0 * k;
    const int64_t ld_src = (i == 0) ? ld_src0 : k;
    // X(S_i) = Linv_ii * B'(S_i)
    TRSM_HIP(gemm_simple<T>(Linv + i * n0 * n0, n0, src, ld_src, nullptr, 0, X + r0 * ldx, ldx,
                            sz, k, sz, 1.0, 0.0, G_A_LOWER | G_A_ZERO_UPPER, s));
    if (i + 1 >= m) break;
    const int64_t t0 = r0 + n0;
    const T* cin = (i == 0) ? B + t0 * ldb : R + t0 * k;
    const int64_t ldci = (i == 0) ? ldb : k;
    if (!look) {
      // B'(T_{i+1}) -= L(T_{i+1}, S_i) X(S_i)
      TRSM_HIP(gemm_simple<T>(L + t0 * ldl + r0, ldl, X + r0 * ldx, ldx, cin, ldci, R + t0 * k, k,
                              n - t0, k, sz, -1.0, 1.0, 0u, s));
      continue;
    }
    TRSM_HIP(hipEventRecord(ev_x[i], s));
    // rows S_{i+1} on the critical stream
    if (i >= 1) TRSM_HIP(hipStreamWaitEvent(s, ev_b[i - 1], 0));
    const int64_t rows_a = std::min(n0, n - t0);
    TRSM_HIP(gemm_simple<T>(L + t0 * ldl + r0, ldl, X + r0 * ldx, ldx, cin, ldci, R + t0 * k, k,
                            rows_a, k, sz, -1.0, 1.0, 0u, s));
    // rows T_{i+2} on the side stream
    const int64_t t1 = t0 + rows_a;
    if (t1 < n) {
      TRSM_HIP(hipStreamWaitEvent(s2, ev_x[i], 0));
      SplitScope side_split(sp ? sp + half : nullptr, half);
      TRSM_HIP(gemm_simple<T>(L + t1 * ldl + r0, ldl, X + r0 * ldx, ldx, cin + rows_a * ldci, ldci,
                              R + t1 * k, k, n - t1, k, sz, -1.0, 1.0, 0u, s2));
      TRSM_HIP(hipEventRecord(ev_b[i], s2));
    } else {
      TRSM_HIP(hipEventRecord(ev_b[i], s2));
    }
  }
  if (look) {
    TRSM_HIP(hipEventRecord(ev_end, s2));
    TRSM_HIP(hipStreamWaitEvent(s, ev_end, 0));
  }
  return TRSM_OK;
}

// The transposed problem L^T X = B: with U = L^T upper triangular the
// blocked sweep runs backward, right-looking:
//   X(S_i)   = Uinv_ii B'(S_i)                   (Uinv_ii = Linv_ii^T)
//   B'(0:i)  = B'(0:i) - U(0:i, S_i) X(S_i)
// for i = m-1 down to 0; B' lives in the workspace R.
template <typename T>
trsm_status sweep_back(trsm_plan_s& P, const T* U, int64_t ldu, const T* Uinv, const T* B,
                       int64_t ldb, T* X, int64_t ldx, T* R, hipStream_t s) {
  const int64_t n = P.n, k = P.k, n0 = P.n0, m = P.m;
  const bool alias = (const void*)X == (const void*)B;
  const int64_t rl = (m - 1) * n0, szl = n - rl;   // the last (possibly ragged) block
  const T* srcl = B + rl * ldb;
  int64_t ld_srcl = ldb;
  if (alias) {
    TRSM_HIP(launch_copy2d<T, T>(B + rl * ldb, ldb, R + rl * k, k, szl, k, 1.0, s));
    srcl = R + rl * k;
    ld_srcl = k;
  }
  for (int64_t i = m - 1; i >= 0; --i) {
    const int64_t r0 = i * n0, sz = std::min(n0, n - r0);
    const bool last = i == m - 1;
    const T* src = last ? srcl : R + r0 * k;
    const int64_t ld_src = last ? ld_srcl : k;
    // X(S_i) = Uinv_ii B'(S_i)
    TRSM_HIP(gemm_simple<T>(Uinv + i * n0 * n0, n0, src, ld_src, nullptr, 0, X + r0 * ldx, ldx,
                            sz, k, sz, 1.0, 0.0, G_A_UPPER, s));
    if (i == 0) break;
    // B'(0:r0) -= U(0:r0, S_i) X(S_i)
    const T* cin = last ? B : R;
    const int64_t ldci = last ? ldb : k;
    TRSM_HIP(gemm_simple<T>(U + r0, ldu, X + r0 * ldx, ldx, cin, ldci, R, k, r0, k, sz, -1.0, 1.0,
                            0u, s));
  }
  return TRSM_OK;
}

// Recursive baseline (Alg. Rec-TRSM order on one GPU): X1 = solve(L11, B1);
// B2 -= L21 X1; X2 = solve(L22, B2); substitution leaves, no inversion.
template <typename T>
trsm_status rec_solve(int64_t n, int64_t k, const T* L, int64_t ldl, T* X, int64_t ldx,
                      int64_t leaf, hipStream_t s) {
  if (n <= 0) return TRSM_OK;
  if (n <= leaf) {
    TRSM_HIP(launch_subst_leaf<T>(L, ldl, X, ldx, n, k, s));
    return TRSM_OK;
  }
  int64_t n1 = ((n / 2 + leaf - 1) / leaf) * leaf;
  if (n1 >= n) n1 = n - leaf;
  TRSM_TRY(rec_solve<T>(n1, k, L, ldl, X, ldx, leaf, s));
  TRSM_HIP(gemm_simple<T>(L + n1 * ldl, ldl, X, ldx, X + n1 * ldx, ldx, X + n1 * ldx, ldx, n - n1,
                          k, n1, -1.0, 1.0, 0u, s));
  return rec_solve<T>(n - n1, k, L + n1 * ldl + n1, ldl, X + n1 * ldx, ldx, leaf, s);
}

// ---------------------------------------------------------------------------
// A4-A6: mixed precision.  Low-precision sweep (binary32 diagonal apply with
// the binary32 copy of Linv, bfloat16/half trailing update with binary32
// accumulation and per-(row, block) power-of-two scales), binary64 residual,
// iterative refinement.
// ---------------------------------------------------------------------------
// Left-looking form for the 16-bit matrix cores: block i's right-hand side
// is updated once, by all solved blocks at the same time,
//   Rl(S_i) -= L(S_i, 0:i n0) X(0:i n0)
// (one product with K = i n0, each block j of K carrying its own scales, see
// LP_SEGMENTS), then X(S_i) = Linv32_ii Rl(S_i).  Same arithmetic per term
// as the right-looking sweep, but the binary32 right-hand side is read and
// written once per block instead of once per step.
template <typename TL>
bool low_sweep_left_ok(const trsm_plan_s& P, const TL* Llow, const TL* XlowT) {
  lp::LpParams q = lp::lp_params();
  q.A = Llow; q.lda = P.n;
  q.B = XlowT; q.ldb = P.n;
  q.K = (int)P.n0;
  // whole 128-byte chunks per block of K (the segments' scales change at
  // chunk boundaries)
  const int64_t bb = P.n0 * (int64_t)sizeof(TL);
  return P.n % 8 == 0 && bb >= lp::kChunk && bb % lp::kChunk == 0 && lp::lp_ok<TL>(q);
}

template <typename TL>
trsm_status low_sweep_left(const trsm_plan_s& P, const float* Linv32, const TL* Llow,
                           const float* rscale, float* Rl, float* D, TL* XlowT, unsigned* amax,
                           float* xinv, int etarget, const TL* Linv16, const float* linv16_rs,
                           hipStream_t s) {
  const int64_t n = P.n, k = P.k, n0 = P.n0, m = P.m;
  unsigned* tamax = amax + 2 * m;          // scales of the coarse sweep's right-hand sides
  float* tinv = (float*)(amax + 3 * m);
  for (int64_t i = 0; i < m; ++i) {
    const int64_t r0 = i * n0, sz = std::min(n0, n - r0);
    if (i > 0) {
      lp::LpParams q = lp::lp_params();
      q.A = Llow + r0 * n; q.lda = n;
      q.B = XlowT; q.ldb = n;
      q.Cin = Rl + r0 * k; q.ldci = k;
      q.Cout = Rl + r0 * k; q.ldco = k;
      q.rscale = rscale + r0 * m; q.ld_rs = m;
      q.sscale = xinv;
      q.seg_chunks = (int)(n0 * (int64_t)sizeof(TL) / lp::kChunk);
      q.M = (int)sz; q.N = (int)k; q.K = (int)r0;
      q.alpha = -1.0f; q.beta = 1.0f;
      q.flags = lp::LP_BETA | lp::LP_SEGMENTS;
      TRSM_HIP(timed(2.0 * sz * k * r0, s, [&] { return lp::launch_lp_gemm<TL, lp::EPI_F32>(q, 1, s); }));
    }
    if (Linv16) {
      // coarse: X(S_i) = Linv_ii B'(S_i) on the 16-bit matrix cores, B'(S_i)
      // rounded with one scale (its columns of XlowT are free until X(S_i)
      // takes them)
      TRSM_HIP(launch_lowx<TL>(Rl + r0 * k, k, sz, k, XlowT + r0, n, tamax + i, tinv + i, etarget, s));
      lp::LpParams q = lp::lp_params();
      q.A = Linv16 + i * n0 * n0; q.lda = n0;
      q.B = XlowT + r0; q.ldb = n;
      q.Cout = D + r0 * k; q.ldco = k;
      q.rscale = linv16_rs + i * n0; q.ld_rs = 1;
      q.ascale = tinv + i;
      q.M = (int)sz; q.N = (int)k; q.K = (int)sz;
      q.flags = lp::LP_ROWSCALE | lp::LP_A_LOWER;
      TRSM_HIP(timed(1.0 * sz * sz * k, s, [&] { return lp::launch_lp_gemm<TL, lp::EPI_F32>(q, 1, s); }));
    } else {
      auto p = gemm_params<float, float, float, float>();
      p.A = Linv32 + i * n0 * n0; p.lda = n0;
      p.B = Rl + r0 * k; p.ldb = k;
      p.Cout = D + r0 * k; p.ldco = k;
      p.M = (int)sz; p.N = (int)k; p.K = (int)sz;
      p.flags = G_A_LOWER | G_A_ZERO_UPPER;
      use_split(p);
      TRSM_HIP(timed(gemm_flops(p, 1), s, [&] {
        return launch_gemm<float, float, float, float, 128, 128, 2, 2, false>(p, 1, s);
      }));
    }
    if (i + 1 < m)
      TRSM_HIP(launch_lowx<TL>(D + r0 * k, k, sz, k, XlowT + r0, n, amax + i, xinv + i, etarget, s));
  }
  return TRSM_OK;
}

template <typename TL>
trsm_status low_sweep(const trsm_plan_s& P, const float* Linv32, const TL* Llow,
                      const float* rscale, const double* rhs, int64_t ldr, double scale, float* Rl,
                      float* D, TL* XlowT, unsigned* amax, float* xinv, hipStream_t s,
                      const TL* Linv16 = nullptr, const float* linv16_rs = nullptr) {
  const int64_t n = P.n, k = P.k, n0 = P.n0, m = P.m;
  // largest magnitude of a solved block -> [2^etarget, 2^(etarget+1)) in the
  // low copy: half keeps headroom below its largest finite value (65504)
  // (e4m3's largest finite value is 448 or 240 depending on the encoding:
  // keep the block maximum below 128)
  const int etarget = std::is_same<TL, f16_t>::value ? 14 : std::is_same<TL, fp8_t>::value ? 6 : 0;
  if (rhs) TRSM_HIP(launch_copy2d<double, float>(rhs, ldr, Rl, k, n, k, scale, s));
  TRSM_HIP(launch_fill_u32(amax, 4 * m, 0u, s));
  if (low_sweep_left_ok<TL>(P, Llow, XlowT))
    return low_sweep_left<TL>(P, Linv32, Llow, rscale, Rl, D, XlowT, amax, xinv, etarget,
                              Linv16, linv16_rs, s);
  for (int64_t i = 0; i < m; ++i) {
    const int64_t r0 = i * n0, sz = std::min(n0, n - r0);
    // D(S_i) = Linv32_ii * Rl(S_i)
    {
      auto p = gemm_params<float, float, float, float>();
      p.A = Linv32 + i * n0 * n0; p.lda = n0;
      p.B = Rl + r0 * k; p.ldb = k;
      p.Cout = D + r0 * k; p.ldco = k;
      p.M = (int)sz; p.N = (int)k; p.K = (int)sz;
      p.flags = G_A_LOWER | G_A_ZERO_UPPER;
      use_split(p);
      TRSM_HIP(timed(gemm_flops(p, 1), s, [&] {
        return launch_gemm<float, float, float, float, 128, 128, 2, 2, false>(p, 1, s);
      }));
    }
    if (i + 1 < m) {
      // XlowT(:, S_i) = low(2^e D(S_i))^T, then Rl(T_i+1) -= Llow * X(S_i)
      TRSM_HIP(launch_lowx<TL>(D + r0 * k, k, sz, k, XlowT + r0, n, amax + i, xinv + i, etarget,
                               s));
      const int64_t t0 = r0 + n0, rows = n - t0;
      if constexpr (!std::is_same<TL, fp8_t>::value) {
        lp::LpParams q = lp::lp_params();
        q.A = Llow + t0 * n + r0; q.lda = n;
        q.B = XlowT + r0; q.ldb = n;          // stored k x n: column c of X is a row
        q.Cin = Rl + t0 * k; q.ldci = k;
        q.Cout = Rl + t0 * k; q.ldco = k;
        q.rscale = rscale + t0 * m + i; q.ld_rs = m;
        q.ascale = xinv + i;                  // undo the block's scale
        q.M = (int)rows; q.N = (int)k; q.K = (int)sz;
        q.alpha = -1.0f; q.beta = 1.0f;
        q.flags = lp::LP_BETA | lp::LP_ROWSCALE;
        if (lp::lp_ok<TL>(q)) {
          TRSM_HIP(timed(2.0 * rows * k * sz, s, [&] {
            return lp::launch_lp_gemm<TL, lp::EPI_F32>(q, 1, s);
          }));
          continue;
        }
      }
      auto p = gemm_params<TL, float, float, float>();
      p.A = Llow + t0 * n + r0; p.lda = n;
      p.B = XlowT + r0; p.ldb = n;            // stored k x n: column c of X is a row
      p.Cin = Rl + t0 * k; p.ldci = k;
      p.Cout = Rl + t0 * k; p.ldco = k;
      p.rscale = rscale + t0 * m + i; p.ld_rs = m;
      p.ascale = xinv + i;                    // undo the block's scale
      p.M = (int)rows; p.N = (int)k; p.K = (int)sz;
      p.alpha = -1.0; p.beta = 1.0;
      p.flags = G_BETA | G_ROWSCALE;
      use_split(p);
      TRSM_HIP(timed(gemm_flops(p, 1), s, [&] {
        return launch_gemm<TL, float, float, float, 128, 128, 2, 2, true>(p, 1, s);
      }));
    }
  }
  return TRSM_OK;
}

double pow2_scale_for(double maxabs) {
  if (!(maxabs > 0.0) || !isfinite(maxabs)) return 1.0;
  return ldexp(1.0, -ilogb(maxabs));
}

// One refinement residual: the correction piece D (binary32; the correction
// it stands for is D 2^yshift) is rounded in place to b bits per column, its
// residues are multiplied with L's residue planes on the int8 matrix cores (P
// moduli), and the recombination updates R (binary64, in the workspace) and
// its binary32 copy, and X according to xmode (0: untouched, 1: X = piece,
// 2: X += piece).  The norms land in the workspace (crt::launch_recombine).
trsm_status crt_residual(const trsm_plan_s& P, const double* L, int64_t ldl, const char* lbuf,
                         float* D, int yshift, int b, int nmod, const double* Rin, int64_t ldri,
                         double* X, int64_t ldx, int xmode, char* ws, hipStream_t s) {
  const int64_t n = P.n, k = P.k, npad = P.npad, ldz = P.ldz;
  const crt::Table t = crt::make_table(nmod);
  unsigned* colmax = (unsigned*)(ws + P.ws_colmax);
  int* ty = (int*)(ws + P.ws_ty);
  int8_t* Q = (int8_t*)(ws + P.ws_q);
  int8_t* Z = (int8_t*)(ws + P.ws_z);
  double* R64 = (double*)(ws + P.ws_r64);
  TRSM_HIP(crt::launch_y_residues(D, k, n, npad, k, colmax, b, t, Q, npad, k * npad, ty, s));
  lp::LpParams q = lp::lp_params();
  q.A = lbuf + P.off_crt_e; q.lda = npad; q.sa = npad * npad;
  q.B = Q; q.ldb = npad; q.sb = k * npad;
  q.Z = Z; q.ldz = ldz; q.sz = npad * ldz;
  q.M = (int)npad; q.N = (int)k; q.K = (int)npad;
  q.flags = lp::LP_A_LOWER;
  for (int p = 0; p < nmod; ++p) q.modulus[p] = t.mod[p];
  TRSM_HIP(timed(1.0 * npad * npad * k * nmod, s, [&] {
    return lp::launch_lp_gemm<int8_t, lp::EPI_MOD>(q, nmod, s);
  }));
  double* rpart = (double*)(ws + P.ws_rpart);
  TRSM_HIP(crt::launch_recombine(Z, ldz, npad * ldz, t, (const int*)(lbuf + P.off_crt_sl), ty, D,
                                 k, yshift, L, ldl, Rin, ldri, R64, k, (float*)(ws + P.ws_rl), X,
                                 ldx, xmode, n, k, rpart, rpart + 4 * crt::kRecBlocks, s));
  return TRSM_OK;
}

// Moduli for a product of an a-bit L with b-bit pieces (|C| < n 2^(a+b), and
// M > 4 |C|), and the largest b those moduli allow.
int crt_moduli(int a, int bmin, int64_t n, int* b_out) {
  const int lgn = (int)ceil(log2((double)std::max<int64_t>(n, 2)));
  const int P = crt::moduli_for_bits((double)(a + bmin + lgn + 2));
  if (P < 0) return -1;
  const crt::Table t = crt::make_table(P);
  // pieces are rounded in binary32 (exact up to 24 bits)
  *b_out = std::min((int)floor(t.log2M) - a - lgn - 2, 24);
  return P;
}

// Iterative refinement with exact residuals.  Each correction D_j of the
// low-precision sweep is rounded to b_j bits per column before it is added, so
// that L times the accumulated X is an exact integer product (crt_residual):
// the residual R_{j+1} = R_j - L D_j is then exact for the L whose strictly
// lower part is rounded to a bits (relative to each row's largest entry), and
// binary64 work is limited to one rounding per element.  The first piece is
// rounded coarsely (about 8 bits: the next correction removes that error as
// well), later ones to 20+ bits.  Stop when the exact residual of the pieces
// so far gives a backward error ||R|| / (||L|| ||X||) <= 4u, when the next
// correction predicted from the observed contraction,
// ||D_j|| * (||D_j|| / ||D_{j-1}||), falls below 1e-14 ||X||, or when a
// correction falls below 1e-15 ||X||; at most 10 corrections.
//
// With a tolerance tol > 0 (trsm_plan_set_tolerance) the target is a relative
// forward error of tol instead of binary64's level: the first piece is the
// full-accuracy sweep (binary32 diagonal apply) rounded to the wide width, so
// that it counts as correction 0 with ||D_0|| = ||X||, and the refinement
// also stops once the error left after adding D_j, predicted as
// ||D_j|| * rho with rho = ||D_j|| / ||D_{j-1}|| <= 1/2, is <= tol ||X||.  A
// 16-bit sweep whose own error is below sqrt(tol) then needs one exact
// residual and one correction.
template <typename TL>
trsm_status solve_mixed(const trsm_plan_s& P, const double* L, int64_t ldl, const char* lbuf,
                        const double* B, int64_t ldb, double* X, int64_t ldx, char* ws,
                        hipStream_t s, trsm_info* info) {
  const int64_t n = P.n, k = P.k;
  const float* Linv32 = (const float*)(lbuf + P.off_linv32);
  const TL* Llow = (const TL*)(lbuf + P.off_llow);
  const float* rscale = (const float*)(lbuf + P.off_rscale);
  double* R64 = (double*)(ws + P.ws_r64);
  float* Rl = (float*)(ws + P.ws_rl);
  float* D = (float*)(ws + P.ws_d);
  TL* XlowT = (TL*)(ws + P.ws_xlow);
  unsigned* amax = (unsigned*)(ws + P.ws_xsc);
  float* xinv = (float*)(ws + P.ws_xsc + 4 * P.m);
  double* part = (double*)(ws + P.ws_part);
  double* dnorm = (double*)(ws + P.ws_norm);
  unsigned* colmax = (unsigned*)(ws + P.ws_colmax);
  double* dpart = (double*)(ws + P.ws_dpart);
  double* dres = dpart + crt::kStatSlabs * crt::kRecBlocks;
  const double* rres = (const double*)(ws + P.ws_rpart) + 4 * crt::kRecBlocks;

  // ||L||_F^2, the residue bit count a (both stored by trsm_invert_diag), max |B|
  double h[4];
  int a = 0;
  double lnorm2 = 0.0;
  TRSM_HIP(launch_sumsq_max(B, ldb, n, k, part, dnorm, s));
  TRSM_HIP(hipMemcpyAsync(h, dnorm, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  TRSM_HIP(hipMemcpyAsync(&lnorm2, lbuf + P.off_lnorm, sizeof(double), hipMemcpyDeviceToHost, s));
  TRSM_HIP(hipMemcpyAsync(&a, lbuf + P.off_crt_a, sizeof(int), hipMemcpyDeviceToHost, s));
  TRSM_HIP(hipStreamSynchronize(s));
  const double lnorm = sqrt(lnorm2);
  const bool alias = (const void*)X == (const void*)B;
  const double u = ldexp(1.0, -53);

  double scale = pow2_scale_for(h[1]);
  // the first sweep's result is rounded to about 8 bits before the first
  // residual, so its diagonal apply may run in 16 bits as well
  const double tol = P.tol;
  const bool coarse = !(P.flags & TRSM_FLAG_NO_REFINE) && !std::is_same<TL, fp8_t>::value &&
                      tol == 0.0;
  TRSM_TRY(low_sweep<TL>(P, Linv32, Llow, rscale, B, ldb, scale, Rl, D, XlowT, amax, xinv, s,
                         coarse ? (const TL*)(lbuf + P.off_linv16) : nullptr,
                         (const float*)(lbuf + P.off_linv16_rs)));
  if (info) {
    info->iterations = 0;
    info->converged = 0;
    info->backward_error = -1.0;
    info->correction = -1.0;
    info->unrefined_error = -1.0;
  }
  if (P.flags & TRSM_FLAG_NO_REFINE) {
    TRSM_HIP(launch_axpy_f32_to_f64(D, k, X, ldx, n, k, 1.0 / scale, true, s));
    if (info) info->converged = 1;
    return TRSM_OK;
  }
  if (alias) return TRSM_EINVAL;  // refinement needs the original B (checked earlier too)

  int b0 = 0, b1 = 0;
  const int P0 = crt_moduli(a, tol > 0.0 ? 20 : 7, n, &b0);
  const int P1 = crt_moduli(a, 20, n, &b1);
  if (P0 < 0 || P1 < 0) return TRSM_EINVAL;

  // correction pieces: the first three stay in their own binary32 buffers
  // and X is assembled from them at the end (one binary64 pass); from the
  // fourth on they are added to X as they come
  float* piece[3] = {D, (float*)(ws + P.ws_d1), (float*)(ws + P.ws_d2)};
  int pshift[3] = {0, 0, 0};
  double prev = -1.0, xnorm = 0.0;
  float* cur = D;
  for (int j = 0; j <= 10; ++j) {
    // ||D|| and the column maxima of the new correction
    TRSM_HIP(launch_fill_u32(colmax, k, 0u, s));
    TRSM_HIP(crt::launch_dstats<float>(cur, k, n, k, colmax, dpart, dres, s));
    const int yshift = -ilogb(scale);   // the correction is cur 2^yshift
    if (j > 0) {
      double dn2 = 0.0;
      TRSM_HIP(hipMemcpyAsync(&dn2, dres, sizeof(double), hipMemcpyDeviceToHost, s));
      TRSM_HIP(hipStreamSynchronize(s));
      const double corr = (xnorm > 0) ? ldexp(sqrt(dn2), yshift) / xnorm : ldexp(sqrt(dn2), yshift);
      if (info) {
        info->iterations = j;
        info->correction = corr;
        if (j == 1) info->unrefined_error = corr;
      }
      bool done = corr <= 1e-15;
      // the previous correction; without a coarse first piece the first
      // sweep's result is correction 0, of relative size 1
      const double before = prev > 0 ? prev : (tol > 0.0 ? 1.0 : -1.0);
      if (!done && before > 0) {
        const double rho = corr / before;
        done = rho <= 0.5 && corr * rho <= std::max(tol, 1e-14);
      }
      prev = corr;
      if (done || j == 10) {
        if (j <= 2)
          TRSM_HIP(crt::launch_assemble(piece[0], pshift[0], j >= 2 ? piece[1] : cur, j >= 2 ? pshift[1] : yshift,
                                        j >= 2 ? cur : nullptr, yshift, k, X, ldx, n, k, false, s));
        else
          TRSM_HIP(crt::launch_assemble(cur, yshift, nullptr, 0, nullptr, 0, k, X, ldx, n, k, true, s));
        if (done && info) info->converged = 1;
        return done ? TRSM_OK : TRSM_ENOTCONVERGED;
      }
    }
    // R -= L round(cur), exactly; the rounded piece stays in cur
    const bool first = j == 0;
    if (j == 2)   // X from the first two pieces; later pieces are added as they come
      TRSM_HIP(crt::launch_assemble(piece[0], pshift[0], piece[1], pshift[1], nullptr, 0, k, X, ldx,
                                    n, k, false, s));
    TRSM_TRY(crt_residual(P, L, ldl, lbuf, cur, yshift, first ? b0 : b1, first ? P0 : P1,
                          first ? B : R64, first ? ldb : k, X, ldx, j >= 2 ? 2 : 0, ws, s));
    if (j < 3) pshift[j] = yshift;
    TRSM_HIP(hipMemcpyAsync(h, rres, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    TRSM_HIP(hipStreamSynchronize(s));
    const double rn = sqrt(h[0]);
    if (j >= 2) {
      xnorm = sqrt(h[2]);
    } else {
      // ||X|| of the pieces so far: ||piece_0|| for the first (its rounding
      // changes the norm by less than 2^-7), good enough for relative tests
      double dn2 = 0.0;
      TRSM_HIP(hipMemcpyAsync(&dn2, dres, sizeof(double), hipMemcpyDeviceToHost, s));
      TRSM_HIP(hipStreamSynchronize(s));
      if (first) xnorm = ldexp(sqrt(dn2), yshift);
    }
    const double berr = (lnorm * xnorm > 0) ? rn / (lnorm * xnorm) : rn;
    if (info) info->backward_error = berr;
    if (rn == 0.0 || berr <= 4.0 * u) {
      // the pieces so far are backward stable (the residual is exact for
      // them): X is their sum (from the third piece on it was updated in place)
      if (j < 2)
        TRSM_HIP(crt::launch_assemble(piece[0], pshift[0], j == 1 ? piece[1] : nullptr, pshift[1],
                                      nullptr, 0, k, X, ldx, n, k, false, s));
      if (info) info->converged = 1;
      return TRSM_OK;
    }
    // the recombination left R in binary32 in Rl (unscaled)
    scale = 1.0;
    cur = piece[std::min(j + 1, 2)];
    TRSM_TRY(low_sweep<TL>(P, Linv32, Llow, rscale, nullptr, k, scale, Rl, cur, XlowT, amax, xinv, s));
  }
  return TRSM_ENOTCONVERGED;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* trsm_status_string(trsm_status s) {
  switch (s) {
    case TRSM_OK: return "TRSM_OK";
    case TRSM_EINVAL: return "TRSM_EINVAL";
    case TRSM_ESINGULAR: return "TRSM_ESINGULAR";
    case TRSM_ENOMEM: return "TRSM_ENOMEM";
    case TRSM_EHIP: return "TRSM_EHIP";
    case TRSM_ENOTCONVERGED: return "TRSM_ENOTCONVERGED";
    case TRSM_EBUSY: return "TRSM_EBUSY";
  }
  return "TRSM_UNKNOWN";
}

int trsm_last_hip_error(void) { return g_last_hip; }

trsm_status trsm_plan(int64_t n, int64_t k, trsm_precision prec, int64_t n0, uint32_t flags,
                      trsm_plan_t* out) {
  if (!out) return TRSM_EINVAL;
  *out = nullptr;
  if (n < 0 || k < 0 || n > (int64_t)1 << 30 || k > (int64_t)1 << 30) return TRSM_EINVAL;
  if (prec != TRSM_F64 && prec != TRSM_F32 && !is_mixed(prec)) return TRSM_EINVAL;
  if (n0 < 0 || (n0 > 0 && !is_pow2(n0))) return TRSM_EINVAL;
  if ((flags & TRSM_FLAG_RECURSIVE) && is_mixed(prec)) return TRSM_EINVAL;
  // the residual's int8 products accumulate up to n terms of |x| <= 2^14 in int32
  if (is_mixed(prec) && n > crt::kMaxN) return TRSM_EINVAL;
  if (flags & ~(TRSM_FLAG_NO_REFINE | TRSM_FLAG_RECURSIVE | TRSM_FLAG_LOOKAHEAD |
                TRSM_FLAG_LARGE_TILES | TRSM_FLAG_TRANSPOSE | TRSM_FLAG_UPPER))
    return TRSM_EINVAL;
  if ((flags & TRSM_FLAG_TRANSPOSE) &&
      (is_mixed(prec) || (flags & (TRSM_FLAG_RECURSIVE | TRSM_FLAG_LOOKAHEAD))))
    return TRSM_EINVAL;
  if ((flags & TRSM_FLAG_UPPER) &&
      (is_mixed(prec) ||
       (flags & (TRSM_FLAG_RECURSIVE | TRSM_FLAG_LOOKAHEAD | TRSM_FLAG_TRANSPOSE))))
    return TRSM_EINVAL;
  if (n * k > ((int64_t)1 << 31) - 1 || n * n > ((int64_t)1 << 31) * 8) return TRSM_EINVAL;
  trsm_plan_s* P = new (std::nothrow) trsm_plan_s();
  if (!P) return TRSM_ENOMEM;
  P->n = n;
  P->k = k;
  P->prec = prec;
  P->n0_paper = paper_rule_n0(n, k);
  if (n0 == 0) {
    int64_t tn0 = 0;
    uint32_t tfl = 0;
    if (n > 0 && k > 0 && tune_lookup(n, k, (int)prec, &tn0, &tfl)) {
      n0 = tn0;
      flags |= tfl;
    } else {
      n0 = auto_n0(n, k, prec);
    }
  }
  P->flags = flags;
  const int64_t cap = next_pow2(n < 1 ? 1 : n);
  if (n0 > cap) n0 = cap;
  P->n0 = n0;
  P->m = n > 0 ? ceil_div(n, n0) : 0;
  P->leaf = std::min<int64_t>(n0, 64);
  const int64_t m = P->m;
  // Linv buffer
  size_t off = 0;
  P->off_linv64 = off;
  off = align_up(off + (size_t)m * n0 * n0 * 8);
  if (prec != TRSM_F64) {
    P->off_linv32 = off;
    off = align_up(off + (size_t)m * n0 * n0 * 4);
  }
  if (is_mixed(prec)) {
    P->off_llow = off;
    off = align_up(off + (size_t)n * n * 2);
    P->off_rscale = off;
    off = align_up(off + (size_t)n * m * 4);
    P->off_lnorm = off;
    off = align_up(off + 8);
    P->off_lpart = off;
    off = align_up(off + 2 * kNormBlocks * 8 + 16);
    P->npad = (n + 63) / 64 * 64;
    P->ldz = (k + 15) / 16 * 16;
    P->off_crt_e = off;
    off = align_up(off + (size_t)crt::kPlanes * P->npad * P->npad);
    P->off_crt_rowmax = off;
    off = align_up(off + (size_t)n * 8);
    P->off_crt_rowpart = off;
    off = align_up(off + (size_t)n * 8);
    P->off_crt_stats = off;
    off = align_up(off + 64);
    P->off_crt_a = off;
    off = align_up(off + 64);
    P->off_crt_sl = off;
    off = align_up(off + (size_t)P->npad * 4);
    P->off_linv16 = off;
    off = align_up(off + (size_t)m * n0 * n0 * 2);
    P->off_linv16_rs = off;
    off = align_up(off + (size_t)m * n0 * 4);
  }
  if (flags & TRSM_FLAG_TRANSPOSE) {
    const size_t es = elem_size(prec);
    P->ldu = (n + 3) / 4 * 4;
    P->off_ut = off;
    off = align_up(off + (size_t)n * P->ldu * es);
    P->off_uinv = off;
    off = align_up(off + (size_t)m * n0 * n0 * es);
  }
  if (flags & TRSM_FLAG_UPPER) {
    // the inverses of U's diagonal blocks; U itself is read in place
    P->off_uinv = off;
    off = align_up(off + (size_t)m * n0 * n0 * elem_size(prec));
  }
  P->off_status = off;
  off = align_up(off + 8);
  P->linv_bytes = (flags & TRSM_FLAG_RECURSIVE) ? 0 : off;
  // workspace
  off = 0;
  if (flags & TRSM_FLAG_RECURSIVE) {
    // in place in X
  } else if (!is_mixed(prec)) {
    P->ws_r = off;
    off = align_up(off + (size_t)n * k * elem_size(prec));
  } else {
    P->ws_r64 = off;
    off = align_up(off + (size_t)n * k * 8);
    P->ws_rl = off;
    off = align_up(off + (size_t)n * k * 4);
    P->ws_d = off;
    off = align_up(off + (size_t)n * k * 4);
    P->ws_xlow = off;
    off = align_up(off + (size_t)n * k * 2);
    P->ws_xsc = off;   // per-block max bits and inverse scales, for X and for the coarse sweep's B'
    off = align_up(off + (size_t)m * 16);
    P->ws_part = off;
    off = align_up(off + 2 * kNormBlocks * 8);
    P->ws_norm = off;
    off = align_up(off + 8 * 8);
    P->ws_d1 = off;
    off = align_up(off + (size_t)n * k * 4);
    P->ws_d2 = off;
    off = align_up(off + (size_t)n * k * 4);
    P->ws_q = off;
    off = align_up(off + (size_t)crt::kPlanes * k * P->npad);
    P->ws_z = off;
    off = align_up(off + (size_t)crt::kPlanes * P->npad * P->ldz);
    P->ws_colmax = off;
    off = align_up(off + (size_t)k * 4);
    P->ws_ty = off;
    off = align_up(off + (size_t)k * 4);
    P->ws_rpart = off;
    off = align_up(off + (size_t)(4 * crt::kRecBlocks + 8) * 8);
    P->ws_dpart = off;
    off = align_up(off + (size_t)(crt::kStatSlabs * crt::kRecBlocks + 8) * 8);
  }
  P->ws_split = off;
  P->ws_split_bytes = split_bytes(n * k);
  off = align_up(off + P->ws_split_bytes);
  P->ws_bytes = off;
  *out = P;
  return TRSM_OK;
}

trsm_status trsm_plan_get_info(trsm_plan_t P, trsm_plan_info* info) {
  if (!P || !info) return TRSM_EINVAL;
  info->n = P->n;
  info->k = P->k;
  info->n0 = P->n0;
  info->m = P->m;
  info->leaf = P->leaf;
  info->n0_paper_rule = P->n0_paper;
  info->precision = (int32_t)P->prec;
  info->flags = P->flags;
  info->linv_bytes = P->linv_bytes;
  info->workspace_bytes = P->ws_bytes;
  info->inv_flops = (double)P->n * (double)P->n0 * (double)P->n0 / 3.0;
  info->solve_flops = (double)P->n * (double)P->n * (double)P->k;
  return TRSM_OK;
}

trsm_status trsm_plan_destroy(trsm_plan_t P) {
  if (!P) return TRSM_OK;
  P->timer.release();
  for (hipEvent_t e : P->events) (void)hipEventDestroy(e);
  if (P->side) (void)hipStreamDestroy(P->side);
  delete P;
  return TRSM_OK;
}

trsm_status trsm_invert_diag(trsm_plan_t P, const void* L, int64_t ldl, void* Linv, void* stream) {
  if (!P) return TRSM_EINVAL;
  if (P->flags & TRSM_FLAG_RECURSIVE) return TRSM_OK;
  if (P->n == 0) return TRSM_OK;
  if (!L || !Linv || ldl < P->n) return TRSM_EINVAL;
  if (((uintptr_t)Linv) % kAlign) return TRSM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  TimerScope timer_scope(&P->timer);
  char* base = (char*)Linv;
  double* L64 = (double*)(base + P->off_linv64);
  const int64_t n = P->n, n0 = P->n0, m = P->m;
  // the status word lives in the caller's buffer; the inversion's products
  // run without split-K scratch, so the call allocates nothing
  unsigned long long* bad = (unsigned long long*)(base + P->off_status);
  P->last_linv = Linv;
  const bool large = P->flags & TRSM_FLAG_LARGE_TILES;
  TilePolicyScope tile_scope(large);
  SplitScope split_scope(nullptr, 0);
  TRSM_HIP(launch_fill_u32((unsigned*)bad, 2, 0xFFFFFFFFu, s));
  // an upper plan inverts the transposed blocks U_ii^T (lower) and
  // transposes the inverses back below
  const bool upper = P->flags & TRSM_FLAG_UPPER;
  if (P->prec == TRSM_F32)
    TRSM_HIP(launch_extract_diag<float>((const float*)L, ldl, n, n0, m, L64, bad, s, upper));
  else
    TRSM_HIP(launch_extract_diag<double>((const double*)L, ldl, n, n0, m, L64, bad, s, upper));
  TRSM_HIP(launch_trtri_leaf(L64, n0, m, P->leaf, s));
  if (P->leaf < n0) {
    TRSM_HIP(rec_tri_inv_levels(L64, n0, m, P->leaf, s));
    TRSM_HIP(launch_zero_upper(L64, n0, m, s));
  }
  if (P->prec != TRSM_F64)
    TRSM_HIP((launch_convert<double, float>(L64, (float*)(base + P->off_linv32), m * n0 * n0, s)));
  if (P->flags & TRSM_FLAG_TRANSPOSE) {
    // U = L^T (zeros below the diagonal) and Uinv_ii = Linv_ii^T
    if (P->prec == TRSM_F32) {
      TRSM_HIP((launch_transpose<float, float>((const float*)L, ldl, (float*)(base + P->off_ut),
                                               P->ldu, n, n, 1, 0, 0, true, s)));
      TRSM_HIP((launch_transpose<float, float>((const float*)(base + P->off_linv32), n0,
                                               (float*)(base + P->off_uinv), n0, n0, n0, m,
                                               n0 * n0, n0 * n0, false, s)));
    } else {
      TRSM_HIP((launch_transpose<double, double>((const double*)L, ldl,
                                                 (double*)(base + P->off_ut), P->ldu, n, n, 1, 0,
                                                 0, true, s)));
      TRSM_HIP((launch_transpose<double, double>(L64, n0, (double*)(base + P->off_uinv), n0, n0,
                                                 n0, m, n0 * n0, n0 * n0, false, s)));
    }
  }
  if (upper) {
    // Uinv_ii = ((U_ii^T)^{-1})^T
    if (P->prec == TRSM_F32)
      TRSM_HIP((launch_transpose<float, float>((const float*)(base + P->off_linv32), n0,
                                               (float*)(base + P->off_uinv), n0, n0, n0, m,
                                               n0 * n0, n0 * n0, false, s)));
    else
      TRSM_HIP((launch_transpose<double, double>(L64, n0, (double*)(base + P->off_uinv), n0, n0,
                                                 n0, m, n0 * n0, n0 * n0, false, s)));
  }
  if (is_mixed(P->prec)) {
    float* rs = (float*)(base + P->off_rscale);
    if (P->prec == TRSM_MIXED_BF16)
      TRSM_HIP(launch_rowscale_copy<bf16_t>(L64, m * n0, n0, (bf16_t*)(base + P->off_linv16),
                                            (float*)(base + P->off_linv16_rs), 1.0f, s));
    else if (P->prec == TRSM_MIXED_F16)
      TRSM_HIP(launch_rowscale_copy<f16_t>(L64, m * n0, n0, (f16_t*)(base + P->off_linv16),
                                           (float*)(base + P->off_linv16_rs), 16384.0f, s));
    if (P->prec == TRSM_MIXED_BF16)
      TRSM_HIP(launch_lowcopy<bf16_t>((const double*)L, ldl, n, n0, m, (bf16_t*)(base + P->off_llow),
                                      rs, 1.0f, s));
    else if (P->prec == TRSM_MIXED_FP8)
      TRSM_HIP(launch_lowcopy<fp8_t>((const double*)L, ldl, n, n0, m, (fp8_t*)(base + P->off_llow),
                                     rs, 128.0f, s));
    else
      TRSM_HIP(launch_lowcopy<f16_t>((const double*)L, ldl, n, n0, m, (f16_t*)(base + P->off_llow),
                                     rs, 16384.0f, s));
    // ||L||_F^2 over the lower triangle, kept for the backward-error test
    double* part = (double*)(base + P->off_lpart);
    double* res = part + 2 * kNormBlocks;
    TRSM_HIP(launch_sumsq_lower<double>((const double*)L, ldl, n, part, res, s));
    TRSM_HIP((launch_copy2d<double, double>(res, 1, (double*)(base + P->off_lnorm), 1, 1, 1, 1.0, s)));
    // residue planes of L's strictly lower part for the residual's exact
    // integer products; the bit count a follows from L's magnitudes
    double* rowmax = (double*)(base + P->off_crt_rowmax);
    double* stats = (double*)(base + P->off_crt_stats);
    int* a_dev = (int*)(base + P->off_crt_a);
    TRSM_HIP(crt::launch_row_stats((const double*)L, ldl, n, rowmax,
                                   (double*)(base + P->off_crt_rowpart), stats, s));
    TRSM_HIP(crt::launch_choose_bits(stats, (const double*)(base + P->off_lnorm),
                                     crt::kTargetBits, a_dev, s));
    const crt::Table t = crt::make_table(crt::kPlanes);
    TRSM_HIP(crt::launch_l_residues((const double*)L, ldl, n, P->npad, rowmax, a_dev, t,
                                    (int8_t*)(base + P->off_crt_e), P->npad,
                                    P->npad * P->npad, (int*)(base + P->off_crt_sl), s));
  }
  return TRSM_OK;
}

trsm_status trsm_plan_last_error(trsm_plan_t P, trsm_status* status, int64_t* index) {
  if (!P || !status || !index) return TRSM_EINVAL;
  unsigned long long v = ~0ull;
  if (P->last_linv)
    TRSM_HIP(hipMemcpy(&v, (const char*)P->last_linv + P->off_status, sizeof(v),
                       hipMemcpyDeviceToHost));
  if (v == ~0ull) {
    *status = TRSM_OK;
    *index = -1;
  } else {
    *status = TRSM_ESINGULAR;
    *index = (int64_t)v;
  }
  return TRSM_OK;
}

}  // extern "C"

namespace {

// trsm_solve's body; the split-K scratch of the products is the given
// region (the plan's section of the workspace, or part of the static scratch
// of trsm_solve_noalloc).
trsm_status solve_impl(trsm_plan_t P, const void* L, int64_t ldl, const void* Linv, const void* B,
                       int64_t ldb, void* X, int64_t ldx, void* workspace, void* split,
                       int64_t split_bytes, void* stream, trsm_info* info) {
  if (!P) return TRSM_EINVAL;
  if (info) {
    info->iterations = 0;
    info->converged = 1;
    info->backward_error = -1.0;
    info->correction = -1.0;
    info->unrefined_error = -1.0;
  }
  const int64_t n = P->n, k = P->k;
  if (n == 0 || k == 0) return TRSM_OK;
  const bool rec = P->flags & TRSM_FLAG_RECURSIVE;
  if (!L || !B || !X || (!rec && !Linv)) return TRSM_EINVAL;
  if (ldl < n || ldb < k || ldx < k) return TRSM_EINVAL;
  if (P->ws_bytes && !workspace) return TRSM_EINVAL;
  if (workspace && ((uintptr_t)workspace) % kAlign) return TRSM_EINVAL;
  if (Linv && ((uintptr_t)Linv) % kAlign) return TRSM_EINVAL;
  const size_t es = elem_size(P->prec);
  const size_t bbytes = ((size_t)(n - 1) * ldb + k) * es, xbytes = ((size_t)(n - 1) * ldx + k) * es;
  if (ranges_overlap(B, bbytes, X, xbytes) && !(B == X && ldb == ldx)) return TRSM_EINVAL;
  if (is_mixed(P->prec) && B == X && !(P->flags & TRSM_FLAG_NO_REFINE)) return TRSM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  TimerScope timer_scope(&P->timer);
  const char* lb = (const char*)Linv;
  char* ws = (char*)workspace;
  const bool large = P->flags & TRSM_FLAG_LARGE_TILES;
  TilePolicyScope tile_scope(large);
  SplitScope split_scope(large ? nullptr : split, large ? 0 : split_bytes);
  if (rec) {
    if (P->prec == TRSM_F64) {
      if (X != B) TRSM_HIP(launch_copy2d<double, double>((const double*)B, ldb, (double*)X, ldx, n, k, 1.0, s));
      return rec_solve<double>(n, k, (const double*)L, ldl, (double*)X, ldx, 64, s);
    }
    if (X != B) TRSM_HIP(launch_copy2d<float, float>((const float*)B, ldb, (float*)X, ldx, n, k, 1.0, s));
    return rec_solve<float>(n, k, (const float*)L, ldl, (float*)X, ldx, 64, s);
  }
  if (P->flags & TRSM_FLAG_UPPER) {
    if (P->prec == TRSM_F64)
      return sweep_back<double>(*P, (const double*)L, ldl, (const double*)(lb + P->off_uinv),
                                (const double*)B, ldb, (double*)X, ldx, (double*)(ws + P->ws_r),
                                s);
    return sweep_back<float>(*P, (const float*)L, ldl, (const float*)(lb + P->off_uinv),
                             (const float*)B, ldb, (float*)X, ldx, (float*)(ws + P->ws_r), s);
  }
  if (P->flags & TRSM_FLAG_TRANSPOSE) {
    if (P->prec == TRSM_F64)
      return sweep_back<double>(*P, (const double*)(lb + P->off_ut), P->ldu,
                                (const double*)(lb + P->off_uinv), (const double*)B, ldb,
                                (double*)X, ldx, (double*)(ws + P->ws_r), s);
    return sweep_back<float>(*P, (const float*)(lb + P->off_ut), P->ldu,
                             (const float*)(lb + P->off_uinv), (const float*)B, ldb, (float*)X,
                             ldx, (float*)(ws + P->ws_r), s);
  }
  switch (P->prec) {
    case TRSM_F64:
      return sweep_right<double>(*P, (const double*)L, ldl, (const double*)(lb + P->off_linv64),
                                 (const double*)B, ldb, (double*)X, ldx, (double*)(ws + P->ws_r), s);
    case TRSM_F32:
      return sweep_right<float>(*P, (const float*)L, ldl, (const float*)(lb + P->off_linv32),
                                (const float*)B, ldb, (float*)X, ldx, (float*)(ws + P->ws_r), s);
    case TRSM_MIXED_BF16:
      return solve_mixed<bf16_t>(*P, (const double*)L, ldl, lb, (const double*)B, ldb, (double*)X,
                                 ldx, ws, s, info);
    case TRSM_MIXED_FP8:
      return solve_mixed<fp8_t>(*P, (const double*)L, ldl, lb, (const double*)B, ldb, (double*)X,
                                ldx, ws, s, info);
    case TRSM_MIXED_F16:
      return solve_mixed<f16_t>(*P, (const double*)L, ldl, lb, (const double*)B, ldb, (double*)X,
                                ldx, ws, s, info);
  }
  return TRSM_EINVAL;
}

// Device scratch of trsm_solve_noalloc: one copy per GPU, held until the
// process ends.  Host code never uses the array's name as an address: its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)2 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

trsm_status scratch_for_current_device(void** out) {
  int dev = 0;
  TRSM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return TRSM_EINVAL;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    TRSM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return TRSM_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TRSM_OK;
}

}  // namespace

extern "C" {

trsm_status trsm_solve(trsm_plan_t P, const void* L, int64_t ldl, const void* Linv, const void* B,
                       int64_t ldb, void* X, int64_t ldx, void* workspace, void* stream,
                       trsm_info* info) {
  if (!P) return TRSM_EINVAL;
  char* ws = (char*)workspace;
  return solve_impl(P, L, ldl, Linv, B, ldb, X, ldx, workspace, ws ? ws + P->ws_split : nullptr,
                    ws ? (int64_t)P->ws_split_bytes : 0, stream, info);
}

size_t trsm_solve_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

trsm_status trsm_solve_noalloc(trsm_plan_t P, const void* L, int64_t ldl, const void* Linv,
                               const void* B, int64_t ldb, void* X, int64_t ldx, void* stream,
                               trsm_info* info) {
  if (!P) return TRSM_EINVAL;
  // binary64 / binary32 plans on one stream (the lookahead's side stream and
  // the per-launch timing events would be created on first use)
  if (is_mixed(P->prec) || (P->flags & TRSM_FLAG_LOOKAHEAD) || P->timer.enabled)
    return TRSM_EINVAL;
  // the workspace's running right-hand side must fit the scratch; what is
  // left of it holds split-K partial products
  const size_t need = P->ws_split;
  if (need > kNoAllocScratchBytes) return TRSM_ENOMEM;
  if (P->n == 0 || P->k == 0) return solve_impl(P, L, ldl, Linv, B, ldb, X, ldx, nullptr, nullptr,
                                                0, stream, info);
  void* base = nullptr;
  TRSM_TRY(scratch_for_current_device(&base));
  const int64_t split = (int64_t)std::min(P->ws_split_bytes, kNoAllocScratchBytes - need);
  return solve_impl(P, L, ldl, Linv, B, ldb, X, ldx, base, (char*)base + need, split, stream,
                    info);
}

size_t trsm_residual_workspace_bytes(int64_t n, int64_t k) {
  if (n < 0 || k < 0) return 0;
  return align_up(2 * kNormBlocks * 8) + align_up(8 * 8) + align_up(split_bytes(n * k));
}

trsm_status trsm_residual(int64_t n, int64_t k, const double* L, int64_t ldl, const double* X,
                          int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                          void* workspace, double* norms, void* stream) {
  if (n < 0 || k < 0 || !norms) return TRSM_EINVAL;
  norms[0] = norms[1] = norms[2] = 0.0;
  if (n == 0 || k == 0) return TRSM_OK;
  if (!L || !X || !B || !R || !workspace) return TRSM_EINVAL;
  if (ldl < n || ldx < k || ldb < k || ldr < k) return TRSM_EINVAL;
  const size_t rb = ((size_t)(n - 1) * ldr + k) * 8;
  if (ranges_overlap(R, rb, X, ((size_t)(n - 1) * ldx + k) * 8) ||
      ranges_overlap(R, rb, B, ((size_t)(n - 1) * ldb + k) * 8) ||
      ranges_overlap(R, rb, L, ((size_t)(n - 1) * ldl + n) * 8))
    return TRSM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)workspace;
  double* dn = (double*)((char*)workspace + align_up(2 * kNormBlocks * 8));
  SplitScope split_scope((char*)workspace + align_up(2 * kNormBlocks * 8) + align_up(8 * 8),
                         (int64_t)split_bytes(n * k));
  TRSM_HIP(gemm_simple<double>(L, ldl, X, ldx, B, ldb, R, ldr, n, k, n, -1.0, 1.0, G_A_LOWER, s));
  TRSM_HIP(launch_sumsq_max(R, ldr, n, k, part, dn, s));
  TRSM_HIP(launch_sumsq_max(X, ldx, n, k, part, dn + 2, s));
  double h[4];
  TRSM_HIP(hipMemcpyAsync(h, dn, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  TRSM_HIP(hipStreamSynchronize(s));
  norms[0] = sqrt(h[0]);
  norms[1] = sqrt(h[2]);
  norms[2] = h[1];
  return TRSM_OK;
}

trsm_status trsm_plan_set_tolerance(trsm_plan_t P, double tol) {
  if (!P || !(tol >= 0.0) || !(tol < 1.0)) return TRSM_EINVAL;
  P->tol = tol;
  return TRSM_OK;
}

trsm_status trsm_plan_set_timing(trsm_plan_t P, int enable) {
  if (!P) return TRSM_EINVAL;
  P->timer.enabled = enable != 0;
  P->timer.used = 0;
  return TRSM_OK;
}

trsm_status trsm_plan_timing(trsm_plan_t P, int64_t* launches, double* ms, double* flops) {
  if (!P || !launches || !ms || !flops) return TRSM_EINVAL;
  LaunchTimer& t = P->timer;
  double tot_ms = 0.0, tot_fl = 0.0;
  for (size_t i = 0; i < t.used; ++i) {
    TRSM_HIP(hipEventSynchronize(t.ev[2 * i + 1]));
    float e = 0.f;
    TRSM_HIP(hipEventElapsedTime(&e, t.ev[2 * i], t.ev[2 * i + 1]));
    tot_ms += e;
    tot_fl += t.flops[i];
  }
  *launches = (int64_t)t.used;
  *ms = tot_ms;
  *flops = tot_fl;
  t.used = 0;
  return TRSM_OK;
}

}  // extern "C"
