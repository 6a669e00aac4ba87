// LU factorization with partial pivoting, P A = L U (binary64), built on the
// triangular solve of Alg. It-Inv-TRSM (C ABI trsm_lu_piv_*, see
// include/trsm.h).  The abstract and Sec. I name LU as a factorization whose
// main subroutine is TRSM; the row exchanges make it apply to every
// nonsingular matrix.
//
// Right-looking with block columns of nb (a power of two), each factored in
// panels of kPw = 32 columns:
//
//   for each block column S_j = [c0, c0 + s):
//     for each panel [c, c + w) of it:
//       factor A(c:n, c:c+w) with row exchanges          (cooperative kernel)
//       exchange the same rows in the block's other columns
//       A(c:c+w, c+w:c0+s) = Lp^{-1} A(c:c+w, c+w:c0+s)  (unit lower, w x w)
//       A(c+w:n, c+w:c0+s) -= A(c+w:n, c:c+w) A(c:c+w, c+w:c0+s)
//     exchange the block's rows in the columns outside it (L's columns to
//       the left, the trailing columns to the right)
//     Linv_jj = L_jj^{-1}  (Alg. Diagonal-Inverter + RecTriInv on the unit
//       lower diagonal block, through trsm_invert_diag)
//     U(S_j, T_j) = Linv_jj A(S_j, T_j)         (the panel solve: one product)
//     A(T_j, T_j) -= L(T_j, S_j) U(S_j, T_j)
//
// The panel kernel keeps one row of the panel per thread in registers, rows
// split over G workgroups that are co-resident (cooperative launch), and
// meets at one device-wide barrier per column: every workgroup publishes its
// best candidate (largest magnitude, the first position on ties, positions
// being the row order after the exchanges so far) together with that row's
// values; after the barrier each picks the winner from the G candidates,
// reads its row, and eliminates its own rows.  The exchanges are kept as
// positions and applied when the panel is written back.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/trsm.h"
#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace trsm {
namespace {

constexpr int kPw = 32;               // panel width
constexpr int kRows = 256;            // panel rows per workgroup (one per thread)
constexpr int kMaxGroups = 256;       // workgroups of a panel: n <= kRows * kMaxGroups
constexpr int kSlot = kPw + 2;        // doubles per candidate slot: |a|, position, row
constexpr unsigned kSpinLimit = 1u << 24;
constexpr size_t kAl = 256;
constexpr size_t kSplitBytes = (size_t)32 << 20;
inline size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

// Status words at the start of the workspace.
struct Words {
  unsigned long long bad;   // smallest column with a zero or non-finite pivot
  unsigned bar;             // barrier arrivals (monotone over the factorization)
  unsigned err;             // a barrier wait gave up
};

__device__ __forceinline__ bool better(double a, int pa, double b, int pb) {
  // larger magnitude first; on equal magnitudes the smaller position
  return a > b || (a == b && pa < pb);
}

// Argmax over the workgroup of (value, position, thread): the result lands in
// s_v / s_p / s_t.  NaN magnitudes never win (comparisons are false).
__device__ __forceinline__ void block_argmax(double v, int p, int t, double* s_v, int* s_p,
                                             int* s_t) {
  __shared__ double wv[kRows / 64];
  __shared__ int wp[kRows / 64], wt[kRows / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int op = __shfl_xor(p, o, 64), ot = __shfl_xor(t, o, 64);
    if (better(ov, op, v, p)) {
      v = ov;
      p = op;
      t = ot;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wv[w] = v;
    wp[w] = p;
    wt[w] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = wv[0];
    int bp = wp[0], bt = wt[0];
    for (int i = 1; i < kRows / 64; ++i)
      if (better(wv[i], wp[i], bv, bp)) {
        bv = wv[i];
        bp = wp[i];
        bt = wt[i];
      }
    *s_v = bv;
    *s_p = bp;
    *s_t = bt;
  }
  __syncthreads();
}

// Panel A(r0:r0+h, c0:c0+w) (w <= kPw) factored with row exchanges by G =
// gridDim.x co-resident workgroups; workgroup g owns rows g*kRows.. of the
// panel.  slots: 2 x G candidate slots (by step parity).  ipiv[c0 + j]
// receives the absolute row exchanged with row r0 + j.  words->bar counts
// barrier arrivals from `base`.
__global__ __launch_bounds__(kRows) void piv_panel_kernel(double* __restrict__ A, int64_t lda,
                                                          int64_t r0, int64_t c0, int h, int w,
                                                          int64_t* __restrict__ ipiv,
                                                          double* __restrict__ slots,
                                                          Words* __restrict__ words,
                                                          unsigned base) {
  __shared__ double s_v;
  __shared__ int s_p, s_t;
  __shared__ double cand[kMaxGroups * kSlot];   // the G candidates of a step
  __shared__ int piv[kPw];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lr = g * kRows + tid;         // this thread's panel row (original order)
  const bool own = lr < h;
  double a[kPw];
#pragma unroll
  for (int c = 0; c < kPw; ++c)
    a[c] = (own && c < w) ? A[(r0 + lr) * lda + c0 + c] : 0.0;
  int pos = lr;                           // position in the exchanged order
  bool act = own;
  for (int j = 0; j < w; ++j) {
    // this workgroup's candidate for column j
    double v = -1.0;
#pragma unroll
    for (int c = 0; c < kPw; ++c)
      if (c == j) v = act ? fabs(a[c]) : -1.0;
    block_argmax(v, act ? pos : INT32_MAX, tid, &s_v, &s_p, &s_t);
    double* slot = slots + ((size_t)(j & 1) * G + g) * kSlot;
    if (tid == s_t) {
      // the candidate, stored at agent scope and released by its own wave
      // before the workgroup meets; thread 0's arrival comes after that
      __hip_atomic_store(&slot[0], s_v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&slot[1], (double)s_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int c = 0; c < kPw; ++c)
        __hip_atomic_store(&slot[2 + c], a[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
    }
    __syncthreads();
    if (tid == 0) {
      const unsigned target = base + (unsigned)G * (unsigned)(j + 1);
      __hip_atomic_fetch_add(&words->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      unsigned spins = 0;
      while (__hip_atomic_load(&words->bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kSpinLimit) {
          atomicOr(&words->err, 1u);
          break;
        }
      }
    }
    __syncthreads();
    // every candidate in one round of agent-scope loads (no stale cache
    // lines; thread 0's acquire and the barrier order them after every
    // workgroup's arrival), then the winner: largest magnitude, first position
    const double* sl = slots + (size_t)(j & 1) * G * kSlot;
    for (int e = tid; e < G * kSlot; e += kRows)
      cand[e] = __hip_atomic_load(&sl[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const double cv = tid < G ? cand[tid * kSlot] : -1.0;
    const int cp = tid < G ? (int)cand[tid * kSlot + 1] : INT32_MAX;
    block_argmax(cv, cp, tid, &s_v, &s_p, &s_t);
    // a position outside j .. h-1 can only come from candidates read after a
    // barrier wait gave up (reported through the error word): fall back to j
    // so that every row still goes back to a row of the panel
    int p = s_p;
    if (p < j || p >= h) {
      p = j;
      if (tid == 0) atomicOr(&words->err, 2u);
    }
    const double best = s_v;
    const double* u = cand + s_t * kSlot + 2;   // the pivot row
    if (tid == 0) piv[j] = p;
    const bool zero = !(best > 0.0) || !(best <= 1.7976931348623157e308);
    if (zero && g == 0 && tid == 0) atomicMin(&words->bad, (unsigned long long)(c0 + j));
    // exchange positions j and p; the pivot row leaves the elimination
    if (act && pos == p) {
      pos = j;
      act = false;
    } else if (act && pos == j) {
      pos = p;
    }
    if (act && !zero) {
      double pj = 0.0, l = 0.0;
#pragma unroll
      for (int c = 0; c < kPw; ++c)
        if (c == j) pj = u[c];
#pragma unroll
      for (int c = 0; c < kPw; ++c)
        if (c == j) l = a[c] / pj;
#pragma unroll
      for (int c = 0; c < kPw; ++c) {
        if (c == j) a[c] = l;
        else if (c > j && c < w) a[c] = fma(-l, u[c], a[c]);
      }
    }
    __syncthreads();   // cand is rewritten at the next step
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < kPw; ++c)
      if (c < w) A[(r0 + pos) * lda + c0 + c] = a[c];
  }
  if (g == 0 && tid < w) ipiv[c0 + tid] = r0 + piv[tid];
}

// Row exchanges "swap rows k and ipiv[k]" for k = k0 .. k1-1, in order, on
// columns [lo1, hi1) and [lo2, hi2) of A (one thread per column).
__global__ __launch_bounds__(256) void swap_rows_kernel(double* __restrict__ A, int64_t lda,
                                                        const int64_t* __restrict__ ipiv,
                                                        int64_t k0, int64_t k1, int64_t lo1,
                                                        int64_t hi1, int64_t lo2, int64_t hi2) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n1 = hi1 - lo1;
  const int64_t c = t < n1 ? lo1 + t : lo2 + (t - n1);
  if (t >= n1 + (hi2 - lo2)) return;
  for (int64_t k = k0; k < k1; ++k) {
    const int64_t q = ipiv[k];
    if (q == k) continue;
    const double x = A[k * lda + c], y = A[q * lda + c];
    A[k * lda + c] = y;
    A[q * lda + c] = x;
  }
}

// B(c:c+w, cols) = Lp^{-1} B(c:c+w, cols) for the unit lower w x w Lp stored
// strictly below the diagonal of A(c:c+w, c:c+w): one thread per column,
// its column in LDS, rows in order (x_i = b_i - sum_{p<i} l_ip x_p).
constexpr int kSolveCols = 64;
__global__ __launch_bounds__(kSolveCols) void unit_lower_solve_kernel(const double* __restrict__ L,
                                                                      double* __restrict__ B,
                                                                      int64_t lda, int w,
                                                                      int64_t ncols) {
  __shared__ double Ls[kPw][kPw + 1];
  __shared__ double xs[kPw][kSolveCols];
  for (int e = threadIdx.x; e < kPw * kPw; e += kSolveCols) {
    const int i = e / kPw, p = e % kPw;
    Ls[i][p] = (i < w && p < i) ? L[i * lda + p] : 0.0;
  }
  const int t = threadIdx.x;
  const int64_t col = (int64_t)blockIdx.x * kSolveCols + t;
  const bool live = col < ncols;
  for (int i = 0; i < w; ++i) xs[i][t] = live ? B[i * lda + col] : 0.0;
  __syncthreads();
  for (int i = 1; i < w; ++i) {
    double acc = xs[i][t];
    for (int p = 0; p < i; ++p) acc = fma(-Ls[i][p], xs[p][t], acc);
    xs[i][t] = acc;
  }
  if (live)
    for (int i = 0; i < w; ++i) B[i * lda + col] = xs[i][t];
}

// W (nb x nb) = the unit lower triangle of the s x s block D: strictly lower
// part from D, ones on the diagonal, zeros above, identity past s.
__global__ __launch_bounds__(256) void unit_lower_copy_kernel(const double* __restrict__ D,
                                                              int64_t ldd, int64_t s,
                                                              double* __restrict__ W, int64_t nb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nb * nb) return;
  const int64_t i = e / nb, c = e % nb;
  W[e] = (c < i) ? ((i < s) ? D[i * ldd + c] : 0.0) : (c == i ? 1.0 : 0.0);
}

#define PIV_HIP(...)                                              \
  do {                                                            \
    hipError_t e_ = (__VA_ARGS__);                                \
    if (e_ != hipSuccess) return (trsm_status)note_hip_error(e_); \
  } while (0)

#define PIV_TRY(...)                 \
  do {                               \
    trsm_status s_ = (__VA_ARGS__);  \
    if (s_ != TRSM_OK) return s_;    \
  } while (0)

struct Layout {
  int64_t nb, m;
  size_t words, slots, w, winv, wu, split, total, inv_bytes, plan_linv;
};

int64_t default_nb(int64_t n) { return n <= 4096 ? 256 : 512; }

inline int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

trsm_status layout_for(int64_t n, int64_t nb, Layout* L) {
  if (n <= 0 || n > (int64_t)kRows * kMaxGroups) return TRSM_EINVAL;
  if (nb < 0 || (nb > 0 && (nb < kPw || (nb & (nb - 1))))) return TRSM_EINVAL;
  if (nb == 0) nb = default_nb(n);
  // a solve plan caps its block size at the next power of two >= n
  nb = std::max<int64_t>(kPw, std::min(nb, pow2_at_least(n)));
  L->nb = nb;
  L->m = (n + nb - 1) / nb;
  trsm_plan_t plan = nullptr;
  PIV_TRY(trsm_plan(nb, 1, TRSM_F64, nb, 0, &plan));
  trsm_plan_info pi;
  const trsm_status st = trsm_plan_get_info(plan, &pi);
  trsm_plan_destroy(plan);
  if (st != TRSM_OK) return st;
  L->plan_linv = pi.linv_bytes;
  L->words = al(sizeof(Words));
  L->slots = al((size_t)2 * kMaxGroups * kSlot * sizeof(double));
  L->w = al((size_t)nb * nb * 8);
  L->winv = al(pi.linv_bytes);
  L->wu = al((size_t)nb * std::max<int64_t>(n - nb, 1) * 8);
  L->split = kSplitBytes;
  L->total = L->words + L->slots + L->w + L->winv + L->wu + L->split;
  L->inv_bytes = (size_t)L->m * nb * nb * 8;
  return TRSM_OK;
}

// C = alpha A B (+ C): binary64 product on the solve path's kernel.
hipError_t prod(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha, bool accumulate,
                uint32_t flags, void* split, size_t split_bytes, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  auto p = gemm_params<double, double, double, float>();
  p.A = A; p.lda = lda;
  p.B = B; p.ldb = ldb;
  p.Cout = C; p.ldco = ldc;
  if (accumulate) {
    p.Cin = C;
    p.ldci = ldc;
    p.beta = 1.0;
    flags |= G_BETA;
  }
  p.M = (int)M; p.N = (int)N; p.K = (int)K;
  p.alpha = alpha;
  p.flags = flags;
  p.part = split;
  p.part_bytes = (int64_t)split_bytes;
  const bool small = gemm_wgs(p.M, p.N, p.K, flags, 128, 128) < kSplitTarget;
  return small ? launch_gemm<double, double, double, float, 64, 64, 2, 2, false>(p, 1, s)
               : launch_gemm<double, double, double, float, 128, 128, 2, 2, false>(p, 1, s);
}

hipError_t swap_rows(double* A, int64_t lda, const int64_t* ipiv, int64_t k0, int64_t k1,
                     int64_t lo1, int64_t hi1, int64_t lo2, int64_t hi2, hipStream_t s) {
  hi1 = std::max(hi1, lo1);
  hi2 = std::max(hi2, lo2);
  const int64_t cols = (hi1 - lo1) + (hi2 - lo2);
  if (cols <= 0 || k1 <= k0) return hipSuccess;
  swap_rows_kernel<<<(unsigned)ceil_div(cols, 256), 256, 0, s>>>(A, lda, ipiv, k0, k1, lo1, hi1,
                                                                 lo2, hi2);
  return hipGetLastError();
}

trsm_status factor(int64_t n, double* A, int64_t lda, const Layout& L, int64_t* ipiv,
                   double* Linv, char* ws, hipStream_t s) {
  const int64_t nb = L.nb;
  Words* words = (Words*)ws;
  char* q = ws + L.words;
  double* slots = (double*)q;  q += L.slots;
  double* W = (double*)q;      q += L.w;
  double* Winv = (double*)q;   q += L.winv;
  double* WU = (double*)q;     q += L.wu;
  void* split = q;
  // words: bad = all ones, bar = 0, err = 0
  PIV_HIP(launch_fill_u32((unsigned*)words, 2, 0xFFFFFFFFu, s));
  PIV_HIP(launch_fill_u32((unsigned*)words + 2, 2, 0u, s));
  trsm_plan_t plan = nullptr;
  PIV_TRY(trsm_plan(nb, 1, TRSM_F64, nb, 0, &plan));
  trsm_status st = TRSM_OK;
  unsigned base = 0;
  for (int64_t j = 0; j < L.m && st == TRSM_OK; ++j) {
    const int64_t c0 = j * nb, sb = std::min(nb, n - c0), e0 = c0 + sb;
    for (int64_t c = c0; c < e0; c += kPw) {
      const int w = (int)std::min<int64_t>(kPw, e0 - c);
      const int h = (int)(n - c);
      const int G = (h + kRows - 1) / kRows;
      double* Ap = A;
      int64_t ldap = lda, r0 = c, cc = c;
      int hh = h, ww = w;
      int64_t* ip = ipiv;
      double* sp = slots;
      Words* wp = words;
      unsigned bs = base;
      void* args[] = {&Ap, &ldap, &r0, &cc, &hh, &ww, &ip, &sp, &wp, &bs};
      hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(piv_panel_kernel),
                                                dim3(G), dim3(kRows), args, 0, s);
      if (e != hipSuccess) {
        st = (trsm_status)note_hip_error(e);
        break;
      }
      base += (unsigned)G * (unsigned)w;
      // the panel's exchanges in the block's other columns
      hipError_t e2 = swap_rows(A, lda, ipiv, c, c + w, c0, c, c + w, e0, s);
      if (e2 == hipSuccess && c + w < e0) {
        // U of the panel rows in the block's remaining columns, then the
        // block's trailing rows
        const int64_t nc = e0 - (c + w);
        unit_lower_solve_kernel<<<(unsigned)ceil_div(nc, kSolveCols), kSolveCols, 0, s>>>(
            A + c * lda + c, A + c * lda + c + w, lda, w, nc);
        e2 = hipGetLastError();
        if (e2 == hipSuccess)
          e2 = prod(A + (c + w) * lda + c, lda, A + c * lda + c + w, lda,
                    A + (c + w) * lda + c + w, lda, n - (c + w), nc, w, -1.0, true, 0u, split,
                    kSplitBytes, s);
      }
      if (e2 != hipSuccess) {
        st = (trsm_status)note_hip_error(e2);
        break;
      }
    }
    if (st != TRSM_OK) break;
    // the block's exchanges in the columns left and right of it
    hipError_t e = swap_rows(A, lda, ipiv, c0, e0, 0, c0, e0, n, s);
    // Linv_jj: the unit lower diagonal block, inverted by Alg.
    // Diagonal-Inverter + RecTriInv (one block of nb rows)
    if (e == hipSuccess) {
      unit_lower_copy_kernel<<<(unsigned)ceil_div(nb * nb, 256), 256, 0, s>>>(
          A + c0 * lda + c0, lda, sb, W, nb);
      e = hipGetLastError();
    }
    if (e != hipSuccess) {
      st = (trsm_status)note_hip_error(e);
      break;
    }
    st = trsm_invert_diag(plan, W, nb, Winv, s);
    if (st != TRSM_OK) break;
    e = launch_copy2d<double, double>(Winv, nb, Linv + j * nb * nb, nb, nb, nb, 1.0, s);
    const int64_t t = n - e0;
    if (e == hipSuccess && t > 0) {
      // U(S_j, T_j) = Linv_jj A(S_j, T_j), then the trailing update
      e = prod(Linv + j * nb * nb, nb, A + c0 * lda + e0, lda, WU, t, sb, t, sb, 1.0, false,
               G_A_LOWER | G_A_ZERO_UPPER, split, kSplitBytes, s);
      if (e == hipSuccess) e = launch_copy2d<double, double>(WU, t, A + c0 * lda + e0, lda, sb, t,
                                                             1.0, s);
      if (e == hipSuccess)
        e = prod(A + e0 * lda + c0, lda, A + c0 * lda + e0, lda, A + e0 * lda + e0, lda, t, t, sb,
                 -1.0, true, 0u, split, kSplitBytes, s);
    }
    if (e != hipSuccess) st = (trsm_status)note_hip_error(e);
  }
  trsm_plan_destroy(plan);
  return st;
}

}  // namespace
}  // namespace trsm

using namespace trsm;

extern "C" {

trsm_status trsm_lu_piv_sizes(int64_t n, int64_t nb, int64_t* nb_used, size_t* inv_bytes,
                              size_t* workspace_bytes) {
  Layout L;
  const trsm_status st = layout_for(n, nb, &L);
  if (st != TRSM_OK) return st;
  if (nb_used) *nb_used = L.nb;
  if (inv_bytes) *inv_bytes = L.inv_bytes;
  if (workspace_bytes) *workspace_bytes = L.total;
  return TRSM_OK;
}

trsm_status trsm_lu_piv_factor(int64_t n, double* A, int64_t lda, int64_t nb, int64_t* ipiv,
                               double* Linv, void* workspace, void* stream) {
  if (!A || !ipiv || !Linv || !workspace || lda < n) return TRSM_EINVAL;
  Layout L;
  const trsm_status st = layout_for(n, nb, &L);
  if (st != TRSM_OK) return st;
  if (((uintptr_t)workspace & 255) || ((uintptr_t)A & 15) || ((uintptr_t)Linv & 15))
    return TRSM_EINVAL;
  return factor(n, A, lda, L, ipiv, Linv, static_cast<char*>(workspace), (hipStream_t)stream);
}

trsm_status trsm_lu_piv_check(const void* workspace, trsm_status* status, int64_t* index) {
  if (!workspace || !status) return TRSM_EINVAL;
  Words w;
  if (hipMemcpy(&w, workspace, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess)
    return (trsm_status)note_hip_error(hipGetLastError());
  if (w.err) {
    *status = TRSM_EHIP;
    if (index) *index = -1;
    return TRSM_OK;
  }
  const bool bad = w.bad != ~0ull;
  *status = bad ? TRSM_ESINGULAR : TRSM_OK;
  if (index) *index = bad ? (int64_t)w.bad : -1;
  return TRSM_OK;
}

trsm_status trsm_row_swaps(int64_t k0, int64_t k1, const int64_t* ipiv, double* B, int64_t ldb,
                           int64_t ncols, void* stream) {
  if (k0 < 0 || k1 < k0 || ncols < 0 || (k1 > k0 && (!ipiv || !B)) || ldb < ncols)
    return TRSM_EINVAL;
  const hipError_t e = swap_rows(B, ldb, ipiv, k0, k1, 0, ncols, 0, 0, (hipStream_t)stream);
  return e == hipSuccess ? TRSM_OK : (trsm_status)note_hip_error(e);
}

}  // extern "C"
