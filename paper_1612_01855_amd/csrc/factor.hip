// Blocked factorizations whose panel steps are the triangular solve of Alg.
// It-Inv-TRSM with whole inverted diagonal blocks: Cholesky A = L L^T (C ABI
// trsm_chol_*) and LU without row exchanges A = L U (trsm_lu_*), both binary64
// (see include/trsm.h).
//
// The abstract and Sec. I name Cholesky as a factorization whose main
// subroutine is TRSM.  Right-looking, block size nb:
//
//   for each diagonal block S_j (nb rows, the last one ragged):
//     factor A(S_j, S_j) = L_jj L_jj^T and form Linv_jj = L_jj^{-1}
//     L(T_j, S_j) = A(T_j, S_j) Linv_jj^T          (the panel solve)
//     A(T_j, T_j) -= L(T_j, S_j) L(T_j, S_j)^T      (lower triangle only)
//
// The panel solve X L_jj^T = A(T_j, S_j) has nb columns of L and n - (j+1) nb
// rows of right-hand sides: the one-large-dimension regime of Sec. VIII,
// where the rule takes n0 equal to the whole triangle (here nb), so it is a
// single product with the inverted block.  The diagonal block is factored
// recursively: halves h and s - h,
//
//   factor D11 -> L11, Linv11;   L21 = D21 Linv11^T;   D22 -= L21 L21^T;
//   factor D22 -> L22, Linv22;   Linv21 = -(Linv22 L21) Linv11,
//
// the last line being Alg. RecTriInv's combine, so the inverse of the block
// is built along the way; 64 x 64 leaves are factored and inverted in LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/trsm.h"
#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace trsm {

namespace {

constexpr int kLeaf = 64;
constexpr int64_t kDefaultNb = 512;
constexpr int64_t kLargeN = 12288;
constexpr int64_t kMidN = 6144;
constexpr int64_t kMaxNb = 4096;
constexpr size_t kCholSplitBytes = (size_t)32 << 20;
constexpr size_t kAl = 256;
inline size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

inline int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Value of lane `lane` (a wave-uniform constant) for every lane.
__device__ __forceinline__ double lane_value(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Leaf: the s x s (s <= 64) diagonal block D (lower triangle read) is
// factored by wave 0 and inverted by wave 1, one step behind it.  Wave 0,
// lane i holding row i of the block in registers (positions past s hold the
// identity), right-looking, step j: every lane takes the pivot a_jj from
// lane j, then
//   l_jj = sqrt(a_jj),  l_ij = a_ij / l_jj   (column j published in LDS),
//   a_ic -= l_ij l_cj                        for c > j.
// Entries above the diagonal are updated too (they are never read), so no
// lane is masked.  Wave 1, lane t holding column t of the inverse (starting
// from the identity), takes column j of L from LDS in the next step:
//   x_jt *= 1 / l_jj,   x_rt -= l_rj x_jt   for r > j,
// i.e. x_rt = (delta_rt - sum_{p<r} l_rp x_pt) / l_rr with the sum taken in
// p order.  The two waves share one register array (each uses it for its
// own role).  L goes back to D's lower triangle (the strict upper triangle
// is not written), the inverse to V (ld ldv; nothing above the diagonal is
// written).  A pivot that is not positive (or NaN) records its global row in
// *bad (the smallest one wins) and is replaced by 1 so that the arithmetic
// stays finite.  LDS reads come in 16-byte pairs issued ahead of their use.
constexpr int kLdc = kLeaf + 2;   // column stride of Lc (16-byte aligned rows)
constexpr int kAhead = 8;         // LDS pair reads in flight
constexpr int kGroup = 8;         // leaf steps between the two waves' barriers

__global__ __launch_bounds__(2 * kLeaf) void chol_leaf_kernel(double* __restrict__ D,
                                                              int64_t ldd, int s,
                                                              double* __restrict__ V,
                                                              int64_t ldv, int64_t row0,
                                                              unsigned long long* bad) {
  __shared__ __attribute__((aligned(16))) double Lc[kLeaf][kLdc];
  __shared__ double rdiag[kLeaf];
  typedef double D2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x, i = tid % kLeaf;
  const bool w0 = tid < kLeaf;    // wave 0 factors, wave 1 inverts
  // coalesced load, all loads of a thread issued before any is used: thread
  // (wave w, lane i) takes column i of rows w, w + 2, ...
  {
    double v[kLeaf / 2];
#pragma unroll
    for (int q = 0; q < kLeaf / 2; ++q) {
      const int r = 2 * q + (w0 ? 0 : 1);
      v[q] = (r < s && i <= r) ? D[(int64_t)r * ldd + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kLeaf / 2; ++q) {
      const int r = 2 * q + (w0 ? 0 : 1);
      Lc[r][i] = (r >= s && r == i) ? 1.0 : v[q];
    }
  }
  __syncthreads();
  double a[kLeaf];   // wave 0: row i of the block; wave 1: column i of the inverse
  if (w0) {
#pragma unroll
    for (int c = 0; c < kLeaf; c += 2) {
      const D2 v = *reinterpret_cast<const D2*>(&Lc[i][c]);
      a[c] = v.x;
      a[c + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kLeaf; ++r) a[r] = (r == i) ? 1.0 : 0.0;
  }
  __syncthreads();
  // the loop is kept free of per-lane branches (they split it into blocks that
  // the register allocator handles badly): failures are collected in `first`.
  // Column j + 1 is finished and published right after its own update in
  // step j, so its square root and division can overlap the rest of step j.
  int first = kLeaf;
  auto publish = [&](int j) {
    double piv = lane_value(a[j], j);
    const bool ok = piv > 0.0;
    first = (!ok && first == kLeaf) ? j : first;
    piv = ok ? piv : 1.0;
    const double d = sqrt(piv);
    const double l = (i == j) ? d : a[j] / d;
    a[j] = l;
    Lc[j][i] = l;
    rdiag[j] = 1.0 / d;
  };
  if (w0) publish(0);
  // Steps go in groups of kGroup between barriers: wave 0 factors group g
  // while wave 1 inverts with the columns of group g - 1.
#pragma unroll
  for (int g = 0; g <= kLeaf / kGroup; ++g) {
    if (w0 && g < kLeaf / kGroup) {
#pragma unroll
      for (int j = g * kGroup; j < (g + 1) * kGroup && j + 1 < kLeaf; ++j) {
        const double l = a[j];
        // l_{j+1,j} straight from lane j + 1: the next pivot's chain
        // does not wait for LDS
        a[j + 1] = fma(-l, lane_value(l, j + 1), a[j + 1]);
        publish(j + 1);
        // the rest of the row, c >= j + 2, in pairs read kAhead pairs ahead
        const int q0 = (j + 2) / 2;
        D2 buf[kLeaf / 2];
#pragma unroll
        for (int q = q0; q < kLeaf / 2 && q < q0 + kAhead; ++q)
          buf[q] = *reinterpret_cast<const D2*>(&Lc[j][2 * q]);
#pragma unroll
        for (int q = q0; q < kLeaf / 2; ++q) {
          if (q + kAhead < kLeaf / 2)
            buf[q + kAhead] = *reinterpret_cast<const D2*>(&Lc[j][2 * (q + kAhead)]);
          if (2 * q >= j + 2) a[2 * q] = fma(-l, buf[q].x, a[2 * q]);
          a[2 * q + 1] = fma(-l, buf[q].y, a[2 * q + 1]);
        }
      }
    }
    if (!w0 && g >= 1) {
#pragma unroll
      for (int jj = (g - 1) * kGroup; jj < g * kGroup; ++jj) {
        // column jj of L was published before the last barrier
        a[jj] *= rdiag[jj];
        const int q0 = (jj + 1) / 2;
        D2 buf[kLeaf / 2];
#pragma unroll
        for (int q = q0; q < kLeaf / 2 && q < q0 + kAhead; ++q)
          buf[q] = *reinterpret_cast<const D2*>(&Lc[jj][2 * q]);
#pragma unroll
        for (int q = q0; q < kLeaf / 2; ++q) {
          if (q + kAhead < kLeaf / 2)
            buf[q + kAhead] = *reinterpret_cast<const D2*>(&Lc[jj][2 * (q + kAhead)]);
          if (2 * q > jj) a[2 * q] = fma(-buf[q].x, a[jj], a[2 * q]);
          a[2 * q + 1] = fma(-buf[q].y, a[jj], a[2 * q + 1]);
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && first < s) atomicMin(bad, (unsigned long long)(row0 + first));
  // L back to D, rows coalesced (element (r, i) is Lc[i][r]), both waves
  for (int r = (w0 ? 0 : 1); r < s; r += 2)
    if (i <= r) D[(int64_t)r * ldd + i] = Lc[i][r];
  __syncthreads();
  // column i of the inverse through LDS, then coalesced rows (r >= i)
  if (!w0) {
#pragma unroll
    for (int r = 0; r < kLeaf; ++r) Lc[r][i] = a[r];
  }
  __syncthreads();
  for (int r = (w0 ? 0 : 1); r < kLeaf; r += 2)
    if (i <= r) V[(int64_t)r * ldv + i] = Lc[r][i];
}

// Linv blocks: zero everywhere except the identity on the padded diagonal of
// the ragged last block; the status word starts at "no failure".
__global__ void chol_init_kernel(double* __restrict__ V, int64_t n, int64_t nb, int64_t m,
                                 unsigned long long* bad) {
  const int64_t per = nb * nb, total = per * m;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) *bad = ~0ull;
  for (int64_t idx = tid; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / per, e = idx % per, i = e / nb, j = e % nb;
    V[idx] = (i == j && b * nb + i >= n) ? 1.0 : 0.0;
  }
}

// LU leaf: the s x s (s <= 64) diagonal block D is factored without row
// exchanges by four waves, right-looking, step j (u_jj the pivot):
//   l_ij = d_ij / u_jj (i > j),  u_jc = d_jc (c >= j),  d_ic -= l_ij u_jc (i, c > j).
// Wave 0 holds row i in lane i and publishes column j of L in LDS; wave 1
// holds column c in lane c and publishes row j of U; after one barrier each
// takes the other's half for its update (both compute the same products, so
// their U parts stay bitwise equal; wave 1 never scales its entries below the
// diagonal, which nothing reads), while wave 2 (column t of L^{-1}, unit
// diagonal) and wave 3 (column t of (U^T)^{-1}, i.e. row t of U^{-1}) take
// step j of their substitutions from the same two published vectors:
//   x_rt -= l_rj x_jt (r > j);   z_jt /= u_jj,  z_rt -= u_jr z_jt (r > j).
// Every wave consumes step j's vectors within step j, so two LDS slots per
// vector suffice (2 KB in all: the leaf fits beside the trailing products'
// workgroups); the block goes between global memory and registers directly.
// Positions past s hold the identity.  L (strictly lower) and U go back to
// D, the inverses to VL (unit lower, diagonal stored) and VU (upper), ld ldv,
// nothing written on their other side.  A zero or non-finite pivot records
// its global row in *bad (the smallest one wins) and is replaced by 1 in the
// divisions of L.  LDS reads come in 16-byte pairs issued ahead of their use.
__global__ __launch_bounds__(4 * kLeaf) void lu_leaf_kernel(double* __restrict__ D,
                                                            int64_t ldd, int s,
                                                            double* __restrict__ VL,
                                                            double* __restrict__ VU,
                                                            int64_t ldv, int64_t row0,
                                                            unsigned long long* bad) {
  __shared__ __attribute__((aligned(16))) double Lr[2][kLdc];   // slot: l_rj, column j of L
  __shared__ __attribute__((aligned(16))) double Ur[2][kLdc];   // slot: u_jc, row j of U
  typedef double D2 __attribute__((ext_vector_type(2)));
  const int tid = threadIdx.x, w = tid / kLeaf, i = tid % kLeaf;
  // wave 0: row i; wave 1: column i; waves 2, 3: column i of the identity
  double a[kLeaf];
  if (w == 0) {
#pragma unroll
    for (int c = 0; c < kLeaf; ++c)
      a[c] = (i < s && c < s) ? D[(int64_t)i * ldd + c] : (c == i ? 1.0 : 0.0);
  } else if (w == 1) {
#pragma unroll
    for (int r = 0; r < kLeaf; ++r)
      a[r] = (r < s && i < s) ? D[(int64_t)r * ldd + i] : (r == i ? 1.0 : 0.0);
  } else {
#pragma unroll
    for (int r = 0; r < kLeaf; ++r) a[r] = (r == i) ? 1.0 : 0.0;
  }
  int first = kLeaf;
  // a[c] -= m * P[c] for c > j, P a published LDS vector read in pairs
  auto axpy = [&](const double* P, double m, int j) {
    const int q0 = (j + 1) / 2;
    D2 buf[kLeaf / 2];
#pragma unroll
    for (int q = q0; q < kLeaf / 2 && q < q0 + kAhead; ++q)
      buf[q] = *reinterpret_cast<const D2*>(P + 2 * q);
#pragma unroll
    for (int q = q0; q < kLeaf / 2; ++q) {
      if (q + kAhead < kLeaf / 2) buf[q + kAhead] = *reinterpret_cast<const D2*>(P + 2 * (q + kAhead));
      if (2 * q > j) a[2 * q] = fma(-m, buf[q].x, a[2 * q]);
      a[2 * q + 1] = fma(-m, buf[q].y, a[2 * q + 1]);
    }
  };
#pragma unroll
  for (int j = 0; j < kLeaf; ++j) {
    const int slot = j & 1;
    if (w == 0) {
      double piv = lane_value(a[j], j);
      const bool ok = (piv != 0.0) && isfinite(piv);
      first = (!ok && first == kLeaf) ? j : first;
      piv = ok ? piv : 1.0;
      const double l = (i > j) ? a[j] / piv : 0.0;
      a[j] = (i > j) ? l : a[j];
      Lr[slot][i] = l;
    } else if (w == 1) {
      Ur[slot][i] = a[j];
    }
    __syncthreads();
    if (w == 0) {
      axpy(&Ur[slot][0], (i > j) ? a[j] : 0.0, j);         // row i: -= l_ij u_j.
    } else if (w == 1) {
      const double u = (i > j) ? a[j] : 0.0;               // column i: -= l_.j u_ji
#pragma unroll
      for (int q = (j + 1) / 2; q < kLeaf / 2; ++q) {
        const D2 v = *reinterpret_cast<const D2*>(&Lr[slot][2 * q]);
        if (2 * q > j) a[2 * q] = fma(-v.x, u, a[2 * q]);
        a[2 * q + 1] = fma(-v.y, u, a[2 * q + 1]);
      }
    } else if (w == 2) {
      axpy(&Lr[slot][0], a[j], j);                         // x_r -= l_rj x_j
    } else {
      a[j] = a[j] / Ur[slot][j];                           // z_j /= u_jj
      axpy(&Ur[slot][0], a[j], j);                         // z_r -= u_jr z_j
    }
  }
  if (tid == 0 && first < s) atomicMin(bad, (unsigned long long)(row0 + first));
  if (w == 0) {
    if (i < s) {
#pragma unroll
      for (int c = 0; c < kLeaf; ++c)
        if (c < s) D[(int64_t)i * ldd + c] = a[c];
    }
  } else if (w == 2) {
#pragma unroll
    for (int r = 0; r < kLeaf; ++r)
      if (r >= i) VL[(int64_t)r * ldv + i] = a[r];
  } else if (w == 3) {
#pragma unroll
    for (int c = 0; c < kLeaf; ++c)
      if (c >= i) VU[(int64_t)i * ldv + c] = a[c];
  }
}

struct Ctx {
  double* A;
  int64_t lda, n, nb;
  double* V = nullptr;      // m inverted diagonal blocks, nb x nb each (LU: of L)
  double* VU = nullptr;     // LU: m inverted diagonal blocks of U
  double* W = nullptr;      // nb x nb: the diagonal block's panel and combine
  double* W2[2] = {};       // (n - nb) x nb each: the outer panel L(T_j, S_j), by parity of j
  double* WU[2] = {};       // LU: nb x (n - nb) each: the outer panel U(S_j, T_j)
  void* split;    // split-K scratch
  size_t split_bytes;
  unsigned long long* bad;
  hipStream_t s;
};

// C = alpha * A op(B) (+ C when accumulate); op(B) = B^T stored as N x K rows
// when BT.  Products with fewer than two 128 x 128 workgroups per compute
// unit take 64 x 64 tiles (and split K when still small, if `split`: the
// products inside a diagonal block are too small for the finishing pass to
// pay off).
template <bool BT>
hipError_t prod(const Ctx& c, const double* A, int64_t lda, const double* B, int64_t ldb,
                double* C, int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha,
                bool accumulate, uint32_t flags, bool split = true) {
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
  p.part = split ? c.split : nullptr;
  p.part_bytes = split ? (int64_t)c.split_bytes : 0;
  const bool small = gemm_wgs(p.M, p.N, p.K, flags, 128, 128) < kSplitTarget;
  return small ? launch_gemm<double, double, double, float, 64, 64, 2, 2, BT>(p, 1, c.s)
               : launch_gemm<double, double, double, float, 128, 128, 2, 2, BT>(p, 1, c.s);
}

#define CHOL_HIP(...)                                           \
  do {                                                          \
    hipError_t e_ = (__VA_ARGS__);                              \
    if (e_ != hipSuccess) return (trsm_status)note_hip_error(e_); \
  } while (0)

#define CHOL_TRY(...)                 \
  do {                                \
    trsm_status s_ = (__VA_ARGS__);   \
    if (s_ != TRSM_OK) return s_;     \
  } while (0)

// Factor the s x s diagonal block at global row r0 and write its inverse at V
// (ld nb).
trsm_status factor_diag(const Ctx& c, int64_t r0, int64_t s, double* V) {
  const int64_t lda = c.lda, nb = c.nb;
  double* D = c.A + r0 * lda + r0;
  if (s <= kLeaf) {
    chol_leaf_kernel<<<1, 2 * kLeaf, 0, c.s>>>(D, lda, (int)s, V, nb, r0, c.bad);
    CHOL_HIP(hipGetLastError());
    return TRSM_OK;
  }
  const int64_t h = kLeaf * ((s + 2 * kLeaf - 1) / (2 * kLeaf));
  const int64_t t = s - h;
  double* D21 = D + h * lda;
  double* D22 = D21 + h;
  double* V21 = V + h * nb;
  double* V22 = V21 + h;
  CHOL_TRY(factor_diag(c, r0, h, V));
  // L21 = D21 Linv11^T.  With h <= 64 the product has one column tile, so
  // each workgroup reads its rows of D21 in full before it writes them and
  // the product runs in place; otherwise it goes through W.
  const double* L21 = D21;
  int64_t ld21 = lda;
  if (h <= kLeaf) {
    CHOL_HIP(prod<true>(c, D21, lda, V, nb, D21, lda, t, h, h, 1.0, false, 0u, false));
  } else {
    CHOL_HIP(prod<true>(c, D21, lda, V, nb, c.W, nb, t, h, h, 1.0, false, 0u, false));
    CHOL_HIP(launch_copy2d<double, double>(c.W, nb, D21, lda, t, h, 1.0, c.s));
    L21 = c.W;
    ld21 = nb;
  }
  // D22 -= L21 L21^T, lower triangle
  CHOL_HIP(prod<true>(c, L21, ld21, L21, ld21, D22, lda, t, t, h, -1.0, true, G_C_LOWER, false));
  CHOL_TRY(factor_diag(c, r0 + h, t, V22));
  // Linv21 = -(Linv22 L21) Linv11
  CHOL_HIP(prod<false>(c, V22, nb, D21, lda, c.W, nb, t, h, t, 1.0, false,
                       G_A_LOWER | G_A_ZERO_UPPER, false));
  CHOL_HIP(prod<false>(c, c.W, nb, V, nb, V21, nb, t, h, h, -1.0, false, G_B_LOWER, false));
  return TRSM_OK;
}

// The library's second stream and its events, per device: the lookahead
// runs the bulk of each trailing update there.  Enqueueing is serialised by
// the mutex (the events are reused from one step to the next: a wait takes
// the event's state at the moment it is enqueued).
struct Side {
  std::mutex mu;
  hipStream_t s2 = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};
constexpr int kMaxDevices = 64;
Side g_side[kMaxDevices];

// The device's side stream and events, created on first use (under the
// device's mutex, which the caller then keeps while it enqueues); they live
// until the process ends.
trsm_status side_for(Side** out, std::unique_lock<std::mutex>* lock) {
  int dev = 0;
  CHOL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return TRSM_EINVAL;
  Side& sd = g_side[dev];
  *lock = std::unique_lock<std::mutex>(sd.mu);
  if (!sd.s2) {
    hipStream_t s2 = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    CHOL_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    for (auto& e : ev) CHOL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int i = 0; i < 3; ++i) sd.ev[i] = ev[i];
    sd.s2 = s2;
  }
  *out = &sd;
  return TRSM_OK;
}

trsm_status init(const Ctx& c, int64_t m) {
  const int64_t total = m * c.nb * c.nb;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
  chol_init_kernel<<<g, 256, 0, c.s>>>(c.V, c.n, c.nb, m, c.bad);
  CHOL_HIP(hipGetLastError());
  return TRSM_OK;
}

// One stream: diagonal block, panel, trailing update, in order.
trsm_status factor_serial(const Ctx& c) {
  const int64_t n = c.n, nb = c.nb, m = (n + nb - 1) / nb, lda = c.lda;
  CHOL_TRY(init(c, m));
  for (int64_t j = 0; j < m; ++j) {
    const int64_t r0 = j * nb, s = std::min(nb, n - r0), t = n - r0 - s;
    double* Vj = c.V + j * nb * nb;
    CHOL_TRY(factor_diag(c, r0, s, Vj));
    if (t <= 0) break;
    double* A21 = c.A + (r0 + s) * lda + r0;
    double* A22 = A21 + s;
    // L(T_j, S_j) = A(T_j, S_j) Linv_jj^T
    CHOL_HIP(prod<true>(c, A21, lda, Vj, nb, c.W2[0], nb, t, s, s, 1.0, false, 0u));
    CHOL_HIP(launch_copy2d<double, double>(c.W2[0], nb, A21, lda, t, s, 1.0, c.s));
    // A(T_j, T_j) -= L(T_j, S_j) L(T_j, S_j)^T, lower triangle
    CHOL_HIP(prod<true>(c, c.W2[0], nb, c.W2[0], nb, A22, lda, t, t, s, -1.0, true, G_C_LOWER));
  }
  return TRSM_OK;
}

// Lookahead over two streams.  Update j, A(T_j, T_j) -= P_j P_j^T, is split
// into the next diagonal block A(S_{j+1}, S_{j+1}) (on the caller's stream,
// the critical chain) and everything below it, A(T_{j+1}, S_{j+1} u T_{j+1})
// (on the side stream).  The side part of update j runs while the chain
// factors diagonal block j+1, whose inputs are complete once the chain's own
// part of update j is done (the side parts of earlier updates, which also
// touched that block, were finished before panel j).  Panel j+1 then waits
// for the side part of update j (event 2), which wrote the rows it reads;
// the side part of update j+1 waits for panel j+1 (event 1).  Panels
// alternate between two buffers, so panel j+1 never overwrites the one the
// side stream may still be reading.
trsm_status factor_lookahead(const Ctx& c, Side& sd) {
  const int64_t n = c.n, nb = c.nb, m = (n + nb - 1) / nb, lda = c.lda;
  hipStream_t s2 = sd.s2;
  Ctx c2 = c;
  c2.s = s2;
  c2.split = nullptr;
  c2.split_bytes = 0;
  CHOL_TRY(init(c, m));
  CHOL_HIP(hipEventRecord(sd.ev[0], c.s));
  CHOL_HIP(hipStreamWaitEvent(s2, sd.ev[0], 0));
  bool pending = false;
  for (int64_t j = 0; j < m; ++j) {
    const int64_t r0 = j * nb, s = std::min(nb, n - r0), t = n - r0 - s;
    double* Vj = c.V + j * nb * nb;
    CHOL_TRY(factor_diag(c, r0, s, Vj));
    if (t <= 0) break;
    double* P = c.W2[j & 1];
    double* A21 = c.A + (r0 + s) * lda + r0;
    double* A22 = A21 + s;
    if (pending) CHOL_HIP(hipStreamWaitEvent(c.s, sd.ev[2], 0));
    CHOL_HIP(prod<true>(c, A21, lda, Vj, nb, P, nb, t, s, s, 1.0, false, 0u));
    CHOL_HIP(launch_copy2d<double, double>(P, nb, A21, lda, t, s, 1.0, c.s));
    const int64_t s1 = std::min(nb, t);
    // the next diagonal block, lower triangle, on the chain
    CHOL_HIP(prod<true>(c, P, nb, P, nb, A22, lda, s1, s1, s, -1.0, true, G_C_LOWER));
    if (t > s1) {
      CHOL_HIP(hipEventRecord(sd.ev[1], c.s));
      CHOL_HIP(hipStreamWaitEvent(s2, sd.ev[1], 0));
      // rows T_{j+1}: block column S_{j+1}, then the lower triangle of T_{j+1}
      CHOL_HIP(prod<true>(c2, P + s1 * nb, nb, P, nb, A22 + s1 * lda, lda, t - s1, s1, s, -1.0,
                          true, 0u));
      CHOL_HIP(prod<true>(c2, P + s1 * nb, nb, P + s1 * nb, nb, A22 + s1 * lda + s1, lda,
                          t - s1, t - s1, s, -1.0, true, G_C_LOWER));
      CHOL_HIP(hipEventRecord(sd.ev[2], s2));
      pending = true;
    } else {
      pending = false;
    }
  }
  // join: the caller's stream sees the side stream's work
  CHOL_HIP(hipEventRecord(sd.ev[2], s2));
  CHOL_HIP(hipStreamWaitEvent(c.s, sd.ev[2], 0));
  return TRSM_OK;
}

// ---------------------------------------------------------------------------
// LU without row exchanges.  Diagonal block of s rows at global row r0, its
// inverses at VL / VU (ld nb): halves h and s - h,
//   factor D11 -> L11, U11, Linv11, Uinv11;
//   L21 = D21 Uinv11;  U12 = Linv11 D12;  D22 -= L21 U12;
//   factor D22 -> L22, U22, Linv22, Uinv22;
//   Linv21 = -(Linv22 L21) Linv11;  Uinv12 = -(Uinv11 U12) Uinv22,
// the last two being Alg. RecTriInv's combine for the lower and the upper
// factor.
trsm_status lu_factor_diag(const Ctx& c, int64_t r0, int64_t s, double* VL, double* VU) {
  const int64_t lda = c.lda, nb = c.nb;
  double* D = c.A + r0 * lda + r0;
  if (s <= kLeaf) {
    lu_leaf_kernel<<<1, 4 * kLeaf, 0, c.s>>>(D, lda, (int)s, VL, VU, nb, r0, c.bad);
    CHOL_HIP(hipGetLastError());
    return TRSM_OK;
  }
  const int64_t h = kLeaf * ((s + 2 * kLeaf - 1) / (2 * kLeaf));
  const int64_t t = s - h;
  double* D12 = D + h;
  double* D21 = D + h * lda;
  double* D22 = D21 + h;
  CHOL_TRY(lu_factor_diag(c, r0, h, VL, VU));
  // L21 = D21 Uinv11 and U12 = Linv11 D12.  With h <= 64 each product has
  // one tile along the dimension it overwrites (columns of L21, rows of U12),
  // so every workgroup reads its part of the operand in full before writing
  // it and the product runs in place; otherwise it goes through W.
  if (h <= kLeaf) {
    CHOL_HIP(prod<false>(c, D21, lda, VU, nb, D21, lda, t, h, h, 1.0, false, 0u, false));
    CHOL_HIP(prod<false>(c, VL, nb, D12, lda, D12, lda, h, t, h, 1.0, false,
                         G_A_LOWER | G_A_ZERO_UPPER, false));
  } else {
    CHOL_HIP(prod<false>(c, D21, lda, VU, nb, c.W, nb, t, h, h, 1.0, false, 0u, false));
    CHOL_HIP(launch_copy2d<double, double>(c.W, nb, D21, lda, t, h, 1.0, c.s));
    CHOL_HIP(prod<false>(c, VL, nb, D12, lda, c.W, nb, h, t, h, 1.0, false,
                         G_A_LOWER | G_A_ZERO_UPPER, false));
    CHOL_HIP(launch_copy2d<double, double>(c.W, nb, D12, lda, h, t, 1.0, c.s));
  }
  // D22 -= L21 U12
  CHOL_HIP(prod<false>(c, D21, lda, D12, lda, D22, lda, t, t, h, -1.0, true, 0u, false));
  CHOL_TRY(lu_factor_diag(c, r0 + h, t, VL + h * nb + h, VU + h * nb + h));
  // Linv21 = -(Linv22 L21) Linv11
  CHOL_HIP(prod<false>(c, VL + h * nb + h, nb, D21, lda, c.W, nb, t, h, t, 1.0, false,
                       G_A_LOWER | G_A_ZERO_UPPER, false));
  CHOL_HIP(prod<false>(c, c.W, nb, VL, nb, VL + h * nb, nb, t, h, h, -1.0, false, G_B_LOWER,
                       false));
  // Uinv12 = -(Uinv11 U12) Uinv22
  CHOL_HIP(prod<false>(c, VU, nb, D12, lda, c.W, nb, h, t, h, 1.0, false, G_A_UPPER, false));
  CHOL_HIP(prod<false>(c, c.W, nb, VU + h * nb + h, nb, VU + h, nb, h, t, t, -1.0, false, 0u,
                       false));
  return TRSM_OK;
}

trsm_status lu_init(const Ctx& c, int64_t m) {
  CHOL_TRY(init(c, m));
  Ctx cu = c;
  cu.V = c.VU;
  return init(cu, m);
}

// One stream: diagonal block, both panels, trailing update, in order.
trsm_status lu_factor_serial(const Ctx& c) {
  const int64_t n = c.n, nb = c.nb, m = (n + nb - 1) / nb, lda = c.lda;
  CHOL_TRY(lu_init(c, m));
  for (int64_t j = 0; j < m; ++j) {
    const int64_t r0 = j * nb, s = std::min(nb, n - r0), t = n - r0 - s;
    double* VLj = c.V + j * nb * nb;
    double* VUj = c.VU + j * nb * nb;
    CHOL_TRY(lu_factor_diag(c, r0, s, VLj, VUj));
    if (t <= 0) break;
    double* A12 = c.A + r0 * lda + r0 + s;
    double* A21 = c.A + (r0 + s) * lda + r0;
    double* A22 = A21 + s;
    const int64_t ldu = n - nb;
    // L(T_j, S_j) = A(T_j, S_j) Uinv_jj;  U(S_j, T_j) = Linv_jj A(S_j, T_j)
    CHOL_HIP(prod<false>(c, A21, lda, VUj, nb, c.W2[0], nb, t, s, s, 1.0, false, 0u));
    CHOL_HIP(launch_copy2d<double, double>(c.W2[0], nb, A21, lda, t, s, 1.0, c.s));
    CHOL_HIP(prod<false>(c, VLj, nb, A12, lda, c.WU[0], ldu, s, t, s, 1.0, false,
                         G_A_LOWER | G_A_ZERO_UPPER));
    CHOL_HIP(launch_copy2d<double, double>(c.WU[0], ldu, A12, lda, s, t, 1.0, c.s));
    // A(T_j, T_j) -= L(T_j, S_j) U(S_j, T_j)
    CHOL_HIP(prod<false>(c, c.W2[0], nb, c.WU[0], ldu, A22, lda, t, t, s, -1.0, true, 0u));
  }
  return TRSM_OK;
}

// Lookahead over two streams, as for Cholesky: update j is split into the
// next diagonal block (on the caller's stream) and the rest, the rows below
// it and the columns right of it (on the side stream), which overlaps the
// factorization of diagonal block j+1; panels j+1 wait for it.
trsm_status lu_factor_lookahead(const Ctx& c, Side& sd) {
  const int64_t n = c.n, nb = c.nb, m = (n + nb - 1) / nb, lda = c.lda;
  const int64_t ldu = n - nb;
  hipStream_t s2 = sd.s2;
  Ctx c2 = c;
  c2.s = s2;
  c2.split = nullptr;
  c2.split_bytes = 0;
  CHOL_TRY(lu_init(c, m));
  CHOL_HIP(hipEventRecord(sd.ev[0], c.s));
  CHOL_HIP(hipStreamWaitEvent(s2, sd.ev[0], 0));
  bool pending = false;
  for (int64_t j = 0; j < m; ++j) {
    const int64_t r0 = j * nb, s = std::min(nb, n - r0), t = n - r0 - s;
    double* VLj = c.V + j * nb * nb;
    double* VUj = c.VU + j * nb * nb;
    CHOL_TRY(lu_factor_diag(c, r0, s, VLj, VUj));
    if (t <= 0) break;
    double* PL = c.W2[j & 1];
    double* PU = c.WU[j & 1];
    double* A12 = c.A + r0 * lda + r0 + s;
    double* A21 = c.A + (r0 + s) * lda + r0;
    double* A22 = A21 + s;
    if (pending) CHOL_HIP(hipStreamWaitEvent(c.s, sd.ev[2], 0));
    CHOL_HIP(prod<false>(c, A21, lda, VUj, nb, PL, nb, t, s, s, 1.0, false, 0u));
    CHOL_HIP(launch_copy2d<double, double>(PL, nb, A21, lda, t, s, 1.0, c.s));
    CHOL_HIP(prod<false>(c, VLj, nb, A12, lda, PU, ldu, s, t, s, 1.0, false,
                         G_A_LOWER | G_A_ZERO_UPPER));
    CHOL_HIP(launch_copy2d<double, double>(PU, ldu, A12, lda, s, t, 1.0, c.s));
    const int64_t s1 = std::min(nb, t);
    // the next diagonal block on the chain
    CHOL_HIP(prod<false>(c, PL, nb, PU, ldu, A22, lda, s1, s1, s, -1.0, true, 0u));
    if (t > s1) {
      CHOL_HIP(hipEventRecord(sd.ev[1], c.s));
      CHOL_HIP(hipStreamWaitEvent(s2, sd.ev[1], 0));
      // rows of S_{j+1} right of its diagonal block, then all rows below it
      CHOL_HIP(prod<false>(c2, PL, nb, PU + s1, ldu, A22 + s1, lda, s1, t - s1, s, -1.0, true,
                           0u));
      CHOL_HIP(prod<false>(c2, PL + s1 * nb, nb, PU, ldu, A22 + s1 * lda, lda, t - s1, t, s,
                           -1.0, true, 0u));
      CHOL_HIP(hipEventRecord(sd.ev[2], s2));
      pending = true;
    } else {
      pending = false;
    }
  }
  CHOL_HIP(hipEventRecord(sd.ev[2], s2));
  CHOL_HIP(hipStreamWaitEvent(c.s, sd.ev[2], 0));
  return TRSM_OK;
}

struct Sizes {
  int64_t nb;
  size_t linv, off_w, off_w2, w2_bytes, off_split, ws;
  size_t off_wu = 0;   // LU only: two nb x (n - nb) panels of U after the split scratch
};

trsm_status sizes_for(int64_t n, int64_t nb, Sizes* z, bool lu = false) {
  if (n < 0 || nb < 0) return TRSM_EINVAL;
  // measured: 128-row blocks are the fastest up to n = 4096, 256-row ones at
  // 8192 and 512-row ones at 16384
  if (nb == 0)
    nb = std::min<int64_t>(
        n >= kLargeN ? kDefaultNb : (n >= kMidN ? kDefaultNb / 2 : kDefaultNb / 4),
        pow2_at_least(std::max<int64_t>(n, kLeaf)));
  if (nb < kLeaf || nb > kMaxNb || (nb & (nb - 1))) return TRSM_EINVAL;
  if (n > (int64_t)1 << 20) return TRSM_EINVAL;
  // no block larger than the matrix rounded up to a power of two (the cap a
  // TRSM plan puts on n0), so that the inverted blocks keep a plan's layout
  nb = std::min<int64_t>(nb, pow2_at_least(std::max<int64_t>(n, kLeaf)));
  const int64_t m = n > 0 ? (n + nb - 1) / nb : 0;
  z->nb = nb;
  // a TRSM_F64 plan's Linv buffer with n0 = nb: the packed inverses, then
  // the 256 bytes of that plan's status word
  z->linv = al((size_t)m * nb * nb * 8) + al(8);
  size_t off = kAl;                                 // status word
  z->off_w = off;
  off += al((size_t)nb * nb * 8);
  z->off_w2 = off;
  z->w2_bytes = al((size_t)std::max<int64_t>(n - nb, 1) * nb * 8);
  off += 2 * al((size_t)std::max<int64_t>(n - nb, 1) * nb * 8);
  z->off_split = off;
  off += kCholSplitBytes;
  if (lu) {
    z->off_wu = off;
    off += 2 * z->w2_bytes;
  }
  z->ws = off;
  return TRSM_OK;
}

}  // namespace
}  // namespace trsm

using namespace trsm;

extern "C" {

trsm_status trsm_chol_sizes(int64_t n, int64_t nb, int64_t* nb_used, size_t* linv_bytes,
                            size_t* workspace_bytes) {
  Sizes z;
  CHOL_TRY(sizes_for(n, nb, &z));
  if (nb_used) *nb_used = z.nb;
  if (linv_bytes) *linv_bytes = z.linv;
  if (workspace_bytes) *workspace_bytes = z.ws;
  return TRSM_OK;
}

trsm_status trsm_chol_factor(int64_t n, double* A, int64_t lda, int64_t nb, double* Linv,
                             void* workspace, void* stream) {
  Sizes z;
  CHOL_TRY(sizes_for(n, nb, &z));
  if (!workspace || (n > 0 && (!A || !Linv)) || lda < std::max<int64_t>(n, 1))
    return TRSM_EINVAL;
  if (((uintptr_t)workspace & (kAl - 1)) || ((uintptr_t)Linv & 15)) return TRSM_EINVAL;
  Ctx c;
  c.A = A;
  c.lda = lda;
  c.n = n;
  c.nb = z.nb;
  c.V = Linv;
  char* w = static_cast<char*>(workspace);
  c.bad = reinterpret_cast<unsigned long long*>(w);
  c.W = reinterpret_cast<double*>(w + z.off_w);
  c.W2[0] = reinterpret_cast<double*>(w + z.off_w2);
  c.W2[1] = reinterpret_cast<double*>(w + z.off_w2 + z.w2_bytes);
  c.split = w + z.off_split;
  c.split_bytes = kCholSplitBytes;
  c.s = static_cast<hipStream_t>(stream);
  if (n == 0) {
    chol_init_kernel<<<1, 64, 0, c.s>>>(nullptr, 0, z.nb, 0, c.bad);
    CHOL_HIP(hipGetLastError());
    return TRSM_OK;
  }
  // the lookahead pays once there are a few blocks to overlap
  if ((n + z.nb - 1) / z.nb <= 2) return factor_serial(c);
  Side* sd = nullptr;
  std::unique_lock<std::mutex> lock;
  CHOL_TRY(side_for(&sd, &lock));
  return factor_lookahead(c, *sd);
}

trsm_status trsm_chol_check(const void* workspace, trsm_status* status, int64_t* index) {
  if (!workspace || !status || !index) return TRSM_EINVAL;
  unsigned long long v = 0;
  CHOL_HIP(hipDeviceSynchronize());
  CHOL_HIP(hipMemcpy(&v, workspace, sizeof(v), hipMemcpyDeviceToHost));
  if (v == ~0ull) {
    *status = TRSM_OK;
    *index = -1;
  } else {
    *status = TRSM_ESINGULAR;
    *index = (int64_t)v;
  }
  return TRSM_OK;
}

trsm_status trsm_lu_sizes(int64_t n, int64_t nb, int64_t* nb_used, size_t* inv_bytes,
                          size_t* workspace_bytes) {
  Sizes z;
  CHOL_TRY(sizes_for(n, nb, &z, true));
  if (nb_used) *nb_used = z.nb;
  if (inv_bytes) *inv_bytes = z.linv;
  if (workspace_bytes) *workspace_bytes = z.ws;
  return TRSM_OK;
}

trsm_status trsm_lu_factor(int64_t n, double* A, int64_t lda, int64_t nb, double* Linv,
                           double* Uinv, void* workspace, void* stream) {
  Sizes z;
  CHOL_TRY(sizes_for(n, nb, &z, true));
  if (!workspace || (n > 0 && (!A || !Linv || !Uinv)) || lda < std::max<int64_t>(n, 1))
    return TRSM_EINVAL;
  if (((uintptr_t)workspace & (kAl - 1)) || ((uintptr_t)Linv & 15) || ((uintptr_t)Uinv & 15))
    return TRSM_EINVAL;
  Ctx c;
  c.A = A;
  c.lda = lda;
  c.n = n;
  c.nb = z.nb;
  c.V = Linv;
  c.VU = Uinv;
  char* w = static_cast<char*>(workspace);
  c.bad = reinterpret_cast<unsigned long long*>(w);
  c.W = reinterpret_cast<double*>(w + z.off_w);
  c.W2[0] = reinterpret_cast<double*>(w + z.off_w2);
  c.W2[1] = reinterpret_cast<double*>(w + z.off_w2 + z.w2_bytes);
  c.WU[0] = reinterpret_cast<double*>(w + z.off_wu);
  c.WU[1] = reinterpret_cast<double*>(w + z.off_wu + z.w2_bytes);
  c.split = w + z.off_split;
  c.split_bytes = kCholSplitBytes;
  c.s = static_cast<hipStream_t>(stream);
  if (n == 0) {
    chol_init_kernel<<<1, 64, 0, c.s>>>(nullptr, 0, z.nb, 0, c.bad);
    CHOL_HIP(hipGetLastError());
    return TRSM_OK;
  }
  if ((n + z.nb - 1) / z.nb <= 2) return lu_factor_serial(c);
  Side* sd = nullptr;
  std::unique_lock<std::mutex> lock;
  CHOL_TRY(side_for(&sd, &lock));
  return lu_factor_lookahead(c, *sd);
}

trsm_status trsm_lu_check(const void* workspace, trsm_status* status, int64_t* index) {
  return trsm_chol_check(workspace, status, index);
}

}  // extern "C"

