// Blocked Cholesky factorization A = L L^T (binary64) whose panel step is the
// triangular solve of Alg. It-Inv-TRSM with whole inverted diagonal blocks,
// and the C ABI trsm_chol_* (see include/trsm.h).
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

#include "../../include/trsm.h"
#include "common.hpp"
#include "gemm.hpp"
#include "kernels.hpp"

namespace trsm {

namespace {

constexpr int kLeaf = 64;
constexpr int64_t kDefaultNb = 256;
constexpr int64_t kMaxNb = 4096;
constexpr size_t kCholSplitBytes = (size_t)32 << 20;
constexpr size_t kAl = 256;
inline size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

inline int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Leaf: the s x s (s <= 64) diagonal block D (lower triangle read) is
// factored in LDS, right-looking, column by column:
//   l_jj = sqrt(d_jj);  l_ij = d_ij / l_jj;  d_ic -= l_ij l_cj  (j < c <= i),
// then inverted by substitution on the identity (thread t owns column t of
// the inverse).  L goes back to D's lower triangle (the strict upper triangle
// is not written), the inverse to V (ld ldv; positions past s hold the
// identity, and nothing above the diagonal is written).  A pivot that is not
// positive (or NaN) records its global row in *bad (the smallest one wins)
// and is replaced by 1 so that the arithmetic stays finite.
__global__ __launch_bounds__(256) void chol_leaf_kernel(double* __restrict__ D, int64_t ldd,
                                                        int s, double* __restrict__ V,
                                                        int64_t ldv, int64_t row0,
                                                        unsigned long long* bad) {
  __shared__ double S[kLeaf][kLeaf + 1];
  __shared__ double X[kLeaf][kLeaf + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kLeaf * kLeaf; e += 256) {
    const int i = e / kLeaf, j = e % kLeaf;
    double v = (i == j) ? 1.0 : 0.0;
    if (i < s && j <= i) v = D[(int64_t)i * ldd + j];
    S[i][j] = v;
    X[i][j] = 0.0;
  }
  __syncthreads();
  const int row = t % kLeaf, cg = t / kLeaf;
  for (int j = 0; j < s; ++j) {
    if (t == 0) {
      double piv = S[j][j];
      if (!(piv > 0.0)) {
        atomicMin(bad, (unsigned long long)(row0 + j));
        piv = 1.0;
      }
      S[j][j] = sqrt(piv);
    }
    __syncthreads();
    if (t > j && t < s) S[t][j] = S[t][j] / S[j][j];
    __syncthreads();
    if (row > j && row < s) {
      const double lij = S[row][j];
      for (int c = j + 1 + cg; c <= row; c += 4) S[row][c] -= lij * S[c][j];
    }
    __syncthreads();
  }
  // inverse: x_tt = 1 / l_tt;  x_it = -(sum_{p<i} l_ip x_pt) / l_ii for i > t;
  // every lane walks the same (i, p) so that l_ip is an LDS broadcast
  if (t < kLeaf) {
    X[t][t] = 1.0 / S[t][t];
    for (int i = 1; i < kLeaf; ++i) {
      if (t < i) {
        double acc = 0.0;
        for (int p = 0; p < i; ++p) acc += S[i][p] * X[p][t];
        X[i][t] = -acc / S[i][i];
      }
    }
  }
  __syncthreads();
  for (int e = t; e < kLeaf * kLeaf; e += 256) {
    const int i = e / kLeaf, j = e % kLeaf;
    if (j > i) continue;
    if (i < s) D[(int64_t)i * ldd + j] = S[i][j];
    V[(int64_t)i * ldv + j] = X[i][j];
  }
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

struct Ctx {
  double* A;
  int64_t lda, n, nb;
  double* V;      // m inverted diagonal blocks, nb x nb each
  double* W;      // nb x nb: the diagonal block's panel and combine
  double* W2;     // (n - nb) x nb: the outer panel L(T_j, S_j)
  void* split;    // split-K scratch
  size_t split_bytes;
  unsigned long long* bad;
  hipStream_t s;
};

// C = alpha * A op(B) (+ C when accumulate); op(B) = B^T stored as N x K rows
// when BT.  Products with fewer than two 128 x 128 workgroups per compute
// unit take 64 x 64 tiles (and split K when still small).
template <bool BT>
hipError_t prod(const Ctx& c, const double* A, int64_t lda, const double* B, int64_t ldb,
                double* C, int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha,
                bool accumulate, uint32_t flags) {
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
  p.part = c.split;
  p.part_bytes = (int64_t)c.split_bytes;
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
    chol_leaf_kernel<<<1, 256, 0, c.s>>>(D, lda, (int)s, V, nb, r0, c.bad);
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
  // L21 = D21 Linv11^T (into W, then back into D21)
  CHOL_HIP(prod<true>(c, D21, lda, V, nb, c.W, nb, t, h, h, 1.0, false, 0u));
  CHOL_HIP(launch_copy2d<double, double>(c.W, nb, D21, lda, t, h, 1.0, c.s));
  // D22 -= L21 L21^T, lower triangle
  CHOL_HIP(prod<true>(c, c.W, nb, c.W, nb, D22, lda, t, t, h, -1.0, true, G_C_LOWER));
  CHOL_TRY(factor_diag(c, r0 + h, t, V22));
  // Linv21 = -(Linv22 L21) Linv11
  CHOL_HIP(prod<false>(c, V22, nb, D21, lda, c.W, nb, t, h, t, 1.0, false,
                       G_A_LOWER | G_A_ZERO_UPPER));
  CHOL_HIP(prod<false>(c, c.W, nb, V, nb, V21, nb, t, h, h, -1.0, false, G_B_LOWER));
  return TRSM_OK;
}

trsm_status factor(const Ctx& c) {
  const int64_t n = c.n, nb = c.nb, m = (n + nb - 1) / nb, lda = c.lda;
  {
    const int64_t total = m * nb * nb;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
    chol_init_kernel<<<g, 256, 0, c.s>>>(c.V, n, nb, m, c.bad);
    CHOL_HIP(hipGetLastError());
  }
  for (int64_t j = 0; j < m; ++j) {
    const int64_t r0 = j * nb, s = std::min(nb, n - r0), t = n - r0 - s;
    double* Vj = c.V + j * nb * nb;
    CHOL_TRY(factor_diag(c, r0, s, Vj));
    if (t <= 0) break;
    double* A21 = c.A + (r0 + s) * lda + r0;
    double* A22 = A21 + s;
    // L(T_j, S_j) = A(T_j, S_j) Linv_jj^T
    CHOL_HIP(prod<true>(c, A21, lda, Vj, nb, c.W2, nb, t, s, s, 1.0, false, 0u));
    CHOL_HIP(launch_copy2d<double, double>(c.W2, nb, A21, lda, t, s, 1.0, c.s));
    // A(T_j, T_j) -= L(T_j, S_j) L(T_j, S_j)^T, lower triangle
    CHOL_HIP(prod<true>(c, c.W2, nb, c.W2, nb, A22, lda, t, t, s, -1.0, true, G_C_LOWER));
  }
  return TRSM_OK;
}

struct Sizes {
  int64_t nb;
  size_t linv, off_w, off_w2, off_split, ws;
};

trsm_status sizes_for(int64_t n, int64_t nb, Sizes* z) {
  if (n < 0 || nb < 0) return TRSM_EINVAL;
  if (nb == 0) nb = std::min<int64_t>(kDefaultNb, pow2_at_least(std::max<int64_t>(n, kLeaf)));
  if (nb < kLeaf || nb > kMaxNb || (nb & (nb - 1))) return TRSM_EINVAL;
  if (n > (int64_t)1 << 20) return TRSM_EINVAL;
  const int64_t m = n > 0 ? (n + nb - 1) / nb : 0;
  z->nb = nb;
  z->linv = al((size_t)m * nb * nb * 8);
  size_t off = kAl;                                 // status word
  z->off_w = off;
  off += al((size_t)nb * nb * 8);
  z->off_w2 = off;
  off += al((size_t)std::max<int64_t>(n - nb, 1) * nb * 8);
  z->off_split = off;
  off += kCholSplitBytes;
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
  c.W2 = reinterpret_cast<double*>(w + z.off_w2);
  c.split = w + z.off_split;
  c.split_bytes = kCholSplitBytes;
  c.s = static_cast<hipStream_t>(stream);
  if (n == 0) {
    chol_init_kernel<<<1, 64, 0, c.s>>>(nullptr, 0, z.nb, 0, c.bad);
    CHOL_HIP(hipGetLastError());
    return TRSM_OK;
  }
  return factor(c);
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

}  // extern "C"
