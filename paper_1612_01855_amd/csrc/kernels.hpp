// Launchers of the non-GEMM kernels (defined in kernels.hip).
#pragma once

#include "common.hpp"

namespace trsm {

// Copy the m diagonal n0 x n0 blocks of L (lower part, zeros above) into the
// packed binary64 buffer Linv; positions past row/column n get the identity.
// Records min(row) of any zero / non-finite diagonal entry in *bad.  With
// `upper`, L is an upper-triangular U and the blocks copied are U_bb^T (the
// lower triangles of the transposed diagonal blocks; U below its diagonal is
// not read).
template <typename TL>
hipError_t launch_extract_diag(const TL* L, int64_t ldl, int64_t n, int64_t n0, int64_t m,
                               double* Linv, unsigned long long* bad, hipStream_t s,
                               bool upper = false);

// Invert, in place, every nb x nb diagonal leaf of every packed block
// (nb <= 64): column-oriented substitution on the identity in LDS.
hipError_t launch_trtri_leaf(double* Linv, int64_t n0, int64_t m, int64_t nb, hipStream_t s);

// Zero the strict upper triangle of every packed block.
hipError_t launch_zero_upper(double* Linv, int64_t n0, int64_t m, hipStream_t s);

// out[i] = (TO) in[i]
template <typename TI, typename TO>
hipError_t launch_convert(const TI* in, TO* out, int64_t count, hipStream_t s);

// Dense 2-D copy / convert with scaling: out[i*ldo+j] = (TO)(scale * in[i*ldi+j]).
template <typename TI, typename TO>
hipError_t launch_copy2d(const TI* in, int64_t ldi, TO* out, int64_t ldo, int64_t rows,
                         int64_t cols, double scale, hipStream_t s);

// X[i*ldx+j] += scale * D[i*ldd+j]  (binary64 X, binary32 D), or X = scale*D
// when `assign`.
hipError_t launch_axpy_f32_to_f64(const float* D, int64_t ldd, double* X, int64_t ldx,
                                  int64_t rows, int64_t cols, double scale, bool assign,
                                  hipStream_t s);

// Low-precision copy of the strictly-lower off-diagonal blocks of L:
// Llow[r*n + c] = l[r][c] * 2^e(r, blk) for c < n0*floor(r/n0), with one
// power-of-two scale per (row, column block) chosen from the row segment's
// largest magnitude (target: largest magnitude near `target`), and
// rscale[r*m + blk] = 2^-e (exact inverse scale).
template <typename TO>
hipError_t launch_lowcopy(const double* L, int64_t ldl, int64_t n, int64_t n0, int64_t m,
                          TO* Llow, float* rscale, float target, hipStream_t s);

// out[r * cols + c] = low(a[r * cols + c] 2^e_r), one power-of-two scale per
// row placing its largest magnitude just below `target`; rs[r] = 2^-e_r.
template <typename TO>
hipError_t launch_rowscale_copy(const double* a, int64_t rows, int64_t cols, TO* out, float* rs,
                               float target, hipStream_t s);

// Low-precision, transposed copy of a solved block of X with a power-of-two
// scale taken from the block's largest magnitude (found on the device):
// XT[c*ldx + r] = low(2^e * D[r*ldd + c]), 2^e placing the largest magnitude
// in [2^etarget, 2^(etarget+1)); writes *xinv = 2^-e (exact inverse).
// *amax is working space and must be zero on entry (launch_fill_u32).
template <typename TO>
hipError_t launch_lowx(const float* D, int64_t ldd, int64_t rows, int64_t cols, TO* XT,
                       int64_t ldx, unsigned* amax, float* xinv, int etarget, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t s);

// Forward substitution on an nb x nb lower-triangular leaf (nb <= 64) for k
// right-hand-side columns, in place on X: the recursive baseline's base case
// (no inversion).  One thread per column.
template <typename T>
hipError_t launch_subst_leaf(const T* L, int64_t ldl, T* X, int64_t ldx, int64_t nb,
                             int64_t k, hipStream_t s);

// Deterministic reductions of a binary64 n x k matrix (fixed block split,
// fixed order): partial sums of squares and maxima into `part` (device,
// 2 * kNormBlocks doubles), then the final values into out[0] = sum of
// squares, out[1] = max |a|.
constexpr int kNormBlocks = 1024;
hipError_t launch_sumsq_max(const double* A, int64_t lda, int64_t rows, int64_t cols,
                            double* part, double* out, hipStream_t s);

// Frobenius norm squared of the lower triangle of L into out[0] (deterministic).
template <typename TL>
hipError_t launch_sumsq_lower(const TL* L, int64_t ldl, int64_t n, double* part, double* out,
                              hipStream_t s);

// A synthetic, well-conditioned system for timing runs: L[i][i] in [1, 2),
// L[i][j] in (-1/n, 1/n) below the diagonal, 0 above; B[i][c] in (-1/2, 1/2)
// (counter-based hash of (i, j, seed)).  L is n x n, B is n x k, both dense
// row-major.
template <typename T>
hipError_t launch_fill_system(T* L, int64_t n, T* B, int64_t k, uint64_t seed, hipStream_t s);

// Transpose of `batch` rows x cols matrices (batch strides si, so elements):
// out[c*ldo + r] = (TO) in[r*ldi + c]; with lower_only, entries with r < c
// (above in's diagonal) are written as zeros instead (out is then the upper
// triangular transpose of in's lower triangle, whose upper part is never read).
template <typename TI, typename TO>
hipError_t launch_transpose(const TI* in, int64_t ldi, TO* out, int64_t ldo, int64_t rows,
                            int64_t cols, int64_t batch, int64_t si, int64_t so, bool lower_only,
                            hipStream_t s);

// Record a HIP error for trsm_last_hip_error() (thread-local); returns
// TRSM_EHIP's numeric value for convenience.
int note_hip_error(hipError_t e);

}  // namespace trsm
