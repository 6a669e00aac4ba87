// Exact integer products for the refinement residual R = B - L X (the
// defect of the postcondition B = L X of Alg. It-Inv-TRSM), evaluated on the
// int8 matrix cores through a residue number system.
//
// L's strictly lower part E is scaled row by row by a power of two and
// rounded to integers of at most `a` bits: Eq[i][j] = round(E[i][j] 2^sL_i).
// A correction piece Y (n x k) is scaled column by column and rounded to at
// most `b` bits: Yq[i][c] = round(Y[i][c] 2^tY_c).  The integer product
// C = Eq Yq has |C| < n 2^(a+b); with pairwise coprime moduli m_p <= 256 whose
// product M exceeds 4 |C|, C is recovered exactly from the P products
// (Eq mod m_p)(Yq mod m_p) mod m_p, each an int8 x int8 -> int32 product with
// no rounding (|sum| < 2^30 for n <= 2^16), by the Chinese remainder theorem.
// Then L Yq 2^-tY = diag(L) Yq 2^-tY + C 2^(-sL - tY) with one binary64
// rounding per element, and R is updated in binary64.  The refinement then
// converges to the solution of the system whose strictly lower part is
// Eq 2^-sL, an L perturbed by at most 2^-a relative to each row's largest
// entry; `a` is chosen from L's own magnitudes so that this perturbation is
// below binary64's backward-error level.
#pragma once

#include "common.hpp"

namespace trsm {
namespace crt {

constexpr int kMaxModuli = 16;
// Residue planes kept per matrix: enough for a + b + log2(n) + 2 <= 94 bits.
constexpr int kPlanes = 12;
// Largest n: n terms of |z| <= 2^14 must stay below 2^30 in int32.
constexpr int64_t kMaxN = (int64_t)1 << 16;
// Target of the perturbation of L's strictly lower part: ||E - Eq 2^-sL||_F
// <= 2^-kTargetBits ||L||_F (about 3.6e-15, binary64's backward-error level).
constexpr double kTargetBits = 48.0;

// Pairwise coprime moduli, largest first (2^8, then odd numbers <= 255), so
// that every residue fits a signed byte.
constexpr int kModuli[kMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                     229, 227, 223, 217, 211, 199, 197, 193};

// Explicit CRT data for the first P moduli: C = (sum_p z_p W_p) mod M, with
// W_p = (M/m_p) * ((M/m_p)^-1 mod m_p) < M split into 24-bit limbs, so that
// every limb product z_p w and every limb sum is an exact binary64 integer.
struct Table {
  int P;
  int mod[kMaxModuli];
  float inv[kMaxModuli];        // 1 / m_p (binary32)
  double invd[kMaxModuli];      // 1 / m_p (binary64)
  double Wd[kMaxModuli][4];     // W_p as four 24-bit limbs (exact binary64 integers)
  double Md4[4];                // M as four 24-bit limbs
  double Md;                    // M rounded to binary64
  double inv_Md;
  double log2M;
};

// Host: the table for the first P moduli (P <= 12, so that M < 2^96).
Table make_table(int P);
// Smallest P whose modulus product satisfies log2 M >= bits (P <= 12), or -1.
int moduli_for_bits(double bits);

// Per-row data of L's strictly lower part: rowmax[i] = max_{j<i} |l_ij| and
// stats[0] += sum_i i rowmax_i^2 (deterministic partials, then a final pass).
hipError_t launch_row_stats(const double* L, int64_t ldl, int64_t n, double* rowmax,
                            double* part, double* stats, hipStream_t s);

// Device: a = clamp(ceil(target_bits + log2(sqrt(stats[0]) / ||L||_F)), 24, 50), from
// stats[0] and lnorm2 = ||L||_F^2 (lower triangle); written to *a_out.
hipError_t launch_choose_bits(const double* stats, const double* lnorm2, double target_bits,
                              int* a_out, hipStream_t s);

// Residue planes of Eq: planes[p * plane + i * lde + j] = Eq[i][j] mod m_p for
// j < i (zero for j >= i, and for rows n <= i < npad), p < P, over columns
// j < min(lde, 256 * ceil((i + 1) / 256)) (the columns the lower-triangular
// products read).  sl[i] receives sL_i.
hipError_t launch_l_residues(const double* L, int64_t ldl, int64_t n, int64_t npad,
                             const double* rowmax, const int* a_dev, const Table& t,
                             int8_t* planes, int64_t lde, int64_t plane, int* sl, hipStream_t s);

// Column maxima of |Y| as binary32 bit patterns rounded up, and the sum of
// squares of Y in binary64 over a fixed partition (partials in `part`, at
// most kRecBlocks entries; the total in out[0]).
template <typename TY>
hipError_t launch_dstats(const TY* Y, int64_t ldy, int64_t n, int64_t k, unsigned* colmax,
                         double* part, double* out, hipStream_t s);

// Round the piece Y (binary32) to b <= 24 bits per column (tY_c from colmax:
// |Yq| <= 2^b 2^-tY_c), in place, and write its residue planes transposed:
// planes[p * plane + c * ldq + i] = Yq[i][c] 2^tY_c mod m_p, with zeros for
// n <= i < npad.  ty[c] receives tY_c.
hipError_t launch_y_residues(float* Y, int64_t ldy, int64_t n, int64_t npad, int64_t k,
                             const unsigned* colmax, int b, const Table& t, int8_t* planes,
                             int64_t ldq, int64_t plane, int* ty, hipStream_t s);

// Recombine: C from the P residue planes Z (n x ldz each), then with the
// rounded piece's value y = Yq 2^yshift:
//   Rout[i][c] = Rin[i][c] - l_ii y[i][c] - C[i][c] 2^(yshift - sL_i - tY_c)
// and Rl[i * k + c] = (float)Rout[i][c] (the next low-precision right-hand
// side); xmode 1: X = y, 2: X += y, 0: X untouched.  Rout may equal Rin.
// Partial sums of squares / maxima go to `part` (fixed split), the final
// values to out[0..3] = {sum Rout^2, max |Rout|, sum X^2, max |X|} (the X
// entries are zero when xmode is 0).
hipError_t launch_recombine(const int8_t* Z, int64_t ldz, int64_t zplane, const Table& t,
                            const int* sl, const int* ty, const float* Yq, int64_t ldy, int yshift,
                            const double* L, int64_t ldl, const double* Rin, int64_t ldri,
                            double* Rout, int64_t ldro, float* Rl, double* X, int64_t ldx,
                            int xmode, int64_t n, int64_t k, double* part, double* out,
                            hipStream_t s);

// X (+)= Y0 2^s0 + Y1 2^s1 + Y2 2^s2 in binary64 (Y1, Y2 may be null).
hipError_t launch_assemble(const float* Y0, int s0, const float* Y1, int s1, const float* Y2,
                           int s2, int64_t ldy, double* X, int64_t ldx, int64_t n, int64_t k,
                           bool accumulate, hipStream_t s);

constexpr int kRecBlocks = 1024;   // fixed block count of the recombination's partials
constexpr int kStatSlabs = 16;     // row slabs of the correction statistics (partials:
                                   // ceil(k / 64) * kStatSlabs, at most kRecBlocks * kStatSlabs)

}  // namespace crt
}  // namespace trsm
