// Tiled matrix-core GEMM for gfx950, the workhorse of every dense product on
// the solve path: the diagonal-block apply X(S_i) = Linv_ii * B'(S_i) and the
// trailing update B'(T_{i+1}) -= L(T_{i+1}, S_i) X(S_i) of Alg. It-Inv-TRSM,
// the two products of each Alg. RecTriInv combine level, the recursive
// baseline's off-diagonal update, and the residual B - L X.
//
//   Cout = beta * Cin + alpha * rowscale .* (op(A) * op(B))        (per batch)
//
// * A is M x K row-major (k contiguous).  B is K x N row-major (n contiguous)
//   or, with BKMAJOR, stored N x K (k contiguous).  Both are staged through
//   LDS k-contiguous, so every lane reads 32 contiguous bytes of a row.
// * G_A_LOWER: A is lower triangular (A[i][k] = 0 for k > i).  Whole tiles
//   past the diagonal are skipped and the diagonal tile is masked, so
//   whatever is stored above A's diagonal is never used.
// * G_B_LOWER: B is lower triangular (B[k][j] = 0 for k < j), same treatment.
// * G_A_UPPER: A is upper triangular and stores zeros below its diagonal;
//   the chunks left of a tile's diagonal are skipped.
// * Optional second output C2 (another precision, optionally transposed,
//   optionally scaled) feeds a following low-precision product.
// * Batches: z -> offset (z / zdiv) * outer + (z % zdiv) * inner.
//
// Work decomposition: a workgroup of WGM x WGN waves owns a BM x BN tile;
// each wave owns (BM/WGM) x (BN/WGN) made of 16x16 MFMA tiles.  K advances in
// chunks of 128 bytes with two LDS stages and one barrier per chunk.  Aligned
// binary64/binary32 products copy their operands from HBM directly into LDS
// (buffer loads with the LDS modifier, no register staging); the general
// path stages them through registers.  Square lower-triangular products are
// folded so that every workgroup gets equal work.  Tiles are visited in groups of GROUP_M row
// tiles (column-major inside a group) so that concurrently running
// workgroups share A and B panels in L2.  The hardware deals consecutive
// workgroup ids to the eight XCDs in turn; dense products regroup the ids so
// that each XCD works on a contiguous range of tiles (2.3x less L2-miss
// traffic), triangular products keep the round-robin order because a
// contiguous range per XCD unbalanced their uneven tile costs (the
// lower-triangular residual ran twice as slow).
#pragma once

#include "common.hpp"

#include <algorithm>
#include <type_traits>

namespace trsm {

enum GemmFlags : uint32_t {
  G_A_LOWER = 1u,
  G_B_LOWER = 2u,
  G_C2_T = 4u,       // C2 stored transposed: C2[col * ldc2 + row]
  G_BETA = 8u,       // read Cin
  G_ROWSCALE = 16u,  // multiply the product by rscale[row * ld_rs]
  G_A_ZERO_UPPER = 32u,  // with G_A_LOWER: A's upper triangle is stored as zeros (no masking)
  G_A_UPPER = 64u,       // A upper triangular with zeros stored below the diagonal: the
                         // zero chunks are skipped (no masking)
  G_C_LOWER = 128u,      // only the lower triangle of a square C (M == N, BM == BN) is
                         // computed: tiles above the diagonal are not launched and elements
                         // above it are left untouched (the symmetric rank-K update)
};

template <typename TIn, typename TCin, typename TCout, typename TC2>
struct GemmParams {
  const TIn* A; int64_t lda; int64_t sa_o, sa_i;
  const TIn* B; int64_t ldb; int64_t sb_o, sb_i;
  const TCin* Cin; int64_t ldci; int64_t sci_o, sci_i;
  TCout* Cout; int64_t ldco; int64_t sco_o, sco_i;
  TC2* C2; int64_t ldc2;
  const float* rscale; int64_t ld_rs;
  const float* ascale;        // if set, alpha is multiplied by *ascale (device value)
  void* part;                 // split-K scratch (element type Mfma<TIn>::Acc), or null
  int64_t part_bytes;         // its size; the launcher picks ksplit to fit
  int ksplit;                 // set by the launcher: K slices (<= 1: no split)
  int M, N, K;
  int zdiv;
  double alpha, beta;
  float c2scale;
  uint32_t flags;
};

template <typename T> struct VecOf;
template <> struct VecOf<double> { typedef double T2 __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float> { typedef float T2 __attribute__((ext_vector_type(4))); };
template <> struct VecOf<bf16_t> { typedef __bf16 T2 __attribute__((ext_vector_type(8))); };
template <> struct VecOf<f16_t> { typedef _Float16 T2 __attribute__((ext_vector_type(8))); };
template <> struct VecOf<fp8_t> { typedef uint8_t T2 __attribute__((ext_vector_type(16))); };

// Buffer descriptor word 3 for the gfx9 family (raw, untyped loads).
constexpr int kBufWord3 = 0x00020000;
// Offsets at or above this value read as zero (outside the descriptor).
constexpr int kBufOOB = 0x7FFFFFF0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, kBufOOB, kBufWord3);
}

template <typename V>
__device__ __forceinline__ V buf_load16(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}


// A square lower-triangular A (M == K) makes the tile cost grow with the
// row index.  Such products are "folded": one workgroup computes row tile t
// and row tile ntm-1-t of the same column, so every workgroup gets the same
// amount of work (and half as many workgroups are launched).
__host__ __device__ inline bool tri_fold(int M, int K, uint32_t flags, int BM) {
  return (flags & (G_A_LOWER | G_A_UPPER)) && M == K && (M + BM - 1) / BM >= 2;
}

// Workgroups one product needs.
__host__ __device__ inline int gemm_wgs(int M, int N, int K, uint32_t flags, int BM, int BN) {
  const int ntm = (M + BM - 1) / BM, ntn = (N + BN - 1) / BN;
  if (flags & G_C_LOWER) return ntm * (ntm + 1) / 2;
  return (tri_fold(M, K, flags, BM) ? (ntm + 1) / 2 : ntm) * ntn;
}

// Tile (tm, tn), tn <= tm, of workgroup `bid` among the t (t + 1) / 2 that
// cover the lower triangle of a t x t tile grid.  Row tiles are paired, a
// with t - 1 - a, so that a run of t + 1 consecutive ids covers one pair
// (a + 1 tiles of row a, then t - a of row t - 1 - a); with a multiple of 8
// workgroups the ids are regrouped so that each XCD takes a contiguous range
// of pairs (they share their rows of A in its L2).
__device__ __forceinline__ void lower_tile(int t, int bid, int nwg, int& tm, int& tn) {
  if ((nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
  const int pr = bid / (t + 1), q = bid - pr * (t + 1);
  if (q <= pr) {
    tm = pr;
    tn = q;
  } else {
    tm = t - 1 - pr;
    tn = q - pr - 1;
  }
}

// Row slot and column of workgroup `bid` among the nwg workgroups of one
// product: groups of GROUP_M row slots, column-major inside a group.  The
// hardware deals consecutive workgroup ids to the eight XCDs in turn;
// products with uniform tile cost (dense, folded, or a single group of row
// slots) regroup the ids so that each XCD works on a contiguous range of
// tiles and its concurrent workgroups share panels in its own L2 (2.3x less
// L2-miss traffic).  Other triangular products keep the round-robin order,
// which spreads their uneven tile costs over the XCDs (a contiguous range of
// row groups per XCD made an unfolded lower-triangular product twice as slow).
template <int GROUP_M, bool XCD_REMAP>
__device__ __forceinline__ void tile_slot(int rows, int ntn, bool uniform, int bid, int nwg,
                                          int& slot, int& tn) {
  const bool remap = XCD_REMAP || uniform || rows <= GROUP_M;
  if (remap && (nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
  const int per_group = GROUP_M * ntn;
  const int grp = bid / per_group;
  const int first_m = grp * GROUP_M;
  const int gsize = min(rows - first_m, GROUP_M);
  const int in_grp = bid % per_group;
  slot = first_m + in_grp % gsize;
  tn = in_grp / gsize;
}

// Reduction range of a tile: whole chunks of BK from kbeg, skipping the zero
// part of a triangular operand.  Returns the number of chunks.
template <int BM, int BK>
__device__ __forceinline__ int chunk_range(int K, uint32_t flags, int r0, int c0, int& kbeg) {
  int kend = K;
  kbeg = 0;
  if (flags & G_A_LOWER) kend = min(K, r0 + BM);
  if (flags & G_A_UPPER) kbeg = (min(r0, K) / BK) * BK;
  if (flags & G_B_LOWER) kbeg = (min(c0, K) / BK) * BK;
  return kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
}

// Split-K: slice s of S covers the global chunks [s*cps, (s+1)*cps) of K,
// intersected with the tile's own range.
template <int BK>
__device__ __forceinline__ int split_range(int K, int s, int S, int nchunks, int& kbeg) {
  if (S <= 1) return nchunks;
  const int nck = (K + BK - 1) / BK, cps = (nck + S - 1) / S;
  const int lo = max(s * cps, kbeg / BK), hi = min((s + 1) * cps, kbeg / BK + nchunks);
  kbeg = lo * BK;
  return hi > lo ? hi - lo : 0;
}

template <typename TIn, typename TCin, typename TCout>
using EpiType = typename std::conditional<std::is_same<TCout, double>::value ||
                                              std::is_same<TCin, double>::value,
                                          double, typename Mfma<TIn>::Acc>::type;

// One output element: Cout = beta*Cin + alpha*rs*v (+ second output).
template <typename TIn, typename TCin, typename TCout, typename TC2, typename Epi>
__device__ __forceinline__ void epi_store(const GemmParams<TIn, TCin, TCout, TC2>& p,
                                          TCout* __restrict__ Co, const TCin* __restrict__ Ci,
                                          int row, int col, Epi v, Epi alpha, Epi beta,
                                          bool use_beta, Epi rs) {
  v = alpha * (v * rs);
  if (use_beta) v += beta * static_cast<Epi>(Ci[(int64_t)row * p.ldci + col]);
  Co[(int64_t)row * p.ldco + col] = static_cast<TCout>(v);
  if (p.C2) {
    const TC2 w = cvt<TC2>(v * static_cast<Epi>(p.c2scale));
    if (p.flags & G_C2_T) p.C2[(int64_t)col * p.ldc2 + row] = w;
    else p.C2[(int64_t)row * p.ldc2 + col] = w;
  }
}

// Epilogue: Cout = beta*Cin + alpha*rowscale*acc (+ optional second output).
// Lane (gi, g) holds column gi and rows out_row(g, r) of every 16x16 tile.
template <typename TIn, typename TCin, typename TCout, typename TC2, int TM, int TN, int WTM,
          int WTN>
__device__ __forceinline__ void gemm_epilogue(const GemmParams<TIn, TCin, TCout, TC2>& p,
                                              const typename Mfma<TIn>::Out (&acc)[TM][TN],
                                              int zo, int zi, int z, int s, int r0, int c0,
                                              int wm, int wn, int g, int gi) {
  using MF = Mfma<TIn>;
  using Acc = typename MF::Acc;
  const int M = p.M, N = p.N;
  if (p.ksplit > 1) {
    // split-K: raw partial sums, summed and finished by gemm_splitk_finish
    Acc* __restrict__ P = static_cast<Acc*>(p.part) + ((int64_t)z * p.ksplit + s) * M * N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wm * WTM + i * 16 + MF::out_row(g, r);
        if (row >= M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int col = c0 + wn * WTN + j * 16 + gi;
          if (col < N) P[(int64_t)row * N + col] = acc[i][j][r];
        }
      }
    return;
  }
  TCout* __restrict__ Co = p.Cout + zo * p.sco_o + zi * p.sco_i;
  const TCin* __restrict__ Ci = p.Cin ? p.Cin + zo * p.sci_o + zi * p.sci_i : nullptr;
  const bool use_beta = (p.flags & G_BETA) && Ci;
  const bool use_rs = (p.flags & G_ROWSCALE) && p.rscale;
  // the epilogue runs in binary64 whenever C is binary64 on either side
  using Epi = EpiType<TIn, TCin, TCout>;
  Epi alpha = static_cast<Epi>(p.alpha);
  if (p.ascale) alpha *= static_cast<Epi>(*p.ascale);
  const Epi beta = static_cast<Epi>(p.beta);
  const bool c_lower = p.flags & G_C_LOWER;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + wm * WTM + i * 16 + MF::out_row(g, r);
      if (row >= M) continue;
      Epi rs = Epi(1);
      if (use_rs) rs = static_cast<Epi>(p.rscale[(int64_t)row * p.ld_rs]);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = c0 + wn * WTN + j * 16 + gi;
        if (col >= N || (c_lower && col > row)) continue;
        epi_store(p, Co, Ci, row, col, static_cast<Epi>(acc[i][j][r]), alpha, beta, use_beta, rs);
      }
    }
  }
}

// Epilogue for products computed with the MFMA operands swapped (the tile of
// C^T is accumulated): lane (gi, g) then holds row gi and the four adjacent
// columns 4g..4g+3 of every 16x16 tile, so binary32 C moves in 16-byte
// vectors.
template <typename TIn, typename TCin, typename TCout, typename TC2, int TM, int TN, int WTM,
          int WTN>
__device__ __forceinline__ void gemm_epilogue_t(const GemmParams<TIn, TCin, TCout, TC2>& p,
                                                const typename Mfma<TIn>::Out (&acc)[TM][TN],
                                                int zo, int zi, int z, int s, int r0, int c0,
                                                int wm, int wn, int g, int gi) {
  using MF = Mfma<TIn>;
  using Acc = typename MF::Acc;
  const int M = p.M, N = p.N;
  if (p.ksplit > 1) {
    Acc* __restrict__ P = static_cast<Acc*>(p.part) + ((int64_t)z * p.ksplit + s) * M * N;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int row = r0 + wm * WTM + i * 16 + gi;
      if (row >= M) continue;
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = c0 + wn * WTN + j * 16 + 4 * g + r;
          if (col < N) P[(int64_t)row * N + col] = acc[i][j][r];
        }
    }
    return;
  }
  TCout* __restrict__ Co = p.Cout + zo * p.sco_o + zi * p.sco_i;
  const TCin* __restrict__ Ci = p.Cin ? p.Cin + zo * p.sci_o + zi * p.sci_i : nullptr;
  const bool use_beta = (p.flags & G_BETA) && Ci;
  const bool use_rs = (p.flags & G_ROWSCALE) && p.rscale;
  using Epi = EpiType<TIn, TCin, TCout>;
  Epi alpha = static_cast<Epi>(p.alpha);
  if (p.ascale) alpha *= static_cast<Epi>(*p.ascale);
  const Epi beta = static_cast<Epi>(p.beta);
  constexpr bool F32C = std::is_same<TCout, float>::value && std::is_same<TCin, float>::value;
  const bool c_lower = p.flags & G_C_LOWER;
  const bool vec = F32C && !p.C2 && !c_lower &&
                   (((uintptr_t)Co | (uintptr_t)(Ci ? Ci : Co) | (uintptr_t)(p.ldco * 4) |
                     (uintptr_t)(p.ldci * 4)) & 15) == 0;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int row = r0 + wm * WTM + i * 16 + gi;
    if (row >= M) continue;
    const Epi rs = use_rs ? static_cast<Epi>(p.rscale[(int64_t)row * p.ld_rs]) : Epi(1);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col0 = c0 + wn * WTN + j * 16 + 4 * g;
      if constexpr (F32C) {
        if (vec && col0 + 3 < N) {
          typedef float F4 __attribute__((ext_vector_type(4)));
          F4 cin = {0.f, 0.f, 0.f, 0.f};
          if (use_beta) cin = *reinterpret_cast<const F4*>(Ci + (int64_t)row * p.ldci + col0);
          F4 o;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            Epi v = alpha * (static_cast<Epi>(acc[i][j][r]) * rs);
            if (use_beta) v += beta * static_cast<Epi>(cin[r]);
            o[r] = static_cast<float>(v);
          }
          *reinterpret_cast<F4*>(Co + (int64_t)row * p.ldco + col0) = o;
          continue;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = col0 + r;
        if (col < N && !(c_lower && col > row))
          epi_store(p, Co, Ci, row, col, static_cast<Epi>(acc[i][j][r]), alpha, beta, use_beta, rs);
      }
    }
  }
}

// s_waitcnt immediate that waits for at most n outstanding vector-memory
// operations and nothing else (gfx9 encoding).
constexpr int vmcnt_imm(int n) {
  return (n & 0xF) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8);
}

// Matrix-core tile with operands copied from HBM straight into LDS by
// buffer loads (no register staging), two LDS stages, one barrier per chunk.
// For one-k-per-lane instructions (binary64, binary32) and 16-byte aligned
// operands.  LDS layout per stage:
//  * A: BM rows of 128 bytes (BK elements), the eight 16-byte pieces of row r
//    stored XOR-swizzled (piece d at position d ^ (r & 7)), so that the 16
//    rows a fragment read touches fall in different banks;
//  * B, row-major (BKMAJOR false): BK rows of BN elements; each wave load
//    instruction writes 1 KB (one or more whole rows) and is followed by 16
//    bytes of padding;
//  * B given as B^T (BKMAJOR true: N rows of K, k contiguous): BN rows of
//    128 bytes swizzled like A, and read like A.
// All fragments of a half-chunk are read before its MFMAs are issued.
// Triangular masks are applied to the fragments, only in chunks that cross
// the diagonal.
template <typename TIn, typename TCin, typename TCout, typename TC2, int BM, int BN, int WGM,
          int WGN, bool BKMAJOR = false>
__device__ __forceinline__ void gemm_tile_dma(const GemmParams<TIn, TCin, TCout, TC2>& p, int z,
                                              int s, const int r0, const int c0) {
  using MF = Mfma<TIn>;
  using Acc = typename MF::Acc;
  using Out = typename MF::Out;
  using V16 = typename VecOf<TIn>::T2;
  constexpr int NW = WGM * WGN;
  constexpr int ES = sizeof(TIn);
  constexpr int VEC = 16 / ES;
  constexpr int BK = 128 / ES;
  constexpr int KL = BK / 4;                     // k per lane group per chunk (32 bytes)
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int A_BYTES = BM * 128;
  constexpr int ROW_B = BN * ES;                 // bytes of one B row
  constexpr int RPI = 1024 / ROW_B;              // B rows per wave instruction
  constexpr int B_INST_TOTAL = BK / RPI;
  constexpr int B_BYTES = BKMAJOR ? BN * 128 : B_INST_TOTAL * (1024 + 16);
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int A_INST = BM / 8 / NW;
  constexpr int B_INST = B_INST_TOTAL / NW;
  constexpr int BT_INST = BN / 8 / NW;
  static_assert(MF::kPerLane == 1, "one k per lane");
  static_assert(RPI * ROW_B == 1024, "a wave instruction must cover whole B rows");
  static_assert(A_INST * NW * 8 == BM && B_INST * NW == B_INST_TOTAL, "even split of loads");
  static_assert(!BKMAJOR || BT_INST * NW * 8 == BN, "even split of B^T loads");
  __shared__ __attribute__((aligned(1024))) char smem[2 * STAGE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN, gi = lane & 15, g = lane >> 4;
  const int zo = z / p.zdiv, zi = z % p.zdiv;
  const TIn* __restrict__ A = p.A + zo * p.sa_o + zi * p.sa_i;
  const TIn* __restrict__ B = p.B + zo * p.sb_o + zi * p.sb_i;
  const int M = p.M, N = p.N, K = p.K;
  const int lda = (int)p.lda, ldb = (int)p.ldb;
  int kbeg;
  int nchunks = chunk_range<BM, BK>(K, p.flags, r0, c0, kbeg);
  nchunks = split_range<BK>(K, s, p.ksplit, nchunks, kbeg);
  const bool a_lower = p.flags & G_A_LOWER;
  const bool b_lower = p.flags & G_B_LOWER;

  Out acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = Acc(0);

  auto issue = [&](int c, int st) {
    const int k0 = kbeg + c * BK;
    char* base = smem + st * STAGE;
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + (int64_t)r0 * lda + k0);
#pragma unroll
    for (int q = 0; q < A_INST; ++q) {
      const int rb = 8 * (wave * A_INST + q);
      const int r = rb + (lane >> 3);
      const int d = (lane & 7) ^ (r & 7);
      const bool ok = (r0 + r < M) && (k0 + d * VEC < K);
      const int off = ok ? (r * lda + d * VEC) * ES : kBufOOB;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ra, (__attribute__((address_space(3))) void*)(base + rb * 128), 16, off, 0, 0, 0);
    }
    if constexpr (BKMAJOR) {
      const __amdgpu_buffer_rsrc_t rbt = make_rsrc(B + (int64_t)c0 * ldb + k0);
#pragma unroll
      for (int q = 0; q < BT_INST; ++q) {
        const int rb = 8 * (wave * BT_INST + q);
        const int r = rb + (lane >> 3);
        const int d = (lane & 7) ^ (r & 7);
        const bool ok = (c0 + r < N) && (k0 + d * VEC < K);
        const int off = ok ? (r * ldb + d * VEC) * ES : kBufOOB;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rbt, (__attribute__((address_space(3))) void*)(base + A_BYTES + rb * 128), 16, off, 0,
            0, 0);
      }
      return;
    }
    const __amdgpu_buffer_rsrc_t rbs = make_rsrc(B + (int64_t)k0 * ldb + c0);
#pragma unroll
    for (int q = 0; q < B_INST; ++q) {
      const int qi = wave * B_INST + q;
      const int kr = qi * RPI + lane / (64 / RPI);
      const int cv = (lane % (64 / RPI)) * VEC;
      const bool ok = (k0 + kr < K) && (c0 + cv < N);
      const int off = ok ? (kr * ldb + cv) * ES : kBufOOB;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rbs, (__attribute__((address_space(3))) void*)(base + A_BYTES + qi * (1024 + 16)), 16,
          off, 0, 0, 0);
    }
  };

  if (nchunks > 0) issue(0, 0);
  for (int c = 0; c < nchunks; ++c) {
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));   // this wave's part of chunk c has landed
    __syncthreads();                            // ... everyone's; and chunk c-1 is consumed
    if (c + 1 < nchunks) issue(c + 1, (c + 1) & 1);
    const char* as = smem + (c & 1) * STAGE;
    const char* bs = as + A_BYTES;
    const int k0 = kbeg + c * BK;
    const bool mask_a = a_lower && !(p.flags & G_A_ZERO_UPPER) && (k0 + BK - 1 > r0 + wm * WTM);
    const bool mask_b = b_lower && (k0 < c0 + wn * WTN + WTN - 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {               // the lane group's two 16-byte pieces of k
      V16 fa[TM];
      TIn fb[VEC][TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm * WTM + i * 16 + gi;
        const int slot = (2 * g + h) ^ (r & 7);
        fa[i] = *reinterpret_cast<const V16*>(as + r * 128 + slot * 16);
      }
      if constexpr (BKMAJOR) {
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int r = wn * WTN + j * 16 + gi;
          const int slot = (2 * g + h) ^ (r & 7);
          const V16 v = *reinterpret_cast<const V16*>(bs + r * 128 + slot * 16);
#pragma unroll
          for (int e = 0; e < VEC; ++e) fb[e][j] = v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int kr = g * KL + h * VEC + e;
#pragma unroll
          for (int j = 0; j < TN; ++j)
            fb[e][j] = *reinterpret_cast<const TIn*>(bs + (kr / RPI) * (1024 + 16) +
                                                     (kr % RPI) * ROW_B +
                                                     (wn * WTN + j * 16 + gi) * ES);
        }
      }
      if (mask_a) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (k0 + g * KL + h * VEC + e > r0 + wm * WTM + i * 16 + gi) fa[i][e] = TIn(0);
      }
      if (mask_b) {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (k0 + g * KL + h * VEC + e < c0 + wn * WTN + j * 16 + gi) fb[e][j] = TIn(0);
      }
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(fa[i][e], fb[e][j], acc[i][j]);
    }
  }
  gemm_epilogue<TIn, TCin, TCout, TC2, TM, TN, WTM, WTN>(p, acc, zo, zi, z, s, r0, c0, wm, wn, g,
                                                        gi);
}

// Register-staged tile: every operand layout and alignment (the general
// path; bfloat16/half products with k-contiguous B, and unaligned operands).
template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR, bool ALIGNED>
__device__ __forceinline__ void gemm_tile_staged(const GemmParams<TIn, TCin, TCout, TC2>& p,
                                                 int z, int s, const int r0, const int c0) {
  using MF = Mfma<TIn>;
  using Acc = typename MF::Acc;
  using Out = typename MF::Out;
  using V16 = typename VecOf<TIn>::T2;          // 16-byte vector of TIn
  constexpr int NT = WGM * WGN * 64;
  constexpr int VEC = 16 / sizeof(TIn);         // elements per 16-byte vector
  constexpr int BK = 128 / sizeof(TIn);         // one 128-byte row segment per chunk
  constexpr int KL = BK / 4;                    // contiguous k per lane group per chunk
  constexpr int STEPS = KL / MF::kPerLane;      // MFMAs per 16x16 tile per chunk
  constexpr int WTM = BM / WGM, WTN = BN / WGN; // wave tile
  constexpr int TM = WTM / 16, TN = WTN / 16;   // MFMA tiles per wave
  // LDS: A as [row][k]; B as [k][n] (row-major B) or [n][k] (BKMAJOR).
  constexpr int LDA_S = BK + VEC;
  constexpr int LDB_S = BKMAJOR ? (BK + VEC) : (BN + VEC);
  constexpr int B_ELEMS = BKMAJOR ? BN * LDB_S : BK * LDB_S;
  constexpr int VPR = BK / VEC;                 // vectors per k segment of one A row
  constexpr int A_ITERS = BM * VPR / NT;
  constexpr int B_VPL = BKMAJOR ? VPR : BN / VEC;   // vectors per stored B line
  constexpr int B_ITERS = (BKMAJOR ? BN * VPR : BK * (BN / VEC)) / NT;
  static_assert(A_ITERS * NT == BM * VPR, "A tile load must divide evenly");
  static_assert(B_ITERS * NT == (BKMAJOR ? BN * VPR : BK * (BN / VEC)), "B tile load must divide evenly");
  static_assert(BKMAJOR || MF::kPerLane == 1, "row-major B needs a one-k-per-lane instruction");
  // With both operands k-contiguous the MFMA can take them in either order;
  // taking B first accumulates the tile of C^T, whose lane layout lets the
  // epilogue move binary32 C in 16-byte vectors.
  constexpr bool SWAP = BKMAJOR && (MF::kPerLane > 1) && std::is_same<Acc, float>::value;

  __shared__ __attribute__((aligned(16))) TIn As[2][BM * LDA_S];
  __shared__ __attribute__((aligned(16))) TIn Bs[2][B_ELEMS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int gi = lane & 15, g = lane >> 4;

  // ---- batch offsets --------------------------------------------------
  const int zo = z / p.zdiv, zi = z % p.zdiv;
  const TIn* __restrict__ A = p.A + zo * p.sa_o + zi * p.sa_i;
  const TIn* __restrict__ B = p.B + zo * p.sb_o + zi * p.sb_i;
  const int M = p.M, N = p.N, K = p.K;
  const int64_t lda = p.lda, ldb = p.ldb;

  const bool a_lower = p.flags & G_A_LOWER;
  const bool b_lower = p.flags & G_B_LOWER;
  int kbeg;
  int nchunks = chunk_range<BM, BK>(K, p.flags, r0, c0, kbeg);
  nchunks = split_range<BK>(K, s, p.ksplit, nchunks, kbeg);

  Out acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = Acc(0);

  // ---- global -> register staging (no per-lane branches) -------------------
  V16 ra[A_ITERS], rb[B_ITERS];

  auto load_a = [&](int k0) {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(A + (int64_t)r0 * lda + k0);
#pragma unroll
    for (int it = 0; it < A_ITERS; ++it) {
      const int idx = tid + it * NT;
      const int row = idx / VPR, kv = (idx % VPR) * VEC;
      const int gr = r0 + row, gk = k0 + kv;
      V16 v;
      if constexpr (ALIGNED) {
        const bool ok = gr < M && gk < K;
        v = buf_load16<V16>(rs, ok ? (int)((row * lda + kv) * (int64_t)sizeof(TIn)) : kBufOOB);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const bool ok = gr < M && gk + e < K;
          const TIn x = A[ok ? (int64_t)gr * lda + gk + e : 0];
          v[e] = ok ? x : TIn(0);
        }
      }
      ra[it] = v;
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int it = 0; it < B_ITERS; ++it) {
      const int idx = tid + it * NT;
      V16 v;
      if constexpr (BKMAJOR) {
        // B stored N x K: a stored row is a column of B.
        const int col = idx / VPR, kv = (idx % VPR) * VEC;
        const int gc = c0 + col, gk = k0 + kv;
        if constexpr (ALIGNED) {
          const __amdgpu_buffer_rsrc_t rs = make_rsrc(B + (int64_t)c0 * ldb + k0);
          const bool ok = gc < N && gk < K;
          v = buf_load16<V16>(rs, ok ? (int)((col * ldb + kv) * (int64_t)sizeof(TIn)) : kBufOOB);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const bool ok = gc < N && gk + e < K;
            const TIn x = B[ok ? (int64_t)gc * ldb + gk + e : 0];
            v[e] = ok ? x : TIn(0);
          }
        }
      } else {
        // B stored K x N: BK rows of BN/VEC vectors.
        const int krow = idx / B_VPL, cv = (idx % B_VPL) * VEC;
        const int gk = k0 + krow, gc = c0 + cv;
        if constexpr (ALIGNED) {
          const __amdgpu_buffer_rsrc_t rs = make_rsrc(B + (int64_t)k0 * ldb + c0);
          const bool ok = gk < K && gc < N;
          v = buf_load16<V16>(rs, ok ? (int)((krow * ldb + cv) * (int64_t)sizeof(TIn)) : kBufOOB);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const bool ok = gk < K && gc + e < N;
            const TIn x = B[ok ? (int64_t)gk * ldb + gc + e : 0];
            v[e] = ok ? x : TIn(0);
          }
        }
      }
      rb[it] = v;
    }
  };
  // Triangular masks are applied when the staged data is written to LDS, so
  // that the global loads of the next chunk stay in flight during the MFMAs.
  auto store_ab = [&](int buf, int k0) {
#pragma unroll
    for (int it = 0; it < A_ITERS; ++it) {
      const int idx = tid + it * NT;
      const int row = idx / VPR, kv = (idx % VPR) * VEC;
      V16 v = ra[it];
      if (a_lower) {
        const int gr = r0 + row, gk = k0 + kv;
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = (gk + e > gr) ? TIn(0) : v[e];
      }
      *reinterpret_cast<V16*>(&As[buf][row * LDA_S + kv]) = v;
    }
#pragma unroll
    for (int it = 0; it < B_ITERS; ++it) {
      const int idx = tid + it * NT;
      const int line = idx / B_VPL, vo = (idx % B_VPL) * VEC;
      V16 v = rb[it];
      if (b_lower) {
        // BKMAJOR: line = column, vo = k offset; else line = k row, vo = column offset
        const int gc = c0 + (BKMAJOR ? line : vo), gk = k0 + (BKMAJOR ? vo : line);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const bool zero = BKMAJOR ? (gk + e < gc) : (gk < gc + e);
          v[e] = zero ? TIn(0) : v[e];
        }
      }
      *reinterpret_cast<V16*>(&Bs[buf][line * LDB_S + vo]) = v;
    }
  };

  // ---- main loop --------------------------------------------------------
  if (nchunks > 0) {
    load_a(kbeg);
    load_b(kbeg);
    store_ab(0, kbeg);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = c + 1 < nchunks;
      if (more) {
        load_a(kbeg + (c + 1) * BK);
        load_b(kbeg + (c + 1) * BK);
      }
      const TIn* as = As[buf];
      const TIn* bs = Bs[buf];
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        // lane group g feeds k = g*KL + s*kPerLane ... + kPerLane - 1
        const int kk = g * KL + s * MF::kPerLane;
        typename MF::Frag fa[TM], fb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          fa[i] = *reinterpret_cast<const typename MF::Frag*>(&as[(wm * WTM + i * 16 + gi) * LDA_S + kk]);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (BKMAJOR)
            fb[j] = *reinterpret_cast<const typename MF::Frag*>(&bs[(wn * WTN + j * 16 + gi) * LDB_S + kk]);
          else
            fb[j] = bs[kk * LDB_S + wn * WTN + j * 16 + gi];
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = SWAP ? MF::mma(fb[j], fa[i], acc[i][j]) : MF::mma(fa[i], fb[j], acc[i][j]);
      }
      if (more) store_ab(buf ^ 1, kbeg + (c + 1) * BK);
      __syncthreads();
    }
  }

  if constexpr (SWAP)
    gemm_epilogue_t<TIn, TCin, TCout, TC2, TM, TN, WTM, WTN>(p, acc, zo, zi, z, s, r0, c0, wm, wn,
                                                            g, gi);
  else
    gemm_epilogue<TIn, TCin, TCout, TC2, TM, TN, WTM, WTN>(p, acc, zo, zi, z, s, r0, c0, wm, wn, g,
                                                          gi);
}


// The output tiles of workgroup `bid` (of nwg) of one batch entry z: one
// tile, or two for a folded triangular product.
template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR, bool ALIGNED, bool CLOWER = false,
          int GROUP_M = 8, bool XCD_REMAP = false>
__device__ __forceinline__ void gemm_tile(const GemmParams<TIn, TCin, TCout, TC2>& p, int z,
                                          int s, int bid, int nwg) {
  const int ntm = (p.M + BM - 1) / BM, ntn = (p.N + BN - 1) / BN;
  if constexpr (CLOWER) {
    int tm, tn;
    lower_tile(ntm, bid, nwg, tm, tn);
    if constexpr (ALIGNED && Mfma<TIn>::kPerLane == 1)
      gemm_tile_dma<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR>(p, z, s, tm * BM, tn * BN);
    else
      gemm_tile_staged<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, ALIGNED>(p, z, s, tm * BM,
                                                                               tn * BN);
    return;
  }
  const bool fold = tri_fold(p.M, p.K, p.flags, BM);
  const bool uniform = fold || !(p.flags & (G_A_LOWER | G_B_LOWER | G_A_UPPER));
  const int rows = fold ? (ntm + 1) / 2 : ntm;
  int slot, tn;
  tile_slot<GROUP_M, XCD_REMAP>(rows, ntn, uniform, bid, nwg, slot, tn);
  auto one = [&](int tm) {
    if constexpr (ALIGNED && Mfma<TIn>::kPerLane == 1)
      gemm_tile_dma<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR>(p, z, s, tm * BM, tn * BN);
    else
      gemm_tile_staged<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, ALIGNED>(p, z, s, tm * BM,
                                                                               tn * BN);
  };
  one(slot);
  if (fold && ntm - 1 - slot != slot) {
    __syncthreads();   // the second tile reuses the LDS stages
    one(ntm - 1 - slot);
  }
}

template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR, bool ALIGNED, bool CLOWER = false>
__global__ __launch_bounds__(WGM * WGN * 64, 2)
void gemm_kernel(GemmParams<TIn, TCin, TCout, TC2> p) {
  gemm_tile<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, ALIGNED, CLOWER>(
      p, blockIdx.z, blockIdx.y, blockIdx.x, gridDim.x);
}

// Split-K finish: the fixed-order sum of the ksplit partial products of
// every element, then the usual epilogue (deterministic: the order of the
// sum never depends on scheduling).
template <typename TIn, typename TCin, typename TCout, typename TC2>
__global__ __launch_bounds__(256) void gemm_splitk_finish(GemmParams<TIn, TCin, TCout, TC2> p,
                                                          int batch) {
  using Acc = typename Mfma<TIn>::Acc;
  using Epi = EpiType<TIn, TCin, TCout>;
  const int64_t MN = (int64_t)p.M * p.N, total = MN * batch;
  const bool use_rs = (p.flags & G_ROWSCALE) && p.rscale;
  Epi alpha = static_cast<Epi>(p.alpha);
  if (p.ascale) alpha *= static_cast<Epi>(*p.ascale);
  const Epi beta = static_cast<Epi>(p.beta);
  const Acc* __restrict__ P = static_cast<const Acc*>(p.part);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(e / MN);
    const int64_t rc = e - z * MN;
    const int row = (int)(rc / p.N), col = (int)(rc - (int64_t)row * p.N);
    if ((p.flags & G_C_LOWER) && col > row) continue;
    const Acc* q = P + (int64_t)z * p.ksplit * MN + rc;
    Acc v = q[0];
    for (int t = 1; t < p.ksplit; ++t) v += q[t * MN];
    const int zo = z / p.zdiv, zi = z % p.zdiv;
    TCout* Co = p.Cout + zo * p.sco_o + zi * p.sco_i;
    const TCin* Ci = p.Cin ? p.Cin + zo * p.sci_o + zi * p.sci_i : nullptr;
    const Epi rs = use_rs ? static_cast<Epi>(p.rscale[(int64_t)row * p.ld_rs]) : Epi(1);
    epi_store(p, Co, Ci, row, col, static_cast<Epi>(v), alpha, beta, (p.flags & G_BETA) && Ci, rs);
  }
}

// Grouped launch: many independent products of one element type in one
// grid.  Entry e owns workgroups [tile_start[e], tile_start[e+1]); within an
// entry the workgroups cover ksplit x tiles (K slice, then tile).
template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR, bool ALIGNED>
__global__ __launch_bounds__(WGM * WGN * 64, 2)
void gemm_grouped_kernel(const GemmParams<TIn, TCin, TCout, TC2>* __restrict__ entries,
                         const int* __restrict__ tile_start, int nentries) {
  const int b = blockIdx.x;
  int lo = 0, hi = nentries - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const GemmParams<TIn, TCin, TCout, TC2>& p = entries[lo];
  const int tiles = gemm_wgs(p.M, p.N, p.K, p.flags, BM, BN);
  const int local = b - tile_start[lo];
  gemm_tile<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, ALIGNED>(p, 0, local / tiles,
                                                                      local % tiles, tiles);
}

// Whether the 16-byte vector path may be used for a product.
template <typename TIn, int BM, int BN, bool BKMAJOR, typename P>
inline bool gemm_aligned(const P& p) {
  constexpr int VEC = 16 / sizeof(TIn);
  constexpr int BK = 128 / sizeof(TIn);
  auto al = [](const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; };
  const int64_t span_a = (int64_t)BM * p.lda * (int64_t)sizeof(TIn);
  const int64_t span_b = (int64_t)(BKMAJOR ? BN : BK) * p.ldb * (int64_t)sizeof(TIn);
  return al(p.A) && al(p.B) && p.lda % VEC == 0 && p.ldb % VEC == 0 && p.sa_o % VEC == 0 &&
         p.sa_i % VEC == 0 && p.sb_o % VEC == 0 && p.sb_i % VEC == 0 && p.K % VEC == 0 &&
         (BKMAJOR || p.N % VEC == 0) && span_a < kBufOOB && span_b < kBufOOB;
}

// Split-K policy: products with at most half a round of workgroups split K
// into S slices (each at least kSplitMinChunks chunks) so that at most one
// round runs (kSplitTarget = two 128 x 128 workgroups per compute unit), as
// far as the scratch in p.part holds the partial products.  Without scratch
// (p.part null) nothing is split.
constexpr int kSplitTarget = 512;
constexpr int kSplitMinChunks = 4;
constexpr int kSplitMax = 16;
template <typename TIn, typename P>
inline int gemm_ksplit(const P& p, int64_t wgs, int batch, int target) {
  if (!p.part || 2 * wgs > target) return 1;
  constexpr int BK = 128 / sizeof(TIn);
  const int64_t nck = (p.K + BK - 1) / BK;
  int64_t S = std::min<int64_t>(target / wgs, nck / kSplitMinChunks);
  S = std::min<int64_t>(S, kSplitMax);
  const int64_t per = (int64_t)p.M * p.N * batch * (int64_t)sizeof(typename Mfma<TIn>::Acc);
  if (per > 0) S = std::min<int64_t>(S, p.part_bytes / per);
  return S > 1 ? (int)S : 1;
}

// Host-side launch helper.  Picks the aligned (16-byte vector) path when every
// operand start, leading dimension and batch stride allows it.
template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR>
inline hipError_t launch_gemm(const GemmParams<TIn, TCin, TCout, TC2>& p, int batch,
                              hipStream_t stream) {
  if (p.M <= 0 || p.N <= 0 || batch <= 0) return hipSuccess;
  if ((p.flags & G_C_LOWER) && (p.M != p.N || BM != BN)) return hipErrorInvalidValue;
  const bool aligned = gemm_aligned<TIn, BM, BN, BKMAJOR>(p);
  const int64_t tiles = gemm_wgs(p.M, p.N, p.K, p.flags, BM, BN);
  GemmParams<TIn, TCin, TCout, TC2> q = p;
  // one round of workgroups: two per compute unit for the 128 x 128 tiles,
  // four for the smaller ones (their registers and LDS allow it)
  const int target = (BM * BN >= 128 * 128) ? kSplitTarget : 2 * kSplitTarget;
  q.ksplit = gemm_ksplit<TIn>(p, tiles * batch, batch, target);
  // lower-triangle products take their own instantiation (tile enumeration)
  const bool clower = p.flags & G_C_LOWER;
  dim3 grid((unsigned)tiles, (unsigned)q.ksplit, (unsigned)batch);
  dim3 block(WGM * WGN * 64);
  if (clower) {
    if (aligned)
      gemm_kernel<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, true, true>
          <<<grid, block, 0, stream>>>(q);
    else
      gemm_kernel<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, false, true>
          <<<grid, block, 0, stream>>>(q);
  } else if (aligned) {
    gemm_kernel<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, true><<<grid, block, 0, stream>>>(q);
  } else {
    gemm_kernel<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, false><<<grid, block, 0, stream>>>(q);
  }
  if (q.ksplit > 1) {
    const int64_t total = (int64_t)p.M * p.N * batch;
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    gemm_splitk_finish<TIn, TCin, TCout, TC2><<<g, 256, 0, stream>>>(q, batch);
  }
  return hipGetLastError();
}

template <typename TIn, typename TCin, typename TCout, typename TC2>
inline GemmParams<TIn, TCin, TCout, TC2> gemm_params() {
  GemmParams<TIn, TCin, TCout, TC2> p{};
  p.zdiv = 1;
  p.alpha = 1.0;
  p.beta = 0.0;
  p.c2scale = 1.0f;
  return p;
}

}  // namespace trsm
