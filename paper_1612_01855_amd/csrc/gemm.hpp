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
// * Optional second output C2 (another precision, optionally transposed,
//   optionally scaled) feeds a following low-precision product.
// * Batches: z -> offset (z / zdiv) * outer + (z % zdiv) * inner.
//
// Work decomposition: a workgroup of WGM x WGN waves owns a BM x BN tile;
// each wave owns (BM/WGM) x (BN/WGN) made of 16x16 MFMA tiles.  K advances in
// chunks of BK with two LDS buffers and a register prefetch of the next
// chunk, one barrier per chunk.  Tiles are visited in groups of GROUP_M row
// tiles (column-major inside a group) so that concurrently running
// workgroups share A and B panels in L2.  The hardware deals consecutive
// workgroup ids to the eight XCDs in turn; dense products regroup the ids so
// that each XCD works on a contiguous range of tiles (2.3x less L2-miss
// traffic), triangular products keep the round-robin order because a
// contiguous range per XCD unbalanced their uneven tile costs (the
// lower-triangular residual ran twice as slow).
#pragma once

#include "common.hpp"

#include <type_traits>

namespace trsm {

enum GemmFlags : uint32_t {
  G_A_LOWER = 1u,
  G_B_LOWER = 2u,
  G_C2_T = 4u,       // C2 stored transposed: C2[col * ldc2 + row]
  G_BETA = 8u,       // read Cin
  G_ROWSCALE = 16u,  // multiply the product by rscale[row * ld_rs]
};

template <typename TIn, typename TCin, typename TCout, typename TC2>
struct GemmParams {
  const TIn* A; int64_t lda; int64_t sa_o, sa_i;
  const TIn* B; int64_t ldb; int64_t sb_o, sb_i;
  const TCin* Cin; int64_t ldci; int64_t sci_o, sci_i;
  TCout* Cout; int64_t ldco; int64_t sco_o, sco_i;
  TC2* C2; int64_t ldc2;
  const float* rscale; int64_t ld_rs;
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

// One BM x BN output tile of one batch entry.  `bid` is the tile's index
// among the nwg tiles of the entry; `z` the batch index.
template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR, bool ALIGNED,
          int GROUP_M = 8, bool XCD_REMAP = false>
__device__ __forceinline__ void gemm_tile(const GemmParams<TIn, TCin, TCout, TC2>& p, int z,
                                          int bid, int nwg) {
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

  // ---- tile coordinates (XCD-aware, grouped) -----------------------------
  const int ntm = (M + BM - 1) / BM, ntn = (N + BN - 1) / BN;
  // Dense products (uniform tile cost): give each XCD a contiguous range of
  // tiles so that its concurrent workgroups share panels in its own L2.
  // Triangular products keep the hardware's round-robin order, which
  // balances their uneven tile costs over the XCDs.
  const bool remap = XCD_REMAP || !(p.flags & (G_A_LOWER | G_B_LOWER));
  if (remap && (nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
  const int per_group = GROUP_M * ntn;
  const int grp = bid / per_group;
  const int first_m = grp * GROUP_M;
  const int gsize = min(ntm - first_m, GROUP_M);
  const int in_grp = bid % per_group;
  const int tm = first_m + in_grp % gsize;
  const int tn = in_grp / gsize;
  const int r0 = tm * BM, c0 = tn * BN;

  const bool a_lower = p.flags & G_A_LOWER;
  const bool b_lower = p.flags & G_B_LOWER;
  int kbeg = 0, kend = K;
  if (a_lower) kend = min(K, r0 + BM);
  if (b_lower) kbeg = (min(c0, K) / BK) * BK;
  const int nchunks = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

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
          for (int j = 0; j < TN; ++j) acc[i][j] = MF::mma(fa[i], fb[j], acc[i][j]);
      }
      if (more) store_ab(buf ^ 1, kbeg + (c + 1) * BK);
      __syncthreads();
    }
  }

  // ---- epilogue ---------------------------------------------------------
  TCout* __restrict__ Co = p.Cout + zo * p.sco_o + zi * p.sco_i;
  const TCin* __restrict__ Ci = p.Cin ? p.Cin + zo * p.sci_o + zi * p.sci_i : nullptr;
  const bool use_beta = (p.flags & G_BETA) && Ci;
  const bool use_rs = (p.flags & G_ROWSCALE) && p.rscale;
  const bool c2t = p.flags & G_C2_T;
  // the epilogue runs in binary64 whenever C is binary64 on either side
  using Epi = typename std::conditional<std::is_same<TCout, double>::value ||
                                            std::is_same<TCin, double>::value,
                                        double, Acc>::type;
  const Epi alpha = static_cast<Epi>(p.alpha);
  const Epi beta = static_cast<Epi>(p.beta);
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
        if (col >= N) continue;
        Epi v = alpha * (static_cast<Epi>(acc[i][j][r]) * rs);
        if (use_beta) v += beta * static_cast<Epi>(Ci[(int64_t)row * p.ldci + col]);
        Co[(int64_t)row * p.ldco + col] = static_cast<TCout>(v);
        if (p.C2) {
          const TC2 w = cvt<TC2>(v * static_cast<Epi>(p.c2scale));
          if (c2t) p.C2[(int64_t)col * p.ldc2 + row] = w;
          else p.C2[(int64_t)row * p.ldc2 + col] = w;
        }
      }
    }
  }
}

template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR, bool ALIGNED>
__global__ __launch_bounds__(WGM * WGN * 64, 2)
void gemm_kernel(GemmParams<TIn, TCin, TCout, TC2> p) {
  gemm_tile<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, ALIGNED>(p, blockIdx.z, blockIdx.x,
                                                                      gridDim.x);
}

// Grouped launch: many independent products of one element type in one
// grid.  Entry e owns workgroups [tile_start[e], tile_start[e+1]); within an
// entry the workgroups cover batch x tiles as in gemm_kernel.
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
  const int tiles = ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN);
  const int local = b - tile_start[lo];
  gemm_tile<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, ALIGNED>(p, local / tiles,
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

// Host-side launch helper.  Picks the aligned (16-byte vector) path when every
// operand start, leading dimension and batch stride allows it.
template <typename TIn, typename TCin, typename TCout, typename TC2,
          int BM, int BN, int WGM, int WGN, bool BKMAJOR>
inline hipError_t launch_gemm(const GemmParams<TIn, TCin, TCout, TC2>& p, int batch,
                              hipStream_t stream) {
  if (p.M <= 0 || p.N <= 0 || batch <= 0) return hipSuccess;
  const bool aligned = gemm_aligned<TIn, BM, BN, BKMAJOR>(p);
  const int64_t tiles = ceil_div(p.M, BM) * ceil_div(p.N, BN);
  dim3 grid((unsigned)tiles, 1, (unsigned)batch);
  dim3 block(WGM * WGN * 64);
  if (aligned)
    gemm_kernel<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, true><<<grid, block, 0, stream>>>(p);
  else
    gemm_kernel<TIn, TCin, TCout, TC2, BM, BN, WGM, WGN, BKMAJOR, false><<<grid, block, 0, stream>>>(p);
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
