// Matrix-core GEMM for 8- and 16-bit operands on gfx950 (bfloat16, half,
// fp8 e4m3, int8), used where the solve runs in low precision: the trailing
// updates of the bfloat16/half/fp8 sweep (the update steps of Alg.
// It-Inv-TRSM on a low-precision copy of L) and the exact integer products of the residual
// B - L X in the refinement (one product per modulus of a residue number
// system; int8 operands, int32 accumulation, no rounding anywhere).
//
//   C = op(A) * op(B)^T,   A: M x K, B: N x K, both k-contiguous row-major.
//
// Work decomposition.  A workgroup of 8 waves (2 x 4) owns a 256 x 256 tile
// of C; each wave owns 128 x 64, i.e. 4 x 2 tiles of the 32 x 32 matrix-core
// instruction (v_mfma_f32_32x32x16_{f16,bf16}, v_mfma_i32_32x32x32_i8: 16
// bytes of k per lane, the two 32-lane halves taking two different 16-byte
// pieces; v_mfma_scale_f32_32x32x64_f8f6f4 for fp8: 32 bytes per lane, two
// pieces each).  K advances in chunks of 128 bytes; both operands of a chunk go
// from HBM straight into LDS (buffer loads with the LDS modifier, no register
// staging), two LDS stages of 64 KB, one barrier per chunk.  Every row of a
// stage holds eight 16-byte pieces; piece d of row r sits at position
// d ^ f(r) with f(r) = ((r >> 1) ^ (r << 2)) & 7, so that the 16 rows a
// fragment read touches fall in distinct banks for both the 128- and the
// 256-byte-per-clock LDS read widths.  Fragments of the next k step are read
// while the matrix instructions of the current one issue.  The matrix
// instruction takes the B fragment as its first operand, so it accumulates
// the tile of C^T: lane l then holds row l % 32 and four consecutive
// columns, which the epilogues move as one vector.
//
// Lower-triangular A (LP_A_LOWER): chunks past a row tile's last row are
// skipped (A must store zeros above its diagonal inside the chunk that
// crosses it); a square lower-triangular product pairs row tile t with row
// tile ntm - 1 - t in one workgroup so that every workgroup gets equal work.
// Batches (grid z) step A, B and the integer output by fixed strides and take
// their own modulus.
#pragma once

#include "common.hpp"

namespace trsm {
namespace lp {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef int i16v __attribute__((ext_vector_type(16)));

template <typename T> struct Mma;
template <> struct Mma<f16_t> {
  typedef h8v Frag;
  typedef f16v Acc;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<bf16_t> {
  typedef b8v Frag;
  typedef f16v Acc;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<int8_t> {
  typedef i4v Frag;
  typedef i16v Acc;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
  }
};
// fp8 (OCP e4m3) on gfx950's f8f6f4 matrix instruction: 64 bytes of k per
// instruction, 32 per lane (two 16-byte pieces), operand formats 0 (e4m3)
// and unit block scales (E8M0 127 = 2^0: the operands carry their own
// power-of-two row and block scales, applied in the epilogue).
template <> struct Mma<fp8_t> {
  typedef i8v Frag;
  typedef f16v Acc;
  static constexpr int kBytes = 64;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
};
// bytes of k one matrix instruction consumes (16 per lane for the 16-bit
// and int8 instructions)
template <typename T> struct KBytes { static constexpr int v = 32; };
template <> struct KBytes<fp8_t> { static constexpr int v = Mma<fp8_t>::kBytes; };

enum LpFlags : uint32_t {
  LP_A_LOWER = 1u,    // A lower triangular (zeros stored above the diagonal)
  LP_BETA = 2u,       // read Cin
  LP_ROWSCALE = 4u,   // multiply by rscale[row * ld_rs]
  LP_SEGMENTS = 8u,   // K is a run of segments with their own scales (below)
};

enum LpEpi { EPI_F32 = 0, EPI_MOD = 1, EPI_RAW = 2 };

constexpr int kMaxBatch = 16;

struct LpParams {
  const void* A; int64_t lda;       // elements
  const void* B; int64_t ldb;
  int M, N, K;
  uint32_t flags;
  // EPI_F32: Cout = beta * Cin + alpha * (*ascale) * rscale[row * ld_rs] * acc
  // With LP_SEGMENTS, K is split into segments of seg_chunks chunks; the
  // products of segment j carry the scale 1 / f(row, j) with
  // f(row, j) = rscale[row * ld_rs + j] * sscale[j] (exact powers of two), and
  // the result is sum_j f(row, j) * (segment j's product): the accumulator is
  // rescaled at every segment boundary and the epilogue applies the last f.
  const float* sscale;
  int seg_chunks;
  float* Cout; int64_t ldco;
  const float* Cin; int64_t ldci;
  const float* rscale; int64_t ld_rs;
  const float* ascale;
  float alpha, beta;
  // EPI_MOD: Z[row * ldz + col] = acc mod modulus[z], in [-(m-1)/2, (m-1)/2]
  // (m odd) or [-128, 127] (m = 256).  EPI_RAW: int32/binary32 acc to Zraw.
  int8_t* Z; int64_t ldz;
  void* Zraw;
  int64_t sa, sb, sz;               // batch strides (elements) of A, B, Z
  int modulus[kMaxBatch];
};

constexpr int kBM = 256, kBN = 256, kWGM = 2, kWGN = 4;
constexpr int kThreads = kWGM * kWGN * 64;
constexpr int kChunk = 128;                        // bytes of k per LDS stage row
constexpr int kStageBytes = (kBM + kBN) * kChunk;  // 64 KB
constexpr int kStages = 2;

__device__ __forceinline__ int piece_pos(int r) { return ((r >> 1) ^ (r << 2)) & 7; }

constexpr int kBufWord3 = 0x00020000;
constexpr int kBufOOB = 0x7FFFFFF0;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, kBufOOB, kBufWord3);
}
constexpr int vmcnt(int n) { return (n & 0xF) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8); }

// Interleaving hints for one chunk: the matrix instructions of k step s
// alternate with the fragment reads of step s + 1.
template <int NM, int NR>
__device__ __forceinline__ void sched_interleave() {
  if constexpr (NM > 0 || NR > 0) {
    if constexpr (NM > 0) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    if constexpr (NR > 0) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    sched_interleave<(NM > 0 ? NM - 1 : 0), (NR > 0 ? NR - 1 : 0)>();
  }
}
template <int S, int KSTEPS, int NM, int NR>
__device__ __forceinline__ void sched_chunk() {
  if constexpr (S < KSTEPS) {
    sched_interleave<NM, (S + 1 < KSTEPS) ? NR : 0>();
    sched_chunk<S + 1, KSTEPS, NM, NR>();
  }
}

__host__ __device__ inline bool lp_fold(const LpParams& p) {
  return (p.flags & LP_A_LOWER) && p.M == p.K && (p.M + kBM - 1) / kBM >= 2;
}
__host__ __device__ inline int lp_tiles(const LpParams& p) {
  const int ntm = (p.M + kBM - 1) / kBM, ntn = (p.N + kBN - 1) / kBN;
  return (lp_fold(p) ? (ntm + 1) / 2 : ntm) * ntn;
}

template <typename T, int EPI>
__device__ __forceinline__ void lp_tile(const LpParams& p, int z, int r0, int c0, char* smem) {
  using MM = Mma<T>;
  using Frag = typename MM::Frag;
  using Acc = typename MM::Acc;
  constexpr int ES = sizeof(T);
  constexpr int WTM = kBM / kWGM, WTN = kBN / kWGN;
  constexpr int TM = WTM / 32, TN = WTN / 32;
  constexpr int A_BYTES = kBM * kChunk;
  constexpr int A_INST = kBM / 8 / (kWGM * kWGN), B_INST = kBN / 8 / (kWGM * kWGN);
  constexpr int LOADS = A_INST + B_INST;
  constexpr int KB = KBytes<T>::v;                 // k bytes per instruction
  constexpr int KSTEPS = kChunk / KB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / kWGN, wn = wave % kWGN;
  const int li = lane & 31, hh = lane >> 5;

  const char* A = static_cast<const char*>(p.A) + (int64_t)z * p.sa * ES;
  const char* B = static_cast<const char*>(p.B) + (int64_t)z * p.sb * ES;
  const int lda = (int)(p.lda * ES), ldb = (int)(p.ldb * ES);
  const int Kb = p.K * ES;
  int kend = Kb;
  if (p.flags & LP_A_LOWER) kend = min(Kb, (r0 + kBM) * ES);
  const int nchunks = (kend + kChunk - 1) / kChunk;
  const __amdgpu_buffer_rsrc_t ra = rsrc(A + (int64_t)r0 * lda);
  const __amdgpu_buffer_rsrc_t rb = rsrc(B + (int64_t)c0 * ldb);
  const int arows = p.M - r0, brows = p.N - c0;

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0;

  // one chunk of both operands into LDS stage st (out of range -> zeros)
  auto issue = [&](int c, int st) {
    const bool live = c < nchunks;
    const int k0 = c * kChunk;
    char* base = smem + st * kStageBytes;
#pragma unroll
    for (int q = 0; q < A_INST; ++q) {
      const int rr = 8 * (wave * A_INST + q);
      const int r = rr + (lane >> 3);
      const int d = (lane & 7) ^ piece_pos(r);
      const int kb = k0 + d * 16;
      const bool ok = live && r < arows && kb < Kb;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ra, (__attribute__((address_space(3))) void*)(base + rr * kChunk), 16,
          ok ? r * lda + kb : kBufOOB, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < B_INST; ++q) {
      const int rr = 8 * (wave * B_INST + q);
      const int r = rr + (lane >> 3);
      const int d = (lane & 7) ^ piece_pos(r);
      const int kb = k0 + d * 16;
      const bool ok = live && r < brows && kb < Kb;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rb, (__attribute__((address_space(3))) void*)(base + A_BYTES + rr * kChunk), 16,
          ok ? r * ldb + kb : kBufOOB, 0, 0, 0);
    }
  };

  if (nchunks > 0) issue(0, 0);
  for (int c = 0; c < nchunks; ++c) {
    __builtin_amdgcn_s_waitcnt(vmcnt(0));   // this wave's part of chunk c has landed
    __syncthreads();                        // ... everyone's; chunk c - 1 is consumed
    const char* as = smem + (c & 1) * kStageBytes;
    const char* bs = as + A_BYTES;
    Frag fa[2][TM], fb[2][TN];
    // lane group hh takes the pieces (KB / 32) (2 s + hh) .. + KB / 32 - 1 of
    // k step s, for A and B alike (so every instruction pairs the same k)
    auto frag = [&](const char* base, int r, int s) {
      if constexpr (KB == 32) {
        return *reinterpret_cast<const Frag*>(base + r * kChunk + (((2 * s + hh) ^ piece_pos(r)) * 16));
      } else {
        const int d = 4 * s + 2 * hh;
        const i4v lo = *reinterpret_cast<const i4v*>(base + r * kChunk + ((d ^ piece_pos(r)) * 16));
        const i4v hi =
            *reinterpret_cast<const i4v*>(base + r * kChunk + (((d + 1) ^ piece_pos(r)) * 16));
        return Frag{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
    };
    auto rd = [&](int s, int set) {
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[set][i] = frag(as, wm * WTM + i * 32 + li, s);
#pragma unroll
      for (int j = 0; j < TN; ++j) fb[set][j] = frag(bs, wn * WTN + j * 32 + li, s);
    };
    rd(0, 0);
    issue(c + 1, (c + 1) & 1);   // past the last chunk: zero-filled, never read
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
      if (s + 1 < KSTEPS) rd(s + 1, (s + 1) & 1);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = MM::mma(fb[s & 1][j], fa[s & 1][i], acc[i][j]);
    }
    sched_chunk<0, KSTEPS, TM * TN, (TM + TN) * (KB / 32)>();
    if ((p.flags & LP_SEGMENTS) && (c + 1) % p.seg_chunks == 0 && c + 1 < nchunks) {
      // leaving segment j for j + 1: acc <- acc * f(row, j) / f(row, j + 1)
      const int j = (c + 1) / p.seg_chunks - 1;
      const float sr = p.sscale[j] / p.sscale[j + 1];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = r0 + wm * WTM + i * 32 + li;
        float f = 1.0f;
        if (row < p.M) {
          const float* rr = p.rscale + (int64_t)row * p.ld_rs;
          f = sr * (rr[j] / rr[j + 1]);
        }
#pragma unroll
        for (int jj = 0; jj < TN; ++jj)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[i][jj][v] *= f;
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(vmcnt(0));    // the zero-filled prefetch past the end

  // ---- epilogues: lane holds row li and columns 8 g + 4 hh + e of each tile ----
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int row = r0 + wm * WTM + i * 32 + li;
    if (row >= p.M) continue;
    if constexpr (EPI == EPI_F32) {
      float sc = p.alpha;
      if (p.ascale) sc *= *p.ascale;
      if (p.flags & LP_SEGMENTS) {
        const int jl = nchunks > 0 ? (nchunks - 1) / p.seg_chunks : 0;
        sc *= p.rscale[(int64_t)row * p.ld_rs + jl] * p.sscale[jl];
      } else if (p.flags & LP_ROWSCALE) {
        sc *= p.rscale[(int64_t)row * p.ld_rs];
      }
      const bool beta = p.flags & LP_BETA;
      float* co = p.Cout + (int64_t)row * p.ldco;
      const float* ci = beta ? p.Cin + (int64_t)row * p.ldci : nullptr;
      const bool vec = ((((uintptr_t)co) | (uintptr_t)(ci ? ci : co)) & 15) == 0;
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int col = c0 + wn * WTN + j * 32 + 8 * g + 4 * hh;
          if (vec && col + 3 < p.N) {
            f4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = sc * acc[i][j][4 * g + e];
            if (beta) {
              const f4 cv = *reinterpret_cast<const f4*>(ci + col);
#pragma unroll
              for (int e = 0; e < 4; ++e) o[e] += p.beta * cv[e];
            }
            *reinterpret_cast<f4*>(co + col) = o;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (col + e < p.N) {
                float o = sc * acc[i][j][4 * g + e];
                if (beta) o += p.beta * ci[col + e];
                co[col + e] = o;
              }
          }
        }
    } else if constexpr (EPI == EPI_MOD) {
      const int m = p.modulus[z];
      const float inv = 1.0f / (float)m;
      const int half = (m - 1) / 2;
      int8_t* zr = p.Z + (int64_t)z * p.sz + (int64_t)row * p.ldz;
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int col = c0 + wn * WTN + j * 32 + 8 * g + 4 * hh;
          uint32_t packed = 0;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int a = acc[i][j][4 * g + e];
            int r;
            if (m == 256) {
              r = (int)(int8_t)(a & 0xFF);
            } else {
              // |a| < 2^30: the binary32 quotient is off by at most one
              const int q = (int)rintf((float)a * inv);
              r = a - q * m;
              r = r > half ? r - m : r;
              r = r < -half ? r + m : r;
            }
            packed |= ((uint32_t)(uint8_t)(int8_t)r) << (8 * e);
          }
          if (col + 3 < p.N) {
            *reinterpret_cast<uint32_t*>(zr + col) = packed;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (col + e < p.N) zr[col + e] = (int8_t)((packed >> (8 * e)) & 0xFF);
          }
        }
    } else {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int col = c0 + wn * WTN + j * 32 + 8 * g + 4 * hh;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e < p.N) {
              if constexpr (std::is_same<T, int8_t>::value)
                static_cast<int*>(p.Zraw)[(int64_t)z * p.sz + (int64_t)row * p.ldz + col + e] =
                    acc[i][j][4 * g + e];
              else
                static_cast<float*>(p.Zraw)[(int64_t)z * p.sz + (int64_t)row * p.ldz + col + e] =
                    acc[i][j][4 * g + e];
            }
        }
    }
  }
}

// Tile (row slot, column tile) of workgroup `bid`: groups of 8 row slots,
// column-major inside a group; the ids are first regrouped so that each of
// the eight XCDs (which the hardware deals consecutive ids to in turn) works
// on a contiguous range of tiles and shares their panels in its own L2.
__device__ __forceinline__ void lp_slot(int rows, int ntn, int bid, int nwg, int& slot, int& tn) {
  if ((nwg & 7) == 0) bid = (bid & 7) * (nwg >> 3) + (bid >> 3);
  constexpr int G = 8;
  const int per_group = G * ntn;
  const int grp = bid / per_group;
  const int first = grp * G;
  const int gsize = min(rows - first, G);
  const int in_grp = bid - grp * per_group;
  slot = first + in_grp % gsize;
  tn = in_grp / gsize;
}

template <typename T, int EPI>
__global__ __launch_bounds__(kThreads, 1) void lp_gemm_kernel(LpParams p) {
  __shared__ __attribute__((aligned(1024))) char smem[kStages * kStageBytes];
  const int ntm = (p.M + kBM - 1) / kBM, ntn = (p.N + kBN - 1) / kBN;
  const bool fold = lp_fold(p);
  const int rows = fold ? (ntm + 1) / 2 : ntm;
  int slot, tn;
  lp_slot(rows, ntn, blockIdx.x, gridDim.x, slot, tn);
  lp_tile<T, EPI>(p, blockIdx.z, slot * kBM, tn * kBN, smem);
  if (fold && ntm - 1 - slot != slot) {
    __syncthreads();   // the second tile reuses the LDS stages
    lp_tile<T, EPI>(p, blockIdx.z, (ntm - 1 - slot) * kBM, tn * kBN, smem);
  }
}

// Whether the operands suit the 16-byte loads (k extent a whole number of
// 16-byte pieces, 16-byte aligned rows, offsets inside the 2 GiB window).
template <typename T>
inline bool lp_ok(const LpParams& p) {
  constexpr int ES = sizeof(T);
  auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  return al(p.A) && al(p.B) && (p.lda * ES) % 16 == 0 && (p.ldb * ES) % 16 == 0 &&
         (p.K * ES) % 16 == 0 && (p.sa * ES) % 16 == 0 && (p.sb * ES) % 16 == 0 &&
         (int64_t)kBM * p.lda * ES < kBufOOB && (int64_t)kBN * p.ldb * ES < kBufOOB;
}

template <typename T, int EPI>
inline hipError_t launch_lp_gemm(const LpParams& p, int batch, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0 || batch <= 0) return hipSuccess;
  if (!lp_ok<T>(p) || batch > kMaxBatch || (p.flags & LP_A_LOWER && p.K > p.M + kBM))
    return hipErrorInvalidValue;
  dim3 grid((unsigned)lp_tiles(p), 1, (unsigned)batch);
  lp_gemm_kernel<T, EPI><<<grid, kThreads, 0, s>>>(p);
  return hipGetLastError();
}

inline LpParams lp_params() {
  LpParams p{};
  p.alpha = 1.0f;
  p.beta = 0.0f;
  return p;
}

}  // namespace lp
}  // namespace trsm
