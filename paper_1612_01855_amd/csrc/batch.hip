// Grouped launches for batches of triangular solves, and the C ABI
// trsm_batch_* (see include/trsm.h).
#include "batch.hpp"

#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/trsm.h"
#include "kernels.hpp"

namespace trsm {

namespace {

// Index of the entry that owns workgroup b (start[] is the prefix array).
__device__ __forceinline__ int owner_of(const int* __restrict__ start, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A sum of squares kept as s * 4^e with s in a safe range, so that it does
// not overflow or underflow whatever the magnitudes summed (the exponent is
// raised to the largest exponent seen and smaller terms are scaled by exact
// powers of two).  Not-finite terms make s not finite.
struct Sq {
  double s;
  int e;
};
constexpr int kSqEmpty = -4000;

__device__ __forceinline__ void sq_add(Sq& a, double x) {
  const double ax = fabs(x);
  if (ax == 0.0) return;
  if (!(ax <= 1.7976931348623157e308)) {
    a.s += ax;   // infinity or NaN
    return;
  }
  const int e = ilogb(ax);
  if (e > a.e) {
    a.s = ldexp(a.s, 2 * (a.e - e));
    a.e = e;
  }
  const double y = ldexp(ax, -a.e);
  a.s += y * y;
}

__device__ __forceinline__ Sq sq_merge(Sq a, Sq b) {
  const int e = max(a.e, b.e);
  return Sq{ldexp(a.s, 2 * (a.e - e)) + ldexp(b.s, 2 * (b.e - e)), e};
}

// Merge over the 64 lanes of a wavefront (butterfly: a fixed order).
__device__ __forceinline__ Sq wave_sq(Sq v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Sq w{__shfl_xor(v.s, o, 64), __shfl_xor(v.e, o, 64)};
    v = sq_merge(v, w);
  }
  return v;
}

// The sum of quantity q over an entry's parts (partial layout of RedEntry),
// by one wavefront in a fixed order.
__device__ __forceinline__ Sq parts_sq(const double* part, int nparts, int q, int lane) {
  Sq v{0.0, kSqEmpty};
  for (int p = lane; p < nparts; p += 64)
    v = sq_merge(v, Sq{part[kPartStride * p + q], (int)part[kPartStride * p + 3 + q]});
  return wave_sq(v);
}

// 2^-e for a sum of squares whose square root lies below 2^e (e clamped to
// +-1000); 1 when the sum is zero or not finite.
__device__ __forceinline__ double pow2_inv_scale(Sq v) {
  if (!(v.s > 0.0) || !(v.s <= 1.7976931348623157e308)) return 1.0;
  int e1;
  (void)frexp(sqrt(v.s), &e1);
  const int e = max(-1000, min(1000, v.e + e1));
  return ldexp(1.0, -e);
}

// Row and column of a thread's elements: those at flat (row-major) index i0,
// i0 + 256, i0 + 512, ... of a rows x cols matrix, stepped without a division
// per element (one 64-bit division for the first).
struct RowCol {
  int64_t r;
  int c, dr, dc, cols;
  __device__ __forceinline__ RowCol(int64_t i0, int ncols) : cols(ncols) {
    r = i0 / ncols;
    c = (int)(i0 - r * ncols);
    dr = 256 / ncols;
    dc = 256 - dr * ncols;
  }
  __device__ __forceinline__ void next() {
    r += dr;
    c += dc;
    if (c >= cols) {
      c -= cols;
      ++r;
    }
  }
};

// One element of each elementwise op: the source type S, the destination
// type D, whether the destination is read (a running sum) and the value
// stored (`old` is the destination's value for the running sums).
template <int OP> struct EwElem;
template <> struct EwElem<EW_F64_TO_F32> {
  typedef double S; typedef float D; static constexpr bool kAdd = false;
  static __device__ __forceinline__ D f(S x, D, double scale, double) {
    return static_cast<float>(scale * x);
  }
};
template <> struct EwElem<EW_F32_TO_F64_SET> {
  typedef float S; typedef double D; static constexpr bool kAdd = false;
  static __device__ __forceinline__ D f(S x, D, double scale, double) {
    return scale * static_cast<double>(x);
  }
};
template <> struct EwElem<EW_F32_TO_F64_ADD> {
  typedef float S; typedef double D; static constexpr bool kAdd = true;
  static __device__ __forceinline__ D f(S x, D old, double scale, double) {
    return old + scale * static_cast<double>(x);
  }
};
template <> struct EwElem<EW_F64_COPY> {
  typedef double S; typedef double D; static constexpr bool kAdd = false;
  static __device__ __forceinline__ D f(S x, D, double scale, double) { return scale * x; }
};
template <> struct EwElem<EW_F32_COPY> {
  typedef float S; typedef float D; static constexpr bool kAdd = false;
  static __device__ __forceinline__ D f(S x, D, double scale, double) {
    return static_cast<float>(scale) * x;
  }
};
template <> struct EwElem<EW_F64_TO_F32_PS> {
  typedef double S; typedef float D; static constexpr bool kAdd = false;
  static __device__ __forceinline__ D f(S x, D, double, double sc) {
    return static_cast<float>(sc * x);
  }
};
template <> struct EwElem<EW_F32_TO_F64_SET_SC> {
  typedef float S; typedef double D; static constexpr bool kAdd = false;
  static __device__ __forceinline__ D f(S x, D, double, double sc) {
    return sc * static_cast<double>(x);
  }
};
template <> struct EwElem<EW_F32_TO_F64_ADD_SC> {
  typedef float S; typedef double D; static constexpr bool kAdd = true;
  static __device__ __forceinline__ D f(S x, D old, double, double sc) {
    return old + sc * static_cast<double>(x);
  }
};
template <> struct EwElem<EW_F64_ADD> {
  typedef double S; typedef double D; static constexpr bool kAdd = true;
  static __device__ __forceinline__ D f(S x, D old, double, double) { return old + x; }
};

// Elements a thread keeps in flight: every load of a group is issued before
// the group's first store, so a workgroup waits for memory once per group
// rather than once per element.
constexpr int kEwGroup = 8;

// The thread's elements i0, i0 + 256, ... below lim of one entry.  Padding
// columns (>= valid_cols) are not read: plain ops store zero there, running
// sums leave them alone.  Loads are not predicated: an element that is not
// read loads element (0, 0) instead (every entry has one valid column) and
// discards it, so the group's loads form one straight run.
template <int OP>
__device__ __forceinline__ void ew_elems(const EwEntry& e, int64_t i0, int64_t lim, double sc) {
  using EL = EwElem<OP>;
  using S = typename EL::S;
  using D = typename EL::D;
  const S* __restrict__ src = static_cast<const S*>(e.src);
  D* __restrict__ dst = static_cast<D*>(e.dst);
  if (i0 >= lim || e.valid_cols <= 0) {
    // nothing to read: plain ops store zeros, running sums are unchanged
    if (!EL::kAdd)
      for (; i0 < lim; i0 += 256) {
        const int64_t r = i0 / e.cols, c = i0 - r * e.cols;
        dst[r * e.ldd + c] = D(0);
      }
    return;
  }
  RowCol rc(i0, e.cols);
  for (; i0 < lim; i0 += 256 * kEwGroup) {
    int64_t so[kEwGroup], dof[kEwGroup];
    bool in[kEwGroup], rd[kEwGroup];
#pragma unroll
    for (int j = 0; j < kEwGroup; ++j) {
      in[j] = i0 + 256 * j < lim;
      rd[j] = in[j] && rc.c < e.valid_cols;
      so[j] = rd[j] ? rc.r * e.lds + rc.c : 0;
      dof[j] = in[j] ? rc.r * e.ldd + rc.c : 0;
      rc.next();
    }
    S x[kEwGroup];
    D old[kEwGroup];
#pragma unroll
    for (int j = 0; j < kEwGroup; ++j) {
      x[j] = src[so[j]];
      old[j] = EL::kAdd ? dst[dof[j]] : D(0);
    }
#pragma unroll
    for (int j = 0; j < kEwGroup; ++j) {
      if (EL::kAdd) {
        if (rd[j]) dst[dof[j]] = EL::f(x[j], old[j], e.scale, sc);
      } else if (in[j]) {
        dst[dof[j]] = rd[j] ? EL::f(x[j], old[j], e.scale, sc) : D(0);
      }
    }
  }
}

// Grouped elementwise kernel: entry e owns workgroups [start[e], start[e+1]),
// each workgroup converts kEwChunk consecutive elements (row-major order) of
// its matrix.
__global__ __launch_bounds__(256) void grouped_ew_kernel(const EwEntry* __restrict__ entries,
                                                         const int* __restrict__ start, int n) {
  const int b = blockIdx.x;
  const int lo = owner_of(start, n, b);
  const EwEntry& e = entries[lo];
  const int64_t total = (int64_t)e.rows * e.cols;
  const int64_t base = (int64_t)(b - start[lo]) * kEwChunk;
  // scaled ops: the scale is uniform over the entry (every workgroup of it
  // derives the same value from the same partial sums, in the same order)
  double sc = 1.0;
  if (e.op == EW_F64_TO_F32_PS) {
    __shared__ double sh;
    if (threadIdx.x < 64) {
      const Sq v = parts_sq(e.part, e.nparts, 0, threadIdx.x);
      if (threadIdx.x == 0) sh = pow2_inv_scale(v);
    }
    __syncthreads();
    sc = sh;
    if (b == start[lo] && threadIdx.x == 0) *e.sc = sc;
  } else if (e.op == EW_F32_TO_F64_SET_SC || e.op == EW_F32_TO_F64_ADD_SC) {
    sc = 1.0 / *e.sc;   // exact: a power of two
  }
  const int64_t i0 = base + threadIdx.x;
  const int64_t lim = min(total, base + kEwChunk);
  switch (e.op) {
    case EW_F64_TO_F32: ew_elems<EW_F64_TO_F32>(e, i0, lim, sc); break;
    case EW_F32_TO_F64_SET: ew_elems<EW_F32_TO_F64_SET>(e, i0, lim, sc); break;
    case EW_F32_TO_F64_ADD: ew_elems<EW_F32_TO_F64_ADD>(e, i0, lim, sc); break;
    case EW_F64_COPY: ew_elems<EW_F64_COPY>(e, i0, lim, sc); break;
    case EW_F64_TO_F32_PS: ew_elems<EW_F64_TO_F32_PS>(e, i0, lim, sc); break;
    case EW_F32_TO_F64_SET_SC: ew_elems<EW_F32_TO_F64_SET_SC>(e, i0, lim, sc); break;
    case EW_F32_TO_F64_ADD_SC: ew_elems<EW_F32_TO_F64_ADD_SC>(e, i0, lim, sc); break;
    case EW_F64_ADD: ew_elems<EW_F64_ADD>(e, i0, lim, sc); break;
    default: ew_elems<EW_F32_COPY>(e, i0, lim, sc); break;
  }
}

// Grouped reductions (see RedOp): entry e owns workgroups [start[e],
// start[e+1]), one per chunk; the three partial sums of a chunk are merged
// per wavefront, then over the four wavefronts in order.  A thread adds its
// elements base + tid, base + tid + 256, ... in that order; it loads them
// kEwGroup at a time (elements past the chunk read as zero, which leaves a
// sum of squares unchanged).
__global__ __launch_bounds__(256) void grouped_red_kernel(const RedEntry* __restrict__ entries,
                                                          const int* __restrict__ start, int n) {
  const int b = blockIdx.x;
  const int lo = owner_of(start, n, b);
  const RedEntry& e = entries[lo];
  const int p = b - start[lo];
  const int64_t total = (int64_t)e.rows * e.cols;
  const int64_t base = (int64_t)p * e.chunk;
  const int64_t end = min(total, base + e.chunk);
  Sq s0{0.0, kSqEmpty}, s1{0.0, kSqEmpty}, s2{0.0, kSqEmpty};
  const double* __restrict__ A = e.a;
  int64_t i0 = base + threadIdx.x;
  // Loads are not predicated: an element that is not read loads element
  // (0, 0) of the same matrix instead and is replaced by zero (the caller's
  // B of RD_LOAD has that element whenever it has a valid row and column).
  const bool a_any = e.op != RD_LOAD || (e.valid_cols > 0 && e.valid_rows > 0);
  if (i0 < end) {
    RowCol rc(i0, e.cols);
    for (; i0 < end; i0 += 256 * kEwGroup) {
      int64_t ao[kEwGroup], bo[kEwGroup], dof[kEwGroup], xof[kEwGroup];
      bool in[kEwGroup], valid[kEwGroup];
#pragma unroll
      for (int j = 0; j < kEwGroup; ++j) {
        in[j] = i0 + 256 * j < end;
        valid[j] = in[j] && rc.c < e.valid_cols && rc.r < e.valid_rows;
        const bool rd = e.op == RD_LOAD ? valid[j] : in[j];
        ao[j] = rd ? rc.r * e.lda + rc.c : 0;
        bo[j] = in[j] ? rc.r * e.ldb + rc.c : 0;
        dof[j] = in[j] ? rc.r * e.ldd + rc.c : 0;
        xof[j] = rc.r * e.ldxo + rc.c;
        rc.next();
      }
      double a[kEwGroup];
      if (e.op == RD_LOAD) {
        if (a_any) {
#pragma unroll
          for (int j = 0; j < kEwGroup; ++j) a[j] = A[ao[j]];
        }
#pragma unroll
        for (int j = 0; j < kEwGroup; ++j) {
          a[j] = a_any && valid[j] ? a[j] : 0.0;
          if (in[j]) e.b[bo[j]] = a[j];
          sq_add(s0, a[j]);
        }
      } else if (e.op == RD_RES) {
#pragma unroll
        for (int j = 0; j < kEwGroup; ++j) a[j] = A[ao[j]];
#pragma unroll
        for (int j = 0; j < kEwGroup; ++j) sq_add(s0, in[j] ? a[j] : 0.0);
      } else {
        const double* __restrict__ X = e.b;
        double x[kEwGroup], d[kEwGroup];
#pragma unroll
        for (int j = 0; j < kEwGroup; ++j) {
          a[j] = A[ao[j]];
          x[j] = X[bo[j]];
          d[j] = 0.0;
        }
        if (e.d) {
          if (e.d_f64) {
#pragma unroll
            for (int j = 0; j < kEwGroup; ++j) d[j] = static_cast<const double*>(e.d)[dof[j]];
          } else {
#pragma unroll
            for (int j = 0; j < kEwGroup; ++j)
              d[j] = static_cast<double>(static_cast<const float*>(e.d)[dof[j]]);
          }
        }
#pragma unroll
        for (int j = 0; j < kEwGroup; ++j) {
          sq_add(s0, in[j] ? a[j] : 0.0);
          sq_add(s1, in[j] ? x[j] : 0.0);
          sq_add(s2, in[j] ? d[j] : 0.0);
          if (valid[j]) e.xo[xof[j]] = x[j];
        }
      }
    }
  }
  __shared__ double rs[4][3];
  __shared__ int re[4][3];
  s0 = wave_sq(s0);
  s1 = wave_sq(s1);
  s2 = wave_sq(s2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rs[w][0] = s0.s; re[w][0] = s0.e;
    rs[w][1] = s1.s; re[w][1] = s1.e;
    rs[w][2] = s2.s; re[w][2] = s2.e;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    Sq v{rs[0][q], re[0][q]};
    for (int j = 1; j < 4; ++j) v = sq_merge(v, Sq{rs[j][q], re[j][q]});
    e.part[kPartStride * p + q] = v.s;
    e.part[kPartStride * p + 3 + q] = (double)v.e;
  }
}

// Final sums: one wavefront per entry.
__global__ __launch_bounds__(64) void grouped_fin_kernel(const FinEntry* __restrict__ entries) {
  const FinEntry& e = entries[blockIdx.x];
  const Sq s0 = parts_sq(e.part, e.nparts, 0, threadIdx.x);
  const Sq s1 = parts_sq(e.part, e.nparts, 1, threadIdx.x);
  const Sq s2 = parts_sq(e.part, e.nparts, 2, threadIdx.x);
  if (threadIdx.x == 0) {
    // a correction computed in scaled units: divide its sum by sc^2
    const int es = e.sc ? ilogb(*e.sc) : 0;
    e.out[0] = s0.s; e.out[1] = (double)s0.e;
    e.out[2] = s1.s; e.out[3] = (double)s1.e;
    e.out[4] = s2.s; e.out[5] = (double)(s2.e - es);
  }
}

// Split-K finish of grouped products: the fixed-order sum of each element's
// ksplit partial sums, then the product's epilogue.  Entry e owns workgroups
// [start[e], start[e+1]), kFinChunk elements each; a thread holds its
// kFinChunk / 256 elements at once, so each slice's loads go out together.
constexpr int kFinChunk = 2048;
template <typename T>
__global__ __launch_bounds__(256) void grouped_split_finish(
    const GemmParams<T, T, T, float>* __restrict__ entries, const int* __restrict__ start,
    int n) {
  using Acc = typename Mfma<T>::Acc;
  using Epi = EpiType<T, T, T>;
  constexpr int U = kFinChunk / 256;
  const int b = blockIdx.x;
  const int lo = owner_of(start, n, b);
  const GemmParams<T, T, T, float>& p = entries[lo];
  const int64_t MN = (int64_t)p.M * p.N;
  const int64_t base = (int64_t)(b - start[lo]) * kFinChunk;
  Epi alpha = static_cast<Epi>(p.alpha);
  if (p.ascale) alpha *= static_cast<Epi>(*p.ascale);
  const Epi beta = static_cast<Epi>(p.beta);
  const bool use_beta = (p.flags & G_BETA) && p.Cin;
  const bool use_rs = (p.flags & G_ROWSCALE) && p.rscale;
  const Acc* __restrict__ P = static_cast<const Acc*>(p.part);
  const int64_t e0 = base + threadIdx.x;
  const int64_t lim = min(MN, base + kFinChunk);
  if (e0 >= lim) return;
  RowCol rc(e0, p.N);
  // Loads are not predicated: an element the finish skips (past the chunk,
  // or above the diagonal of a lower-triangular C) loads the thread's first
  // element instead, which lies inside every buffer read here, and drops it.
  int row[U], col[U];
  int64_t pe[U];
  bool ok[U];
  Acc v[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    row[j] = (int)rc.r;
    col[j] = rc.c;
    ok[j] = e0 + 256 * j < lim && !((p.flags & G_C_LOWER) && col[j] > row[j]);
    pe[j] = ok[j] ? e0 + 256 * j : e0;
    rc.next();
  }
#pragma unroll
  for (int j = 0; j < U; ++j) v[j] = P[pe[j]];
  for (int t = 1; t < p.ksplit; ++t) {
    const Acc* __restrict__ Pt = P + t * MN;
    Acc w[U];
#pragma unroll
    for (int j = 0; j < U; ++j) w[j] = Pt[pe[j]];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] += w[j];
  }
  // the epilogue of every element (the same arithmetic as the products'
  // unsplit epilogue), with its row scales and C inputs loaded up front
  Epi rs[U], ci[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const int rj = ok[j] ? row[j] : row[0];
    const int cj = ok[j] ? col[j] : col[0];
    rs[j] = use_rs ? static_cast<Epi>(p.rscale[(int64_t)rj * p.ld_rs]) : Epi(1);
    ci[j] = use_beta ? static_cast<Epi>(p.Cin[(int64_t)rj * p.ldci + cj]) : Epi(0);
  }
#pragma unroll
  for (int j = 0; j < U; ++j) {
    if (!ok[j]) continue;
    Epi y = alpha * (static_cast<Epi>(v[j]) * rs[j]);
    if (use_beta) y += beta * ci[j];
    p.Cout[(int64_t)row[j] * p.ldco + col[j]] = static_cast<T>(y);
    if (p.C2) {
      const float w = cvt<float>(y * static_cast<Epi>(p.c2scale));
      if (p.flags & G_C2_T) p.C2[(int64_t)col[j] * p.ldc2 + row[j]] = w;
      else p.C2[(int64_t)row[j] * p.ldc2 + col[j]] = w;
    }
  }
}

constexpr int kBM = 128, kBN = 128;
// Aligned products of at most kNarrowN columns (skinny right-hand sides) use
// 128 x 32 tiles of four waves stacked along M: a quarter of the matrix-core
// work of a 128 x 128 tile on padding.  The k order of every element is the
// same as with the wide tiles, so the bits are too.
constexpr int kNarrowN = 32;

// Waits of the persistent sweep give up (and set the error word) after this
// many polls of about a microsecond; by construction a wait always ends long
// before (the awaited task was taken from the queue earlier by a running
// workgroup).
constexpr unsigned kSpinLimit = 1u << 22;
// Blocks of X folded into a task's running right-hand side per pass.
constexpr int kPassBlocks = 4;

template <typename T, bool ALIGNED>
__device__ __forceinline__ void persist_tile(const GemmParams<T, T, T, float>& p) {
  if constexpr (ALIGNED)
    gemm_tile_dma<T, T, T, float, kPB, kPB, 2, 2>(p, 0, 0, 0, 0);
  else
    gemm_tile_staged<T, T, T, float, kPB, kPB, 2, 2, false, false>(p, 0, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ GemmParams<T, T, T, float> persist_params() {
  GemmParams<T, T, T, float> p{};
  p.zdiv = 1;
  p.alpha = 1.0;
  p.c2scale = 1.0f;
  return p;
}

// Persistent left-looking sweep over many systems.  Workgroups take tasks
// (system p, step i, column tile c) from a queue (an atomic head) in
// step-major order.  A task accumulates R(S_i, c) = B(S_i, c) - sum over the
// blocks j < i of L(S_i, S_j) X(S_j, c) in passes over fixed groups of
// kPassBlocks blocks: before a pass it waits until the tile's counter shows
// the group finished (acquire), and the pass reads and updates R through the
// epilogue; then X(S_i, c) = Linv_ii R(S_i, c) and the counter advances
// (release).  Tasks of later steps therefore work through the finished
// blocks while earlier steps complete, and the fixed groups keep the
// arithmetic (and so the result bits) independent of timing.  A task only
// ever waits for tasks taken from the queue before it, by workgroups that
// are running, so every wait ends.
template <typename T, bool ALIGNED>
__global__ __launch_bounds__(256, 2) void persist_sweep_kernel(
    const PersistItem<T>* __restrict__ items, const PersistTask* __restrict__ tasks, int ntasks,
    unsigned* __restrict__ cnt, int ncnt) {
  __shared__ int s_task;
  unsigned* head = cnt + ncnt;
  unsigned* err = cnt + ncnt + 1;
  for (;;) {
    __syncthreads();   // every thread has read s_task of the previous round
    if (threadIdx.x == 0) s_task = (int)atomicAdd(head, 1u);
    __syncthreads();
    const int t = s_task;
    if (t >= ntasks) return;
    const PersistTask tk = tasks[t];
    const PersistItem<T> it = items[tk.item];
    unsigned* mine = cnt + it.cnt + tk.ctile;
    const int nb = it.nb;
    const int r0 = tk.step * nb, sz = min(nb, it.n - r0);
    const int c0 = tk.ctile * kPB, nc = min(kPB, it.k - c0);
    int done = 0;   // blocks of X already folded into R(S_i, c)
    do {
      const int avail = min(done + kPassBlocks, tk.step);   // this pass: blocks done..avail-1
      if (threadIdx.x == 0 && avail > 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(mine, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
               (unsigned)avail) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins > kSpinLimit) {
            atomicOr(err, 1u);
            break;
          }
        }
      }
      __syncthreads();
      __threadfence();   // acquire for every wave: no stale X(S_j, c) in the caches
      // R(S_i, c) = (first pass ? B : R)(S_i, c) - L(S_i, blocks done..avail) X(..., c)
      auto p = persist_params<T>();
      p.A = it.L + (int64_t)r0 * it.ldl + (int64_t)done * nb; p.lda = it.ldl;
      p.B = it.X + (int64_t)done * nb * it.ldx + c0; p.ldb = it.ldx;
      p.Cin = done == 0 ? it.B + (int64_t)r0 * it.ldb + c0 : it.R + (int64_t)r0 * it.ldr + c0;
      p.ldci = done == 0 ? it.ldb : it.ldr;
      p.Cout = it.R + (int64_t)r0 * it.ldr + c0; p.ldco = it.ldr;
      p.M = sz; p.N = nc; p.K = (avail - done) * nb;
      p.alpha = -1.0; p.beta = 1.0;
      p.flags = G_BETA;
      persist_tile<T, ALIGNED>(p);
      done = avail;
      __threadfence();
      __syncthreads();
    } while (done < tk.step);
    {
      // X(S_i, c) = Linv_ii R(S_i, c)
      auto p = persist_params<T>();
      p.A = it.Linv + (int64_t)tk.step * nb * nb; p.lda = nb;
      p.B = it.R + (int64_t)r0 * it.ldr + c0; p.ldb = it.ldr;
      p.Cout = it.X + (int64_t)r0 * it.ldx + c0; p.ldco = it.ldx;
      p.M = sz; p.N = nc; p.K = sz;
      p.flags = G_A_LOWER | G_A_ZERO_UPPER;
      persist_tile<T, ALIGNED>(p);
    }
    __threadfence();   // release: X(S_i, c) is visible before the counter moves
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
hipError_t launch_persist(const void* items, const void* tasks, int ntasks, unsigned* cnt,
                          int ncnt, bool aligned, hipStream_t s) {
  hipError_t e = launch_fill_u32(cnt, ncnt + 2, 0u, s);
  if (e != hipSuccess || ntasks <= 0) return e;
  const unsigned grid = (unsigned)std::min(ntasks, kPersistMaxWG);
  const auto* it = static_cast<const PersistItem<T>*>(items);
  const auto* tk = static_cast<const PersistTask*>(tasks);
  if (aligned)
    persist_sweep_kernel<T, true><<<grid, 256, 0, s>>>(it, tk, ntasks, cnt, ncnt);
  else
    persist_sweep_kernel<T, false><<<grid, 256, 0, s>>>(it, tk, ntasks, cnt, ncnt);
  return hipGetLastError();
}

}  // namespace

void LaunchList::clear() {
  host_.clear();
  phases_.clear();
}

template <typename T>
size_t LaunchList::append(const T* data, size_t n) {
  size_t off = (host_.size() + 15) / 16 * 16;
  host_.resize(off + n * sizeof(T));
  if (n) memcpy(host_.data() + off, data, n * sizeof(T));
  return off;
}

namespace {
// Split of one grouped product (see SweepItem::part): products with at most
// half a round of 128 x 128 workgroups cut K into up to kSplitMax slices of
// at least kSplitMinChunks chunks each, as far as the scratch holds them.
template <typename T>
int grouped_ksplit(const GemmParams<T, T, T, float>& p) {
  if (!p.part) return 1;
  return grouped_split_slices(p.M, p.N, p.K, p.flags, p.part_bytes, (int)sizeof(T));
}
}  // namespace

int grouped_split_slices(int M, int N, int K, uint32_t flags, int64_t part_bytes, int elem) {
  if (M <= 0 || N <= 0) return 1;
  const int64_t tiles = gemm_wgs(M, N, K, flags, kBM, kBN);
  if (2 * tiles > kSplitTarget) return 1;
  const int64_t nck = (K + 128 / elem - 1) / (128 / elem);   // chunks of 128 bytes
  int64_t S = std::min<int64_t>(kSplitTarget / tiles, nck / kSplitMinChunks);
  S = std::min<int64_t>(S, kSplitMax);
  S = std::min<int64_t>(S, part_bytes / ((int64_t)M * N * elem));   // binary32/64 partials
  return S > 1 ? (int)S : 1;
}

template <typename P>
void LaunchList::add_gemm(int kind, int split_kind, std::vector<P> entries) {
  if (entries.empty()) return;
  using T = typename std::remove_const<typename std::remove_pointer<decltype(P::A)>::type>::type;
  // sub-launches: aligned narrow, aligned wide, unaligned (wide tiles)
  std::vector<P> sub[3];
  std::vector<P> split;
  for (P& e : entries) {
    e.ksplit = grouped_ksplit<T>(e);
    if (e.ksplit > 1) split.push_back(e);
    const bool al = gemm_aligned<T, kBM, kBN, false>(e);
    sub[!al ? 2 : (e.N <= kNarrowN ? 0 : 1)].push_back(e);
  }
  for (int v = 0; v < 3; ++v) {
    if (sub[v].empty()) continue;
    Phase ph{};
    ph.kind = kind;
    ph.count = (int)sub[v].size();
    ph.aligned = v < 2;
    ph.narrow = v == 0;
    const int bn = ph.narrow ? kNarrowN : kBN;
    std::vector<int> st(sub[v].size() + 1, 0);
    for (size_t i = 0; i < sub[v].size(); ++i) {
      const P& e = sub[v][i];
      st[i + 1] = st[i] + gemm_wgs(e.M, e.N, e.K, e.flags, kBM, bn) * e.ksplit;
    }
    ph.total = st.back();
    ph.entries_off = append(sub[v].data(), sub[v].size());
    ph.start_off = append(st.data(), st.size());
    if (ph.total > 0) phases_.push_back(ph);
  }
  if (split.empty()) return;
  Phase fin{};
  fin.kind = split_kind;
  fin.count = (int)split.size();
  std::vector<int> fs(split.size() + 1, 0);
  for (size_t i = 0; i < split.size(); ++i)
    fs[i + 1] = fs[i] + (int)ceil_div((int64_t)split[i].M * split[i].N, kFinChunk);
  fin.total = fs.back();
  fin.entries_off = append(split.data(), split.size());
  fin.start_off = append(fs.data(), fs.size());
  phases_.push_back(fin);
}

void LaunchList::add_gemm64(const std::vector<GemmP64>& entries) {
  add_gemm(PH_GEMM_F64, PH_SPLIT_F64, entries);
}

void LaunchList::add_gemm32(const std::vector<GemmP32>& entries) {
  add_gemm(PH_GEMM_F32, PH_SPLIT_F32, entries);
}

void LaunchList::add_ew(const std::vector<EwEntry>& entries) {
  if (entries.empty()) return;
  Phase ph{};
  ph.kind = PH_EW;
  ph.count = (int)entries.size();
  ph.aligned = false;
  std::vector<int> st(entries.size() + 1, 0);
  for (size_t i = 0; i < entries.size(); ++i)
    st[i + 1] = st[i] + (int)ceil_div((int64_t)entries[i].rows * entries[i].cols, kEwChunk);
  ph.total = st.back();
  ph.entries_off = append(entries.data(), entries.size());
  ph.start_off = append(st.data(), st.size());
  if (ph.total > 0) phases_.push_back(ph);
}

void red_split(int64_t rows, int64_t cols, int* chunk, int* nparts) {
  const int64_t total = rows * cols;
  int64_t c = std::max<int64_t>(kEwChunk, ceil_div(ceil_div(total, kRedMaxParts), 256) * 256);
  *chunk = (int)c;
  *nparts = (int)std::max<int64_t>(1, ceil_div(total, c));
}

void LaunchList::add_red(const std::vector<RedEntry>& entries) {
  if (entries.empty()) return;
  Phase ph{};
  ph.kind = PH_RED;
  ph.count = (int)entries.size();
  std::vector<int> st(entries.size() + 1, 0);
  for (size_t i = 0; i < entries.size(); ++i) st[i + 1] = st[i] + entries[i].nparts;
  ph.total = st.back();
  ph.entries_off = append(entries.data(), entries.size());
  ph.start_off = append(st.data(), st.size());
  if (ph.total > 0) phases_.push_back(ph);
}

void LaunchList::add_fin(const std::vector<FinEntry>& entries) {
  if (entries.empty()) return;
  Phase ph{};
  ph.kind = PH_FIN;
  ph.count = (int)entries.size();
  ph.total = ph.count;
  ph.entries_off = append(entries.data(), entries.size());
  ph.start_off = ph.entries_off;
  phases_.push_back(ph);
}

template <typename T>
void LaunchList::add_persist(const std::vector<PersistItem<T>>& items,
                             const std::vector<PersistTask>& tasks, unsigned* counters,
                             int ncounters, bool aligned) {
  Phase ph{};
  ph.kind = std::is_same<T, double>::value ? PH_PERSIST_F64 : PH_PERSIST_F32;
  ph.count = (int)items.size();
  ph.ntasks = (int)tasks.size();
  ph.total = std::min(ph.ntasks, kPersistMaxWG);
  ph.aligned = aligned;
  ph.counters = counters;
  ph.ncounters = ncounters;
  ph.entries_off = append(items.data(), items.size());
  ph.start_off = append(tasks.data(), tasks.size());
  if (ph.ntasks > 0) phases_.push_back(ph);
}
template void LaunchList::add_persist<double>(const std::vector<PersistItem<double>>&,
                                              const std::vector<PersistTask>&, unsigned*, int, bool);
template void LaunchList::add_persist<float>(const std::vector<PersistItem<float>>&,
                                             const std::vector<PersistTask>&, unsigned*, int, bool);

hipError_t LaunchList::run(const void* dev, hipStream_t s) const {
  const char* base = static_cast<const char*>(dev);
  for (const Phase& ph : phases_) {
    if (ph.kind == PH_PERSIST_F64 || ph.kind == PH_PERSIST_F32) {
      const void* items = base + ph.entries_off;
      const void* tasks = base + ph.start_off;
      hipError_t e = ph.kind == PH_PERSIST_F64
                         ? launch_persist<double>(items, tasks, ph.ntasks, ph.counters,
                                                  ph.ncounters, ph.aligned, s)
                         : launch_persist<float>(items, tasks, ph.ntasks, ph.counters,
                                                 ph.ncounters, ph.aligned, s);
      if (e != hipSuccess) return e;
      continue;
    }
    const int* st = reinterpret_cast<const int*>(base + ph.start_off);
    dim3 grid((unsigned)ph.total);
    if (ph.kind == PH_GEMM_F64) {
      const GemmP64* e = reinterpret_cast<const GemmP64*>(base + ph.entries_off);
      if (ph.narrow)
        gemm_grouped_kernel<double, double, double, float, kBM, kNarrowN, 4, 1, false, true>
            <<<grid, 256, 0, s>>>(e, st, ph.count);
      else if (ph.aligned)
        gemm_grouped_kernel<double, double, double, float, kBM, kBN, 2, 2, false, true>
            <<<grid, 256, 0, s>>>(e, st, ph.count);
      else
        gemm_grouped_kernel<double, double, double, float, kBM, kBN, 2, 2, false, false>
            <<<grid, 256, 0, s>>>(e, st, ph.count);
    } else if (ph.kind == PH_GEMM_F32) {
      const GemmP32* e = reinterpret_cast<const GemmP32*>(base + ph.entries_off);
      if (ph.narrow)
        gemm_grouped_kernel<float, float, float, float, kBM, kNarrowN, 4, 1, false, true>
            <<<grid, 256, 0, s>>>(e, st, ph.count);
      else if (ph.aligned)
        gemm_grouped_kernel<float, float, float, float, kBM, kBN, 2, 2, false, true>
            <<<grid, 256, 0, s>>>(e, st, ph.count);
      else
        gemm_grouped_kernel<float, float, float, float, kBM, kBN, 2, 2, false, false>
            <<<grid, 256, 0, s>>>(e, st, ph.count);
    } else if (ph.kind == PH_SPLIT_F64) {
      const GemmP64* e = reinterpret_cast<const GemmP64*>(base + ph.entries_off);
      grouped_split_finish<double><<<grid, 256, 0, s>>>(e, st, ph.count);
    } else if (ph.kind == PH_SPLIT_F32) {
      const GemmP32* e = reinterpret_cast<const GemmP32*>(base + ph.entries_off);
      grouped_split_finish<float><<<grid, 256, 0, s>>>(e, st, ph.count);
    } else if (ph.kind == PH_RED) {
      const RedEntry* e = reinterpret_cast<const RedEntry*>(base + ph.entries_off);
      grouped_red_kernel<<<grid, 256, 0, s>>>(e, st, ph.count);
    } else if (ph.kind == PH_FIN) {
      const FinEntry* e = reinterpret_cast<const FinEntry*>(base + ph.entries_off);
      grouped_fin_kernel<<<grid, 64, 0, s>>>(e);
    } else {
      const EwEntry* e = reinterpret_cast<const EwEntry*>(base + ph.entries_off);
      grouped_ew_kernel<<<grid, 256, 0, s>>>(e, st, ph.count);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

template <typename T>
void record_sweep(LaunchList& list, const std::vector<SweepItem<T>>& items) {
  int64_t max_m = 0;
  for (const auto& it : items) max_m = std::max(max_m, ceil_div(it.n, it.n0));
  for (int64_t i = 0; i < max_m; ++i) {
    std::vector<GemmParams<T, T, T, float>> trmm, upd;
    for (const auto& it : items) {
      const int64_t n0 = it.n0;
      const int64_t m = ceil_div(it.n, n0);
      if (i >= m || it.k == 0) continue;
      const int64_t r0 = i * n0, sz = std::min(n0, it.n - r0);
      // X(S_i) = Linv_ii * B'(S_i)
      auto p = gemm_params<T, T, T, float>();
      p.A = it.Linv + i * n0 * n0; p.lda = n0;
      p.B = (i == 0) ? it.B : it.R + r0 * it.ldr;
      p.ldb = (i == 0) ? it.ldb : it.ldr;
      p.Cout = it.X + r0 * it.ldx; p.ldco = it.ldx;
      p.M = (int)sz; p.N = (int)it.k; p.K = (int)sz;
      p.flags = G_A_LOWER | G_A_ZERO_UPPER;
      p.part = it.part; p.part_bytes = it.part_bytes;
      trmm.push_back(p);
      if (i + 1 < m) {
        // B'(T_{i+1}) = B'(T_{i+1}) - L(T_{i+1}, S_i) X(S_i)
        const int64_t t0 = r0 + n0;
        auto q = gemm_params<T, T, T, float>();
        q.A = it.L + t0 * it.ldl + r0; q.lda = it.ldl;
        q.B = it.X + r0 * it.ldx; q.ldb = it.ldx;
        q.Cin = (i == 0) ? it.B + t0 * it.ldb : it.R + t0 * it.ldr;
        q.ldci = (i == 0) ? it.ldb : it.ldr;
        q.Cout = it.R + t0 * it.ldr; q.ldco = it.ldr;
        q.M = (int)(it.n - t0); q.N = (int)it.k; q.K = (int)sz;
        q.alpha = -1.0; q.beta = 1.0;
        q.flags = G_BETA;
        q.part = it.part; q.part_bytes = it.part_bytes;
        upd.push_back(q);
      }
    }
    if constexpr (std::is_same<T, double>::value) {
      list.add_gemm64(trmm);
      list.add_gemm64(upd);
    } else {
      list.add_gemm32(trmm);
      list.add_gemm32(upd);
    }
  }
}

template void record_sweep<double>(LaunchList&, const std::vector<SweepItem<double>>&);
template void record_sweep<float>(LaunchList&, const std::vector<SweepItem<float>>&);

template <typename T>
void record_sweep_back(LaunchList& list, const std::vector<SweepItem<T>>& items) {
  int64_t max_m = 0;
  for (const auto& it : items) max_m = std::max(max_m, ceil_div(it.n, it.n0));
  for (int64_t j = 0; j < max_m; ++j) {
    std::vector<GemmParams<T, T, T, float>> diag, upd;
    for (const auto& it : items) {
      const int64_t n0 = it.n0;
      const int64_t m = ceil_div(it.n, n0);
      if (j >= m || it.k == 0) continue;
      const int64_t i = m - 1 - j;
      const int64_t r0 = i * n0, sz = std::min(n0, it.n - r0);
      // X(S_i) = Uinv_ii * B'(S_i)
      auto p = gemm_params<T, T, T, float>();
      p.A = it.Linv + i * n0 * n0; p.lda = n0;
      p.B = (j == 0) ? it.B + r0 * it.ldb : it.R + r0 * it.ldr;
      p.ldb = (j == 0) ? it.ldb : it.ldr;
      p.Cout = it.X + r0 * it.ldx; p.ldco = it.ldx;
      p.M = (int)sz; p.N = (int)it.k; p.K = (int)sz;
      p.flags = G_A_UPPER;
      p.part = it.part; p.part_bytes = it.part_bytes;
      diag.push_back(p);
      if (i > 0) {
        // B'(0:r0) = B'(0:r0) - U(0:r0, S_i) X(S_i)
        auto q = gemm_params<T, T, T, float>();
        q.A = it.L + r0; q.lda = it.ldl;
        q.B = it.X + r0 * it.ldx; q.ldb = it.ldx;
        q.Cin = (j == 0) ? it.B : it.R;
        q.ldci = (j == 0) ? it.ldb : it.ldr;
        q.Cout = it.R; q.ldco = it.ldr;
        q.M = (int)r0; q.N = (int)it.k; q.K = (int)sz;
        q.alpha = -1.0; q.beta = 1.0;
        q.flags = G_BETA;
        q.part = it.part; q.part_bytes = it.part_bytes;
        upd.push_back(q);
      }
    }
    if constexpr (std::is_same<T, double>::value) {
      list.add_gemm64(diag);
      list.add_gemm64(upd);
    } else {
      list.add_gemm32(diag);
      list.add_gemm32(upd);
    }
  }
}
template void record_sweep_back<double>(LaunchList&, const std::vector<SweepItem<double>>&);
template void record_sweep_back<float>(LaunchList&, const std::vector<SweepItem<float>>&);

template <typename T>
int persist_counter_words(const std::vector<SweepItem<T>>& items) {
  int64_t c = 0;
  for (const auto& it : items)
    if (it.n > 0 && it.k > 0) c += ceil_div(it.k, kPB);
  return (int)c;
}
template int persist_counter_words<double>(const std::vector<SweepItem<double>>&);
template int persist_counter_words<float>(const std::vector<SweepItem<float>>&);

template <typename T>
void record_persist(LaunchList& list, const std::vector<SweepItem<T>>& items, unsigned* counters) {
  constexpr int VEC = 16 / sizeof(T);
  auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  std::vector<PersistItem<T>> pis;
  std::vector<int> order;
  bool aligned = true;
  int cnt = 0;
  for (const auto& it : items) {
    if (it.n <= 0 || it.k <= 0) continue;
    PersistItem<T> q{};
    q.L = it.L; q.ldl = it.ldl;
    q.Linv = it.Linv;
    q.B = it.B; q.ldb = it.ldb;
    q.X = it.X; q.ldx = it.ldx;
    q.R = it.R; q.ldr = it.ldr;
    q.n = (int)it.n; q.k = (int)it.k;
    q.nb = (int)it.n0;
    q.m = (int)ceil_div(it.n, it.n0);
    q.nct = (int)ceil_div(it.k, kPB);
    q.cnt = cnt;
    cnt += q.nct;
    aligned &= al(q.L) && al(q.Linv) && al(q.X) && al(q.R) && q.ldl % VEC == 0 &&
               q.ldx % VEC == 0 && q.ldr % VEC == 0 && q.nb % VEC == 0 && q.n % VEC == 0 &&
               q.k % VEC == 0 && (int64_t)kPB * q.ldl * (int64_t)sizeof(T) < kBufOOB &&
               (int64_t)q.n * q.ldx * (int64_t)sizeof(T) < kBufOOB &&
               (int64_t)q.n * q.ldr * (int64_t)sizeof(T) < kBufOOB;
    pis.push_back(q);
  }
  // step-major task order, systems with more steps first within a step
  std::vector<int> idx(pis.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return pis[a].m > pis[b].m; });
  int max_m = 0;
  for (const auto& q : pis) max_m = std::max(max_m, q.m);
  std::vector<PersistTask> tasks;
  for (int i = 0; i < max_m; ++i)
    for (int j : idx) {
      if (i >= pis[j].m) continue;
      for (int c = 0; c < pis[j].nct; ++c) tasks.push_back(PersistTask{j, i, c, 0});
    }
  list.add_persist<T>(pis, tasks, counters, cnt, aligned);
}
template void record_persist<double>(LaunchList&, const std::vector<SweepItem<double>>&, unsigned*);
template void record_persist<float>(LaunchList&, const std::vector<SweepItem<float>>&, unsigned*);

}  // namespace trsm

// ---------------------------------------------------------------------------
// C ABI: batches
// ---------------------------------------------------------------------------
using namespace trsm;

struct trsm_batch_s {
  std::vector<trsm_batch_item> items;
  trsm_precision prec = TRSM_F64;
  int64_t n0 = 128;
  size_t table_bytes = 0;      // upper bound, reserved at the head of the workspace
  size_t ws_bytes = 0;
  std::vector<size_t> r_off;   // offset of each item's running right-hand side
  size_t cnt_off = 0;          // persistent sweep (n0 == kPB): its counter words
  LaunchList list;
  void* pinned = nullptr;      // host staging of the table (page-locked)
  size_t pinned_bytes = 0;
  // captured graph, valid for (graph_ws, graph_stream)
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void* graph_ws = nullptr;
  hipStream_t graph_stream = nullptr;
};

namespace {

constexpr size_t kAlignB = 256;
inline size_t alignb(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

bool is_pow2_64(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// leading dimension of a system's running right-hand side (16-byte rows)
int64_t ldr_for(int64_t k) { return std::max<int64_t>((k + 3) / 4 * 4, 4); }

size_t linv32_offset(int64_t n, int64_t n0) {
  const int64_t m = ceil_div(n, n0);
  return alignb((size_t)m * n0 * n0 * 8);
}

template <typename T>
void build_list(trsm_batch_s* b, char* ws) {
  std::vector<SweepItem<T>> its;
  for (size_t i = 0; i < b->items.size(); ++i) {
    const trsm_batch_item& x = b->items[i];
    SweepItem<T> s{};
    s.n = x.n;
    s.k = x.k;
    s.n0 = effective_n0(x.n, b->n0);
    s.L = static_cast<const T*>(x.L);
    s.ldl = x.ldl;
    const char* lb = static_cast<const char*>(x.Linv);
    s.Linv = reinterpret_cast<const T*>(
        lb + (std::is_same<T, float>::value ? linv32_offset(x.n, s.n0) : 0));
    s.B = static_cast<const T*>(x.B);
    s.ldb = x.ldb;
    s.X = static_cast<T*>(x.X);
    s.ldx = x.ldx;
    s.R = reinterpret_cast<T*>(ws + b->r_off[i]);
    s.ldr = ldr_for(x.k);
    its.push_back(s);
  }
  b->list.clear();
  if (b->n0 == kPB)
    record_persist<T>(b->list, its, reinterpret_cast<unsigned*>(ws + b->cnt_off));
  else
    record_sweep<T>(b->list, its);
}

}  // namespace

extern "C" {

trsm_status trsm_batch_create(int32_t count, const trsm_batch_item* items, trsm_precision prec,
                              int64_t n0, trsm_batch_t* out) {
  if (!out) return TRSM_EINVAL;
  *out = nullptr;
  if (count < 0 || (count > 0 && !items)) return TRSM_EINVAL;
  if (prec != TRSM_F64 && prec != TRSM_F32) return TRSM_EINVAL;
  if (!is_pow2_64(n0)) return TRSM_EINVAL;
  const size_t es = prec == TRSM_F32 ? 4 : 8;
  for (int32_t i = 0; i < count; ++i) {
    const trsm_batch_item& x = items[i];
    if (x.n < 0 || x.k < 0 || x.n > (1 << 30) || x.k > (1 << 30)) return TRSM_EINVAL;
    if (x.n == 0 || x.k == 0) continue;
    if (!x.L || !x.Linv || !x.B || !x.X) return TRSM_EINVAL;
    if (x.ldl < x.n || x.ldb < x.k || x.ldx < x.k) return TRSM_EINVAL;
    if (((uintptr_t)x.Linv) % kAlignB) return TRSM_EINVAL;
    // X must not overlap B (the batch has no in-place path)
    const uintptr_t b0 = (uintptr_t)x.B, b1 = b0 + ((size_t)(x.n - 1) * x.ldb + x.k) * es;
    const uintptr_t x0 = (uintptr_t)x.X, x1 = x0 + ((size_t)(x.n - 1) * x.ldx + x.k) * es;
    if (b0 < x1 && x0 < b1) return TRSM_EINVAL;
  }
  trsm_batch_s* b = new (std::nothrow) trsm_batch_s();
  if (!b) return TRSM_ENOMEM;
  b->items.assign(items, items + count);
  b->prec = prec;
  b->n0 = n0;
  // table size: record once with a null workspace to measure it
  size_t off = 0;
  b->r_off.resize(count);
  int64_t tiles = 0;
  for (int32_t i = 0; i < count; ++i) {
    b->r_off[i] = off;
    off = alignb(off + (size_t)items[i].n * ldr_for(items[i].k) * es);
    if (items[i].n > 0 && items[i].k > 0) tiles += ceil_div(items[i].k, kPB);
  }
  b->cnt_off = off;
  off = alignb(off + (size_t)(tiles + 2) * 4);
  if (prec == TRSM_F64) build_list<double>(b, nullptr);
  else build_list<float>(b, nullptr);
  b->table_bytes = alignb(b->list.table_bytes() + 64);
  for (int32_t i = 0; i < count; ++i) b->r_off[i] += b->table_bytes;
  b->cnt_off += b->table_bytes;
  b->ws_bytes = b->table_bytes + off;
  *out = b;
  return TRSM_OK;
}

trsm_status trsm_batch_workspace_bytes(trsm_batch_t b, size_t* bytes) {
  if (!b || !bytes) return TRSM_EINVAL;
  *bytes = b->ws_bytes;
  return TRSM_OK;
}

trsm_status trsm_batch_run(trsm_batch_t b, void* workspace, void* stream, int32_t use_graph) {
  if (!b) return TRSM_EINVAL;
  if (b->items.empty()) return TRSM_OK;
  if (!workspace || ((uintptr_t)workspace) % kAlignB) return TRSM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (use_graph && !s) return TRSM_EINVAL;  // the legacy default stream cannot be captured
  auto fail = [](hipError_t e) { return (trsm_status)note_hip_error(e); };
  if (use_graph && b->exec && b->graph_ws == workspace && b->graph_stream == s) {
    hipError_t e = hipGraphLaunch(b->exec, s);
    return e == hipSuccess ? TRSM_OK : fail(e);
  }
  char* ws = static_cast<char*>(workspace);
  if (b->prec == TRSM_F64) build_list<double>(b, ws);
  else build_list<float>(b, ws);
  const size_t tb = b->list.table_bytes();
  if (tb > b->table_bytes) return TRSM_EINVAL;  // cannot happen: same recording
  if (b->pinned_bytes < tb) {
    if (b->pinned) (void)hipHostFree(b->pinned);
    b->pinned = nullptr;
    b->pinned_bytes = 0;
    if (hipHostMalloc(&b->pinned, tb, hipHostMallocDefault) != hipSuccess) return TRSM_ENOMEM;
    b->pinned_bytes = tb;
  }
  memcpy(b->pinned, b->list.host_table(), tb);
  if (!use_graph) {
    hipError_t e = hipMemcpyAsync(ws, b->pinned, tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = b->list.run(ws, s);
    return e == hipSuccess ? TRSM_OK : fail(e);
  }
  // capture the table upload and every launch into one graph
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipError_t e0 = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e0 != hipSuccess) return fail(e0);
  hipError_t e1 = hipMemcpyAsync(ws, b->pinned, tb, hipMemcpyHostToDevice, s);
  hipError_t e2 = e1 == hipSuccess ? b->list.run(ws, s) : e1;
  hipGraph_t g = nullptr;
  hipError_t e3 = hipStreamEndCapture(s, &g);
  if (e2 != hipSuccess || e3 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return fail(e2 != hipSuccess ? e2 : (e3 != hipSuccess ? e3 : hipErrorUnknown));
  }
  hipError_t e4 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e4 != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->exec = nullptr;
    return fail(e4);
  }
  b->graph = g;
  b->graph_ws = workspace;
  b->graph_stream = s;
  hipError_t e5 = hipGraphLaunch(b->exec, s);
  return e5 == hipSuccess ? TRSM_OK : fail(e5);
}

trsm_status trsm_batch_check(trsm_batch_t b, const void* workspace) {
  if (!b || !workspace) return TRSM_EINVAL;
  if (b->n0 != kPB || b->items.empty()) return TRSM_OK;
  int64_t tiles = 0;
  for (const auto& x : b->items)
    if (x.n > 0 && x.k > 0) tiles += ceil_div(x.k, kPB);
  unsigned err = 0;
  const char* w = static_cast<const char*>(workspace) + b->cnt_off + (size_t)(tiles + 1) * 4;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&err, w, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return (trsm_status)note_hip_error(e);
  return err ? TRSM_EHIP : TRSM_OK;
}

trsm_status trsm_batch_destroy(trsm_batch_t b) {
  if (!b) return TRSM_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->pinned) (void)hipHostFree(b->pinned);
  delete b;
  return TRSM_OK;
}

}  // extern "C"
