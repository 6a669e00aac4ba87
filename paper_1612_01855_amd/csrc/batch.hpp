// Grouped ("batched") launches: the blocked sweep of Alg. It-Inv-TRSM for
// many independent systems of uneven n and k at once.  Every phase of the
// sweep (the diagonal apply of step i, the trailing update of step i) becomes
// ONE grouped launch covering the tiles of every system that has that phase;
// systems with fewer blocks simply drop out of later phases.  The launch list
// is recorded once per batch into a device table and can be replayed from a
// captured hipGraph.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "gemm.hpp"

namespace trsm {

// Elementwise conversion/copy over many matrices in one launch.
enum EwOp : int {
  EW_F64_TO_F32 = 0,      // dst(float)  = scale * src(double)
  EW_F32_TO_F64_SET = 1,  // dst(double) = scale * src(float)
  EW_F32_TO_F64_ADD = 2,  // dst(double) += scale * src(float)
  EW_F64_COPY = 3,        // dst(double) = scale * src(double)
  EW_F32_COPY = 4,        // dst(float)  = scale * src(float)
  // Scaled conversions of a served request's running right-hand side.  Its
  // scale s is a power of two taken from the sums of squares held in `part`
  // (nparts partials, see RedEntry): s = 2^-e with the Frobenius norm below
  // 2^e, so every scaled entry is below 1 in magnitude and binary32 keeps the
  // matrix's leading bits whatever its size.
  EW_F64_TO_F32_PS = 5,   // dst(float)  = s * src(double); stores s in *sc
  EW_F32_TO_F64_SET_SC = 6,  // dst(double)  = src(float) / *sc
  EW_F32_TO_F64_ADD_SC = 7,  // dst(double) += src(float) / *sc
  EW_F64_ADD = 8,         // dst(double) += src(double)
};

// rows x cols elements are written; source columns at or beyond
// `valid_cols` are not read and produce zeros (padding of internal buffers).
struct EwEntry {
  const void* src;
  int64_t lds;
  void* dst;
  int64_t ldd;
  int rows, cols;
  double scale;
  int op;
  int valid_cols;
  const double* part;     // EW_F64_TO_F32_PS: partial sums of squares (quantity 0)
  double* sc;             // the scale (written by _PS, read by _SC ops)
  int nparts;
};

// Deterministic grouped reductions of the serving pipeline.  Entry e is split
// into nparts chunks of `chunk` consecutive elements (row-major, rows x cols);
// chunk p writes its three sums of squares, each as s * 4^x with s in a safe
// range (no overflow or underflow for any finite data), to
// part[kPartStride p + q] = s_q and part[kPartStride p + 3 + q] = x_q, in a
// fixed order, so a request's sums do not depend on what else is in its batch.
enum RedOp : int {
  RD_LOAD = 0,   // b = a (rows >= valid_rows and columns >= valid_cols: zero);
                 // part.x = sum a^2
  RD_RES = 1,    // part.x = sum a^2
  RD_NORMS = 2,  // part = {sum a^2, sum b^2, sum d^2}; xo = b (valid rows and columns)
};
constexpr int kRedMaxParts = 256;
constexpr int kPartStride = 8;

struct RedEntry {
  const double* a; int64_t lda;   // LOAD: the caller's B; RES, NORMS: the residual
  double* b; int64_t ldb;         // LOAD: the padded copy (written); NORMS: X (read)
  const void* d; int64_t ldd;     // NORMS: the last correction, or null
  double* xo; int64_t ldxo;       // NORMS: the caller's X (written)
  double* part;                   // nparts x kPartStride partials
  int rows, cols, valid_rows, valid_cols, chunk, nparts, op, d_f64;
};

// Final sums of a reduction over all parts: out[2q] = s_q, out[2q+1] = x_q
// (the sum of squares of quantity q is s_q 4^x_q), with the third sum
// divided by (*sc)^2 when sc is set (a correction computed in scaled units).
// `out` may be mapped host memory.
struct FinEntry {
  const double* part;
  const double* sc;
  double* out;
  int nparts;
};

// chunk and nparts of a reduction over rows x cols elements
void red_split(int64_t rows, int64_t cols, int* chunk, int* nparts);

// K slices that phase launches give a product (see SweepItem::part) with
// part_bytes of scratch; elem = bytes of its (binary32 or binary64) elements.
int grouped_split_slices(int M, int N, int K, uint32_t flags, int64_t part_bytes, int elem);

constexpr int kEwChunk = 4096;  // elements per workgroup in grouped elementwise launches

enum PhaseKind : int { PH_GEMM_F64 = 0, PH_GEMM_F32 = 1, PH_EW = 2, PH_PERSIST_F64 = 3,
                       PH_PERSIST_F32 = 4, PH_RED = 5, PH_FIN = 6, PH_SPLIT_F64 = 7,
                       PH_SPLIT_F32 = 8 };

// Persistent sweep (left-looking Alg. It-Inv-TRSM over many systems in one
// launch).  A task is (system, step i, column tile c):
//   R(S_i, c) = B(S_i, c) - L(S_i, 0:i n0) X(0:i n0, c);  X(S_i, c) = Linv_ii R(S_i, c)
// with n0 = kPB.  Task (i, c) needs tasks (0..i-1, c) of its system: one
// counter per (system, column tile) holds the number of finished steps.
constexpr int kPB = 64;          // rows of a step (the block size n0) and columns of a tile
constexpr int kPersistMaxWG = 1024;

template <typename T>
struct PersistItem {
  const T* L; int64_t ldl;
  const T* Linv;                 // m packed kPB x kPB inverses
  const T* B; int64_t ldb;
  T* X; int64_t ldx;
  T* R; int64_t ldr;             // n x k workspace
  int n, k, m, nct;              // nct = ceil(k / kPB)
  int cnt;                       // index of this system's first counter
  int nb;                        // block size of Linv: kPB, or next_pow2(n) < kPB when m == 1
};

struct PersistTask {
  int item, step, ctile, pad;
};

using GemmP64 = GemmParams<double, double, double, float>;
using GemmP32 = GemmParams<float, float, float, float>;

// A recorded list of grouped launches.  Host side: entries are appended per
// phase; upload() packs them (and the per-phase workgroup prefix tables)
// into one contiguous block that lives in device memory; run() issues the
// launches on a stream.
class LaunchList {
 public:
  void clear();
  void add_gemm64(const std::vector<GemmP64>& entries);
  void add_gemm32(const std::vector<GemmP32>& entries);
  void add_ew(const std::vector<EwEntry>& entries);
  void add_red(const std::vector<RedEntry>& entries);
  void add_fin(const std::vector<FinEntry>& entries);
  // One persistent launch (preceded by clearing its counters): `counters`
  // (device, ncounters + 2 words: the per-tile counters, the queue head and
  // an error word that is set if a wait ever gives up) lives in the caller's
  // workspace.
  template <typename T>
  void add_persist(const std::vector<PersistItem<T>>& items, const std::vector<PersistTask>& tasks,
                   unsigned* counters, int ncounters, bool aligned);
  size_t table_bytes() const { return host_.size(); }
  size_t phases() const { return phases_.size(); }
  // Host copy of the packed table (to be copied to `dev` before run()).
  const void* host_table() const { return host_.data(); }
  // Launch every phase, reading the packed table at device address `dev`.
  hipError_t run(const void* dev, hipStream_t s) const;

 private:
  struct Phase {
    int kind;
    size_t entries_off;  // byte offset of the entry array in the table
    size_t start_off;    // byte offset of the int prefix array (n + 1 values); tasks (persistent)
    int count;
    int total;           // workgroups
    bool aligned;
    bool narrow = false;            // products of at most kNarrowN columns: 128 x 32 tiles
    unsigned* counters = nullptr;   // persistent: counters, queue head, error word
    int ncounters = 0;
    int ntasks = 0;
  };
  template <typename T>
  size_t append(const T* data, size_t n);
  template <typename P>
  void add_gemm(int kind, int split_kind, std::vector<P> entries);
  std::vector<char> host_;
  std::vector<Phase> phases_;
};

// One system of a batch in working precision T.  n0 is the system's own
// diagonal block size (the plan caps it at the next power of two >= n).
template <typename T>
struct SweepItem {
  int64_t n, k, n0;
  const T* L; int64_t ldl;      // lower triangle read
  const T* Linv;                // m packed n0 x n0 inverses (element type T)
  const T* B; int64_t ldb;      // right-hand side (read)
  T* X; int64_t ldx;            // solution (written)
  T* R; int64_t ldr;            // running right-hand side (workspace, n x k)
  // Optional split-K scratch for this item's products (phase launches): a
  // product with few tiles and a deep K is cut into K slices whose partial
  // sums are added in a fixed order by a following finish launch.  The
  // split depends only on the product's shape and part_bytes, so an item's
  // bits do not depend on what else is in the batch.
  void* part = nullptr; int64_t part_bytes = 0;
};

// Append the 2m-1 phases of the right-looking sweep for all items; phase i
// of every item goes into the same grouped launch.
template <typename T>
void record_sweep(LaunchList& list, const std::vector<SweepItem<T>>& items);

// Append the backward sweep of the transposed problem for all items: here
// L is U = L^T (upper triangular, zeros below the diagonal) and Linv holds
// the blocks Uinv_ii = Linv_ii^T; phase j of every item is its step
// i = m - 1 - j: X(S_i) = Uinv_ii B'(S_i), B'(0:i n0) -= U(0:i n0, S_i) X(S_i).
template <typename T>
void record_sweep_back(LaunchList& list, const std::vector<SweepItem<T>>& items);

// Append the persistent sweep for all items (each with n0 == kPB): tasks in
// step-major order, the systems with the most steps first.  `counters` as in
// LaunchList::add_persist (one per column tile of every system).
template <typename T>
void record_persist(LaunchList& list, const std::vector<SweepItem<T>>& items, unsigned* counters);

// Counter words record_persist needs for these items (tiles + head + error).
template <typename T>
int persist_counter_words(const std::vector<SweepItem<T>>& items);

// The block size a plan made with (n, n0) uses: n0 capped at the next power
// of two >= n.
inline int64_t effective_n0(int64_t n, int64_t n0) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return n0 > p ? p : n0;
}

}  // namespace trsm
