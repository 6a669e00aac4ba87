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
};

constexpr int kEwChunk = 4096;  // elements per workgroup in grouped elementwise launches

enum PhaseKind : int { PH_GEMM_F64 = 0, PH_GEMM_F32 = 1, PH_EW = 2 };

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
    size_t start_off;    // byte offset of the int prefix array (n + 1 values)
    int count;
    int total;           // workgroups
    bool aligned;
  };
  template <typename T>
  size_t append(const T* data, size_t n);
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
};

// Append the 2m-1 phases of the right-looking sweep for all items; phase i
// of every item goes into the same grouped launch.
template <typename T>
void record_sweep(LaunchList& list, const std::vector<SweepItem<T>>& items);

// The block size a plan made with (n, n0) uses: n0 capped at the next power
// of two >= n.
inline int64_t effective_n0(int64_t n, int64_t n0) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return n0 > p ? p : n0;
}

}  // namespace trsm
