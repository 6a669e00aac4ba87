// Shared device/host helpers for the gfx950 triangular-solve kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace trsm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

typedef __bf16 bf16_t;
typedef _Float16 f16_t;
// 8-bit float (e4m3: 4 exponent bits, 3 mantissa bits) held as its bit
// pattern; produced by the hardware conversion and consumed by the 8-bit
// matrix-core instruction, which use the same encoding.
typedef uint8_t fp8_t;

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Matrix-core traits.  Every 16x16 output tile is produced by the 16x16xK
// MFMA of the element type.  Operands: lane l feeds row l%16 of A and
// column l%16 of B with kPerLane reduction indices; which k a lane feeds is
// picked by the kernel (any permutation of k, used consistently for both
// operands, gives the same sum up to rounding order).  Results: lane l holds
// column l%16, and its four values r = 0..3 are rows out_row(l/16, r) --
// 4*(l/16) + r for the binary32-accumulating instructions, 4*r + l/16 for the
// binary64 one (checked on gfx950 against a host product).
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<double> {
  using Acc = double;
  using Frag = double;   // one element per lane
  using Out = d4;
  static constexpr int kPerLane = 1;   // k values per lane per instruction
  static __device__ __forceinline__ Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int r) { return 4 * r + g; }
};

template <> struct Mfma<float> {
  using Acc = float;
  using Frag = float;
  using Out = f4;
  static constexpr int kPerLane = 1;
  static __device__ __forceinline__ Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int r) { return 4 * g + r; }
};

template <> struct Mfma<bf16_t> {
  using Acc = float;
  using Frag = bf16x8;
  using Out = f4;
  static constexpr int kPerLane = 8;
  static __device__ __forceinline__ Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int r) { return 4 * g + r; }
};

template <> struct Mfma<f16_t> {
  using Acc = float;
  using Frag = f16x8;
  using Out = f4;
  static constexpr int kPerLane = 8;
  static __device__ __forceinline__ Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int r) { return 4 * g + r; }
};

template <> struct Mfma<fp8_t> {
  using Acc = float;
  using Frag = long;   // eight 8-bit values
  using Out = f4;
  static constexpr int kPerLane = 8;
  static __device__ __forceinline__ Out mma(Frag a, Frag b, Out c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int g, int r) { return 4 * g + r; }
};

template <typename To, typename From>
__device__ __forceinline__ To cvt(From v) { return static_cast<To>(v); }
// round to nearest e4m3 (saturating conversion of the hardware)
template <> __device__ __forceinline__ fp8_t cvt<fp8_t, float>(float v) {
  return (fp8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xFF);
}
template <> __device__ __forceinline__ fp8_t cvt<fp8_t, double>(double v) {
  return cvt<fp8_t, float>(static_cast<float>(v));
}
template <> __device__ __forceinline__ bf16_t cvt<bf16_t, float>(float v) { return static_cast<bf16_t>(v); }
template <> __device__ __forceinline__ bf16_t cvt<bf16_t, double>(double v) { return static_cast<bf16_t>(static_cast<float>(v)); }
template <> __device__ __forceinline__ f16_t cvt<f16_t, double>(double v) { return static_cast<f16_t>(static_cast<float>(v)); }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace trsm
