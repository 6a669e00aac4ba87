// Non-GEMM kernels of the gfx950 triangular solver: diagonal-block
// extraction, the LDS leaf of the recursive triangular inversion, the
// substitution leaf of the recursive baseline, precision conversions and
// deterministic norm reductions.
#include "kernels.hpp"

#include <math.h>

namespace trsm {

namespace {

// threads for a workgroup that walks one row of n0 elements
inline unsigned row_threads(int64_t n0) { return (unsigned)std::min<int64_t>(256, (n0 + 63) / 64 * 64); }

inline unsigned grid_for(int64_t work, int threads, int64_t cap = 1 << 20) {
  int64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Alg. Diagonal-Inverter, data movement: the block diagonal L_D is copied
// into its own packed buffer (one n0 x n0 binary64 block per S_i).
// ---------------------------------------------------------------------------
template <typename TL>
__global__ __launch_bounds__(256) void extract_diag_kernel(const TL* __restrict__ L, int64_t ldl,
                                                           int64_t n, int64_t n0,
                                                           double* __restrict__ Linv,
                                                           unsigned long long* bad, bool upper) {
  // one row of one packed block per workgroup (row index b n0 + i is also
  // the global row of L), threads along its columns
  const int64_t gr = blockIdx.x;
  const int64_t b = gr / n0, i = gr - b * n0;
  double* __restrict__ out = Linv + gr * n0;
  for (int64_t j = threadIdx.x; j < n0; j += blockDim.x) {
    const int64_t gc = b * n0 + j;
    double v;
    if (gr < n && gc < n) {
      v = (j <= i) ? static_cast<double>(upper ? L[gc * ldl + gr] : L[gr * ldl + gc]) : 0.0;
      if (i == j && (!(v != 0.0) || !isfinite(v))) atomicMin(bad, (unsigned long long)gr);
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    out[j] = v;
  }
}

// ---------------------------------------------------------------------------
// Alg. RecTriInv base case ("sequential inversion"): the nb x nb leaf is
// inverted by substitution on the identity.  Thread t owns column t of the
// inverse, kept in registers:
//   x[i] = (delta(i, t) - sum_{p<i} l[i][p] x[p]) / l[i][i],   i = 0 .. 63,
// which is zero above the diagonal (i < t) and 1 / l[t][t] on it.  Every lane
// reads the same l[i][p] (an LDS broadcast); the sum runs in four partial
// sums.  Rows and columns at or beyond nb hold the identity.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void trtri_leaf_kernel(double* __restrict__ Linv, int64_t n0,
                                                        int64_t nb, int64_t lpb) {
  __shared__ __attribute__((aligned(16))) double Ls[64][64];
  const int64_t leaf = blockIdx.x;
  const int64_t b = leaf / lpb, q = leaf % lpb;
  double* P = Linv + b * n0 * n0 + q * nb * (n0 + 1);
  const int t = threadIdx.x;
  for (int i = 0; i < 64; ++i) {
    double v;
    if (i < nb && t < nb) v = (t <= i) ? P[(int64_t)i * n0 + t] : 0.0;
    else v = (i == t) ? 1.0 : 0.0;
    Ls[i][t] = v;
  }
  __syncthreads();
  double x[64];
  const double* L0 = &Ls[0][0];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    // Row i is read in groups of 16 entries, each group only after the
    // previous one is in use (and row i only after x[i-1] exists): the
    // column of x already takes 128 registers, and reading the whole
    // triangle ahead would spill.  The empty asm statements only make an
    // offset depend on an earlier result.
    int off = i * 64;
    if (i > 0) asm volatile("" : "+v"(off) : "v"(x[i - 1]));
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (16 * g >= i) break;
      int goff = off + 16 * g;
      if (g > 0) asm volatile("" : "+v"(goff) : "v"(s4[3]));
      const double* Lr = L0 + goff;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int p = 16 * g + e;
        if (p < i) s4[p & 3] = fma(Lr[e], x[p], s4[p & 3]);
      }
    }
    const double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    x[i] = ((i == t ? 1.0 : 0.0) - s) / Ls[i][i];
  }
#pragma unroll
  for (int i = 0; i < 64; ++i)
    if (i < nb && t < nb && t <= i) P[(int64_t)i * n0 + t] = x[i];
}

__global__ __launch_bounds__(256) void zero_upper_kernel(double* __restrict__ Linv, int64_t n0) {
  // one row of one packed block per workgroup: its columns past the diagonal
  const int64_t row = blockIdx.x;
  const int64_t i = row % n0;
  double* __restrict__ out = Linv + row * n0;
  for (int64_t j = i + 1 + threadIdx.x; j < n0; j += blockDim.x) out[j] = 0.0;
}

template <typename TI, typename TO>
__global__ void convert_kernel(const TI* __restrict__ in, TO* __restrict__ out, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = cvt<TO>(in[i]);
}

template <typename TI, typename TO>
__global__ void copy2d_kernel(const TI* __restrict__ in, int64_t ldi, TO* __restrict__ out,
                              int64_t ldo, int64_t rows, int64_t cols, double scale) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i % cols;
    out[r * ldo + c] = cvt<TO>(static_cast<double>(in[r * ldi + c]) * scale);
  }
}

__global__ void axpy_kernel(const float* __restrict__ D, int64_t ldd, double* __restrict__ X,
                            int64_t ldx, int64_t rows, int64_t cols, double scale, int assign) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i % cols;
    const double d = scale * static_cast<double>(D[r * ldd + c]);
    if (assign) X[r * ldx + c] = d;
    else X[r * ldx + c] += d;
  }
}

// One wave per (row r, column block c).  Waves for c >= floor(r / n0) (the
// diagonal block and beyond) only write a unit scale.
template <typename TO>
__global__ __launch_bounds__(256) void lowcopy_kernel(const double* __restrict__ L, int64_t ldl,
                                                      int64_t n, int64_t n0, int64_t m,
                                                      TO* __restrict__ Llow,
                                                      float* __restrict__ rscale, float target) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wid >= n * m) return;
  const int64_t r = wid / m, c = wid % m;
  if (c >= r / n0) {
    if (lane == 0) rscale[r * m + c] = 1.0f;
    return;
  }
  const double* src = L + r * ldl + c * n0;
  double mx = 0.0;
  for (int64_t j = lane; j < n0; j += 64) mx = fmax(mx, fabs(src[j]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  int e = 0;
  if (mx > 0.0) e = ilogb((double)target) - ilogb(mx) - 1;
  TO* dst = Llow + r * n + c * n0;
  for (int64_t j = lane; j < n0; j += 64) dst[j] = cvt<TO>(ldexp(src[j], e));
  if (lane == 0) rscale[r * m + c] = ldexpf(1.0f, -e);
}

// out[r * cols + c] = low(a[r * cols + c] 2^e_r) with one power-of-two scale
// per row (its largest magnitude placed just below `target`) and
// rs[r] = 2^-e_r; one wave per row.
template <typename TO>
__global__ __launch_bounds__(256) void rowscale_copy_kernel(const double* __restrict__ a,
                                                            int64_t rows, int64_t cols,
                                                            TO* __restrict__ out,
                                                            float* __restrict__ rs, float target) {
  const int lane = threadIdx.x & 63;
  const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (r >= rows) return;
  const double* src = a + r * cols;
  double mx = 0.0;
  for (int64_t j = lane; j < cols; j += 64) mx = fmax(mx, fabs(src[j]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  int e = 0;
  if (mx > 0.0) e = ilogb((double)target) - ilogb(mx) - 1;
  for (int64_t j = lane; j < cols; j += 64) out[r * cols + j] = cvt<TO>(ldexp(src[j], e));
  if (lane == 0) rs[r] = ldexpf(1.0f, -e);
}

// Largest |D| over a rows x cols block as float bits: the bit patterns of
// non-negative floats order like their values (and a NaN orders above
// infinity, so it is not lost).  out[0] must start at zero.
__global__ __launch_bounds__(256) void absmax_bits_kernel(const float* __restrict__ D, int64_t ldd,
                                                          int64_t rows, int64_t cols,
                                                          unsigned* __restrict__ out) {
  __shared__ unsigned wmax[4];
  unsigned mx = 0;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
    for (int64_t c = threadIdx.x; c < cols; c += blockDim.x)
      mx = max(mx, __float_as_uint(D[r * ldd + c]) & 0x7FFFFFFFu);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (unsigned)__shfl_xor((int)mx, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    if (mx) atomicMax(out, mx);
  }
}

__global__ void fill_u32_kernel(unsigned* __restrict__ p, int64_t count, unsigned v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// XT[c * ldx + r] = low(2^e * D[r * ldd + c]) with 2^e putting the block's
// largest magnitude in [2^etarget, 2^(etarget+1)); *xinv = 2^-e.  64 x 64
// tiles transposed through LDS.
template <typename TO>
__global__ __launch_bounds__(256) void lowx_kernel(const float* __restrict__ D, int64_t ldd,
                                                   int64_t rows, int64_t cols, TO* __restrict__ XT,
                                                   int64_t ldx, const unsigned* __restrict__ amax,
                                                   float* __restrict__ xinv, int etarget) {
  __shared__ float tile[64][65];
  const float mx = __uint_as_float(*amax);
  int e = 0;
  if (mx > 0.0f && isfinite(mx)) e = etarget - ilogbf(mx);
  if (blockIdx.x == 0 && threadIdx.x == 0) *xinv = ldexpf(1.0f, -e);
  const int64_t ntc = (cols + 63) / 64;
  const int64_t tr = (blockIdx.x / ntc) * 64, tc = (blockIdx.x % ntc) * 64;
  const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
#pragma unroll 4
  for (int j = 0; j < 16; ++j) {
    const int64_t r = tr + hi + 4 * j, c = tc + lo;
    tile[hi + 4 * j][lo] = (r < rows && c < cols) ? D[r * ldd + c] : 0.0f;
  }
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < 16; ++j) {
    const int64_t c = tc + hi + 4 * j, r = tr + lo;
    if (r < rows && c < cols) XT[c * ldx + r] = cvt<TO>(ldexpf(tile[lo][hi + 4 * j], e));
  }
}

// Uniform in [0, 1) from a 64-bit counter (splitmix64 finaliser).
__device__ inline double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

template <typename T>
__global__ void fill_system_kernel(T* __restrict__ L, int64_t n, T* __restrict__ B, int64_t k,
                                   uint64_t seed) {
  const int64_t tl = n * n, total = tl + n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double u = hash_unit(seed * 0x100000001B3ull + (uint64_t)e);
    if (e < tl) {
      const int64_t i = e / n, j = e - i * n;
      L[e] = (T)(j == i ? 1.0 + u : (j < i ? (2.0 * u - 1.0) / (double)n : 0.0));
    } else {
      B[e - tl] = (T)(u - 0.5);
    }
  }
}

// 64 x 64 tiles transposed through LDS; one workgroup per (matrix, tile).
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void transpose_kernel(const TI* __restrict__ in, int64_t ldi,
                                                        TO* __restrict__ out, int64_t ldo,
                                                        int64_t rows, int64_t cols, int64_t si,
                                                        int64_t so, int64_t tiles_per,
                                                        bool lower_only) {
  __shared__ TO tile[64][65];
  const int64_t b = blockIdx.x / tiles_per, t = blockIdx.x % tiles_per;
  const int64_t ntc = (cols + 63) / 64;
  const int64_t tr = (t / ntc) * 64, tc = (t % ntc) * 64;
  const TI* src = in + b * si;
  TO* dst = out + b * so;
  const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
#pragma unroll 4
  for (int j = 0; j < 16; ++j) {
    const int64_t r = tr + hi + 4 * j, c = tc + lo;
    TO v = TO(0);
    if (r < rows && c < cols && !(lower_only && r < c)) v = (TO)src[r * ldi + c];
    tile[hi + 4 * j][lo] = v;
  }
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < 16; ++j) {
    const int64_t c = tc + hi + 4 * j, r = tr + lo;
    if (r < rows && c < cols) dst[c * ldo + r] = tile[lo][hi + 4 * j];
  }
}

// Recursive baseline leaf: forward substitution, one thread per column.
template <typename T>
__global__ __launch_bounds__(64) void subst_leaf_kernel(const T* __restrict__ L, int64_t ldl,
                                                        T* __restrict__ X, int64_t ldx,
                                                        int64_t nb, int64_t k) {
  __shared__ T Ls[64][65];
  __shared__ T Xs[64][65];
  const int t = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * 64 + t;
  for (int i = 0; i < nb; ++i) Ls[i][t] = (t < nb && t <= i) ? L[(int64_t)i * ldl + t] : T(0);
  __syncthreads();
  if (c < k) {
    for (int i = 0; i < nb; ++i) {
      T s = X[(int64_t)i * ldx + c];
      for (int p = 0; p < i; ++p) s -= Ls[i][p] * Xs[p][t];
      const T x = s / Ls[i][i];
      Xs[i][t] = x;
      X[(int64_t)i * ldx + c] = x;
    }
  }
}

// Deterministic reductions: a fixed grid of kNormBlocks blocks; block b takes
// rows b, b + kNormBlocks, ... in order and thread t of it the columns t,
// t + 256, ... of each row (whole rows per block: coalesced, no index
// division), then a fixed-shape reduction: butterflies inside each wavefront
// and a fixed sum of the four wavefronts' results.
__device__ inline void block_reduce2(double& s, double& mx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  __shared__ double ws[4], wm[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    ws[w] = s;
    wm[w] = mx;
  }
  __syncthreads();
  s = (ws[0] + ws[1]) + (ws[2] + ws[3]);
  mx = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
}

__global__ __launch_bounds__(256) void sumsq_max_part(const double* __restrict__ A, int64_t lda,
                                                      int64_t rows, int64_t cols,
                                                      double* __restrict__ part) {
  double s = 0.0, mx = 0.0;
  for (int64_t r = blockIdx.x; r < rows; r += kNormBlocks) {
    const double* __restrict__ a = A + r * lda;
    for (int64_t c = threadIdx.x; c < cols; c += 256) {
      const double v = a[c];
      s += v * v;
      mx = fmax(mx, fabs(v));
    }
  }
  block_reduce2(s, mx);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[kNormBlocks + blockIdx.x] = mx;
  }
}

template <typename TL>
__global__ __launch_bounds__(256) void sumsq_lower_part(const TL* __restrict__ L, int64_t ldl,
                                                        int64_t n, double* __restrict__ part) {
  double s = 0.0, mx = 0.0;
  for (int64_t r = blockIdx.x; r < n; r += kNormBlocks) {
    const TL* __restrict__ l = L + r * ldl;
    for (int64_t c = threadIdx.x; c <= r; c += 256) {
      const double v = static_cast<double>(l[c]);
      s += v * v;
      mx = fmax(mx, fabs(v));
    }
  }
  block_reduce2(s, mx);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[kNormBlocks + blockIdx.x] = mx;
  }
}

__global__ __launch_bounds__(256) void reduce_final(const double* __restrict__ part,
                                                    double* __restrict__ out) {
  double s = 0.0, mx = 0.0;
  for (int i = threadIdx.x; i < kNormBlocks; i += 256) {
    s += part[i];
    mx = fmax(mx, part[kNormBlocks + i]);
  }
  block_reduce2(s, mx);
  if (threadIdx.x == 0) {
    out[0] = s;
    out[1] = mx;
  }
}

}  // namespace

template <typename TL>
hipError_t launch_extract_diag(const TL* L, int64_t ldl, int64_t n, int64_t n0, int64_t m,
                               double* Linv, unsigned long long* bad, hipStream_t s, bool upper) {
  if (m <= 0) return hipSuccess;
  extract_diag_kernel<TL><<<(unsigned)(m * n0), row_threads(n0), 0, s>>>(L, ldl, n, n0, Linv, bad,
                                                                         upper);
  return hipGetLastError();
}
template hipError_t launch_extract_diag<double>(const double*, int64_t, int64_t, int64_t, int64_t,
                                                double*, unsigned long long*, hipStream_t, bool);
template hipError_t launch_extract_diag<float>(const float*, int64_t, int64_t, int64_t, int64_t,
                                               double*, unsigned long long*, hipStream_t, bool);

hipError_t launch_trtri_leaf(double* Linv, int64_t n0, int64_t m, int64_t nb, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t lpb = n0 / nb;
  trtri_leaf_kernel<<<(unsigned)(m * lpb), 64, 0, s>>>(Linv, n0, nb, lpb);
  return hipGetLastError();
}

hipError_t launch_zero_upper(double* Linv, int64_t n0, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  zero_upper_kernel<<<(unsigned)(m * n0), row_threads(n0), 0, s>>>(Linv, n0);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_convert(const TI* in, TO* out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  convert_kernel<TI, TO><<<grid_for(count, 256), 256, 0, s>>>(in, out, count);
  return hipGetLastError();
}
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);

template <typename TI, typename TO>
hipError_t launch_copy2d(const TI* in, int64_t ldi, TO* out, int64_t ldo, int64_t rows,
                         int64_t cols, double scale, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  copy2d_kernel<TI, TO><<<grid_for(rows * cols, 256), 256, 0, s>>>(in, ldi, out, ldo, rows, cols,
                                                                   scale);
  return hipGetLastError();
}
template hipError_t launch_copy2d<double, double>(const double*, int64_t, double*, int64_t,
                                                  int64_t, int64_t, double, hipStream_t);
template hipError_t launch_copy2d<float, float>(const float*, int64_t, float*, int64_t, int64_t,
                                                int64_t, double, hipStream_t);
template hipError_t launch_copy2d<double, float>(const double*, int64_t, float*, int64_t, int64_t,
                                                 int64_t, double, hipStream_t);
template hipError_t launch_copy2d<float, double>(const float*, int64_t, double*, int64_t, int64_t,
                                                 int64_t, double, hipStream_t);

hipError_t launch_axpy_f32_to_f64(const float* D, int64_t ldd, double* X, int64_t ldx,
                                  int64_t rows, int64_t cols, double scale, bool assign,
                                  hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  axpy_kernel<<<grid_for(rows * cols, 256), 256, 0, s>>>(D, ldd, X, ldx, rows, cols, scale,
                                                         assign ? 1 : 0);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_lowcopy(const double* L, int64_t ldl, int64_t n, int64_t n0, int64_t m,
                          TO* Llow, float* rscale, float target, hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  const int64_t waves = n * m;
  lowcopy_kernel<TO><<<grid_for(waves * 64, 256, INT64_MAX), 256, 0, s>>>(L, ldl, n, n0, m, Llow,
                                                                          rscale, target);
  return hipGetLastError();
}
template <typename TO>
hipError_t launch_rowscale_copy(const double* a, int64_t rows, int64_t cols, TO* out, float* rs,
                               float target, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  rowscale_copy_kernel<TO><<<grid_for(rows * 64, 256, INT64_MAX), 256, 0, s>>>(a, rows, cols, out,
                                                                              rs, target);
  return hipGetLastError();
}
template hipError_t launch_rowscale_copy<bf16_t>(const double*, int64_t, int64_t, bf16_t*, float*,
                                                 float, hipStream_t);
template hipError_t launch_rowscale_copy<f16_t>(const double*, int64_t, int64_t, f16_t*, float*,
                                                float, hipStream_t);

template hipError_t launch_lowcopy<bf16_t>(const double*, int64_t, int64_t, int64_t, int64_t,
                                           bf16_t*, float*, float, hipStream_t);
template hipError_t launch_lowcopy<f16_t>(const double*, int64_t, int64_t, int64_t, int64_t,
                                          f16_t*, float*, float, hipStream_t);
template hipError_t launch_lowcopy<fp8_t>(const double*, int64_t, int64_t, int64_t, int64_t,
                                          fp8_t*, float*, float, hipStream_t);

hipError_t launch_fill_u32(unsigned* p, int64_t count, unsigned v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_u32_kernel<<<(unsigned)ceil_div(count, 256), 256, 0, s>>>(p, count, v);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_lowx(const float* D, int64_t ldd, int64_t rows, int64_t cols, TO* XT,
                       int64_t ldx, unsigned* amax, float* xinv, int etarget, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  absmax_bits_kernel<<<(unsigned)std::min<int64_t>(rows, 2048), 256, 0, s>>>(D, ldd, rows, cols, amax);
  const int64_t tiles = ceil_div(rows, 64) * ceil_div(cols, 64);
  lowx_kernel<TO><<<(unsigned)tiles, 256, 0, s>>>(D, ldd, rows, cols, XT, ldx, amax, xinv, etarget);
  return hipGetLastError();
}
template hipError_t launch_lowx<bf16_t>(const float*, int64_t, int64_t, int64_t, bf16_t*, int64_t,
                                        unsigned*, float*, int, hipStream_t);
template hipError_t launch_lowx<f16_t>(const float*, int64_t, int64_t, int64_t, f16_t*, int64_t,
                                       unsigned*, float*, int, hipStream_t);
template hipError_t launch_lowx<fp8_t>(const float*, int64_t, int64_t, int64_t, fp8_t*, int64_t,
                                       unsigned*, float*, int, hipStream_t);

template <typename T>
hipError_t launch_fill_system(T* L, int64_t n, T* B, int64_t k, uint64_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_system_kernel<T><<<grid_for(n * n + n * k, 256, 16384), 256, 0, s>>>(L, n, B, k, seed);
  return hipGetLastError();
}
template hipError_t launch_fill_system<double>(double*, int64_t, double*, int64_t, uint64_t,
                                               hipStream_t);
template hipError_t launch_fill_system<float>(float*, int64_t, float*, int64_t, uint64_t,
                                              hipStream_t);

template <typename TI, typename TO>
hipError_t launch_transpose(const TI* in, int64_t ldi, TO* out, int64_t ldo, int64_t rows,
                            int64_t cols, int64_t batch, int64_t si, int64_t so, bool lower_only,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
  const int64_t per = ceil_div(rows, 64) * ceil_div(cols, 64);
  transpose_kernel<TI, TO><<<(unsigned)(per * batch), 256, 0, s>>>(in, ldi, out, ldo, rows, cols,
                                                                   si, so, per, lower_only);
  return hipGetLastError();
}
template hipError_t launch_transpose<double, double>(const double*, int64_t, double*, int64_t,
                                                     int64_t, int64_t, int64_t, int64_t, int64_t,
                                                     bool, hipStream_t);
template hipError_t launch_transpose<float, float>(const float*, int64_t, float*, int64_t, int64_t,
                                                   int64_t, int64_t, int64_t, int64_t, bool,
                                                   hipStream_t);

template <typename T>
hipError_t launch_subst_leaf(const T* L, int64_t ldl, T* X, int64_t ldx, int64_t nb, int64_t k,
                             hipStream_t s) {
  if (nb <= 0 || k <= 0) return hipSuccess;
  subst_leaf_kernel<T><<<(unsigned)ceil_div(k, 64), 64, 0, s>>>(L, ldl, X, ldx, nb, k);
  return hipGetLastError();
}
template hipError_t launch_subst_leaf<double>(const double*, int64_t, double*, int64_t, int64_t,
                                              int64_t, hipStream_t);
template hipError_t launch_subst_leaf<float>(const float*, int64_t, float*, int64_t, int64_t,
                                             int64_t, hipStream_t);

hipError_t launch_sumsq_max(const double* A, int64_t lda, int64_t rows, int64_t cols,
                            double* part, double* out, hipStream_t s) {
  sumsq_max_part<<<kNormBlocks, 256, 0, s>>>(A, lda, rows, cols, part);
  reduce_final<<<1, 256, 0, s>>>(part, out);
  return hipGetLastError();
}

template <typename TL>
hipError_t launch_sumsq_lower(const TL* L, int64_t ldl, int64_t n, double* part, double* out,
                              hipStream_t s) {
  sumsq_lower_part<TL><<<kNormBlocks, 256, 0, s>>>(L, ldl, n, part);
  reduce_final<<<1, 256, 0, s>>>(part, out);
  return hipGetLastError();
}
template hipError_t launch_sumsq_lower<double>(const double*, int64_t, int64_t, double*, double*,
                                               hipStream_t);
template hipError_t launch_sumsq_lower<float>(const float*, int64_t, int64_t, double*, double*,
                                              hipStream_t);

}  // namespace trsm
