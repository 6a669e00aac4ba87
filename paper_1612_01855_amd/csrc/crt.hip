// Residue-number-system kernels of the refinement residual (see crt.hpp).
#include "crt.hpp"

#include <algorithm>
#include <cmath>

namespace trsm {
namespace crt {

namespace {

typedef unsigned __int128 u128;

int modinv(int a, int m) {
  // extended Euclid: a * x = 1 (mod m), gcd(a, m) = 1
  long t = 0, nt = 1, r = m, nr = a % m;
  while (nr != 0) {
    const long q = r / nr;
    long tmp = t - q * nt; t = nt; nt = tmp;
    tmp = r - q * nr; r = nr; nr = tmp;
  }
  return (int)(t < 0 ? t + m : t);
}

double u128_to_double(u128 v) {
  const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
  return std::ldexp((double)hi, 64) + (double)lo;
}

// x mod m in the symmetric range of a signed byte, for an integer-valued
// binary64 |x| <= 2^53: the quotient is off by at most one, and
// x - q m is exact.
__device__ __forceinline__ int sym_mod_d(double x, int m, double inv_m) {
  const double q = floor(x * inv_m);
  double r = fma(-q, (double)m, x);
  r = r < 0.0 ? r + m : r;
  r = r >= (double)m ? r - m : r;
  const int ri = (int)r;
  return ri > (m - 1) / 2 ? ri - m : ri;
}

// x mod m in the symmetric range of a signed byte, for |x| < 2^30: the
// binary32 quotient is off by at most one.
__device__ __forceinline__ int sym_mod_i(int x, int m, float inv_m) {
  const int q = (int)rintf((float)x * inv_m);
  int r = x - q * m;
  r = r < 0 ? r + m : r;
  r = r >= m ? r - m : r;
  return r > (m - 1) / 2 ? r - m : r;
}

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// rowmax[i] = max_{j<i} |l_ij|; one 256-thread block per row.
__global__ __launch_bounds__(256) void row_max_kernel(const double* __restrict__ L, int64_t ldl,
                                                       int64_t n, double* __restrict__ rowmax,
                                                       double* __restrict__ contrib) {
  const int64_t i = blockIdx.x;
  const double* li = L + i * ldl;
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < i; j += 256) m = fmax(m, fabs(li[j]));
  m = warp_max(m);
  __shared__ double sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double r = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
    rowmax[i] = r;
    contrib[i] = (double)i * r * r;
  }
}

// Fixed-order sum of v[0..count) by one block: out[0] = sum.
__global__ __launch_bounds__(1024) void sum_fixed_kernel(const double* __restrict__ v,
                                                          int64_t count, double* __restrict__ out) {
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < count; e += 1024) s += v[e];
  s = warp_sum(s);
  __shared__ double sm[16];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sm[w];
    out[0] = t;
  }
}

__global__ void choose_bits_kernel(const double* stats, const double* lnorm2, double target,
                                   int* a_out) {
  const double s = stats[0], l = lnorm2[0];
  int a = 24;
  if (s > 0.0 && l > 0.0) a = (int)ceil(target + 0.5 * log2(s / l));
  a_out[0] = a < 24 ? 24 : (a > 50 ? 50 : a);
}

// Eight consecutive columns of one row per thread, all P planes.
__global__ __launch_bounds__(256) void l_residues_kernel(const double* __restrict__ L, int64_t ldl,
                                                          int64_t n, const double* __restrict__ rowmax,
                                                          const int* __restrict__ a_dev, Table t,
                                                          int8_t* __restrict__ planes, int64_t lde,
                                                          int64_t plane, int* __restrict__ sl) {
  const int64_t i = blockIdx.y;
  const int64_t j0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
  const int64_t jend = min(lde, ((i + 256) / 256) * 256);
  if (j0 >= jend) return;
  int s = 0;
  if (i < n) {
    const double rm = rowmax[i];
    s = rm > 0.0 ? a_dev[0] - 1 - ilogb(rm) : 0;
  }
  if (j0 == 0) sl[i] = s;
  double v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t j = j0 + e;
    v[e] = (i < n && j < i) ? rint(ldexp(L[i * ldl + j], s)) : 0.0;
  }
#pragma unroll
  for (int p = 0; p < kPlanes; ++p) {
    if (p >= t.P) break;
    const int m = t.mod[p];
    const double inv = t.invd[p];
    uint64_t packed = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      packed |= (uint64_t)(uint8_t)(int8_t)sym_mod_d(v[e], m, inv) << (8 * e);
    *reinterpret_cast<uint64_t*>(planes + p * plane + i * lde + j0) = packed;
  }
}

// Block (x, y) takes the 64-column strip x and the rows of slab y (four row
// groups of 64 threads, rows y, y + 4 S, ... for group 0): column maxima by
// atomic max (order-independent), one partial sum of squares per block in a
// fixed order.
template <typename TY>
__global__ __launch_bounds__(256) void dstats_kernel(const TY* __restrict__ Y, int64_t ldy,
                                                      int64_t n, int64_t k,
                                                      unsigned* __restrict__ colmax,
                                                      double* __restrict__ part) {
  __shared__ float smax[4][64];
  __shared__ double ssum[4];
  const int cl = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + cl;
  const int64_t stride = 4 * (int64_t)gridDim.y;
  double ss = 0.0;
  float m = 0.0f;
  if (c < k) {
    int64_t i = (int64_t)blockIdx.y * 4 + rg;
    for (; i + 3 * stride < n; i += 4 * stride) {
      double a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = fabs((double)Y[(i + u * stride) * ldy + c]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ss += a[u] * a[u];
        m = fmaxf(m, (float)a[u]);
      }
    }
    for (; i < n; i += stride) {
      const double a = fabs((double)Y[i * ldy + c]);
      ss += a * a;
      m = fmaxf(m, (float)a);
    }
  }
  // binary32 rounds to nearest: the next float up bounds every magnitude
  smax[rg][cl] = m > 0.0f ? nextafterf(m, INFINITY) : 0.0f;
  __syncthreads();
  if (rg == 0 && c < k) {
    const float mm = fmaxf(fmaxf(smax[0][cl], smax[1][cl]), fmaxf(smax[2][cl], smax[3][cl]));
    if (mm > 0.0f) atomicMax(colmax + c, __float_as_uint(mm));
  }
  ss = warp_sum(ss);
  if (cl == 0) ssum[rg] = ss;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ssum[0] + ssum[1] + ssum[2] + ssum[3];
}

__device__ __forceinline__ int col_shift(unsigned bits, int b) {
  const float m = __uint_as_float(bits);
  return m > 0.0f ? b - 1 - ilogbf(m) : 0;
}

// 64 x 64 tile of Y per block: thread (column cl, row group g) rounds rows
// 16 g .. 16 g + 15 of its column to integers, writes the exact binary32 value
// of the rounded piece (Yq = q 2^-t) back, and stores the residues of four
// rows as one 32-bit word in LDS; the words then leave as 16-byte pieces of
// the transposed planes (row c of a plane holds column c of Y).
__global__ __launch_bounds__(256) void y_residues_kernel(float* __restrict__ Y, int64_t ldy,
                                                          int64_t n, int64_t k,
                                                          const unsigned* __restrict__ colmax,
                                                          int b, Table t,
                                                          int8_t* __restrict__ planes, int64_t ldq,
                                                          int64_t plane, int* __restrict__ ty) {
  __shared__ uint32_t tile[kPlanes][64][17];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int cl = tid & 63, g = tid >> 6;
  const int64_t c = c0 + cl;
  const int sh = c < k ? col_shift(colmax[c], b) : 0;
  if (blockIdx.y == 0 && g == 0 && c < k) ty[c] = sh;
  int q[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + 16 * g + r;
    q[r] = (i < n && c < k) ? (int)rintf(ldexpf(Y[i * ldy + c], sh)) : 0;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + 16 * g + r;
    if (i < n && c < k) Y[i * ldy + c] = ldexpf((float)q[r], -sh);
  }
#pragma unroll
  for (int p = 0; p < kPlanes; ++p) {
    if (p >= t.P) break;
    const int m = t.mod[p];
    const float inv = t.inv[p];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t word = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        word |= (uint32_t)(uint8_t)(int8_t)sym_mod_i(q[4 * w + e], m, inv) << (8 * e);
      tile[p][cl][4 * g + w] = word;
    }
  }
  __syncthreads();
  // thread -> column row (tid >> 2) of the tile, 16 bytes (4 words) each
  const int crow = tid >> 2, part = tid & 3;
  if (c0 + crow < k) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) {
      if (p >= t.P) break;
      u4 o = {tile[p][crow][4 * part], tile[p][crow][4 * part + 1], tile[p][crow][4 * part + 2],
              tile[p][crow][4 * part + 3]};
      *reinterpret_cast<u4*>(planes + p * plane + (c0 + crow) * ldq + i0 + 16 * part) = o;
    }
  }
}

// X = sum_p Yp 2^shift_p (binary64) for up to three binary32 pieces.
__global__ __launch_bounds__(256) void assemble_kernel(const float* __restrict__ Y0, int s0,
                                                        const float* __restrict__ Y1, int s1,
                                                        const float* __restrict__ Y2, int s2,
                                                        int64_t ldy, double* __restrict__ X,
                                                        int64_t ldx, int64_t n, int64_t k,
                                                        bool accumulate) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x)
    for (int64_t c = threadIdx.x; c < k; c += 256) {
      double v = accumulate ? X[i * ldx + c] : 0.0;
      v += ldexp((double)Y0[i * ldy + c], s0);
      if (Y1) v += ldexp((double)Y1[i * ldy + c], s1);
      if (Y2) v += ldexp((double)Y2[i * ldy + c], s2);
      X[i * ldx + c] = v;
    }
}

// One block per row (rows blockIdx.x, blockIdx.x + gridDim.x, ...), threads
// over columns: fixed partition, so the partial norms are deterministic.
__global__ __launch_bounds__(256) void recombine_kernel(
    const int8_t* __restrict__ Z, int64_t ldz, int64_t zplane, Table t,
    const int* __restrict__ sl, const int* __restrict__ ty, const float* __restrict__ Yq, int64_t ldy,
    int yshift, const double* __restrict__ L, int64_t ldl, const double* Rin, int64_t ldri, double* Rout,
    int64_t ldro, float* __restrict__ Rl, double* __restrict__ X, int64_t ldx, int xmode,
    int64_t n, int64_t k, double* __restrict__ part) {
  double r2 = 0.0, rmax = 0.0, x2 = 0.0, xmax = 0.0;
  const double two24 = 16777216.0, inv24 = 1.0 / 16777216.0;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const double lii = L[i * ldl + i];
    const int si = sl[i];
    for (int64_t c0 = 4 * (int64_t)threadIdx.x; c0 < k; c0 += 1024) {
      const int nc = (int)min<int64_t>(4, k - c0);
      // all loads of the four columns first
      uint32_t zw[kPlanes];
      const int8_t* zp = Z + i * ldz + c0;
#pragma unroll
      for (int p = 0; p < kPlanes; ++p) {
        zw[p] = 0;
        if (p < t.P) {
          if (nc == 4) {
            zw[p] = *reinterpret_cast<const uint32_t*>(zp + p * zplane);
          } else {
            for (int e = 0; e < nc; ++e) zw[p] |= (uint32_t)(uint8_t)zp[p * zplane + e] << (8 * e);
          }
        }
      }
      float yv[4];
      double rin[4], rout[4];
      int tcv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        yv[e] = e < nc ? Yq[i * ldy + c0 + e] : 0.0f;
        rin[e] = e < nc ? Rin[i * ldri + c0 + e] : 0.0;
        tcv[e] = e < nc ? ty[c0 + e] : 0;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (e >= nc) break;
        const int64_t c = c0 + e;
        // S = sum_p z_p W_p in four 24-bit limbs, each an exact binary64 integer
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) {
          if (p >= t.P) break;
          const double z = (double)(int8_t)((zw[p] >> (8 * e)) & 0xFF);
          a0 = fma(z, t.Wd[p][0], a0);
          a1 = fma(z, t.Wd[p][1], a1);
          a2 = fma(z, t.Wd[p][2], a2);
          a3 = fma(z, t.Wd[p][3], a3);
        }
        const double Sd = fma(fma(fma(a3, two24, a2), two24, a1), two24, a0);
        // C = S - q M, |C| < M / 4: q is the nearest integer to S / M
        const double q = rint(Sd * t.inv_Md);
        double d0 = fma(-q, t.Md4[0], a0), d1 = fma(-q, t.Md4[1], a1);
        double d2 = fma(-q, t.Md4[2], a2), d3 = fma(-q, t.Md4[3], a3);
        double cr = floor(d0 * inv24);
        d0 = fma(-cr, two24, d0);
        d1 += cr;
        cr = floor(d1 * inv24);
        d1 = fma(-cr, two24, d1);
        d2 += cr;
        cr = floor(d2 * inv24);
        d2 = fma(-cr, two24, d2);
        d3 += cr;
        const double Cv = fma(fma(fma(d3, two24, d2), two24, d1), two24, d0);
        const double yq = ldexp((double)yv[e], yshift);
        const double r = rin[e] - lii * yq - ldexp(Cv, yshift - si - tcv[e]);
        rout[e] = r;
        r2 += r * r;
        rmax = fmax(rmax, fabs(r));
        if (xmode) {
          const double xn = xmode == 1 ? yq : X[i * ldx + c] + yq;
          X[i * ldx + c] = xn;
          x2 += xn * xn;
          xmax = fmax(xmax, fabs(xn));
        }
      }
      if (nc == 4 && k % 4 == 0 && ldro % 2 == 0 && (((uintptr_t)Rout | (uintptr_t)Rl) & 15) == 0) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        typedef float f4v __attribute__((ext_vector_type(4)));
        *reinterpret_cast<d2v*>(Rout + i * ldro + c0) = d2v{rout[0], rout[1]};
        *reinterpret_cast<d2v*>(Rout + i * ldro + c0 + 2) = d2v{rout[2], rout[3]};
        *reinterpret_cast<f4v*>(Rl + i * k + c0) =
            f4v{(float)rout[0], (float)rout[1], (float)rout[2], (float)rout[3]};
      } else {
        for (int e = 0; e < nc; ++e) {
          Rout[i * ldro + c0 + e] = rout[e];
          Rl[i * k + c0 + e] = (float)rout[e];
        }
      }
    }
  }
  r2 = warp_sum(r2);
  x2 = warp_sum(x2);
  rmax = warp_max(rmax);
  xmax = warp_max(xmax);
  __shared__ double sm[4][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w][0] = r2;
    sm[w][1] = rmax;
    sm[w][2] = x2;
    sm[w][3] = xmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + 4 * (int64_t)blockIdx.x;
    o[0] = sm[0][0] + sm[1][0] + sm[2][0] + sm[3][0];
    o[1] = fmax(fmax(sm[0][1], sm[1][1]), fmax(sm[2][1], sm[3][1]));
    o[2] = sm[0][2] + sm[1][2] + sm[2][2] + sm[3][2];
    o[3] = fmax(fmax(sm[0][3], sm[1][3]), fmax(sm[2][3], sm[3][3]));
  }
}

__global__ __launch_bounds__(64) void recombine_final_kernel(const double* __restrict__ part,
                                                              int blocks, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double r2 = 0.0, rmax = 0.0, x2 = 0.0, xmax = 0.0;
  for (int b = 0; b < blocks; ++b) {
    r2 += part[4 * b];
    rmax = fmax(rmax, part[4 * b + 1]);
    x2 += part[4 * b + 2];
    xmax = fmax(xmax, part[4 * b + 3]);
  }
  out[0] = r2;
  out[1] = rmax;
  out[2] = x2;
  out[3] = xmax;
}

}  // namespace

Table make_table(int P) {
  Table t{};
  t.P = P;
  u128 M = 1;
  for (int p = 0; p < P; ++p) {
    t.mod[p] = kModuli[p];
    M *= (u128)kModuli[p];
  }
  const u128 mask = ((u128)1 << 24) - 1;
  for (int p = 0; p < P; ++p) {
    const int m = kModuli[p];
    const u128 Mp = M / (u128)m;
    const int inv = modinv((int)(Mp % (u128)m), m);
    const u128 W = (Mp * (u128)inv) % M;
    t.inv[p] = 1.0f / (float)m;
    t.invd[p] = 1.0 / (double)m;
    for (int l = 0; l < 4; ++l) t.Wd[p][l] = (double)(uint64_t)((W >> (24 * l)) & mask);
  }
  for (int l = 0; l < 4; ++l) t.Md4[l] = (double)(uint64_t)((M >> (24 * l)) & mask);
  t.Md = u128_to_double(M);
  t.inv_Md = 1.0 / t.Md;
  t.log2M = std::log2(t.Md);
  return t;
}

int moduli_for_bits(double bits) {
  double l = 0.0;
  for (int p = 0; p < 12; ++p) {
    l += std::log2((double)kModuli[p]);
    if (l >= bits) return p + 1;
  }
  return -1;
}

hipError_t launch_row_stats(const double* L, int64_t ldl, int64_t n, double* rowmax, double* part,
                            double* stats, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  row_max_kernel<<<(unsigned)n, 256, 0, s>>>(L, ldl, n, rowmax, part);
  sum_fixed_kernel<<<1, 1024, 0, s>>>(part, n, stats);
  return hipGetLastError();
}

hipError_t launch_choose_bits(const double* stats, const double* lnorm2, double target_bits,
                              int* a_out, hipStream_t s) {
  choose_bits_kernel<<<1, 1, 0, s>>>(stats, lnorm2, target_bits, a_out);
  return hipGetLastError();
}

hipError_t launch_l_residues(const double* L, int64_t ldl, int64_t n, int64_t npad,
                             const double* rowmax, const int* a_dev, const Table& t,
                             int8_t* planes, int64_t lde, int64_t plane, int* sl, hipStream_t s) {
  if (npad <= 0) return hipSuccess;
  dim3 grid((unsigned)((lde + 2047) / 2048), (unsigned)npad);
  l_residues_kernel<<<grid, 256, 0, s>>>(L, ldl, n, rowmax, a_dev, t, planes, lde, plane, sl);
  return hipGetLastError();
}

template <typename TY>
hipError_t launch_dstats(const TY* Y, int64_t ldy, int64_t n, int64_t k, unsigned* colmax,
                         double* part, double* out, hipStream_t s) {
  const int64_t strips = (k + 63) / 64;
  if (strips <= 0 || n <= 0) return hipSuccess;
  if (strips > kRecBlocks) return hipErrorInvalidValue;
  dstats_kernel<TY><<<dim3((unsigned)strips, kStatSlabs), 256, 0, s>>>(Y, ldy, n, k, colmax, part);
  sum_fixed_kernel<<<1, 1024, 0, s>>>(part, strips * kStatSlabs, out);
  return hipGetLastError();
}

hipError_t launch_y_residues(float* Y, int64_t ldy, int64_t n, int64_t npad, int64_t k,
                             const unsigned* colmax, int b, const Table& t, int8_t* planes,
                             int64_t ldq, int64_t plane, int* ty, hipStream_t s) {
  if (npad <= 0 || k <= 0) return hipSuccess;
  if (b > 24) return hipErrorInvalidValue;   // pieces must stay exact in binary32
  dim3 grid((unsigned)((k + 63) / 64), (unsigned)(npad / 64));
  y_residues_kernel<<<grid, 256, 0, s>>>(Y, ldy, n, k, colmax, b, t, planes, ldq, plane, ty);
  return hipGetLastError();
}

hipError_t launch_recombine(const int8_t* Z, int64_t ldz, int64_t zplane, const Table& t,
                            const int* sl, const int* ty, const float* Yq, int64_t ldy, int yshift,
                            const double* L, int64_t ldl, const double* Rin, int64_t ldri,
                            double* Rout, int64_t ldro, float* Rl, double* X, int64_t ldx,
                            int xmode, int64_t n, int64_t k, double* part, double* out,
                            hipStream_t s) {
  recombine_kernel<<<kRecBlocks, 256, 0, s>>>(Z, ldz, zplane, t, sl, ty, Yq, ldy, yshift, L, ldl,
                                              Rin, ldri, Rout, ldro, Rl, X, ldx, xmode, n, k, part);
  recombine_final_kernel<<<1, 64, 0, s>>>(part, kRecBlocks, out);
  return hipGetLastError();
}

hipError_t launch_assemble(const float* Y0, int s0, const float* Y1, int s1, const float* Y2,
                           int s2, int64_t ldy, double* X, int64_t ldx, int64_t n, int64_t k,
                           bool accumulate, hipStream_t s) {
  if (n <= 0 || k <= 0) return hipSuccess;
  assemble_kernel<<<(unsigned)std::min<int64_t>(n, 4096), 256, 0, s>>>(Y0, s0, Y1, s1, Y2, s2, ldy,
                                                                      X, ldx, n, k, accumulate);
  return hipGetLastError();
}

template hipError_t launch_dstats<float>(const float*, int64_t, int64_t, int64_t, unsigned*,
                                         double*, double*, hipStream_t);
template hipError_t launch_dstats<double>(const double*, int64_t, int64_t, int64_t, unsigned*,
                                          double*, double*, hipStream_t);
}  // namespace crt
}  // namespace trsm
