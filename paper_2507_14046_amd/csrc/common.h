// Shared device helpers of the D2IP HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define D2IP_WAVE 64

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

// float -> bf16 bits, round to nearest even (finite inputs; NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of a double (blockDim.x multiple of 64, <= 1024); result
// valid in thread 0.  `sh` needs blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

constexpr float kLnEps = 1e-5f;  // LayerNorm epsilon (inside the square root)

// Normalisation statistics of one LayerNorm: mean and 1/sqrt(var + eps).
struct LnStat {
  float mean, rstd;
};

// Coefficients of the LayerNorm backward: dh = rstd*(gamma_c*dz - A - xhat*B).
struct LnBwd {
  float A, B;
};

// Per-block FP64 partial pairs written by the producer of a LayerNorm input
// (sum, sum of squares) or of its backward ((sum_c gamma_c sum gz),
// (sum_c gamma_c sum gz*xhat)); every consumer block reduces them itself.
struct PairRef {
  const double* part;  // [nparts][2]
  int nparts;
  double count;        // elements normalised together
};

// Block-wide sums of the (a, b) pairs of up to two partial arrays, in a fixed
// order; the same values in all threads.  Thread t adds pairs t, t + 256, ...
// (the first four loads of each array issued together), waves combine by a
// butterfly, then the four wave totals are added in wave order.  Contains
// barriers: every thread of the block must call it (blockDim.x == 256).
__device__ __forceinline__ void block_pair_sums(const double* p1, int n1, const double* p2, int n2,
                                                double& s1, double& s2, double& s3, double& s4) {
  __shared__ double sh[4][4];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  double ra[4], rb[4], rc[4], rd[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = t + 256 * k;
    ra[k] = i < n1 ? p1[2 * i] : 0.0;
    rb[k] = i < n1 ? p1[2 * i + 1] : 0.0;
    rc[k] = i < n2 ? p2[2 * i] : 0.0;
    rd[k] = i < n2 ? p2[2 * i + 1] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a += ra[k];
    b += rb[k];
    c += rc[k];
    d += rd[k];
  }
  for (int i = t + 1024; i < n1; i += 256) {
    a += p1[2 * i];
    b += p1[2 * i + 1];
  }
  for (int i = t + 1024; i < n2; i += 256) {
    c += p2[2 * i];
    d += p2[2 * i + 1];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  d = wave_sum(d);
  const int w = t >> 6;
  __syncthreads();
  if ((t & 63) == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
    sh[2][w] = c;
    sh[3][w] = d;
  }
  __syncthreads();
  s1 = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
  s2 = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  s3 = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
  s4 = (sh[3][0] + sh[3][1]) + (sh[3][2] + sh[3][3]);
}

__device__ __forceinline__ LnStat stat_from(double s1, double s2, double count) {
  const double mean = s1 / count;
  double var = s2 / count - mean * mean;
  if (var < 0.0) var = 0.0;
  LnStat st;
  st.mean = (float)mean;
  st.rstd = (float)(1.0 / sqrt(var + (double)kLnEps));
  return st;
}

__device__ __forceinline__ LnStat stat_of(const PairRef& r) {
  double s1, s2, s3, s4;
  block_pair_sums(r.part, r.nparts, nullptr, 0, s1, s2, s3, s4);
  return stat_from(s1, s2, r.count);
}

__device__ __forceinline__ LnBwd coef_of(const PairRef& r) {
  double s1, s2, s3, s4;
  block_pair_sums(r.part, r.nparts, nullptr, 0, s1, s2, s3, s4);
  LnBwd c;
  c.A = (float)(s1 / r.count);
  c.B = (float)(s2 / r.count);
  return c;
}

// Statistics and LayerNorm-backward coefficients from one combined reduction.
__device__ __forceinline__ void stat_coef_of(const PairRef& st, const PairRef& bw, LnStat& s,
                                             LnBwd& c) {
  double s1, s2, s3, s4;
  block_pair_sums(st.part, st.nparts, bw.part, bw.nparts, s1, s2, s3, s4);
  s = stat_from(s1, s2, st.count);
  c.A = (float)(s3 / bw.count);
  c.B = (float)(s4 / bw.count);
}

// Members of an instance group share every shape; member b's data lives
// b * istride bytes after member 0's.  A kernel shifts its per-member pointers.
template <class T>
__host__ __device__ __forceinline__ T* ishift(T* p, long long off) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<typename std::remove_const<T>::type*>(p)) + off)
           : p;
}
