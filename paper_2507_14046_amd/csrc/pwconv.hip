// Pointwise (1x1x1) convolution of the depthwise-separable convolutions of
// the lightweight backbone (Sec. III-D) as FP32 matrix-core GEMMs on
// channels-last tensors: the forward Y[V][N] = X[V][K] W^T + b (W [N][K]), the
// input gradient gX = gY W (the same kernel with W read transposed), and the
// weight gradient gW = gY^T X, gb = column sums of gY, split over voxel
// chunks into partials that a second kernel adds in a fixed order.
//
// The matrix-core step is v_mfma_f32_16x16x4f32: lane l = l16 + 16 g supplies
// A[row l16][k slot g] and B[k slot g][col l16] and receives D[row 4 g + r]
// [col l16] in register r.  The k index behind slot g in step s is 4 g + s of
// the current 16-wide k group, so one float4 LDS read per lane feeds four
// consecutive steps (the order of a sum over k does not change its terms).
#include <algorithm>

#include "kernels.h"

namespace d2ip {
namespace {

constexpr int kPwM = 128;   // rows (voxels) per block: 4 waves x 32
constexpr int kPwN = 64;    // columns per block: 4 tiles of 16
constexpr int kPwKC = 32;   // k per LDS stage
constexpr int kPwLd = kPwKC + 4;  // LDS row stride (floats): float4 aligned, fewer bank conflicts
constexpr int kPwWgBlocks = 1024;  // weight-gradient grid target (chunks x tiles)
constexpr int kPwGroup = 32;       // chunks per first-stage partial sum

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float comp(const float4& v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// 32 rows x 64 columns of a wave over one LDS stage: As [rows][kPwLd] holds
// the block's A rows, Bs [cols][kPwLd] its B columns (k contiguous).
__device__ __forceinline__ void pw_stage_mma(const float* As, const float* Bs, int wave, int l16,
                                             int g, f32x4 (&acc)[2][4]) {
#pragma unroll
  for (int k16 = 0; k16 < kPwKC; k16 += 16) {
    float4 a[2], b[4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
      a[rt] = *reinterpret_cast<const float4*>(As + (wave * 32 + rt * 16 + l16) * kPwLd + k16 +
                                               4 * g);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      b[ct] = *reinterpret_cast<const float4*>(Bs + (ct * 16 + l16) * kPwLd + k16 + 4 * g);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mfma4(comp(a[rt], s), comp(b[ct], s), acc[rt][ct]);
  }
}

// Y[M][N] = X[M][K] B + bias with B[k][n] = W[n][k] (transw = 0, W [N][K]) or
// W[k][n] (transw = 1, W [K][N]).  K and N multiples of 4.  Grid:
// (ceil(M / 128), ceil(N / 64)).
__global__ __launch_bounds__(256) void k_pw_gemm(const float* __restrict__ X,
                                                 const float* __restrict__ W,
                                                 const float* __restrict__ bias,
                                                 float* __restrict__ Y, int M, int K, int N,
                                                 int transw) {
  __shared__ __align__(16) float As[kPwM * kPwLd];
  __shared__ __align__(16) float Bs[kPwN * kPwLd];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g = lane >> 4;
  const size_t m0 = (size_t)blockIdx.x * kPwM;
  const int n0 = blockIdx.y * kPwN;
  f32x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  // stage loads: A 128 rows x 32 k as 1024 float4 (rows contiguous in k,
  // coalesced), B 64 columns x 32 k; the next stage's loads are issued before
  // this stage's MFMAs
  float4 ra[4], rb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i, r = e >> 3, c4 = (e & 7) * 4;
      const bool ok = m0 + r < (size_t)M && k0 + c4 < K;
      const size_t row = ok ? m0 + r : 0;
      ra[i] = *reinterpret_cast<const float4*>(X + row * K + (ok ? k0 + c4 : 0));
      if (!ok) ra[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = tid + 256 * i;
      if (!transw) {  // W [N][K]: column n is a contiguous run of k
        const int n = e >> 3, c4 = (e & 7) * 4;
        const bool ok = n0 + n < N && k0 + c4 < K;
        rb[i] = *reinterpret_cast<const float4*>(W + (size_t)(ok ? n0 + n : 0) * K +
                                                 (ok ? k0 + c4 : 0));
        if (!ok) rb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      } else {  // W [K][N]: row k holds the block's 64 columns contiguously
        const int k = e >> 4, n4 = (e & 15) * 4;
        const bool ok = k0 + k < K && n0 + n4 < N;
        rb[i] = *reinterpret_cast<const float4*>(W + (size_t)(ok ? k0 + k : 0) * N +
                                                 (ok ? n0 + n4 : 0));
        if (!ok) rb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += kPwKC) {
    __syncthreads();  // the previous stage is consumed
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i, r = e >> 3, c4 = (e & 7) * 4;
      *reinterpret_cast<float4*>(As + r * kPwLd + c4) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = tid + 256 * i;
      if (!transw) {
        const int n = e >> 3, c4 = (e & 7) * 4;
        *reinterpret_cast<float4*>(Bs + n * kPwLd + c4) = rb[i];
      } else {
        const int k = e >> 4, n4 = (e & 15) * 4;
        Bs[(n4 + 0) * kPwLd + k] = rb[i].x;
        Bs[(n4 + 1) * kPwLd + k] = rb[i].y;
        Bs[(n4 + 2) * kPwLd + k] = rb[i].z;
        Bs[(n4 + 3) * kPwLd + k] = rb[i].w;
      }
    }
    __syncthreads();
    if (k0 + kPwKC < K) load(k0 + kPwKC);  // uniform
    pw_stage_mma(As, Bs, wave, l16, g, acc);
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int n = n0 + ct * 16 + l16;
    if (n >= N) continue;
    const float bv = bias ? bias[n] : 0.f;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t m = m0 + wave * 32 + rt * 16 + 4 * g + r;
        if (m < (size_t)M) Y[m * N + n] = acc[rt][ct][r] + bv;
      }
  }
}

// Weight-gradient partials: block (chunk, n tile, k tile) computes over the
// chunk's `chunk` voxels v the 64 x 64 tile P[n][k] = sum_v G[v][n] X[v][k] (G = gY
// [M][N], X [M][K]) and, in k tile 0, the column sums of G; both go to
// part[chunk][N * K + N] (n-major).  Grid: (chunks, ceil(N / 64),
// ceil(K / 64)); both operands are staged transposed (v contiguous).
__global__ __launch_bounds__(256) void k_pw_wgrad(const float* __restrict__ X,
                                                  const float* __restrict__ G, float* part,
                                                  int M, int K, int N, int chunk) {
  __shared__ __align__(16) float As[kPwM * kPwLd];  // rows: 64 n of G (only 64 used)
  __shared__ __align__(16) float Bs[kPwN * kPwLd];  // rows: 64 k of X
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, g = lane >> 4;
  const int n0 = blockIdx.y * 64, kk0 = blockIdx.z * 64;
  const size_t v0 = (size_t)blockIdx.x * chunk;
  const size_t v1 = v0 + chunk < (size_t)M ? v0 + chunk : (size_t)M;
  // each wave owns 16 rows (n) x 64 columns (k): one row tile, four column tiles
  f32x4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  float csum = 0.f;  // column sum of G for n = n0 + tid (tid < 64, k tile 0)
  // 32 voxels x 64 columns of G and of X as 512 float4 each; the next
  // stage's loads are issued before this stage's MFMAs
  float4 rg[2], rx[2];
  auto load = [&](size_t vb) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = tid + 256 * i, v = e >> 4, c4 = (e & 15) * 4;
      const bool vok = vb + v < v1;
      const size_t row = vok ? vb + v : v0;
      const bool gok = vok && n0 + c4 < N, xok = vok && kk0 + c4 < K;
      rg[i] = *reinterpret_cast<const float4*>(G + row * N + (gok ? n0 + c4 : 0));
      rx[i] = *reinterpret_cast<const float4*>(X + row * K + (xok ? kk0 + c4 : 0));
      if (!gok) rg[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!xok) rx[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  load(v0);
  for (size_t vb = v0; vb < v1; vb += kPwKC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int e = tid + 256 * i, v = e >> 4, c4 = (e & 15) * 4;
      As[(c4 + 0) * kPwLd + v] = rg[i].x;
      As[(c4 + 1) * kPwLd + v] = rg[i].y;
      As[(c4 + 2) * kPwLd + v] = rg[i].z;
      As[(c4 + 3) * kPwLd + v] = rg[i].w;
      Bs[(c4 + 0) * kPwLd + v] = rx[i].x;
      Bs[(c4 + 1) * kPwLd + v] = rx[i].y;
      Bs[(c4 + 2) * kPwLd + v] = rx[i].z;
      Bs[(c4 + 3) * kPwLd + v] = rx[i].w;
    }
    __syncthreads();
    if (vb + kPwKC < v1) load(vb + kPwKC);  // uniform
    if (blockIdx.z == 0 && tid < 64) {
#pragma unroll
      for (int v = 0; v < kPwKC; v += 4) {
        const float4 q = *reinterpret_cast<const float4*>(As + tid * kPwLd + v);
        csum += ((q.x + q.y) + (q.z + q.w));
      }
    }
#pragma unroll
    for (int k16 = 0; k16 < kPwKC; k16 += 16) {
      const float4 a = *reinterpret_cast<const float4*>(As + (wave * 16 + l16) * kPwLd + k16 +
                                                        4 * g);
      float4 b[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
        b[ct] = *reinterpret_cast<const float4*>(Bs + (ct * 16 + l16) * kPwLd + k16 + 4 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma4(comp(a, s), comp(b[ct], s), acc[ct]);
    }
  }
  float* P = part + (size_t)blockIdx.x * ((size_t)N * K + N);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int k = kk0 + ct * 16 + l16;
    if (k >= K) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = n0 + wave * 16 + 4 * g + r;
      if (n < N) P[(size_t)n * K + k] = acc[ct][r];
    }
  }
  if (blockIdx.z == 0 && tid < 64 && n0 + tid < N) P[(size_t)N * K + n0 + tid] = csum;
}

// First stage of the partial sum: out[r][e] = sum of part[chunk][e] over the
// chunks r * kPwGroup .. (r + 1) * kPwGroup - 1, in chunk order.  Grid:
// (ceil(per / 256), groups).
__global__ __launch_bounds__(256) void k_pw_psum(const float* __restrict__ part, int nchunks,
                                                 size_t per, float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  const int c0 = blockIdx.y * kPwGroup, c1 = min(nchunks, c0 + kPwGroup);
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(c + u) * per + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  float r[7];  // the rest: every load issued, then added in the same order
#pragma unroll
  for (int u = 0; u < 7; ++u) r[u] = c + u < c1 ? part[(size_t)(c + u) * per + e] : 0.f;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (c + u < c1) a[u] += r[u];
  out[(size_t)blockIdx.y * per + e] =
      ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// out[e] = sum over chunks of part[chunk][e] in chunk order, eight loads in
// flight; e < N * K goes to gw (n-major = [N][K]), the rest to gb.
__global__ __launch_bounds__(256) void k_pw_wreduce(const float* __restrict__ part, int nchunks,
                                                    size_t per, int NK, float* gw, float* gb) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int c = 0;
  for (; c + 8 <= nchunks; c += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(c + u) * per + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  float r[7];  // the rest: every load issued, then added in the same order
#pragma unroll
  for (int u = 0; u < 7; ++u) r[u] = c + u < nchunks ? part[(size_t)(c + u) * per + e] : 0.f;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (c + u < nchunks) a[u] += r[u];
  const float s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  if (e < (size_t)NK) {
    if (gw) gw[e] = s;
  } else if (gb) {
    gb[e - NK] = s;
  }
}

// Voxel chunks of the weight gradient: about kPwWgBlocks blocks in all, each
// chunk a multiple of 32 voxels.
void pw_chunks(size_t M, int K, int N, int* chunk, int* nchunks) {
  const int tiles = ((N + 63) / 64) * ((K + 63) / 64);
  const size_t want = std::max<size_t>(1, (kPwWgBlocks + tiles - 1) / tiles);
  size_t len = (M + want - 1) / want;
  len = std::max<size_t>(kPwKC, (len + kPwKC - 1) / kPwKC * kPwKC);
  *chunk = (int)len;
  *nchunks = (int)((M + len - 1) / len);
}

}  // namespace

// Floats of `part`: the chunk partials, then the first-stage group sums.
size_t pw_partials(size_t M, int K, int N) {
  int chunk, nchunks;
  pw_chunks(M, K, N, &chunk, &nchunks);
  const size_t groups = (nchunks + kPwGroup - 1) / kPwGroup;
  return ((size_t)nchunks + groups) * ((size_t)N * K + N);
}

void pw_gemm(const float* X, const float* W, const float* bias, float* Y, size_t M, int K, int N,
             bool transw, hipStream_t s) {
  hipLaunchKernelGGL(k_pw_gemm, dim3((unsigned)((M + kPwM - 1) / kPwM), (N + kPwN - 1) / kPwN),
                     dim3(256), 0, s, X, W, bias, Y, (int)M, K, N, transw ? 1 : 0);
}

void pw_wgrad(const float* X, const float* G, float* part, float* gw, float* gb, size_t M, int K,
              int N, hipStream_t s) {
  int chunk, nchunks;
  pw_chunks(M, K, N, &chunk, &nchunks);
  hipLaunchKernelGGL(k_pw_wgrad, dim3(nchunks, (N + 63) / 64, (K + 63) / 64), dim3(256), 0, s, X,
                     G, part, (int)M, K, N, chunk);
  // chunk partials summed in groups of kPwGroup, then the group sums (two
  // short fixed-order passes instead of one long serial one)
  const size_t per = (size_t)N * K + N;
  const int groups = (nchunks + kPwGroup - 1) / kPwGroup;
  float* sums = part + (size_t)nchunks * per;
  const unsigned eb = (unsigned)((per + 255) / 256);
  hipLaunchKernelGGL(k_pw_psum, dim3(eb, groups), dim3(256), 0, s, part, nchunks, per, sums);
  hipLaunchKernelGGL(k_pw_wreduce, dim3(eb), dim3(256), 0, s, sums, groups, per, N * K, gw, gb);
}

}  // namespace d2ip
