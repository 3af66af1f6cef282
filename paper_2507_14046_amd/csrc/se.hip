// Squeeze-and-Excitation unit of the 3D-FastResUNet (Sec. III-D) on
// channels-last FP32 tensors [V][C] (C a multiple of 4): the channel means
// s = (1/V) sum_v x[v], the gate e = sigmoid(W2 relu(W1 s + b1) + b2) and
// y[v][c] = e[c] x[v][c], with the backward.  The voxel passes are HBM-bound
// streams of float4 rows; the excitation MLP (C x H weights) runs in one
// block.  Column sums go through per-chunk partials, summed in groups by a
// wide pass and then over the groups, in a fixed order (FP64 above the chunks).
#include <algorithm>

#include "kernels.h"

namespace d2ip {
namespace {

constexpr int kSeChunks = 1024;  // voxel chunks of a column-sum pass (at most)

// part[chunk][c] = sum over the chunk's voxels of a[v][c] (* b[v][c] when b is
// given).  Thread (r, q) of R = 256 / C4 row lanes and C4 = C / 4 quads sums
// rows r, r + R, ... of its quad; the R lanes are then added in order.
__global__ __launch_bounds__(256) void k_se_colsum(const float* __restrict__ a,
                                                   const float* __restrict__ b, int V, int C,
                                                   int chunk, float* __restrict__ part) {
  __shared__ float4 red[256];
  const int C4 = C >> 2, R = 256 / C4;
  const int q = threadIdx.x % C4, r = threadIdx.x / C4;
  const int v0 = blockIdx.x * chunk, v1 = min(V, v0 + chunk);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r < R) {
    int v = v0 + r;
    for (; v + 3 * R < v1; v += 4 * R) {
      float4 t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        t[u] = *reinterpret_cast<const float4*>(a + (size_t)(v + u * R) * C + 4 * q);
        if (b) {
          const float4 m = *reinterpret_cast<const float4*>(b + (size_t)(v + u * R) * C + 4 * q);
          t[u].x *= m.x;
          t[u].y *= m.y;
          t[u].z *= m.z;
          t[u].w *= m.w;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc.x += t[u].x;
        acc.y += t[u].y;
        acc.z += t[u].z;
        acc.w += t[u].w;
      }
    }
    for (; v < v1; v += R) {
      float4 t = *reinterpret_cast<const float4*>(a + (size_t)v * C + 4 * q);
      if (b) {
        const float4 m = *reinterpret_cast<const float4*>(b + (size_t)v * C + 4 * q);
        t.x *= m.x;
        t.y *= m.y;
        t.z *= m.z;
        t.w *= m.w;
      }
      acc.x += t.x;
      acc.y += t.y;
      acc.z += t.z;
      acc.w += t.w;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < C4) {
    float4 s = red[threadIdx.x];
    for (int rr = 1; rr < R; ++rr) {
      const float4 t = red[rr * C4 + threadIdx.x];
      s.x += t.x;
      s.y += t.y;
      s.z += t.z;
      s.w += t.w;
    }
    *reinterpret_cast<float4*>(part + (size_t)blockIdx.x * C + 4 * threadIdx.x) = s;
  }
}

constexpr int kSeGroup = 32;  // chunk partials per first-stage sum

// First stage of the column sums: gsum[g][c] = sum of part[k][c] over the
// chunks k of group g, in chunk order (FP64).  Grid: (ceil(C / 256), groups).
__global__ __launch_bounds__(256) void k_se_psum(const float* __restrict__ part, int nchunks,
                                                 int C, double* __restrict__ gsum) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= C) return;
  const int k0 = blockIdx.y * kSeGroup, k1 = min(nchunks, k0 + kSeGroup);
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int k = k0;
  for (; k + 8 <= k1; k += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(k + u) * C + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  float r[7];  // the rest: every load issued, then added in the same order
#pragma unroll
  for (int u = 0; u < 7; ++u) r[u] = k + u < k1 ? part[(size_t)(k + u) * C + c] : 0.f;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (k + u < k1) a[u] += r[u];
  gsum[(size_t)blockIdx.y * C + c] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Column c of the group sums in a fixed order (eight loads in flight).
__device__ __forceinline__ double se_sum(const double* gsum, int ngroups, int C, int c) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int g = 0;
  for (; g + 8 <= ngroups; g += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = gsum[(size_t)(g + u) * C + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  double r[7];  // the rest: every load issued, then added in the same order
#pragma unroll
  for (int u = 0; u < 7; ++u) r[u] = g + u < ngroups ? gsum[(size_t)(g + u) * C + c] : 0.0;
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (g + u < ngroups) a[u] += r[u];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// One block: s, z = relu(W1 s + b1), e = sigmoid(W2 z + b2) into
// st = [s (C), e (C), z (H)] (e 16-byte aligned for the scaling pass).
__global__ __launch_bounds__(256) void k_se_mlp(const double* __restrict__ gsum, int ngroups,
                                                int V, int C, int H, const float* __restrict__ w1,
                                                const float* __restrict__ b1,
                                                const float* __restrict__ w2,
                                                const float* __restrict__ b2, float* st) {
  extern __shared__ float sh[];  // s (C), z (H)
  float* s = sh;
  float* z = sh + C;
  for (int c = threadIdx.x; c < C; c += 256) {
    s[c] = (float)(se_sum(gsum, ngroups, C, c) / (double)V);
    st[c] = s[c];
  }
  __syncthreads();
  for (int h = threadIdx.x; h < H; h += 256) {
    float a = b1[h];
    for (int c = 0; c < C; ++c) a += w1[(size_t)h * C + c] * s[c];
    z[h] = fmaxf(a, 0.f);
    st[2 * C + h] = z[h];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) {
    float a = b2[c];
    for (int h = 0; h < H; ++h) a += w2[(size_t)c * H + h] * z[h];
    st[C + c] = 1.f / (1.f + expf(-a));
  }
}

// One block: the excitation's backward from ge = column sums of gy * x.
// Writes the weight and bias gradients (any may be null) and
// gsv[c] = (dL/ds[c]) / V for the input gradient.
__global__ __launch_bounds__(256) void k_se_mlp_bwd(const double* __restrict__ gsum, int ngroups,
                                                    int V, int C, int H,
                                                    const float* __restrict__ w1,
                                                    const float* __restrict__ w2,
                                                    const float* __restrict__ st, float* gw1,
                                                    float* gb1, float* gw2, float* gb2,
                                                    float* gsv) {
  extern __shared__ float sh[];  // ga2 (C), ga1 (H)
  float* ga2 = sh;
  float* ga1 = sh + C;
  const float* s = st;
  const float* e = st + C;
  const float* z = st + 2 * C;
  for (int c = threadIdx.x; c < C; c += 256) {
    const float ge = (float)se_sum(gsum, ngroups, C, c);
    ga2[c] = ge * e[c] * (1.f - e[c]);
    if (gb2) gb2[c] = ga2[c];
  }
  __syncthreads();
  if (gw2)
    for (int i = threadIdx.x; i < C * H; i += 256) gw2[i] = ga2[i / H] * z[i % H];
  for (int h = threadIdx.x; h < H; h += 256) {
    float g = 0.f;
    for (int c = 0; c < C; ++c) g += w2[(size_t)c * H + h] * ga2[c];
    ga1[h] = z[h] > 0.f ? g : 0.f;
    if (gb1) gb1[h] = ga1[h];
  }
  __syncthreads();
  if (gw1)
    for (int i = threadIdx.x; i < H * C; i += 256) gw1[i] = ga1[i / C] * s[i % C];
  if (gsv)
    for (int c = threadIdx.x; c < C; c += 256) {
      float g = 0.f;
      for (int h = 0; h < H; ++h) g += w1[(size_t)h * C + c] * ga1[h];
      gsv[c] = g / (float)V;
    }
}

// y = a * e[c] (+ add[c]) over float4 elements.
__global__ __launch_bounds__(256) void k_se_scale(const float* __restrict__ a,
                                                  const float* __restrict__ e,
                                                  const float* __restrict__ add, float* y,
                                                  size_t n4, int C4) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256) {
    const int q = (int)(i % C4);
    const float4 v = reinterpret_cast<const float4*>(a)[i];
    const float4 g = reinterpret_cast<const float4*>(e)[q];
    float4 o = make_float4(v.x * g.x, v.y * g.y, v.z * g.z, v.w * g.w);
    if (add) {
      const float4 t = reinterpret_cast<const float4*>(add)[q];
      o.x += t.x;
      o.y += t.y;
      o.z += t.z;
      o.w += t.w;
    }
    reinterpret_cast<float4*>(y)[i] = o;
  }
}

void se_chunks(int V, int C, int* chunk, int* nchunks) {
  const int R = 256 / (C / 4);
  int len = (V + kSeChunks - 1) / kSeChunks;
  len = ((len + 4 * R - 1) / (4 * R)) * 4 * R;  // whole unrolled passes
  *chunk = len;
  *nchunks = (V + len - 1) / len;
}

}  // namespace

int se_groups(int nchunks) { return (nchunks + kSeGroup - 1) / kSeGroup; }

// Floats of the workspace: two chunk-partial arrays, two group-sum arrays
// (doubles), the state [s, e, z] and gsv.
size_t se_scratch(int V, int C, int H) {
  int chunk, nchunks;
  se_chunks(V, C, &chunk, &nchunks);
  return 2 * (size_t)nchunks * C + 4 * (size_t)se_groups(nchunks) * C +
         (size_t)((2 * C + H + 3) / 4 * 4) + C;
}

namespace {
struct SeWs {
  float *part, *part2, *st, *gsv;
  double *gsum, *gsum2;
  int chunk, nchunks, ngroups;
};
SeWs se_ws(float* ws, int V, int C, int H) {
  SeWs w;
  se_chunks(V, C, &w.chunk, &w.nchunks);
  w.ngroups = se_groups(w.nchunks);
  w.part = ws;
  w.part2 = ws + (size_t)w.nchunks * C;
  // C % 4 == 0 keeps every piece below 16-byte aligned (doubles 8-byte)
  w.gsum = reinterpret_cast<double*>(w.part2 + (size_t)w.nchunks * C);
  w.gsum2 = w.gsum + (size_t)w.ngroups * C;
  w.st = reinterpret_cast<float*>(w.gsum2 + (size_t)w.ngroups * C);
  w.gsv = w.st + (2 * C + H + 3) / 4 * 4;  // 16-byte aligned
  return w;
}
unsigned se_grid(size_t n4) { return (unsigned)std::min<size_t>((n4 + 255) / 256, 8192); }
}  // namespace

void se_forward(const float* x, const float* w1, const float* b1, const float* w2,
                const float* b2, float* y, int V, int C, int H, float* ws, hipStream_t s) {
  const SeWs w = se_ws(ws, V, C, H);
  hipLaunchKernelGGL(k_se_colsum, dim3(w.nchunks), dim3(256), 0, s, x, nullptr, V, C, w.chunk,
                     w.part);
  hipLaunchKernelGGL(k_se_psum, dim3((C + 255) / 256, w.ngroups), dim3(256), 0, s, w.part,
                     w.nchunks, C, w.gsum);
  hipLaunchKernelGGL(k_se_mlp, dim3(1), dim3(256), (size_t)(C + H) * sizeof(float), s, w.gsum,
                     w.ngroups, V, C, H, w1, b1, w2, b2, w.st);
  const size_t n4 = (size_t)V * C / 4;
  hipLaunchKernelGGL(k_se_scale, dim3(se_grid(n4)), dim3(256), 0, s, x, w.st + C, nullptr, y,
                     n4, C / 4);
}

void se_backward(const float* x, const float* w1, const float* b1, const float* w2,
                 const float* b2, const float* gy, float* gx, float* gw1, float* gb1, float* gw2,
                 float* gb2, int V, int C, int H, float* ws, hipStream_t s) {
  const SeWs w = se_ws(ws, V, C, H);
  // the forward state (s, z, e), recomputed from x
  hipLaunchKernelGGL(k_se_colsum, dim3(w.nchunks), dim3(256), 0, s, x, nullptr, V, C, w.chunk,
                     w.part);
  hipLaunchKernelGGL(k_se_colsum, dim3(w.nchunks), dim3(256), 0, s, gy, x, V, C, w.chunk,
                     w.part2);
  hipLaunchKernelGGL(k_se_psum, dim3((C + 255) / 256, w.ngroups), dim3(256), 0, s, w.part,
                     w.nchunks, C, w.gsum);
  hipLaunchKernelGGL(k_se_psum, dim3((C + 255) / 256, w.ngroups), dim3(256), 0, s, w.part2,
                     w.nchunks, C, w.gsum2);
  hipLaunchKernelGGL(k_se_mlp, dim3(1), dim3(256), (size_t)(C + H) * sizeof(float), s, w.gsum,
                     w.ngroups, V, C, H, w1, b1, w2, b2, w.st);
  hipLaunchKernelGGL(k_se_mlp_bwd, dim3(1), dim3(256), (size_t)(C + H) * sizeof(float), s,
                     w.gsum2, w.ngroups, V, C, H, w1, w2, w.st, gw1, gb1, gw2, gb2, w.gsv);
  if (gx) {
    const size_t n4 = (size_t)V * C / 4;
    hipLaunchKernelGGL(k_se_scale, dim3(se_grid(n4)), dim3(256), 0, s, gy, w.st + C, w.gsv, gx,
                       n4, C / 4);
  }
}

}  // namespace d2ip
