// View quality and feature fusion (arXiv 2603.03935, Sec. III-C, Eqs. 2-3),
// the per-observation consumers of the instance embeddings:
//   Q = S_size S_angle S_sem S_dist per observation;
//   S_angle = mean over a detection's voxels of max(0, -r.n);
//   fusion: per map instance, the observation of the largest Q above the
//   stored Q replaces the stored feature (the first of equal Q).
// All three are streaming passes bound by HBM bandwidth (a few reads per
// element, no reuse); one wavefront per row, fixed reduction order.
#include "disc_device.h"

namespace disc {

__device__ __forceinline__ float wave_sum_f(float a) {
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  return a;
}

// one wavefront per observation; 4 per workgroup
__global__ __launch_bounds__(256) void k_quality(const int32_t* area, const float* dbar, const float* emb,
                                                 const float* g, const float* angle, int m, int e, float inv_hw,
                                                 float lambda, float* q, float* comp) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= m) return;
  const float* y = emb + (int64_t)i * e;
  float yy = 0.f, gg = 0.f, yg = 0.f;
  for (int c = lane * 4; c < e; c += 256) {
    const float4 a = *reinterpret_cast<const float4*>(y + c);
    const float4 b = *reinterpret_cast<const float4*>(g + c);
    yy += a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w;
    gg += b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w;
    yg += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
  }
  yy = wave_sum_f(yy);
  gg = wave_sum_f(gg);
  yg = wave_sum_f(yg);
  if (lane != 0) return;
  const float size = fminf(lambda * (float)area[i] * inv_hw, 1.0f);
  float sem = (yy > 0.f && gg > 0.f) ? yg / (__builtin_sqrtf(yy) * __builtin_sqrtf(gg)) : 0.f;
  sem = fminf(fmaxf(sem, 0.f), 1.f);
  const float dist = 0.5f + 0.5f * dbar[i];
  const float ang = angle ? angle[i] : 1.0f;
  q[i] = size * ang * sem * dist;
  if (comp) *reinterpret_cast<float4*>(comp + 4 * (int64_t)i) = make_float4(size, ang, sem, dist);
}

// one wavefront per detection: mean of max(0, -r.n) over its voxels
__global__ __launch_bounds__(256) void k_angle(const float* rays, const float* normals, int nv, const int32_t* off,
                                               int m, float* angle) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= m) return;
  const int a = min(max(off[i], 0), nv), b = min(max(off[i + 1], 0), nv);
  float s = 0.f;
  for (int v = a + lane; v < b; v += 64) {
    const float* r = rays + 3 * (int64_t)v;
    const float* n = normals + 3 * (int64_t)v;
    const float c = -(r[0] * n[0] + r[1] * n[1] + r[2] * n[2]);
    s += fmaxf(c, 0.f);
  }
  s = wave_sum_f(s);
  if (lane == 0) angle[i] = b > a ? s / (float)(b - a) : 0.f;
}

// Order-preserving key: larger quality first, then the lower observation
// index; never 0 (0 marks "no bid").
__device__ __forceinline__ uint64_t fuse_key(float v, int i) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)o << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
}

__global__ __launch_bounds__(256) void k_fuse_clear(const int32_t* ids, int m, int n_map, uint64_t* best) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int t = ids[i];
  if (t >= 0 && t < n_map) best[t] = 0;
}

__global__ __launch_bounds__(256) void k_fuse_bid(const int32_t* ids, const float* q, int m, const float* map_q,
                                                  int n_map, uint64_t* best) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int t = ids[i];
  if (t < 0 || t >= n_map) return;
  const float v = q[i];
  if (v > map_q[t]) atomicMax(reinterpret_cast<unsigned long long*>(best + t), (unsigned long long)fuse_key(v, i));
}

// one wavefront per observation: the winner of its instance copies its row
__global__ __launch_bounds__(256) void k_fuse_apply(const int32_t* ids, const float* q, const float* emb, int m, int e,
                                                    float* map_q, float* map_emb, int n_map, int32_t* won,
                                                    const uint64_t* best) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= m) return;
  const int t = ids[i];
  const bool win = t >= 0 && t < n_map && best[t] == fuse_key(q[i], i);
  if (lane == 0 && won) won[i] = win ? 1 : 0;
  if (!win) return;
  const float* src = emb + (int64_t)i * e;
  float* dst = map_emb + (int64_t)t * e;
  for (int c = lane * 4; c < e; c += 256)
    *reinterpret_cast<float4*>(dst + c) = *reinterpret_cast<const float4*>(src + c);
  if (lane == 0) map_q[t] = q[i];
}

void launch_quality(const int32_t* area, const float* dbar, const float* emb, const float* g, const float* angle, int m,
                    int e, int img_h, int img_w, float lambda, float* q, float* comp, hipStream_t st) {
  if (m <= 0) return;
  const float inv_hw = (float)(1.0 / ((double)img_h * (double)img_w));
  hipLaunchKernelGGL(k_quality, dim3((m + 3) / 4), dim3(256), 0, st, area, dbar, emb, g, angle, m, e, inv_hw, lambda, q,
                     comp);
}

void launch_angle(const float* rays, const float* normals, int nv, const int32_t* off, int m, float* angle,
                  hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_angle, dim3((m + 3) / 4), dim3(256), 0, st, rays, normals, nv, off, m, angle);
}

void launch_fuse(const int32_t* ids, const float* q, const float* emb, int m, int e, float* map_q, float* map_emb,
                 int n_map, int32_t* won, uint64_t* best, hipStream_t st) {
  if (m <= 0) return;
  const int nb = (m + 255) / 256;
  hipLaunchKernelGGL(k_fuse_clear, dim3(nb), dim3(256), 0, st, ids, m, n_map, best);
  hipLaunchKernelGGL(k_fuse_bid, dim3(nb), dim3(256), 0, st, ids, q, m, map_q, n_map, best);
  hipLaunchKernelGGL(k_fuse_apply, dim3((m + 3) / 4), dim3(256), 0, st, ids, q, emb, m, e, map_q, map_emb, n_map, won,
                     best);
}

}  // namespace disc
