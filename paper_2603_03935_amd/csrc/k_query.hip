// Open-vocabulary query over the instance embeddings (arXiv 2603.03935,
// Sec. III-C: instances are retrieved by the cosine similarity of their
// embedding with a text embedding; Sec. IV evaluates exactly this):
//   sim[j][i] = cos(text_j, emb_i)  (0 when either vector is zero)
//   for each query j, the k instances of highest similarity, higher first,
//   ties to the lower instance index.
// The similarity matrix is one dense contraction (q x m, K = e) on FP32 MFMA
// (v_mfma_f32_32x32x2f32, FP32 accumulation); the ranking is a per-query
// selection that takes the k largest keys in k passes over the row.
#include "disc_device.h"

namespace disc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int BF16>
__device__ __forceinline__ float4 load_row4(const void* base, int64_t off) {
  if (BF16) {
    const uint2 v = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + off);
    return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u), __uint_as_float(v.y << 16),
                       __uint_as_float(v.y & 0xFFFF0000u));
  }
  return *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + off);
}

// inv[r] = 1 / ||row r|| (0 for a zero row); one wavefront per row
template <int BF16>
__global__ __launch_bounds__(256) void k_invnorm(const void* x, int rows, int e, float* inv) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= rows) return;
  float a = 0.f;
  for (int c = lane * 4; c < e; c += 256) {
    const float4 v = load_row4<BF16>(x, (int64_t)r * e + c);
    a += v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
  }
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) inv[r] = a > 0.f ? 1.0f / __builtin_sqrtf(a) : 0.f;
}

// sim tile: 64 queries x 64 instances per workgroup (4 wavefronts of 32 x 32),
// K in steps of 16 staged through LDS.
template <int BF16>
__global__ __launch_bounds__(256) void k_sim(const float* emb, int m, const void* text, int q, int e,
                                             const float* inv_emb, const float* inv_text, float* sim) {
  constexpr int BK = 16;
  const int q0 = blockIdx.y * 64, i0 = blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wq = wv >> 1, wi = wv & 1;
  __shared__ float Ts[64][BK + 1];
  __shared__ float Ys[64][BK + 1];
  floatx16 acc = {};
  // loaders: 64 rows x 16 k = 1024 floats per operand, 4 per thread
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  for (int k0 = 0; k0 < e; k0 += BK) {
    const float4 tv = q0 + lr < q ? load_row4<BF16>(text, (int64_t)(q0 + lr) * e + k0 + lk) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 yv = i0 + lr < m ? *reinterpret_cast<const float4*>(emb + (int64_t)(i0 + lr) * e + k0 + lk)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    Ts[lr][lk] = tv.x; Ts[lr][lk + 1] = tv.y; Ts[lr][lk + 2] = tv.z; Ts[lr][lk + 3] = tv.w;
    Ys[lr][lk] = yv.x; Ys[lr][lk + 1] = yv.y; Ys[lr][lk + 2] = yv.z; Ys[lr][lk + 3] = yv.w;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const float a = Ts[32 * wq + (lane & 31)][kk + (lane >> 5)];
      const float bb = Ys[32 * wi + (lane & 31)][kk + (lane >> 5)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc, 0, 0, 0);
    }
  }
  const int i = i0 + 32 * wi + (lane & 31);
  if (i >= m) return;
  const float yi = inv_emb[i];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int j = q0 + 32 * wq + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (j < q) sim[(int64_t)j * m + i] = acc[v] * yi * inv_text[j];
  }
}

// Order-preserving 64-bit key: larger score first, then smaller index.
__device__ __forceinline__ uint64_t rank_key(float s, int i) {
  const uint32_t b = __float_as_uint(s);
  const uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)o << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)i);
}

// one workgroup per query: k passes, each takes the largest key below the last
__global__ __launch_bounds__(256) void k_topk(const float* sim, int m, int q, int k, float* scores, int32_t* idx) {
  const int j = blockIdx.x;
  if (j >= q) return;
  const float* row = sim + (int64_t)j * m;
  __shared__ uint64_t red[4];
  uint64_t last = ~0ull;
  for (int r = 0; r < k; ++r) {
    uint64_t best = 0;
    for (int i = threadIdx.x; i < m; i += 256) {
      const uint64_t key = rank_key(row[i], i);
      if (key < last && key > best) best = key;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const uint64_t t = __shfl_xor(best, o);
      best = t > best ? t : best;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    best = red[0];
    for (int w = 1; w < 4; ++w) best = red[w] > best ? red[w] : best;
    __syncthreads();
    if (threadIdx.x == 0) {
      if (best == 0) {
        idx[(int64_t)j * k + r] = -1;
        scores[(int64_t)j * k + r] = -__builtin_inff();
      } else {
        const int i = (int)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFu));
        idx[(int64_t)j * k + r] = i;
        scores[(int64_t)j * k + r] = row[i];
      }
    }
    last = best;
  }
}

void launch_query(const float* emb, int m, const void* text, int text_bf16, int q, int e, int k, float* inv,
                  float* sim, float* scores, int32_t* idx, hipStream_t st) {
  float* inv_emb = inv;
  float* inv_text = inv + m;
  if (m > 0) hipLaunchKernelGGL(k_invnorm<0>, dim3((m + 3) / 4), dim3(256), 0, st, emb, m, e, inv_emb);
  if (text_bf16)
    hipLaunchKernelGGL(k_invnorm<1>, dim3((q + 3) / 4), dim3(256), 0, st, text, q, e, inv_text);
  else
    hipLaunchKernelGGL(k_invnorm<0>, dim3((q + 3) / 4), dim3(256), 0, st, text, q, e, inv_text);
  if (m > 0) {
    const dim3 grid((m + 63) / 64, (q + 63) / 64);
    if (text_bf16)
      hipLaunchKernelGGL(k_sim<1>, grid, dim3(256), 0, st, emb, m, text, q, e, inv_emb, inv_text, sim);
    else
      hipLaunchKernelGGL(k_sim<0>, grid, dim3(256), 0, st, emb, m, text, q, e, inv_emb, inv_text, sim);
  }
  hipLaunchKernelGGL(k_topk, dim3(q), dim3(256), 0, st, sim, m, q, k, scores, idx);
}

}  // namespace disc
