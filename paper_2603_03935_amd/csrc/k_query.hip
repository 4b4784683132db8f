// Open-vocabulary query over the instance embeddings (arXiv 2603.03935,
// Sec. III-C: instances are retrieved by the cosine similarity of their
// embedding with a text embedding; Sec. IV evaluates exactly this):
//   sim[j][i] = cos(text_j, emb_i)  (0 when either vector is zero)
//   for each query j, the k instances of highest similarity, higher first,
//   ties to the lower instance index.
// The similarity matrix is one dense contraction (q x m, K = e) on FP32 MFMA
// (v_mfma_f32_32x32x2f32, FP32 accumulation); the ranking is a per-query
// selection that takes the k largest keys in k passes over the row.
#include <type_traits>

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

// ---------------------------------------------------------------------------
// Weighted similarity heat-map of text queries over one frame's patches
// (Sec. III-C, the feature-similarity figure):
//   heat[j][p] = D_p cos(text_j, y_p),  y_p = f_p^T P,
// D of Eq. (1).  The patch tokens are projected by one FP32-MFMA contraction
// (G x E, K = C); each projected row's inverse norm is folded with D_p into
// one per-patch factor, and the cosine contraction above (k_sim) applies it.
// ---------------------------------------------------------------------------
template <int TOK>
__device__ __forceinline__ float4 load_tok4(const void* base, const float* scale, int64_t row, int c, int C) {
  const int64_t off = row * C + c;
  if (TOK == 0) return *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + off);
  if (TOK == 1) return load_row4<1>(base, off);
  // e4m3fn codes times the token's scale (every code value is exact in FP32)
  const uint32_t q = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(base) + off);
  const float sc = scale[row];
  const float4 x = e4m3x4_to_f32(q);
  return make_float4(x.x * sc, x.y * sc, x.z * sc, x.w * sc);
}

// Y[G][E] = tokens[G][C] P[C][E]: 64 x 64 tiles (4 wavefronts of 32 x 32),
// K in steps of 16 through LDS; TOK 0 F32, 1 BF16, 2 FP8 + scale; PB: P in BF16.
template <int TOK, int PB>
__global__ __launch_bounds__(256) void k_tokproj(const void* tok, const float* scale, int G, int C, const void* P,
                                                 int E, float* Y) {
  constexpr int BK = 16;
  const int g0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wg = wv >> 1, wn = wv & 1;
  __shared__ float As[64][BK + 1];
  __shared__ float Bs[64][BK + 1];
  floatx16 acc = {};
  const int lr = tid >> 2, lk = (tid & 3) * 4;         // A: row lr, channels lk..lk+3
  const int bk = tid >> 4, bn = (tid & 15) * 4;        // B: channel bk, columns bn..bn+3
  for (int k0 = 0; k0 < C; k0 += BK) {
    const float4 av = g0 + lr < G ? load_tok4<TOK>(tok, scale, g0 + lr, k0 + lk, C) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 bv = load_row4<PB>(P, (int64_t)(k0 + bk) * E + n0 + bn);
    __syncthreads();
    As[lr][lk] = av.x; As[lr][lk + 1] = av.y; As[lr][lk + 2] = av.z; As[lr][lk + 3] = av.w;
    Bs[bn][bk] = bv.x; Bs[bn + 1][bk] = bv.y; Bs[bn + 2][bk] = bv.z; Bs[bn + 3][bk] = bv.w;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const float a = As[32 * wg + (lane & 31)][kk + (lane >> 5)];
      const float b = Bs[32 * wn + (lane & 31)][kk + (lane >> 5)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }
  // acc[v]: row 32 wg + 8 (v >> 2) + 4 (lane >> 5) + (v & 3), column 32 wn + (lane & 31)
  const int n = n0 + 32 * wn + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int g = g0 + 32 * wg + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (g < G) Y[(int64_t)g * E + n] = acc[v];
  }
}

// f[p] = D[p] / ||Y_p|| (0 for a zero row); one wavefront per row
__global__ __launch_bounds__(256) void k_heat_factor(const float* Y, int G, int E, const float* D, float* f) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= G) return;
  float a = 0.f;
  for (int c = lane * 4; c < E; c += 256) {
    const float4 v = *reinterpret_cast<const float4*>(Y + (int64_t)r * E + c);
    a += v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
  }
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) f[r] = a > 0.f ? D[r] / __builtin_sqrtf(a) : 0.f;
}

void launch_heatmap(const void* tok, int tok_dtype, const float* scale, int G, int C, const void* P, int p_bf16, int E,
                    const void* text, int text_bf16, int q, const float* D, float* Y, float* fac, float* inv_text,
                    float* heat, hipStream_t st) {
  const dim3 pg((G + 63) / 64, E / 64);
  auto proj = [&](auto tk, auto pb) {
    constexpr int T = decltype(tk)::value, B = decltype(pb)::value;
    hipLaunchKernelGGL((k_tokproj<T, B>), pg, dim3(256), 0, st, tok, scale, G, C, P, E, Y);
  };
  using Z = std::integral_constant<int, 0>;
  using O = std::integral_constant<int, 1>;
  using T2 = std::integral_constant<int, 2>;
  if (tok_dtype == 0) { if (p_bf16) proj(Z{}, O{}); else proj(Z{}, Z{}); }
  else if (tok_dtype == 1) { if (p_bf16) proj(O{}, O{}); else proj(O{}, Z{}); }
  else { if (p_bf16) proj(T2{}, O{}); else proj(T2{}, Z{}); }
  hipLaunchKernelGGL(k_heat_factor, dim3((G + 3) / 4), dim3(256), 0, st, Y, G, E, D, fac);
  if (text_bf16)
    hipLaunchKernelGGL(k_invnorm<1>, dim3((q + 3) / 4), dim3(256), 0, st, text, q, E, inv_text);
  else
    hipLaunchKernelGGL(k_invnorm<0>, dim3((q + 3) / 4), dim3(256), 0, st, text, q, E, inv_text);
  const dim3 grid((G + 63) / 64, (q + 63) / 64);
  if (text_bf16)
    hipLaunchKernelGGL(k_sim<1>, grid, dim3(256), 0, st, Y, G, text, q, E, fac, inv_text, heat);
  else
    hipLaunchKernelGGL(k_sim<0>, grid, dim3(256), 0, st, Y, G, text, q, E, fac, inv_text, heat);
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
