// Token statistics of Eq. (1) (arXiv 2603.03935, Sec. III-C) and the per-mask
// weight finalisation.
//
// Eq. (1): D_p = ||f_p - mean|| / (mean_q ||f_q - mean|| + eps).  Inside the
// weighted mean of the tokens every weight carries the same factor
// 1/(mean r + eps), which cancels, so the fused path weights with
// r_p = ||f_p - mean|| directly; D itself is produced only for the stage entry
// point.  Statistics are per frame (batching never mixes frames).
#include "disc_device.h"

namespace disc {



// e4m3fn code -> BF16 bits of the same value (exact: e4m3 values are BF16 values)

// four consecutive channels of token p as floats (value = scale * code for FP8)
__device__ __forceinline__ float4 load4(const void* base, int dtype, const float* scale, int64_t p, int C, int c) {
  const int64_t off = p * C + c;
  if (dtype == 0) return *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + off);
  if (dtype == 1) {
    const uint2 v = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + off);
    return make_float4(bf16_to_f32(v.x & 0xFFFFu), bf16_to_f32(v.x >> 16), bf16_to_f32(v.y & 0xFFFFu),
                       bf16_to_f32(v.y >> 16));
  }
  const uint32_t v = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(base) + off);
  const float s = scale[p];
  const float4 x = e4m3x4_to_f32(v);
  return make_float4(s * x.x, s * x.y, s * x.z, s * x.w);
}

// Partial channel sums of one (frame, chunk): colsum_chunk (the device
// helpers header); a standalone launch, or workgroups of the mask scan's
// launch for small batches.
template <int TOK>
__global__ __launch_bounds__(256) void k_colsum(Batch b, Work wk) {
  colsum_chunk<TOK>(b, wk, blockIdx.y, blockIdx.x);
}

// mean[f][c] = (sum of the chunk partials in chunk order) / G.  PACK >= 0:
// the rows of the grid past the frames write the projection's k-packed BF16
// copy (PACK = 1: P stored as BF16).
template <int PACK>
__global__ __launch_bounds__(256) void k_mean(Batch b, Work wk, const void* proj, uint4* ppack) {
  if constexpr (PACK >= 0) {
    if ((int)blockIdx.y >= b.n_frames) {
      const int64_t t = ((int64_t)(blockIdx.y - b.n_frames) * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
      pack_proj_chunk<PACK>(proj, b.C, b.E, ppack, t);
      return;
    }
  }
  const int f = blockIdx.y, c = blockIdx.x * 256 + threadIdx.x;
  if (f >= b.dyn[0] || c >= b.C) return;
  frame_mean_channel(b, wk, f, c);
}

// r_p = ||f_p - mean|| over the tokens of a frame.  A thread owns one vector
// of VEC channels (16 or 32 bytes of a token row, as k_colsum reads them)
// and reads it for tpt <= 8 tokens, so its slice of the mean is read once;
// the nthr = min(C / VEC, 256) threads of a token row sit side by side,
// R = 256 / nthr rows of them, so a workgroup covers tpt·R consecutive tokens
// and every 16-byte load instruction of a wavefront reads 1 KB of one or two
// token rows.  The per-thread partial sums of each token are added in thread
// order from LDS.
template <int TOK>
__global__ __launch_bounds__(256) void k_resid(Batch b, Work wk, int tpt) {
  constexpr int VEC = TOK == 2 ? 16 : 8;
  const int f = blockIdx.y;
  if (f >= b.dyn[0]) return;
  const FrameDesc fd = b.frames[f];
  const int G = fd.G, C = b.C;
  const int nch = C / VEC, nthr = min(nch, 256), R = 256 / nthr, ntok = tpt * R;
  const int p0 = blockIdx.x * ntok;
  if (p0 >= G) return;
  const int tid = threadIdx.x, ro = tid / nthr, cl = tid % nthr;
  const float* mu = wk.mean + (int64_t)f * C;
  float ss[8];
  for (int i = 0; i < 8; ++i) ss[i] = 0.f;
  if (ro < R) {
    for (int cg = cl; cg < nch; cg += nthr) {
      const int c = cg * VEC;
      float m[VEC];
      for (int j = 0; j < VEC; j += 4) {
        const float4 q = *reinterpret_cast<const float4*>(mu + c + j);
        m[j] = q.x; m[j + 1] = q.y; m[j + 2] = q.z; m[j + 3] = q.w;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = p0 + ro + R * i;
        if (i < tpt && p < G) {
          float v[VEC];
          load_vec<TOK>(fd.tokens, fd.scale, p, C, c, v);
          for (int j = 0; j < VEC; ++j) {
            const float dd = v[j] - m[j];
            ss[i] += dd * dd;
          }
        }
      }
    }
  }
  __shared__ float part[8 * 256];  // [token of the group][thread of its row]
  if (ro < R)
    for (int i = 0; i < tpt; ++i) part[(ro + R * i) * nthr + cl] = ss[i];
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  for (int t = wv; t < ntok; t += 4) {
    float x = 0.f;
    for (int k = lane; k < nthr; k += 64) x += part[t * nthr + k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0 && p0 + t < G) wk.r[fd.r_base + p0 + t] = __builtin_sqrtf(x);
  }
}

// token rows side by side in a k_resid workgroup
inline int resid_rows(int C, int tok_dtype) { return 256 / std::min(C / (tok_dtype == 2 ? 16 : 8), 256); }

// Token statistics of every frame: chunk partial sums, the frame mean, then r.
void launch_token_stats(const Batch& b, const Work& w, int gmax, hipStream_t st, bool colsum_done,
                        const void* pack_proj, int proj_bf16, bool mean_done) {
  const dim3 cgrid(b.nchunk, b.n_frames);
  if (colsum_done) {
  } else if (b.tok_dtype == 0) {
    hipLaunchKernelGGL(k_colsum<0>, cgrid, dim3(256), 0, st, b, w);
  } else if (b.tok_dtype == 1) {
    hipLaunchKernelGGL(k_colsum<1>, cgrid, dim3(256), 0, st, b, w);
  } else {
    hipLaunchKernelGGL(k_colsum<2>, cgrid, dim3(256), 0, st, b, w);
  }
  const int mx = (b.C + 255) / 256;
  uint4* pp = reinterpret_cast<uint4*>(w.ppack);
  if (mean_done) {
  } else if (!pack_proj) {
    hipLaunchKernelGGL(k_mean<-1>, dim3(mx, b.n_frames), dim3(256), 0, st, b, w, nullptr, nullptr);
  } else {
    const int64_t np = (int64_t)(b.C / 8) * b.E, row = (int64_t)mx * 256;
    const dim3 mg(mx, b.n_frames + (unsigned)((np + row - 1) / row));
    if (proj_bf16) hipLaunchKernelGGL(k_mean<1>, mg, dim3(256), 0, st, b, w, pack_proj, pp);
    else hipLaunchKernelGGL(k_mean<0>, mg, dim3(256), 0, st, b, w, pack_proj, pp);
  }
  // 8 tokens per thread, fewer where that would leave under 1024 workgroups
  const int R = resid_rows(b.C, b.tok_dtype);
  int tpt = 8;
  while (tpt > 1 && (int64_t)((gmax + tpt * R - 1) / (tpt * R)) * b.n_frames < 1024) tpt /= 2;
  const dim3 rgrid((gmax + tpt * R - 1) / (tpt * R), b.n_frames);
  if (b.tok_dtype == 2) hipLaunchKernelGGL(k_resid<2>, rgrid, dim3(256), 0, st, b, w, tpt);
  else if (b.tok_dtype == 1) hipLaunchKernelGGL(k_resid<1>, rgrid, dim3(256), 0, st, b, w, tpt);
  else hipLaunchKernelGGL(k_resid<0>, rgrid, dim3(256), 0, st, b, w, tpt);
}

// D = r / (mean(r) + eps) for one frame (stage entry point only).
__global__ __launch_bounds__(1024) void k_d_from_r(const float* r, int G, float eps, float* D) {
  __shared__ float red[16];
  float a = 0.f;
  for (int p = threadIdx.x; p < G; p += 1024) a += r[p];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  float tot = 0.f;
  for (int i = 0; i < 16; ++i) tot += red[i];
  const float denom = tot / (float)G + eps;
  for (int p = threadIdx.x; p < G; p += 1024) D[p] = r[p] / denom;
}

void launch_d_from_r(const float* r, int G, float eps, float* D, hipStream_t st) {
  hipLaunchKernelGGL(k_d_from_r, dim3(1), dim3(1024), 0, st, r, G, eps, D);
}

// Mean of r per frame, for the frames that ask for the mean distinctiveness
// of their masks (one workgroup per frame, fixed summation order).
__global__ __launch_bounds__(256) void k_rbar(Batch b, Work wk) {
  const int f = blockIdx.x;
  if (f >= b.dyn[0]) return;
  const FrameDesc fd = b.frames[f];
  if (!fd.dbar) return;
  const float* r = wk.r + fd.r_base;
  float a = 0.f;
  for (int p = threadIdx.x; p < fd.G; p += 256) a += r[p];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) wk.rbar[f] = (((red[0] + red[1]) + red[2]) + red[3]) / (float)fd.G;
}

void launch_rbar(const Batch& b, const Work& w, hipStream_t st) {
  if (b.n_frames > 0) hipLaunchKernelGGL(k_rbar, dim3(b.n_frames), dim3(256), 0, st, b, w);
}

// ---------------------------------------------------------------------------
// Weight finalisation, one workgroup per mask.
//   w_p = s_p * r_p (distinct) or s_p, times scale_p for FP8 tokens (the GEMM
//   then multiplies the raw e4m3 codes), rounded to the GEMM operand type and
//   written as a dense row (zeros outside the mask's patch rectangle).
//   Z = sum of the rounded weights (per token value: w_p / scale_p for FP8) in
//   compensated (Neumaier) FP32 summation.  Z == 0 with a non-empty mask and
//   distinctiveness on (every touched patch equals the frame mean) falls back
//   to w = s.
// ---------------------------------------------------------------------------
struct Neu {
  float s, c;
};
__device__ __forceinline__ void neu_add(Neu& a, float x) {
  const float t = a.s + x;
  if (fabsf(a.s) >= fabsf(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ Neu neu_merge(Neu a, Neu b) {
  neu_add(a, b.s);
  a.c += b.c;
  return a;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);  // finite, non-negative weights only
}

// The term a weight adds to Z, in token-value units: the rounded GEMM operand,
// divided by the token's scale for FP8 tokens.  A token whose scale is 0 (an
// all-zero token) adds nothing to the pooled sum, but its weight still counts
// in Z, as in the FP64 definition: the unscaled weight, rounded like an
// operand.
template <int BF16>
__device__ __forceinline__ float z_term(float wr, float wu, bool fp8, float sc) {
  if (!fp8) return wr;
  if (sc != 0.f) return wr / sc;
  return BF16 ? __uint_as_float((uint32_t)f32_to_bf16_rne(wu) << 16) : wu;
}

// The GEMM weights of one mask: a dense row of Gs elements (G rounded up to
// 8), the weight inside the mask's patch rectangle and exact zeros elsewhere,
// stored 8 elements at a time (the pooling GEMM loads whole 8-element chunks
// and needs no masking).  Chunks outside the rectangle are plain zero stores.
template <int BF16>
__device__ float write_row(const Batch& b, const Work& wk, const FrameDesc& fd, int64_t rowoff, int pr0, int pr1,
                           int pc0, int pc1, bool use_r, Neu& z, float& ssum) {
  const int gw = fd.gw, G = fd.G, nch = fd.Gs / 8;
  const bool fp8 = b.tok_dtype == 2;
  const float* r = wk.r + fd.r_base;
  const int rlo = pr1 >= pr0 ? pr0 * gw + pc0 : G, rhi = pr1 >= pr0 ? pr1 * gw + pc1 : -1;
  for (int c = threadIdx.x; c < nch; c += 256) {
    const int p0 = 8 * c;
    float wv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) wv[e] = 0.f;
    if (p0 <= rhi && p0 + 7 >= rlo) {
      // every load of the chunk first (in bounds: the row holds Gs >= p0 + 8
      // elements, r and the scales G), then the elements inside the rectangle
      const float4* sp = reinterpret_cast<const float4*>(wk.s + rowoff + p0);
      const float4 sa = sp[0], sb = sp[1];
      const float s8[8] = {sa.x, sa.y, sa.z, sa.w, sb.x, sb.y, sb.z, sb.w};
      float r8[8], c8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int p = min(p0 + e, G - 1);
        r8[e] = use_r ? r[p] : 1.f;
        c8[e] = fp8 ? fd.scale[p] : 1.f;
      }
      int pr = p0 / gw, pc = p0 - pr * gw;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int p = p0 + e;
        if (p < G && pr >= pr0 && pr <= pr1 && pc >= pc0 && pc <= pc1) {
          const float sv = s8[e];
          ssum += sv;
          const float wu = use_r ? sv * r8[e] : sv;
          const float sc = c8[e];
          float w = fp8 ? wu * sc : wu;
          if (BF16) w = __uint_as_float((uint32_t)f32_to_bf16_rne(w) << 16);
          wv[e] = w;
          const float zt = z_term<BF16>(w, wu, fp8, sc);
          if (zt != 0.f) neu_add(z, zt);
        }
        if (++pc == gw) {
          pc = 0;
          ++pr;
        }
      }
    }
    if (BF16) {
      uint32_t h[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) h[e] = (__float_as_uint(wv[2 * e]) >> 16) | (__float_as_uint(wv[2 * e + 1]) & 0xFFFF0000u);
      *reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(wk.W) + rowoff + p0) = make_uint4(h[0], h[1], h[2], h[3]);
    } else {
      float4* dst = reinterpret_cast<float4*>(reinterpret_cast<float*>(wk.W) + rowoff + p0);
      dst[0] = make_float4(wv[0], wv[1], wv[2], wv[3]);
      dst[1] = make_float4(wv[4], wv[5], wv[6], wv[7]);
    }
  }
  return 0.f;
}

__device__ Neu block_neu(Neu z, float* red) {
  // wave butterfly, then the four waves in order
  for (int o = 32; o > 0; o >>= 1) {
    Neu t;
    t.s = __shfl_xor(z.s, o);
    t.c = __shfl_xor(z.c, o);
    // combine in a lane-independent order so every lane holds the same value
    const int lane = threadIdx.x & 63;
    z = (lane & o) ? neu_merge(t, z) : neu_merge(z, t);
  }
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[wv * 2] = z.s;
    red[wv * 2 + 1] = z.c;
  }
  __syncthreads();
  Neu tot{red[0], red[1]};
  for (int i = 1; i < 4; ++i) tot = neu_merge(tot, Neu{red[2 * i], red[2 * i + 1]});
  return tot;
}

template <int BF16>
__global__ __launch_bounds__(256) void k_weights(Batch b, Work wk) {
  const int g = blockIdx.x;
  if (g >= b.dyn[1]) return;
  const FrameDesc fd = b.frames[b.mask_frame[g]];
  const int64_t rowoff = fd.w_base + (int64_t)(g - fd.mask_base) * fd.Gs;
  const int4 bb = wk.bbox[g];
  const int P = fd.patch;
  int pr0 = bb.x / P, pr1 = bb.y / P, pc0 = bb.z / P, pc1 = bb.w / P;
  const bool empty = bb.x > bb.y;
  if (empty) pr1 = -1;
  __shared__ float red[8];
  __shared__ float ssum_sh[4];
  Neu z{0.f, 0.f};
  float ssum = 0.f;
  write_row<BF16>(b, wk, fd, rowoff, pr0, pr1, pc0, pc1, b.distinct != 0, z, ssum);
  Neu tot = block_neu(z, red);
  for (int o = 32; o > 0; o >>= 1) ssum += __shfl_xor(ssum, o);
  if ((threadIdx.x & 63) == 0) ssum_sh[threadIdx.x >> 6] = ssum;
  __syncthreads();
  const float stot = ssum_sh[0] + ssum_sh[1] + ssum_sh[2] + ssum_sh[3];
  float Z = tot.s + tot.c;
  if (!empty && stot > 0.f && Z == 0.f && b.distinct) {
    __syncthreads();
    Neu z2{0.f, 0.f};
    float s2 = 0.f;
    write_row<BF16>(b, wk, fd, rowoff, pr0, pr1, pc0, pc1, false, z2, s2);
    tot = block_neu(z2, red);
    Z = tot.s + tot.c;
  }
  if (threadIdx.x == 0) {
    wk.Z[g] = Z;
    wk.mstat[g] = wk.fbad[b.mask_frame[g]] ? 3 : (empty || !(stot > 0.f)) ? 1 : 0;
  }
}

// One workgroup per (chunk of tokens, frame): a scale that is NaN, infinite
// or negative flags its frame (its masks then get status 3 and zero rows).
__global__ __launch_bounds__(256) void k_scale_check(Batch b, Work wk) {
  const int f = blockIdx.y;
  if (f >= b.dyn[0]) return;
  const FrameDesc fd = b.frames[f];
  bool bad = false;
  for (int p = blockIdx.x * 256 + threadIdx.x; p < fd.G; p += gridDim.x * 256) {
    const float s = fd.scale[p];
    bad |= !(s >= 0.f && s <= 3.402823466e38f);  // false for NaN, +-inf and negatives
  }
  if (bad) atomicOr(&wk.fbad[f], 1);
}

void launch_scale_check(const Batch& b, const Work& w, int gmax, hipStream_t st) {
  if (b.n_frames <= 0) return;
  hipLaunchKernelGGL(k_scale_check, dim3(std::max(1, std::min(32, (gmax + 255) / 256)), b.n_frames), dim3(256), 0, st,
                     b, w);
}

void launch_weights(const Batch& b, const Work& w, hipStream_t st) {
  if (b.M <= 0) return;
  if (b.gemm_bf16)
    hipLaunchKernelGGL(k_weights<1>, dim3(b.M), dim3(256), 0, st, b, w);
  else
    hipLaunchKernelGGL(k_weights<0>, dim3(b.M), dim3(256), 0, st, b, w);
}

// Stage output of disc_patch_weights: dense w[m][G] = s * D (or s), D from
// Eq. (1) with eps (single frame).
__global__ __launch_bounds__(256) void k_dense_weights(Batch b, Work wk, float* out, float eps) {
  const int g = blockIdx.x;
  if (g >= b.dyn[1]) return;
  const FrameDesc fd = b.frames[b.mask_frame[g]];
  const int G = fd.G, gw = fd.gw, P = fd.patch;
  const int4 bb = wk.bbox[g];
  const bool empty = bb.x > bb.y;
  const int pr0 = bb.x / P, pr1 = bb.y / P, pc0 = bb.z / P, pc1 = bb.w / P;
  const int64_t rowoff = fd.w_base + (int64_t)(g - fd.mask_base) * fd.Gs;
  __shared__ float denom_sh;
  if (b.distinct) {
    __shared__ float red[4];
    float a = 0.f;
    for (int p = threadIdx.x; p < G; p += 256) a += wk.r[fd.r_base + p];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) denom_sh = (red[0] + red[1] + red[2] + red[3]) / (float)G + eps;
    __syncthreads();
  }
  for (int p = threadIdx.x; p < G; p += 256) {
    const int pr = p / gw, pc = p - pr * gw;
    float v = 0.f;
    if (!empty && pr >= pr0 && pr <= pr1 && pc >= pc0 && pc <= pc1) {
      v = wk.s[rowoff + p];
      if (b.distinct) v *= wk.r[fd.r_base + p] / denom_sh;
    }
    out[(int64_t)(g - fd.mask_base) * G + p] = v;
  }
}

void launch_dense_weights(const Batch& b, const Work& w, float* out, float eps, hipStream_t st) {
  if (b.M > 0) hipLaunchKernelGGL(k_dense_weights, dim3(b.M), dim3(256), 0, st, b, w, out, eps);
}

// Caller-given weights (disc_pool_project): copy w[m][G] into the GEMM operand
// (times scale_p for FP8 tokens), Z = compensated sum of the rounded weights,
// status 1 for an all-zero row.  The mask bounding box is set to the whole
// frame so the pooling GEMM visits every patch.
template <int BF16>
__global__ __launch_bounds__(256) void k_user_weights(Batch b, Work wk, const float* wts) {
  const int g = blockIdx.x;
  if (g >= b.dyn[1]) return;
  const FrameDesc fd = b.frames[b.mask_frame[g]];
  const int G = fd.G;
  const int64_t rowoff = fd.w_base + (int64_t)(g - fd.mask_base) * fd.Gs;
  const bool fp8 = b.tok_dtype == 2;
  __shared__ float red[8];
  Neu z{0.f, 0.f};
  for (int p = G + threadIdx.x; p < fd.Gs; p += 256) {  // the row's tail: zeros (the GEMM loads 8 at a time)
    if (BF16) reinterpret_cast<uint16_t*>(wk.W)[rowoff + p] = 0;
    else reinterpret_cast<float*>(wk.W)[rowoff + p] = 0.f;
  }
  for (int p = threadIdx.x; p < G; p += 256) {
    const float wu = wts[(int64_t)(g - fd.mask_base) * G + p];
    const float sc = fp8 ? fd.scale[p] : 1.f;
    const float wv = fp8 ? wu * sc : wu;
    float wr;
    if (BF16) {
      const uint16_t hb = f32_to_bf16_rne(wv);
      reinterpret_cast<uint16_t*>(wk.W)[rowoff + p] = hb;
      wr = __uint_as_float((uint32_t)hb << 16);
    } else {
      reinterpret_cast<float*>(wk.W)[rowoff + p] = wv;
      wr = wv;
    }
    const float zt = z_term<BF16>(wr, wu, fp8, sc);
    if (zt != 0.f) neu_add(z, zt);
  }
  const Neu tot = block_neu(z, red);
  if (threadIdx.x == 0) {
    const float Z = tot.s + tot.c;
    wk.Z[g] = Z;
    wk.mstat[g] = wk.fbad[b.mask_frame[g]] ? 3 : Z > 0.f ? 0 : 1;
    wk.bbox[g] = make_int4(0, fd.h - 1, 0, fd.w - 1);
  }
}

void launch_user_weights(const Batch& b, const Work& w, const float* wts, hipStream_t st) {
  if (b.M <= 0) return;
  if (b.gemm_bf16)
    hipLaunchKernelGGL(k_user_weights<1>, dim3(b.M), dim3(256), 0, st, b, w, wts);
  else
    hipLaunchKernelGGL(k_user_weights<0>, dim3(b.M), dim3(256), 0, st, b, w, wts);
}

}  // namespace disc
