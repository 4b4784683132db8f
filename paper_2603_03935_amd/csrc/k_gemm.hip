// The two dense contractions of DISC's single-pass feature extraction
// (arXiv 2603.03935, Sec. III-C), on MFMA with FP32 accumulation:
//   pooling     X_f = W_f (m_f x G_f) . T_f (G_f x C) / Z, one GEMM per frame
//               (ragged batch: each frame has its own token map);
//   projection  Y = X (M x C) . P (C x E) over all masks of the batch, with the
//               L2 normalisation fused into the epilogue (a workgroup owns
//               complete output rows).
// BF16 operands use v_mfma_f32_32x32x16_bf16, FP32 operands
// v_mfma_f32_32x32x2f32.  FP8 (e4m3fn) tokens are widened exactly to BF16
// while staged into LDS; their per-token scales are already in the weights.
#include "disc_device.h"

namespace disc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even (finite inputs)
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// e4m3fn code -> bf16 bits (exact: every e4m3 value is a bf16 value)
__device__ __forceinline__ uint16_t e4m3_to_bf16(uint32_t code) {
  const uint32_t sign = (code & 0x80u) << 8;
  const uint32_t mag = code & 0x7Fu;
  if (mag == 0x7Fu) return (uint16_t)(sign | 0x7FC0u);
  if (mag >= 8u) return (uint16_t)(sign | ((mag << 4) + (120u << 7)));
  const float v = (float)mag * 0x1p-9f;  // subnormal e4m3 -> normal bf16
  return (uint16_t)(sign | (__float_as_uint(v) >> 16));
}
__device__ __forceinline__ float e4m3_to_f32g(uint32_t code) { return bf2f(e4m3_to_bf16(code)); }

// 8 consecutive elements of a token row as GEMM operands (zero past G)
template <int TOK, int BF16>
__device__ __forceinline__ void load_tok8(const void* base, int64_t off, bool ok, uint16_t* ob, float* of) {
  if (!ok) {
    for (int j = 0; j < 8; ++j) {
      if (BF16) ob[j] = 0; else of[j] = 0.f;
    }
    return;
  }
  if (TOK == 0) {
    const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + off);
    const float4 a = p[0], c = p[1];
    const float v[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
    for (int j = 0; j < 8; ++j) {
      if (BF16) ob[j] = f2bf(v[j]); else of[j] = v[j];
    }
  } else if (TOK == 1) {
    const uint4 a = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(base) + off);
    const uint32_t v[4] = {a.x, a.y, a.z, a.w};
    for (int j = 0; j < 4; ++j) {
      const uint16_t lo = (uint16_t)(v[j] & 0xFFFFu), hi = (uint16_t)(v[j] >> 16);
      if (BF16) { ob[2 * j] = lo; ob[2 * j + 1] = hi; } else { of[2 * j] = bf2f(lo); of[2 * j + 1] = bf2f(hi); }
    }
  } else {
    const uint2 a = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint8_t*>(base) + off);
    for (int j = 0; j < 8; ++j) {
      const uint32_t code = ((j < 4 ? a.x : a.y) >> (8 * (j & 3))) & 0xFFu;
      if (BF16) ob[j] = e4m3_to_bf16(code); else of[j] = e4m3_to_f32g(code);
    }
  }
}

// ---------------------------------------------------------------------------
// pooling: tile 64 masks x 64 channels, K = patches in chunks of 32
// ---------------------------------------------------------------------------
constexpr int PBM = 64, PBN = 64, PBK = 32;

template <int BF16, int TOK>
__global__ __launch_bounds__(256) void k_pool(Batch b, Work wk, const int4* tiles) {
  const int4 t = tiles[blockIdx.x];
  const FrameDesc fd = b.frames[t.x];
  const int m0 = t.y, n0 = t.z, C = b.C;
  const int mrows = min(PBM, fd.m - m0);
  const int G = fd.G;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;

  __shared__ int kmin_sh, kmax_sh;
  __shared__ __attribute__((aligned(16))) uint16_t As16[BF16 ? PBM * (PBK + 8) : 1];
  __shared__ __attribute__((aligned(16))) uint16_t Bs16[BF16 ? PBK * PBN : 1];
  __shared__ float As32[BF16 ? 1 : PBM * (PBK + 1)];
  __shared__ __attribute__((aligned(16))) float Bs32[BF16 ? 1 : PBK * PBN];

  if (tid == 0) {
    kmin_sh = INT32_MAX;
    kmax_sh = 0;
  }
  __syncthreads();
  if (tid < mrows) {
    const int4 bb = wk.bbox[fd.mask_base + m0 + tid];
    if (bb.x <= bb.y) {
      atomicMin(&kmin_sh, (bb.x / fd.patch) * fd.gw);
      atomicMax(&kmax_sh, (bb.y / fd.patch + 1) * fd.gw);
    }
  }
  __syncthreads();
  const int kbeg = (kmin_sh / PBK) * PBK, kend = min(kmax_sh, G);

  floatx16 acc;
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;

  const int64_t wrow0 = fd.w_base + (int64_t)m0 * fd.Gs;
  // A loader: row tid/4, 8 consecutive k at (tid%4)*8
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  // B loader: k row tid/8, 8 consecutive channels at (tid%8)*8
  const int bk = tid >> 3, bn = (tid & 7) * 8;

  for (int k0 = kbeg; k0 < kend; k0 += PBK) {
    // ---- stage A (weights) ----
    {
      const int kk = k0 + ak;
      const bool rok = ar < mrows;
      if (BF16) {
        const uint16_t* src = reinterpret_cast<const uint16_t*>(wk.W) + wrow0 + (int64_t)ar * fd.Gs + kk;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (rok && kk + 8 <= G) {
          v = *reinterpret_cast<const uint4*>(src);
        } else if (rok) {
          uint16_t tmp[8];
          for (int j = 0; j < 8; ++j) tmp[j] = (kk + j < G) ? src[j] : (uint16_t)0;
          v = make_uint4(tmp[0] | (tmp[1] << 16), tmp[2] | (tmp[3] << 16), tmp[4] | (tmp[5] << 16), tmp[6] | (tmp[7] << 16));
        }
        *reinterpret_cast<uint4*>(&As16[ar * (PBK + 8) + ak]) = v;
      } else {
        const float* src = reinterpret_cast<const float*>(wk.W) + wrow0 + (int64_t)ar * fd.Gs + kk;
        for (int j = 0; j < 8; ++j) As32[ar * (PBK + 1) + ak + j] = (rok && kk + j < G) ? src[j] : 0.f;
      }
    }
    // ---- stage B (tokens) ----
    {
      const int kr = k0 + bk;
      const bool ok = kr < G;
      const int64_t off = (int64_t)kr * C + n0 + bn;
      if (BF16) {
        uint16_t ob[8];
        load_tok8<TOK, 1>(fd.tokens, off, ok, ob, nullptr);
        uint4 v = make_uint4(ob[0] | (ob[1] << 16), ob[2] | (ob[3] << 16), ob[4] | (ob[5] << 16), ob[6] | (ob[7] << 16));
        *reinterpret_cast<uint4*>(&Bs16[bk * PBN + bn]) = v;
      } else {
        float of[8];
        load_tok8<TOK, 0>(fd.tokens, off, ok, nullptr, of);
        *reinterpret_cast<float4*>(&Bs32[bk * PBN + bn]) = make_float4(of[0], of[1], of[2], of[3]);
        *reinterpret_cast<float4*>(&Bs32[bk * PBN + bn + 4]) = make_float4(of[4], of[5], of[6], of[7]);
      }
    }
    __syncthreads();
    // ---- MFMA ----
    const int lr = lane & 31, lk = lane >> 5;
    if (BF16) {
      for (int kk = 0; kk < PBK; kk += 16) {
        const u16x8 av = *reinterpret_cast<const u16x8*>(&As16[(32 * wm + lr) * (PBK + 8) + kk + 8 * lk]);
        u16x8 bv;
        for (int j = 0; j < 8; ++j) bv[j] = Bs16[(kk + 8 * lk + j) * PBN + 32 * wn + lr];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
      }
    } else {
      for (int kk = 0; kk < PBK; kk += 2) {
        const float a = As32[(32 * wm + lr) * (PBK + 1) + kk + lk];
        const float bb = Bs32[(kk + lk) * PBN + 32 * wn + lr];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // ---- epilogue: divide by Z, store X (GEMM dtype) and the optional FP32 pooled output ----
  const int col = n0 + 32 * wn + (lane & 31);
  for (int v = 0; v < 16; ++v) {
    const int r = 32 * wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int mi = m0 + r;
    if (mi >= fd.m) continue;
    const int g = fd.mask_base + mi;
    const float Z = wk.Z[g];
    const float val = (wk.mstat[g] == 0 && Z > 0.f) ? acc[v] / Z : 0.f;
    if (BF16)
      reinterpret_cast<uint16_t*>(wk.X)[(int64_t)g * C + col] = f2bf(val);
    else
      reinterpret_cast<float*>(wk.X)[(int64_t)g * C + col] = val;
    if (fd.pooled) fd.pooled[(int64_t)mi * C + col] = val;
  }
}

void launch_pool(const Batch& b, const Work& w, const int4* tiles, int n_tiles, hipStream_t st) {
  if (n_tiles <= 0) return;
  const dim3 grid(n_tiles), block(256);
  if (b.gemm_bf16) {
    if (b.tok_dtype == 0) hipLaunchKernelGGL((k_pool<1, 0>), grid, block, 0, st, b, w, tiles);
    else if (b.tok_dtype == 1) hipLaunchKernelGGL((k_pool<1, 1>), grid, block, 0, st, b, w, tiles);
    else hipLaunchKernelGGL((k_pool<1, 2>), grid, block, 0, st, b, w, tiles);
  } else {
    if (b.tok_dtype == 0) hipLaunchKernelGGL((k_pool<0, 0>), grid, block, 0, st, b, w, tiles);
    else if (b.tok_dtype == 1) hipLaunchKernelGGL((k_pool<0, 1>), grid, block, 0, st, b, w, tiles);
    else hipLaunchKernelGGL((k_pool<0, 2>), grid, block, 0, st, b, w, tiles);
  }
}

// ---------------------------------------------------------------------------
// projection + L2 normalisation: 32 rows x all E columns per workgroup; each
// wavefront covers E/4 columns as NT tiles of 32 x 32.
// ---------------------------------------------------------------------------
template <int BF16>
struct ProjCfg {
  static constexpr int BK = BF16 ? 32 : 16;
};

template <int BF16, int NT, int PBF16>
__global__ __launch_bounds__(256) void k_proj(Batch b, Work wk, const void* proj) {
  constexpr int BK = ProjCfg<BF16>::BK;
  constexpr int E = NT * 128;
  const int C = b.C;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int gbase = blockIdx.x * 32;
  __shared__ __attribute__((aligned(16))) uint16_t As16[BF16 ? 32 * (BK + 8) : 1];
  __shared__ __attribute__((aligned(16))) uint16_t Bs16[BF16 ? BK * E : 1];
  __shared__ float As32[BF16 ? 1 : 32 * (BK + 1)];
  __shared__ __attribute__((aligned(16))) float Bs32[BF16 ? 1 : BK * E];
  __shared__ float red[4][32];
  __shared__ float* orow[32];
  __shared__ int32_t* srow[32];
  __shared__ int st_in[32];

  if (tid < 32) {
    const int g = gbase + tid;
    if (g < b.M) {
      const FrameDesc& fd = b.frames[b.mask_frame[g]];
      orow[tid] = fd.out + (int64_t)(g - fd.mask_base) * b.E;
      srow[tid] = fd.status ? fd.status + (g - fd.mask_base) : nullptr;
      st_in[tid] = wk.mstat[g];
    } else {
      orow[tid] = nullptr;
      srow[tid] = nullptr;
      st_in[tid] = 1;
    }
  }

  floatx16 acc[NT];
  for (int t = 0; t < NT; ++t)
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;

  const int lr = lane & 31, lk = lane >> 5;
  for (int k0 = 0; k0 < C; k0 += BK) {
    // A: 32 rows x BK of X
    if (BF16) {
      const int r = tid >> 3, kk = (tid & 7) * 4;  // 32 x 32, 4 per thread
      const int g = gbase + r;
      uint2 v = make_uint2(0, 0);
      if (g < b.M) v = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(wk.X) + (int64_t)g * C + k0 + kk);
      *reinterpret_cast<uint2*>(&As16[r * (BK + 8) + kk]) = v;
    } else {
      const int r = tid >> 3, kk = (tid & 7) * 2;  // 32 x 16, 2 per thread
      const int g = gbase + r;
      float2 v = make_float2(0.f, 0.f);
      if (g < b.M) v = *reinterpret_cast<const float2*>(reinterpret_cast<const float*>(wk.X) + (int64_t)g * C + k0 + kk);
      As32[r * (BK + 1) + kk] = v.x;
      As32[r * (BK + 1) + kk + 1] = v.y;
    }
    // B: BK rows x E of P (8 elements per step)
    for (int idx = tid * 8; idx < BK * E; idx += 256 * 8) {
      const int kr = idx / E, cc = idx - kr * E;
      const int64_t off = (int64_t)(k0 + kr) * E + cc;
      if (BF16) {
        if (PBF16) {
          *reinterpret_cast<uint4*>(&Bs16[idx]) = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(proj) + off);
        } else {
          const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(proj) + off);
          const float4 a = p[0], c = p[1];
          *reinterpret_cast<uint4*>(&Bs16[idx]) =
              make_uint4(f2bf(a.x) | (f2bf(a.y) << 16), f2bf(a.z) | (f2bf(a.w) << 16), f2bf(c.x) | (f2bf(c.y) << 16),
                         f2bf(c.z) | (f2bf(c.w) << 16));
        }
      } else {
        if (PBF16) {
          const uint4 a = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(proj) + off);
          const uint32_t v[4] = {a.x, a.y, a.z, a.w};
          for (int j = 0; j < 4; ++j) {
            Bs32[idx + 2 * j] = bf2f((uint16_t)(v[j] & 0xFFFFu));
            Bs32[idx + 2 * j + 1] = bf2f((uint16_t)(v[j] >> 16));
          }
        } else {
          const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(proj) + off);
          *reinterpret_cast<float4*>(&Bs32[idx]) = p[0];
          *reinterpret_cast<float4*>(&Bs32[idx + 4]) = p[1];
        }
      }
    }
    __syncthreads();
    for (int t = 0; t < NT; ++t) {
      const int cb = wv * (E / 4) + 32 * t;
      if (BF16) {
        for (int kk = 0; kk < BK; kk += 16) {
          const u16x8 av = *reinterpret_cast<const u16x8*>(&As16[lr * (BK + 8) + kk + 8 * lk]);
          u16x8 bv;
          for (int j = 0; j < 8; ++j) bv[j] = Bs16[(kk + 8 * lk + j) * E + cb + lr];
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
        }
      } else {
        for (int kk = 0; kk < BK; kk += 2) {
          const float a = As32[lr * (BK + 1) + kk + lk];
          const float bb = Bs32[(kk + lk) * E + cb + lr];
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // ---- L2 normalisation over each row's E columns ----
  float ss[16];
  for (int v = 0; v < 16; ++v) {
    float a = 0.f;
    for (int t = 0; t < NT; ++t) a += acc[t][v] * acc[t][v];
    for (int o = 1; o < 32; o <<= 1) a += __shfl_xor(a, o);
    ss[v] = a;
  }
  if (lr == 0)
    for (int v = 0; v < 16; ++v) red[wv][8 * (v >> 2) + 4 * lk + (v & 3)] = ss[v];
  __syncthreads();
  for (int v = 0; v < 16; ++v) {
    const int r = 8 * (v >> 2) + 4 * lk + (v & 3);
    float* o = orow[r];
    if (o == nullptr) continue;
    const float tot = red[0][r] + red[1][r] + red[2][r] + red[3][r];
    const bool zero = st_in[r] != 0 || !(tot > 0.f);
    const float inv = zero ? 0.f : 1.0f / __builtin_sqrtf(tot);
    for (int t = 0; t < NT; ++t) o[wv * (E / 4) + 32 * t + lr] = acc[t][v] * inv;
  }
  if (tid < 32 && orow[tid] != nullptr && srow[tid] != nullptr) {
    const float tot = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    *srow[tid] = st_in[tid] != 0 ? 1 : (tot > 0.f ? 0 : 2);
  }
}

template <int BF16, int PBF16>
static void launch_proj_t(const Batch& b, const Work& w, const void* proj, hipStream_t st) {
  const dim3 grid((b.M + 31) / 32), block(256);
  switch (b.E / 128) {
    case 1: hipLaunchKernelGGL((k_proj<BF16, 1, PBF16>), grid, block, 0, st, b, w, proj); break;
    case 2: hipLaunchKernelGGL((k_proj<BF16, 2, PBF16>), grid, block, 0, st, b, w, proj); break;
    case 3: hipLaunchKernelGGL((k_proj<BF16, 3, PBF16>), grid, block, 0, st, b, w, proj); break;
    case 4: hipLaunchKernelGGL((k_proj<BF16, 4, PBF16>), grid, block, 0, st, b, w, proj); break;
    case 5: hipLaunchKernelGGL((k_proj<BF16, 5, PBF16>), grid, block, 0, st, b, w, proj); break;
    case 6: hipLaunchKernelGGL((k_proj<BF16, 6, PBF16>), grid, block, 0, st, b, w, proj); break;
    case 7: hipLaunchKernelGGL((k_proj<BF16, 7, PBF16>), grid, block, 0, st, b, w, proj); break;
    default: hipLaunchKernelGGL((k_proj<BF16, 8, PBF16>), grid, block, 0, st, b, w, proj); break;
  }
}

void launch_proj(const Batch& b, const Work& w, const void* proj, int proj_bf16, hipStream_t st) {
  if (b.M <= 0) return;
  if (b.gemm_bf16) {
    if (proj_bf16) launch_proj_t<1, 1>(b, w, proj, st); else launch_proj_t<1, 0>(b, w, proj, st);
  } else {
    if (proj_bf16) launch_proj_t<0, 1>(b, w, proj, st); else launch_proj_t<0, 0>(b, w, proj, st);
  }
}

}  // namespace disc
