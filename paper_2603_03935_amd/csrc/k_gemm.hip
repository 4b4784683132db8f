// The two dense contractions of DISC's single-pass feature extraction
// (arXiv 2603.03935, Sec. III-C), on MFMA with FP32 accumulation:
//   pooling     X_f = W_f (m_f x G_f) . T_f (G_f x C) / Z, one GEMM per frame
//               (ragged batch: each frame has its own token map);
//   projection  Y = X (M x C) . P (C x E) over all masks of the batch, then
//               a row pass applies the L2 normalisation.
// K is accumulated in fixed groups (kPoolKG patches, kProjKG channels) whose
// sums are added in group order.  When a batch has too few tiles to fill the
// GPU, a tile's K groups are spread over several workgroups that store their
// group sums, and a second pass adds them in the same order: the result is the
// same bits either way, so a mask's embedding does not depend on its batch.
// BF16 operands use v_mfma_f32_32x32x16_bf16, FP32 operands
// v_mfma_f32_32x32x2f32.  FP8 (e4m3fn) tokens are widened exactly to BF16
// while staged into LDS; their per-token scales are already in the weights.
#include "disc_device.h"

namespace disc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

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
    const float4 x0 = e4m3x4_to_f32(a.x), x1 = e4m3x4_to_f32(a.y);
    const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    for (int j = 0; j < 8; ++j) {
      if (BF16) ob[j] = (uint16_t)(__float_as_uint(v[j]) >> 16); else of[j] = v[j];  // exact either way
    }
  }
}

// ---------------------------------------------------------------------------
// pooling: tile 64 masks x 64 channels, K = patches in chunks of 32.
// A (weights, k contiguous) is staged row-major; for BF16 operands B is read
// from the caller's [G][C] tokens and transposed into LDS (8 consecutive
// patches of one channel contiguous, BF16; FP8 codes widened exactly by the
// hardware conversion), so the MFMA operand of a lane is one 16-byte LDS
// read.  The next K chunk is fetched into registers while the current one
// is multiplied.  A workgroup may take NT = 1, 2 or 4 adjacent 64-channel
// tiles of the same masks (one A fetch for NT x 64 channels); the tile list,
// the K order and therefore the result do not depend on NT, which the pooling
// autotuner picks per problem shape.
// ---------------------------------------------------------------------------
constexpr int PBM = 64, PBN = 64, PBK = 32;
constexpr int PAS = PBK + 8;  // LDS row stride (elements) of A and B
// B rows (channels) hold the step's 32 patches as four 8-patch chunks; chunk
// c of row r sits at position c ^ ((r >> 4) & 3), so that the staging
// writes (4 channels x 16 patch pairs of a wavefront, rows 80 bytes apart)
// fall in 64 different banks.  The MFMA reads (16 bytes of 8 consecutive
// rows with one chunk) see the same bank pattern as without the swizzle.
__device__ __forceinline__ int bsw(int row, int chunk) { return chunk ^ ((row >> 4) & 3); }

template <int TOK>
__device__ __forceinline__ uint16_t tok_bf16(const void* base, int64_t off) {
  if (TOK == 0) return f2bf(reinterpret_cast<const float*>(base)[off]);
  if (TOK == 1) return reinterpret_cast<const uint16_t*>(base)[off];
  return (uint16_t)(__float_as_uint(e4m3x4_to_f32(reinterpret_cast<const uint8_t*>(base)[off]).x) >> 16);
}

// K range [kbeg, kend) of a tile: the union of its masks' patch-row ranges
// (rows of patches outside every mask's box hold zero weights for all of them).
// Tile row i of a frame holds mask perm[mask_base + i] (masks ordered by the
// first patch row of their box, so that a tile's range is narrow); which masks
// share a tile never changes a mask's result.
__device__ __forceinline__ void tile_krange(const Work& wk, const FrameDesc& fd, int m0, int mrows, int tid,
                                            int* kmin_sh, int* kmax_sh, int& kbeg, int& kend, int kalign = PBK) {
  if (tid == 0) {
    *kmin_sh = INT32_MAX;
    *kmax_sh = 0;
  }
  __syncthreads();
  if (tid < mrows) {
    const int4 bb = wk.bbox[fd.mask_base + wk.perm[fd.mask_base + m0 + tid]];
    if (bb.x <= bb.y) {
      atomicMin(kmin_sh, (bb.x / fd.patch) * fd.gw);
      atomicMax(kmax_sh, (bb.y / fd.patch + 1) * fd.gw);
    }
  }
  __syncthreads();
  kbeg = (*kmin_sh / kalign) * kalign;
  kend = min(*kmax_sh, fd.G);
}

// The tile's rows resolved once (all threads call it; it synchronises):
// (global mask index, index in the frame, Z bits, 1 if the row is stored
// divided by Z else 0), or g = -1 past the frame's masks.
__device__ __forceinline__ void pool_rows(const Work& wk, const FrameDesc& fd, int m0, int tid, int4* rows,
                                          int nrows = PBM) {
  if (tid < nrows) {
    int4 v = make_int4(-1, 0, 0, 0);
    if (m0 + tid < fd.m) {
      const int mi = wk.perm[fd.mask_base + m0 + tid];
      const int g = fd.mask_base + mi;
      const float Z = wk.Z[g];
      v = make_int4(g, mi, __float_as_int(Z), (wk.mstat[g] == 0 && Z > 0.f) ? 1 : 0);
    }
    rows[tid] = v;
  }
  __syncthreads();
}

// divide by Z, store X (GEMM dtype) and the optional FP32 pooled output
template <int BF16>
__device__ __forceinline__ void pool_store(const Work& wk, const FrameDesc& fd, const int4* rows, int n0, int C,
                                           int lane, int wm, int wn, const floatx16& acc) {
  const int col = n0 + 32 * wn + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = 32 * wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int4 rw = rows[r];
    if (rw.x < 0) continue;
    const float val = rw.w ? acc[v] / __int_as_float(rw.z) : 0.f;
    if (BF16)
      reinterpret_cast<uint16_t*>(wk.X)[(int64_t)rw.x * C + col] = f2bf(val);
    else
      reinterpret_cast<float*>(wk.X)[(int64_t)rw.x * C + col] = val;
    if (fd.pooled) fd.pooled[(int64_t)rw.y * C + col] = val;
  }
}

// grid: (tiles / NT) x S; workgroup (super-tile, s) takes the s-th share of the
// K groups of NT adjacent tiles.  MW = 2: 128 masks (the tile and the next
// mask tile of its frame, its partner, whose tiles are C / 64 entries later in
// the list) share each token chunk, which halves the token reads; the
// partner's own workgroups return at once.  Every mask row sees the same K
// steps and group folds either way, so the bits do not depend on MW.
template <int BF16, int TOK, int NT, int MW>
__global__ __launch_bounds__(256) void k_pool(Batch b, Work wk, const int4* tiles) {
  constexpr int BN = PBN * NT;  // channels per workgroup
  // K step: 64 patches with BF16 operands (two A chunks and two token
  // passes per thread), 32 with FP32 operands
  constexpr int KS = BF16 ? 2 * PBK : PBK, KP = KS + 8, NKS = KS / PBK;
  const int S = MW == 1 ? b.pool_split : 1;
  const int nlive = b.dyn[2] / NT * S;  // live workgroups (NT divides the channel tiles of a mask tile)
  if ((int)blockIdx.x >= nlive) return;
  // without split K, one XCD takes consecutive super-tiles (the channel tiles
  // of one mask tile share its weight rows through that XCD's L2; 16 frames
  // of 1080p with 500 masks each: pooling 0.44 -> 0.29 ms); split launches
  // (small batches) keep the plain
  // order, which measured faster for them
  const int vb = S == 1 ? xcd_remap(blockIdx.x, nlive) : (int)blockIdx.x;
  const int stix = vb / S, sidx = vb - stix * S;
  const int tix = stix * NT;  // first 64-channel tile
  const int4 t = tiles[tix];
  if (MW == 2 && t.w < 0) return;  // the second half of a 128-mask tile
  const FrameDesc fd = b.frames[t.x];
  const int m0 = t.y, n0 = t.z, C = b.C;
  const int mrows = min(PBM * MW, fd.m - m0);
  const int G = fd.G;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;

  __shared__ int kmin_sh, kmax_sh;
  __shared__ __attribute__((aligned(16))) uint16_t As16[BF16 ? PBM * MW * KP : 1];
  __shared__ __attribute__((aligned(16))) uint16_t Bs16[BF16 ? BN * KP : 1];
  __shared__ float As32[BF16 ? 1 : PBM * MW * (PBK + 1)];
  __shared__ __attribute__((aligned(16))) float Bs32[BF16 ? 1 : PBK * BN];

  int kbeg, kend;
  tile_krange(wk, fd, m0, mrows, tid, &kmin_sh, &kmax_sh, kbeg, kend, KS);
  const int gbeg = kbeg / kPoolKG, gend = kbeg < kend ? (kend + kPoolKG - 1) / kPoolKG : gbeg;
  const int per = (gend - gbeg + S - 1) / S;
  const int ga = gbeg + sidx * per, gb = min(gend, ga + per);
  const int kstart = max(kbeg, ga * kPoolKG), kstop = min(kend, gb * kPoolKG);
  if (S > 1 && sidx == 0 && tid <= PBM) {
    // for the reduce pass: the tiles' K groups and rows (no wait here)
    int4 v = make_int4(gbeg, gend, 0, 0);
    if (tid < PBM) {
      v = make_int4(-1, 0, 0, 0);
      if (m0 + tid < fd.m) {
        const int mi = wk.perm[fd.mask_base + m0 + tid];
        const int g = fd.mask_base + mi;
        const float Z = wk.Z[g];
        v = make_int4(g, mi, __float_as_int(Z), (wk.mstat[g] == 0 && Z > 0.f) ? 1 : 0);
      }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) wk.ptile[(int64_t)(tix + j) * (PBM + 1) + (tid < PBM ? 1 + tid : 0)] = v;
  }

  const floatx16 zero16 = {};
  floatx16 total[MW][NT], acc[MW][NT];
#pragma unroll
  for (int h = 0; h < MW; ++h)
#pragma unroll
    for (int j = 0; j < NT; ++j) total[h][j] = acc[h][j] = zero16;

  const int ar = tid >> 2, ak = (tid & 3) * 8;        // A: rows ar (+ 64 h), first k of 8
  bool arow_ok[MW];
  int64_t wrow0[MW];
#pragma unroll
  for (int h = 0; h < MW; ++h) {
    arow_ok[h] = ar + 64 * h < mrows;
    wrow0[h] = fd.w_base + (int64_t)(arow_ok[h] ? wk.perm[fd.mask_base + m0 + 64 * h + ar] : 0) * fd.Gs;
  }
  // B (BF16): the caller's [G][C] tokens, patches 2 pp, 2 pp + 1 and
  // channels c4 .. c4 + 3 (+ 64 j) per thread, transposed into LDS as
  // (patch pair, channel) words
  const int bpp = tid >> 4, bc4 = (tid & 15) * 4;
  // B (FP32): patch tid >> 3, channels 8*(tid & 7) + 64 j .. +7
  const int bk32 = tid >> 3, bn32 = (tid & 7) * 8;

  // FP32 operands: two register sets, the loads of step k + 2 PBK are in
  // flight while step k computes (small batches are latency-bound).  BF16:
  // one set, one step ahead (more resident workgroups hide the latency).
  constexpr int DIST = BF16 ? 1 : 2;
  uint4 ra16[2][MW][NKS];
  uint4 rbr[2][NT][NKS][2];  // raw token words of patches 2 pp, 2 pp + 1 (+ 32 per pass): BF16 .xy, FP8 .x
  float ra32[2][MW][8], rb32[2][NT][8];

  auto fetch = [&](int k0, int q) {
    const int kk = k0 + ak;
    // weight rows are Gs (a multiple of 8) long and hold exact zeros outside
    // the mask's patch rectangle
    if (BF16) {
#pragma unroll
      for (int h = 0; h < MW; ++h)
#pragma unroll
        for (int a = 0; a < NKS; ++a) {
          const int ka = kk + PBK * a;
          const uint16_t* src = reinterpret_cast<const uint16_t*>(wk.W) + wrow0[h] + ka;
          ra16[q][h][a] = arow_ok[h] && ka < G ? *reinterpret_cast<const uint4*>(src) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
      for (int a = 0; a < NKS; ++a) {
        const int kb = k0 + PBK * a + 2 * bpp;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (kb + h < G) {
              const int64_t off = (int64_t)(kb + h) * C + n0 + 64 * j + bc4;
              if (TOK == 0) {
                v = *reinterpret_cast<const uint4*>(reinterpret_cast<const float*>(fd.tokens) + off);
              } else if (TOK == 1) {
                const uint2 t2 = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(fd.tokens) + off);
                v.x = t2.x;
                v.y = t2.y;
              } else {
                v.x = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(fd.tokens) + off);
              }
            }
            rbr[q][j][a][h] = v;
          }
        }
      }
    } else {
      // weight rows start on 8 elements (Gs and the frame bases are multiples of 8)
#pragma unroll
      for (int h = 0; h < MW; ++h) {
        const float* src = reinterpret_cast<const float*>(wk.W) + wrow0[h] + kk;
        if (arow_ok[h] && kk < G) {
          const float4 x = reinterpret_cast<const float4*>(src)[0], y = reinterpret_cast<const float4*>(src)[1];
          ra32[q][h][0] = x.x; ra32[q][h][1] = x.y; ra32[q][h][2] = x.z; ra32[q][h][3] = x.w;
          ra32[q][h][4] = y.x; ra32[q][h][5] = y.y; ra32[q][h][6] = y.z; ra32[q][h][7] = y.w;
        } else {
          for (int j = 0; j < 8; ++j) ra32[q][h][j] = 0.f;
        }
      }
      const int kr = k0 + bk32;
#pragma unroll
      for (int j = 0; j < NT; ++j) load_tok8<TOK, 0>(fd.tokens, (int64_t)kr * C + n0 + bn32 + 64 * j, kr < G, nullptr, rb32[q][j]);
    }
  };
  auto stage = [&](int q) {
    if (BF16) {
#pragma unroll
      for (int h = 0; h < MW; ++h)
#pragma unroll
        for (int a = 0; a < NKS; ++a) *reinterpret_cast<uint4*>(&As16[(ar + 64 * h) * KP + ak + PBK * a]) = ra16[q][h][a];
#pragma unroll
      for (int a = 0; a < NKS; ++a)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        // channel bc4 + e: patches 2 pp and 2 pp + 1 as one word (BF16 bits)
        uint32_t wd[4];
        const int pp = bpp + (PBK / 2) * a;  // patch pair within the step
        const uint4 v0 = rbr[q][j][a][0], v1 = rbr[q][j][a][1];
        if (TOK == 0) {
          const uint32_t a[4] = {v0.x, v0.y, v0.z, v0.w}, c[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) wd[e] = f2bf(__uint_as_float(a[e])) | ((uint32_t)f2bf(__uint_as_float(c[e])) << 16);
        } else if (TOK == 1) {
          wd[0] = __builtin_amdgcn_perm(v1.x, v0.x, 0x05040100u);
          wd[1] = __builtin_amdgcn_perm(v1.x, v0.x, 0x07060302u);
          wd[2] = __builtin_amdgcn_perm(v1.y, v0.y, 0x05040100u);
          wd[3] = __builtin_amdgcn_perm(v1.y, v0.y, 0x07060302u);
        } else {
          // e4m3fn codes: exact floats, whose upper halves are the BF16 bits
          const float4 x0 = e4m3x4_to_f32(v0.x), x1 = e4m3x4_to_f32(v1.x);
          wd[0] = __builtin_amdgcn_perm(__float_as_uint(x1.x), __float_as_uint(x0.x), 0x07060302u);
          wd[1] = __builtin_amdgcn_perm(__float_as_uint(x1.y), __float_as_uint(x0.y), 0x07060302u);
          wd[2] = __builtin_amdgcn_perm(__float_as_uint(x1.z), __float_as_uint(x0.z), 0x07060302u);
          wd[3] = __builtin_amdgcn_perm(__float_as_uint(x1.w), __float_as_uint(x0.w), 0x07060302u);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 64 * j + bc4 + e;
          *reinterpret_cast<uint32_t*>(&Bs16[row * KP + bsw(row, pp >> 2) * 8 + ((2 * pp) & 7)]) = wd[e];
        }
      }
    } else {
#pragma unroll
      for (int h = 0; h < MW; ++h)
        for (int j = 0; j < 8; ++j) As32[(ar + 64 * h) * (PBK + 1) + ak + j] = ra32[q][h][j];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        *reinterpret_cast<float4*>(&Bs32[bk32 * BN + bn32 + 64 * j]) = make_float4(rb32[q][j][0], rb32[q][j][1], rb32[q][j][2], rb32[q][j][3]);
        *reinterpret_cast<float4*>(&Bs32[bk32 * BN + bn32 + 64 * j + 4]) = make_float4(rb32[q][j][4], rb32[q][j][5], rb32[q][j][6], rb32[q][j][7]);
      }
    }
  };
  // a finished K group: add it to the running total, or store it for the reduce pass
  auto fold = [&](int grp) {
#pragma unroll
    for (int h = 0; h < MW; ++h)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        if (S == 1) {
          total[h][j] += acc[h][j];
        } else {
          // sub-tile j of this wavefront lies in 64-channel tile tix + j (MW = 1)
          float4* dst = reinterpret_cast<float4*>(wk.ppart + (((int64_t)(tix + j) * b.kgroups + grp) * (PBM * PBN)) + tid * 16);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            dst[i] = make_float4(acc[h][j][4 * i], acc[h][j][4 * i + 1], acc[h][j][4 * i + 2], acc[h][j][4 * i + 3]);
        }
        acc[h][j] = zero16;
      }
  };

  const int lr = lane & 31, lk = lane >> 5;
  // K groups of this share, each folded once, in order
  int cur = ga;
  auto advance = [&](int g) {
    while (cur < g) {
      fold(cur);
      ++cur;
    }
  };
  // one K step on register set q; kf: the step to fetch into q meanwhile
  auto step = [&](int k0, int q, int kf) {
    advance(k0 / kPoolKG);
    stage(q);
    __syncthreads();
    if (kf < kstop) fetch(kf, q);
    if (BF16) {
#pragma unroll
      for (int kk = 0; kk < KS; kk += 16) {
        u16x8 av[MW];
#pragma unroll
        for (int h = 0; h < MW; ++h) av[h] = *reinterpret_cast<const u16x8*>(&As16[(64 * h + 32 * wm + lr) * KP + kk + 8 * lk]);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int row = 64 * j + 32 * wn + lr;
          const u16x8 bv = *reinterpret_cast<const u16x8*>(&Bs16[row * KP + bsw(row, (kk >> 3) + lk) * 8]);
#pragma unroll
          for (int h = 0; h < MW; ++h)
            acc[h][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[h]),
                                                                __builtin_bit_cast(bf16x8, bv), acc[h][j], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < PBK; kk += 2) {
        float a[MW];
#pragma unroll
        for (int h = 0; h < MW; ++h) a[h] = As32[(64 * h + 32 * wm + lr) * (PBK + 1) + kk + lk];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const float bb = Bs32[(kk + lk) * BN + 64 * j + 32 * wn + lr];
#pragma unroll
          for (int h = 0; h < MW; ++h) acc[h][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[h], bb, acc[h][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  };
  if (kstart < kstop) fetch(kstart, 0);
  if (DIST == 2) {
    if (kstart + PBK < kstop) fetch(kstart + PBK, 1);
    for (int k0 = kstart; k0 < kstop; k0 += 2 * PBK) {
      step(k0, 0, k0 + 2 * PBK);
      if (k0 + PBK >= kstop) break;
      step(k0 + PBK, 1, k0 + 3 * PBK);
    }
  } else {
    for (int k0 = kstart; k0 < kstop; k0 += KS) step(k0, 0, k0 + KS);
  }
  advance(gb);
  if (S == 1) {
    __shared__ int4 rows[PBM * MW];
    pool_rows(wk, fd, m0, tid, rows, PBM * MW);
#pragma unroll
    for (int h = 0; h < MW; ++h)
#pragma unroll
      for (int j = 0; j < NT; ++j) pool_store<BF16>(wk, fd, rows + 64 * h, n0 + 64 * j, C, lane, wm, wn, total[h][j]);
  }
}

// split K: add each tile's stored group sums in group order, then store
template <int BF16>
__global__ __launch_bounds__(256) void k_pool_reduce(Batch b, Work wk, const int4* tiles) {
  const int tix = blockIdx.x;
  if (tix >= b.dyn[2]) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
  // the tile's K groups and rows, as the first share of the split pass wrote them
  const int4* info = wk.ptile + (int64_t)tix * (PBM + 1);
  __shared__ int4 rows[PBM];
  if (tid < PBM) rows[tid] = info[1 + tid];
  const int4 kr = info[0];
  const int4 t = tiles[tix];
  floatx16 total = {};
  const float* gpart = wk.ppart + ((int64_t)tix * b.kgroups) * (PBM * PBN) + tid * 16;
  for (int grp = kr.x; grp < kr.y; ++grp) {
    const float4* src = reinterpret_cast<const float4*>(gpart + (int64_t)grp * (PBM * PBN));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 v = src[i];
      total[4 * i] += v.x;
      total[4 * i + 1] += v.y;
      total[4 * i + 2] += v.z;
      total[4 * i + 3] += v.w;
    }
  }
  __syncthreads();
  pool_store<BF16>(wk, b.frames[t.x], rows, t.z, b.C, lane, wm, wn, total);
}

template <int BF16, int TOK>
static void launch_pool_t(const Batch& b, const Work& w, const int4* tiles, int nt, int mw, hipStream_t st) {
  const dim3 block(256);
  const int S = mw == 2 ? 1 : b.pool_split;
  if (mw == 2) {
    if (nt == 2)
      hipLaunchKernelGGL((k_pool<BF16, TOK, 2, 2>), dim3(b.n_tiles / 2), block, 0, st, b, w, tiles);
    else
      hipLaunchKernelGGL((k_pool<BF16, TOK, 1, 2>), dim3(b.n_tiles), block, 0, st, b, w, tiles);
    return;
  }
  if (nt == 4)
    hipLaunchKernelGGL((k_pool<BF16, TOK, 4, 1>), dim3(b.n_tiles / 4 * S), block, 0, st, b, w, tiles);
  else if (nt == 2)
    hipLaunchKernelGGL((k_pool<BF16, TOK, 2, 1>), dim3(b.n_tiles / 2 * S), block, 0, st, b, w, tiles);
  else
    hipLaunchKernelGGL((k_pool<BF16, TOK, 1, 1>), dim3(b.n_tiles * S), block, 0, st, b, w, tiles);
  if (S > 1) hipLaunchKernelGGL((k_pool_reduce<BF16>), dim3(b.n_tiles), block, 0, st, b, w, tiles);
}

// NT must divide C / 64 (the tiles of one mask tile are consecutive in the list)
bool pool_nt_valid(int C, int nt) { return nt == 1 || ((C / 64) % nt == 0); }

void launch_pool(const Batch& b, const Work& w, const int4* tiles, hipStream_t st, int nt, int mw) {
  if (b.n_tiles <= 0) return;
  if (!pool_nt_valid(b.C, nt)) nt = 1;
  if (mw == 2 && nt > 2) nt = 2;
  if (b.gemm_bf16) {
    if (b.tok_dtype == 0) launch_pool_t<1, 0>(b, w, tiles, nt, mw, st);
    else if (b.tok_dtype == 1) launch_pool_t<1, 1>(b, w, tiles, nt, mw, st);
    else launch_pool_t<1, 2>(b, w, tiles, nt, mw, st);
  } else {
    if (b.tok_dtype == 0) launch_pool_t<0, 0>(b, w, tiles, nt, mw, st);
    else if (b.tok_dtype == 1) launch_pool_t<0, 1>(b, w, tiles, nt, mw, st);
    else launch_pool_t<0, 2>(b, w, tiles, nt, mw, st);
  }
}

// ---------------------------------------------------------------------------
// projection with FP32 operands: tile 32 rows x 128 columns (4 wavefronts of
// 32 x 32, v_mfma_f32_32x32x2f32), K = C in groups of kProjKG channels.  grid:
// (row tiles x S, E / 128).  With S = 1 the workgroup writes the
// unnormalised rows; otherwise each writes its groups' sums to qpart and
// k_norm adds them in group order.  (BF16 operands: k_proj_bf16.)  PBF16: P
// is stored as BF16 (widened exactly).
// ---------------------------------------------------------------------------
template <int PBF16>
__global__ __launch_bounds__(256) void k_proj(Batch b, Work wk, const void* proj) {
  constexpr int BK = 16;
  const int C = b.C, E = b.E, S = b.proj_split;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rt = blockIdx.x / S, sidx = blockIdx.x - rt * S;
  const int gbase = rt * 32, c0 = blockIdx.y * 128;
  const int M = b.dyn[1];
  if (gbase >= M) return;
  const int ngr = (C + kProjKG - 1) / kProjKG;
  const int per = (ngr + S - 1) / S;
  const int ga = sidx * per, gb = min(ngr, ga + per);
  const int kstart = ga * kProjKG, kstop = min(C, gb * kProjKG);
  __shared__ float As32[32 * (BK + 1)];
  __shared__ __attribute__((aligned(16))) float Bs32[BK * 128];

  const floatx16 zero16 = {};
  floatx16 total = zero16, acc = zero16;

  // A loaders: 32 rows x 16 k (2 per thread); B loaders: [k][col] (k tid >> 4, 8 columns)
  const int ar = tid >> 3, ak = (tid & 7) * 2;
  const int ga_row = gbase + ar;
  const int bk32 = tid >> 4, bc32 = (tid & 15) * 8;
  float2 ra32 = make_float2(0.f, 0.f);
  float rb32[8];

  auto fetch = [&](int k0) {
    ra32 = ga_row < M ? *reinterpret_cast<const float2*>(reinterpret_cast<const float*>(wk.X) + (int64_t)ga_row * C + k0 + ak)
                      : make_float2(0.f, 0.f);
    const int64_t off = (int64_t)(k0 + bk32) * E + c0 + bc32;
    if (PBF16) {
      const uint4 a = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(proj) + off);
      const uint32_t v[4] = {a.x, a.y, a.z, a.w};
      for (int j = 0; j < 4; ++j) {
        rb32[2 * j] = bf2f((uint16_t)(v[j] & 0xFFFFu));
        rb32[2 * j + 1] = bf2f((uint16_t)(v[j] >> 16));
      }
    } else {
      const float4* q = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(proj) + off);
      const float4 a = q[0], c = q[1];
      rb32[0] = a.x; rb32[1] = a.y; rb32[2] = a.z; rb32[3] = a.w;
      rb32[4] = c.x; rb32[5] = c.y; rb32[6] = c.z; rb32[7] = c.w;
    }
  };
  auto stage = [&]() {
    As32[ar * (BK + 1) + ak] = ra32.x;
    As32[ar * (BK + 1) + ak + 1] = ra32.y;
    *reinterpret_cast<float4*>(&Bs32[bk32 * 128 + bc32]) = make_float4(rb32[0], rb32[1], rb32[2], rb32[3]);
    *reinterpret_cast<float4*>(&Bs32[bk32 * 128 + bc32 + 4]) = make_float4(rb32[4], rb32[5], rb32[6], rb32[7]);
  };
  const int lr = lane & 31, lk = lane >> 5;
  const int col = c0 + 32 * wv + lr;
  auto fold = [&](int grp) {
    if (S == 1) {
      total += acc;
    } else {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int g = gbase + 8 * (v >> 2) + 4 * lk + (v & 3);
        if (g < M) wk.qpart[((int64_t)grp * b.M + g) * E + col] = acc[v];
      }
    }
    acc = zero16;
  };

  int cur = kstart / kProjKG;
  if (kstart < kstop) fetch(kstart);
  for (int k0 = kstart; k0 < kstop; k0 += BK) {
    if (k0 / kProjKG != cur) {
      fold(cur);
      cur = k0 / kProjKG;
    }
    stage();
    __syncthreads();
    if (k0 + BK < kstop) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const float a = As32[lr * (BK + 1) + kk + lk];
      const float bb = Bs32[(kk + lk) * 128 + 32 * wv + lr];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bb, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if (kstart < kstop) fold(cur);
  if (S > 1) return;
  // ---- store the unnormalised rows (row pointers resolved once per tile) ----
  __shared__ float* rowp[32];
  if (tid < 32) {
    const int g = gbase + tid;
    float* p = nullptr;
    if (g < M) {
      const FrameDesc& fd = b.frames[b.mask_frame[g]];
      p = fd.out + (int64_t)(g - fd.mask_base) * E;
    }
    rowp[tid] = p;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = 8 * (v >> 2) + 4 * lk + (v & 3);
    if (gbase + r < M) rowp[r][col] = total[v];
  }
}

// ---------------------------------------------------------------------------
// BF16 projection, large tiles: 128 rows x 128 columns per workgroup, 4
// wavefronts of 64 x 64 (2 x 2 MFMA 32x32x16 tiles each).  A = X rows (k
// contiguous), B = a k-packed copy of P ([C/8][E][8], written by
// k_pack_proj: 8 consecutive k of one column in 16 bytes), both staged in LDS
// as [row][k] / [column][k] so every load is 16 bytes.  Each element adds
// its k in fixed order within fixed K groups (kProjKG channels) and the group
// sums in group order, whether one workgroup runs the whole K or the groups
// are split over several (then k_norm adds them): the same bits either way.
// ---------------------------------------------------------------------------
template <int PBF16>
__global__ __launch_bounds__(256) void k_pack_proj(const void* proj, int C, int E, uint4* ppack) {
  pack_proj_chunk<PBF16>(proj, C, E, ppack, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// TM x TN output tile per workgroup, each wavefront (TM / 2) x (TN / 2) as
// MI x NJ MFMA tiles of 32 x 32.  64 x 64 tiles (51 KB of LDS, three
// workgroups per CU) measured faster than 128 x 128 ones (136 KB, one per
// CU) at every batch size measured (3749 masks: 44 -> 34 us, 8000 masks:
// 91 -> 82 us); every
// output element sees the same MFMA K steps and K groups with either shape.
template <int TM, int TN>
__global__ __launch_bounds__(256) void k_proj_bf16(Batch b, Work wk) {
  constexpr int BK = 128, AS = BK + 8, MI = TM / 64, NJ = TN / 64;
  constexpr int NA = TM * (BK / 8) / 256, NB = TN * (BK / 8) / 256;  // 16-byte chunks per thread
  const int C = b.C, E = b.E, S = b.proj_split;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
  const int rt = blockIdx.x / S, sidx = blockIdx.x - rt * S;
  const int gbase = rt * TM, c0 = blockIdx.y * TN;
  const int M = b.dyn[1];
  if (gbase >= M) return;
  const int ngr = (C + kProjKG - 1) / kProjKG;
  const int per = (ngr + S - 1) / S;
  const int ga = sidx * per, gb = min(ngr, ga + per);
  const int kstart = ga * kProjKG, kstop = min(C, gb * kProjKG);
  __shared__ __attribute__((aligned(16))) uint16_t As[TM * AS];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN * AS];
  // running sum of the K groups (unsplit K), one float4 slot set per thread:
  // slot (4 (NJ i + j) + v / 4) of thread t at [slot][t]
  __shared__ float4 Ts[4 * MI * NJ * 256];

  const floatx16 zero16 = {};
  floatx16 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = zero16;
  if (S == 1)
    for (int t = 0; t < 4 * MI * NJ; ++t) Ts[t * 256 + tid] = make_float4(0.f, 0.f, 0.f, 0.f);

  // loaders, NA / NB chunks of 8 k (16 bytes) per thread: A chunk
  // q = tid + 256 i is row q >> 4, k 8 (q & 15); B chunk q is k group q / TN
  // of column q % TN.  Chunks past the K range (C a multiple of 64 only)
  // load zeros and their MFMAs are skipped.
  const uint16_t* X = reinterpret_cast<const uint16_t*>(wk.X);
  const uint4* pp = reinterpret_cast<const uint4*>(wk.ppack);
  uint4 ra[NA], rb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + 256 * i, r = q >> 4, ka = k0 + 8 * (q & 15);
      ra[i] = gbase + r < M && ka < kstop ? *reinterpret_cast<const uint4*>(X + (int64_t)(gbase + r) * C + ka)
                                          : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + 256 * i, kb = k0 + 8 * (q / TN);
      rb[i] = kb < kstop ? pp[(int64_t)(kb >> 3) * E + c0 + (q % TN)] : make_uint4(0, 0, 0, 0);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int q = tid + 256 * i;
      *reinterpret_cast<uint4*>(&As[(q >> 4) * AS + 8 * (q & 15)]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int q = tid + 256 * i;
      *reinterpret_cast<uint4*>(&Bs[(q % TN) * AS + 8 * (q / TN)]) = rb[i];
    }
  };
  const int lr = lane & 31, lk = lane >> 5;
  auto fold = [&](int grp) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (S == 1) {
#pragma unroll
          for (int v4 = 0; v4 < 4; ++v4) {
            float4& t = Ts[(4 * (NJ * i + j) + v4) * 256 + tid];
            float4 u = t;
            u.x += acc[i][j][4 * v4];
            u.y += acc[i][j][4 * v4 + 1];
            u.z += acc[i][j][4 * v4 + 2];
            u.w += acc[i][j][4 * v4 + 3];
            t = u;
          }
        } else {
          const int col = c0 + (TN / 2) * wn + 32 * j + lr;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int g = gbase + (TM / 2) * wm + 32 * i + 8 * (v >> 2) + 4 * lk + (v & 3);
            if (g < M) wk.qpart[((int64_t)grp * b.M + g) * E + col] = acc[i][j][v];
          }
        }
        acc[i][j] = zero16;
      }
  };

  int cur = kstart / kProjKG;
  if (kstart < kstop) fetch(kstart);
  for (int k0 = kstart; k0 < kstop; k0 += BK) {
    if (k0 / kProjKG != cur) {
      fold(cur);
      cur = k0 / kProjKG;
    }
    stage();
    __syncthreads();
    if (k0 + BK < kstop) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      if (k0 + kk >= kstop) break;
      u16x8 av[MI], bv[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        av[i] = *reinterpret_cast<const u16x8*>(&As[((TM / 2) * wm + 32 * i + lr) * AS + kk + 8 * lk]);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        bv[j] = *reinterpret_cast<const u16x8*>(&Bs[((TN / 2) * wn + 32 * j + lr) * AS + kk + 8 * lk]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[i]),
                                                              __builtin_bit_cast(bf16x8, bv[j]), acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  if (kstart < kstop) fold(cur);
  if (S > 1) return;
  // output row pointers of the tile, resolved once
  __shared__ float* rowp[TM];
  if (tid < TM) {
    const int g = gbase + tid;
    float* p = nullptr;
    if (g < M) {
      const FrameDesc& fd = b.frames[b.mask_frame[g]];
      p = fd.out + (int64_t)(g - fd.mask_base) * E;
    }
    rowp[tid] = p;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int col = c0 + (TN / 2) * wn + 32 * j + lr;
#pragma unroll
      for (int v4 = 0; v4 < 4; ++v4) {
        const float4 t = Ts[(4 * (NJ * i + j) + v4) * 256 + tid];
        const float tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = (TM / 2) * wm + 32 * i + 8 * v4 + 4 * lk + u;
          if (gbase + r < M) rowp[r][col] = tv[u];
        }
      }
    }
}

// One wavefront per row: (split K: add the group sums in group order and)
// normalise.  The sum of squares has a fixed order: each lane sums its columns
// lane*4 + 256 i in order, then a fixed butterfly over the lanes.
__global__ __launch_bounds__(256) void k_norm(Batch b, Work wk) {
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= b.dyn[1]) return;
  const int E = b.E, S = b.proj_split;
  const int ngr = (b.C + kProjKG - 1) / kProjKG;
  const FrameDesc& fd = b.frames[b.mask_frame[g]];
  const int i = g - fd.mask_base;
  float* o = fd.out + (int64_t)i * E;
  float4 v[4];  // E <= 1024: at most 4 chunks of 4 columns per lane
  float ss = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (S == 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (lane * 4 + 256 * k < E) v[k] = *reinterpret_cast<const float4*>(o + lane * 4 + 256 * k);
  } else {
    // group sums added in group order; the four chunks of a group load together
    for (int grp = 0; grp < ngr; ++grp) {
      const float* qp = wk.qpart + ((int64_t)grp * b.M + g) * E;
      float4 q[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        q[k] = lane * 4 + 256 * k < E ? *reinterpret_cast<const float4*>(qp + lane * 4 + 256 * k)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[k].x += q[k].x;
        v[k].y += q[k].y;
        v[k].z += q[k].z;
        v[k].w += q[k].w;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = lane * 4 + 256 * k;
    if (c >= E) continue;
    ss += v[k].x * v[k].x;
    ss += v[k].y * v[k].y;
    ss += v[k].z * v[k].z;
    ss += v[k].w * v[k].w;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  const int st_in = wk.mstat[g];
  const bool zero = st_in != 0 || !(ss > 0.f);
  const float inv = zero ? 0.f : 1.0f / __builtin_sqrtf(ss);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = lane * 4 + 256 * k;
    if (c < E) *reinterpret_cast<float4*>(o + c) = make_float4(v[k].x * inv, v[k].y * inv, v[k].z * inv, v[k].w * inv);
  }
  if (lane == 0 && fd.status) fd.status[i] = st_in != 0 ? st_in : (ss > 0.f ? 0 : 2);
}

void launch_proj(const Batch& b, const Work& w, const void* proj, int proj_bf16, hipStream_t st, bool packed) {
  if (b.M <= 0) return;
  const dim3 block(256);
  if (b.gemm_bf16) {
    const int64_t np = (int64_t)(b.C / 8) * b.E;
    const dim3 pg((unsigned)((np + 255) / 256));
    if (packed) {
    } else if (proj_bf16) {
      hipLaunchKernelGGL((k_pack_proj<1>), pg, block, 0, st, proj, b.C, b.E, reinterpret_cast<uint4*>(w.ppack));
    } else {
      hipLaunchKernelGGL((k_pack_proj<0>), pg, block, 0, st, proj, b.C, b.E, reinterpret_cast<uint4*>(w.ppack));
    }
    hipLaunchKernelGGL((k_proj_bf16<64, 64>), dim3((b.M + 63) / 64 * b.proj_split, b.E / 64), block, 0, st, b, w);
  } else {
    const dim3 grid((b.M + 31) / 32 * b.proj_split, b.E / 128);
    if (proj_bf16) hipLaunchKernelGGL((k_proj<1>), grid, block, 0, st, b, w, proj);
    else hipLaunchKernelGGL((k_proj<0>), grid, block, 0, st, b, w, proj);
  }
  hipLaunchKernelGGL(k_norm, dim3((b.M + 3) / 4), dim3(256), 0, st, b, w);
}

}  // namespace disc
