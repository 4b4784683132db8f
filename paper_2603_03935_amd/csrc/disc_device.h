// Internal declarations shared by the libdisc HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace disc {

// ---------------------------------------------------------------------------
// Distance-transform work decomposition.
//
// A work item is (mask, strip): SW(P) = 64 - 64 % P consecutive pixel columns
// starting on a patch boundary.  The item's rows (bounding-box height + one
// padding row above and below, n rows) are split into bands of B rows, one
// wavefront per band.  The row count picks the class c (n <= class_rows(c)).
// One EDT workgroup has kEdtWaves wavefronts and processes a packet of
// kEdtWaves / K items of one class side by side.  Two band layouts share the
// classes: mode 0 (short bands, for small batches where the longest item sets
// the time) and mode 1 (longer bands and fewer merge steps, for batches that
// fill the GPU many times over):
//   class        0    1    2    3    4     5
//   rows        32   64  128  256  512  1152
//   mode 0 B,K  32,1 32,2 32,4 32,8 32,16 96,12
//   mode 1 B,K  32,1 64,1 64,2 64,4 64,8  96,12
// ---------------------------------------------------------------------------
constexpr int kClasses = 6;
constexpr int kEdtWaves = 16;
__host__ __device__ constexpr int class_rows(int c) { return c == 5 ? 1152 : (32 << c); }
__host__ __device__ constexpr int class_band(int mode, int c) { return c == 5 ? 96 : (mode == 0 || c == 0) ? 32 : 64; }
__host__ __device__ constexpr int class_waves(int mode, int c) { return class_rows(c) / class_band(mode, c); }
__host__ __device__ constexpr int class_items(int mode, int c) { return kEdtWaves / class_waves(mode, c); }
constexpr int kMaxRows = 1152;      // bbox height + 2
constexpr int kMinPatch = 8;
constexpr int kMaxPatch = 64;
constexpr int kItemStripBits = 8;   // item = (mask << 8) | strip
constexpr int kMaxC = 2048;
// Frame mean: partial channel sums over chunks of stat_chunk(G) tokens (a
// multiple of 32 chosen from G alone, so at most 64 chunks per frame), added
// in chunk order.
__host__ __device__ inline int stat_chunk(int G) { return 32 * ((G + 32 * 64 - 1) / (32 * 64)); }
__host__ __device__ inline int stat_nchunk(int G) { return (G + stat_chunk(G) - 1) / stat_chunk(G); }
// The GEMMs accumulate K in fixed groups (pooling: 256 patches, projection:
// 256 channels) and add the group sums in order, so splitting K over several
// workgroups (for small batches) gives the same bits as one pass.
constexpr int kPoolKG = 256;
constexpr int kProjKG = 256;
constexpr int kTargetWGs = 512;  // workgroups that fill the 256 CUs twice

__host__ __device__ inline int strip_width(int patch) { return 64 - (64 % patch); }

// LDS of one EDT workgroup (every class fits kMaxRows rows): a 16-byte record
// per row, the per-column stack bitmaps (one bit per row) and the partial
// patch sums of every 16-row block of the items' rows (a block meets at most
// 3 patch rows of at least 8 pixels).  Patch sums are always formed per
// 16-row block, whatever the layout or band height, so the order of the
// additions (and the result) depends only on the mask.
constexpr int kBlkRows = 16;
constexpr int kEdtBmWords = kMaxRows / 32 + 1;
constexpr int kEdtBlocks = kMaxRows / kBlkRows;
constexpr int kEdtPartRows = 3;
// Direct search: a packet of at most 512 rows may be shared by up to
// kDirSplitMax workgroups when the batch has few packets; their block partial
// sums go to a global buffer of kDirSplitPackets packets.
constexpr int kDirSplitMax = 2;
constexpr int kDirSplitPackets = 512;
constexpr int kDirPartFloats = 512 / kBlkRows * kEdtPartRows * 8;  // per packet

// Per-mask record of the distance transform (written by the mask scan).
struct MaskRec {
  const uint64_t* bits;    // the mask's first row
  float* srow;             // the mask's spatial-weight row
  int32_t y0, y1, x0, x1;  // bounding box
  int32_t n, patch, gw, wq;
  int32_t w, h, xs0, g;    // frame width/height, first strip column, global mask index
};

__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even (finite inputs)
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// The four e4m3fn codes of w (lowest byte first) as floats, by the hardware
// conversion (exact: sign x 2^(e - 7) x (1 + m / 8), subnormals m x 2^-9,
// codes 0x7F and 0xFF NaN).  Every e4m3fn value is also exact in BF16 (its
// FP32 bits end in 16 zeros).
__device__ __forceinline__ float4 e4m3x4_to_f32(uint32_t w) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  const f2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  return make_float4(lo.x, lo.y, hi.x, hi.y);
}

// Workgroup b of a launch runs on XCD b % 8 (each XCD has its own L2).
// xcd_remap gives each XCD a contiguous range of the n live workgroups of a
// launch (a bijection of [0, n)), so workgroups that read the same data (the
// channel tiles of one mask tile, the strips of one mask) share an L2.
constexpr int kXcds = 8;
// Work lists of the distance transform: each class has kLists sub-lists,
// mask g appending its strips to sub-list g % kLists, so that the scan's
// atomics spread over kClasses x kLists counters instead of kClasses (one
// hot counter per class serialised thousands of device-scope atomics).  A
// class's items are its sub-lists one after another.
constexpr int kLists = 8;
// Counters zeroed whenever a batch is staged: the sub-list sizes
// [kClasses][kLists], then the direct EDT's packet queues (one counter per
// XCD and launch: kDirQueue .. + 7 for classes 0-4, the next 8 for class 5),
// then the per-frame FP8 scale flags.
constexpr int kDirQueue = kClasses * kLists;
constexpr int kCounters = 64;
static_assert(kDirQueue + 2 * kXcds <= kCounters, "counters");
// items of class c (each sub-list capped at item_cap)
__device__ __forceinline__ int class_count(const int32_t* counts, int item_cap, int c) {
  int n = 0;
#pragma unroll
  for (int j = 0; j < kLists; ++j) n += min(counts[c * kLists + j], item_cap);
  return n;
}
// item k of class c (k below class_count): the item word of its sub-list
__device__ __forceinline__ int class_item(const int32_t* counts, const int32_t* items, int item_cap, int c, int k) {
  int j = 0;
  for (; j < kLists - 1; ++j) {
    const int n = min(counts[c * kLists + j], item_cap);
    if (k < n) break;
    k -= n;
  }
  return items[((int64_t)c * kLists + j) * item_cap + k];
}
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + min(x, r) + k;
}

// One frame of a (possibly ragged) batch, in device memory.
struct FrameDesc {
  const void* tokens;     // [G][C] in tok_dtype
  const float* scale;     // [G] for FP8 tokens
  const uint64_t* bits;   // [m][h][wq]
  float* out;             // [m][E]
  int32_t* status;        // [m] or null
  float* pooled;          // [m][C] or null
  float* dbar;            // [m] or null: mean D over the mask's pixels
  int32_t* area_out;      // [m] or null: pixel counts
  int32_t gh, gw, patch, G;
  int32_t h, w, wq, m;
  int32_t mask_base;      // global index of this frame's first mask
  int32_t Gs;             // row stride of the per-mask weight rows (G rounded up to 8)
  int64_t w_base;         // element offset of this frame's [m][Gs] block in s/W
  int64_t r_base;         // offset of this frame's G entries in r
};

// Scalar arguments shared by the kernels of one call.  n_frames and M are
// capacities (they size the grids); the live counts are read from device
// memory (dyn), so one captured graph of the kernel set serves every batch
// that fits the capacities.
struct Batch {
  const FrameDesc* frames;
  const int32_t* mask_frame;  // [M] frame of each global mask
  const int32_t* dyn;         // device: [0] frames, [1] masks, [2] pooling tiles
  int32_t n_frames, M, C, E;
  int32_t tok_dtype;          // disc_dtype of the tokens
  int32_t gemm_bf16;          // 1: BF16 operands, 0: FP32 operands
  int32_t spatial, distinct;
  int32_t nchunk;             // token-statistics chunks per frame (capacity)
  int32_t item_cap;           // capacity of each work sub-list (and the sub-list stride)
  int32_t n_tiles;            // pooling tiles (capacity)
  int32_t kgroups;            // pooling K groups of the largest frame
  int32_t pool_split, proj_split;  // workgroups sharing one GEMM tile's K range
  float eps;                  // Eq. (1) epsilon (only the mean distinctiveness uses it)
  int32_t max_rows;           // tallest frame + 2 (the tallest distance-transform item)
};

// Workspace pointers (device).
struct Work {
  int4* bbox;          // [M] (y0, y1, x0, x1); y0 > y1 for an empty mask
  int32_t* area;       // [M]
  int32_t* meta;       // [M] (class << 16) | strips, -1 empty
  MaskRec* mrec;       // [M]
  int32_t* items;      // [kClasses][kLists][item_cap] (mask << 8) | strip: the sub-lists of each class
  int32_t* counts;     // [kCounters] sub-list sizes and EDT queues (zeroed when a batch is staged)
  int32_t* fbad;       // [frames] 1 when a frame's FP8 scales include a non-finite or negative value (zeroed when staged)
  float* psum;         // [F][nchunk][C]
  float* mean;         // [F][C]
  float* r;            // [sum G]
  float* rbar;         // [F] mean of r per frame (frames that ask for dbar)
  float* s;            // [sum m*Gs] spatial weights
  void* W;             // [sum m*Gs] GEMM-dtype weights
  float* Z;            // [M] weight sums
  int32_t* mstat;      // [M] 0 ok, 1 empty
  int32_t* perm;       // [M] pooling order: perm[mask_base + i] = frame-local mask of tile row i
  void* X;             // [M][C] pooled features in the GEMM dtype
  float* ppart;        // pooling group sums [tile][kgroups][64*64] (split K only)
  int4* ptile;         // per pooling tile: (first, end K group), then its 64 rows as pool_rows gives them (split K only)
  float* qpart;        // projection group sums [C/256][M][E] (split K only)
  float* edt_part;     // direct EDT block partial sums of shared packets [kDirSplitPackets][kDirPartFloats]
  void* ppack;         // k-packed BF16 copy of P [C/8][E][8] (BF16 GEMMs)
};

// Host-side launchers (stream = hipStream_t).
// any_dbar: some frame of the batch asks for the mean distinctiveness (its
// float sum is formed per scan thread, so such batches always use one width)
// colsum: when scan_takes_colsum(b, any_dbar), the scan's launch also takes
// the token statistics' channel sums (launch_token_stats then runs with
// colsum_done)
void launch_scan(const Batch& b, const Work& w, hipStream_t st, bool any_dbar = true, bool colsum = false);
bool scan_takes_colsum(const Batch& b, bool any_dbar);
// Pooling order of frame f's masks: a counting sort over 256 buckets by the
// first patch row of the box (empty masks last), so that each 64-mask pooling
// tile reads a narrow band of token rows.  A frame of more than kPoolBigMin
// masks first puts its largest boxes (up to kPoolBig of them, by a
// histogram of log2 box area) into the first tiles: a few large masks in a
// tile make its rows' union most of the frame, so they share their tiles
// (a CPU model of 1080p frames of 500 masks: 15 % less issued work).  The order within a
// bucket follows the atomics and may differ from run to run: which masks
// share a tile never changes a mask's result.  Any block size >= 256 (the
// first 256 threads own the buckets); all threads of the block call it.
constexpr int kPoolBig = 128, kPoolBigMin = 256;
__device__ inline void pool_order_frame(const Batch& b, const Work& wk, int f, int* cnt, int* wsum) {
  const FrameDesc& fd = b.frames[f];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nt = blockDim.x;
  const int m = fd.m, base = fd.mask_base, P = fd.patch;
  auto abucket = [&](const int4& bb) {  // 0 .. 63, larger boxes higher
    const float area = (float)(bb.y - bb.x + 1) * (float)(bb.w - bb.z + 1);
    return min(63, (int)(2.f * __log2f(area)));
  };
  int big_from = 64;  // area buckets >= big_from go first
  if (m > kPoolBigMin) {
    if (tid < 64) cnt[tid] = 0;
    __syncthreads();
    for (int i = tid; i < m; i += nt) {
      const int4 bb = wk.bbox[base + i];
      if (bb.x <= bb.y) atomicAdd(&cnt[abucket(bb)], 1);
    }
    __syncthreads();
    // the lowest bucket t with at most kPoolBig boxes in buckets >= t
    int acc = 0, t = 64;
    for (int k = 63; k >= 0; --k) {
      acc += cnt[k];
      if (acc > kPoolBig) break;
      t = k;
    }
    big_from = t;
    __syncthreads();
  }
  auto key = [&](int i) {
    const int4 bb = wk.bbox[base + i];
    if (bb.x > bb.y) return 255;
    return abucket(bb) >= big_from ? 0 : 1 + min(bb.x / P, 253);
  };
  if (tid < 256) cnt[tid] = 0;
  __syncthreads();
  for (int i = tid; i < m; i += nt) atomicAdd(&cnt[key(i)], 1);
  __syncthreads();
  // exclusive prefix of the 256 bucket counts (the first four wavefronts)
  int v = 0, x = 0;
  if (tid < 256) {
    v = cnt[tid];
    x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(x, o);
      if (lane >= o) x += t;
    }
    if (lane == 63) wsum[wv] = x;
  }
  __syncthreads();
  if (tid < 256) {
    int before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    cnt[tid] = before + x - v;
  }
  __syncthreads();
  for (int i = tid; i < m; i += nt) wk.perm[base + atomicAdd(&cnt[key(i)], 1)] = i;
  __syncthreads();
}

// Token statistics: partial channel sums over chunks of stat_chunk(G) tokens
// of a frame, folded in chunk order into the frame mean by k_mean.  The first
// 256 threads of the block do the work (the same partition and order in a
// 256-thread k_colsum workgroup and in the 1024-thread mask-scan workgroups
// that carry it for small batches); every thread of the block must call it.
// Each thread reads 16-byte vectors (VEC channels) of several token rows.
template <int TOK>
__device__ __forceinline__ void load_vec(const void* base, const float* scale, int64_t p, int C, int c, float* v) {
  const int64_t off = p * C + c;
  if (TOK == 0) {
    const float4* q = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + off);
    const float4 a = q[0], d = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = d.x; v[5] = d.y; v[6] = d.z; v[7] = d.w;
  } else if (TOK == 1) {
    const uint4 a = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(base) + off);
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
    for (int j = 0; j < 4; ++j) {
      v[2 * j] = bf16_to_f32(w[j] & 0xFFFFu);
      v[2 * j + 1] = bf16_to_f32(w[j] >> 16);
    }
  } else {
    const uint4 a = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint8_t*>(base) + off);
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
    const float sc = scale[p];
    for (int j = 0; j < 4; ++j) {
      const float4 x = e4m3x4_to_f32(w[j]);
      v[4 * j] = sc * x.x;
      v[4 * j + 1] = sc * x.y;
      v[4 * j + 2] = sc * x.z;
      v[4 * j + 3] = sc * x.w;
    }
  }
}

template <int TOK>
__device__ inline void colsum_chunk(const Batch& b, const Work& wk, int f, int chunk) {
  constexpr int VEC = TOK == 2 ? 16 : 8;
  if (f >= b.dyn[0]) return;
  const FrameDesc fd = b.frames[f];
  const int G = fd.G, C = b.C;
  const int nch = stat_nchunk(G);
  if (chunk >= nch) return;
  const int tpr = C / VEC, rpp = 256 / tpr;
  const int tid = threadIdx.x, cg = tid % tpr, ro = tid / tpr;
  const int p0 = chunk * stat_chunk(G), p1 = min(p0 + stat_chunk(G), G);
  __shared__ float part[256 * 16];
  float acc[VEC];
  for (int j = 0; j < VEC; ++j) acc[j] = 0.f;
  if (ro < rpp) {
    int p = p0 + ro;
    for (; p + 3 * rpp < p1; p += 4 * rpp) {
      float v0[VEC], v1[VEC], v2[VEC], v3[VEC];
      load_vec<TOK>(fd.tokens, fd.scale, p, C, cg * VEC, v0);
      load_vec<TOK>(fd.tokens, fd.scale, p + rpp, C, cg * VEC, v1);
      load_vec<TOK>(fd.tokens, fd.scale, p + 2 * rpp, C, cg * VEC, v2);
      load_vec<TOK>(fd.tokens, fd.scale, p + 3 * rpp, C, cg * VEC, v3);
      for (int j = 0; j < VEC; ++j) acc[j] += ((v0[j] + v1[j]) + v2[j]) + v3[j];
    }
    for (; p < p1; p += rpp) {
      float v0[VEC];
      load_vec<TOK>(fd.tokens, fd.scale, p, C, cg * VEC, v0);
      for (int j = 0; j < VEC; ++j) acc[j] += v0[j];
    }
    for (int j = 0; j < VEC; ++j) part[ro * C + cg * VEC + j] = acc[j];
  }
  __syncthreads();
  float* ps = wk.psum + ((int64_t)f * b.nchunk + chunk) * C;
  if (tid < 256) {
    for (int c = tid; c < C; c += 256) {
      float a = 0.f;
      for (int r = 0; r < rpp; ++r) a += part[r * C + c];
      ps[c] = a;
    }
  }
}

// One thread t of the projection's k-packed BF16 copy: column n, channels
// 8 kg .. 8 kg + 7 of P ([C][E], FP32 or BF16 bits) as 16 bytes at ppack[t]
// ([C/8][E][8]).
template <int PBF16>
__device__ __forceinline__ void pack_proj_chunk(const void* proj, int C, int E, uint4* ppack, int64_t t) {
  if (t >= (int64_t)(C / 8) * E) return;
  const int kg = (int)(t / E), n = (int)(t - (int64_t)kg * E);
  uint32_t q[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t off = (int64_t)(kg * 8 + j) * E + n;
    q[j] = PBF16 ? reinterpret_cast<const uint16_t*>(proj)[off] : f2bf(reinterpret_cast<const float*>(proj)[off]);
  }
  ppack[t] = make_uint4(q[0] | (q[1] << 16), q[2] | (q[3] << 16), q[4] | (q[5] << 16), q[6] | (q[7] << 16));
}

// mean[f][c] of the token statistics: the chunk partials of channel c in
// chunk order, divided by G (one thread per channel; k_mean, or the
// distance transform's last launch for small batches)
__device__ __forceinline__ void frame_mean_channel(const Batch& b, const Work& wk, int f, int c) {
  const int G = b.frames[f].G;
  const int nch = stat_nchunk(G);
  const float* ps = wk.psum + (int64_t)f * b.nchunk * b.C + c;
  float a = 0.f;
#pragma unroll 8
  for (int j = 0; j < nch; ++j) a += ps[(int64_t)j * b.C];
  wk.mean[(int64_t)f * b.C + c] = a * (1.0f / (float)G);
}

void launch_pool_order(const Batch& b, const Work& w, hipStream_t st);
// order_pool: also order every frame's masks for the pooling (as
// launch_pool_order), inside the launch that follows the distance transform
// take_mean (direct search only, mode -1 or 2): the last launch also takes
// the token statistics' frame means (the channel sums must be done) and,
// given pack_proj (BF16 GEMMs), writes the projection's k-packed P
void launch_edt(const Batch& b, const Work& w, int32_t* e_out, int num_cus, hipStream_t st, int mode = -1,
                bool order_pool = false, bool take_mean = false, const void* pack_proj = nullptr, int proj_bf16 = 0);
void edt_prepare();
// Frame means and residual norms r (gmax: the largest G).
// colsum_done: the channel sums were taken by the mask scan's launch.
// pack_proj (BF16 GEMMs): also write the projection's k-packed BF16 copy
// (proj_bf16: P is stored as BF16), from the workgroups of the frame-mean
// launch, so the projection stage skips that launch.
// mean_done: the frame means were taken by the distance transform's last
// launch (launch_edt with take_mean; pack_proj is then not used).
void launch_token_stats(const Batch& b, const Work& w, int gmax, hipStream_t st, bool colsum_done = false,
                        const void* pack_proj = nullptr, int proj_bf16 = 0, bool mean_done = false);
void launch_weights(const Batch& b, const Work& w, hipStream_t st);
void launch_rbar(const Batch& b, const Work& w, hipStream_t st);
// FP8 tokens: flag the frames whose scales hold a non-finite or negative value
void launch_scale_check(const Batch& b, const Work& w, int gmax, hipStream_t st);
void launch_quality(const int32_t* area, const float* dbar, const float* emb, const float* g, const float* angle, int m,
                    int e, int img_h, int img_w, float lambda, float* q, float* comp, hipStream_t st);
void launch_angle(const float* rays, const float* normals, int nv, const int32_t* off, int m, float* angle,
                  hipStream_t st);
// geometry (k_geom.hip); cam = 18 floats (fx, fy, cx, cy, R[9], t[3], dmin, dmax)
size_t scan_scratch_ints(int n);
void launch_bp_count(const float* depth, const uint64_t* bits, int m, int h, int w, int s, const float* cam,
                     int32_t* counts, int32_t* offsets, int32_t* scratch, hipStream_t st);
void launch_bp_write(const float* depth, const uint64_t* bits, int m, int h, int w, int s, const float* cam,
                     const int32_t* offsets, float* points, hipStream_t st);
size_t dbscan_ws_bytes(int n);
void launch_dbscan(const float* pts, const int32_t* off, int m, int n, float eps, int min_pts, int32_t* keep,
                   char* ws, hipStream_t st);
size_t voxel_ws_bytes(int n, int m);
void launch_voxelize(const float* pts, const int32_t* off, const int32_t* keep, int m, int n, float v, int32_t* voff,
                     int32_t* vox, int32_t* status, char* ws, hipStream_t st);
void launch_overlap(const int32_t* va, const int32_t* oa, int na, const int32_t* vb, const int32_t* ob, int nb,
                    const int32_t* pairs, int np, int32_t* out, hipStream_t st);
void launch_fuse(const int32_t* ids, const float* q, const float* emb, int m, int e, float* map_q, float* map_emb,
                 int n_map, int32_t* won, uint64_t* best, hipStream_t st);
// nt: 64-channel tiles per workgroup (1, 2 or 4; any value gives the same result)
// A pooling tile (frame, m0, n0, pair flag): the flag is 1 when the frame's
// next mask tile (m0 + 64) exists and joins this one in a 128-mask
// workgroup, 0 when this tile stays alone, -1 when it is the second of a pair.
__host__ __device__ inline int pool_pair_flag(int m0, int m) { return (m0 & 64) ? -1 : (m0 + 64 < m ? 1 : 0); }
// nt: 64-channel tiles per workgroup (1, 2, 4); mw: 64-mask tiles per
// workgroup (1, or 2 with nt <= 2 and K not split)
void launch_pool(const Batch& b, const Work& w, const int4* tiles, hipStream_t st, int nt = 1, int mw = 1);
bool pool_nt_valid(int C, int nt);
// packed: the k-packed BF16 copy of P is already in the workspace (written
// by launch_token_stats' pack_proj)
void launch_proj(const Batch& b, const Work& w, const void* proj, int proj_bf16, hipStream_t st, bool packed = false);
// stage helpers
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// open-vocabulary query: inv holds m + q floats of scratch
void launch_query(const float* emb, int m, const void* text, int text_bf16, int q, int e, int k, float* inv,
                  float* sim, float* scores, int32_t* idx, hipStream_t st);
void launch_pack(const uint8_t* u8, int m, int h, int w, uint64_t* bits, hipStream_t st);
void launch_dense_weights(const Batch& b, const Work& w, float* out, float eps, hipStream_t st);
void launch_d_from_r(const float* r, int G, float eps, float* D, hipStream_t st);
void launch_heatmap(const void* tok, int tok_dtype, const float* scale, int G, int C, const void* P, int p_bf16, int E,
                    const void* text, int text_bf16, int q, const float* D, float* Y, float* fac, float* inv_text,
                    float* heat, hipStream_t st);
void launch_user_weights(const Batch& b, const Work& w, const float* wts, hipStream_t st);
void launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st);

}  // namespace disc
