// Mask scan (bounding box + area per mask), which also appends each mask's
// distance-transform work items to its class's lists (small batches; larger
// ones build the lists in k_lists); the bit-packing and fill helpers.
#include "disc_device.h"

namespace disc {

// ---------------------------------------------------------------------------
// k_scan: one workgroup per mask (1024 threads for small batches without
// D-bar, so that a mask is read in a couple of rounds of loads, else 256:
// D-bar's float sum depends on the width, and must not depend on the batch)
// streams the mask's h*wq words once (the only
// full read of the mask bits) and reduces min/max row, min/max column and the
// pixel count.  Columns >= w in the last word of a row are ignored.
// For frames that ask for it, the same pass sums r_p over the mask's pixels
// (each pixel takes its patch's r) and writes the mean distinctiveness
//   dbar = sum_x r_p(x) / (|M| (mean(r) + eps))
// i.e. D of Eq. (1) averaged over the mask's pixels; the token statistics
// (r and its mean) run before the scan.
// ---------------------------------------------------------------------------
__device__ inline int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ inline int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ inline int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// append = 1: each mask appends its strips to its class's work sub-list
// (one device-scope atomic per mask); 0: k_lists builds the lists afterwards
// from the masks' (class, strips) records.  CS >= 0: the workgroups past the
// first scan_blocks take the token statistics' channel-sum chunks (tokens of
// type CS; chunk-major per frame, as k_colsum's grid), so a small batch
// saves that launch.
template <int kScanThreads, int CS = -1>
__global__ __launch_bounds__(kScanThreads) void k_scan(Batch b, Work wk, int append, int scan_blocks = 0) {
  constexpr int kScanWaves = kScanThreads / 64;
  const int g = blockIdx.x;
  if constexpr (CS >= 0) {
    if (g >= scan_blocks) {
      const int k = g - scan_blocks;
      colsum_chunk<CS>(b, wk, k / b.nchunk, k % b.nchunk);
      return;
    }
  }
  if (g >= b.dyn[1]) return;
  const FrameDesc fd = b.frames[b.mask_frame[g]];
  const int wq = fd.wq, h = fd.h;
  const uint64_t* mb = fd.bits + (int64_t)(g - fd.mask_base) * h * wq;
  const uint64_t last_valid = (fd.w & 63) ? ((1ull << (fd.w & 63)) - 1) : ~0ull;
  const int64_t nwords = (int64_t)h * wq;

  int ymin = INT32_MAX, ymax = -1, xmin = INT32_MAX, xmax = -1, area = 0;
  const float* rf = fd.dbar ? wk.r + fd.r_base : nullptr;
  const int P = fd.patch;
  float rsum = 0.f;
  // words tid, tid + kScanThreads, ... in groups of four independent loads in flight;
  // (row, word) of each load without a division per word
  auto visit = [&](uint64_t v, int row, int k) {
    if (k == wq - 1) v &= last_valid;
    if (v) {
      ymin = min(ymin, row);
      ymax = max(ymax, row);
      xmin = min(xmin, 64 * k + __builtin_ctzll(v));
      xmax = max(xmax, 64 * k + 63 - __builtin_clzll(v));
      area += __builtin_popcountll(v);
      if (rf) {
        // split the word at patch-column boundaries; set bits lie at columns < w,
        // so every patch read is inside the frame's gh x gw grid
        const float* rrow = rf + (int64_t)(row / P) * fd.gw;
        int pc = (64 * k) / P, lo = 0;
        while (lo < 64) {
          const int hi = min((pc + 1) * P - 64 * k, 64);
          const uint64_t seg = v & (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
          if (seg) rsum += (float)__builtin_popcountll(seg) * rrow[pc];
          lo = hi;
          ++pc;
        }
      }
    }
  };
  int row = threadIdx.x / wq, k = threadIdx.x % wq;
  const int drow = kScanThreads / wq, dk = kScanThreads % wq;
  auto step = [&](int& r, int& kk) {
    r += drow;
    kk += dk;
    if (kk >= wq) {
      kk -= wq;
      r += 1;
    }
  };
  int64_t i = threadIdx.x;
  for (; i + 3 * kScanThreads < nwords; i += 4 * kScanThreads) {
    uint64_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load(mb + i + q * kScanThreads);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      visit(v[q], row, k);
      step(row, k);
    }
  }
  for (; i < nwords; i += kScanThreads) {
    visit(__builtin_nontemporal_load(mb + i), row, k);
    step(row, k);
  }
  ymin = wave_min(ymin);
  ymax = wave_max(ymax);
  xmin = wave_min(xmin);
  xmax = wave_max(xmax);
  area = wave_sum(area);
  for (int o = 32; o > 0; o >>= 1) rsum += __shfl_xor(rsum, o);
  __shared__ float rred[kScanWaves];
  __shared__ int red[kScanWaves][5];
  __shared__ int app[3];  // class, strips, first slot in the class list
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[wv][0] = ymin;
    red[wv][1] = ymax;
    red[wv][2] = xmin;
    red[wv][3] = xmax;
    red[wv][4] = area;
    rred[wv] = rsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kScanWaves; ++i) {
      ymin = min(ymin, red[i][0]);
      ymax = max(ymax, red[i][1]);
      xmin = min(xmin, red[i][2]);
      xmax = max(xmax, red[i][3]);
      area += red[i][4];
    }
    int meta = -1;
    app[1] = 0;
    if (area > 0) {
      const int SW = strip_width(P);
      const int xs0 = (xmin / P) * P;
      const int strips = (xmax + 1 - xs0 + SW - 1) / SW;
      const int n = ymax - ymin + 3;
      int cls = kClasses;
      for (int c = 0; c < kClasses; ++c)
        if (n <= class_rows(c)) {
          cls = c;
          break;
        }
      meta = (cls << 16) | strips;  // cls == kClasses would mean "too tall": rejected on the host
      wk.bbox[g] = make_int4(ymin, ymax, xmin, xmax);
      MaskRec r;
      r.bits = mb;
      r.srow = wk.s + fd.w_base + (int64_t)(g - fd.mask_base) * fd.Gs;
      r.y0 = ymin;
      r.y1 = ymax;
      r.x0 = xmin;
      r.x1 = xmax;
      r.n = n;
      r.patch = P;
      r.gw = fd.gw;
      r.wq = wq;
      r.w = fd.w;
      r.h = h;
      r.xs0 = xs0;
      r.g = g;
      wk.mrec[g] = r;
      if (cls < kClasses && append) {
        // the order of items inside a class's lists does not affect any result
        app[0] = cls;
        app[1] = strips;
        app[2] = atomicAdd(wk.counts + cls * kLists + g % kLists, strips);
      }
    } else {
      wk.bbox[g] = make_int4(1, 0, 1, 0);
    }
    wk.area[g] = area;
    wk.meta[g] = meta;
    const int64_t li = g - fd.mask_base;
    if (fd.area_out) fd.area_out[li] = area;
    if (fd.dbar) {
      float tot = rred[0];
      for (int i = 1; i < kScanWaves; ++i) tot += rred[i];
      const int f = b.mask_frame[g];
      fd.dbar[li] = area > 0 ? (tot / (float)area) / (wk.rbar[f] + b.eps) : 0.f;
    }
  }
  __syncthreads();
  const int strips = app[1];
  if (strips > 0) {
    int32_t* list = wk.items + ((int64_t)app[0] * kLists + g % kLists) * b.item_cap + app[2];
    for (int j = threadIdx.x; j < strips; j += kScanThreads)
      if (app[2] + j < b.item_cap) list[j] = (g << kItemStripBits) | j;
  }
}

// ---------------------------------------------------------------------------
// k_lists: the work sub-lists of batches of more than kListsMasks masks.  A
// mask's atomic append at the end of its scan workgroup kept the workgroup
// (and its CU slot) waiting for the atomic's round trip: for large batches
// the scan only records (class, strips) per mask.  One workgroup per (class
// c < 5, sub-list j) writes the items of the masks g = j, j + kLists, ... of
// that class in mask order (a block-wide prefix sum of their strips).  The
// items taller than 512 rows (class 5), whose search costs differ by two
// orders of magnitude, are written by one more workgroup in decreasing order
// of an estimated cost (counting sort over kCostBuckets buckets of
// n * min(n, box width), a mask's strips kept together), filling the
// sub-lists one after another: the XCD queues of the direct search then hand
// out the longest packets first.
// ---------------------------------------------------------------------------
constexpr int kListsMasks = 512;
constexpr int kCostBuckets = 64;

__device__ __forceinline__ int tall_cost_bucket(const Work& wk, int g) {
  const int4 bb = wk.bbox[g];
  const int n = bb.y - bb.x + 3, bw = bb.w - bb.z + 1;
  const float key = (float)n * (float)min(n, bw);  // >= 1
  return min(kCostBuckets - 1, (int)(2.f * __log2f(key)));
}

__device__ __forceinline__ void lists_tall(const Batch& b, const Work& wk) {
  __shared__ int cnt[kCostBuckets], cur[kCostBuckets];
  const int M = b.dyn[1];
  const int cap = b.item_cap;
  if (threadIdx.x < kCostBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  // eight masks per thread and round, their records loaded together
  for (int g0 = 0; g0 < M; g0 += 8 * 1024) {
    int mt[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int g = g0 + 1024 * i + (int)threadIdx.x;
      mt[i] = g < M ? wk.meta[g] : -1;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (mt[i] >= 0 && (mt[i] >> 16) == 5)
        atomicAdd(&cnt[tall_cost_bucket(wk, g0 + 1024 * i + (int)threadIdx.x)], mt[i] & 0xFFFF);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;  // descending cost: the last bucket first
    for (int k = kCostBuckets - 1; k >= 0; --k) {
      cur[k] = acc;
      acc += cnt[k];
    }
    cnt[0] = acc;  // the class's item count
  }
  __syncthreads();
  const int total = cnt[0];
  int32_t* list = wk.items + (int64_t)5 * kLists * cap;  // sub-lists 0 .. kLists - 1 back to back
  for (int g0 = 0; g0 < M; g0 += 8 * 1024) {
    int mt[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int g = g0 + 1024 * i + (int)threadIdx.x;
      mt[i] = g < M ? wk.meta[g] : -1;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (mt[i] < 0 || (mt[i] >> 16) != 5) continue;
      const int g = g0 + 1024 * i + (int)threadIdx.x, strips = mt[i] & 0xFFFF;
      const int first = atomicAdd(&cur[tall_cost_bucket(wk, g)], strips);
      for (int k = 0; k < strips; ++k)
        if (first + k < kLists * cap) list[first + k] = (g << kItemStripBits) | k;
    }
  }
  if (threadIdx.x < kLists)
    wk.counts[5 * kLists + threadIdx.x] = max(0, min(cap, total - (int)threadIdx.x * cap));
}

// grid: (kClasses - 1) * kLists workgroups for classes 0-4, plus one for
// class 5 when the batch can have such items (it runs beside the others)
__global__ __launch_bounds__(1024) void k_lists(Batch b, Work wk) {
  if ((int)blockIdx.x == (kClasses - 1) * kLists) {
    lists_tall(b, wk);
    return;
  }
  const int c = blockIdx.x / kLists, j = blockIdx.x % kLists;
  const int M = b.dyn[1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ int wsum[16];
  int32_t* list = wk.items + ((int64_t)c * kLists + j) * b.item_cap;
  int total = 0;  // items of the sub-list so far
  for (int i0 = 0; j + kLists * i0 < M; i0 += 1024) {
    const int g = j + kLists * (i0 + (int)threadIdx.x);
    const int meta = g < M ? wk.meta[g] : -1;
    const int v = (meta >= 0 && (meta >> 16) == c) ? (meta & 0xFFFF) : 0;
    // inclusive scan over the wavefront, then over the wavefront totals
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(x, o);
      if (lane >= o) x += t;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int before = 0, all = 0;
    for (int k = 0; k < 16; ++k) {
      const int t = wsum[k];
      before += k < wv ? t : 0;
      all += t;
    }
    const int first = total + before + x - v;
    for (int k = 0; k < v; ++k)
      if (first + k < b.item_cap) list[first + k] = (g << kItemStripBits) | k;
    total += all;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (threadIdx.x == 0) wk.counts[c * kLists + j] = total;
}

bool scan_takes_colsum(const Batch& b, bool any_dbar) { return b.M > 0 && !any_dbar; }

void launch_scan(const Batch& b, const Work& w, hipStream_t st, bool any_dbar, bool colsum) {
  if (b.M <= 0) return;
  const int append = b.M <= kListsMasks ? 1 : 0;
  colsum = colsum && scan_takes_colsum(b, any_dbar);
  const int nb = b.M + (colsum ? b.nchunk * b.n_frames : 0), sb = (int)b.M;
  if (b.M <= 512 && !any_dbar) {
    if (!colsum) hipLaunchKernelGGL((k_scan<1024>), dim3(b.M), dim3(1024), 0, st, b, w, append, 0);
    else if (b.tok_dtype == 0) hipLaunchKernelGGL((k_scan<1024, 0>), dim3(nb), dim3(1024), 0, st, b, w, append, sb);
    else if (b.tok_dtype == 1) hipLaunchKernelGGL((k_scan<1024, 1>), dim3(nb), dim3(1024), 0, st, b, w, append, sb);
    else hipLaunchKernelGGL((k_scan<1024, 2>), dim3(nb), dim3(1024), 0, st, b, w, append, sb);
  } else {
    if (!colsum) hipLaunchKernelGGL((k_scan<256>), dim3(b.M), dim3(256), 0, st, b, w, append, 0);
    else if (b.tok_dtype == 0) hipLaunchKernelGGL((k_scan<256, 0>), dim3(nb), dim3(256), 0, st, b, w, append, sb);
    else if (b.tok_dtype == 1) hipLaunchKernelGGL((k_scan<256, 1>), dim3(nb), dim3(256), 0, st, b, w, append, sb);
    else hipLaunchKernelGGL((k_scan<256, 2>), dim3(nb), dim3(256), 0, st, b, w, append, sb);
  }
  if (!append) {
    // class-5 counters stay 0 (zeroed when staged) when no item can be that tall
    const int tall = b.max_rows > class_rows(kClasses - 2) ? 1 : 0;
    hipLaunchKernelGGL(k_lists, dim3((kClasses - 1) * kLists + tall), dim3(1024), 0, st, b, w);
  }
}

// ---------------------------------------------------------------------------
// k_pool_order: one workgroup per frame orders its masks for the pooling
// tiles by the first patch row of their box (counting sort over 256 buckets,
// empty masks last), so that each 64-mask tile reads a narrow band of token
// rows.  The order within a bucket follows the atomics and may differ from
// run to run: which masks share a tile never changes a mask's result.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pool_order(Batch b, Work wk) {
  __shared__ int cnt[256];
  __shared__ int wsum[4];
  for (int f = blockIdx.x; f < b.dyn[0]; f += gridDim.x) pool_order_frame(b, wk, f, cnt, wsum);
}

void launch_pool_order(const Batch& b, const Work& w, hipStream_t st) {
  if (b.n_frames > 0 && b.M > 0) hipLaunchKernelGGL(k_pool_order, dim3(b.n_frames), dim3(256), 0, st, b, w);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
}

__global__ void k_copy_f32(const float* src, float* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
}

// one thread per output word: 64 bytes -> 64 bits
__global__ void k_pack(const uint8_t* u8, int m, int h, int w, uint64_t* bits) {
  const int wq = (w + 63) / 64;
  const int64_t nwords = (int64_t)m * h * wq;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rowi = i / wq;
    const int k = (int)(i - rowi * wq);
    const uint8_t* src = u8 + rowi * w + 64 * k;
    const int nb = min(64, w - 64 * k);
    uint64_t v = 0;
    for (int j = 0; j < nb; ++j) v |= (uint64_t)(src[j] != 0) << j;
    bits[i] = v;
  }
}

void launch_pack(const uint8_t* u8, int m, int h, int w, uint64_t* bits, hipStream_t st) {
  const int64_t nwords = (int64_t)m * h * ((w + 63) / 64);
  if (nwords <= 0) return;
  int64_t blocks = (nwords + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, st, u8, m, h, w, bits);
}

}  // namespace disc
