// Geometry workload of the mapping pipeline (arXiv 2603.03935, Sec. III-B):
// each segment's depth pixels are back-projected to world points, DBSCAN
// removes the noise points, the rest are voxelised, and segments are
// associated with map instances by exact voxel overlap (Sec. III-B, the
// voxel-overlap refinement).
//
// Where floating point decides an integer (which points are neighbours
// within eps, which voxel a point falls in) every operation is an explicitly
// rounded single-precision one in a fixed order (no contraction into FMA), so
// the decisions are reproducible operation by operation.
//
// Kernels:
//   back-projection  one workgroup per mask, one wavefront per row; rows in
//                    chunks of 16 with a running base, so each mask's points
//                    come out in row-major pixel order;
//   DBSCAN           a global hash grid of (segment, cell) keys with cells of
//                    side eps: insert (64-bit CAS), counting sort of the
//                    points by slot, then per point a scan of the 27
//                    neighbouring cells for the core test and the border
//                    test (early exit);
//   voxels           a global hash set of (segment, voxel) keys gives the
//                    distinct voxels and their count per segment; each
//                    segment's keys are gathered and sorted in LDS (bitonic);
//   overlap          one workgroup per (segment, instance) pair: the longer
//                    list is staged in LDS chunk by chunk and the keys of the
//                    shorter list are binary-searched there.
#include "disc_device.h"

namespace disc {

// ---------------------------------------------------------------------------
// exclusive scan of int32 (two levels, up to 4096 * 4096 elements)
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 4096;  // elements per workgroup (1024 threads x 4)

__device__ __forceinline__ int block_exscan_1024(int v, int* sh) {
  // inclusive wave scan
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (threadIdx.x < 16) {
    int s = sh[threadIdx.x];
    for (int o = 1; o < 16; o <<= 1) {
      const int t = __shfl_up(s, o, 16);
      if ((threadIdx.x & 15) >= o) s += t;
    }
    sh[16 + threadIdx.x] = s;  // inclusive over waves
  }
  __syncthreads();
  const int before = wv > 0 ? sh[16 + wv - 1] : 0;
  const int total = sh[31];
  __syncthreads();
  sh[32] = total;
  return before + x - v;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(const int32_t* in, int n, int32_t* out, int32_t* sums) {
  __shared__ int sh[40];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  int v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = base + k < n ? in[base + k] : 0;
  const int t = v[0] + v[1] + v[2] + v[3];
  int ex = block_exscan_1024(t, sh);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = sh[32];
}

__global__ __launch_bounds__(1024) void k_scan_add(int32_t* out, int n, const int32_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  const int add = sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < n) out[base + k] += add;
}

// out[i] = sum of in[j < i]; out[n] = total when out has n + 1 entries
// (write_total).  scratch: 2 * ceil(n / 4096) + 1 int32.
void exclusive_scan(const int32_t* in, int n, int32_t* out, bool write_total, int32_t* scratch, hipStream_t st) {
  const int nb = (n + kScanBlock - 1) / kScanBlock;
  if (n <= 0) {
    if (write_total) launch_fill_u32(reinterpret_cast<uint32_t*>(out), 0u, 1, st);
    return;
  }
  int32_t* sums = scratch;
  int32_t* sums_ex = scratch + nb;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, st, in, n, out, sums);
  // nb <= 4096: one workgroup scans the block sums (and writes the total)
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, sums, nb, sums_ex, sums_ex + nb);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, st, out, n, sums_ex);
  if (write_total) hipMemcpyAsync(out + n, sums_ex + nb, 4, hipMemcpyDeviceToDevice, st);
}

// ---------------------------------------------------------------------------
// back-projection
// ---------------------------------------------------------------------------
struct Cam {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float dmin, dmax;
};

// valid pixel bits of word k of row y (lane l = column 64k + l), this lane's
// depth in z
__device__ __forceinline__ bool pixel_valid(const uint64_t* row, int k, int y, int w, int s, const float* depth,
                                            const Cam& c, float& z) {
  const int lane = threadIdx.x & 63;
  const uint64_t word = row[k];
  const int x = 64 * k + lane;
  z = 0.f;
  if (!((word >> lane) & 1ull) || x >= w || (x % s) != 0) return false;
  z = depth[(int64_t)y * w + x];
  return __builtin_isfinite(z) && z >= c.dmin && z <= c.dmax;
}

__device__ __forceinline__ int row_count(const uint64_t* row, int y, int wq, int w, int s, const float* depth,
                                         const Cam& c) {
  int cnt = 0;
  for (int k = 0; k < wq; ++k) {
    if (row[k] == 0ull) continue;  // uniform
    float z;
    const bool v = pixel_valid(row, k, y, w, s, depth, c, z);
    cnt += __builtin_popcountll(__ballot(v));
  }
  return cnt;
}

// one workgroup (16 wavefronts) per mask: valid-pixel counts
__global__ __launch_bounds__(1024) void k_bp_count(const float* depth, const uint64_t* bits, int m, int h, int w, int s,
                                                   Cam c, int32_t* counts) {
  const int i = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = (w + 63) / 64;
  const uint64_t* mb = bits + (int64_t)i * h * wq;
  int cnt = 0;
  for (int y = s * wv; y < h; y += 16 * s) cnt += row_count(mb + (int64_t)y * wq, y, wq, w, s, depth, c);
  __shared__ int red[16];
  if (lane == 0) red[wv] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < 16; ++k) t += red[k];
    counts[i] = t;
  }
}

// (contraction off in this scope: every product and sum is rounded on its
// own; the division is the correctly rounded one)
__device__ __forceinline__ void world_point(const Cam& c, int x, int y, float z, float* out) {
#pragma clang fp contract(off)
  const float xc = (((float)x - c.cx) * z) / c.fx;
  const float yc = (((float)y - c.cy) * z) / c.fy;
#pragma unroll
  for (int k = 0; k < 3; ++k) out[k] = ((c.R[3 * k] * xc + c.R[3 * k + 1] * yc) + c.R[3 * k + 2] * z) + c.t[k];
}

// one workgroup per mask: rows in chunks of 16 (one per wavefront), points
// written in row-major order from offsets[i]
__global__ __launch_bounds__(1024) void k_bp_write(const float* depth, const uint64_t* bits, int m, int h, int w, int s,
                                                   Cam c, const int32_t* offsets, float* points) {
  const int i = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wq = (w + 63) / 64;
  const uint64_t* mb = bits + (int64_t)i * h * wq;
  __shared__ int rc[16];
  int64_t run = offsets[i];
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int y0 = 0; y0 < h; y0 += 16 * s) {
    const int y = y0 + s * wv;
    const uint64_t* row = mb + (int64_t)y * wq;
    const int cnt = y < h ? row_count(row, y, wq, w, s, depth, c) : 0;
    if (lane == 0) rc[wv] = cnt;
    __syncthreads();
    int64_t pos = run;
    int tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wv) pos += rc[k];
      tot += rc[k];
    }
    if (y < h && cnt > 0) {
      for (int k = 0; k < wq; ++k) {
        if (row[k] == 0ull) continue;
        float z;
        const bool v = pixel_valid(row, k, y, w, s, depth, c, z);
        const uint64_t b = __ballot(v);
        if (v) {
          float p[3];
          world_point(c, 64 * k + lane, y, z, p);
          float* o = points + 3 * (pos + __builtin_popcountll(b & below));
          o[0] = p[0];
          o[1] = p[1];
          o[2] = p[2];
        }
        pos += __builtin_popcountll(b);
      }
    }
    run += tot;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// hash grid shared by DBSCAN and the voxel sets
// ---------------------------------------------------------------------------
constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint32_t hash64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)k;
}

// 16-bit biased cell coordinate (cells beyond +-32767 are clamped: the
// distance tests below never depend on the cell a point is filed under
// being its true cell, only on each point being filed once)
__device__ __forceinline__ uint64_t cell16(int v) { return (uint64_t)(min(max(v, -32767), 32767) + 32768); }

__device__ __forceinline__ uint64_t cell_key(int seg, int cx, int cy, int cz) {
  return ((uint64_t)seg << 48) | (cell16(cx) << 32) | (cell16(cy) << 16) | cell16(cz);
}

__device__ __forceinline__ int cell_of(float p, float e) { return (int)floorf(p / e); }

// insert (or find) a key; returns its slot
__device__ __forceinline__ uint32_t hash_insert(uint64_t* keys, uint32_t mask, uint64_t key, bool& fresh) {
  uint32_t h = hash64(key) & mask;
  fresh = false;
  for (;;) {
    const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long*>(keys + h), (unsigned long long)kEmpty,
                                    (unsigned long long)key);
    if (prev == kEmpty) {
      fresh = true;
      return h;
    }
    if (prev == key) return h;
    h = (h + 1) & mask;
  }
}

// slot of a key, or -1 (the table is never full: size >= 2 x keys)
__device__ __forceinline__ int hash_find(const uint64_t* keys, uint32_t mask, uint64_t key) {
  uint32_t h = hash64(key) & mask;
  for (;;) {
    const uint64_t k = keys[h];
    if (k == key) return (int)h;
    if (k == kEmpty) return -1;
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int seg_of(const int32_t* off, int m, int i) {
  int lo = 0, hi = m;  // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// counter[key] += (number of active lanes with that key), one atomic per
// distinct key in the wavefront; returns the old value plus this lane's rank
// among the lanes with its key (lanes whose key repeats are usually
// neighbours: points are grouped by segment and cell)
__device__ __forceinline__ int agg_atomic_add(int32_t* counter, int key, bool active) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint64_t pending = __ballot(active);
  int result = 0;
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int k = __shfl(key, leader);
    const uint64_t same = __ballot(active && key == k) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter + k, __builtin_popcountll(same));
    base = __shfl(base, leader);
    if ((same >> lane) & 1ull) result = base + __builtin_popcountll(same & below);
    pending &= ~same;
  }
  return result;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// DBSCAN noise removal
// ---------------------------------------------------------------------------
struct DbWork {
  uint64_t* keys;  // [T]
  int32_t* cnt;    // [T]
  int32_t* start;  // [T]
  int32_t* cur;    // [T]
  int32_t* slot;   // [n]
  int32_t* idx;    // [n] point indices grouped by slot
  int32_t* core;   // [n] core flag of each sorted position
  float4* spts;    // [n] the points in slot order
  uint32_t mask;   // T - 1
};

__global__ __launch_bounds__(256) void k_db_insert(const float* pts, const int32_t* off, int m, int n, float eps,
                                                   DbWork d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool act = i < n;
  int h = 0;
  if (act) {
    const int seg = seg_of(off, m, i);
    const float* p = pts + 3 * (int64_t)i;
    bool fresh;
    h = (int)hash_insert(d.keys, d.mask, cell_key(seg, cell_of(p[0], eps), cell_of(p[1], eps), cell_of(p[2], eps)),
                         fresh);
    d.slot[i] = h;
  }
  agg_atomic_add(d.cnt, h, act);
}

// counting sort by slot: idx[pos] = point, spts[pos] = its coordinates
__global__ __launch_bounds__(256) void k_db_fill(const float* pts, int n, DbWork d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool act = i < n;
  const int h = act ? d.slot[i] : 0;
  const int r = agg_atomic_add(d.cur, h, act);
  if (!act) return;
  const int pos = d.start[h] + r;
  d.idx[pos] = i;
  const float* p = pts + 3 * (int64_t)i;
  d.spts[pos] = make_float4(p[0], p[1], p[2], __int_as_float(h));
}

__device__ __forceinline__ float sqdist(const float* p, const float* q) {
#pragma clang fp contract(off)
  const float dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
  return (dx * dx + dy * dy) + dz * dz;
}

// Over sorted positions t (points of one cell are adjacent, so a wavefront
// mostly scans the same neighbour lists).  PASS 0: core test (stop at
// min_pts neighbours); PASS 1: border test (stop at the first core
// neighbour), keep written at the point's original index.  The point's own
// cell is visited first.
template <int PASS>
__global__ __launch_bounds__(256) void k_db_scan(const int32_t* off, int m, int n, float eps, int min_pts, DbWork d,
                                                 int32_t* keep) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  if (PASS == 1 && d.core[t]) {
    keep[d.idx[t]] = 1;
    return;
  }
  const float4 pt = d.spts[t];
  const float p[3] = {pt.x, pt.y, pt.z};
  const int seg = (int)(d.keys[__float_as_int(pt.w)] >> 48);
  const float e2 = eps * eps;
  const int cx = cell_of(p[0], eps), cy = cell_of(p[1], eps), cz = cell_of(p[2], eps);
  // clamped cell coordinates can repeat at the edge of the key range: visit
  // each distinct neighbouring cell once (clamping is monotonic, so repeats
  // are adjacent)
  auto rep = [](int c, int dd) { return dd > -1 && cell16(c + dd) == cell16(c + dd - 1); };
  int found = 0;
  bool done = false;
  for (int k27 = 0; k27 < 27 && !done; ++k27) {
    // offsets in the order (0,0,0), then the other 26
    const int c = k27 == 0 ? 13 : (k27 <= 13 ? k27 - 1 : k27);
    const int dz = c / 9 - 1, dy = (c / 3) % 3 - 1, dx = c % 3 - 1;
    if (rep(cz, dz) || rep(cy, dy) || rep(cx, dx)) continue;
    const int h = hash_find(d.keys, d.mask, cell_key(seg, cx + dx, cy + dy, cz + dz));
    if (h < 0) continue;
    const int b = d.start[h], e = b + d.cnt[h];
    for (int k = b; k < e; ++k) {
      const float4 q = d.spts[k];
      const float qq[3] = {q.x, q.y, q.z};
      if (sqdist(p, qq) <= e2 && (PASS == 0 || d.core[k])) {
        if (++found >= (PASS == 0 ? min_pts : 1)) {
          done = true;
          break;
        }
      }
    }
  }
  if (PASS == 0) d.core[t] = done ? 1 : 0;
  else keep[d.idx[t]] = done ? 1 : 0;
}

// ---------------------------------------------------------------------------
// voxel sets
// ---------------------------------------------------------------------------
struct VoxWork {
  uint64_t* keys;   // [T] hash set of (segment, voxel)
  int32_t* vcnt;    // [m]
  int32_t* vcur;    // [m]
  uint64_t* tmp;    // [T] gathered keys, grouped by segment
  int32_t* fresh;   // [n] slot of the key this point inserted first, or -1
  uint32_t mask;
};

// voxel coordinates must fit 16 bits signed (|v| <= 32767): a point outside
// sets its segment's status to 1 and is left out
__global__ __launch_bounds__(256) void k_vox_insert(const float* pts, const int32_t* off, const int32_t* keep, int m,
                                                    int n, float v, VoxWork d, int32_t* status) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  bool fresh = false;
  int seg = 0, h = -1;
  if (i < n && (!keep || keep[i])) {
    seg = seg_of(off, m, i);
    const float* p = pts + 3 * (int64_t)i;
    const int vx = cell_of(p[0], v), vy = cell_of(p[1], v), vz = cell_of(p[2], v);
    if (vx < -32767 || vx > 32767 || vy < -32767 || vy > 32767 || vz < -32767 || vz > 32767) {
      if (status) status[seg] = 1;
    } else {
      h = (int)hash_insert(d.keys, d.mask, cell_key(seg, vx, vy, vz), fresh);
    }
  }
  if (i < n) d.fresh[i] = fresh ? h : -1;
  agg_atomic_add(d.vcnt, seg, fresh);
}

// over the points (grouped by segment, so a wavefront's appends share one
// counter): the point that inserted a key appends it to its segment's range
__global__ __launch_bounds__(256) void k_vox_gather(VoxWork d, int n, const int32_t* voff) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int h = i < n ? d.fresh[i] : -1;
  const bool act = h >= 0;
  const uint64_t k = act ? d.keys[h] : 0ull;
  const int seg = act ? (int)(k >> 48) : 0;
  const int r = agg_atomic_add(d.vcur, seg, act);
  if (act) d.tmp[voff[seg] + r] = k;
}

// One workgroup per segment sorts its keys (distinct, so every key has one
// rank).  Up to kVoxSortMax keys: a bitonic sort in LDS.  More: each chunk of
// kVoxSortMax keys is sorted in LDS and written back in place, then every
// key's rank is its place in its own chunk plus, for every other chunk,
// the number of that chunk's keys below it (a binary search with the chunk
// in LDS); the keys are scattered to their ranks in `sorted` (this segment's
// range of a scratch array) and written out from there.  The ranks are kept
// in the segment's output rows until the scatter.
constexpr int kVoxSortMax = 8192;

__device__ void vox_bitonic(uint64_t* sk, int n) {
  int N = 1;
  while (N < n) N <<= 1;
  for (int k = n + threadIdx.x; k < N; k += 1024) sk[k] = kEmpty;
  __syncthreads();
  for (int size = 2; size <= N; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N / 2; t += 1024) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = sk[lo], c = sk[hi];
        if ((a > c) == up) {
          sk[lo] = c;
          sk[hi] = a;
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ void vox_write(int32_t* o, uint64_t key) {
  o[0] = (int32_t)((key >> 32) & 0xFFFF) - 32768;
  o[1] = (int32_t)((key >> 16) & 0xFFFF) - 32768;
  o[2] = (int32_t)(key & 0xFFFF) - 32768;
}

__global__ __launch_bounds__(1024) void k_vox_sort(uint64_t* tmp, const int32_t* voff, int32_t* vox, uint64_t* sorted) {
  __shared__ uint64_t sk[kVoxSortMax];
  const int seg = blockIdx.x;
  const int b = voff[seg], n = voff[seg + 1] - b;
  if (n == 0) return;
  if (n <= kVoxSortMax) {
    for (int k = threadIdx.x; k < n; k += 1024) sk[k] = tmp[b + k];
    vox_bitonic(sk, n);
    for (int k = threadIdx.x; k < n; k += 1024) vox_write(vox + 3 * (int64_t)(b + k), sk[k]);
    return;
  }
  const int nch = (n + kVoxSortMax - 1) / kVoxSortMax;
  // sorted chunks, in place; each key's rank starts at its place in its chunk
  for (int c = 0; c < nch; ++c) {
    const int c0 = c * kVoxSortMax, len = min(kVoxSortMax, n - c0);
    for (int k = threadIdx.x; k < len; k += 1024) sk[k] = tmp[b + c0 + k];
    vox_bitonic(sk, len);
    for (int k = threadIdx.x; k < len; k += 1024) {
      tmp[b + c0 + k] = sk[k];
      vox[3 * (int64_t)(b + c0 + k)] = k;
    }
    __syncthreads();
  }
  // plus the keys below it in every other chunk
  for (int c = 0; c < nch; ++c) {
    const int c0 = c * kVoxSortMax, len = min(kVoxSortMax, n - c0);
    for (int k = threadIdx.x; k < len; k += 1024) sk[k] = tmp[b + c0 + k];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 1024) {
      if (i >= c0 && i < c0 + len) continue;
      const uint64_t key = tmp[b + i];
      int lo = 0, hi = len;  // first entry not below key
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sk[mid] < key) lo = mid + 1;
        else hi = mid;
      }
      vox[3 * (int64_t)(b + i)] += lo;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += 1024) sorted[b + vox[3 * (int64_t)(b + i)]] = tmp[b + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 1024) vox_write(vox + 3 * (int64_t)(b + i), sorted[b + i]);
}

// ---------------------------------------------------------------------------
// voxel overlap of (segment, instance) pairs
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t vox_code(const int32_t* v) {
  return ((uint64_t)(uint32_t)(v[0] + (1 << 20)) << 42) | ((uint64_t)(uint32_t)(v[1] + (1 << 20)) << 21) |
         (uint64_t)(uint32_t)(v[2] + (1 << 20));
}

// One workgroup per (segment, instance) pair: the longer list is staged in
// LDS in chunks of kOvChunk codes and every key of the shorter list that
// falls inside a chunk's range is binary-searched there.  Voxel coordinates
// within +-2^20 (the voxel sets above are within +-32767).
constexpr int kOvChunk = 4096;

__global__ __launch_bounds__(256) void k_overlap(const int32_t* va, const int32_t* oa, const int32_t* vb,
                                                 const int32_t* ob, const int32_t* pairs, int np, int na, int nb,
                                                 int32_t* out) {
  __shared__ uint64_t sb[kOvChunk];
  __shared__ int red[4];
  const int pr = blockIdx.x;
  const int i = pairs[2 * pr], j = pairs[2 * pr + 1];
  int cnt = 0;
  if (i >= 0 && i < na && j >= 0 && j < nb) {  // uniform over the workgroup
    int a0 = oa[i], a1 = oa[i + 1], b0 = ob[j], b1 = ob[j + 1];
    const int32_t* s = va;  // keys of the shorter list are searched in the longer
    const int32_t* l = vb;
    if (a1 - a0 > b1 - b0) {
      s = vb;
      l = va;
      const int t0 = a0, t1 = a1;
      a0 = b0;
      a1 = b1;
      b0 = t0;
      b1 = t1;
    }
    if (a1 > a0) {
      for (int c0 = b0; c0 < b1; c0 += kOvChunk) {
        const int len = min(kOvChunk, b1 - c0);
        __syncthreads();
        for (int k = threadIdx.x; k < len; k += 256) sb[k] = vox_code(l + 3 * (int64_t)(c0 + k));
        __syncthreads();
        const uint64_t first = sb[0], last = sb[len - 1];
        for (int k = a0 + threadIdx.x; k < a1; k += 256) {
          const uint64_t key = vox_code(s + 3 * (int64_t)k);
          if (key < first || key > last) continue;
          int lo = 0, hi = len;  // first element >= key
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sb[mid] < key) lo = mid + 1;
            else hi = mid;
          }
          cnt += (lo < len && sb[lo] == key) ? 1 : 0;
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) out[pr] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static Cam to_cam(const float* cam) {
  Cam c;
  c.fx = cam[0];
  c.fy = cam[1];
  c.cx = cam[2];
  c.cy = cam[3];
  for (int k = 0; k < 9; ++k) c.R[k] = cam[4 + k];
  for (int k = 0; k < 3; ++k) c.t[k] = cam[13 + k];
  c.dmin = cam[16];
  c.dmax = cam[17];
  return c;
}

size_t scan_scratch_ints(int n) { return 2 * (size_t)((n + kScanBlock - 1) / kScanBlock) + 2; }

void launch_bp_count(const float* depth, const uint64_t* bits, int m, int h, int w, int s, const float* cam,
                     int32_t* counts, int32_t* offsets, int32_t* scratch, hipStream_t st) {
  if (m > 0)
    hipLaunchKernelGGL(k_bp_count, dim3(m), dim3(1024), 0, st, depth, bits, m, h, w, s, to_cam(cam), counts);
  exclusive_scan(counts, m, offsets, true, scratch, st);
}

void launch_bp_write(const float* depth, const uint64_t* bits, int m, int h, int w, int s, const float* cam,
                     const int32_t* offsets, float* points, hipStream_t st) {
  if (m > 0)
    hipLaunchKernelGGL(k_bp_write, dim3(m), dim3(1024), 0, st, depth, bits, m, h, w, s, to_cam(cam), offsets, points);
}

static uint32_t table_size(int n) {
  uint32_t T = 1024;
  while (T < 2u * (uint32_t)n) T <<= 1;
  return T;
}

size_t dbscan_ws_bytes(int n) {
  const size_t T = table_size(n);
  return T * 8 + 3 * T * 4 + 3 * (size_t)n * 4 + (size_t)n * 16 + scan_scratch_ints((int)T) * 4 + 4096;
}

void launch_dbscan(const float* pts, const int32_t* off, int m, int n, float eps, int min_pts, int32_t* keep,
                   char* ws, hipStream_t st) {
  if (n <= 0) return;
  const uint32_t T = table_size(n);
  DbWork d;
  char* p = ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  d.keys = reinterpret_cast<uint64_t*>(take((size_t)T * 8));
  d.cnt = reinterpret_cast<int32_t*>(take((size_t)T * 4));
  d.start = reinterpret_cast<int32_t*>(take((size_t)T * 4));
  d.cur = reinterpret_cast<int32_t*>(take((size_t)T * 4));
  d.slot = reinterpret_cast<int32_t*>(take((size_t)n * 4));
  d.idx = reinterpret_cast<int32_t*>(take((size_t)n * 4));
  d.core = reinterpret_cast<int32_t*>(take((size_t)n * 4));
  d.spts = reinterpret_cast<float4*>(take((size_t)n * 16));
  int32_t* scratch = reinterpret_cast<int32_t*>(take(scan_scratch_ints((int)T) * 4));
  d.mask = T - 1;
  hipLaunchKernelGGL(k_fill_u64, dim3((T + 255) / 256), dim3(256), 0, st, d.keys, kEmpty, (int64_t)T);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d.cnt), 0u, T, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d.cur), 0u, T, st);
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_db_insert, dim3(nb), dim3(256), 0, st, pts, off, m, n, eps, d);
  exclusive_scan(d.cnt, (int)T, d.start, false, scratch, st);
  hipLaunchKernelGGL(k_db_fill, dim3(nb), dim3(256), 0, st, pts, n, d);
  hipLaunchKernelGGL(k_db_scan<0>, dim3(nb), dim3(256), 0, st, off, m, n, eps, min_pts, d, keep);
  hipLaunchKernelGGL(k_db_scan<1>, dim3(nb), dim3(256), 0, st, off, m, n, eps, min_pts, d, keep);
}

size_t voxel_ws_bytes(int n, int m) {
  const size_t T = table_size(n);
  return 2 * T * 8 + 2 * (size_t)(m + 1) * 4 + (size_t)n * 4 + 4 + scan_scratch_ints(m) * 4 + 4096;
}

// distinct voxels per segment -> voff [m + 1]; their keys gathered by
// segment and sorted -> vox [voff[m]][3]
void launch_voxelize(const float* pts, const int32_t* off, const int32_t* keep, int m, int n, float v, int32_t* voff,
                     int32_t* vox, int32_t* status, char* ws, hipStream_t st) {
  const uint32_t T = table_size(n);
  VoxWork d;
  char* p = ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  d.keys = reinterpret_cast<uint64_t*>(take((size_t)T * 8));
  d.tmp = reinterpret_cast<uint64_t*>(take((size_t)T * 8));
  d.vcnt = reinterpret_cast<int32_t*>(take((size_t)(m + 1) * 4));
  d.vcur = reinterpret_cast<int32_t*>(take((size_t)(m + 1) * 4));
  d.fresh = reinterpret_cast<int32_t*>(take((size_t)n * 4 + 4));
  int32_t* scratch = reinterpret_cast<int32_t*>(take(scan_scratch_ints(m) * 4));
  d.mask = T - 1;
  hipLaunchKernelGGL(k_fill_u64, dim3((T + 255) / 256), dim3(256), 0, st, d.keys, kEmpty, (int64_t)T);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d.vcnt), 0u, m + 1, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(d.vcur), 0u, m + 1, st);
  if (status && m > 0) launch_fill_u32(reinterpret_cast<uint32_t*>(status), 0u, m, st);
  if (n > 0)
    hipLaunchKernelGGL(k_vox_insert, dim3((n + 255) / 256), dim3(256), 0, st, pts, off, keep, m, n, v, d, status);
  exclusive_scan(d.vcnt, m, voff, true, scratch, st);
  if (n > 0) hipLaunchKernelGGL(k_vox_gather, dim3((n + 255) / 256), dim3(256), 0, st, d, n, voff);
  // the hash table is free once the keys are gathered: it holds the scattered keys of large segments
  if (m > 0) hipLaunchKernelGGL(k_vox_sort, dim3(m), dim3(1024), 0, st, d.tmp, voff, vox, d.keys);
}

void launch_overlap(const int32_t* va, const int32_t* oa, int na, const int32_t* vb, const int32_t* ob, int nb,
                    const int32_t* pairs, int np, int32_t* out, hipStream_t st) {
  if (np > 0) hipLaunchKernelGGL(k_overlap, dim3(np), dim3(256), 0, st, va, oa, vb, ob, pairs, np, na, nb, out);
}

}  // namespace disc
