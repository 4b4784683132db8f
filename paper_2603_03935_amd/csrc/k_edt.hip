// Exact squared Euclidean distance transform of each mask fused with the
// per-patch reduction of sqrt(EDT): the "distance-weighted" part of DISC's
// single-pass extraction (arXiv 2603.03935, abstract and Sec. V), feeding the
// weights of Sec. III-C.
//
// Separable exact EDT: g = horizontal distance to the nearest pixel outside
// the mask (row pass), then e(y) = min_y' (y - y')^2 + g(y')^2 along each
// column (lower envelope of parabolas, Felzenszwalb & Huttenlocher).
// Pixels outside the frame count as outside the mask.  Only the mask's
// bounding box plus a one-pixel ring is processed: for a pixel in the box some
// nearest outside pixel lies in that ring or inside the box, so the result is
// the full-plane one.
//
// GPU decomposition (one workgroup per (mask, column strip) work item, taken
// from a per-class queue by a persistent grid):
//   * lanes = 64 consecutive columns, wavefront k = rows [96k, 96k+96) of the
//     padded box ("band");
//   * row pass straight from the packed bits: each lane fetches, for one row of
//     its band, the 64-bit window of the strip and the run lengths that
//     continue past the window's ends (all rows in parallel); the sequential
//     pass broadcasts each row with readlane and every lane finds its nearest
//     zero bit with clz/ctz;
//   * each band builds the lower envelope of its own rows; the envelope is a
//     stack of row indices kept as a 96-bit bitmap in registers (exact integer
//     intersection tests, 64-bit cross products);
//   * band envelopes are merged pairwise in LDS (the merged envelope keeps a
//     prefix of the upper one and a suffix of the lower one: pop dominated
//     sites at the junction);
//   * each band walks the final envelope over its rows, producing e exactly,
//     and sums sqrt(e) over each patch (segmented lane reduction per patch
//     row; a patch row split between two bands is finished in fixed order).
#include <mutex>

#include "disc_device.h"

namespace disc {

__device__ __forceinline__ uint64_t valid_bits(int k, int wq, int w) {
  return (k == wq - 1 && (w & 63)) ? ((1ull << (w & 63)) - 1) : ~0ull;
}

// mask pixels in an unbroken run ending at column x (inclusive), going left
__device__ __forceinline__ int run_left(const uint64_t* row, int x, int wq, int w) {
  if (x < 0) return 0;
  int k = x >> 6;
  const int bpos = x & 63;
  uint64_t wd = row[k] & valid_bits(k, wq, w);
  const uint64_t z = ~wd & ((2ull << bpos) - 1);
  if (z) return bpos - 63 + __builtin_clzll(z);
  int L = bpos + 1;
  for (--k; k >= 0; --k) {
    wd = row[k];
    if (~wd) return L + __builtin_clzll(~wd);
    L += 64;
  }
  return L;
}

// mask pixels in an unbroken run starting at column x, going right
__device__ __forceinline__ int run_right(const uint64_t* row, int x, int wq, int w) {
  if (x >= w) return 0;
  int k = x >> 6;
  const int bpos = x & 63;
  uint64_t wd = row[k] & valid_bits(k, wq, w);
  const uint64_t z = ~wd & (~0ull << bpos);
  if (z) return __builtin_ctzll(z) - bpos;
  int R = 64 - bpos;
  for (++k; k < wq; ++k) {
    wd = row[k] & valid_bits(k, wq, w);
    if (~wd) return R + __builtin_ctzll(~wd);
    R += 64;
  }
  return R;
}

// bits [xs, xs+64) of a row (columns >= w read as 0)
__device__ __forceinline__ uint64_t load_window(const uint64_t* row, int xs, int wq, int w) {
  const int k = xs >> 6, bpos = xs & 63;
  const uint64_t lo = row[k] & valid_bits(k, wq, w);
  if (bpos == 0) return lo;
  const uint64_t hi = (k + 1 < wq) ? (row[k + 1] & valid_bits(k + 1, wq, w)) : 0ull;
  return (lo >> bpos) | (hi << (64 - bpos));
}

// horizontal distance of window bit l to the nearest zero, runs extending
// L bits past the left end and R bits past the right end
__device__ __forceinline__ int g_from_window(uint64_t win, int l, int L, int R) {
  const uint64_t inv = ~win;
  const uint64_t zl = inv & ((2ull << l) - 1);
  const int dl = zl ? (l - 63 + __builtin_clzll(zl)) : (l + 1 + L);
  const uint64_t zr = inv & (~0ull << l);
  const int dr = zr ? (__builtin_ctzll(zr) - l) : (64 - l + R);
  return min(dl, dr);
}

// Site m (p < m < q, parabola heights F) never lies strictly below both p and
// q: q overtakes p no later than m does, i.e. Aq/(q-p) <= Am/(m-p) with
// A = F - Fp + (site^2 - p^2).  |A| < 2^22 and the row distances < 2^11, so
// both products are below 2^33 and exact in double precision (FP64 FMA runs
// at the FP32 rate on gfx950, unlike 64-bit integer products).
__device__ __forceinline__ bool dominated(int p, int Fp, int m, int Fm, int q, int Fq) {
  const int Am = (Fm - Fp) + (m - p) * (m + p);
  const int Aq = (Fq - Fp) + (q - p) * (q + p);
  return (double)Aq * (double)(m - p) <= (double)Am * (double)(q - p);
}

__device__ __forceinline__ int parab(int site, int F, int y) { return (y - site) * (y - site) + F; }

// --- the band's stack bitmap in three registers (rows b0 .. b0+95) ---
__device__ __forceinline__ void bm_set(uint32_t& w0, uint32_t& w1, uint32_t& w2, int rel) {
  const uint32_t bit = 1u << (rel & 31);
  const int wi = rel >> 5;
  if (wi == 0) w0 |= bit;
  else if (wi == 1) w1 |= bit;
  else w2 |= bit;
}
__device__ __forceinline__ void bm_clear(uint32_t& w0, uint32_t& w1, uint32_t& w2, int rel) {
  const uint32_t bit = ~(1u << (rel & 31));
  const int wi = rel >> 5;
  if (wi == 0) w0 &= bit;
  else if (wi == 1) w1 &= bit;
  else w2 &= bit;
}
// highest set bit strictly below rel (one always exists: the band's first row)
__device__ __forceinline__ int bm_prev(uint32_t w0, uint32_t w1, uint32_t w2, int rel) {
  const int wi = rel >> 5;
  const uint32_t below = (rel & 31) ? ((1u << (rel & 31)) - 1u) : 0u;
  const uint32_t c2 = wi == 2 ? (w2 & below) : (wi > 2 ? w2 : 0u);
  const uint32_t c1 = wi == 1 ? (w1 & below) : (wi > 1 ? w1 : 0u);
  const uint32_t c0 = wi == 0 ? (w0 & below) : w0;
  if (c2) return 64 + 31 - __builtin_clz(c2);
  if (c1) return 32 + 31 - __builtin_clz(c1);
  return 31 - __builtin_clz(c0);
}

// --- the column's bitmap in LDS: bm[word][lane] ---
// highest set row r with lo <= r < pos (lo a multiple of 32), or -1
__device__ __forceinline__ int lds_prev(const uint32_t* bm, int lane, int pos, int lo) {
  const int x = pos - 1;
  if (x < lo) return -1;
  int wi = x >> 5;
  uint32_t wd = bm[wi * 64 + lane] & (0xFFFFFFFFu >> (31 - (x & 31)));
  const int wlo = lo >> 5;
  for (;;) {
    if (wd) return wi * 32 + 31 - __builtin_clz(wd);
    if (--wi < wlo) return -1;
    wd = bm[wi * 64 + lane];
  }
}
// lowest set row r with pos <= r < hi, or -1
__device__ __forceinline__ int lds_next(const uint32_t* bm, int lane, int pos, int hi) {
  if (pos >= hi) return -1;
  int wi = pos >> 5;
  uint32_t wd = bm[wi * 64 + lane] & (0xFFFFFFFFu << (pos & 31));
  const int whi = (hi + 31) >> 5;
  for (;;) {
    if (wd) {
      const int r = wi * 32 + __builtin_ctz(wd);
      return r < hi ? r : -1;
    }
    if (++wi >= whi) return -1;
    wd = bm[wi * 64 + lane];
  }
}

__device__ __forceinline__ int gsq(const int16_t* g_lds, int row, int lane) {
  const int v = g_lds[row * 64 + lane];
  return v * v;
}

// Merge the envelope of rows [lo, jb) with the envelope of rows [jb, hi).
__device__ void merge_junction(const int16_t* g_lds, uint32_t* bm, int lane, int lo, int jb, int hi) {
  int a1 = lds_prev(bm, lane, jb, lo);
  int b1 = lds_next(bm, lane, jb, hi);
  if (a1 < 0 || b1 < 0) return;
  int a2 = lds_prev(bm, lane, a1, lo);
  int b2 = lds_next(bm, lane, b1 + 1, hi);
  int Fa1 = gsq(g_lds, a1, lane), Fb1 = gsq(g_lds, b1, lane);
  int Fa2 = a2 >= 0 ? gsq(g_lds, a2, lane) : 0;
  int Fb2 = b2 >= 0 ? gsq(g_lds, b2, lane) : 0;
  for (;;) {
    if (a2 >= 0 && dominated(a2, Fa2, a1, Fa1, b1, Fb1)) {
      bm[(a1 >> 5) * 64 + lane] &= ~(1u << (a1 & 31));
      a1 = a2;
      Fa1 = Fa2;
      a2 = lds_prev(bm, lane, a1, lo);
      Fa2 = a2 >= 0 ? gsq(g_lds, a2, lane) : 0;
      continue;
    }
    if (b2 >= 0 && dominated(a1, Fa1, b1, Fb1, b2, Fb2)) {
      bm[(b1 >> 5) * 64 + lane] &= ~(1u << (b1 & 31));
      b1 = b2;
      Fb1 = Fb2;
      b2 = lds_next(bm, lane, b1 + 1, hi);
      Fb2 = b2 >= 0 ? gsq(g_lds, b2, lane) : 0;
      continue;
    }
    break;
  }
}

template <int SPATIAL>  // 0: EDT, 1: AREA (pixel counts, no transform)
__global__ __launch_bounds__(768) void k_edt(Batch b, Work wk, int cls, int rows_cap, int32_t* e_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int16_t* g_lds = reinterpret_cast<int16_t*>(smem);
  uint32_t* bm = reinterpret_cast<uint32_t*>(smem + edt_g_bytes(rows_cap));
  float* part = reinterpret_cast<float*>(smem + edt_g_bytes(rows_cap) + edt_bm_bytes(rows_cap));
  __shared__ int item_sh;

  // the band index is wave-uniform; make that visible so row loops run on scalars
  const int lane = threadIdx.x & 63, kb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), K = blockDim.x >> 6;
  const int32_t* list = wk.items + (int64_t)cls * b.item_cap;
  const int count = wk.counts[cls];
  const int nbm = edt_bm_words(rows_cap);
  const int npart = edt_part_rows(rows_cap) * 16;

  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_sh = atomicAdd(wk.counters + cls, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_sh);
    if (it >= count) break;
    const int item = list[it];
    const int g = item >> kItemStripBits, strip = item & ((1 << kItemStripBits) - 1);
    const FrameDesc fd = b.frames[b.mask_frame[g]];
    const int4 bb = wk.bbox[g];
    const int y0 = bb.x, y1 = bb.y, x0 = bb.z, x1 = bb.w;
    const int P = fd.patch, SW = strip_width(P);
    const int xs = (x0 / P) * P + strip * SW;
    const int n = y1 - y0 + 3;
    const bool lane_ok = lane < SW;
    const int col = xs + lane;
    const int wq = fd.wq, fw = fd.w;
    const uint64_t* mb = fd.bits + (int64_t)(g - fd.mask_base) * fd.h * wq;

    for (int i = threadIdx.x; i < nbm * 64; i += blockDim.x) bm[i] = 0u;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) part[i] = 0.f;
    __syncthreads();

    const int b0 = kb * kBand, b1 = min(b0 + kBand, n);

    // ---- row pass, part 1: lane l fetches the strip window of rows b0 + l and
    // b0 + 64 + l, plus the run lengths that continue past the window's ends
    // (only needed when the edge pixel is inside the mask).  All rows of the
    // band are fetched in parallel; the sequential part reads them back with
    // readlane.
    uint32_t wlo0 = 0, whi0 = 0, wlo1 = 0, whi1 = 0;
    int L0 = 0, R0 = 0, L1 = 0, R1 = 0;
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int u = b0 + lane + 64 * rr;
      if (u < b1 && u > 0 && u < n - 1) {
        const uint64_t* row = mb + (int64_t)(y0 - 1 + u) * wq;
        const uint64_t win = load_window(row, xs, wq, fw);
        const int L = (win & 1ull) ? run_left(row, xs - 1, wq, fw) : 0;
        const int R = (win >> 63) ? run_right(row, xs + 64, wq, fw) : 0;
        if (rr == 0) {
          wlo0 = (uint32_t)win; whi0 = (uint32_t)(win >> 32); L0 = L; R0 = R;
        } else {
          wlo1 = (uint32_t)win; whi1 = (uint32_t)(win >> 32); L1 = L; R1 = R;
        }
      }
    }

    // ---- row pass, part 2 + this band's lower envelope (sequential in u) ----
    uint32_t w0 = 0, w1 = 0, w2 = 0;
    int cnt = 0, s1 = 0, s2 = 0, F1 = 0, F2 = 0;
    for (int u = b0; u < b1; ++u) {
      const int src = (u - b0) & 63;
      const bool hi = (u - b0) >= 64;
      const uint32_t lo32 = __builtin_amdgcn_readlane(hi ? wlo1 : wlo0, src);
      const uint32_t hi32 = __builtin_amdgcn_readlane(hi ? whi1 : whi0, src);
      const int L = __builtin_amdgcn_readlane(hi ? L1 : L0, src);
      const int R = __builtin_amdgcn_readlane(hi ? R1 : R0, src);
      const uint64_t win = ((uint64_t)hi32 << 32) | lo32;
      const int gv = lane_ok ? g_from_window(win, lane, L, R) : 0;
      g_lds[u * 64 + lane] = (int16_t)gv;
      if (SPATIAL == 0) {
        const int Fu = gv * gv;
        while (cnt >= 2 && dominated(s2, F2, s1, F1, u, Fu)) {
          bm_clear(w0, w1, w2, s1 - b0);
          --cnt;
          s1 = s2;
          F1 = F2;
          if (cnt >= 2) {
            s2 = b0 + bm_prev(w0, w1, w2, s1 - b0);
            F2 = gsq(g_lds, s2, lane);
          }
        }
        bm_set(w0, w1, w2, u - b0);
        s2 = s1;
        F2 = F1;
        s1 = u;
        F1 = Fu;
        ++cnt;
      }
    }
    if (SPATIAL == 0 && b0 < n) {
      const int wb = b0 >> 5;
      bm[wb * 64 + lane] = w0;
      if (wb + 1 < nbm) bm[(wb + 1) * 64 + lane] = w1;
      if (wb + 2 < nbm) bm[(wb + 2) * 64 + lane] = w2;
    }
    __syncthreads();

    // ---- merge band envelopes pairwise ----
    if (SPATIAL == 0) {
      for (int step = 1; step < K; step <<= 1) {
        if ((kb % (2 * step)) == 0 && kb + step < K) {
          const int jb = (kb + step) * kBand;
          if (jb < n) merge_junction(g_lds, bm, lane, kb * kBand, jb, min((kb + 2 * step) * kBand, n));
        }
        __syncthreads();
      }
    }

    // ---- final walk: e over the band's rows, sqrt(e) summed per patch ----
    const int prbase = y0 / P;
    float acc = 0.f;
    int cur_pr = -1;
    int c = 0, Fc = 0, nx = -1, Fn = 0;
    if (SPATIAL == 0 && b0 < n) {
      c = lds_prev(bm, lane, b0 + 1, 0);
      Fc = gsq(g_lds, c, lane);
      for (;;) {
        const int p = lds_prev(bm, lane, c, 0);
        if (p < 0) break;
        const int Fp = gsq(g_lds, p, lane);
        if (parab(p, Fp, b0) <= parab(c, Fc, b0)) {
          c = p;
          Fc = Fp;
        } else {
          break;
        }
      }
      nx = lds_next(bm, lane, c + 1, n);
      Fn = nx >= 0 ? gsq(g_lds, nx, lane) : 0;
    }
    auto flush = [&](int pr, float v) {
      v = lane_ok ? v : 0.f;
      const int inseg = lane % P;
      for (int o = 1; o < P; o <<= 1) {
        const float t = __shfl_down(v, o);
        if (inseg + o < P && lane + o < 64) v += t;
      }
      if (inseg == 0 && lane_ok) {
        const int q = lane / P;
        const int first_row = max(pr * P, y0);
        const int band_first = max(y0 - 1 + b0, y0);
        const int slot = band_first <= first_row ? 0 : 1;
        part[((pr - prbase) * 8 + q) * 2 + slot] = v;
      }
    };
    for (int u = b0; u < b1; ++u) {
      int e;
      if (SPATIAL == 0) {
        while (nx >= 0 && parab(nx, Fn, u) <= parab(c, Fc, u)) {
          c = nx;
          Fc = Fn;
          nx = lds_next(bm, lane, c + 1, n);
          Fn = nx >= 0 ? gsq(g_lds, nx, lane) : 0;
        }
        e = (u - c) * (u - c) + Fc;
      } else {
        e = g_lds[u * 64 + lane] > 0 ? 1 : 0;
      }
      if (u >= 1 && u <= n - 2) {
        const int Y = y0 - 1 + u;
        const int pr = Y / P;
        if (pr != cur_pr) {
          if (cur_pr >= 0) flush(cur_pr, acc);
          cur_pr = pr;
          acc = 0.f;
        }
        acc += SPATIAL == 0 ? __builtin_amdgcn_sqrtf((float)e) : (float)e;  // e >= 0 integer: no denormals
        if (e_out != nullptr && lane_ok && col >= x0 && col <= x1)
          e_out[(int64_t)g * fd.h * fw + (int64_t)Y * fw + col] = e;
      }
    }
    if (cur_pr >= 0) flush(cur_pr, acc);
    __syncthreads();

    // ---- write the strip's patch sums ----
    const int npc = SW / P;
    const int npr = y1 / P - prbase + 1;
    const int pc0 = xs / P;
    float* srow = wk.s + fd.w_base + (int64_t)(g - fd.mask_base) * fd.Gs;
    for (int idx = threadIdx.x; idx < npr * npc; idx += blockDim.x) {
      const int prl = idx / npc, q = idx - prl * npc;
      const int pc = pc0 + q;
      if (pc < fd.gw) srow[(prbase + prl) * fd.gw + pc] = part[(prl * 8 + q) * 2] + part[(prl * 8 + q) * 2 + 1];
    }
  }
}

// Per-class LDS attribute and resident workgroups per CU, computed once
// (outside any stream capture).
static std::once_flag g_edt_once;
static int g_edt_per_cu[2][kClasses];

void edt_prepare() {
  std::call_once(g_edt_once, [] {
    for (int sp = 0; sp < 2; ++sp)
      for (int c = 0; c < kClasses; ++c) {
        const int threads = 64 * class_bands(c);
        const size_t lds = (size_t)edt_lds_bytes(class_rows(c));
        const void* fn = sp == 0 ? reinterpret_cast<const void*>(&k_edt<0>) : reinterpret_cast<const void*>(&k_edt<1>);
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
        g_edt_per_cu[sp][c] = per_cu;
      }
  });
}

void launch_edt(const Batch& b, const Work& w, int32_t* e_out, int num_cus, hipStream_t st) {
  edt_prepare();
  const int sp = b.spatial == 0 ? 0 : 1;
  for (int c = 0; c < kClasses; ++c) {
    const int threads = 64 * class_bands(c);
    const int rows = class_rows(c);
    const size_t lds = (size_t)edt_lds_bytes(rows);
    const int grid = num_cus * g_edt_per_cu[sp][c];
    if (sp == 0)
      hipLaunchKernelGGL(k_edt<0>, dim3(grid), dim3(threads), lds, st, b, w, c, rows, e_out);
    else
      hipLaunchKernelGGL(k_edt<1>, dim3(grid), dim3(threads), lds, st, b, w, c, rows, e_out);
  }
}

}  // namespace disc
