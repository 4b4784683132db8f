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
// Two kernels compute it.  The default, k_edt_direct, tabulates g per (row,
// column) in LDS and searches each pixel's column outward (see there).  The
// lower-envelope kernel k_edt (layouts 0 and 1) is kept as a second,
// independent computation of the same bits.
//
// Envelope decomposition (one workgroup per (mask, column strip) work item; a grid
// sized to the resident capacity takes the items of a class in a fixed stride):
//   * lanes = 64 consecutive columns, wavefront k = rows [96k, 96k+96) of the
//     padded box ("band");
//   * row records straight from the packed bits: each lane reads, for one row
//     of its band, the strip's 64-bit window and the run lengths that continue
//     past the window's ends, and stores the (at most two) runs crossing the
//     window as intervals, so that g of any column is two min/max operations
//     (windows crossed by more runs keep the bits and use clz/ctz);
//   * each band builds the lower envelope of its own rows; the envelope is a
//     stack of row indices kept as a 96-bit bitmap in registers (exact
//     intersection tests: cross products below 2^33, exact in FP64);
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

// mask pixels in an unbroken run ending at column x (inclusive), going left;
// the walk stops once the count reaches cap (the result is then >= cap, not
// the run's length: callers that clamp g at cap or below lose nothing)
__device__ __forceinline__ int run_left(const uint64_t* row, int x, int wq, int w, int cap = INT32_MAX) {
  if (x < 0) return 0;
  int k = x >> 6;
  const int bpos = x & 63;
  uint64_t wd = row[k] & valid_bits(k, wq, w);
  const uint64_t z = ~wd & ((2ull << bpos) - 1);
  if (z) return bpos - 63 + __builtin_clzll(z);
  int L = bpos + 1;
  for (--k; k >= 0 && L < cap; --k) {
    wd = row[k];
    if (~wd) return L + __builtin_clzll(~wd);
    L += 64;
  }
  return L;
}

// mask pixels in an unbroken run starting at column x, going right (the walk
// stops at cap as in run_left)
__device__ __forceinline__ int run_right(const uint64_t* row, int x, int wq, int w, int cap = INT32_MAX) {
  if (x >= w) return 0;
  int k = x >> 6;
  const int bpos = x & 63;
  uint64_t wd = row[k] & valid_bits(k, wq, w);
  const uint64_t z = ~wd & (~0ull << bpos);
  if (z) return __builtin_ctzll(z) - bpos;
  int R = 64 - bpos;
  for (++k; k < wq && R < cap; ++k) {
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

// Row record (16 bytes): the strip window's bits (x, y) and up to two runs of
// mask pixels crossing the window as open intervals (a, b) in window
// coordinates, the run lengths past the window's ends folded in, so that
// g(l) = max(0, min(l - a, b - l)).  z = a1 | b1 << 16, w = a2 | b2 << 16.
// A window crossed by three or more runs stores b1 = -32768 and w = L | R << 16
// (run lengths past the two ends) and takes the bit path.
constexpr int kManyRuns = -32768;

__device__ __forceinline__ uint4 make_rowrec(uint64_t win, int L, int R) {
  int a[2] = {0, 0}, bnd[2] = {0, 0};
  int nr = 0;
  uint64_t t = win;
  while (t != 0ull && nr < 3) {
    const int s0 = __builtin_ctzll(t);
    const uint64_t zeros = ~t & (~0ull << s0);
    const int e0 = zeros ? __builtin_ctzll(zeros) - 1 : 63;
    if (nr < 2) {
      a[nr] = (s0 == 0 ? -L : s0) - 1;
      bnd[nr] = (e0 == 63 ? 63 + R : e0) + 1;
    }
    ++nr;
    t = e0 == 63 ? 0ull : (t & (~0ull << (e0 + 1)));
  }
  const uint32_t lo = (uint32_t)win, hi = (uint32_t)(win >> 32);
  if (nr >= 3) return make_uint4(lo, hi, (uint32_t)(0xFFFFu | ((uint32_t)(uint16_t)kManyRuns << 16)), (uint32_t)L | ((uint32_t)R << 16));
  return make_uint4(lo, hi, (uint32_t)(uint16_t)a[0] | ((uint32_t)(uint16_t)bnd[0] << 16),
                    (uint32_t)(uint16_t)a[1] | ((uint32_t)(uint16_t)bnd[1] << 16));
}

// g of window column l from a record with at most two runs
__device__ __forceinline__ int g_runs(uint4 r, int l) {
  const int a1 = (int)(int16_t)(r.z & 0xFFFFu), b1 = (int)r.z >> 16;
  const int a2 = (int)(int16_t)(r.w & 0xFFFFu), b2 = (int)r.w >> 16;
  return max(0, max(min(l - a1, b1 - l), min(l - a2, b2 - l)));
}

// horizontal distance g of window column l from a row record
__device__ __forceinline__ int g_rec(uint4 r, int l) {
  const int b1 = (int)r.z >> 16;
  if (b1 == kManyRuns) return g_from_window(((uint64_t)r.y << 32) | r.x, l, (int)(r.w & 0xFFFFu), (int)(r.w >> 16));
  return g_runs(r, l);
}

// Site m (p < m < q, parabola heights F) never lies strictly below both p and
// q: q overtakes p no later than m does, i.e. Aq/(q-p) <= Am/(m-p) with
// A = F - Fp + (site^2 - p^2).  |A| < 2^27 (g < 2^14) and the row distances
// are below 2^11, so both products are below 2^38: exact 64-bit integer
// products.
__device__ __forceinline__ bool dominated(int p, int Fp, int m, int Fm, int q, int Fq) {
  const int Am = (Fm - Fp) + __mul24(m - p, m + p);
  const int Aq = (Fq - Fp) + __mul24(q - p, q + p);
  return (int64_t)Aq * (m - p) <= (int64_t)Am * (q - p);
}

__device__ __forceinline__ int parab(int site, int F, int y) { return __mul24(y - site, y - site) + F; }

// --- the band's stack bitmap in NW (1..3) registers, rows b0 .. b0 + 32 NW - 1 ---
template <int NW>
struct BandBits {
  uint32_t w0 = 0u, w1 = 0u, w2 = 0u;
  __device__ __forceinline__ void set(int rel) {
    if (NW == 1) {
      w0 |= 1u << rel;
    } else {
      const uint32_t bit = 1u << (rel & 31);
      const int wi = rel >> 5;
      w0 = wi == 0 ? (w0 | bit) : w0;
      w1 = wi == 1 ? (w1 | bit) : w1;
      if (NW > 2) w2 = wi == 2 ? (w2 | bit) : w2;
    }
  }
  __device__ __forceinline__ void clear(int rel) {
    if (NW == 1) {
      w0 &= ~(1u << rel);
    } else {
      const uint32_t bit = ~(1u << (rel & 31));
      const int wi = rel >> 5;
      w0 = wi == 0 ? (w0 & bit) : w0;
      w1 = wi == 1 ? (w1 & bit) : w1;
      if (NW > 2) w2 = wi == 2 ? (w2 & bit) : w2;
    }
  }
  // highest set bit strictly below rel (one always exists: the band's first row)
  __device__ __forceinline__ int prev(int rel) const {
    if (NW == 1) return 31 - __builtin_clz(w0 & ((1u << rel) - 1u));
    const int wi = rel >> 5;
    const uint32_t below = (rel & 31) ? ((1u << (rel & 31)) - 1u) : 0u;
    const uint32_t c0 = wi == 0 ? (w0 & below) : w0;
    const uint32_t c1 = wi == 1 ? (w1 & below) : (wi > 1 ? w1 : 0u);
    const uint32_t c2 = NW > 2 ? (wi == 2 ? (w2 & below) : 0u) : 0u;
    if (c2) return 64 + 31 - __builtin_clz(c2);
    if (c1) return 32 + 31 - __builtin_clz(c1);
    return 31 - __builtin_clz(c0);
  }
  // lowest set bit at or above rel (0 <= rel < 32 NW), or -1
  __device__ __forceinline__ int next(int rel) const {
    if (NW == 1) {
      const uint32_t m = w0 & (0xFFFFFFFFu << rel);
      return m ? __builtin_ctz(m) : -1;
    }
    const int wi = rel >> 5;
    const uint32_t above = 0xFFFFFFFFu << (rel & 31);
    const uint32_t c0 = wi == 0 ? (w0 & above) : 0u;
    const uint32_t c1 = wi == 1 ? (w1 & above) : (wi < 1 ? w1 : 0u);
    const uint32_t c2 = NW > 2 ? (wi == 2 ? (w2 & above) : (wi < 2 ? w2 : 0u)) : 0u;
    if (c0) return __builtin_ctz(c0);
    if (c1) return 32 + __builtin_ctz(c1);
    if (c2) return 64 + __builtin_ctz(c2);
    return -1;
  }
  __device__ __forceinline__ uint32_t word(int i) const { return i == 0 ? w0 : i == 1 ? w1 : w2; }
};

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

// g^2 of column `lane` in row `row`, recomputed from the row's record
// (g < 2^16, so the square is one 24-bit multiply)
__device__ __forceinline__ int sq16(int g) {
  const uint32_t v = (uint32_t)g & 0xFFFFu;
  return (int)(v * v);
}
// many = some row of the packet crosses three or more runs (uniform): else
// the records decode without the bit path and without a branch
__device__ __forceinline__ int gsq(const uint4* rec, int row, int lane, bool lane_ok, bool many) {
  const uint4 r = rec[row];
  const int g = many ? g_rec(r, lane) : g_runs(r, lane);
  return lane_ok ? sq16(g) : 0;
}

// Merge the envelope of rows [lo, jb) with the envelope of rows [jb, hi)
// (lo and jb multiples of 32): pop dominated sites on either side of the
// junction.  The bitmap words holding the two innermost sites stay in
// registers while sites are popped and are written back once at the end.
__device__ void merge_junction(const uint4* rec, uint32_t* bm, int lane, bool lane_ok, bool many, int lo, int jb,
                               int hi) {
  int a1 = lds_prev(bm, lane, jb, lo);
  int b1 = lds_next(bm, lane, jb, hi);
  if (a1 < 0 || b1 < 0) return;
  int uwi = a1 >> 5, lwi = b1 >> 5;  // words holding a1 and b1
  uint32_t uwd = bm[uwi * 64 + lane], lwd = bm[lwi * 64 + lane];
  bool udirty = false, ldirty = false;
  // next site below a1 / above b1, from the cached word first
  auto below = [&](int a) -> int {
    const uint32_t m = uwd & ((1u << (a & 31)) - 1u);
    if (m) return (uwi << 5) + 31 - __builtin_clz(m);
    return lds_prev(bm, lane, uwi << 5, lo);
  };
  auto above = [&](int b) -> int {
    const uint32_t m = (b & 31) == 31 ? 0u : (lwd & (0xFFFFFFFEu << (b & 31)));
    if (m) {
      const int r = (lwi << 5) + __builtin_ctz(m);
      return r < hi ? r : -1;
    }
    return lds_next(bm, lane, (lwi + 1) << 5, hi);
  };
  int a2 = below(a1);
  int b2 = above(b1);
  int Fa1 = gsq(rec, a1, lane, lane_ok, many), Fb1 = gsq(rec, b1, lane, lane_ok, many);
  int Fa2 = a2 >= 0 ? gsq(rec, a2, lane, lane_ok, many) : 0;
  int Fb2 = b2 >= 0 ? gsq(rec, b2, lane, lane_ok, many) : 0;
  for (;;) {
    if (a2 >= 0 && dominated(a2, Fa2, a1, Fa1, b1, Fb1)) {
      uwd &= ~(1u << (a1 & 31));
      udirty = true;
      a1 = a2;
      Fa1 = Fa2;
      if ((a1 >> 5) != uwi) {
        bm[uwi * 64 + lane] = uwd;
        uwi = a1 >> 5;
        uwd = bm[uwi * 64 + lane];
        udirty = false;
      }
      a2 = below(a1);
      Fa2 = a2 >= 0 ? gsq(rec, a2, lane, lane_ok, many) : 0;
      continue;
    }
    if (b2 >= 0 && dominated(a1, Fa1, b1, Fb1, b2, Fb2)) {
      lwd &= ~(1u << (b1 & 31));
      ldirty = true;
      b1 = b2;
      Fb1 = Fb2;
      if ((b1 >> 5) != lwi) {
        bm[lwi * 64 + lane] = lwd;
        lwi = b1 >> 5;
        lwd = bm[lwi * 64 + lane];
        ldirty = false;
      }
      b2 = above(b1);
      Fb2 = b2 >= 0 ? gsq(rec, b2, lane, lane_ok, many) : 0;
      continue;
    }
    break;
  }
  if (udirty) bm[uwi * 64 + lane] = uwd;
  if (ldirty) bm[lwi * 64 + lane] = lwd;
}

// Partial patch sums of one 16-row block: the per-lane sums v of the block's
// rows in patch row pr are added across the P lanes of each patch (a fixed
// tree) and stored at (block, patch row within the block, patch column).
__device__ __forceinline__ void flush_patch_part(float* part, int lane, bool lane_ok, int P, int y0, int blk, int pr,
                                                 float v) {
  v = lane_ok ? v : 0.f;
  const int inseg = lane % P;
  for (int o = 1; o < P; o <<= 1) {
    const float t = __shfl_down(v, o);
    if (inseg + o < P && lane + o < 64) v += t;
  }
  const int pf_blk = (y0 - 1 + max(blk * kBlkRows, 1)) / P;  // first patch row the block meets
  if (inseg == 0 && lane_ok) part[(blk * kEdtPartRows + (pr - pf_blk)) * 8 + lane / P] = v;
}

// The strip's patch sums: each patch row adds the partial sums of the 16-row
// blocks that meet it, in block order.  Wavefront j of the K that share the
// item takes every K-th patch.
__device__ __forceinline__ void strip_patch_sums(const float* part, float* srow, int lane, int j, int K, int P, int SW,
                                                 int xs, int y0, int y1, int gw) {
  const int npc = SW / P;
  const int prbase = y0 / P;
  const int npr = y1 / P - prbase + 1;
  const int pc0 = xs / P;
  for (int idx = j * 64 + lane; idx < npr * npc; idx += K * 64) {
    const int prl = idx / npc, q = idx - prl * npc;
    const int pc = pc0 + q;
    const int pr = prbase + prl;
    const int ua = max(pr * P, y0) - y0 + 1, ub = min(pr * P + P - 1, y1) - y0 + 1;
    float v = 0.f;
    for (int kk = ua / kBlkRows; kk <= ub / kBlkRows; ++kk) {
      const int pf_blk = (y0 - 1 + max(kk * kBlkRows, 1)) / P;
      v += part[(kk * kEdtPartRows + (pr - pf_blk)) * 8 + q];
    }
    if (pc < gw) srow[pr * gw + pc] = v;
  }
}

// Packets: the items of class c are grouped class_items(c) at a time; the
// packets of the tallest class come first so that the longest work starts
// first.  Returns the class of packet p (or -1 past the end) and the item word
// of wavefront kb's slot in it (or -1 when that slot is empty).
__device__ __forceinline__ int packet_slot(int mode, const int* ccnt, const int32_t* counts, const int32_t* items,
                                           int item_cap, int p, int kb, int& word) {
  word = -1;
#pragma unroll
  for (int c = kClasses - 1; c >= 0; --c) {
    const int ipp = class_items(mode, c);
    const int cnt = ccnt[c];
    const int np = (cnt + ipp - 1) / ipp;
    if (p < np) {
      const int slot = kb / class_waves(mode, c);
      const int k = p * ipp + slot;
      if (slot < ipp && k < cnt) word = class_item(counts, items, item_cap, c, k);
      return c;
    }
    p -= np;
  }
  return -1;
}

// One packet: wavefront kb holds band j of the item in slot kb / K (its mask
// record broadcast from pf; word < 0: no item).  `prefetch` is called once,
// after the row records are in LDS, to start loading the next packet.
template <int SPATIAL, int B, bool WE, typename Prefetch>
__device__ __forceinline__ void edt_packet(int K, uint32_t pf, int word, uint4* rec_all, uint32_t* bm_all,
                                           float* part_all, int lane, int kb, int32_t* e_out, Prefetch prefetch) {
  constexpr int NW = B / 32;
  const int rows_c = B * K;
  const int slot = kb / K, j = kb - slot * K;  // item slot in the packet, band in the item
  const bool has = word >= 0;
  const int strip = has ? (word & ((1 << kItemStripBits) - 1)) : 0;
  auto fld = [&](int q) { return (int)__builtin_amdgcn_readlane(pf, q); };
  const uint64_t* mb = reinterpret_cast<const uint64_t*>(((uint64_t)(uint32_t)fld(1) << 32) | (uint32_t)fld(0));
  float* srow = reinterpret_cast<float*>(((uint64_t)(uint32_t)fld(3) << 32) | (uint32_t)fld(2));
  const int y0 = fld(4), y1 = fld(5), x0 = fld(6), x1 = fld(7);
  const int n = has ? fld(8) : 0;
  const int P = has ? fld(9) : kMinPatch;
  const int gw = fld(10), wq = fld(11), fw = fld(12), fh = fld(13), xs0 = fld(14), gidx = fld(15);
  const int SW = strip_width(P);
  const int xs = xs0 + strip * SW;
  const bool lane_ok = lane < SW;
  const int col = xs + lane;
  // this item's rows and bitmap words in LDS (rows_c is a multiple of 32)
  uint4* rec = rec_all + slot * rows_c;
  uint32_t* bm = bm_all + (slot * rows_c / 32) * 64;
  float* part = part_all + (slot * rows_c / kBlkRows) * kEdtPartRows * 8;  // this item's blocks

  const int b0 = j * B, b1 = min(b0 + B, n);

  // ---- row records: lane l reads rows b0 + l (and b0 + 64 + l) of its band:
  // the strip's 64-bit window and the run lengths past the window's ends
  // (only read when the edge pixel is inside the mask).
  constexpr int NR = (B + 63) / 64;
  uint4 rreg[NR];  // this lane's rows' records, kept for the sequential pass
  bool my_many = false;
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    const int u = b0 + lane + 64 * rr;
    rreg[rr] = make_uint4(0u, 0u, 0u, 0u);  // padding row: no runs
    if (lane + 64 * rr < B && u < b1) {
      if (u > 0 && u < n - 1) {
        const uint64_t* row = mb + (int64_t)(y0 - 1 + u) * wq;
        const uint64_t win = load_window(row, xs, wq, fw);
        const int L = (win & 1ull) ? run_left(row, xs - 1, wq, fw) : 0;
        const int R = (win >> 63) ? run_right(row, xs + 64, wq, fw) : 0;
        rreg[rr] = make_rowrec(win, L, R);
      }
      rec[u] = rreg[rr];
      my_many |= ((int)rreg[rr].z >> 16) == kManyRuns;
    }
  }
  const bool many = __builtin_amdgcn_readfirstlane(__syncthreads_or(my_many ? 1 : 0)) != 0;
  prefetch();

  // ---- this band's lower envelope (sequential in u; row u's record is
  // broadcast from the lane that read it) ----
  if (SPATIAL == 0 && b0 < n) {
    BandBits<NW> w;
    // Stack top s1 and the site below it, s2, with K = F + site^2.  The top
    // is dominated by a new site u iff (Ku - K2)(s1 - s2) <= (K1 - K2)(u - s2)
    // (the three-site test above in this form); the products are below 2^39,
    // exact in 64-bit integers.  d12 = s1 - s2 and dK = K1 - K2 are kept
    // while the stack is unchanged.
    int depth = 0, s1 = 0, s2 = 0, K1 = 0, K2 = 0;
    int d12 = 0, dK = 0;
    for (int u = b0; u < b1; ++u) {
      uint4 ru;
      if (NR == 1) {
        const int k = u - b0;
        ru = make_uint4(__builtin_amdgcn_readlane(rreg[0].x, k), __builtin_amdgcn_readlane(rreg[0].y, k),
                        __builtin_amdgcn_readlane(rreg[0].z, k), __builtin_amdgcn_readlane(rreg[0].w, k));
      } else {
        ru = rec[u];  // one broadcast LDS read
      }
      const int gu = many ? g_rec(ru, lane) : g_runs(ru, lane);
      const int Ku = (lane_ok ? sq16(gu) : 0) + u * u;
      bool pop = depth >= 2 && (int64_t)(Ku - K2) * d12 <= (int64_t)dK * (u - s2);
      while (pop) {
        w.clear(s1 - b0);
        --depth;
        s1 = s2;
        K1 = K2;
        pop = false;
        if (depth >= 2) {
          s2 = b0 + w.prev(s1 - b0);
          K2 = gsq(rec, s2, lane, lane_ok, many) + __mul24(s2, s2);
          d12 = s1 - s2;
          dK = K1 - K2;
          pop = (int64_t)(Ku - K2) * d12 <= (int64_t)dK * (u - s2);
        }
      }
      w.set(u - b0);
      s2 = s1;
      K2 = K1;
      s1 = u;
      K1 = Ku;
      ++depth;
      d12 = s1 - s2;
      dK = K1 - K2;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) bm[((b0 >> 5) + i) * 64 + lane] = w.word(i);
  }
  __syncthreads();

  // ---- merge band envelopes pairwise ----
  if (SPATIAL == 0) {
    for (int step = 1; step < K; step <<= 1) {
      if ((j % (2 * step)) == 0 && j + step < K) {
        const int jb = (j + step) * B;
        if (jb < n) merge_junction(rec, bm, lane, lane_ok, many, j * B, jb, min((j + 2 * step) * B, n));
      }
      __syncthreads();
    }
  }

  // ---- final walk: e over the band's rows, sqrt(e) summed per patch ----
  const int pfirst = (y0 - 1 + max(b0, 1)) / P;  // first patch row this band meets
  float acc = 0.f;
  int c = 0, Fc = 0, nx = -1, Fn = 0;
  if (SPATIAL == 0 && b0 < n) {
    c = lds_prev(bm, lane, b0 + 1, 0);
    Fc = gsq(rec, c, lane, lane_ok, many);
    for (;;) {
      const int q = lds_prev(bm, lane, c, 0);
      if (q < 0) break;
      const int Fq = gsq(rec, q, lane, lane_ok, many);
      if (parab(q, Fq, b0) <= parab(c, Fc, b0)) {
        c = q;
        Fc = Fq;
      } else {
        break;
      }
    }
    nx = lds_next(bm, lane, c + 1, n);
    Fn = nx >= 0 ? gsq(rec, nx, lane, lane_ok, many) : 0;
  }
  // the band's own bitmap word(s) stay in registers for the walk
  const int cw0 = b0 >> 5;
  BandBits<NW> cw;
  if (SPATIAL == 0 && b0 < n) {
    cw.w0 = bm[cw0 * 64 + lane];
    if (NW > 1) cw.w1 = bm[(cw0 + 1) * 64 + lane];
    if (NW > 2) cw.w2 = bm[(cw0 + 2) * 64 + lane];
  }
  // lowest envelope row r with pos <= r < n, or -1: from the band's own
  // bitmap words in registers when pos lies in them (no branch), else (rare)
  // from LDS
  auto next_site = [&](int pos) -> int {
    const int base = cw0 << 5;
    const int rel = pos - base;
    const bool in = (unsigned)rel < 32u * NW;
    const int r0 = cw.next(in ? rel : 0);
    int r = (in && r0 >= 0) ? base + r0 : -1;
    if (r < 0) r = lds_next(bm, lane, in ? base + 32 * NW : pos, n);
    return r < n ? r : -1;
  };
  auto flush = [&](int blk, int pr, float v) { flush_patch_part(part, lane, lane_ok, P, y0, blk, pr, v); };
  // rows 0 and n-1 are padding and produce nothing: walk rows [ua, ub) in
  // segments that end where a patch row or a 16-row block ends (flush points)
  const int ua = max(b0, 1), ub = min(b1, n - 1);
  int pr = (y0 - 1 + ua) / P;               // patch row of row u
  int pr_next = (pr + 1) * P - (y0 - 1);    // first row of the next patch row
  int blk = ua / kBlkRows, blk_next = (blk + 1) * kBlkRows;
  // site nx takes over from c at row u iff Fn - Fc <= (nx - c)(2u - c - nx);
  // without a next site the test is made false (dF = 2^30, dc = 0)
  int dF = nx >= 0 ? Fn - Fc : (1 << 30), dc = nx >= 0 ? nx - c : 0, sc = nx + c;
  int u = ua;
  while (u < ub) {
    const int seg_end = min(ub, min(pr_next, blk_next));
    for (; u < seg_end; ++u) {
      int e;
      if (SPATIAL == 0) {
        while (dF <= __mul24(dc, 2 * u - sc)) {
          c = nx;
          Fc = Fn;
          nx = next_site(c + 1);
          Fn = nx >= 0 ? gsq(rec, nx, lane, lane_ok, many) : 0;
          dF = nx >= 0 ? Fn - Fc : (1 << 30);
          dc = nx >= 0 ? nx - c : 0;
          sc = nx + c;
        }
        e = __mul24(u - c, u - c) + Fc;
      } else {
        e = gsq(rec, u, lane, lane_ok, many) > 0 ? 1 : 0;
      }
      acc += SPATIAL == 0 ? __builtin_amdgcn_sqrtf((float)e) : (float)e;  // e >= 0 integer: no denormals
      if (WE && lane_ok && col >= x0 && col <= x1)
        e_out[(int64_t)gidx * fh * fw + (int64_t)(y0 - 1 + u) * fw + col] = e;
    }
    if (u < ub) {  // u is a flush point
      flush(blk, pr, acc);
      acc = 0.f;
      if (u == pr_next) {
        ++pr;
        pr_next += P;
      }
      if (u == blk_next) {
        ++blk;
        blk_next += kBlkRows;
      }
    }
  }
  if (ua < ub) flush(blk, pr, acc);
  __syncthreads();

  if (has) strip_patch_sums(part, srow, lane, j, K, P, SW, xs, y0, y1, gw);
  __syncthreads();
}

// Band layout for this launch (uniform over the grid): mode 1 when the work
// in mode-0 wavefronts exceeds four times what the grid holds at once.
__device__ __forceinline__ int pick_mode(const int32_t* counts, int item_cap, int mode_arg) {
  if (mode_arg >= 0) return mode_arg;
  int64_t waves0 = 0;
  for (int c = 0; c < kClasses; ++c) waves0 += (int64_t)class_count(counts, item_cap, c) * class_waves(0, c);
  return waves0 > 4ll * gridDim.x * kEdtWaves ? 1 : 0;
}

// SPATIAL 0: EDT, 1: AREA (pixel counts, no transform); WE: also write e
template <int SPATIAL, bool WE>
__global__ __launch_bounds__(kEdtWaves * 64) __attribute__((amdgpu_waves_per_eu(8))) void k_edt(
    const int32_t* __restrict__ counts, const int32_t* __restrict__ items, int item_cap,
    const MaskRec* __restrict__ mrec, int32_t* e_out, int mode_arg) {
  __shared__ uint4 rec_all[kMaxRows];
  __shared__ uint32_t bm_all[kEdtBmWords * 64];
  __shared__ float part_all[kEdtBlocks * kEdtPartRows * 8];

  // the wavefront index is uniform; make that visible so row loops run on scalars
  const int lane = threadIdx.x & 63, kb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int mode = pick_mode(counts, item_cap, mode_arg);
  int total = 0;
  int cnt[kClasses];
  for (int c = 0; c < kClasses; ++c) cnt[c] = class_count(counts, item_cap, c);
  for (int c = 0; c < kClasses; ++c) total += (cnt[c] + class_items(mode, c) - 1) / class_items(mode, c);

  // Packets are taken in a fixed stride (no shared queue).  Each wavefront
  // prefetches the record of its item in the next packet into one VGPR per
  // lane (lane j holds dword j) and broadcasts it with readlane.
  int p = blockIdx.x;
  if (p >= total) return;
  int word = -1;
  int cls = packet_slot(mode, cnt, counts, items, item_cap, p, kb, word);
  uint32_t pf = 0u;
  if (word >= 0 && lane < 16) pf = reinterpret_cast<const uint32_t*>(mrec + (word >> kItemStripBits))[lane];

  for (; p < total; p += gridDim.x) {
    int ncls = -1, nword = -1;
    uint32_t npf = pf;
    auto prefetch = [&]() {
      if (p + (int)gridDim.x < total) {
        ncls = packet_slot(mode, cnt, counts, items, item_cap, p + gridDim.x, kb, nword);
        if (nword >= 0 && lane < 16) npf = reinterpret_cast<const uint32_t*>(mrec + (nword >> kItemStripBits))[lane];
      }
    };
    const int B = class_band(mode, cls), K = class_waves(mode, cls);
    if (B == 96)
      edt_packet<SPATIAL, 96, WE>(K, pf, word, rec_all, bm_all, part_all, lane, kb, e_out, prefetch);
    else if (B == 64)
      edt_packet<SPATIAL, 64, WE>(K, pf, word, rec_all, bm_all, part_all, lane, kb, e_out, prefetch);
    else
      edt_packet<SPATIAL, 32, WE>(K, pf, word, rec_all, bm_all, part_all, lane, kb, e_out, prefetch);
    cls = ncls;
    word = nword;
    pf = npf;
  }
}

// ---------------------------------------------------------------------------
// Direct column search (layouts -1 and 2).  With g tabulated per (row,
// column) in LDS, the column pass e(u) = min_v (u - v)^2 + g(v)^2 is searched
// outward from u: distance d is visited while d^2 is below the best value so
// far, so a pixel costs about its own distance in steps, and no row or column
// waits on another (no envelope, no band merges).  Rows 0 and n-1 of an item
// are padding (g = 0): a search that reaches one of them ends there.  The
// sums of sqrt(e) are formed as by the envelope walk (per 16-row block and
// patch row, rows in order, the same lane tree), so all layouts give the same
// bits.
//
// Packets: class c <= 4 items (2^c x 32 rows) are packed 16 >> c to a packet
// of 512 rows, a class-5 item (up to 1152 rows) is a packet alone.  A
// workgroup tabulates g for the whole packet, then its 16 wavefronts take the
// packet's 16-row blocks in a stride.  When the batch has few packets (at
// most half the resident workgroups), up to kDirSplitMax workgroups share a
// packet: each tabulates it and searches every S-th block, the block partial
// sums go to global memory and k_edt_dsums adds them.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int direct_items(int c) { return c == 5 ? 1 : (kEdtWaves >> c); }
// run lengths past a strip window's ends are needed up to the largest g the
// tables keep (576, the bound of the tallest class); AREA needs only g > 0
constexpr int kDirRunCap = 576;
constexpr int kDirRows = 4;   // rows searched together
constexpr int kDirSteps = 4;  // distances per search step (windows start on 4-row words)
// A group's search reads at most kDirRows + kDirSteps - 2 rows past its item
// on either side (a row that is done keeps being updated while another row of
// its group searches; a step visits kDirSteps distances): zeroed guard rows
// at the ends of the table, real rows of the neighbouring slot elsewhere
// (every slot row is written, 0 past its item, so every value read is a
// g <= 8448 and the arithmetic cannot overflow; a candidate read past the
// item can no longer win).
constexpr int kDirGuard = 12;
static_assert(kDirGuard >= kDirRows + kDirSteps - 2 && kDirGuard % 4 == 0, "guard rows");
static_assert(kDirRows == 4 && kDirSteps == 4 && kBlkRows % kDirRows == 0, "search windows are whole 4-row words");

// the packets of the classes in the kernel's range (tallest first)
__device__ __forceinline__ int direct_count(const int32_t* counts, int item_cap, bool tall, int* cnt) {
  int total = 0;
#pragma unroll
  for (int c = 0; c < kClasses; ++c) {
    cnt[c] = tall == (c == 5) ? class_count(counts, item_cap, c) : 0;
    total += (cnt[c] + direct_items(c) - 1) / direct_items(c);
  }
  return total;
}
// workgroups per packet (uniform over the launch)
__device__ __forceinline__ int direct_split(bool tall, int total, int grid) {
  return (!tall && total > 0 && 2 * total <= grid && total <= kDirSplitPackets) ? min(kDirSplitMax, grid / total) : 1;
}
// class of packet p, its first item index and the class's item count
__device__ __forceinline__ int direct_packet_class(const int* cnt, int p, int& first, int& ccount) {
#pragma unroll
  for (int c = kClasses - 1; c >= 0; --c) {
    const int ipp = direct_items(c);
    const int np = (cnt[c] + ipp - 1) / ipp;
    if (p < np) {
      first = p * ipp;
      ccount = cnt[c];
      return c;
    }
    p -= np;
  }
  return -1;
}
// item words and mask records of packet p's slots into LDS (recs: 16 dwords per slot)
__device__ __forceinline__ int direct_load_packet(const int* cnt, const int32_t* counts, const int32_t* items,
                                                  int item_cap, const MaskRec* mrec, int p, uint32_t* recs, int* words) {
  int first = 0, ccount = 0;
  const int cls = direct_packet_class(cnt, p, first, ccount);
  const int ipp = direct_items(cls);
  if ((int)threadIdx.x < ipp * 16) {
    const int sl = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int k = first + sl;
    const int word = k < ccount ? class_item(counts, items, item_cap, cls, k) : -1;
    if (q == 0) words[sl] = word;
    recs[sl * 16 + q] = word >= 0 ? reinterpret_cast<const uint32_t*>(mrec + (word >> kItemStripBits))[q] : 0u;
  }
  __syncthreads();
  return cls;
}

struct DirItem {
  const uint64_t* mb;
  float* srow;
  int y0, y1, x0, x1, n, P, gw, wq, fw, fh, gidx, SW, xs;
  bool has;
};
__device__ __forceinline__ DirItem direct_item(const uint32_t* recs, const int* words, int slot) {
  auto fld = [&](int q) { return (int)__builtin_amdgcn_readfirstlane(recs[slot * 16 + q]); };
  DirItem it;
  const int word = __builtin_amdgcn_readfirstlane(words[slot]);
  it.has = word >= 0;
  it.mb = reinterpret_cast<const uint64_t*>(((uint64_t)(uint32_t)fld(1) << 32) | (uint32_t)fld(0));
  it.srow = reinterpret_cast<float*>(((uint64_t)(uint32_t)fld(3) << 32) | (uint32_t)fld(2));
  it.y0 = fld(4);
  it.y1 = fld(5);
  it.x0 = fld(6);
  it.x1 = fld(7);
  it.n = it.has ? fld(8) : 0;
  it.P = it.has ? fld(9) : kMinPatch;
  it.gw = fld(10);
  it.wq = fld(11);
  it.fw = fld(12);
  it.fh = fld(13);
  it.gidx = fld(15);
  it.SW = strip_width(it.P);
  it.xs = fld(14) + (it.has ? (word & ((1 << kItemStripBits) - 1)) : 0) * it.SW;
  return it;
}

// The patch sums of packet slots from their block partial sums (part: the
// packet's blocks, kEdtPartRows x 8 floats each): wavefront kb of the
// 16 / ipp that share a slot.
__device__ __forceinline__ void direct_strip_sums(int cls, const uint32_t* recs, const int* words, const float* part,
                                                  int lane, int kb) {
  const int ipp = direct_items(cls), rows_c = class_rows(cls);
  const int K = kEdtWaves / ipp, slot = kb / K, j = kb - slot * K;
  const DirItem it = direct_item(recs, words, slot);
  if (it.has)
    strip_patch_sums(part + (slot * rows_c / kBlkRows) * kEdtPartRows * 8, it.srow, lane, j, K, it.P, it.SW, it.xs,
                     it.y0, it.y1, it.gw);
}

typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ us2 as_us2(uint32_t x) { return __builtin_bit_cast(us2, x); }
__device__ __forceinline__ us2 sq2(uint32_t x) { const us2 v = as_us2(x); return v * v; }
__device__ __forceinline__ int max4(us2 a, us2 b) {
  const us2 m = __builtin_elementwise_max(a, b);
  return max((int)m.x, (int)m.y);
}

// PK = 1: items of at most 512 rows.  Every e is then at most 255^2 (rows 0
// and n - 1 are padding with g = 0, and min(u, n - 1 - u) <= 255), so g is
// clamped to 255 (a candidate with g >= 255 is >= 255^2 >= e either way: no
// e changes) and the table holds g^2 (< 2^16).  The search runs in packed
// 16-bit arithmetic, two rows per instruction: sums saturate at 65535, which
// is never below the best value (<= 65025).
// PK = 2: taller items (up to 1152 rows).  Every e is at most 575^2, so g is
// clamped to 576, and the table holds T(g) = g^2 for g < 255 and
// 255^2 + (g - 255) above (at most 65346, 16 bits; T(g) <= g^2 and T grows
// with g).  The packed search over T is exact for every row whose e is below
// 255^2 (each clamped candidate is at least 255^2); a group in which some row
// ends at 255^2 or above is searched again in exact 32-bit arithmetic,
// decoding g^2 from T.  Those are the rows more than 254 pixels from the
// mask's outside, a small share of the tallest items.
// PK = 0: the table holds g and the search is exact 32-bit (AREA of the
// taller items).
// The g table of a packet (PK 1: min(g, 255)^2; PK 2: T(min(g, 576)); PK 0:
// g; 0 past each slot's item), 16 bits per (row, column), four rows per
// 64-bit word.
template <int PK>
__device__ __forceinline__ void direct_table(int cls, const uint32_t* recs, const int* words, uint2* gt_all,
                                             int lane, int kb) {
  const int rows_c = class_rows(cls), ipp = direct_items(cls);
  const int nbs = rows_c / kBlkRows;  // blocks per slot
  const int nblk = ipp * nbs;         // blocks of the packet

  // ---- g table: every block of every slot (0 past the slot's item).  A
  // wavefront takes up to four blocks per round: lane l reads row l & 15 of
  // the (l >> 4)-th block (its window and the run lengths past the window's
  // ends), so the global reads of the round overlap; then each block's rows
  // are broadcast and decoded by all lanes, four rows per 64-bit word. ----
  for (int b1 = kb; b1 < nblk; b1 += 4 * kEdtWaves) {
    uint4 r = make_uint4(0u, 0u, 0u, 0u);  // padding row: no runs
    {
      const int bl = b1 + kEdtWaves * (lane >> 4);
      if (bl < nblk) {
        const int slot = bl / nbs;
        const int word = words[slot];
        const uint32_t* rc = recs + slot * 16;
        const int n = word >= 0 ? (int)rc[8] : 0;
        const int u = (bl - slot * nbs) * kBlkRows + (lane & 15);
        if (u > 0 && u < n - 1) {
          const uint64_t* mb = reinterpret_cast<const uint64_t*>(((uint64_t)rc[1] << 32) | rc[0]);
          const int y0 = (int)rc[4], wq = (int)rc[11], fw = (int)rc[12];
          const int xs = (int)rc[14] + (word & ((1 << kItemStripBits) - 1)) * strip_width((int)rc[9]);
          const uint64_t* row = mb + (int64_t)(y0 - 1 + u) * wq;
          const uint64_t win = load_window(row, xs, wq, fw);
          // the table clamps g at 576 or below: runs past the window's ends
          // matter up to that length
          const int L = (win & 1ull) ? run_left(row, xs - 1, wq, fw, kDirRunCap) : 0;
          const int R = (win >> 63) ? run_right(row, xs + 64, wq, fw, kDirRunCap) : 0;
          r = make_rowrec(win, L, R);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int b = b1 + kEdtWaves * t;
      if (b >= nblk) break;
      const int slot = b / nbs, r0 = (b - slot * nbs) * kBlkRows;
      const DirItem it = direct_item(recs, words, slot);
      const bool lane_ok = lane < it.SW;
      uint2* gt = gt_all + ((slot * rows_c + r0) >> 2) * 64 + lane;
      const s16x2 l2 = {(short)lane, (short)lane};
#pragma unroll
      for (int k4 = 0; k4 < kBlkRows; k4 += 4) {
        if (r0 + k4 >= it.n - 1) {  // padding rows only
          gt[(k4 >> 2) * 64] = make_uint2(0u, 0u);
          continue;
        }
        uint32_t wd[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {  // rows k4 + 2q and k4 + 2q + 1
          const int src = 16 * t + k4 + 2 * q;
          const uint32_t z0 = __builtin_amdgcn_readlane(r.z, src), w0 = __builtin_amdgcn_readlane(r.w, src);
          const uint32_t z1 = __builtin_amdgcn_readlane(r.z, src + 1), w1 = __builtin_amdgcn_readlane(r.w, src + 1);
          if (((int)z0 >> 16) != kManyRuns && ((int)z1 >> 16) != kManyRuns) {
            // both rows have at most two runs: g of the two rows at once in
            // packed 16-bit arithmetic (every endpoint and difference is
            // below 2^15 in magnitude), as g_runs computes it
            const s16x2 a1 = __builtin_bit_cast(s16x2, (z0 & 0xFFFFu) | (z1 << 16));
            const s16x2 b1 = __builtin_bit_cast(s16x2, (z0 >> 16) | (z1 & 0xFFFF0000u));
            const s16x2 a2 = __builtin_bit_cast(s16x2, (w0 & 0xFFFFu) | (w1 << 16));
            const s16x2 b2 = __builtin_bit_cast(s16x2, (w0 >> 16) | (w1 & 0xFFFF0000u));
            const s16x2 zero = {0, 0};
            s16x2 g = __builtin_elementwise_max(
                __builtin_elementwise_max(__builtin_elementwise_min(l2 - a1, b1 - l2), __builtin_elementwise_min(l2 - a2, b2 - l2)),
                zero);
            if (PK == 1) {
              const s16x2 cap = {255, 255};
              const us2 gc = __builtin_bit_cast(us2, __builtin_elementwise_min(g, cap));
              wd[q] = lane_ok ? __builtin_bit_cast(uint32_t, gc * gc) : 0u;
            } else if (PK == 2) {
              const s16x2 cap = {255, 255}, top = {576, 576};
              const us2 g1 = __builtin_bit_cast(us2, __builtin_elementwise_min(g, top));
              const us2 gc = __builtin_bit_cast(us2, __builtin_elementwise_min(g, cap));
              wd[q] = lane_ok ? __builtin_bit_cast(uint32_t, gc * gc + (g1 - gc)) : 0u;
            } else {
              wd[q] = lane_ok ? __builtin_bit_cast(uint32_t, g) : 0u;
            }
          } else {
            uint32_t h[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const uint4 ru =
                  make_uint4(__builtin_amdgcn_readlane(r.x, src + e), __builtin_amdgcn_readlane(r.y, src + e),
                             __builtin_amdgcn_readlane(r.z, src + e), __builtin_amdgcn_readlane(r.w, src + e));
              h[e] = lane_ok ? (uint32_t)g_rec(ru, lane) : 0u;
              if (PK == 1) h[e] = min(h[e], 255u) * min(h[e], 255u);
              if (PK == 2) h[e] = min(h[e], 255u) * min(h[e], 255u) + (min(h[e], 576u) - min(h[e], 255u));
            }
            wd[q] = h[0] | (h[1] << 16);
          }
        }
        gt[(k4 >> 2) * 64] = make_uint2(wd[0], wd[1]);
      }
    }
  }
}

// The squared distances (AREA: 1 inside, 0 outside) of the kDirRows rows of
// one group, whose first table word is `base` (one lane per column; RS: the
// table's words per row quad).  Rows are searched together, kDirSteps
// distances per step: the candidates at distances d .. d + kDirSteps - 1 come
// from consecutive table rows on each side, and a step runs while any row of
// the group can still improve (rows that are done are updated with
// candidates that cannot win).
template <int SPATIAL, int PK, int RS>
__device__ __forceinline__ void direct_group(const uint2* base, int* best) {
  int bmax = 0;
  // g^2 of a table entry (PK 1: the entry itself, PK 2: decoded from T)
  auto gsq_of = [](int t) { return PK == 1 ? t : PK == 2 ? (t < 65025 ? t : (t - 64770) * (t - 64770)) : t * t; };
  // initial values: the rows' own entries, g^2 (exact = false with PK 2:
  // T itself, for the packed search)
  auto init_exact = [&](bool exact) {
    bmax = 0;
#pragma unroll
    for (int q = 0; q < kDirRows / 4; ++q) {
      const uint2 w = base[q * RS];
      const int g4[4] = {(int)(w.x & 0xFFFFu), (int)(w.x >> 16), (int)(w.y & 0xFFFFu), (int)(w.y >> 16)};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        best[4 * q + k] = SPATIAL != 0 ? (g4[k] > 0 ? 1 : 0) : (PK == 2 && !exact) ? g4[k] : gsq_of(g4[k]);
        bmax = max(bmax, best[4 * q + k]);
      }
    }
  };
  // exact 32-bit search.  d = 1 (mod 4): the windows start on words, up
  // at u0 - d - 3, down at u0 + d - 1 (one row early)
  auto search32 = [&]() {
    for (int d = 1; d * d < bmax; d += kDirSteps) {
      constexpr int NQ = (kDirRows + kDirSteps) / 4;  // words per window
      const uint2* pu = base - ((d + kDirSteps - 1) >> 2) * RS;
      const uint2* pd = base + ((d - 1) >> 2) * RS;
      int su[4 * NQ], sd[4 * NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const uint2 x = pu[q * RS], y = pd[q * RS];
        const int xa = (int)(x.x & 0xFFFFu), xb = (int)(x.x >> 16), xc = (int)(x.y & 0xFFFFu), xd = (int)(x.y >> 16);
        const int ya = (int)(y.x & 0xFFFFu), yb = (int)(y.x >> 16), yc = (int)(y.y & 0xFFFFu), yd = (int)(y.y >> 16);
        su[4 * q] = gsq_of(xa);
        su[4 * q + 1] = gsq_of(xb);
        su[4 * q + 2] = gsq_of(xc);
        su[4 * q + 3] = gsq_of(xd);
        sd[4 * q] = gsq_of(ya);
        sd[4 * q + 1] = gsq_of(yb);
        sd[4 * q + 2] = gsq_of(yc);
        sd[4 * q + 3] = gsq_of(yd);
      }
      bmax = 0;
#pragma unroll
      for (int k = 0; k < kDirRows; ++k) {
#pragma unroll
        for (int i = 0; i < kDirSteps; ++i)  // row u0 + k at distance d + i: up index k - i + 3, down k + i + 1
          best[k] = min(best[k], (d + i) * (d + i) + min(su[k - i + kDirSteps - 1], sd[k + i + 1]));
        bmax = max(bmax, best[k]);
      }
    }
  };
  init_exact(false);
  if (SPATIAL == 0 && PK != 0) {
    // packed: rows (0,1) and (2,3) of the group in one register each;
    // the window rows as aligned pairs (2j, 2j+1) and odd pairs
    // (2j+1, 2j+2); the table holds g^2.
    const int b0v = best[0], b1v = best[1], b2v = best[2], b3v = best[3];
    us2 B[2] = {as_us2((uint32_t)b0v | ((uint32_t)b1v << 16)), as_us2((uint32_t)b2v | ((uint32_t)b3v << 16))};
    int pmax = max(max(b0v, b1v), max(b2v, b3v));
    for (int d = 1; d * d < pmax; d += kDirSteps) {
      const uint2* pu = base - ((d + kDirSteps - 1) >> 2) * RS;
      const uint2* pd = base + ((d - 1) >> 2) * RS;
      const uint2 u0w = pu[0], u1w = pu[RS], d0w = pd[0], d1w = pd[RS];
      const uint32_t U[4] = {u0w.x, u0w.y, u1w.x, u1w.y};
      const uint32_t Dn[4] = {d0w.x, d0w.y, d1w.x, d1w.y};
      uint32_t Uo[3], Do[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        Uo[j] = __builtin_amdgcn_alignbyte(U[j + 1], U[j], 2);
        Do[j] = __builtin_amdgcn_alignbyte(Dn[j + 1], Dn[j], 2);
      }
#pragma unroll
      for (int i = 0; i < kDirSteps; ++i) {
        // (d + i)^2 is the same for every lane: scalar arithmetic, one
        // scalar operand of the packed adds
        const uint32_t dd = (uint32_t)min((d + i) * (d + i), 65535);
        const us2 D = as_us2(dd | (dd << 16));
#pragma unroll
        for (int q = 0; q < 2; ++q) {  // rows 2q, 2q + 1 at distance d + i
          const uint32_t up = (i & 1) ? U[(3 + 2 * q - i) >> 1] : Uo[(2 + 2 * q - i) >> 1];
          const uint32_t dn = (i & 1) ? Dn[(1 + 2 * q + i) >> 1] : Do[(2 * q + i) >> 1];
          B[q] = __builtin_elementwise_min(
              B[q], __builtin_elementwise_add_sat(__builtin_elementwise_min(as_us2(up), as_us2(dn)), D));
        }
      }
      pmax = max4(B[0], B[1]);
    }
    best[0] = B[0].x;
    best[1] = B[0].y;
    best[2] = B[1].x;
    best[3] = B[1].y;
    if (PK == 2 && max(max(best[0], best[1]), max(best[2], best[3])) >= 65025) {
      // some row of the group is at least 255 from the outside: exact search
      init_exact(true);
      search32();
    }
  } else if (SPATIAL == 0) {
    search32();
  }
}

template <int SPATIAL, bool WE, int PK>
__device__ __forceinline__ void direct_packet(int cls, int s, int S, const uint32_t* recs, const int* words,
                                              uint2* gt_all, float* part, int lane, int kb, int32_t* e_out,
                                              int32_t* queue, int nb, int& next) {
  const int rows_c = class_rows(cls), ipp = direct_items(cls);
  const int nbs = rows_c / kBlkRows;  // blocks per slot
  const int nblk = ipp * nbs;         // blocks of the packet

  direct_table<PK>(cls, recs, words, gt_all, lane, kb);
  __syncthreads();
  // the workgroup's next packet (no barrier waits for this atomic before the
  // packet's end)
  if (queue && threadIdx.x == 0) next = nb + atomicAdd(queue, 1);

  // ---- search: this workgroup's blocks (every S-th from s), one wavefront
  // per block in a stride, kDirRows rows at a time (direct_group); each
  // group's rows are then added in row order. ----
  for (int b = s + S * kb; b < nblk; b += S * kEdtWaves) {
    const int slot = b / nbs, lb = b - slot * nbs, b0 = lb * kBlkRows;
    const DirItem it = direct_item(recs, words, slot);
    const int n = it.n, P = it.P, y0 = it.y0;
    const int ua = max(b0, 1), ub = min(b0 + kBlkRows, n - 1);
    if (ua >= ub) continue;
    const bool lane_ok = lane < it.SW;
    const int col = it.xs + lane;
    float* bpart = part + (slot * nbs) * kEdtPartRows * 8;  // the slot's blocks
    int pr = (y0 - 1 + ua) / P;             // patch row of row u
    int pr_next = (pr + 1) * P - (y0 - 1);  // first row of the next patch row
    float acc = 0.f;
    const uint2* tb = gt_all + ((slot * rows_c + b0) >> 2) * 64 + lane;  // the block's first word
#pragma unroll
    for (int gi = 0; gi < kBlkRows; gi += kDirRows) {
      if (b0 + gi >= ub) break;
      const uint2* base = tb + (gi >> 2) * 64;  // row u0 = b0 + gi
      int best[kDirRows];
      direct_group<SPATIAL, PK, 64>(base, best);
#pragma unroll
      for (int k = 0; k < kDirRows; ++k) {
        const int u = b0 + gi + k;
        if (u < ua || u >= ub) continue;
        if (u == pr_next) {
          flush_patch_part(bpart, lane, lane_ok, P, y0, lb, pr, acc);
          acc = 0.f;
          ++pr;
          pr_next += P;
        }
        const int e = best[k];
        acc += SPATIAL == 0 ? __builtin_amdgcn_sqrtf((float)e) : (float)e;  // e >= 0 integer: no denormals
        if (WE && lane_ok && col >= it.x0 && col <= it.x1)
          e_out[(int64_t)it.gidx * it.fh * it.fw + (int64_t)(y0 - 1 + u) * it.fw + col] = e;
      }
    }
    flush_patch_part(bpart, lane, lane_ok, P, y0, lb, pr, acc);
  }
  __syncthreads();
}

// ROWS: table rows of one workgroup (512: classes 0-4, 1152: class 5)
template <int SPATIAL, bool WE, int ROWS>
__global__ __launch_bounds__(kEdtWaves * 64) __attribute__((amdgpu_waves_per_eu(ROWS > 512 ? 4 : 8))) void k_edt_direct(
    int32_t* __restrict__ counts, const int32_t* __restrict__ items, int item_cap,
    const MaskRec* __restrict__ mrec, int32_t* e_out, float* gpart) {
  __shared__ uint2 gt_all[(ROWS + 2 * kDirGuard) / 4 * 64];  // g table, 4 rows per word; zero guard rows at each end
  __shared__ float part_all[kEdtBlocks * kEdtPartRows * 8];
  __shared__ uint32_t recs[kEdtWaves * 16];
  __shared__ int words[kEdtWaves];
  __shared__ int taken;
  const int lane = threadIdx.x & 63, kb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < (ROWS + 2 * kDirGuard) / 4 * 64; i += kEdtWaves * 64) gt_all[i] = make_uint2(0u, 0u);
  int cnt[kClasses];
  const int total = direct_count(counts, item_cap, ROWS > 512, cnt);
  const int S = direct_split(ROWS > 512, total, gridDim.x);
  // Virtual packets (packet, share) in chunks of kXcds: chunk c belongs to
  // XCD c % kXcds.  The XCD's nb workgroups take its first nb packets one
  // each, then the rest in order from a queue of their own (a counter per
  // XCD: a workgroup that finishes early takes the next packet instead of
  // waiting for a fixed share of the list).  The shares of a packet and
  // neighbouring packets (the strips of one mask, in scan order) then read
  // the same mask rows through one L2, and every XCD starts with the tallest
  // packets.  Which workgroup takes a packet never changes its result.
  const int N = total * S;
  const bool by_xcd = gridDim.x >= kXcds;  // else one queue in plain order
  const int x = by_xcd ? blockIdx.x % kXcds : 0;
  const int nb = by_xcd ? (gridDim.x - x + kXcds - 1) / kXcds : gridDim.x;
  // no queue when the XCD's list ends within its first nb packets
  const bool queued = (by_xcd ? kXcds * (x + kXcds * (nb / kXcds)) + nb % kXcds : nb) < N;
  int32_t* queue = queued ? counts + kDirQueue + (ROWS > 512 ? kXcds : 0) + x : nullptr;
  int next = N;  // past every list (by_xcd: t >= N gives vp >= N)
  for (int t = by_xcd ? blockIdx.x / kXcds : blockIdx.x;;) {
    const int vp = by_xcd ? kXcds * (x + kXcds * (t / kXcds)) + t % kXcds : t;
    if (vp >= N) break;  // the XCD's list is in increasing order: nothing after it either
    const int p = vp / S, s = vp - p * S;
    const int cls = direct_load_packet(cnt, counts, items, item_cap, mrec, p, recs, words);
    float* part = S == 1 ? part_all : gpart + (int64_t)p * kDirPartFloats;
    direct_packet<SPATIAL, WE, (ROWS <= 512 ? 1 : SPATIAL == 0 ? 2 : 0)>(cls, s, S, recs, words, gt_all + kDirGuard / 4 * 64, part, lane, kb, e_out,
                                                                         queue, nb, next);
    if (S == 1) {
      direct_strip_sums(cls, recs, words, part_all, lane, kb);
      __syncthreads();
    }
    // every thread has read the previous value of taken (barriers above)
    if (threadIdx.x == 0) taken = next;
    __syncthreads();
    t = taken;
  }
}

// Patch sums of the packets that k_edt_direct shared between workgroups
// (nothing to do when it shared none); grid: one workgroup per CU.  With
// order_pool it first orders every frame's masks for the pooling (one
// workgroup per frame, in a stride); with take_mean it takes the token
// statistics' frame means (frame f on workgroup grid - 1 - f, in a stride)
// and, given pack_proj, writes the projection's k-packed BF16 copy of P.
__global__ __launch_bounds__(kEdtWaves * 64) void k_edt_dsums(Batch b, const int32_t* __restrict__ counts,
                                                              const int32_t* __restrict__ items, int item_cap,
                                                              const MaskRec* __restrict__ mrec, const float* gpart,
                                                              int direct_grid, Work wk, int order_pool,
                                                              int take_mean, const void* pack_proj, int proj_bf16) {
  __shared__ uint32_t recs[kEdtWaves * 16];
  __shared__ int words[kEdtWaves];
  if (take_mean)
    for (int f = (int)gridDim.x - 1 - (int)blockIdx.x; f < b.dyn[0]; f += gridDim.x)
      for (int c = threadIdx.x; c < b.C; c += blockDim.x) frame_mean_channel(b, wk, f, c);
  if (pack_proj) {
    const int64_t np = (int64_t)(b.C / 8) * b.E, step = (int64_t)gridDim.x * blockDim.x;
    uint4* pp = reinterpret_cast<uint4*>(wk.ppack);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < np; t += step) {
      if (proj_bf16) pack_proj_chunk<1>(pack_proj, b.C, b.E, pp, t);
      else pack_proj_chunk<0>(pack_proj, b.C, b.E, pp, t);
    }
  }
  if (order_pool) {
    __shared__ int ocnt[256];
    __shared__ int owsum[4];
    for (int f = blockIdx.x; f < b.dyn[0]; f += gridDim.x) pool_order_frame(b, wk, f, ocnt, owsum);
  }
  const int lane = threadIdx.x & 63, kb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int cnt[kClasses];
  const int total = direct_count(counts, item_cap, false, cnt);
  if (direct_split(false, total, direct_grid) == 1) return;
  for (int p = blockIdx.x; p < total; p += gridDim.x) {
    const int cls = direct_load_packet(cnt, counts, items, item_cap, mrec, p, recs, words);
    direct_strip_sums(cls, recs, words, gpart + (int64_t)p * kDirPartFloats, lane, kb);
    __syncthreads();
  }
}

// Resident workgroups per CU of each kernel variant, computed once (outside
// any stream capture): envelope EDT and AREA (layouts 0 and 1), then the
// direct search for (EDT, EDT writing e, AREA) x (classes 0-4, class 5).
static std::once_flag g_edt_once;
static int g_edt_per_cu[8];

static const void* edt_variant(int v) {
  switch (v) {
    case 0: return reinterpret_cast<const void*>(&k_edt<0, false>);
    case 1: return reinterpret_cast<const void*>(&k_edt<1, false>);
    case 2: return reinterpret_cast<const void*>(&k_edt_direct<0, false, 512>);
    case 3: return reinterpret_cast<const void*>(&k_edt_direct<0, true, 512>);
    case 4: return reinterpret_cast<const void*>(&k_edt_direct<1, false, 512>);
    case 5: return reinterpret_cast<const void*>(&k_edt_direct<0, false, kMaxRows>);
    case 6: return reinterpret_cast<const void*>(&k_edt_direct<0, true, kMaxRows>);
    default: return reinterpret_cast<const void*>(&k_edt_direct<1, false, kMaxRows>);
  }
}

void edt_prepare() {
  std::call_once(g_edt_once, [] {
    for (int v = 0; v < 8; ++v) {
      int per_cu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edt_variant(v), kEdtWaves * 64, 0) != hipSuccess ||
          per_cu < 1)
        per_cu = 1;
      g_edt_per_cu[v] = per_cu;
    }
  });
}

// Layout -1 (default) and 2 run the direct search; 0 and 1 the envelope
// kernel in that band layout.  e_out (squared distances of the bounding
// boxes) is written by the direct search only (callers that pass it use the
// default layout); the AREA variants never produce distances.
void launch_edt(const Batch& b, const Work& w, int32_t* e_out, int num_cus, hipStream_t st, int mode,
                bool order_pool, bool take_mean, const void* pack_proj, int proj_bf16) {
  edt_prepare();
  const dim3 blk(kEdtWaves * 64);
  if (mode == 0 || mode == 1) {
    if (order_pool) launch_pool_order(b, w, st);
    const int v = b.spatial != 0 ? 1 : 0;
    const dim3 grid(num_cus * g_edt_per_cu[v]);
    if (v == 0)
      hipLaunchKernelGGL((k_edt<0, false>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, nullptr, mode);
    else
      hipLaunchKernelGGL((k_edt<1, false>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, nullptr, mode);
    return;
  }
  const int kind = b.spatial != 0 ? 2 : (e_out ? 1 : 0);
  auto go = [&](int dv) {
    const dim3 grid(num_cus * g_edt_per_cu[dv]);
    float* gp = w.edt_part;
    switch (dv) {
      case 2: hipLaunchKernelGGL((k_edt_direct<0, false, 512>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, e_out, gp); break;
      case 3: hipLaunchKernelGGL((k_edt_direct<0, true, 512>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, e_out, gp); break;
      case 4: hipLaunchKernelGGL((k_edt_direct<1, false, 512>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, e_out, gp); break;
      case 5: hipLaunchKernelGGL((k_edt_direct<0, false, kMaxRows>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, e_out, gp); break;
      case 6: hipLaunchKernelGGL((k_edt_direct<0, true, kMaxRows>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, e_out, gp); break;
      default: hipLaunchKernelGGL((k_edt_direct<1, false, kMaxRows>), grid, blk, 0, st, w.counts, w.items, b.item_cap, w.mrec, e_out, gp); break;
    }
    return (int)grid.x;
  };
  // items taller than 512 rows (class 5) first, when the batch can have any;
  // then the rest, whose packets may be shared (their patch sums follow)
  if (b.max_rows > 512) go(5 + kind);
  const int g = go(2 + kind);
  const int op = order_pool && b.n_frames > 0 && b.M > 0 ? 1 : 0;
  hipLaunchKernelGGL(k_edt_dsums, dim3(num_cus), blk, 0, st, b, w.counts, w.items, b.item_cap, w.mrec, w.edt_part, g, w,
                     op, take_mean && b.n_frames > 0 ? 1 : 0, take_mean ? pack_proj : nullptr, proj_bf16);
}

}  // namespace disc
