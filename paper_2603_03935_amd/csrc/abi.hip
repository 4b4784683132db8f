// C ABI of libdisc: argument validation, workspaces and the kernel sequence
// of DISC's single-pass feature extraction (arXiv 2603.03935, Sec. III-C).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cstring>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/disc.h"
#include "disc_device.h"
#include "host.h"

using namespace disc;

namespace disc {
namespace host {

thread_local std::string g_err;

disc_status fail(disc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

disc_status ok() {
  g_err.clear();
  return DISC_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// A strip is at least 33 columns wide for every patch size in [8, 64]
// (SW = 64 - 64 % P), so 256 strips, the most an item word encodes, cover
// 256 * 33 columns.
constexpr int kMaxWidth = 256 * 33;

// --------------------------------------------------------------------------
// validation
// --------------------------------------------------------------------------
disc_status check_tokens(const disc_tokens* t, const char* who) {
  if (!t) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: tokens is NULL", who);
  if (!t->data) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: tokens->data is NULL", who);
  if (t->dtype < DISC_F32 || t->dtype > DISC_F8E4M3)
    return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: unknown token dtype %d", who, t->dtype);
  if (t->gh <= 0 || t->gw <= 0 || t->c <= 0)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: token grid %dx%dx%d must be positive", who, t->gh, t->gw, t->c);
  if (t->patch < kMinPatch || t->patch > kMaxPatch)
    return fail(DISC_ERR_LIMIT, "%s: patch %d outside [%d, %d]", who, t->patch, kMinPatch, kMaxPatch);
  if (t->c % 64 != 0 || t->c > kMaxC)
    return fail(DISC_ERR_LIMIT, "%s: channels %d must be a multiple of 64 up to %d", who, t->c, kMaxC);
  if ((t->dtype == DISC_F8E4M3) != (t->scale != nullptr))
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: per-token scales are required for FP8 tokens and only for them", who);
  if (!aligned16(t->data) || (t->scale && !aligned16(t->scale)))
    return fail(DISC_ERR_ALIGNMENT, "%s: token pointers must be 16-byte aligned", who);
  return DISC_OK;
}

disc_status check_masks(const disc_masks* m, const char* who) {
  if (!m) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: masks is NULL", who);
  if (m->m < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative mask count", who);
  if (m->h <= 0 || m->w <= 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: frame %dx%d must be positive", who, m->h, m->w);
  if (m->m > 0 && !m->bits) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: masks->bits is NULL", who);
  if (m->h > kMaxRows - 2) return fail(DISC_ERR_LIMIT, "%s: frame height %d exceeds %d", who, m->h, kMaxRows - 2);
  if (m->w > kMaxWidth) return fail(DISC_ERR_LIMIT, "%s: frame width %d exceeds %d", who, m->w, kMaxWidth);
  if (m->bits && !aligned16(m->bits)) return fail(DISC_ERR_ALIGNMENT, "%s: mask bits must be 16-byte aligned", who);
  if ((int64_t)m->m * m->h * ((m->w + 63) / 64) > (int64_t)1 << 40)
    return fail(DISC_ERR_LIMIT, "%s: mask batch too large", who);
  return DISC_OK;
}

disc_status check_grid(const disc_tokens* t, const disc_masks* m, const char* who) {
  const int gh = (m->h + t->patch - 1) / t->patch, gw = (m->w + t->patch - 1) / t->patch;
  if (t->gh != gh || t->gw != gw)
    return fail(DISC_ERR_SHAPE, "%s: token grid %dx%d does not cover a %dx%d frame with %d-px patches (expected %dx%d)",
                who, t->gh, t->gw, m->h, m->w, t->patch, gh, gw);
  return DISC_OK;
}

disc_status check_proj(const disc_proj* p, int c, const char* who) {
  if (!p) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: proj is NULL", who);
  if (!p->data) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: proj->data is NULL", who);
  if (p->dtype != DISC_F32 && p->dtype != DISC_BF16)
    return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: projection dtype must be F32 or BF16", who);
  if (p->c != c) return fail(DISC_ERR_SHAPE, "%s: proj has %d input channels, tokens have %d", who, p->c, c);
  if (p->e <= 0 || p->e % 128 != 0 || p->e > 1024)
    return fail(DISC_ERR_LIMIT, "%s: embedding width %d must be a multiple of 128 up to 1024", who, p->e);
  if (!aligned16(p->data)) return fail(DISC_ERR_ALIGNMENT, "%s: proj must be 16-byte aligned", who);
  return DISC_OK;
}

disc_status check_out(const disc_out* o, int m, int e, const char* who) {
  if (!o) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: out is NULL", who);
  if (m > 0 && !o->data) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: out->data is NULL", who);
  if (o->m != m) return fail(DISC_ERR_SHAPE, "%s: out has %d rows for %d masks", who, o->m, m);
  if (o->e != e) return fail(DISC_ERR_SHAPE, "%s: out has width %d, projection %d", who, o->e, e);
  if ((o->data && !aligned16(o->data)) || (o->pooled && !aligned16(o->pooled)) ||
      (o->mask_status && (reinterpret_cast<uintptr_t>(o->mask_status) & 3u)) ||
      (o->dbar && (reinterpret_cast<uintptr_t>(o->dbar) & 3u)) || (o->area && (reinterpret_cast<uintptr_t>(o->area) & 3u)))
    return fail(DISC_ERR_ALIGNMENT, "%s: output pointers must be 16-byte aligned (status, dbar, area: 4)", who);
  return DISC_OK;
}

disc_status check_opts(const disc_options* o, const char* who) {
  if (!o) return DISC_OK;
  if (o->spatial != DISC_SPATIAL_EDT && o->spatial != DISC_SPATIAL_AREA)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: spatial mode %d", who, o->spatial);
  if (o->distinct != 0 && o->distinct != 1) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: distinct must be 0 or 1", who);
  if (!(o->eps >= 0.f)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: eps must be >= 0", who);
  if (o->gemm_dtype != -1 && o->gemm_dtype != DISC_F32 && o->gemm_dtype != DISC_BF16)
    return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: gemm dtype must be F32, BF16 or -1", who);
  if (o->workspace && !aligned16(o->workspace)) return fail(DISC_ERR_ALIGNMENT, "%s: workspace must be 16-byte aligned", who);
  if (o->edt_layout < -1 || o->edt_layout > 2)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: edt_layout must be -1, 0, 1 or 2", who);
  if (o->pool_tile != -1 && o->pool_tile != 1 && o->pool_tile != 2 && o->pool_tile != 4)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: pool_tile must be -1, 1, 2 or 4", who);
  if (o->pool_rows != -1 && o->pool_rows != 64 && o->pool_rows != 128)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: pool_rows must be -1, 64 or 128", who);
  return DISC_OK;
}

disc_status hip_fail(hipError_t e, const char* what) {
  return fail(DISC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// --------------------------------------------------------------------------
// workspace layout
// --------------------------------------------------------------------------


Layout make_layout(const Shape& s) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (size_t)round_up((int64_t)std::max<size_t>(bytes, 1), 256);
    return at;
  };
  L.frames = take(sizeof(FrameDesc) * s.n_frames);
  L.mask_frame = take(4 * (size_t)s.M);
  L.tiles = take(16 * (size_t)s.n_tiles);
  L.dyn = take(16);
  L.counts = take(4 * (kCounters + (size_t)s.n_frames));  // work-list and queue counters, then the per-frame scale flags
  L.staged_end = off;
  L.bbox = take(16 * (size_t)s.M);
  L.area = take(4 * (size_t)s.M);
  L.meta = take(4 * (size_t)s.M);
  L.mrec = take(sizeof(MaskRec) * (size_t)s.M);
  L.items = take(4 * (size_t)kClasses * kLists * s.item_cap);
  L.psum = take(4 * (size_t)s.n_frames * s.nchunk * s.C);
  L.mean = take(4 * (size_t)s.n_frames * s.C);
  L.r = take(4 * (size_t)s.sumG);
  L.rbar = take(4 * (size_t)s.n_frames);
  L.s = take(4 * (size_t)s.sumMGs);
  L.W = take((s.gemm_bf16 ? 2 : 4) * (size_t)s.sumMGs);
  L.Z = take(4 * (size_t)s.M);
  L.mstat = take(4 * (size_t)s.M);
  L.perm = take(4 * (size_t)s.M);
  L.X = take((s.gemm_bf16 ? 2 : 4) * (size_t)s.M * s.C);
  L.ppart = take(s.pool_split > 1 ? 4 * (size_t)s.n_tiles * s.kgroups * 64 * 64 : 0);
  L.ptile = take(s.pool_split > 1 ? 16 * (size_t)s.n_tiles * 65 : 0);
  L.qpart = take(s.proj_split > 1 ? 4 * (size_t)((s.C + kProjKG - 1) / kProjKG) * s.M * s.E : 0);
  L.ppack = take(s.gemm_bf16 ? 2 * (size_t)s.C * s.E : 0);
  L.edt_part = take(4 * (size_t)kDirSplitPackets * kDirPartFloats);
  L.extra = take((size_t)s.extra_bytes);
  L.total = off;
  return L;
}

// --------------------------------------------------------------------------
// per (device, stream) workspace cache with a pinned staging buffer
// --------------------------------------------------------------------------
struct WsEntry {
  void* dev = nullptr;
  size_t dev_bytes = 0;
  void* host = nullptr;
  size_t host_bytes = 0;
  hipEvent_t ev = nullptr;
  bool ev_pending = false;
};

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, WsEntry> g_ws;
std::map<int, int> g_cus;

int num_cus(int dev) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_cus.find(dev);
  if (it != g_cus.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
  g_cus[dev] = n;
  return n;
}

struct Ctx {
  int dev = 0;
  hipStream_t st = nullptr;
  char* dev_ws = nullptr;
  char* host_stage = nullptr;
  WsEntry* entry = nullptr;
};

disc_status acquire(hipStream_t st, const Layout& L, const disc_options* opts, Ctx& cx) {
  // The staged descriptors go through a host buffer that the next call on
  // this stream reuses, and a new shape may time the pooling candidates or
  // grow the workspace: none of that may be recorded into a graph.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(DISC_ERR_INVALID_ARGUMENT,
                "the stream is being captured: this entry point stages through a reused host buffer; "
                "capture disc_embed_masks_noalloc instead");
  hipError_t e = hipGetDevice(&cx.dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  cx.st = st;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  WsEntry& w = g_ws[{cx.dev, st}];
  cx.entry = &w;
  if (!w.ev) {
    if ((e = hipEventCreateWithFlags(&w.ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  }
  if (w.ev_pending) {  // the previous call's upload must have consumed the staging buffer
    if ((e = hipEventSynchronize(w.ev)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    w.ev_pending = false;
  }
  if (w.host_bytes < L.staged_end) {
    if (w.host) (void)hipHostFree(w.host);
    w.host = nullptr;
    w.host_bytes = 0;
    const size_t want = (size_t)round_up((int64_t)(L.staged_end * 5 / 4) + 4096, 4096);
    if ((e = hipHostMalloc(&w.host, want, hipHostMallocDefault)) != hipSuccess)
      return fail(DISC_ERR_OUT_OF_MEMORY, "pinned staging of %zu bytes: %s", want, hipGetErrorString(e));
    w.host_bytes = want;
  }
  cx.host_stage = static_cast<char*>(w.host);
  if (opts && opts->workspace) {
    if (opts->workspace_bytes < L.total)
      return fail(DISC_ERR_OUT_OF_MEMORY, "workspace of %zu bytes is smaller than the %zu required", opts->workspace_bytes, L.total);
    cx.dev_ws = static_cast<char*>(opts->workspace);
    return DISC_OK;
  }
  if (w.dev_bytes < L.total) {
    if (w.dev) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(w.dev);
    }
    w.dev = nullptr;
    w.dev_bytes = 0;
    const size_t want = (size_t)round_up((int64_t)(L.total * 5 / 4) + (1 << 20), 1 << 20);
    if ((e = hipMalloc(&w.dev, want)) != hipSuccess)
      return fail(DISC_ERR_OUT_OF_MEMORY, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
    w.dev_bytes = want;
  }
  cx.dev_ws = static_cast<char*>(w.dev);
  return DISC_OK;
}

disc_status upload(Ctx& cx, const Layout& L) {
  hipError_t e = hipMemcpyAsync(cx.dev_ws, cx.host_stage, L.staged_end, hipMemcpyHostToDevice, cx.st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if ((e = hipEventRecord(cx.entry->ev, cx.st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  cx.entry->ev_pending = true;
  return DISC_OK;
}

Work work_ptrs(char* base, const Layout& L) {
  Work w;
  w.bbox = reinterpret_cast<int4*>(base + L.bbox);
  w.area = reinterpret_cast<int32_t*>(base + L.area);
  w.meta = reinterpret_cast<int32_t*>(base + L.meta);
  w.mrec = reinterpret_cast<MaskRec*>(base + L.mrec);
  w.items = reinterpret_cast<int32_t*>(base + L.items);
  w.counts = reinterpret_cast<int32_t*>(base + L.counts);
  w.fbad = w.counts + kCounters;
  w.psum = reinterpret_cast<float*>(base + L.psum);
  w.mean = reinterpret_cast<float*>(base + L.mean);
  w.r = reinterpret_cast<float*>(base + L.r);
  w.rbar = reinterpret_cast<float*>(base + L.rbar);
  w.s = reinterpret_cast<float*>(base + L.s);
  w.W = base + L.W;
  w.Z = reinterpret_cast<float*>(base + L.Z);
  w.mstat = reinterpret_cast<int32_t*>(base + L.mstat);
  w.perm = reinterpret_cast<int32_t*>(base + L.perm);
  w.X = base + L.X;
  w.ppart = reinterpret_cast<float*>(base + L.ppart);
  w.ptile = reinterpret_cast<int4*>(base + L.ptile);
  w.qpart = reinterpret_cast<float*>(base + L.qpart);
  w.ppack = base + L.ppack;
  w.edt_part = reinterpret_cast<float*>(base + L.edt_part);
  return w;
}

// --------------------------------------------------------------------------
// batch description
// --------------------------------------------------------------------------


// One frame's descriptor, appended to the capacity totals of a plan.
FrameDesc plan_frame(const FrameIn& f, int C, Shape& s, PlanAcc& a) {
  FrameDesc d{};
  d.tokens = f.tokens;
  d.scale = f.scale;
  d.bits = f.bits;
  d.out = f.out;
  d.status = f.status;
  d.pooled = f.pooled;
  d.dbar = f.dbar;
  d.area_out = f.area;
  if (f.dbar) s.want_dbar = true;
  s.max_rows = std::max(s.max_rows, std::min(f.h + 2, kMaxRows));
  d.gh = f.gh;
  d.gw = f.gw;
  d.patch = f.patch;
  d.G = f.gh * f.gw;
  d.h = f.h;
  d.w = f.w;
  d.wq = (f.w + 63) / 64;
  d.m = f.m;
  d.mask_base = (int32_t)a.M;
  d.Gs = (int32_t)round_up(d.G, 8);
  d.w_base = a.sumMGs;
  d.r_base = a.sumG;
  a.M += f.m;
  a.sumG += d.G;
  a.sumMGs += (int64_t)f.m * d.Gs;
  a.gmax = std::max(a.gmax, d.G);
  a.nchunk = std::max(a.nchunk, stat_nchunk(d.G));
  {
    // the frame's masks are g = mask_base .. mask_base + m - 1; mask g
    // appends at most `strips` items to sub-list g % kLists of its class
    const int64_t strips = (f.w + strip_width(f.patch) - 1) / strip_width(f.patch) + 1;
    const int64_t g0 = d.mask_base, g1 = g0 + f.m;
    for (int j = 0; j < kLists; ++j) {
      const int64_t first = g0 + ((j - g0 % kLists) + kLists) % kLists;  // first g >= g0 with g % kLists == j
      const int64_t n = first < g1 ? (g1 - 1 - first) / kLists + 1 : 0;
      a.item_sub[j] += n * strips;
    }
  }
  a.n_tiles += (f.m + 63) / 64 * (C / 64);
  return d;
}

// Shape totals and the workspace layout once every frame is in.
void finish_plan(Plan& p, const PlanAcc& a) {
  Shape& s = p.shape;
  s.M = a.M;
  s.sumG = a.sumG;
  s.sumMGs = a.sumMGs;
  s.gmax = a.gmax;
  s.nchunk = a.nchunk;
  int64_t cap = 1;
  for (int j = 0; j < kLists; ++j) cap = std::max(cap, a.item_sub[j]);
  s.item_cap = (int)std::min<int64_t>(cap, INT32_MAX / 2 / kLists);
  s.n_tiles = a.n_tiles;
  choose_splits(s);
  p.L = make_layout(s);
}

void begin_plan(Plan& p, int n_frames, int C, int E, int gemm_bf16, int tok_dtype) {
  Shape& s = p.shape;
  s.n_frames = n_frames;
  s.want_dbar = false;
  s.max_rows = 0;
  s.C = C;
  s.E = E;
  s.gemm_bf16 = gemm_bf16;
}

void build_plan(const std::vector<FrameIn>& fr, int C, int E, int gemm_bf16, Plan& p, int tok_dtype) {
  begin_plan(p, (int)fr.size(), C, E, gemm_bf16, tok_dtype);
  PlanAcc a;
  p.fds.resize(fr.size());
  for (size_t i = 0; i < fr.size(); ++i) {
    const FrameIn& f = fr[i];
    p.fds[i] = plan_frame(f, C, p.shape, a);
    for (int j = 0; j < f.m; ++j) p.mask_frame.push_back((int32_t)i);
    for (int m0 = 0; m0 < f.m; m0 += 64)
      for (int n0 = 0; n0 < C; n0 += 64) p.tiles.push_back(make_int4((int)i, m0, n0, pool_pair_flag(m0, f.m)));
  }
  finish_plan(p, a);
}

void choose_splits(Shape& s) {
  s.kgroups = std::max(1, (s.gmax + kPoolKG - 1) / kPoolKG);
  const int pool_tiles = std::max(1, s.n_tiles);
  s.pool_split = pool_tiles >= kTargetWGs ? 1 : std::min(s.kgroups, (kTargetWGs + pool_tiles - 1) / pool_tiles);
  const int qgroups = std::max(1, (s.C + kProjKG - 1) / kProjKG);
  // BF16 tiles (64 x 64) run a whole K in a few microseconds, so they split K
  // only when too few to spread over the chip: the group sums cost 8 bytes
  // per group, row and column of extra traffic.
  const int rows = s.gemm_bf16 ? 64 : 32, cols = s.gemm_bf16 ? 64 : 128;
  const int64_t proj_tiles = std::max<int64_t>(1, (s.M + rows - 1) / rows * (s.E / cols));
  const int64_t enough = s.gemm_bf16 ? kTargetWGs / 2 : kTargetWGs;
  s.proj_split = proj_tiles >= enough ? 1 : (int)std::min<int64_t>(qgroups, (kTargetWGs + proj_tiles - 1) / proj_tiles);
}

void stage_host(const Plan& p, char* host, char* dev) {
  std::vector<FrameDesc> fds = p.fds;
  (void)dev;
  std::memcpy(host + p.L.frames, fds.data(), sizeof(FrameDesc) * fds.size());
  if (!p.mask_frame.empty()) std::memcpy(host + p.L.mask_frame, p.mask_frame.data(), 4 * p.mask_frame.size());
  if (!p.tiles.empty()) std::memcpy(host + p.L.tiles, p.tiles.data(), 16 * p.tiles.size());
  const int32_t dyn[4] = {p.shape.n_frames, (int32_t)p.shape.M, p.shape.n_tiles, 0};
  std::memcpy(host + p.L.dyn, dyn, sizeof dyn);
  std::memset(host + p.L.counts, 0, 4 * (kCounters + (size_t)p.shape.n_frames));
}

Batch make_batch(const Plan& p, char* dev, int tok_dtype, int spatial, int distinct) {
  Batch b{};
  b.frames = reinterpret_cast<const FrameDesc*>(dev + p.L.frames);
  b.mask_frame = reinterpret_cast<const int32_t*>(dev + p.L.mask_frame);
  b.dyn = reinterpret_cast<const int32_t*>(dev + p.L.dyn);
  b.n_frames = p.shape.n_frames;
  b.M = (int32_t)p.shape.M;
  b.C = p.shape.C;
  b.E = p.shape.E;
  b.tok_dtype = tok_dtype;
  b.gemm_bf16 = p.shape.gemm_bf16;
  b.spatial = spatial;
  b.distinct = distinct;
  b.nchunk = p.shape.nchunk;
  b.item_cap = p.shape.item_cap;
  b.n_tiles = p.shape.n_tiles;
  b.kgroups = p.shape.kgroups;
  b.pool_split = p.shape.pool_split;
  b.proj_split = p.shape.proj_split;
  b.max_rows = p.shape.max_rows > 0 ? p.shape.max_rows : kMaxRows;
  return b;
}

disc_status check_launch(const char* who) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DISC_ERR_DEVICE, "%s: kernel launch failed: %s", who, hipGetErrorString(e));
  return DISC_OK;
}

int resolve_gemm(const disc_options* o, int tok_dtype, int proj_dtype) {
  const int g = o ? o->gemm_dtype : -1;
  if (g == DISC_F32) return 0;
  if (g == DISC_BF16) return 1;
  return (tok_dtype == DISC_F32 && proj_dtype == DISC_F32) ? 0 : 1;
}

disc_options defaults() {
  disc_options o;
  disc_options_default(&o);
  return o;
}

FrameIn frame_in(const disc_tokens& t, const disc_masks& m, const disc_out& o) {
  FrameIn f;
  f.tokens = t.data;
  f.scale = t.scale;
  f.bits = m.bits;
  f.out = o.data;
  f.status = o.mask_status;
  f.pooled = o.pooled;
  f.dbar = o.dbar;
  f.area = o.area;
  f.gh = t.gh;
  f.gw = t.gw;
  f.patch = t.patch;
  f.h = m.h;
  f.w = m.w;
  f.m = m.m;
  return f;
}

// Validate a ragged batch and describe it.
disc_status describe(const disc_tokens* tokens, const disc_masks* masks, int32_t n, const disc_proj* proj, disc_out* out,
                     const disc_options* opts, const char* who, std::vector<FrameIn>& fr) {
  if (n < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative frame count", who);
  if (n > 0 && (!tokens || !masks || !out)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL frame arrays", who);
  disc_status st;
  if ((st = check_opts(opts, who))) return st;
  for (int i = 0; i < n; ++i) {
    if ((st = check_tokens(&tokens[i], who))) return st;
    if ((st = check_masks(&masks[i], who))) return st;
    if ((st = check_grid(&tokens[i], &masks[i], who))) return st;
    if (tokens[i].c != tokens[0].c) return fail(DISC_ERR_SHAPE, "%s: frames differ in channel count", who);
    if (tokens[i].dtype != tokens[0].dtype) return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: frames differ in token dtype", who);
  }
  if (n > 0) {
    if ((st = check_proj(proj, tokens[0].c, who))) return st;
    for (int i = 0; i < n; ++i)
      if ((st = check_out(&out[i], masks[i].m, proj->e, who))) return st;
  }
  fr.resize(n);
  for (int i = 0; i < n; ++i) fr[i] = frame_in(tokens[i], masks[i], out[i]);
  return DISC_OK;
}

// Validate one frame (the checks describe() applies) without building vectors.
disc_status describe_one(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj, disc_out* out,
                         const disc_options* opts, const char* who, FrameIn& f) {
  if (!tokens || !masks || !out) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL frame arguments", who);
  disc_status st;
  if ((st = check_opts(opts, who))) return st;
  if ((st = check_tokens(tokens, who))) return st;
  if ((st = check_masks(masks, who))) return st;
  if ((st = check_grid(tokens, masks, who))) return st;
  if ((st = check_proj(proj, tokens->c, who))) return st;
  if ((st = check_out(out, masks->m, proj->e, who))) return st;
  f = frame_in(*tokens, *masks, *out);
  return DISC_OK;
}


// --------------------------------------------------------------------------
// per-stage tracing: events around each stage on the caller's stream
// --------------------------------------------------------------------------
enum Stage { ST_SCAN = 0, ST_STATS, ST_EDT, ST_WEIGHTS, ST_POOL, ST_PROJ, ST_COUNT };
const char* kStageNames[ST_COUNT] = {"scan", "token_stats", "edt", "weights", "pool", "proj"};

struct TraceRec {
  int stage;
  hipEvent_t a, b;
};
std::mutex g_tr_mu;
bool g_trace_on = false;
uint32_t g_trace_mask = 0xFFFFFFFFu;
std::vector<TraceRec> g_tr_pending;
std::vector<hipEvent_t> g_tr_free;
double g_tr_ms[ST_COUNT] = {};
int64_t g_tr_n[ST_COUNT] = {};

hipEvent_t tr_event() {
  if (!g_tr_free.empty()) {
    hipEvent_t e = g_tr_free.back();
    g_tr_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct StageTimer {
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(int s, hipStream_t stream) : stage(s), st(stream) {
    if (s < 0) return;
    std::lock_guard<std::mutex> lk(g_tr_mu);
    if (!g_trace_on || !((g_trace_mask >> s) & 1u)) return;
    a = tr_event();
    (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_tr_mu);
    hipEvent_t b = tr_event();
    (void)hipEventRecord(b, st);
    g_tr_pending.push_back({stage, a, b});
  }
};

void tr_collect() {
  std::lock_guard<std::mutex> lk(g_tr_mu);
  for (auto& r : g_tr_pending) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_tr_ms[r.stage] += ms;
      g_tr_n[r.stage] += 1;
    }
    g_tr_free.push_back(r.a);
    g_tr_free.push_back(r.b);
  }
  g_tr_pending.clear();
}

// --------------------------------------------------------------------------
// Pooling autotuner.  The pooling GEMM can give each workgroup 1, 2 or 4
// adjacent 64-channel tiles (wider tiles fetch each weight row once for more
// channels but hold more accumulators, so fewer workgroups fit per CU).  The
// first call with a new problem signature, outside graph capture, runs every
// valid width on its own data (each run writes the same bits), times the
// second of two runs of each with HIP events, and keeps the fastest; later
// calls (and captured graphs) use the stored choice, or a size rule before
// one exists.
// --------------------------------------------------------------------------
namespace {
struct PoolKey {
  int C, bf16, tok, n_tiles, split, kgroups;
  bool operator<(const PoolKey& o) const {
    return std::tie(C, bf16, tok, n_tiles, split, kgroups) < std::tie(o.C, o.bf16, o.tok, o.n_tiles, o.split, o.kgroups);
  }
};
std::mutex g_tune_mu;
std::map<PoolKey, int> g_tune;

// launch the pooling GEMM for a choice nt | (unsplit << 4) | ((mw - 1) << 5)
void launch_pool_choice(const Batch& b, const Work& w, const int4* tiles, hipStream_t st, int choice) {
  const int nt = choice & 15, mw = 1 + ((choice >> 5) & 1);
  if ((choice >> 4) & 1) {
    Batch b1 = b;
    b1.pool_split = 1;
    launch_pool(b1, w, tiles, st, nt, mw);
  } else {
    launch_pool(b, w, tiles, st, nt, mw);
  }
}

int pool_nt_rule(const Shape& s) {
  for (int nt : {4, 2})
    if (pool_nt_valid(s.C, nt) && s.n_tiles / nt * s.pool_split >= 4 * kTargetWGs) return nt;
  return 1;
}
}  // namespace

// The pooling launch of a problem shape: channels per workgroup (NT x 64),
// masks per workgroup (64 or 128) and whether K is split over several
// workgroups.  Every choice gives the same bits (each mask row sees the same
// K steps, and fixed K groups are added in group order), so the first call of
// a shape times each candidate twice and keeps the fastest; captured graphs
// and untuned calls use a rule.  Returned as nt | (unsplit << 4) | ((mw - 1)
// << 5).
int pool_tile_choice(const Plan& p, int tok_dtype, const disc_options& o, bool tune, const Batch& b, const Work& w,
                     const int4* tiles, hipStream_t st, bool* ran) {
  *ran = false;
  if (o.pool_tile > 0 || o.pool_rows > 0) {
    const int nt = o.pool_tile > 0 && pool_nt_valid(p.shape.C, o.pool_tile) ? o.pool_tile : 1;
    return o.pool_rows == 128 ? std::min(nt, 2) | (1 << 5) : nt;
  }
  const Shape& s = p.shape;
  const PoolKey key{s.C, s.gemm_bf16, tok_dtype, s.n_tiles, s.pool_split, s.kgroups};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  if (!tune) return pool_nt_rule(s);
  std::vector<int> cand;
  for (int uns = 0; uns < (s.pool_split > 1 ? 2 : 1); ++uns)
    for (int nt : {1, 2, 4})
      if (pool_nt_valid(s.C, nt)) cand.push_back(nt | (uns << 4));
  for (int nt : {1, 2})  // 128-mask workgroups, K never split
    if (pool_nt_valid(s.C, nt) && s.M > 64) cand.push_back(nt | (1 << 5));
  std::vector<hipEvent_t> ev(4 * cand.size());
  for (auto& e : ev) (void)hipEventCreate(&e);
  for (size_t i = 0; i < cand.size(); ++i)
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(ev[4 * i + 2 * rep], st);
      launch_pool_choice(b, w, tiles, st, cand[i]);
      (void)hipEventRecord(ev[4 * i + 2 * rep + 1], st);
    }
  (void)hipEventSynchronize(ev.back());
  int best = cand[0];
  float best_ms = 1e30f;
  bool timed = true;  // keep a choice only when every candidate was timed
  for (size_t i = 0; i < cand.size(); ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[4 * i + 2], ev[4 * i + 3]) != hipSuccess) {
      timed = false;
      continue;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = cand[i];
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (timed) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  *ran = true;  // X already holds the pooled result (every run writes the same bits)
  return best;
}

void enqueue_path(const Plan& p, char* dev_ws, int tok_dtype, const disc_options& o, const disc_proj* proj, int cus,
                  hipStream_t st, bool trace, bool tune) {
  const int sid = trace ? 0 : -1;
  Batch b = make_batch(p, dev_ws, tok_dtype, o.spatial, o.distinct);
  b.eps = o.eps;
  const Work w = work_ptrs(dev_ws, p.L);
  const int4* tiles = reinterpret_cast<const int4*>(dev_ws + p.L.tiles);
  // token statistics first: the mask scan folds r into the mean
  // distinctiveness.  Without that, the scan's launch also takes the
  // statistics' channel sums, the last launch of the distance transform
  // (direct search) the frame means and the BF16 packing of P, and the rest
  // of the statistics follow the distance transform (launches fewer; the
  // stage trace then counts those parts under the scan and the distance
  // transform).
  const bool want_r = o.distinct || p.shape.want_dbar;
  const bool stats = want_r || tok_dtype == DISC_F8E4M3;
  const bool fused = want_r && scan_takes_colsum(b, p.shape.want_dbar);
  const bool mean_in_edt = fused && o.edt_layout != 0 && o.edt_layout != 1;
  // with BF16 GEMMs the launch that takes the frame means also packs P for
  // the projection
  const bool packed = want_r && b.gemm_bf16;
  auto run_stats = [&](bool colsum_done) {
    StageTimer t(sid < 0 ? -1 : ST_STATS, st);
    if (tok_dtype == DISC_F8E4M3) launch_scale_check(b, w, p.shape.gmax, st);
    if (want_r)
      launch_token_stats(b, w, p.shape.gmax, st, colsum_done, packed && !mean_in_edt ? proj->data : nullptr,
                         proj->dtype == DISC_BF16, mean_in_edt);
    if (p.shape.want_dbar) launch_rbar(b, w, st);
  };
  if (stats && !fused) run_stats(false);
  { StageTimer t(sid < 0 ? -1 : ST_SCAN, st); launch_scan(b, w, st, p.shape.want_dbar, fused); }
  // the pooling order rides on the launch after the distance transform
  {
    StageTimer t(sid < 0 ? -1 : ST_EDT, st);
    launch_edt(b, w, nullptr, cus, st, o.edt_layout, true, mean_in_edt, packed ? proj->data : nullptr,
               proj->dtype == DISC_BF16);
  }
  if (fused) run_stats(true);
  { StageTimer t(sid < 0 ? -1 : ST_WEIGHTS, st); launch_weights(b, w, st); }
  {
    StageTimer t(sid < 0 ? -1 : ST_POOL, st);
    bool ran = false;
    const int nt = pool_tile_choice(p, tok_dtype, o, tune, b, w, tiles, st, &ran);
    if (!ran) launch_pool_choice(b, w, tiles, st, nt);
  }
  { StageTimer t(sid < 0 ? -1 : ST_PROJ, st); launch_proj(b, w, proj->data, proj->dtype == DISC_BF16, st, packed); }
}

}  // namespace host
}  // namespace disc

using namespace disc::host;

// ==========================================================================
// exported entry points
// ==========================================================================
extern "C" {

void disc_options_default(disc_options* o) {
  if (!o) return;
  o->spatial = DISC_SPATIAL_EDT;
  o->distinct = 1;
  o->eps = 1e-6f;
  o->gemm_dtype = -1;
  o->workspace = nullptr;
  o->workspace_bytes = 0;
  o->edt_layout = -1;
  o->pool_tile = -1;
  o->pool_rows = -1;
}

int32_t disc_abi_version(void) { return DISC_ABI_VERSION; }

const char* disc_last_error(void) { return g_err.c_str(); }

size_t disc_workspace_bytes(const disc_tokens* tokens, const disc_masks* masks, int32_t n_frames, const disc_proj* proj,
                            const disc_options* opts) {
  std::vector<FrameIn> fr;
  std::vector<disc_out> outs(std::max(n_frames, 0));
  for (int i = 0; i < n_frames && masks; ++i) {
    outs[i].data = reinterpret_cast<float*>(16);
    outs[i].m = masks[i].m;
    outs[i].e = proj ? proj->e : 0;
    outs[i].mask_status = nullptr;
    outs[i].pooled = nullptr;
  }
  if (describe(tokens, masks, n_frames, proj, outs.data(), opts, "disc_workspace_bytes", fr) != DISC_OK) return 0;
  if (n_frames == 0) return 0;
  Plan p;
  build_plan(fr, tokens[0].c, proj->e, resolve_gemm(opts, tokens[0].dtype, proj->dtype), p, tokens[0].dtype);
  return p.L.total;
}

disc_status disc_embed_frames(const disc_tokens* tokens, const disc_masks* masks, int32_t n_frames, const disc_proj* proj,
                              disc_out* out, const disc_options* opts, void* stream) {
  const char* who = "disc_embed_frames";
  std::vector<FrameIn> fr;
  disc_status st = describe(tokens, masks, n_frames, proj, out, opts, who, fr);
  if (st) return st;
  const disc_options o = opts ? *opts : defaults();
  int64_t M = 0;
  for (auto& f : fr) M += f.m;
  if (n_frames == 0 || M == 0) return ok();
  Plan p;
  build_plan(fr, tokens[0].c, proj->e, resolve_gemm(&o, tokens[0].dtype, proj->dtype), p, tokens[0].dtype);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), p.L, &o, cx))) return st;
  stage_host(p, cx.host_stage, cx.dev_ws);
  if ((st = upload(cx, p.L))) return st;
  enqueue_path(p, cx.dev_ws, tokens[0].dtype, o, proj, num_cus(cx.dev), cx.st, true, true);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_embed_masks_ex(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj, disc_out* out,
                                const disc_options* opts, void* stream) {
  return disc_embed_frames(tokens, masks, 1, proj, out, opts, stream);
}

disc_status disc_embed_masks(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj, disc_out* out) {
  return disc_embed_frames(tokens, masks, 1, proj, out, nullptr, nullptr);
}

disc_status disc_release_workspace(void) {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto& kv : g_ws) {
    if (kv.second.dev) (void)hipFree(kv.second.dev);
    if (kv.second.host) (void)hipHostFree(kv.second.host);
    if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
  }
  g_ws.clear();
  return ok();
}

disc_status disc_edt_sq(const disc_masks* masks, int32_t* e, void* stream) {
  const char* who = "disc_edt_sq";
  disc_status st;
  if ((st = check_masks(masks, who))) return st;
  if (masks->m == 0) return ok();
  if (!e) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: e is NULL", who);
  if (!aligned16(e)) return fail(DISC_ERR_ALIGNMENT, "%s: e must be 16-byte aligned", who);
  FrameIn f;
  f.bits = masks->bits;
  f.patch = 16;
  f.h = masks->h;
  f.w = masks->w;
  f.gh = (f.h + 15) / 16;
  f.gw = (f.w + 15) / 16;
  f.m = masks->m;
  Plan p;
  build_plan({f}, 64, 128, 0, p);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), p.L, nullptr, cx))) return st;
  stage_host(p, cx.host_stage, cx.dev_ws);
  if ((st = upload(cx, p.L))) return st;
  const Batch b = make_batch(p, cx.dev_ws, DISC_F32, DISC_SPATIAL_EDT, 0);
  const Work w = work_ptrs(cx.dev_ws, p.L);
  launch_fill_u32(reinterpret_cast<uint32_t*>(e), 0u, (int64_t)masks->m * masks->h * masks->w, cx.st);
  launch_scan(b, w, cx.st);
  launch_edt(b, w, e, num_cus(cx.dev), cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_patch_weights(const disc_tokens* tokens, const disc_masks* masks, int32_t patch, const disc_options* opts,
                               float* wout, void* stream) {
  const char* who = "disc_patch_weights";
  disc_status st;
  if ((st = check_opts(opts, who))) return st;
  const disc_options o = opts ? *opts : defaults();
  if ((st = check_masks(masks, who))) return st;
  if (patch < kMinPatch || patch > kMaxPatch) return fail(DISC_ERR_LIMIT, "%s: patch %d outside [%d, %d]", who, patch, kMinPatch, kMaxPatch);
  if (o.distinct) {
    if ((st = check_tokens(tokens, who))) return st;
    if (tokens->patch != patch) return fail(DISC_ERR_SHAPE, "%s: patch %d differs from tokens->patch %d", who, patch, tokens->patch);
    if ((st = check_grid(tokens, masks, who))) return st;
  }
  if (masks->m == 0) return ok();
  if (!wout) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: w is NULL", who);
  if (!aligned16(wout)) return fail(DISC_ERR_ALIGNMENT, "%s: w must be 16-byte aligned", who);
  FrameIn f;
  f.bits = masks->bits;
  f.patch = patch;
  f.h = masks->h;
  f.w = masks->w;
  f.gh = (f.h + patch - 1) / patch;
  f.gw = (f.w + patch - 1) / patch;
  f.m = masks->m;
  if (o.distinct) {
    f.tokens = tokens->data;
    f.scale = tokens->scale;
  }
  const int C = o.distinct ? tokens->c : 64;
  Plan p;
  build_plan({f}, C, 128, 0, p);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), p.L, nullptr, cx))) return st;
  stage_host(p, cx.host_stage, cx.dev_ws);
  if ((st = upload(cx, p.L))) return st;
  const Batch b = make_batch(p, cx.dev_ws, o.distinct ? tokens->dtype : DISC_F32, o.spatial, o.distinct);
  const Work w = work_ptrs(cx.dev_ws, p.L);
  launch_scan(b, w, cx.st);
  if (o.distinct) launch_token_stats(b, w, p.shape.gmax, cx.st);
  launch_edt(b, w, nullptr, num_cus(cx.dev), cx.st, o.edt_layout);
  launch_dense_weights(b, w, wout, o.eps, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_token_stats(const disc_tokens* tokens, float eps, float* mean, float* r, float* D, void* stream) {
  const char* who = "disc_token_stats";
  disc_status st;
  if ((st = check_tokens(tokens, who))) return st;
  if (!(eps >= 0.f)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: eps must be >= 0", who);
  if ((mean && !aligned16(mean)) || (r && !aligned16(r)) || (D && !aligned16(D)))
    return fail(DISC_ERR_ALIGNMENT, "%s: outputs must be 16-byte aligned", who);
  FrameIn f;
  f.tokens = tokens->data;
  f.scale = tokens->scale;
  f.gh = tokens->gh;
  f.gw = tokens->gw;
  f.patch = tokens->patch;
  f.h = tokens->gh * tokens->patch;
  f.w = tokens->gw * tokens->patch;
  f.m = 0;
  Plan p;
  build_plan({f}, tokens->c, 128, 0, p);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), p.L, nullptr, cx))) return st;
  stage_host(p, cx.host_stage, cx.dev_ws);
  if ((st = upload(cx, p.L))) return st;
  const Batch b = make_batch(p, cx.dev_ws, tokens->dtype, 0, 1);
  const Work w = work_ptrs(cx.dev_ws, p.L);
  const int G = tokens->gh * tokens->gw;
  launch_token_stats(b, w, G, cx.st);
  if (mean) launch_copy_f32(w.mean, mean, tokens->c, cx.st);
  if (r) launch_copy_f32(w.r, r, G, cx.st);
  if (D) launch_d_from_r(w.r, G, eps, D, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_query_heatmap(const disc_tokens* tokens, const disc_proj* proj, const void* text, int32_t text_dtype,
                               int32_t q, float eps, float* heat, void* stream) {
  const char* who = "disc_query_heatmap";
  disc_status st;
  if ((st = check_tokens(tokens, who))) return st;
  if ((st = check_proj(proj, tokens->c, who))) return st;
  if (q < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative query count", who);
  if (q > (1 << 20)) return fail(DISC_ERR_LIMIT, "%s: at most 2^20 queries per call", who);
  if (text_dtype != DISC_F32 && text_dtype != DISC_BF16)
    return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: text dtype must be F32 or BF16", who);
  if (!(eps >= 0.f)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: eps must be >= 0", who);
  if (q == 0) return ok();
  if (!text || !heat) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: text and heat must not be NULL", who);
  if (!aligned16(text) || !aligned16(heat)) return fail(DISC_ERR_ALIGNMENT, "%s: text and heat must be 16-byte aligned", who);
  const int G = tokens->gh * tokens->gw, C = tokens->c, E = proj->e;
  FrameIn f;
  f.tokens = tokens->data;
  f.scale = tokens->scale;
  f.gh = tokens->gh;
  f.gw = tokens->gw;
  f.patch = tokens->patch;
  f.h = tokens->gh * tokens->patch;
  f.w = tokens->gw * tokens->patch;
  f.m = 0;
  Plan p;
  build_plan({f}, C, 128, 0, p);
  // projected tokens Y [G][E], D [G], per-patch factors [G], text inverse norms [q]
  const int64_t yb = round_up(4 * (int64_t)G * E, 256), gb = round_up(4 * (int64_t)G, 256);
  p.shape.extra_bytes = yb + 2 * gb + round_up(4 * (int64_t)q, 256);
  p.L = make_layout(p.shape);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), p.L, nullptr, cx))) return st;
  stage_host(p, cx.host_stage, cx.dev_ws);
  if ((st = upload(cx, p.L))) return st;
  const Batch b = make_batch(p, cx.dev_ws, tokens->dtype, 0, 1);
  const Work w = work_ptrs(cx.dev_ws, p.L);
  char* x = cx.dev_ws + p.L.extra;
  float* Y = reinterpret_cast<float*>(x);
  float* D = reinterpret_cast<float*>(x + yb);
  float* fac = reinterpret_cast<float*>(x + yb + gb);
  float* inv_text = reinterpret_cast<float*>(x + yb + 2 * gb);
  launch_token_stats(b, w, G, cx.st);
  launch_d_from_r(w.r, G, eps, D, cx.st);
  launch_heatmap(tokens->data, tokens->dtype, tokens->scale, G, C, proj->data, proj->dtype == DISC_BF16, E, text,
                 text_dtype == DISC_BF16, q, D, Y, fac, inv_text, heat, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_pool_project(const disc_tokens* tokens, const float* wts, int32_t m, const disc_proj* proj, disc_out* out,
                              int32_t gemm_dtype, void* stream) {
  const char* who = "disc_pool_project";
  disc_status st;
  if ((st = check_tokens(tokens, who))) return st;
  if (m < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative mask count", who);
  if ((st = check_proj(proj, tokens->c, who))) return st;
  if ((st = check_out(out, m, proj->e, who))) return st;
  if (gemm_dtype != -1 && gemm_dtype != DISC_F32 && gemm_dtype != DISC_BF16)
    return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: gemm dtype must be F32, BF16 or -1", who);
  if (m == 0) return ok();
  if (!wts) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: w is NULL", who);
  if (!aligned16(wts)) return fail(DISC_ERR_ALIGNMENT, "%s: w must be 16-byte aligned", who);
  disc_options o = defaults();
  o.gemm_dtype = gemm_dtype;
  FrameIn f;
  f.tokens = tokens->data;
  f.scale = tokens->scale;
  f.gh = tokens->gh;
  f.gw = tokens->gw;
  f.patch = tokens->patch;
  f.h = tokens->gh * tokens->patch;
  f.w = tokens->gw * tokens->patch;
  f.m = m;
  f.out = out->data;
  f.status = out->mask_status;
  f.pooled = out->pooled;
  Plan p;
  build_plan({f}, tokens->c, proj->e, resolve_gemm(&o, tokens->dtype, proj->dtype), p, tokens->dtype);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), p.L, nullptr, cx))) return st;
  stage_host(p, cx.host_stage, cx.dev_ws);
  if ((st = upload(cx, p.L))) return st;
  const Batch b = make_batch(p, cx.dev_ws, tokens->dtype, 0, 1);
  const Work w = work_ptrs(cx.dev_ws, p.L);
  const int4* tiles = reinterpret_cast<const int4*>(cx.dev_ws + p.L.tiles);
  if (tokens->dtype == DISC_F8E4M3) launch_scale_check(b, w, p.shape.gmax, cx.st);
  launch_user_weights(b, w, wts, cx.st);
  launch_pool_order(b, w, cx.st);
  launch_pool(b, w, tiles, cx.st, o.pool_tile > 0 ? o.pool_tile : 1, o.pool_rows == 128 ? 2 : 1);
  launch_proj(b, w, proj->data, proj->dtype == DISC_BF16, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_pack_masks(const uint8_t* u8, int32_t m, int32_t h, int32_t w, uint64_t* bits, void* stream) {
  const char* who = "disc_pack_masks";
  if (m < 0 || h <= 0 || w <= 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: bad shape %dx%dx%d", who, m, h, w);
  if (m == 0) return ok();
  if (!u8 || !bits) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  if (!aligned16(bits)) return fail(DISC_ERR_ALIGNMENT, "%s: bits must be 16-byte aligned", who);
  launch_pack(u8, m, h, w, bits, static_cast<hipStream_t>(stream));
  disc_status st;
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_query_topk(const float* emb, int32_t m, const void* text, int32_t text_dtype, int32_t q, int32_t e,
                            int32_t k, float* sim, float* scores, int32_t* idx, void* stream) {
  const char* who = "disc_query_topk";
  if (m < 0 || q < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative count (m %d, q %d)", who, m, q);
  if (e <= 0 || e % 16 != 0 || e > 4096)
    return fail(DISC_ERR_LIMIT, "%s: embedding width %d must be a multiple of 16 up to 4096", who, e);
  if (k < 1 || k > 256) return fail(DISC_ERR_LIMIT, "%s: k = %d outside [1, 256]", who, k);
  if (m > (1 << 24)) return fail(DISC_ERR_LIMIT, "%s: m = %d exceeds 2^24", who, m);
  if (text_dtype != DISC_F32 && text_dtype != DISC_BF16)
    return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: text dtype must be F32 or BF16", who);
  if (q == 0) return ok();
  if (!text || !sim || !scores || !idx || (m > 0 && !emb)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  if ((m > 0 && !aligned16(emb)) || !aligned16(text) || !aligned16(sim) || !aligned16(scores) || !aligned16(idx))
    return fail(DISC_ERR_ALIGNMENT, "%s: pointers must be 16-byte aligned", who);
  Layout L{};
  L.staged_end = 0;
  L.total = (size_t)round_up(4 * ((int64_t)m + q), 256);
  Ctx cx;
  disc_status st;
  if ((st = acquire(static_cast<hipStream_t>(stream), L, nullptr, cx))) return st;
  launch_query(emb, m, text, text_dtype == DISC_BF16, q, e, k, reinterpret_cast<float*>(cx.dev_ws), sim, scores, idx,
               cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_view_quality(const int32_t* area, const float* dbar, const float* emb, const float* g,
                              const float* angle, int32_t m, int32_t e, int32_t img_h, int32_t img_w, float lambda,
                              float* q, float* comp, void* stream) {
  const char* who = "disc_view_quality";
  if (m < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative count %d", who, m);
  if (e <= 0 || e % 4 != 0 || e > 4096)
    return fail(DISC_ERR_LIMIT, "%s: embedding width %d must be a multiple of 4 up to 4096", who, e);
  if (img_h < 1 || img_w < 1) return fail(DISC_ERR_SHAPE, "%s: image size %d x %d", who, img_h, img_w);
  if (!(lambda > 0.f) || lambda > 1e30f) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: lambda must be positive", who);
  if (m == 0) return ok();
  if (!area || !dbar || !emb || !g || !q) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  if (!aligned16(emb) || !aligned16(g) || (comp && !aligned16(comp)))
    return fail(DISC_ERR_ALIGNMENT, "%s: emb, g and comp must be 16-byte aligned", who);
  launch_quality(area, dbar, emb, g, angle, m, e, img_h, img_w, lambda, q, comp, static_cast<hipStream_t>(stream));
  disc_status st;
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_angle_score(const float* rays, const float* normals, int32_t nv, const int32_t* off, int32_t m,
                             float* angle, void* stream) {
  const char* who = "disc_angle_score";
  if (m < 0 || nv < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative count (m %d, nv %d)", who, m, nv);
  if (nv > (1 << 29)) return fail(DISC_ERR_LIMIT, "%s: nv = %d exceeds 2^29", who, nv);
  if (m == 0) return ok();
  if (!off || !angle || (nv > 0 && (!rays || !normals)))
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  launch_angle(rays, normals, nv, off, m, angle, static_cast<hipStream_t>(stream));
  disc_status st;
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_fuse(const int32_t* ids, const float* q, const float* emb, int32_t m, int32_t e, float* map_q,
                      float* map_emb, int32_t n_map, int32_t* won, void* stream) {
  const char* who = "disc_fuse";
  if (m < 0 || n_map < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative count (m %d, n_map %d)", who, m, n_map);
  if (e <= 0 || e % 4 != 0 || e > 4096)
    return fail(DISC_ERR_LIMIT, "%s: embedding width %d must be a multiple of 4 up to 4096", who, e);
  if (n_map > (1 << 28)) return fail(DISC_ERR_LIMIT, "%s: n_map = %d exceeds 2^28", who, n_map);
  if (m == 0) return ok();
  if (!ids || !q || !emb || (n_map > 0 && (!map_q || !map_emb)))
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  if (!aligned16(emb) || (n_map > 0 && !aligned16(map_emb)))
    return fail(DISC_ERR_ALIGNMENT, "%s: emb and map_emb must be 16-byte aligned", who);
  Layout L{};
  L.staged_end = 0;
  L.total = (size_t)round_up(8 * (int64_t)std::max(n_map, 1), 256);
  Ctx cx;
  disc_status st;
  if ((st = acquire(static_cast<hipStream_t>(stream), L, nullptr, cx))) return st;
  launch_fuse(ids, q, emb, m, e, map_q, map_emb, n_map, won, reinterpret_cast<uint64_t*>(cx.dev_ws), cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

static disc_status geom_masks(const float* depth, const disc_masks* masks, const disc_camera* cam, int32_t stride,
                              const char* who) {
  disc_status st;
  if ((st = check_masks(masks, who))) return st;
  if (!cam) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: cam is NULL", who);
  if (stride < 1 || stride > 64) return fail(DISC_ERR_LIMIT, "%s: stride %d outside [1, 64]", who, stride);
  if (masks->m > 0 && !depth) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: depth is NULL", who);
  if (!(cam->fx != 0.f) || !(cam->fy != 0.f)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: zero focal length", who);
  return DISC_OK;
}

static void cam_floats(const disc_camera* c, float* f) {
  f[0] = c->fx;
  f[1] = c->fy;
  f[2] = c->cx;
  f[3] = c->cy;
  for (int k = 0; k < 9; ++k) f[4 + k] = c->R[k];
  for (int k = 0; k < 3; ++k) f[13 + k] = c->t[k];
  f[16] = c->depth_min;
  f[17] = c->depth_max;
}

disc_status disc_backproject_count(const float* depth, const disc_masks* masks, const disc_camera* cam,
                                   int32_t stride, int32_t* offsets, void* stream) {
  const char* who = "disc_backproject_count";
  disc_status st;
  if ((st = geom_masks(depth, masks, cam, stride, who))) return st;
  if (!offsets) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: offsets is NULL", who);
  const int m = masks->m;
  Layout L{};
  L.staged_end = 0;
  L.total = (size_t)round_up(4 * ((int64_t)m + 1 + (int64_t)scan_scratch_ints(m)), 256);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), L, nullptr, cx))) return st;
  float cf[18];
  cam_floats(cam, cf);
  int32_t* counts = reinterpret_cast<int32_t*>(cx.dev_ws);
  launch_bp_count(depth, masks->bits, m, masks->h, masks->w, stride, cf, counts, offsets, counts + m + 1, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_backproject(const float* depth, const disc_masks* masks, const disc_camera* cam, int32_t stride,
                             const int32_t* offsets, float* points, void* stream) {
  const char* who = "disc_backproject";
  disc_status st;
  if ((st = geom_masks(depth, masks, cam, stride, who))) return st;
  if (masks->m == 0) return ok();
  if (!offsets || !points) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  float cf[18];
  cam_floats(cam, cf);
  launch_bp_write(depth, masks->bits, masks->m, masks->h, masks->w, stride, cf, offsets, points,
                  static_cast<hipStream_t>(stream));
  if ((st = check_launch(who))) return st;
  return ok();
}

static disc_status check_cloud(const float* points, const int32_t* offsets, int32_t m, int32_t n, const char* who) {
  if (m < 0 || n < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative count (m %d, n %d)", who, m, n);
  if (m > 65535) return fail(DISC_ERR_LIMIT, "%s: m = %d exceeds 65535 segments", who, m);
  if (n > (1 << 23)) return fail(DISC_ERR_LIMIT, "%s: n = %d exceeds 2^23 points", who, n);
  if (!offsets || (n > 0 && !points)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  return DISC_OK;
}

disc_status disc_dbscan_denoise(const float* points, const int32_t* offsets, int32_t m, int32_t n, float eps,
                                int32_t min_pts, int32_t* keep, void* stream) {
  const char* who = "disc_dbscan_denoise";
  disc_status st;
  if ((st = check_cloud(points, offsets, m, n, who))) return st;
  if (!(eps > 0.f) || eps > 1e30f) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: eps must be positive", who);
  if (min_pts < 1) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: min_pts must be >= 1", who);
  if (n == 0) return ok();
  if (!keep) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: keep is NULL", who);
  Layout L{};
  L.staged_end = 0;
  L.total = (size_t)round_up((int64_t)dbscan_ws_bytes(n), 256);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), L, nullptr, cx))) return st;
  launch_dbscan(points, offsets, m, n, eps, min_pts, keep, cx.dev_ws, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_voxelize(const float* points, const int32_t* offsets, const int32_t* keep, int32_t m, int32_t n,
                          float voxel, int32_t* voffsets, int32_t* voxels, int32_t* status, void* stream) {
  const char* who = "disc_voxelize";
  disc_status st;
  if ((st = check_cloud(points, offsets, m, n, who))) return st;
  if (!(voxel > 0.f) || voxel > 1e30f) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: voxel must be positive", who);
  if (!voffsets || (n > 0 && !voxels)) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  Layout L{};
  L.staged_end = 0;
  L.total = (size_t)round_up((int64_t)voxel_ws_bytes(n, m), 256);
  Ctx cx;
  if ((st = acquire(static_cast<hipStream_t>(stream), L, nullptr, cx))) return st;
  launch_voxelize(points, offsets, keep, m, n, voxel, voffsets, voxels, status, cx.dev_ws, cx.st);
  if ((st = check_launch(who))) return st;
  return ok();
}

disc_status disc_voxel_overlap(const int32_t* va, const int32_t* oa, int32_t na, const int32_t* vb,
                               const int32_t* ob, int32_t nb, const int32_t* pairs, int32_t np, int32_t* counts,
                               void* stream) {
  const char* who = "disc_voxel_overlap";
  if (na < 0 || nb < 0 || np < 0) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: negative count", who);
  if (np == 0) return ok();
  if (!oa || !ob || !pairs || !counts) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL pointer", who);
  launch_overlap(va, oa, na, vb, ob, nb, pairs, np, counts, static_cast<hipStream_t>(stream));
  disc_status st;
  if ((st = check_launch(who))) return st;
  return ok();
}

}  // extern "C"

extern "C" {

void disc_trace_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_tr_mu);
  g_trace_on = on != 0;
}

void disc_trace_select(uint32_t stage_mask) {
  std::lock_guard<std::mutex> lk(g_tr_mu);
  g_trace_mask = stage_mask;
}

void disc_trace_reset(void) {
  tr_collect();
  std::lock_guard<std::mutex> lk(g_tr_mu);
  for (int i = 0; i < ST_COUNT; ++i) {
    g_tr_ms[i] = 0.0;
    g_tr_n[i] = 0;
  }
}

int32_t disc_trace_read(int32_t stage, double* total_ms, int64_t* count) {
  if (stage < 0 || stage >= ST_COUNT) return -1;
  tr_collect();
  std::lock_guard<std::mutex> lk(g_tr_mu);
  if (total_ms) *total_ms = g_tr_ms[stage];
  if (count) *count = g_tr_n[stage];
  return 0;
}

const char* disc_trace_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : nullptr;
}

}  // extern "C"
