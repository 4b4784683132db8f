// Continuous-batching request loop over DISC's single-pass feature extraction
// (arXiv 2603.03935, Sec. III-C; frames arrive from an RGB-D stream and every
// frame's masks are embedded as they come).  See include/disc.h for the
// contract.  Lanes (stream + resident workspace + pinned staging + optional
// captured graph) pull FIFO-packed batches from one queue.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"

using namespace disc;
using namespace disc::host;

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  uint64_t ticket;
  FrameIn fin;
  Clock::time_point t_sub;
};

struct Ticket {
  int state = 0;  // 0 waiting, 1 in flight, 2 done
  int32_t result = DISC_OK;
};

struct Lane {
  hipStream_t st = nullptr;
  char* dev_ws = nullptr;
  char* host_stage = nullptr;
  hipEvent_t ev = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_ready = false;
  std::thread th;
};

// Capacity shape of one lane: every batch the lane accepts fits it, so one
// workspace and one captured kernel set serve all of them.
Shape capacity_shape(const disc_server_config& c, int E, int gemm_bf16) {
  Shape s;
  const int gh = (c.max_h + c.min_patch - 1) / c.min_patch, gw = (c.max_w + c.min_patch - 1) / c.min_patch;
  const int G = gh * gw, Gs = (int)round_up(G, 8);
  s.n_frames = c.max_frames;
  s.M = c.max_masks;
  s.sumG = (int64_t)c.max_frames * G;
  s.sumMGs = (int64_t)c.max_masks * Gs;
  s.C = c.c;
  s.E = E;
  s.gmax = G;
  s.nchunk = 64;  // stat_nchunk(G) <= 64 for every frame size
  // a strip is at least 33 columns wide for every patch size in [8, 64]
  // per work sub-list: at most ceil(max_masks / kLists) masks, each with at
  // most max_w / 32 + 1 strips (a strip is at least 33 columns wide)
  s.item_cap = (int)std::min<int64_t>(((int64_t)c.max_masks + kLists - 1) / kLists * ((c.max_w + 31) / 32 + 1) + 1,
                                      INT32_MAX / 2 / kLists);
  s.n_tiles = ((c.max_masks + 63) / 64 + c.max_frames) * (c.c / 64);
  s.gemm_bf16 = gemm_bf16;
  s.want_dbar = true;  // any request may ask for the mean distinctiveness
  s.max_rows = c.max_h + 2;
  choose_splits(s);
  return s;
}

}  // namespace

struct disc_server {
  disc_server_config cfg{};
  disc_options opts{};
  int gemm_bf16 = 1;
  int dev = 0, cus = 256;
  Plan cap;  // capacity plan (layout of every lane's workspace)
  std::vector<Lane> lanes;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> pending;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  int in_flight = 0;
  bool stopping = false;
  uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, batch_frames = 0;
  // latencies of the last kLatWindow successful requests (a ring)
  static constexpr size_t kLatWindow = (size_t)1 << 20;
  std::vector<double> lat_ms;
  size_t lat_next = 0;
  void add_latency(double ms) {
    if (lat_ms.size() < kLatWindow) {
      lat_ms.push_back(ms);
    } else {
      lat_ms[lat_next] = ms;
      lat_next = (lat_next + 1) % kLatWindow;
    }
  }

  void lane_loop(int li);
  int32_t run_batch(Lane& ln, const std::vector<Request>& batch);
  int32_t capture(Lane& ln);
};

// Stage a batch's descriptors into the capacity layout (graph replay).
static void stage_capacity(const Plan& actual, const Plan& cap, char* host) {
  std::memcpy(host + cap.L.frames, actual.fds.data(), sizeof(FrameDesc) * actual.fds.size());
  if (!actual.mask_frame.empty())
    std::memcpy(host + cap.L.mask_frame, actual.mask_frame.data(), 4 * actual.mask_frame.size());
  if (!actual.tiles.empty()) std::memcpy(host + cap.L.tiles, actual.tiles.data(), 16 * actual.tiles.size());
  const int32_t dyn[4] = {actual.shape.n_frames, (int32_t)actual.shape.M, actual.shape.n_tiles, 0};
  std::memcpy(host + cap.L.dyn, dyn, sizeof dyn);
  std::memset(host + cap.L.counts, 0, 4 * (kCounters + (size_t)cap.shape.n_frames));
}

int32_t disc_server::capture(Lane& ln) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(ln.st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return DISC_ERR_DEVICE;
  (void)hipMemcpyAsync(ln.dev_ws, ln.host_stage, cap.L.staged_end, hipMemcpyHostToDevice, ln.st);
  enqueue_path(cap, ln.dev_ws, cfg.tok_dtype, opts, &cfg.proj, cus, ln.st, /*trace=*/false);
  e = hipStreamEndCapture(ln.st, &graph);
  if (e != hipSuccess || !graph) return DISC_ERR_DEVICE;
  e = hipGraphInstantiate(&ln.gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return DISC_ERR_DEVICE;
  ln.graph_ready = true;
  return DISC_OK;
}

int32_t disc_server::run_batch(Lane& ln, const std::vector<Request>& batch) {
  std::vector<FrameIn> fr;
  fr.reserve(batch.size());
  for (const Request& r : batch) fr.push_back(r.fin);
  Plan p;
  build_plan(fr, cfg.c, cfg.proj.e, gemm_bf16, p, cfg.tok_dtype);
  hipError_t e;
  if (cfg.use_graph) {
    if (!ln.graph_ready && capture(ln) != DISC_OK) return DISC_ERR_DEVICE;
    stage_capacity(p, cap, ln.host_stage);
    if ((e = hipGraphLaunch(ln.gexec, ln.st)) != hipSuccess) return DISC_ERR_DEVICE;
  } else {
    stage_host(p, ln.host_stage, ln.dev_ws);
    if ((e = hipMemcpyAsync(ln.dev_ws, ln.host_stage, p.L.staged_end, hipMemcpyHostToDevice, ln.st)) != hipSuccess)
      return DISC_ERR_DEVICE;
    enqueue_path(p, ln.dev_ws, cfg.tok_dtype, opts, &cfg.proj, cus, ln.st);
    if (hipPeekAtLastError() != hipSuccess) {
      (void)hipGetLastError();
      return DISC_ERR_DEVICE;
    }
  }
  if ((e = hipEventRecord(ln.ev, ln.st)) != hipSuccess) return DISC_ERR_DEVICE;
  if ((e = hipEventSynchronize(ln.ev)) != hipSuccess) return DISC_ERR_DEVICE;
  return DISC_OK;
}

void disc_server::lane_loop(int li) {
  Lane& ln = lanes[li];
  if (!cfg.dry_run) (void)hipSetDevice(dev);
  for (;;) {
    std::vector<Request> batch;
    uint64_t batch_id = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stopping || (!pending.empty() && in_flight < cfg.max_slots); });
      if (pending.empty() && stopping) return;
      const Clock::time_point now = Clock::now();
      int frames = 0, masks = 0;
      while (!pending.empty()) {
        Request& r = pending.front();
        if (cfg.admission_timeout_ms > 0 && ms_since(r.t_sub, now) > cfg.admission_timeout_ms) {
          Ticket& t = tickets[r.ticket];
          t.state = 2;
          t.result = DISC_ERR_ADMISSION;
          ++failed;
          pending.pop_front();
          continue;
        }
        if (frames + 1 > cfg.max_frames || masks + r.fin.m > cfg.max_masks ||
            in_flight + (int)batch.size() + 1 > cfg.max_slots)
          break;
        frames += 1;
        masks += r.fin.m;
        tickets[r.ticket].state = 1;
        batch.push_back(r);
        pending.pop_front();
      }
      if (batch.empty()) {
        cv_done.notify_all();
        continue;
      }
      in_flight += (int)batch.size();
      batch_id = batches++;
      batch_frames += batch.size();
    }
    int32_t res = DISC_OK;
    if ((int64_t)cfg.fault_batch == (int64_t)batch_id)
      res = DISC_ERR_DEVICE;
    else if (!cfg.dry_run)
      res = run_batch(ln, batch);
    else if (cfg.dry_run > 1)
      std::this_thread::sleep_for(std::chrono::microseconds(cfg.dry_run));
    const Clock::time_point done = Clock::now();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (const Request& r : batch) {
        Ticket& t = tickets[r.ticket];
        t.state = 2;
        t.result = res;
        if (res == DISC_OK) {
          ++completed;
          add_latency(ms_since(r.t_sub, done));
        } else {
          ++failed;
        }
      }
      in_flight -= (int)batch.size();
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" {

void disc_server_config_default(disc_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->tok_dtype = DISC_BF16;
  c->c = 1024;
  c->max_frames = 16;
  c->max_masks = 1024;
  c->max_h = 720;
  c->max_w = 1280;
  c->min_patch = 14;
  c->max_slots = 64;
  c->lanes = 2;
  c->mem_budget = (size_t)4 << 30;
  c->use_graph = 1;
  c->dry_run = 0;
  c->fault_batch = -1;
  c->admission_timeout_ms = 0.0;
  disc_options_default(&c->opts);
}

disc_status disc_server_create(const disc_server_config* cfg, disc_server** out) {
  const char* who = "disc_server_create";
  if (!cfg || !out) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL argument", who);
  *out = nullptr;
  disc_status st;
  if ((st = check_opts(&cfg->opts, who))) return st;
  if (cfg->tok_dtype < DISC_F32 || cfg->tok_dtype > DISC_F8E4M3) return fail(DISC_ERR_UNSUPPORTED_DTYPE, "%s: token dtype", who);
  if (cfg->c <= 0 || cfg->c % 64 || cfg->c > kMaxC) return fail(DISC_ERR_LIMIT, "%s: channels %d", who, cfg->c);
  if (!cfg->dry_run && (st = check_proj(&cfg->proj, cfg->c, who))) return st;
  if (cfg->dry_run && (cfg->proj.e <= 0 || cfg->proj.e % 128 || cfg->proj.e > 1024 || cfg->proj.c != cfg->c))
    return fail(DISC_ERR_SHAPE, "%s: projection shape", who);
  if (cfg->max_frames < 1 || cfg->max_masks < 1 || cfg->max_slots < 1 || cfg->lanes < 1 || cfg->lanes > 8)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: capacities must be positive (lanes 1..8)", who);
  if (cfg->max_h < 1 || cfg->max_w < 1 || cfg->max_h > kMaxRows - 2 || cfg->min_patch < kMinPatch || cfg->min_patch > kMaxPatch)
    return fail(DISC_ERR_LIMIT, "%s: frame capacity %dx%d / patch %d outside the limits", who, cfg->max_h, cfg->max_w,
                cfg->min_patch);
  disc_server* s = new disc_server();
  s->cfg = *cfg;
  s->opts = cfg->opts;
  s->opts.workspace = nullptr;
  s->opts.workspace_bytes = 0;
  s->gemm_bf16 = resolve_gemm(&s->opts, cfg->tok_dtype, cfg->dry_run ? DISC_BF16 : cfg->proj.dtype);
  s->cap.shape = capacity_shape(*cfg, cfg->proj.e, s->gemm_bf16);
  s->cap.L = make_layout(s->cap.shape);
  const size_t per_lane = s->cap.L.total;
  int nl = (int)std::min<size_t>((size_t)cfg->lanes, cfg->mem_budget / std::max<size_t>(per_lane, 1));
  if (nl < 1) {
    delete s;
    return fail(DISC_ERR_OUT_OF_MEMORY, "%s: a lane needs %zu bytes, the budget is %zu", who, per_lane, cfg->mem_budget);
  }
  s->lanes.resize(nl);
  if (!cfg->dry_run) {
    hipError_t e;
    if ((e = hipGetDevice(&s->dev)) != hipSuccess) {
      delete s;
      return hip_fail(e, who);
    }
    s->cus = num_cus(s->dev);
    edt_prepare();
    for (Lane& ln : s->lanes) {
      bool okl = hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) == hipSuccess &&
                 hipMalloc(reinterpret_cast<void**>(&ln.dev_ws), per_lane) == hipSuccess &&
                 hipHostMalloc(reinterpret_cast<void**>(&ln.host_stage), s->cap.L.staged_end, hipHostMallocDefault) == hipSuccess &&
                 hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming) == hipSuccess;
      if (!okl) {
        disc_server_destroy(s);
        return fail(DISC_ERR_OUT_OF_MEMORY, "%s: lane allocation failed", who);
      }
    }
  }
  for (int i = 0; i < nl; ++i) s->lanes[i].th = std::thread(&disc_server::lane_loop, s, i);
  *out = s;
  return ok();
}

disc_status disc_server_submit(disc_server* s, const disc_tokens* t, const disc_masks* m, disc_out* o, uint64_t* ticket) {
  const char* who = "disc_server_submit";
  if (!s || !ticket) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: NULL argument", who);
  disc_status st;
  if ((st = check_tokens(t, who)) || (st = check_masks(m, who)) || (st = check_grid(t, m, who))) return st;
  if ((st = check_out(o, m->m, s->cfg.proj.e, who))) return st;
  const disc_server_config& c = s->cfg;
  if (t->dtype != c.tok_dtype || t->c != c.c || m->m > c.max_masks || m->h > c.max_h || m->w > c.max_w ||
      t->patch < c.min_patch) {
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->rejected;
    return fail(DISC_ERR_ADMISSION, "%s: request (%d masks, %dx%d, patch %d, dtype %d, c %d) exceeds the server capacity",
                who, m->m, m->h, m->w, t->patch, t->dtype, t->c);
  }
  Request r;
  r.fin.tokens = t->data;
  r.fin.scale = t->scale;
  r.fin.bits = m->bits;
  r.fin.out = o->data;
  r.fin.status = o->mask_status;
  r.fin.pooled = o->pooled;
  r.fin.dbar = o->dbar;
  r.fin.area = o->area;
  r.fin.gh = t->gh;
  r.fin.gw = t->gw;
  r.fin.patch = t->patch;
  r.fin.h = m->h;
  r.fin.w = m->w;
  r.fin.m = m->m;
  r.t_sub = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(DISC_ERR_INVALID_ARGUMENT, "%s: server is stopping", who);
    r.ticket = s->next_ticket++;
    s->tickets[r.ticket] = Ticket{};
    if (m->m == 0) {  // nothing to compute
      s->tickets[r.ticket].state = 2;
      ++s->completed;
      s->add_latency(0.0);
    } else {
      s->pending.push_back(r);
    }
    ++s->submitted;
    *ticket = r.ticket;
  }
  s->cv_work.notify_one();
  return ok();
}

disc_status disc_server_poll(disc_server* s, uint64_t ticket, int32_t* done, int32_t* result) {
  if (!s || !done) return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_poll: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_poll: unknown ticket");
  *done = it->second.state == 2;
  if (result) *result = it->second.result;
  if (*done) s->tickets.erase(it);  // reported: the ticket is forgotten
  return ok();
}

disc_status disc_server_wait(disc_server* s, uint64_t ticket, int32_t* result) {
  if (!s) return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->tickets.find(ticket) == s->tickets.end())
    return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_wait: unknown ticket");
  s->cv_done.wait(lk, [&] { return s->tickets[ticket].state == 2; });
  auto it = s->tickets.find(ticket);
  if (result) *result = it->second.result;
  s->tickets.erase(it);  // reported: the ticket is forgotten
  return ok();
}

disc_status disc_server_drain(disc_server* s) {
  if (!s) return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_drain: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->in_flight == 0; });
  return ok();
}

disc_status disc_server_get_stats(disc_server* s, disc_server_stats* st) {
  if (!s || !st) return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_get_stats: NULL argument");
  std::vector<double> v;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof *st);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->rejected = s->rejected;
    st->batches = s->batches;
    st->mean_batch_frames = s->batches ? (double)s->batch_frames / (double)s->batches : 0.0;
    st->lanes = (int32_t)s->lanes.size();
    st->lane_workspace_bytes = s->cap.L.total;
    v = s->lat_ms;  // copied under the lock, sorted outside it
  }
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5))]; };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    st->max_ms = v.back();
    double sum = 0.0;
    for (double x : v) sum += x;
    st->mean_ms = sum / (double)v.size();
  }
  return ok();
}

disc_status disc_server_reset_stats(disc_server* s) {
  if (!s) return fail(DISC_ERR_INVALID_ARGUMENT, "disc_server_reset_stats: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->submitted = s->completed = s->failed = s->rejected = s->batches = s->batch_frames = 0;
  s->lat_ms.clear();
  s->lat_next = 0;
  return ok();
}

void disc_server_destroy(disc_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->in_flight == 0; });
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (Lane& ln : s->lanes)
    if (ln.th.joinable()) ln.th.join();
  if (!s->cfg.dry_run) {
    for (Lane& ln : s->lanes) {
      if (ln.gexec) (void)hipGraphExecDestroy(ln.gexec);
      if (ln.ev) (void)hipEventDestroy(ln.ev);
      if (ln.st) (void)hipStreamSynchronize(ln.st);
      if (ln.dev_ws) (void)hipFree(ln.dev_ws);
      if (ln.host_stage) (void)hipHostFree(ln.host_stage);
      if (ln.st) (void)hipStreamDestroy(ln.st);
    }
  }
  delete s;
}

}  // extern "C"
