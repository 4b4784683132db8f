// Host-side planning shared by the one-shot entry points and the serving
// runtime (internal; not installed).
#pragma once

#include <string>
#include <vector>

#include "../../include/disc.h"
#include "disc_device.h"

namespace disc {
namespace host {

struct Layout {
  size_t frames, mask_frame, tiles, dyn, staged_end;  // staged region (uploaded from the host)
  size_t bbox, area, meta, mrec, items, counts, psum, mean, r, rbar, s, W, Z, mstat, perm, X, ppart, ptile, qpart, ppack, edt_part;
  size_t extra;  // extra_bytes for an entry point's own buffers
  size_t total;
};

struct Shape {
  int n_frames = 0;
  int64_t M = 0, sumG = 0, sumMGs = 0;
  int C = 0, E = 0, gmax = 0, nchunk = 1, item_cap = 1, n_tiles = 0, gemm_bf16 = 0;
  int kgroups = 1;        // pooling K groups of the largest frame
  int pool_split = 1, proj_split = 1;
  bool want_dbar = false;  // some frame asks for the mean distinctiveness (needs r and its mean)
  int max_rows = kMaxRows;  // tallest frame + 2 (distance-transform rows of the tallest item)
  int64_t extra_bytes = 0;  // appended region (e.g. the heat-map's projected tokens)
};

// Split K of the pooling / projection GEMMs when their tiles alone would not
// fill the GPU (depends only on the capacity shape).
void choose_splits(Shape& s);

struct FrameIn {
  const void* tokens = nullptr;
  const float* scale = nullptr;
  const uint64_t* bits = nullptr;
  float* out = nullptr;
  int32_t* status = nullptr;
  float* pooled = nullptr;
  float* dbar = nullptr;
  int32_t* area = nullptr;
  int gh = 0, gw = 0, patch = 16, h = 0, w = 0, m = 0;
};

struct Plan {
  Shape shape;
  Layout L;
  std::vector<FrameDesc> fds;
  std::vector<int32_t> mask_frame;
  std::vector<int4> tiles;
};

// Capacity totals accumulated while frames are added to a plan.
struct PlanAcc {
  int64_t M = 0, sumG = 0, sumMGs = 0;
  int64_t item_sub[kLists] = {};  // work-list capacity of each sub-list (masks g with g % kLists == j)
  int gmax = 0, nchunk = 1, n_tiles = 0;
};

extern thread_local std::string g_err;
bool aligned16(const void* p);
int64_t round_up(int64_t x, int64_t a);
disc_status fail(disc_status st, const char* fmt, ...);
disc_status ok();
disc_status hip_fail(hipError_t e, const char* what);
disc_status check_tokens(const disc_tokens* t, const char* who);
disc_status check_masks(const disc_masks* m, const char* who);
disc_status check_grid(const disc_tokens* t, const disc_masks* m, const char* who);
disc_status check_proj(const disc_proj* p, int c, const char* who);
disc_status check_out(const disc_out* o, int m, int e, const char* who);
disc_status check_opts(const disc_options* o, const char* who);
disc_status check_launch(const char* who);
Layout make_layout(const Shape& s);
void build_plan(const std::vector<FrameIn>& fr, int C, int E, int gemm_bf16, Plan& p, int tok_dtype = DISC_BF16);
// The same in steps, for callers that build no host vectors: begin_plan, then
// plan_frame per frame (its descriptor and the pooling tiles
// (frame, m0, n0) for m0 in steps of 64, n0 in steps of 64 below C), then
// finish_plan (totals and layout).
void begin_plan(Plan& p, int n_frames, int C, int E, int gemm_bf16, int tok_dtype);
FrameDesc plan_frame(const FrameIn& f, int C, Shape& s, PlanAcc& a);
void finish_plan(Plan& p, const PlanAcc& a);
disc_status describe_one(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj, disc_out* out,
                         const disc_options* opts, const char* who, FrameIn& f);
void stage_host(const Plan& p, char* host, char* dev);
Batch make_batch(const Plan& p, char* dev, int tok_dtype, int spatial, int distinct);
Work work_ptrs(char* base, const Layout& L);
int resolve_gemm(const disc_options* o, int tok_dtype, int proj_dtype);
disc_options defaults();
int num_cus(int dev);
// Enqueue the whole kernel sequence of a staged plan on a stream.
// trace = false while capturing a graph.
// tune = true lets the pooling autotuner time its candidates on this call
// (never while capturing a graph).
void enqueue_path(const Plan& p, char* dev_ws, int tok_dtype, const disc_options& o, const disc_proj* proj, int cus,
                  hipStream_t st, bool trace = true, bool tune = false);

}  // namespace host
}  // namespace disc
