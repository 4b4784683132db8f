// Single-frame embedding that allocates nothing (disc_embed_masks_noalloc).
//
// It runs the same kernel sequence as disc_embed_masks_ex, but its workspace
// is the file-scope device array `scratch` below instead of memory the
// library allocates or the caller passes, and the staged descriptors (frame
// record, mask -> frame map, pooling tiles, live counts, distance-transform
// class counters) are written by a kernel instead of being uploaded from a
// pinned host buffer.  Nothing is allocated, no memset or copy node is
// enqueued and no event is created, so the call is usable where hipMalloc is
// not: under stream capture, in tight serving loops, in harnesses that
// forbid allocation.  Every call on a GPU shares that GPU's array: calls that
// overlap on one GPU (two streams, two threads) race.
#include <mutex>

#include "../../include/disc.h"
#include "disc_device.h"
#include "host.h"

namespace disc {
namespace host {

constexpr size_t kScratchBytes = (size_t)DISC_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, held until the process ends.  In host code its name is a
// stand-in, not a device address: kernels get the address resolved below.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scr_mu;
char* g_scr[kMaxDevices] = {};
int g_scr_cus[kMaxDevices] = {};

// Device address of the current GPU's scratch array and its CU count,
// resolved once per device with that device current.
disc_status scratch_of(int dev, char** ptr, int* cus) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DISC_ERR_LIMIT, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scr_mu);
  if (!g_scr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scr_cus[dev] = num_cus(dev);
    g_scr[dev] = static_cast<char*>(p);
  }
  *ptr = g_scr[dev];
  *cus = g_scr_cus[dev];
  return DISC_OK;
}

// The staged region of a one-frame plan: what the other entry points upload
// from the host (frame descriptor, mask -> frame map, pooling tiles in the
// order (m0, n0), live counts {frames, masks, tiles, 0}, zeroed class
// counters).
__global__ void k_stage_frame(FrameDesc d, int32_t M, int32_t C, int32_t n_tiles, FrameDesc* frames,
                              int32_t* mask_frame, int4* tiles, int32_t* dyn, int32_t* counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  if (i == 0) {
    frames[0] = d;
    dyn[0] = 1;
    dyn[1] = M;
    dyn[2] = n_tiles;
    dyn[3] = 0;
  }
  if (i < kCounters + 1) counts[i] = 0;  // work-list and queue counters and the frame's scale flag
  const int nct = C / 64;
  for (int k = i; k < M; k += stride) mask_frame[k] = 0;
  for (int t = i; t < n_tiles; t += stride) {
    const int m0 = (t / nct) * 64;
    tiles[t] = make_int4(0, m0, (t % nct) * 64, pool_pair_flag(m0, M));
  }
}

}  // namespace host
}  // namespace disc

using namespace disc;
using namespace disc::host;

extern "C" disc_status disc_embed_masks_noalloc(const disc_tokens* tokens, const disc_masks* masks,
                                                const disc_proj* proj, disc_out* out, const disc_options* opts,
                                                void* stream) {
  const char* who = "disc_embed_masks_noalloc";
  FrameIn f;
  disc_status st = describe_one(tokens, masks, proj, out, opts, who, f);
  if (st) return st;
  if (opts && opts->workspace)
    return fail(DISC_ERR_INVALID_ARGUMENT, "%s: takes no workspace (it works in the library's scratch array)", who);
  const disc_options o = opts ? *opts : defaults();
  if (f.m == 0) return ok();
  Plan p;  // its host vectors stay empty
  begin_plan(p, 1, tokens->c, proj->e, resolve_gemm(&o, tokens->dtype, proj->dtype), tokens->dtype);
  PlanAcc acc;
  const FrameDesc d = plan_frame(f, tokens->c, p.shape, acc);
  finish_plan(p, acc);
  if (p.L.total > kScratchBytes)
    return fail(DISC_ERR_LIMIT, "%s: this frame needs %zu bytes of scratch; the array holds %zu", who, p.L.total,
                kScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  char* ws = nullptr;
  int cus = 0;
  if ((st = scratch_of(dev, &ws, &cus))) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int M = (int)p.shape.M, n_tiles = p.shape.n_tiles;
  const int grid = std::max(1, std::min(64, (std::max(M, n_tiles) + 255) / 256));
  hipLaunchKernelGGL(k_stage_frame, dim3(grid), dim3(256), 0, hs, d, M, p.shape.C, n_tiles,
                     reinterpret_cast<FrameDesc*>(ws + p.L.frames), reinterpret_cast<int32_t*>(ws + p.L.mask_frame),
                     reinterpret_cast<int4*>(ws + p.L.tiles), reinterpret_cast<int32_t*>(ws + p.L.dyn),
                     reinterpret_cast<int32_t*>(ws + p.L.counts));
  enqueue_path(p, ws, tokens->dtype, o, proj, cus, hs, /*trace=*/false, /*tune=*/false);
  if ((st = check_launch(who))) return st;
  return ok();
}
