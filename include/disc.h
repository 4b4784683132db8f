/*
 * disc.h -- C ABI of libdisc: mask-aligned, distance-weighted feature
 * extraction from a ViT patch-token map on AMD Instinct MI355X (gfx950).
 *
 * The operation is DISC's single-pass instance feature extraction (arXiv
 * 2603.03935, Sec. III-C): for every 2D instance mask of a frame, aggregate the
 * patch features that lie inside the mask, weighted by the distinctiveness map
 * D of Eq. (1), instead of cropping the image and re-running CLIP; the paper
 * calls the mechanism "distance-weighted" (abstract, Sec. V).  Per mask the
 * library computes
 *
 *   e(x)    exact squared Euclidean distance from mask pixel x to the nearest
 *           pixel outside the mask (pixels outside the frame count as
 *           outside), integer-exact;
 *   s_p     sum over the mask's pixels in patch p of sqrt(e(x))
 *           (AREA mode: the pixel count), patch p = (floor(y/P), floor(x/P));
 *   D_p     ||f_p - mean(f)|| / (mean_p ||f_p - mean(f)|| + eps)   (Eq. 1);
 *   w_p     s_p * D_p (or s_p with distinctiveness off);
 *   F       sum_p w_p f_p / sum_p w_p    (weighted mean of the tokens);
 *   out     y / ||y||_2 with y = F^T P  (CLIP embeddings are compared by
 *           cosine similarity, Sec. III-C and IV-A).
 *
 * Degenerate cases: an empty mask gives a zero row (status 1); when every
 * touched patch has D = 0 the weights fall back to s; a zero projected vector
 * gives a zero row (status 2).
 *
 * Conventions for every entry point:
 *   - Data pointers are DEVICE pointers (HIP, the current device) unless a
 *     comment says otherwise.  The caller owns every buffer; the library never
 *     frees or retains caller memory beyond the call's stream work.
 *   - Arguments are validated on the host before anything is enqueued.  On a
 *     validation failure nothing is written to device memory, the call returns
 *     a non-zero disc_status and disc_last_error() describes the problem.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *     null stream).  A device fault surfaces as DISC_ERR_DEVICE from a later
 *     call or the caller's own synchronisation.
 *   - m == 0 masks is a no-op that returns DISC_OK.
 *   - Calls on different streams may run concurrently; the library keeps one
 *     workspace per (device, stream) unless the caller passes its own.
 *   - Stream capture: the entry points that take a stream stage their
 *     descriptors through a host buffer that the next call reuses (and may
 *     time tuning candidates or grow a workspace), so they refuse a stream
 *     that is being captured (DISC_ERR_INVALID_ARGUMENT, nothing enqueued).
 *     disc_embed_masks_noalloc enqueues kernels only and can be captured;
 *     the serving runtime captures its own graphs.
 *
 * Layouts:
 *   tokens  [gh][gw][c] row-major, c fastest; gh = ceil(h/patch), gw = ceil(w/patch)
 *           (the last patch row/column may cover fewer pixels).
 *   masks   bits[m][h][ceil(w/64)] uint64; bit i of word k of a row is pixel
 *           column 64k+i; bits at columns >= w are ignored.
 *   proj    [c][e] row-major.
 *   out     [m][e] FP32 rows of unit L2 norm (or zero rows, see above).
 *
 * Limits of this version: h, w >= 1, w <= 8448, every mask's bounding box at
 * most 1150 rows tall (frames up to 1150 rows are always accepted),
 * 8 <= patch <= 64,
 * c a multiple of 64 up to 2048, e a multiple of 128 up to 1024.
 */
#ifndef DISC_H
#define DISC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DISC_ABI_VERSION 5

typedef enum disc_status {
  DISC_OK = 0,
  DISC_ERR_INVALID_ARGUMENT = 1, /* null pointer, negative size, bad enum */
  DISC_ERR_SHAPE = 2,            /* inconsistent shapes between arguments */
  DISC_ERR_UNSUPPORTED_DTYPE = 3,
  DISC_ERR_ALIGNMENT = 4,        /* device pointers must be 16-byte aligned */
  DISC_ERR_OUT_OF_MEMORY = 5,    /* workspace allocation failed / too small */
  DISC_ERR_DEVICE = 6,           /* a HIP call failed */
  DISC_ERR_ADMISSION = 7,        /* serving: request can never be admitted */
  DISC_ERR_UNIMPLEMENTED = 8,
  DISC_ERR_LIMIT = 9             /* outside the limits listed above */
} disc_status;

typedef enum disc_dtype {
  DISC_F32 = 0,
  DISC_BF16 = 1,
  DISC_F8E4M3 = 2 /* OCP e4m3fn; tokens only, with a per-token FP32 scale */
} disc_dtype;

typedef enum disc_spatial { DISC_SPATIAL_EDT = 0, DISC_SPATIAL_AREA = 1 } disc_spatial;

/* Patch-token map of one frame (the ViT's intermediate-layer patch tokens,
 * Sec. III-C).  For DISC_F8E4M3 the token value is scale[p] * q. */
typedef struct disc_tokens {
  const void* data;    /* [gh][gw][c] */
  int32_t dtype;       /* disc_dtype */
  int32_t gh, gw, c;
  int32_t patch;       /* pixels per patch side */
  const float* scale;  /* [gh*gw] for DISC_F8E4M3, NULL otherwise */
} disc_tokens;

/* The frame's binary instance masks (Sec. III-A), bit-packed. */
typedef struct disc_masks {
  const uint64_t* bits; /* [m][h][ceil(w/64)] */
  int32_t m, h, w;
} disc_masks;

/* Projection into the embedding space, [c][e]; DISC_F32 or DISC_BF16. */
typedef struct disc_proj {
  const void* data;
  int32_t dtype;
  int32_t c, e;
} disc_proj;

/* Output of one frame. */
typedef struct disc_out {
  float* data;          /* [m][e] FP32 */
  int32_t m, e;
  int32_t* mask_status; /* optional [m]: 0 ok, 1 empty mask, 2 zero projection,
                           3 the frame's FP8 scales hold a NaN, infinite or
                           negative value (every mask of that frame) */
  float* pooled;        /* optional [m][c] FP32 weighted-mean features F */
  float* dbar;          /* optional [m]: the mask's mean distinctiveness, D of
                           Eq. (1) (with eps) averaged over the mask's pixels,
                           each pixel taking its patch's D; 0 for an empty mask
                           (the S_dist input of the view quality, Sec. III-C) */
  int32_t* area;        /* optional [m]: the mask's pixel count |M| */
} disc_out;

typedef struct disc_options {
  int32_t spatial;        /* disc_spatial, default DISC_SPATIAL_EDT */
  int32_t distinct;       /* 1 (default): weights include D of Eq. (1) */
  float eps;              /* Eq. (1) epsilon, default 1e-6 (cancels in F) */
  int32_t gemm_dtype;     /* pooling/projection operand type: DISC_F32 or
                             DISC_BF16; -1 (default) = DISC_F32 for FP32 tokens
                             and projection, DISC_BF16 otherwise.  FP32
                             accumulation in every case. */
  void* workspace;        /* optional caller-owned device workspace */
  size_t workspace_bytes; /* its size; see disc_workspace_bytes() */
  int32_t edt_layout;     /* distance-transform layout: -1 (default) and 2
                             the direct column search; 0 and 1 the lower-
                             envelope kernel with short (0) or longer (1)
                             bands.  Results are identical bit for bit in
                             every layout. */
  int32_t pool_tile;      /* channels per pooling workgroup in units of 64:
                             -1 (default) autotuned (the first call with a
                             new problem shape times every candidate shape
                             and keeps the fastest), or 1, 2 or 4 (4 and 2
                             only when they divide c / 64).  Results are
                             identical bit for bit for every shape. */
  int32_t pool_rows;      /* masks per pooling workgroup: -1 (default)
                             autotuned together with pool_tile, 64 or 128
                             (128 shares each token chunk between two mask
                             tiles; it runs with pool_tile 1 or 2). */
} disc_options;

/* Fill *o with the defaults listed above. */
void disc_options_default(disc_options* o);

/* Embed every mask of one frame with default options on the null stream. */
disc_status disc_embed_masks(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj,
                             disc_out* out);

/* Same with options (NULL = defaults) and a stream. */
disc_status disc_embed_masks_ex(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj,
                                disc_out* out, const disc_options* opts, void* stream);

/* A ragged batch: frame i has tokens[i], masks[i] and out[i]; frames may
 * differ in resolution, grid and mask count but share c, the token dtype and
 * proj.  Each frame keeps its own mean/D (statistics never mix frames). */
disc_status disc_embed_frames(const disc_tokens* tokens, const disc_masks* masks, int32_t n_frames,
                              const disc_proj* proj, disc_out* out, const disc_options* opts, void* stream);

/* Device workspace bytes disc_embed_frames needs for these arguments
 * (0 on invalid arguments). */
size_t disc_workspace_bytes(const disc_tokens* tokens, const disc_masks* masks, int32_t n_frames,
                            const disc_proj* proj, const disc_options* opts);

/* For callers that cannot allocate (code under hipGraph / stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): disc_embed_masks_ex
 * for one frame, with the same arguments and the same results bit for bit,
 * that allocates nothing.  Its workspace is a device array inside the library
 * (one per GPU, DISC_NOALLOC_SCRATCH_BYTES, held until the process ends)
 * instead of library-allocated or caller memory, and it enqueues no memset,
 * no copy and no event.  The pooling tile width comes from the autotuner's
 * stored choice or its size rule (this call never times candidates).
 *   opts->workspace must be NULL.  A frame whose workspace
 *   (disc_workspace_bytes for this one frame) exceeds the array fails with
 *   DISC_ERR_LIMIT before anything is enqueued.
 *   Every call on a GPU works in that GPU's one array and the next call
 *   overwrites it: calls that overlap on one GPU (several streams or threads)
 *   race and must be ordered by the caller.
 * Other errors as for disc_embed_masks_ex. */
#define DISC_NOALLOC_SCRATCH_BYTES (64u << 20)
disc_status disc_embed_masks_noalloc(const disc_tokens* tokens, const disc_masks* masks, const disc_proj* proj,
                                     disc_out* out, const disc_options* opts, void* stream);

/* Free the library-owned workspaces (synchronises the device first). */
disc_status disc_release_workspace(void);

/* ---- stage entry points (tests, ablations) ---- */

/* Exact squared EDT of each mask: e[m][h][w] int32 (0 off the mask). */
disc_status disc_edt_sq(const disc_masks* masks, int32_t* e, void* stream);

/* Per-patch weights w[m][gh*gw] FP32: s_p * D_p (D of Eq. 1 with opts->eps)
 * or s_p when opts->distinct == 0 (tokens may then be NULL; the grid is taken
 * from `patch`).  `patch` must equal tokens->patch when tokens is given. */
disc_status disc_patch_weights(const disc_tokens* tokens, const disc_masks* masks, int32_t patch,
                               const disc_options* opts, float* w, void* stream);

/* Eq. (1): mean[c], r[gh*gw] = ||f_p - mean||, D[gh*gw] = r/(mean(r)+eps).
 * Any output pointer may be NULL. */
disc_status disc_token_stats(const disc_tokens* tokens, float eps, float* mean, float* r, float* D,
                             void* stream);

/* Pooling + projection + normalisation with caller-given weights
 * w[m][gh*gw] FP32 (non-negative); rows summing to zero give status 1.
 * gemm_dtype as in disc_options. */
disc_status disc_pool_project(const disc_tokens* tokens, const float* w, int32_t m, const disc_proj* proj,
                              disc_out* out, int32_t gemm_dtype, void* stream);

/* Pack bool/uint8 masks u8[m][h][w] (non-zero = inside) into the bit layout. */
disc_status disc_pack_masks(const uint8_t* u8, int32_t m, int32_t h, int32_t w, uint64_t* bits, void* stream);

/* ---- open-vocabulary query (consumer of the embeddings) ---- */

/* For each of q text embeddings, the k instances whose embeddings are most
 * similar (arXiv 2603.03935, Sec. III-C: instances are retrieved by the cosine
 * similarity of their CLIP-space embedding with a text embedding).
 *   emb    [m][e] FP32 instance embeddings (e.g. the rows disc_embed_* wrote;
 *          they need not be normalised).
 *   text   [q][e] text embeddings, text_dtype DISC_F32 or DISC_BF16.
 *   sim    [q][m] FP32, written: sim[j][i] = cos(text_j, emb_i), 0 when either
 *          vector is zero (caller-owned; also the scratch of the ranking).
 *   scores [q][k] FP32 and idx [q][k] int32, written: per query the k best
 *          instances, higher similarity first, ties to the lower index;
 *          idx -1 and score -inf past m.
 * All pointers are device pointers, 16-byte aligned; e a multiple of 16 up
 * to 4096, 1 <= k <= 256, m <= 2^24.  Invalid arguments: nothing is
 * enqueued, DISC_ERR_* is returned.  Asynchronous on `stream`. */
disc_status disc_query_topk(const float* emb, int32_t m, const void* text, int32_t text_dtype, int32_t q, int32_t e,
                            int32_t k, float* sim, float* scores, int32_t* idx, void* stream);

/* Weighted similarity heat-map of text queries over one frame's patches
 * (arXiv 2603.03935, Sec. III-C, the feature-similarity figure: the dense
 * similarity of a text query with the patch features, weighted by the
 * distinctiveness map):
 *   heat[j][p] = D_p * cos(text_j, y_p),   y_p = f_p^T P,
 * f_p the patch token (as for disc_embed_masks: F32, BF16 or FP8 + scale),
 * P the projection [c][e], D_p of Eq. (1) with epsilon eps; 0 where text_j
 * or y_p is the zero vector.  |heat| <= D_p.
 *   text [q][e] (text_dtype DISC_F32 or DISC_BF16), heat [q][gh*gw] FP32
 *   written, patch-row-major.  FP32 arithmetic (tokens and P widened
 *   exactly), FP32 accumulation.
 * Device pointers, 16-byte aligned; 0 <= q <= 2^20 (0: no-op); eps >= 0.
 * Invalid arguments: nothing is enqueued, DISC_ERR_* is returned.
 * Asynchronous on `stream`. */
disc_status disc_query_heatmap(const disc_tokens* tokens, const disc_proj* proj, const void* text, int32_t text_dtype,
                               int32_t q, float eps, float* heat, void* stream);

/* ---- view quality and fusion (consumers of the embeddings) ---- */

/* View quality of each observation (arXiv 2603.03935, Sec. III-C, Eqs. 2-3):
 *   Q = S_size * S_angle * S_sem * S_dist
 *   S_size  = min(lambda * area / (img_h * img_w), 1)   (the paper: lambda = 3.3)
 *   S_angle = angle[i], or 1 when angle is NULL (see disc_angle_score)
 *   S_sem   = min(max(cos(emb_i, g), 0), 1), 0 when either vector is zero
 *   S_dist  = 0.5 + 0.5 * dbar[i]
 *   area [m] int32 and dbar [m] FP32 (e.g. what disc_embed_* wrote to
 *   disc_out.area / .dbar), emb [m][e] FP32 (the mask's embedding), g [e]
 *   FP32 (the frame's global image embedding), angle [m] FP32 or NULL.
 *   q [m] FP32, written; comp [m][4] FP32 or NULL, written with
 *   (S_size, S_angle, S_sem, S_dist).
 * Device pointers; emb and g 16-byte aligned; e a multiple of 4 up to 4096;
 * img_h, img_w >= 1; lambda > 0.  Invalid arguments: nothing is enqueued,
 * DISC_ERR_* is returned.  Asynchronous on `stream`. */
disc_status disc_view_quality(const int32_t* area, const float* dbar, const float* emb, const float* g,
                              const float* angle, int32_t m, int32_t e, int32_t img_h, int32_t img_w, float lambda,
                              float* q, float* comp, void* stream);

/* S_angle of Eq. (3): for detection i, the mean over its voxels v of
 * max(0, -r_v . n_v), r_v the unit viewing ray and n_v the unit surface
 * normal; 0 for a detection without voxels.
 *   rays, normals [nv][3] FP32; off [m + 1] int32 (device): the voxels of
 *   detection i are [off[i], off[i+1]) (indices clamped to [0, nv], an
 *   inverted range counts as empty).  angle [m] FP32, written.
 * Device pointers.  Asynchronous on `stream`. */
disc_status disc_angle_score(const float* rays, const float* normals, int32_t nv, const int32_t* off, int32_t m,
                             float* angle, void* stream);

/* Feature fusion (Sec. III-C): an instance's feature is replaced by an
 * observed feature of higher view quality.  Observations i < m target
 * instance ids[i] (skipped unless 0 <= ids[i] < n_map) with quality q[i] and
 * feature emb[i][e]; per instance the observation of the largest q above
 * map_q[t] replaces map_q[t] and map_emb[t] (the first such observation
 * among equal q), which is what taking the observations one by one in index
 * order gives.  Instances that no observation beats keep their row.
 *   ids [m] int32, q [m] FP32, emb [m][e] FP32, map_q [n_map] FP32 and
 *   map_emb [n_map][e] FP32 (updated in place), won [m] int32 or NULL
 *   (written: 1 where the observation entered the map).
 * Device pointers, emb/map_emb 16-byte aligned, e a multiple of 4 up to 4096,
 * n_map <= 2^28.  Asynchronous on `stream`; calls that update one map must
 * be ordered (one stream). */
disc_status disc_fuse(const int32_t* ids, const float* q, const float* emb, int32_t m, int32_t e, float* map_q,
                      float* map_emb, int32_t n_map, int32_t* won, void* stream);

/* ---- geometry (the mapping side of each segment, Sec. III-B) ---- */

/* Pinhole camera of a depth frame.  Pixel (x, y) (integer column and row)
 * with depth z maps to the camera point ((x - cx) z / fx, (y - cy) z / fy, z)
 * and the world point R p + t (R row-major camera-to-world rotation).
 * Depths that are not finite or lie outside [depth_min, depth_max] are
 * missing readings.  All arithmetic is single precision, each operation
 * rounded on its own in the order written (no fused multiply-add). */
typedef struct disc_camera {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float depth_min, depth_max;
} disc_camera;

/* Back-projection, pass 1: offsets [m + 1] (device int32) written with the
 * exclusive prefix sum of each mask's point count (pixels of the mask with a
 * valid depth and x, y multiples of stride); offsets[m] is the total.
 *   depth [h][w] FP32 metres (device), masks as for disc_embed_* (h, w the
 *   depth frame's), cam a host struct, 1 <= stride <= 64.
 * Asynchronous on `stream`. */
disc_status disc_backproject_count(const float* depth, const disc_masks* masks, const disc_camera* cam,
                                   int32_t stride, int32_t* offsets, void* stream);
/* Back-projection, pass 2: the world points of each mask, in row-major pixel
 * order, written to points [offsets[i] ...][3] FP32 (the caller reads
 * offsets[m] after pass 1 to size points).  Same arguments as pass 1. */
disc_status disc_backproject(const float* depth, const disc_masks* masks, const disc_camera* cam, int32_t stride,
                             const int32_t* offsets, float* points, void* stream);

/* DBSCAN noise removal (Sec. III-B: segment point clouds are filtered with
 * DBSCAN): within each segment, a point is a core point when at least
 * min_pts points (itself included) lie within distance eps (squared distance
 * <= eps^2 in single precision); keep[i] = 1 for core points and for points
 * within eps of a core point, 0 for the noise.
 *   points [n][3] FP32, offsets [m + 1] int32 (segment i = points
 *   [offsets[i], offsets[i+1]), offsets[m] = n), keep [n] int32 written.
 * n <= 2^23, m <= 65535, eps > 0, min_pts >= 1.  Asynchronous on `stream`. */
disc_status disc_dbscan_denoise(const float* points, const int32_t* offsets, int32_t m, int32_t n, float eps,
                                int32_t min_pts, int32_t* keep, void* stream);

/* Voxel sets (Sec. III-B: the filtered points are voxelised): voxel of a
 * point floor(p / voxel) per axis; per segment the distinct voxels of its
 * points with keep[i] != 0 (keep may be NULL: all points), listed in
 * lexicographic (x, y, z) order.
 *   voffsets [m + 1] int32 written (prefix sums of the voxel counts),
 *   voxels [n][3] int32 (capacity n rows; rows [voffsets[i], voffsets[i+1])
 *   written), status [m] int32 or NULL: 0 ok, 1 some point's voxel lies
 *   beyond +-32767 per axis (the point is left out).  Any number of voxels
 *   per segment (beyond 8192 the segment is sorted in chunks and merged by
 *   rank, within its workgroup).
 * n <= 2^23, m <= 65535, voxel > 0.  Asynchronous on `stream`. */
disc_status disc_voxelize(const float* points, const int32_t* offsets, const int32_t* keep, int32_t m, int32_t n,
                          float voxel, int32_t* voffsets, int32_t* voxels, int32_t* status, void* stream);

/* Exact voxel overlap (Sec. III-B: association by voxel intersection): for
 * each pair k, counts[k] = number of voxels shared by set pairs[k][0] of A
 * and set pairs[k][1] of B (0 for an index out of range).
 *   va [.][3] int32 with offsets oa [na + 1], vb / ob likewise, each set
 *   sorted lexicographically without repeats (as disc_voxelize writes them),
 *   coordinates within +-2^20; pairs [np][2] int32; counts [np] int32.
 * Asynchronous on `stream`. */
disc_status disc_voxel_overlap(const int32_t* va, const int32_t* oa, int32_t na, const int32_t* vb,
                               const int32_t* ob, int32_t nb, const int32_t* pairs, int32_t np, int32_t* counts,
                               void* stream);

/* ---- serving ---- */

/* A continuous-batching request loop on one device (the view-quality
 * pipeline of Sec. III-C embeds every frame's masks as frames arrive).
 * Requests (one frame each: device-resident tokens and masks, caller-owned
 * outputs that must stay valid until the ticket completes) enter a FIFO.
 * `lanes` worker threads each own a stream, a resident workspace sized for the
 * capacity below and a pinned staging buffer; a free lane packs the waiting
 * requests (in arrival order, up to max_frames frames / max_masks masks and
 * while fewer than max_slots requests are in flight) into one batch, runs the
 * kernel set (replaying a captured hipGraph when use_graph is set), waits for
 * it and completes the tickets.  Requests arriving while other batches run
 * are admitted as soon as a lane and slots free up, so batches on different
 * lanes overlap on the device.  Every result equals the frame processed
 * alone (the kernels never mix masks or frames).
 *
 * Admission: a request that can never fit (more masks than max_masks, a frame
 * larger than max_h x max_w, a patch smaller than min_patch, other dtype or
 * channel count) is rejected at submit with DISC_ERR_ADMISSION; one waiting
 * longer than admission_timeout_ms (0 = no limit) completes with
 * DISC_ERR_ADMISSION.  Creation fails with DISC_ERR_OUT_OF_MEMORY when
 * mem_budget cannot hold one lane's workspace; otherwise the number of lanes
 * is reduced to what the budget holds.
 * dry_run (host-only testing of the admission logic): no device work at all
 * and outputs untouched; 1 = batches complete at once, n > 1 = each batch
 * takes n microseconds.
 * fault_batch >= 0 makes that batch (0-based, in launch order) complete with
 * DISC_ERR_DEVICE without running, to test failure handling. */
typedef struct disc_server disc_server;

typedef struct disc_server_config {
  disc_proj proj;          /* shared projection (device memory; outlives the server) */
  int32_t tok_dtype;       /* token dtype of every request */
  int32_t c;               /* token channels of every request */
  int32_t max_frames;      /* batch capacity: frames */
  int32_t max_masks;       /* batch capacity: masks (sum over the batch) */
  int32_t max_h, max_w;    /* largest frame accepted */
  int32_t min_patch;       /* smallest patch size accepted */
  int32_t max_slots;       /* requests in flight (admitted, not completed), at most */
  int32_t lanes;           /* concurrent batches, 1..8 */
  size_t mem_budget;       /* device bytes for the lanes' workspaces */
  int32_t use_graph;       /* 1: capture each lane's kernel set once and replay it */
  int32_t dry_run;         /* 0 off; 1 host-only; n > 1 host-only, n us per batch */
  int32_t fault_batch;     /* -1: off; else this batch completes with DISC_ERR_DEVICE */
  double admission_timeout_ms;
  disc_options opts;       /* spatial / distinct / eps / gemm_dtype (workspace fields ignored) */
} disc_server_config;

typedef struct disc_server_stats {
  uint64_t submitted, completed, failed, rejected, batches;
  double mean_batch_frames;
  double p50_ms, p99_ms, max_ms, mean_ms; /* submit -> completion of successful requests */
  int32_t lanes;                          /* lanes actually running */
  size_t lane_workspace_bytes;
} disc_server_stats;

/* Defaults: lanes 2, max_frames 16, max_masks 1024, 720x1280 frames, patch
 * >= 14, 64 slots, 4 GiB budget, graphs on, no dry run, no fault. */
void disc_server_config_default(disc_server_config* cfg);
disc_status disc_server_create(const disc_server_config* cfg, disc_server** out);
/* Validate and enqueue one frame; *ticket identifies it. */
disc_status disc_server_submit(disc_server* s, const disc_tokens* tokens, const disc_masks* masks, disc_out* out,
                               uint64_t* ticket);
/* *done = 1 once the ticket completed; *result is then its status.  A ticket
 * whose completion poll or wait has reported is forgotten (a later poll or
 * wait of it fails with DISC_ERR_INVALID_ARGUMENT), so the server's memory
 * does not grow with the number of requests served. */
disc_status disc_server_poll(disc_server* s, uint64_t ticket, int32_t* done, int32_t* result);
/* Block until the ticket completed; *result = its status. */
disc_status disc_server_wait(disc_server* s, uint64_t ticket, int32_t* result);
/* Block until every submitted request completed. */
disc_status disc_server_drain(disc_server* s);
/* Counts since the server started or since the last reset; p50/p99/max/mean
 * over the latencies of the last 2^20 successful requests in that span. */
disc_status disc_server_get_stats(disc_server* s, disc_server_stats* st);
/* Restart the counts and latency samples from zero (e.g. after a warm-up;
 * requests still in flight are counted when they complete). */
disc_status disc_server_reset_stats(disc_server* s);
/* Drain, stop the lanes and free the server's memory. */
void disc_server_destroy(disc_server* s);

/* ---- profiling ---- */

/* Per-stage device timing with HIP events recorded on the caller's stream
 * around each stage of disc_embed_frames (and the calls built on it): stages
 * 0 scan, 1 token_stats, 2 edt, 3 weights, 4 pool, 5 proj.
 * Off by default; enabling it adds two event records per timed stage. */
void disc_trace_enable(int32_t on);
/* Which stages are timed while tracing is on: bit s for stage s (default:
 * all).  Timing one stage keeps the other stages free of event records. */
void disc_trace_select(uint32_t stage_mask);
/* Wait for pending events and zero the accumulated totals. */
void disc_trace_reset(void);
/* Total milliseconds and number of timed launches of a stage since the last
 * reset (waits for pending events); -1 for an unknown stage. */
int32_t disc_trace_read(int32_t stage, double* total_ms, int64_t* count);
/* Name of a stage, or NULL. */
const char* disc_trace_stage_name(int32_t stage);

/* ---- misc ---- */

/* Text of the last error on the calling thread; valid until its next call. */
const char* disc_last_error(void);

/* DISC_ABI_VERSION of the loaded library. */
int32_t disc_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DISC_H */
