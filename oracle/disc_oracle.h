/*
 * disc_oracle.h -- plain FP64 CPU oracle for DISC's mask-aligned,
 * distance-weighted feature extraction (arXiv 2603.03935, Sec. III-C).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this
 * library: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the
 * HIP library; the two only see the same seeded inputs.
 *
 * Everything is single-threaded, double precision (integers for the distance
 * transform), and deliberately simple.  Each function names the passage of the
 * paper it follows.  Where the paper is silent the reading taken is stated
 * next to the function; the readings are:
 *
 *   R-EDT   squared Euclidean distance between pixel centres from a mask pixel
 *           to the nearest pixel that is not in the mask, with every pixel
 *           outside the frame counted as not in the mask; 0 off the mask.
 *   R-PATCH pixel (y, x) belongs to patch (floor(y/P), floor(x/P)); the grid
 *           is ceil(H/P) x ceil(W/P), so the last patch row/column may be
 *           partial.
 *   R-SPAT  spatial weight of patch p for mask m is the sum over the mask's
 *           pixels in p of sqrt(EDT) (mode 0, default) or their count (mode 1).
 *   R-WGT   per-patch weight = spatial weight x distinctiveness D (Eq. 1)
 *           when `distinct` is set, else the spatial weight alone.
 *   R-POOL  the instance feature is the weighted mean of the patch tokens.
 *   R-ZERO  empty mask -> zero row, status 1; all weights zero with D on ->
 *           fall back to the spatial weights; zero projected vector -> zero
 *           row, status 2.
 *   R-PROJ  y = F^T P with no bias, then y / ||y||_2.
 *   R-QUERY open-vocabulary query (Sec. III-C, the figure of the weighted
 *           similarity heat-map; Sec. IV): the similarity of a text
 *           embedding t and an instance embedding y is cos(t, y) (0 when
 *           either is the zero vector); a query returns the k instances of
 *           highest similarity, higher first, ties to the lower index.
 *   R-HEAT  weighted similarity heat-map of a text query (Sec. III-C, the
 *           feature-similarity figure): per patch p, D_p of Eq. (1) times
 *           cos(t, y_p) with y_p = f_p^T P the patch token projected into the
 *           embedding space (0 when either vector is zero).
 *   R-Q     view quality (Sec. III-C, Eqs. 2-3): Q = S_size S_angle S_sem
 *           S_dist with S_size = min(lambda |M| / (H W), 1), lambda = 3.3;
 *           S_dist = 0.5 + 0.5 Dbar, Dbar = D of Eq. (1) averaged over the
 *           mask's pixels (each pixel takes its patch's D; 0 for an empty
 *           mask); S_sem = min(max(cos(y, g), 0), 1) with y the mask's
 *           embedding and g the frame's global image embedding; S_angle =
 *           mean over the detection's voxels of max(0, -r.n) (0 without
 *           voxels), or a caller-given value.
 *   R-FUSE  an observation replaces its instance's feature when its Q is
 *           strictly higher than the instance's; observations are taken in
 *           index order (so among equal Q the first wins).
 *
 * Parity status: every function below is pinned by tests that do not use the
 * oracle itself (brute force, closed forms, a library routine, invariants).
 * Whether R-EDT/R-SPAT/R-WGT is what the authors ran is NOT pinnable: the paper
 * ships no code and prints no per-mask values (parity to the authors'
 * implementation is unpinned).
 *
 * Layouts (all host memory, row-major, caller-owned):
 *   masks  bits[m][h][wq], wq = ceil(w/64); bit i of word k is pixel 64k+i of
 *          that row; bits at columns >= w are ignored.
 *   tokens f[G][C] doubles, G = gh*gw, patch-row-major.
 *   proj   P[C][E] doubles.
 * Return value: 0 on success, -1 on a bad argument (nothing written).
 */
#ifndef DISC_ORACLE_H
#define DISC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Input decoding (exact).  bf16 -> double; OCP e4m3fn code -> double (NaN for
 * the two NaN codes); FP8 tokens with a per-token scale: f = scale[p] * q. */
void disc_oracle_decode_bf16(const uint16_t* in, int64_t n, double* out);
double disc_oracle_e4m3_value(uint8_t code);
void disc_oracle_decode_e4m3(const uint8_t* q, const float* scale, int64_t G, int64_t C, double* out);
void disc_oracle_decode_f32(const float* in, int64_t n, double* out);

/* R-EDT for one mask: e[h][w] (int32). */
int disc_oracle_edt_sq(const uint64_t* bits, int32_t h, int32_t w, int32_t* e);
/* Same for m masks: e[m][h][w]. */
int disc_oracle_edt_sq_batch(const uint64_t* bits, int32_t m, int32_t h, int32_t w, int32_t* e);

/* R-SPAT: s[m][G], G = gh*gw.  spatial: 0 = EDT, 1 = AREA. */
int disc_oracle_spatial_weights(const uint64_t* bits, int32_t m, int32_t h, int32_t w,
                                int32_t patch, int32_t gh, int32_t gw, int32_t spatial, double* s);

/* Eq. (1): mean[C], r[G] = ||f_p - mean||, D[G] = r / (mean(r) + eps). */
int disc_oracle_token_stats(const double* f, int32_t G, int32_t C, double eps,
                            double* mean, double* r, double* D);

/* The whole path for one frame.  out[m][E], status[m]; optional (may be NULL):
 * pooled[m][C] (the weighted-mean feature), Z[m] (sum of the weights used),
 * wts[m][G] (the weights used). */
int disc_oracle_embed(const double* f, int32_t gh, int32_t gw, int32_t C, int32_t patch,
                      const uint64_t* bits, int32_t m, int32_t h, int32_t w,
                      const double* P, int32_t E, int32_t spatial, int32_t distinct, double eps,
                      double* out, int32_t* status, double* pooled, double* Z, double* wts);

/* Pooling + projection + normalisation with caller-given weights wts[m][G].
 * A row whose weights sum to zero gives a zero row and status 1. */
int disc_oracle_pool_project(const double* f, int32_t G, int32_t C, const double* wts, int32_t m,
                             const double* P, int32_t E, double* out, int32_t* status, double* pooled);

/* R-QUERY: sim[q][m] (may be NULL) = cos(text_j, emb_i); for each query j the
 * k best instances: idx[j][r], scores[j][r], r = 0..k-1 (idx -1 and score
 * -inf past m).  emb[m][e], text[q][e]. */
int disc_oracle_query_topk(const double* emb, int32_t m, const double* text, int32_t q, int32_t e, int32_t k,
                           double* sim, double* scores, int32_t* idx);

/* R-HEAT: heat[q][G] = D_p cos(text_j, f_p^T P) for tokens f[G][C],
 * projection P[C][E], text[q][E]; D with epsilon eps (Eq. 1). */
int disc_oracle_query_heatmap(const double* f, int32_t G, int32_t C, const double* P, int32_t E,
                              const double* text, int32_t q, double eps, double* heat);

/* R-Q: Dbar[m] and area |M| [m] of each mask, given D[G] of the frame. */
int disc_oracle_mask_dbar(const uint64_t* bits, int32_t m, int32_t h, int32_t w, int32_t patch, int32_t gh,
                          int32_t gw, const double* D, double* dbar, int32_t* area);
/* R-Q: S_angle[m] from voxel view rays and normals r[nv][3], n[nv][3], the
 * voxels of mask i being [off[i], off[i+1]). */
int disc_oracle_angle_score(const double* rays, const double* normals, const int32_t* off, int32_t m,
                            double* angle);
/* R-Q: Q[m] and the factors comp[m][4] = (S_size, S_angle, S_sem, S_dist)
 * (comp may be NULL).  angle may be NULL (S_angle = 1). emb[m][e], g[e]. */
int disc_oracle_view_quality(const int32_t* area, const double* dbar, const double* emb, const double* g,
                             const double* angle, int32_t m, int32_t e, int32_t H, int32_t W, double lambda,
                             double* Q, double* comp);
/* R-FUSE: update map_q[n_map], map_emb[n_map][e] in place from observations
 * (ids[m] in [0, n_map), or < 0 to skip; q[m]; emb[m][e]); won[m] (may be
 * NULL) = 1 where the observation ends up in the map. */
int disc_oracle_fuse(const int32_t* ids, const double* q, const double* emb, int32_t m, int32_t e,
                     double* map_q, double* map_emb, int32_t n_map, int32_t* won);

#ifdef __cplusplus
}
#endif

#endif /* DISC_ORACLE_H */
