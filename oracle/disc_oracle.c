/*
 * disc_oracle.c -- FP64 reference for DISC's single-pass, distance-weighted,
 * mask-aligned feature extraction (arXiv 2603.03935, Sec. III-C; the
 * "distance-weighted" extraction is named in the abstract and Sec. V).
 *
 * TEST INFRASTRUCTURE ONLY (see disc_oracle.h).  Single-threaded, plain C99,
 * no fast-math.  The readings R-* are listed in the header.
 */
#include "disc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Input decoding                                                       */
/* ------------------------------------------------------------------ */

void disc_oracle_decode_bf16(const uint16_t* in, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    uint32_t u = ((uint32_t)in[i]) << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    out[i] = (double)f;
  }
}

void disc_oracle_decode_f32(const float* in, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (double)in[i];
}

/* OCP 8-bit floating point, E4M3 "fn" variant: 1 sign bit, 4 exponent bits
 * (bias 7), 3 mantissa bits, no infinities, S.1111.111 is NaN. */
double disc_oracle_e4m3_value(uint8_t code) {
  int sign = (code >> 7) & 1;
  int ex = (code >> 3) & 15;
  int man = code & 7;
  double v;
  if (ex == 15 && man == 7) return NAN;
  if (ex == 0)
    v = ldexp((double)man, -9); /* subnormal: man/8 * 2^(1-7) */
  else
    v = ldexp(1.0 + man / 8.0, ex - 7);
  return sign ? -v : v;
}

void disc_oracle_decode_e4m3(const uint8_t* q, const float* scale, int64_t G, int64_t C, double* out) {
  for (int64_t p = 0; p < G; ++p)
    for (int64_t c = 0; c < C; ++c)
      out[p * C + c] = (double)scale[p] * disc_oracle_e4m3_value(q[p * C + c]);
}

/* ------------------------------------------------------------------ */
/* R-EDT: exact squared Euclidean distance transform                    */
/* ------------------------------------------------------------------ */

static int mask_bit(const uint64_t* bits, int32_t wq, int32_t w, int32_t y, int32_t x) {
  if (x < 0 || x >= w) return 0;
  return (int)((bits[(int64_t)y * wq + (x >> 6)] >> (x & 63)) & 1u);
}

/* One-dimensional squared distance transform of a sampled function f over
 * n samples: out[q] = min_v (q - v)^2 + f[v].  Felzenszwalb & Huttenlocher's
 * lower envelope of parabolas; the intersection abscissae are rationals with
 * small denominators, exactly ordered in double precision. */
static void dt1d(const int64_t* f, int n, int64_t* out, int* v, double* z) {
  int k = 0;
  v[0] = 0;
  z[0] = -HUGE_VAL; /* z[k]: left end of the interval where parabola v[k] is lowest */
  z[1] = HUGE_VAL;
  for (int q = 1; q < n; ++q) {
    double s;
    for (;;) {
      const int p = v[k];
      s = ((double)(f[q] + (int64_t)q * q) - (double)(f[p] + (int64_t)p * p)) / (double)(2 * q - 2 * p);
      if (s > z[k]) break; /* z[0] = -inf ends the loop at k = 0 */
      --k;
    }
    ++k;
    v[k] = q;
    z[k] = s;
    z[k + 1] = HUGE_VAL;
  }
  k = 0;
  for (int q = 0; q < n; ++q) {
    while (z[k + 1] < (double)q) ++k;
    const int64_t d = (int64_t)(q - v[k]);
    out[q] = d * d + f[v[k]];
  }
}

/* R-EDT on the frame padded by a one-pixel background ring, so every mask
 * pixel has a finite distance.  Row pass (two linear sweeps) then column pass
 * (lower envelope) -- the standard separable exact EDT, run over the whole
 * frame for every mask. */
int disc_oracle_edt_sq(const uint64_t* bits, int32_t h, int32_t w, int32_t* e) {
  if (!bits || !e || h <= 0 || w <= 0) return -1;
  const int32_t wq = (w + 63) / 64;
  const int H = h + 2, W = w + 2;
  int64_t* g = (int64_t*)malloc(sizeof(int64_t) * (size_t)H * W);
  int64_t* col = (int64_t*)malloc(sizeof(int64_t) * (size_t)H);
  int64_t* res = (int64_t*)malloc(sizeof(int64_t) * (size_t)H);
  int* v = (int*)malloc(sizeof(int) * (size_t)H);
  double* z = (double*)malloc(sizeof(double) * (size_t)(H + 1));
  if (!g || !col || !res || !v || !z) {
    free(g); free(col); free(res); free(v); free(z);
    return -1;
  }
  /* Row pass: horizontal distance to the nearest background pixel. */
  for (int Y = 0; Y < H; ++Y) {
    int64_t* row = g + (int64_t)Y * W;
    for (int X = 0; X < W; ++X) {
      int inside = (Y >= 1 && Y <= h && X >= 1 && X <= w) ? mask_bit(bits, wq, w, Y - 1, X - 1) : 0;
      if (!inside)
        row[X] = 0;
      else
        row[X] = row[X - 1] + 1; /* X >= 1 here because X = 0 is padding */
    }
    for (int X = W - 2; X >= 0; --X)
      if (row[X + 1] + 1 < row[X]) row[X] = row[X + 1] + 1;
  }
  /* Column pass on squared horizontal distances. */
  for (int X = 1; X <= w; ++X) {
    for (int Y = 0; Y < H; ++Y) {
      int64_t gv = g[(int64_t)Y * W + X];
      col[Y] = gv * gv;
    }
    dt1d(col, H, res, v, z);
    for (int Y = 1; Y <= h; ++Y) e[(int64_t)(Y - 1) * w + (X - 1)] = (int32_t)res[Y];
  }
  free(g); free(col); free(res); free(v); free(z);
  return 0;
}

int disc_oracle_edt_sq_batch(const uint64_t* bits, int32_t m, int32_t h, int32_t w, int32_t* e) {
  if (m < 0 || h <= 0 || w <= 0) return -1;
  const int64_t wq = (w + 63) / 64;
  for (int32_t i = 0; i < m; ++i) {
    int rc = disc_oracle_edt_sq(bits + (int64_t)i * h * wq, h, w, e + (int64_t)i * h * w);
    if (rc) return rc;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* R-SPAT / R-PATCH: per-patch spatial weights                          */
/* ------------------------------------------------------------------ */

int disc_oracle_spatial_weights(const uint64_t* bits, int32_t m, int32_t h, int32_t w,
                                int32_t patch, int32_t gh, int32_t gw, int32_t spatial, double* s) {
  if (!bits || !s || m < 0 || h <= 0 || w <= 0 || patch <= 0) return -1;
  if (gh != (h + patch - 1) / patch || gw != (w + patch - 1) / patch) return -1;
  if (spatial != 0 && spatial != 1) return -1;
  const int64_t wq = (w + 63) / 64;
  const int64_t G = (int64_t)gh * gw;
  int32_t* e = (int32_t*)malloc(sizeof(int32_t) * (size_t)h * w);
  if (!e) return -1;
  for (int32_t i = 0; i < m; ++i) {
    const uint64_t* mb = bits + (int64_t)i * h * wq;
    double* si = s + (int64_t)i * G;
    for (int64_t p = 0; p < G; ++p) si[p] = 0.0;
    if (spatial == 0) disc_oracle_edt_sq(mb, h, w, e);
    for (int32_t y = 0; y < h; ++y)
      for (int32_t x = 0; x < w; ++x) {
        if (!mask_bit(mb, (int32_t)wq, w, y, x)) continue;
        int64_t p = (int64_t)(y / patch) * gw + (x / patch);
        si[p] += (spatial == 0) ? sqrt((double)e[(int64_t)y * w + x]) : 1.0;
      }
  }
  free(e);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. (1): distinctiveness map                                         */
/* ------------------------------------------------------------------ */

int disc_oracle_token_stats(const double* f, int32_t G, int32_t C, double eps,
                            double* mean, double* r, double* D) {
  if (!f || G <= 0 || C <= 0) return -1;
  double* mu = (double*)calloc((size_t)C, sizeof(double));
  double* rr = (double*)malloc(sizeof(double) * (size_t)G);
  if (!mu || !rr) {
    free(mu); free(rr);
    return -1;
  }
  /* spatial mean of all patch features */
  for (int32_t p = 0; p < G; ++p)
    for (int32_t c = 0; c < C; ++c) mu[c] += f[(int64_t)p * C + c];
  for (int32_t c = 0; c < C; ++c) mu[c] /= (double)G;
  /* residual norms and their mean over the grid */
  double rbar = 0.0;
  for (int32_t p = 0; p < G; ++p) {
    double acc = 0.0;
    for (int32_t c = 0; c < C; ++c) {
      double d = f[(int64_t)p * C + c] - mu[c];
      acc += d * d;
    }
    rr[p] = sqrt(acc);
    rbar += rr[p];
  }
  rbar /= (double)G;
  if (mean)
    for (int32_t c = 0; c < C; ++c) mean[c] = mu[c];
  if (r)
    for (int32_t p = 0; p < G; ++p) r[p] = rr[p];
  if (D)
    for (int32_t p = 0; p < G; ++p) D[p] = rr[p] / (rbar + eps);
  free(mu);
  free(rr);
  return 0;
}

/* ------------------------------------------------------------------ */
/* R-POOL / R-PROJ: pooling, projection, normalisation                  */
/* ------------------------------------------------------------------ */

/* One row: F = (1/Z) sum_p w_p f_p, y = F^T P, out = y/||y||. */
static int32_t pool_project_row(const double* f, int32_t G, int32_t C, const double* wrow, double Z,
                                const double* P, int32_t E, double* F, double* y, double* out) {
  for (int32_t c = 0; c < C; ++c) F[c] = 0.0;
  for (int32_t p = 0; p < G; ++p) {
    double wp = wrow[p];
    if (wp == 0.0) continue;
    const double* fp = f + (int64_t)p * C;
    for (int32_t c = 0; c < C; ++c) F[c] += wp * fp[c];
  }
  for (int32_t c = 0; c < C; ++c) F[c] /= Z;
  for (int32_t j = 0; j < E; ++j) y[j] = 0.0;
  for (int32_t c = 0; c < C; ++c) {
    const double* Pc = P + (int64_t)c * E;
    for (int32_t j = 0; j < E; ++j) y[j] += F[c] * Pc[j];
  }
  double nn = 0.0;
  for (int32_t j = 0; j < E; ++j) nn += y[j] * y[j];
  nn = sqrt(nn);
  if (nn == 0.0) {
    for (int32_t j = 0; j < E; ++j) out[j] = 0.0;
    return 2;
  }
  for (int32_t j = 0; j < E; ++j) out[j] = y[j] / nn;
  return 0;
}

int disc_oracle_pool_project(const double* f, int32_t G, int32_t C, const double* wts, int32_t m,
                             const double* P, int32_t E, double* out, int32_t* status, double* pooled) {
  if (!f || !wts || !P || !out || G <= 0 || C <= 0 || E <= 0 || m < 0) return -1;
  double* F = (double*)malloc(sizeof(double) * (size_t)C);
  double* y = (double*)malloc(sizeof(double) * (size_t)E);
  if (!F || !y) {
    free(F); free(y);
    return -1;
  }
  for (int32_t i = 0; i < m; ++i) {
    const double* wr = wts + (int64_t)i * G;
    double Z = 0.0;
    for (int32_t p = 0; p < G; ++p) Z += wr[p];
    int32_t st;
    if (Z == 0.0) {
      for (int32_t j = 0; j < E; ++j) out[(int64_t)i * E + j] = 0.0;
      for (int32_t c = 0; c < C; ++c) F[c] = 0.0;
      st = 1;
    } else {
      st = pool_project_row(f, G, C, wr, Z, P, E, F, y, out + (int64_t)i * E);
    }
    if (status) status[i] = st;
    if (pooled)
      for (int32_t c = 0; c < C; ++c) pooled[(int64_t)i * C + c] = F[c];
  }
  free(F);
  free(y);
  return 0;
}

/* ------------------------------------------------------------------ */
/* The whole path for one frame                                         */
/* ------------------------------------------------------------------ */

int disc_oracle_embed(const double* f, int32_t gh, int32_t gw, int32_t C, int32_t patch,
                      const uint64_t* bits, int32_t m, int32_t h, int32_t w,
                      const double* P, int32_t E, int32_t spatial, int32_t distinct, double eps,
                      double* out, int32_t* status, double* pooled, double* Zout, double* wts) {
  if (!f || !bits || !P || !out || gh <= 0 || gw <= 0 || C <= 0 || E <= 0 || m < 0) return -1;
  if (gh != (h + patch - 1) / patch || gw != (w + patch - 1) / patch) return -1;
  const int32_t G = gh * gw;
  double* s = (double*)malloc(sizeof(double) * (size_t)m * G + 1);
  double* D = (double*)malloc(sizeof(double) * (size_t)G);
  double* wrow = (double*)malloc(sizeof(double) * (size_t)G);
  double* F = (double*)malloc(sizeof(double) * (size_t)C);
  double* y = (double*)malloc(sizeof(double) * (size_t)E);
  int rc = -1;
  if (!s || !D || !wrow || !F || !y) goto done;
  if (disc_oracle_spatial_weights(bits, m, h, w, patch, gh, gw, spatial, s)) goto done;
  if (disc_oracle_token_stats(f, G, C, eps, NULL, NULL, D)) goto done;
  for (int32_t i = 0; i < m; ++i) {
    const double* si = s + (int64_t)i * G;
    double S = 0.0, Z = 0.0;
    for (int32_t p = 0; p < G; ++p) S += si[p];
    for (int32_t p = 0; p < G; ++p) {
      wrow[p] = distinct ? si[p] * D[p] : si[p];
      Z += wrow[p];
    }
    int32_t st;
    if (S == 0.0) { /* empty mask */
      for (int32_t p = 0; p < G; ++p) wrow[p] = 0.0;
      Z = 0.0;
      for (int32_t j = 0; j < E; ++j) out[(int64_t)i * E + j] = 0.0;
      for (int32_t c = 0; c < C; ++c) F[c] = 0.0;
      st = 1;
    } else {
      if (Z == 0.0) { /* every touched patch has zero distinctiveness */
        for (int32_t p = 0; p < G; ++p) wrow[p] = si[p];
        Z = S;
      }
      st = pool_project_row(f, G, C, wrow, Z, P, E, F, y, out + (int64_t)i * E);
    }
    if (status) status[i] = st;
    if (Zout) Zout[i] = Z;
    if (pooled)
      for (int32_t c = 0; c < C; ++c) pooled[(int64_t)i * C + c] = F[c];
    if (wts)
      for (int32_t p = 0; p < G; ++p) wts[(int64_t)i * G + p] = wrow[p];
  }
  rc = 0;
done:
  free(s); free(D); free(wrow); free(F); free(y);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Open-vocabulary query (R-QUERY)                                      */
/* ------------------------------------------------------------------ */

static double norm2(const double* v, int32_t n) {
  double a = 0.0;
  for (int32_t i = 0; i < n; ++i) a += v[i] * v[i];
  return sqrt(a);
}

int disc_oracle_query_topk(const double* emb, int32_t m, const double* text, int32_t q, int32_t e, int32_t k,
                           double* sim, double* scores, int32_t* idx) {
  if (!emb || !text || !scores || !idx || m < 0 || q < 0 || e <= 0 || k <= 0) return -1;
  double* row = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  char* used = (char*)malloc((size_t)(m > 0 ? m : 1));
  if (!row || !used) {
    free(row); free(used);
    return -1;
  }
  for (int32_t j = 0; j < q; ++j) {
    const double* t = text + (int64_t)j * e;
    const double nt = norm2(t, e);
    for (int32_t i = 0; i < m; ++i) {
      const double* y = emb + (int64_t)i * e;
      const double ny = norm2(y, e);
      double d = 0.0;
      for (int32_t c = 0; c < e; ++c) d += t[c] * y[c];
      row[i] = (nt > 0.0 && ny > 0.0) ? d / (nt * ny) : 0.0;
      used[i] = 0;
      if (sim) sim[(int64_t)j * m + i] = row[i];
    }
    /* k passes of "best remaining": higher score first, then lower index */
    for (int32_t r = 0; r < k; ++r) {
      int32_t best = -1;
      for (int32_t i = 0; i < m; ++i)
        if (!used[i] && (best < 0 || row[i] > row[best])) best = i;
      idx[(int64_t)j * k + r] = best;
      scores[(int64_t)j * k + r] = best >= 0 ? row[best] : -INFINITY;
      if (best >= 0) used[best] = 1;
    }
  }
  free(row);
  free(used);
  return 0;
}

/* R-HEAT: weighted dense similarity of one text query with every patch
 * (Sec. III-C, the feature-similarity figure): the patch token projected into
 * the embedding space, y_p = f_p^T P, compared with t_j by cosine similarity
 * and weighted by the patch's distinctiveness D_p of Eq. (1). */
int disc_oracle_query_heatmap(const double* f, int32_t G, int32_t C, const double* P, int32_t E,
                              const double* text, int32_t q, double eps, double* heat) {
  if (!f || !P || !text || !heat || G <= 0 || C <= 0 || E <= 0 || q < 0) return -1;
  double* D = (double*)malloc(sizeof(double) * (size_t)G);
  double* y = (double*)malloc(sizeof(double) * (size_t)E);
  if (!D || !y) {
    free(D); free(y);
    return -1;
  }
  if (disc_oracle_token_stats(f, G, C, eps, NULL, NULL, D)) {
    free(D); free(y);
    return -1;
  }
  for (int32_t p = 0; p < G; ++p) {
    /* y_p = f_p^T P */
    for (int32_t k = 0; k < E; ++k) y[k] = 0.0;
    for (int32_t c = 0; c < C; ++c) {
      const double fc = f[(int64_t)p * C + c];
      const double* Pc = P + (int64_t)c * E;
      for (int32_t k = 0; k < E; ++k) y[k] += fc * Pc[k];
    }
    const double ny = norm2(y, E);
    for (int32_t j = 0; j < q; ++j) {
      const double* t = text + (int64_t)j * E;
      const double nt = norm2(t, E);
      double d = 0.0;
      for (int32_t k = 0; k < E; ++k) d += t[k] * y[k];
      heat[(int64_t)j * G + p] = (nt > 0.0 && ny > 0.0) ? D[p] * (d / (nt * ny)) : 0.0;
    }
  }
  free(D);
  free(y);
  return 0;
}

/* ------------------------------------------------------------------ */
/* View quality and fusion (R-Q, R-FUSE)                                */
/* ------------------------------------------------------------------ */

int disc_oracle_mask_dbar(const uint64_t* bits, int32_t m, int32_t h, int32_t w, int32_t patch, int32_t gh,
                          int32_t gw, const double* D, double* dbar, int32_t* area) {
  if (!bits || !D || !dbar || !area || m < 0 || h <= 0 || w <= 0 || patch <= 0) return -1;
  if (gh != (h + patch - 1) / patch || gw != (w + patch - 1) / patch) return -1;
  const int32_t wq = (w + 63) / 64;
  for (int32_t i = 0; i < m; ++i) {
    const uint64_t* mb = bits + (int64_t)i * h * wq;
    double acc = 0.0;
    int32_t cnt = 0;
    for (int32_t y = 0; y < h; ++y)
      for (int32_t x = 0; x < w; ++x)
        if ((mb[(int64_t)y * wq + x / 64] >> (x % 64)) & 1u) {
          acc += D[(int64_t)(y / patch) * gw + (x / patch)];
          ++cnt;
        }
    area[i] = cnt;
    dbar[i] = cnt > 0 ? acc / (double)cnt : 0.0;
  }
  return 0;
}

int disc_oracle_angle_score(const double* rays, const double* normals, const int32_t* off, int32_t m,
                            double* angle) {
  if (!off || !angle || m < 0) return -1;
  for (int32_t i = 0; i < m; ++i) {
    const int32_t a = off[i], b = off[i + 1];
    if (b < a) return -1;
    double s = 0.0;
    for (int32_t v = a; v < b; ++v) {
      const double* r = rays + (int64_t)3 * v;
      const double* n = normals + (int64_t)3 * v;
      const double c = -(r[0] * n[0] + r[1] * n[1] + r[2] * n[2]);
      s += c > 0.0 ? c : 0.0;
    }
    angle[i] = b > a ? s / (double)(b - a) : 0.0;
  }
  return 0;
}

int disc_oracle_view_quality(const int32_t* area, const double* dbar, const double* emb, const double* g,
                             const double* angle, int32_t m, int32_t e, int32_t H, int32_t W, double lambda,
                             double* Q, double* comp) {
  if (!area || !dbar || !emb || !g || !Q || m < 0 || e <= 0 || H <= 0 || W <= 0) return -1;
  const double ng = norm2(g, e);
  for (int32_t i = 0; i < m; ++i) {
    const double* y = emb + (int64_t)i * e;
    double size = lambda * (double)area[i] / ((double)H * (double)W);
    if (size > 1.0) size = 1.0;
    const double ny = norm2(y, e);
    double d = 0.0;
    for (int32_t c = 0; c < e; ++c) d += y[c] * g[c];
    double sem = (ny > 0.0 && ng > 0.0) ? d / (ny * ng) : 0.0;
    if (sem < 0.0) sem = 0.0;
    if (sem > 1.0) sem = 1.0;
    const double dist = 0.5 + 0.5 * dbar[i];
    const double ang = angle ? angle[i] : 1.0;
    Q[i] = size * ang * sem * dist;
    if (comp) {
      comp[4 * (int64_t)i] = size;
      comp[4 * (int64_t)i + 1] = ang;
      comp[4 * (int64_t)i + 2] = sem;
      comp[4 * (int64_t)i + 3] = dist;
    }
  }
  return 0;
}

int disc_oracle_fuse(const int32_t* ids, const double* q, const double* emb, int32_t m, int32_t e,
                     double* map_q, double* map_emb, int32_t n_map, int32_t* won) {
  if (!ids || !q || !emb || !map_q || !map_emb || m < 0 || e <= 0 || n_map < 0) return -1;
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_map > 0 ? n_map : 1));
  if (!owner) return -1;
  for (int32_t t = 0; t < n_map; ++t) owner[t] = -1;
  for (int32_t i = 0; i < m; ++i) {
    const int32_t t = ids[i];
    if (t < 0 || t >= n_map) continue;
    if (q[i] > map_q[t]) {
      map_q[t] = q[i];
      for (int32_t c = 0; c < e; ++c) map_emb[(int64_t)t * e + c] = emb[(int64_t)i * e + c];
      owner[t] = i;
    }
  }
  if (won) {
    for (int32_t i = 0; i < m; ++i) won[i] = 0;
    for (int32_t t = 0; t < n_map; ++t)
      if (owner[t] >= 0) won[owner[t]] = 1;
  }
  free(owner);
  return 0;
}
