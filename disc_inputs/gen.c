/*
 * gen.c -- seeded synthetic inputs for DISC feature extraction.
 *
 * Holds none of the method's arithmetic: it only draws masks, token maps and
 * projections (and the quantised forms a caller would hand over).  Both the
 * HIP library's tests/benchmark and the CPU oracle consume these inputs.
 *
 * Random numbers: SplitMix64 derives an independent xoshiro256** stream per
 * (seed, stream index); uniforms use the top 53 bits; normals use the
 * Box-Muller transform in double precision.  Every mask and every token row
 * owns its own stream, so results do not depend on the thread count.
 *
 * Mask layout: bits[m][h][wq], wq = ceil(w/64), bit i of word k = pixel 64k+i;
 * bits at columns >= w stay zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
  uint64_t s[4];
} rng_t;

static uint64_t splitmix64(uint64_t* x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void rng_init(rng_t* r, uint64_t seed, uint64_t stream) {
  uint64_t x = seed * 0xD1342543DE82EF95ull + stream * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
  for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t* r) {
  uint64_t* s = r->s;
  const uint64_t result = rotl(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

/* uniform in [0, 1) */
static double rng_u01(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
static double rng_uniform(rng_t* r, double a, double b) { return a + (b - a) * rng_u01(r); }

/* standard normal, Box-Muller (one value per call; the pair's second value is
 * discarded so the stream position is independent of call parity) */
static double rng_normal(rng_t* r) {
  double u1 = rng_u01(r);
  double u2 = rng_u01(r);
  if (u1 < 0x1.0p-60) u1 = 0x1.0p-60;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ------------------------------------------------------------------ */
/* Rasterisation helpers (pixel centres at (x + 0.5, y + 0.5))          */
/* ------------------------------------------------------------------ */

static void set_run(uint64_t* row, int32_t w, int64_t xa, int64_t xb) { /* inclusive */
  if (xa < 0) xa = 0;
  if (xb > w - 1) xb = w - 1;
  for (int64_t x = xa; x <= xb;) {
    int64_t k = x >> 6, b0 = x & 63;
    int64_t b1 = (xb >> 6) == k ? (xb & 63) : 63;
    uint64_t msk = (b1 == 63 ? ~0ull : ((1ull << (b1 + 1)) - 1)) & ~((1ull << b0) - 1);
    row[k] |= msk;
    x = (k + 1) << 6;
  }
}

/* pixel x is filled iff its centre x + 0.5 lies in [xl, xr] */
static void fill_centres(uint64_t* row, int32_t w, double xl, double xr) {
  double a = ceil(xl - 0.5), b = floor(xr - 0.5);
  if (b < 0 || a > w - 1 || a > b) return;
  set_run(row, w, (int64_t)a, (int64_t)b);
}

/* even-odd rule: pixel filled iff its centre x + 0.5 lies in [c0, c1) */
static void fill_half_open(uint64_t* row, int32_t w, double c0, double c1) {
  double a = ceil(c0 - 0.5), b = ceil(c1 - 0.5) - 1.0;
  if (b < 0 || a > w - 1 || a > b) return;
  set_run(row, w, (int64_t)a, (int64_t)b);
}

static int mask_empty(const uint64_t* bits, int64_t nwords) {
  for (int64_t i = 0; i < nwords; ++i)
    if (bits[i]) return 0;
  return 1;
}

static void raster_ellipse(uint64_t* bits, int32_t h, int32_t w, int32_t wq, double cx, double cy,
                           double a, double b, double th) {
  const double c = cos(th), s = sin(th);
  /* ((dx c + dy s)/a)^2 + ((-dx s + dy c)/b)^2 <= 1, solved for dx per row */
  const double A = c * c / (a * a) + s * s / (b * b);
  const double ext = sqrt(a * a * s * s + b * b * c * c); /* half height of the bbox */
  int64_t y0 = (int64_t)floor(cy - ext - 1), y1 = (int64_t)ceil(cy + ext + 1);
  if (y0 < 0) y0 = 0;
  if (y1 > h - 1) y1 = h - 1;
  for (int64_t y = y0; y <= y1; ++y) {
    const double dy = (double)y + 0.5 - cy;
    const double B = 2.0 * dy * c * s * (1.0 / (a * a) - 1.0 / (b * b));
    const double Cq = dy * dy * (s * s / (a * a) + c * c / (b * b)) - 1.0;
    const double disc = B * B - 4.0 * A * Cq;
    if (disc < 0) continue;
    const double sq = sqrt(disc);
    fill_centres(bits + y * wq, w, cx + (-B - sq) / (2 * A), cx + (-B + sq) / (2 * A));
  }
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

static void raster_polygon(uint64_t* bits, int32_t h, int32_t w, int32_t wq, const double* px,
                           const double* py, int n) {
  double ymin = py[0], ymax = py[0];
  for (int i = 1; i < n; ++i) {
    if (py[i] < ymin) ymin = py[i];
    if (py[i] > ymax) ymax = py[i];
  }
  int64_t y0 = (int64_t)floor(ymin - 1), y1 = (int64_t)ceil(ymax + 1);
  if (y0 < 0) y0 = 0;
  if (y1 > h - 1) y1 = h - 1;
  double xs[32];
  for (int64_t y = y0; y <= y1; ++y) {
    const double yc = (double)y + 0.5;
    int k = 0;
    for (int i = 0; i < n; ++i) {
      const int j = (i + 1) % n;
      const double ya = py[i], yb = py[j];
      if ((ya <= yc && yc < yb) || (yb <= yc && yc < ya))
        xs[k++] = px[i] + (yc - ya) * (px[j] - px[i]) / (yb - ya);
    }
    qsort(xs, (size_t)k, sizeof(double), cmp_double);
    for (int i = 0; i + 1 < k; i += 2) fill_half_open(bits + y * wq, w, xs[i], xs[i + 1]);
  }
}

/* ------------------------------------------------------------------ */
/* Mask generators                                                      */
/* ------------------------------------------------------------------ */

/* Filled ellipses: semi-axes ~ U(amin, amax) independently, centre uniform in
 * the frame, angle ~ U[0, pi); resampled while empty. */
void disc_gen_masks_ellipses(uint64_t seed, int32_t m, int32_t h, int32_t w, double amin, double amax,
                             uint64_t* bits) {
  const int32_t wq = (w + 63) / 64;
  const int64_t per = (int64_t)h * wq;
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t i = 0; i < m; ++i) {
    rng_t r;
    rng_init(&r, seed, 0x100000000ull + (uint64_t)i);
    uint64_t* mb = bits + (int64_t)i * per;
    do {
      memset(mb, 0, sizeof(uint64_t) * (size_t)per);
      double a = rng_uniform(&r, amin, amax), b = rng_uniform(&r, amin, amax);
      double cx = rng_uniform(&r, 0, w), cy = rng_uniform(&r, 0, h);
      double th = rng_uniform(&r, 0, M_PI);
      raster_ellipse(mb, h, w, wq, cx, cy, a, b, th);
    } while (mask_empty(mb, per));
  }
}

/* Instance-like masks: target area A = exp(U(ln lo, ln hi)) * h * w; with
 * probability 1/2 an ellipse of aspect exp(U(0, ln 4)), otherwise a star
 * polygon with 3..12 vertices at sorted random angles and radii U(0.5, 1),
 * scaled to area A; random centre; resampled while empty. */
void disc_gen_masks_mixed(uint64_t seed, int32_t m, int32_t h, int32_t w, double lo, double hi,
                          uint64_t* bits) {
  const int32_t wq = (w + 63) / 64;
  const int64_t per = (int64_t)h * wq;
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t i = 0; i < m; ++i) {
    rng_t r;
    rng_init(&r, seed, 0x200000000ull + (uint64_t)i);
    uint64_t* mb = bits + (int64_t)i * per;
    do {
      memset(mb, 0, sizeof(uint64_t) * (size_t)per);
      const double area = exp(rng_uniform(&r, log(lo), log(hi))) * (double)h * (double)w;
      const double cx = rng_uniform(&r, 0, w), cy = rng_uniform(&r, 0, h);
      const double th = rng_uniform(&r, 0, M_PI);
      if (rng_u01(&r) < 0.5) {
        const double rho = exp(rng_uniform(&r, 0.0, log(4.0)));
        const double a = sqrt(area * rho / M_PI), b = sqrt(area / (rho * M_PI));
        raster_ellipse(mb, h, w, wq, cx, cy, a, b, th);
      } else {
        const int n = 3 + (int)(rng_next(&r) % 10u);
        double ang[12], rad[12], px[12], py[12];
        for (int k = 0; k < n; ++k) {
          ang[k] = rng_uniform(&r, 0, 2 * M_PI);
          rad[k] = rng_uniform(&r, 0.5, 1.0);
        }
        qsort(ang, (size_t)n, sizeof(double), cmp_double);
        double unit = 0.0; /* area of the unit-scale star polygon */
        for (int k = 0; k < n; ++k) {
          const int j = (k + 1) % n;
          double dth = ang[j] - ang[k];
          if (j == 0) dth += 2 * M_PI;
          unit += 0.5 * rad[k] * rad[j] * sin(dth);
        }
        if (unit <= 1e-9) continue; /* degenerate: draw again */
        const double sc = sqrt(area / unit);
        for (int k = 0; k < n; ++k) {
          px[k] = cx + sc * rad[k] * cos(ang[k] + th);
          py[k] = cy + sc * rad[k] * sin(ang[k] + th);
        }
        raster_polygon(mb, h, w, wq, px, py, n);
      }
    } while (mask_empty(mb, per));
  }
}

/* ------------------------------------------------------------------ */
/* Quantisers (what a caller would hand over)                           */
/* ------------------------------------------------------------------ */

/* double -> bfloat16 bits, round to nearest even, from the double itself */
static uint16_t bf16_from_double(double v) {
  if (v == 0.0) return signbit(v) ? 0x8000u : 0u;
  int e;
  double m = frexp(fabs(v), &e);        /* |v| = m 2^e, m in [0.5, 1) */
  double q = rint(ldexp(m, 8));          /* 8 significant bits, ties to even */
  float f = (float)ldexp(q, e - 8);      /* exact */
  if (v < 0) f = -f;
  uint32_t u;
  memcpy(&u, &f, sizeof u);
  return (uint16_t)(u >> 16);
}

/* double -> OCP e4m3fn code, round to nearest even, saturating at +-448 */
static uint8_t e4m3_from_double(double v) {
  uint8_t sign = (v < 0) ? 0x80u : 0u;
  double a = fabs(v);
  if (a >= 448.0) return sign | 0x7Eu;
  if (a < 0x1.0p-6) { /* subnormal range: multiples of 2^-9 */
    double q = rint(ldexp(a, 9));
    if (q >= 8.0) return sign | 0x08u; /* rounded up to the smallest normal */
    return sign | (uint8_t)q;
  }
  int e;
  double m = frexp(a, &e); /* a = m 2^e, m in [0.5,1) -> a = (2m) 2^(e-1) */
  double q = rint(ldexp(m, 4)); /* 4 significant bits: 8..16 */
  int ex = e - 1;
  if (q >= 16.0) {
    q = 8.0;
    ex += 1;
  }
  if (ex > 8 || (ex == 8 && q > 14.0)) return sign | 0x7Eu;
  return sign | (uint8_t)(((ex + 7) << 3) | ((int)q - 8));
}

void disc_gen_quantize_bf16(const double* in, int64_t n, uint16_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = bf16_from_double(in[i]);
}

void disc_gen_quantize_e4m3(const double* in, int64_t n, uint8_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = e4m3_from_double(in[i]);
}

/* Per-token scaled FP8: scale_p = amax_p / 448 (rounded to float; 1 for an all
 * zero token), q = e4m3(v / scale_p). */
static void quantize_row_fp8(const double* v, int32_t C, uint8_t* q, float* scale) {
  double amax = 0.0;
  for (int32_t c = 0; c < C; ++c)
    if (fabs(v[c]) > amax) amax = fabs(v[c]);
  float sc = amax > 0 ? (float)(amax / 448.0) : 1.0f;
  *scale = sc;
  for (int32_t c = 0; c < C; ++c) q[c] = e4m3_from_double(v[c] / (double)sc);
}

void disc_gen_quantize_fp8_rows(const double* in, int64_t G, int32_t C, uint8_t* q, float* scale) {
  for (int64_t p = 0; p < G; ++p) quantize_row_fp8(in + p * C, C, q + p * C, scale + p);
}

/* ------------------------------------------------------------------ */
/* Token maps and projections                                           */
/* ------------------------------------------------------------------ */

/* dtype: 0 = f32, 1 = bf16, 2 = e4m3fn + per-token scale, 3 = f64.
 * Values i.i.d. N(0, sd^2); row p draws from stream (seed, p). */
void disc_gen_normal_rows(uint64_t seed, uint64_t stream_base, int64_t rows, int32_t C, double sd,
                          int32_t dtype, void* out, float* scale) {
#pragma omp parallel
  {
    double* tmp = (double*)malloc(sizeof(double) * (size_t)C);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < rows; ++p) {
      rng_t r;
      rng_init(&r, seed, stream_base + (uint64_t)p);
      for (int32_t c = 0; c < C; ++c) tmp[c] = sd * rng_normal(&r);
      if (dtype == 0) {
        float* o = (float*)out + p * C;
        for (int32_t c = 0; c < C; ++c) o[c] = (float)tmp[c];
      } else if (dtype == 1) {
        uint16_t* o = (uint16_t*)out + p * C;
        for (int32_t c = 0; c < C; ++c) o[c] = bf16_from_double(tmp[c]);
      } else if (dtype == 2) {
        quantize_row_fp8(tmp, C, (uint8_t*)out + p * C, scale + p);
      } else {
        double* o = (double*)out + p * C;
        for (int32_t c = 0; c < C; ++c) o[c] = tmp[c];
      }
    }
    free(tmp);
  }
}

/* Structured token map (test-only variant): the gh x gw grid is split into
 * `regions` Voronoi cells around random seeds; each cell carries a random
 * N(0,1) vector, every token adds N(0, noise^2), and `outliers` random tokens
 * are multiplied by `outlier_gain`.  Output in double (quantise separately). */
void disc_gen_structured_tokens(uint64_t seed, int32_t gh, int32_t gw, int32_t C, int32_t regions,
                                double noise, int32_t outliers, double outlier_gain, double* out) {
  rng_t r;
  rng_init(&r, seed, 0x300000000ull);
  if (regions < 1) regions = 1;
  double* cy = (double*)malloc(sizeof(double) * (size_t)regions);
  double* cx = (double*)malloc(sizeof(double) * (size_t)regions);
  double* val = (double*)malloc(sizeof(double) * (size_t)regions * C);
  for (int32_t k = 0; k < regions; ++k) {
    cy[k] = rng_uniform(&r, 0, gh);
    cx[k] = rng_uniform(&r, 0, gw);
    for (int32_t c = 0; c < C; ++c) val[(int64_t)k * C + c] = rng_normal(&r);
  }
  for (int32_t i = 0; i < gh; ++i)
    for (int32_t j = 0; j < gw; ++j) {
      int32_t best = 0;
      double bd = 1e300;
      for (int32_t k = 0; k < regions; ++k) {
        double dy = i + 0.5 - cy[k], dx = j + 0.5 - cx[k];
        double d = dy * dy + dx * dx;
        if (d < bd) {
          bd = d;
          best = k;
        }
      }
      double* o = out + ((int64_t)i * gw + j) * C;
      for (int32_t c = 0; c < C; ++c) o[c] = val[(int64_t)best * C + c] + noise * rng_normal(&r);
    }
  for (int32_t k = 0; k < outliers; ++k) {
    int64_t p = (int64_t)(rng_next(&r) % (uint64_t)((int64_t)gh * gw));
    for (int32_t c = 0; c < C; ++c) out[p * C + c] *= outlier_gain;
  }
  free(cy);
  free(cx);
  free(val);
}

/* ------------------------------------------------------------------ */
/* Counts                                                               */
/* ------------------------------------------------------------------ */

/* Poisson(mean) draws clipped to [lo, hi] (Knuth's product method). */
void disc_gen_poisson_counts(uint64_t seed, int32_t n, double mean, int32_t lo, int32_t hi, int32_t* out) {
  rng_t r;
  rng_init(&r, seed, 0x400000000ull);
  const double L = exp(-mean);
  for (int32_t i = 0; i < n; ++i) {
    int32_t k = 0;
    double p = 1.0;
    do {
      ++k;
      p *= rng_u01(&r);
    } while (p > L);
    k -= 1;
    if (k < lo) k = lo;
    if (k > hi) k = hi;
    out[i] = k;
  }
}

/* Exponential inter-arrival gaps with the given mean (seconds). */
void disc_gen_exponential(uint64_t seed, uint64_t stream, int32_t n, double mean, double* out) {
  rng_t r;
  rng_init(&r, seed, 0x500000000ull + stream);
  for (int32_t i = 0; i < n; ++i) {
    double u = rng_u01(&r);
    out[i] = -mean * log(1.0 - u);
  }
}
