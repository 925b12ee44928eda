/*
 * Seeded synthetic sparse matrices and vectors.
 *
 * This module only produces inputs: CRS arrays (row pointers, column
 * indices, values) and dense vectors. It contains none of the SELL-C-sigma
 * arithmetic. Both the CPU oracle and the GPU library consume its output.
 *
 * Random numbers come from a counter-based form of splitmix64
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): value i of stream s under seed k is
 *     mix64(key(k, s) + (i + 1) * GAMMA),  key(k, s) = mix64(k * GAMMA + s + 1)
 * which is exactly output i of a splitmix64 sequence whose state starts at
 * key(k, s). Every element is therefore addressable without generating the
 * ones before it, and the same numbers come out for any traversal order.
 *
 * Uniform [0,1): (r >> 11) * 2^-53.  Normal: Box-Muller with u1 in (0,1].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed * GAMMA + stream + 1);
}

static inline uint64_t draw(uint64_t key, uint64_t i) {
  return mix64(key + (i + 1) * GAMMA);
}

static inline double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

uint64_t synth_draw_u64(uint64_t seed, uint64_t stream, uint64_t i) {
  return draw(stream_key(seed, stream), i);
}

/* out[t] = value (start + t) of the stream, for t < count. */
void synth_u64(uint64_t seed, uint64_t stream, uint64_t start, int64_t count,
               uint64_t *out) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t t = 0; t < count; ++t) out[t] = draw(key, start + (uint64_t)t);
}

/* out[t] = a + (b - a) * U[0,1) for element t of the stream. */
void synth_uniform(uint64_t seed, uint64_t stream, double a, double b,
                   int64_t count, double *out) {
  uint64_t key = stream_key(seed, stream);
  for (int64_t t = 0; t < count; ++t)
    out[t] = a + (b - a) * u01(draw(key, (uint64_t)t));
}

/* ------------------------------------------------------------------ */
/* 2D 5-point Laplacian on an m x m grid, row i = ix + m*iy.            */
/* Diagonal 4, each existing neighbour -1, columns ascending.           */
/* ------------------------------------------------------------------ */
void synth_lap5_size(int64_t m, int64_t *n, int64_t *nnz) {
  *n = m * m;
  *nnz = m <= 0 ? 0 : 5 * m * m - 4 * m;
}

void synth_lap5(int64_t m, int64_t *rpt, int32_t *col, double *val) {
  int64_t k = 0;
  rpt[0] = 0;
  for (int64_t iy = 0; iy < m; ++iy)
    for (int64_t ix = 0; ix < m; ++ix) {
      int64_t i = ix + m * iy;
      if (iy > 0) { col[k] = (int32_t)(i - m); val[k++] = -1.0; }
      if (ix > 0) { col[k] = (int32_t)(i - 1); val[k++] = -1.0; }
      col[k] = (int32_t)i; val[k++] = 4.0;
      if (ix + 1 < m) { col[k] = (int32_t)(i + 1); val[k++] = -1.0; }
      if (iy + 1 < m) { col[k] = (int32_t)(i + m); val[k++] = -1.0; }
      rpt[i + 1] = k;
    }
}

/* ------------------------------------------------------------------ */
/* 3D 27-point stencil on an m^3 grid, row i = ix + m*iy + m^2*iz.      */
/* Every existing neighbour (including the centre) gets a value drawn   */
/* U[lo, hi) from stream 1, indexed by the entry's CRS position; with   */
/* ones != 0 every value is 1. Columns ascending (dz, dy, dx order).    */
/* ------------------------------------------------------------------ */
void synth_stencil27_size(int64_t m, int64_t *n, int64_t *nnz) {
  *n = m * m * m;
  int64_t t = m <= 0 ? 0 : 3 * m - 2;
  *nnz = t * t * t;
}

void synth_stencil27(int64_t m, uint64_t seed, double lo, double hi, int ones,
                     int64_t *rpt, int32_t *col, double *val) {
  uint64_t key = stream_key(seed, 1);
  int64_t k = 0;
  rpt[0] = 0;
  for (int64_t iz = 0; iz < m; ++iz)
    for (int64_t iy = 0; iy < m; ++iy)
      for (int64_t ix = 0; ix < m; ++ix) {
        int64_t i = ix + m * (iy + m * iz);
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t z = iz + dz;
          if (z < 0 || z >= m) continue;
          for (int dy = -1; dy <= 1; ++dy) {
            int64_t y = iy + dy;
            if (y < 0 || y >= m) continue;
            for (int dx = -1; dx <= 1; ++dx) {
              int64_t x = ix + dx;
              if (x < 0 || x >= m) continue;
              col[k] = (int32_t)(x + m * (y + m * z));
              val[k] = ones ? 1.0 : lo + (hi - lo) * u01(draw(key, (uint64_t)k));
              ++k;
            }
          }
        }
        rpt[i + 1] = k;
      }
}

/* ------------------------------------------------------------------ */
/* Irregular matrix with power-law row lengths.                          */
/*                                                                      */
/* Row lengths: P(L = k) proportional to k^-expo for lmin <= k <= lmax,  */
/* drawn by inverse CDF from stream 1 (one draw per row), then capped at */
/* max(1, n/2) so that drawing distinct columns stays cheap.             */
/* ------------------------------------------------------------------ */
void synth_powerlaw_lengths(int64_t n, uint64_t seed, double expo, int64_t lmin,
                            int64_t lmax, int64_t *len) {
  int64_t nk = lmax - lmin + 1;
  double *cum = (double *)malloc(sizeof(double) * (size_t)nk);
  double z = 0.0;
  for (int64_t t = 0; t < nk; ++t) {
    z += pow((double)(lmin + t), -expo);
    cum[t] = z;
  }
  int64_t cap = n / 2 > 1 ? n / 2 : 1;
  uint64_t key = stream_key(seed, 1);
  for (int64_t i = 0; i < n; ++i) {
    double target = u01(draw(key, (uint64_t)i)) * z;
    /* smallest t with cum[t] > target */
    int64_t a = 0, b = nk - 1;
    while (a < b) {
      int64_t mid = (a + b) / 2;
      if (cum[mid] > target) b = mid; else a = mid + 1;
    }
    int64_t L = lmin + a;
    len[i] = L > cap ? cap : L;
  }
  free(cum);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Columns and values, given rpt (prefix sums of the lengths).
 *
 * Each entry flips a fair coin (stream 2, indexed by CRS position): heads
 * draws from the band [max(0, i - band/2), min(n, i + band/2)) (stream 3),
 * tails draws uniformly from [0, n) (stream 4). At most half of the band
 * may be taken by band draws; later heads become tails. A column already
 * present in the row is drawn again with the next attempt counter, so
 * each row holds distinct columns. Columns are then sorted ascending and
 * values are N(0,1) by Box-Muller (streams 5 and 6, by CRS position).
 */
int synth_powerlaw_fill(int64_t n, uint64_t seed, int64_t band,
                        const int64_t *rpt, int32_t *col, double *val) {
  uint64_t kcoin = stream_key(seed, 2), kband = stream_key(seed, 3);
  uint64_t kuni = stream_key(seed, 4), kv1 = stream_key(seed, 5),
           kv2 = stream_key(seed, 6);
  int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t c = 0; c < n; ++c) stamp[c] = -1;
  int64_t half = band / 2;
  for (int64_t i = 0; i < n; ++i) {
    int64_t lo = i - half < 0 ? 0 : i - half;
    int64_t hi = i + half > n ? n : i + half;
    int64_t W = hi - lo, band_left = W / 2;
    for (int64_t g = rpt[i]; g < rpt[i + 1]; ++g) {
      int heads = (int)(draw(kcoin, (uint64_t)g) >> 63);
      if (heads && band_left > 0) --band_left; else heads = 0;
      uint64_t k = heads ? kband : kuni;
      int64_t span = heads ? W : n, base = heads ? lo : 0;
      int64_t c = -1;
      for (uint64_t att = 0; att < 65536; ++att) {
        uint64_t r = draw(k, ((uint64_t)g << 16) | att);
        c = base + (int64_t)(u01(r) * (double)span);
        if (c >= base + span) c = base + span - 1;
        if (stamp[c] != i) break;
        c = -1;
      }
      if (c < 0) { free(stamp); return -1; }
      stamp[c] = i;
      col[g] = (int32_t)c;
    }
    qsort(col + rpt[i], (size_t)(rpt[i + 1] - rpt[i]), sizeof(int32_t), cmp_i32);
    for (int64_t g = rpt[i]; g < rpt[i + 1]; ++g) {
      double u1 = 1.0 - u01(draw(kv1, (uint64_t)g));
      double u2 = u01(draw(kv2, (uint64_t)g));
      val[g] = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
    }
  }
  free(stamp);
  return 0;
}

/*
 * Rectangular nrows x ncols matrix with given row pointers: every row draws
 * its columns uniformly from [0, ncols) without repetition (stream 7,
 * indexed by CRS position and attempt), sorted ascending; values N(0,1)
 * (streams 8 and 9). Rows must be no longer than ncols / 2.
 */
int synth_uniform_fill(int64_t nrows, int64_t ncols, uint64_t seed, const int64_t *rpt,
                       int32_t *col, double *val) {
  uint64_t kc = stream_key(seed, 7), kv1 = stream_key(seed, 8), kv2 = stream_key(seed, 9);
  int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncols > 0 ? ncols : 1));
  if (!stamp) return -1;
  for (int64_t c = 0; c < ncols; ++c) stamp[c] = -1;
  for (int64_t i = 0; i < nrows; ++i) {
    for (int64_t g = rpt[i]; g < rpt[i + 1]; ++g) {
      int64_t c = -1;
      for (uint64_t att = 0; att < 65536; ++att) {
        c = (int64_t)(u01(draw(kc, ((uint64_t)g << 16) | att)) * (double)ncols);
        if (c >= ncols) c = ncols - 1;
        if (stamp[c] != i) break;
        c = -1;
      }
      if (c < 0) { free(stamp); return -1; }
      stamp[c] = i;
      col[g] = (int32_t)c;
    }
    qsort(col + rpt[i], (size_t)(rpt[i + 1] - rpt[i]), sizeof(int32_t), cmp_i32);
    for (int64_t g = rpt[i]; g < rpt[i + 1]; ++g) {
      double u1 = 1.0 - u01(draw(kv1, (uint64_t)g));
      double u2 = u01(draw(kv2, (uint64_t)g));
      val[g] = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
    }
  }
  free(stamp);
  return 0;
}
