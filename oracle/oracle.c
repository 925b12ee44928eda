/*
 * CPU ORACLE for SELL-C-sigma sparse matrix-vector multiplication.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file. It is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg. It shares no code, header, table or helper
 * with the GPU implementation.
 *
 * Source: Kreutzer, Hager, Wellein, Fehske, Bishop, "A unified sparse matrix
 * data format for efficient general sparse matrix-vector multiply on modern
 * processors with wide SIMD units" (arXiv:1307.6209).
 *
 * Every routine is the plain definition, written out:
 *   - CRS storage and the CRS kernel: Sect. 3.1, Listing "CRS spMVM kernel".
 *   - SELL-C-sigma storage: Sect. 3.3 (chunks of C rows, padding to the
 *     longest row of the chunk, column-major inside a chunk, cs[]/cl[]).
 *   - Sorting scope sigma: Sect. 3.4 (rows sorted by descending length
 *     within windows of sigma consecutive rows).
 *   - Chunk occupancy beta: Sect. 3.4, Eqs. (beta), (nc), (max).
 *   - Coefficient of variation zeta: Sect. 5, Eq. (eq:cv).
 *   - SELL kernel semantics: Sect. 3.3, Listing "SELL-4-sigma spMVM kernel",
 *     generalised from C = 4 to any C.
 *
 * Readings where the paper is silent (each also recorded in the design notes):
 *   - ties in the length sort keep the original row order (stable sort);
 *   - windows start at row 0 and step by sigma; the last one may be short;
 *   - padding slots hold value 0 and column index 0 (Sect. 4, the remark
 *     on padded column indices under Eq. (sellbalance));
 *   - within a row, entries keep their CRS order;
 *   - column ids stay the original ones (rows are permuted, x and y stay in
 *     the caller's order; y is overwritten);
 *   - the sums in Eqs. (beta) and (eq:cv) run over N_c chunks / N rows;
 *   - beta := 1 when the padded size is 0.
 *
 * Arithmetic: double, compiled with -ffp-contract=off (no fused multiply-add),
 * summed in CRS order. A long double (x87 80-bit, 64-bit significand)
 * companion gives the reference for error bounds.
 *
 * Reduced precision (not covered by the paper, which uses double only):
 * value rounding to binary32 and to bfloat16, both round-to-nearest-even,
 * written from the IEEE-754 definition of rounding to a p-bit significand.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* CRS validation (Sect. 3.1: rpt[] row offsets, col[] column indices) */
/* 0 ok, 1 rpt[0] != 0, 2 rpt decreasing, 3 rpt[n] != nnz,             */
/* 4 column index outside [0, m), 5 negative sizes                      */
/* ------------------------------------------------------------------ */
int or_crs_validate(int64_t n, int64_t m, int64_t nnz, const int64_t *rpt,
                    const int32_t *col) {
  if (n < 0 || m < 0 || nnz < 0) return 5;
  if (rpt[0] != 0) return 1;
  for (int64_t i = 0; i < n; ++i)
    if (rpt[i + 1] < rpt[i]) return 2;
  if (rpt[n] != nnz) return 3;
  for (int64_t j = 0; j < nnz; ++j)
    if (col[j] < 0 || (int64_t)col[j] >= m) return 4;
  return 0;
}

/* ------------------------------------------------------------------ */
/* CRS spMVM (Listing "CRS spMVM kernel") with y set to zero first:      */
/*   y[i] = sum_{j = rpt[i]}^{rpt[i+1]-1} val[j] * x[col[j]]            */
/* summed in CRS order. Rows are independent, so the row loop may run    */
/* on several threads without changing any result bit. sched selects the */
/* OpenMP schedule the paper uses for its CPU runs (Sect. 5): 0 STATIC,  */
/* 1 GUIDED with chunk 1.                                                */
/* ------------------------------------------------------------------ */
void or_crs_spmv(int64_t n, const int64_t *rpt, const int32_t *col,
                 const double *val, const double *x, double *y, int nthreads,
                 int sched) {
  if (nthreads < 1) nthreads = 1;
  if (sched == 1) {
#pragma omp parallel for num_threads(nthreads) schedule(guided, 1)
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t j = rpt[i]; j < rpt[i + 1]; ++j) s += val[j] * x[col[j]];
      y[i] = s;
    }
  } else {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t j = rpt[i]; j < rpt[i + 1]; ++j) s += val[j] * x[col[j]];
      y[i] = s;
    }
  }
}

/* Same sum in long double, rounded once to double at the end. */
void or_crs_spmv_ld(int64_t n, const int64_t *rpt, const int32_t *col,
                    const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(guided, 64)
  for (int64_t i = 0; i < n; ++i) {
    long double s = 0.0L;
    for (int64_t j = rpt[i]; j < rpt[i + 1]; ++j)
      s += (long double)val[j] * (long double)x[col[j]];
    y[i] = (double)s;
  }
}

/* (|A| |x|)_i in long double, rounded to double: the scale of the
 * componentwise error bounds. */
void or_crs_absmv(int64_t n, const int64_t *rpt, const int32_t *col,
                  const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(guided, 64)
  for (int64_t i = 0; i < n; ++i) {
    long double s = 0.0L;
    for (int64_t j = rpt[i]; j < rpt[i + 1]; ++j)
      s += fabsl((long double)val[j]) * fabsl((long double)x[col[j]]);
    y[i] = (double)s;
  }
}

/* Block form Y = A X with X (m x k) and Y (n x k) row-major: column v of Y
 * is the CRS spMVM of column v of X. Long double, plus |A||X|. */
void or_crs_spmmv_ld(int64_t n, const int64_t *rpt, const int32_t *col,
                     const double *val, const double *X, int64_t k, double *Y,
                     double *absY) {
#pragma omp parallel for schedule(guided, 64)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t v = 0; v < k; ++v) {
      long double s = 0.0L, a = 0.0L;
      for (int64_t j = rpt[i]; j < rpt[i + 1]; ++j) {
        long double p = (long double)val[j] * (long double)X[(int64_t)col[j] * k + v];
        s += p;
        a += fabsl(p);
      }
      Y[i * k + v] = (double)s;
      if (absY) absY[i * k + v] = (double)a;
    }
  }
}

/* ------------------------------------------------------------------ */
/* SELL-C-sigma layout (Sects. 3.3 and 3.4)                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t len;
  int64_t row;
} len_row;

/* longer rows first; equal lengths keep ascending original row index */
static int cmp_len_desc(const void *a, const void *b) {
  const len_row *p = (const len_row *)a, *q = (const len_row *)b;
  if (p->len != q->len) return p->len > q->len ? -1 : 1;
  return (p->row > q->row) - (p->row < q->row);
}

/*
 * perm[p] = original row stored at sorted position p (p < n).
 * Windows [w*sigma, min((w+1)*sigma, n)) are sorted independently by
 * descending row length (ties: original order). sigma = 1 is the identity.
 * cl[i] = max length over the chunk's rows (Eq. (max), rows taken in
 * sorted order; positions p >= n are padding rows of length 0).
 * cs[0] = 0, cs[i+1] = cs[i] + C * cl[i]; cs has nc + 1 entries,
 * nc = ceil(n / C) (Eq. (nc) for the padded row count).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int or_sell_layout(int64_t n, const int64_t *rpt, int32_t C, int64_t sigma,
                   int32_t *perm, int32_t *cl, int64_t *cs) {
  if (C < 1 || sigma < 1 || n < 0) return -1;
  int64_t nc = (n + C - 1) / C;
  for (int64_t w0 = 0; w0 < n; w0 += sigma) {
    int64_t w1 = w0 + sigma < n ? w0 + sigma : n;
    int64_t cnt = w1 - w0;
    len_row *buf = (len_row *)malloc(sizeof(len_row) * (size_t)cnt);
    if (!buf) return -1;
    for (int64_t t = 0; t < cnt; ++t) {
      buf[t].row = w0 + t;
      buf[t].len = rpt[w0 + t + 1] - rpt[w0 + t];
    }
    qsort(buf, (size_t)cnt, sizeof(len_row), cmp_len_desc);
    for (int64_t t = 0; t < cnt; ++t) perm[w0 + t] = (int32_t)buf[t].row;
    free(buf);
  }
  cs[0] = 0;
  for (int64_t i = 0; i < nc; ++i) {
    int64_t mx = 0;
    for (int64_t r = 0; r < C; ++r) {
      int64_t p = i * C + r;
      if (p < n) {
        int64_t row = perm[p];
        int64_t len = rpt[row + 1] - rpt[row];
        if (len > mx) mx = len;
      }
    }
    cl[i] = (int32_t)mx;
    cs[i + 1] = cs[i] + (int64_t)C * mx;
  }
  return 0;
}

/*
 * Chunk i, chunk column j < cl[i], lane r < C live at cs[i] + j*C + r.
 * The slot holds entry j of row perm[i*C + r] (CRS order) when that row
 * exists and has more than j entries; otherwise value 0 and column 0.
 */
void or_sell_fill(int64_t n, const int64_t *rpt, const int32_t *col,
                  const double *val, int32_t C, const int32_t *perm,
                  const int32_t *cl, const int64_t *cs, int32_t *scol,
                  double *sval) {
  int64_t nc = (n + C - 1) / C;
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t j = 0; j < cl[i]; ++j)
      for (int64_t r = 0; r < C; ++r) {
        int64_t idx = cs[i] + j * C + r;
        int64_t p = i * C + r;
        scol[idx] = 0;
        sval[idx] = 0.0;
        if (p < n) {
          int64_t row = perm[p];
          if (j < rpt[row + 1] - rpt[row]) {
            scol[idx] = col[rpt[row] + j];
            sval[idx] = val[rpt[row] + j];
          }
        }
      }
}

/*
 * Symmetric permutation P A P^T of a square CRS matrix (Sect. 3.4: after the
 * row sort, column indices are permuted accordingly so that an iterative
 * solver can work in the permuted index space). Row p of the result is row
 * perm[p] of A, entries in their CRS order, each column c renamed iperm[c]
 * with iperm[perm[p]] = p. rpt2 has n + 1 entries, col2/val2 nnz.
 */
int or_crs_symperm(int64_t n, const int64_t *rpt, const int32_t *col, const double *val,
                   const int32_t *perm, int64_t *rpt2, int32_t *col2, double *val2) {
  int32_t *iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!iperm) return -1;
  for (int64_t p = 0; p < n; ++p) iperm[perm[p]] = (int32_t)p;
  rpt2[0] = 0;
  for (int64_t p = 0; p < n; ++p) {
    int64_t row = perm[p], k = rpt2[p];
    for (int64_t j = rpt[row]; j < rpt[row + 1]; ++j, ++k) {
      col2[k] = iperm[col[j]];
      val2[k] = val[j];
    }
    rpt2[p + 1] = k;
  }
  free(iperm);
  return 0;
}

/* Chunk occupancy, Eq. (beta): nnz over the stored slots. */
double or_sell_beta(int64_t nnz, int64_t padded) {
  return padded == 0 ? 1.0 : (double)nnz / (double)padded;
}

/* Coefficient of variation of the row lengths, Eq. (eq:cv). */
double or_row_zeta(int64_t n, const int64_t *rpt) {
  if (n == 0) return 0.0;
  long double mean = (long double)rpt[n] / (long double)n, ss = 0.0L;
  if (mean == 0.0L) return 0.0;
  for (int64_t i = 0; i < n; ++i) {
    long double d = (long double)(rpt[i + 1] - rpt[i]) - mean;
    ss += d * d;
  }
  return (double)(sqrtl(ss / (long double)n) / mean);
}

/*
 * SELL spMVM (Listing "SELL-4-sigma spMVM kernel", any C): for every chunk
 * i and lane r, sum val * x[col] over the chunk columns j < cl[i] in order,
 * then store the sum at y[perm[i*C + r]] for rows that exist. Padding adds
 * 0 * x[0].
 */
void or_sell_spmv(int64_t n, int32_t C, const int32_t *perm, const int32_t *cl,
                  const int64_t *cs, const int32_t *scol, const double *sval,
                  const double *x, double *y) {
  int64_t nc = (n + C - 1) / C;
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t r = 0; r < C; ++r) {
      int64_t p = i * C + r;
      if (p >= n) continue;
      double s = 0.0;
      for (int64_t j = 0; j < cl[i]; ++j) {
        int64_t idx = cs[i] + j * C + r;
        s += sval[idx] * x[scol[idx]];
      }
      y[perm[p]] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Rounding of double values to narrower formats, nearest-even.          */
/* ------------------------------------------------------------------ */

/* binary32: the C conversion rounds to nearest-even under the default
 * floating-point environment. */
void or_round_f32(int64_t count, const double *in, float *out) {
  for (int64_t t = 0; t < count; ++t) out[t] = (float)in[t];
}

/*
 * bfloat16 (1 sign, 8 exponent, 7 fraction bits; same exponent range as
 * binary32). For finite d: the spacing of representable numbers around d is
 * 2^(e-7) where 2^e <= |d| < 2^(e+1), but never below the subnormal spacing
 * 2^-133. d / spacing is exact (a power-of-two scaling), rint() rounds it to
 * the nearest integer with ties to even, and scaling back is exact. A result
 * above the largest bfloat16 becomes infinity. The bits are the upper half
 * of the binary32 encoding of the (exactly representable) result.
 */
static uint16_t round_bf16_one(double d) {
  if (isnan(d)) return 0x7FC0;
  if (isinf(d)) return d > 0 ? 0x7F80 : 0xFF80;
  double r = 0.0;
  if (d != 0.0) {
    int e;
    frexp(d, &e);          /* |d| = f * 2^e with f in [0.5, 1): 2^(e-1) <= |d| */
    int qexp = (e - 1) - 7; /* spacing exponent for an 8-bit significand */
    if (qexp < -133) qexp = -133;
    double q = ldexp(d, -qexp);
    r = ldexp(rint(q), qexp);
  } else {
    r = d;
  }
  const double bf16_max = 0x1.FEp127; /* (2 - 2^-7) * 2^127 */
  float f;
  if (fabs(r) > bf16_max) f = r > 0 ? INFINITY : -INFINITY;
  else f = (float)r; /* exact */
  uint32_t bits;
  memcpy(&bits, &f, 4);
  return (uint16_t)(bits >> 16);
}

void or_round_bf16(int64_t count, const double *in, uint16_t *out) {
  for (int64_t t = 0; t < count; ++t) out[t] = round_bf16_one(in[t]);
}

/* bfloat16 bits to double (exact). */
void or_bf16_to_f64(int64_t count, const uint16_t *in, double *out) {
  for (int64_t t = 0; t < count; ++t) {
    uint32_t bits = (uint32_t)in[t] << 16;
    float f;
    memcpy(&f, &bits, 4);
    out[t] = (double)f;
  }
}
