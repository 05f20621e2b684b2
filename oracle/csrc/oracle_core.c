/*
 * FP64 reference kernels for the D-GAMP-CT oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; it is compiled into a separate shared object that only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark use.
 * It shares no source with the GPU library.
 *
 * Contents
 *   oracle_line_segments  exact intersection of one line with the pixel grid
 *                         (Siddon-style parametric crossings), the weights
 *                         a_ij = |L_i intersect pixel_j| of the system matrix
 *                         (Sec. 2.1, eq. linCT).
 *   oracle_project        z = A mu, ray by ray (Sec. 2.1, eq. linCT).
 *   oracle_backproject    g = A^T s with the very same per-ray weights.
 *   oracle_nlm            plain non-local means (patch-based plug-in
 *                         denoiser D of Sec. 4.3), written as the textbook
 *                         double sum over search offsets and patch pixels.
 *
 * Grid convention: an I x I grid of square pixels of side h centred on the
 * origin; pixel (row i, column j) has centre ((j-(I-1)/2) h, ((I-1)/2-i) h),
 * row 0 on top.  A line is {u : <u, n> = s} with unit normal n.
 *
 * Edge rule: a line lying exactly on a pixel edge meets the closed squares of
 * both neighbours along its whole length; it is given half of the chord in
 * each (the mean of the two one-sided limits of the chord as the line moves
 * off the edge).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Split a coordinate measured in pixel units from the grid's low edge into
 * the pixel(s) it falls in: one pixel with weight 1 in the interior, two
 * pixels with weight 1/2 each on an edge.  Returns the number of entries. */
static int locate(double c, int I, int *cell, double *w) {
  double f = floor(c);
  int n = 0;
  if (f == c) { /* exactly on an edge */
    int k = (int)f;
    if (k - 1 >= 0 && k - 1 < I) { cell[n] = k - 1; w[n] = 0.5; n++; }
    if (k >= 0 && k < I) { cell[n] = k; w[n] = 0.5; n++; }
  } else {
    int k = (int)f;
    if (k >= 0 && k < I) { cell[n] = k; w[n] = 1.0; n++; }
  }
  return n;
}

/* Exact chord lengths of the line {<u,n> = s} through every pixel it meets.
 * idx/len must hold 8*I+32 entries and lam 2*I+8.  Returns the entry count.
 * Lengths are in the units of h. */
int oracle_line_segments(int I, double h, double nx, double ny, double s,
                         int32_t *idx, double *len, double *lam) {
  const double half = 0.5 * I * h;
  const double p0x = s * nx, p0y = s * ny; /* foot of the normal */
  const double dx = -ny, dy = nx;           /* direction along the line */
  double lo = -INFINITY, hi = INFINITY;
  if (dx != 0.0) {
    double a = (-half - p0x) / dx, b = (half - p0x) / dx;
    lo = fmax(lo, fmin(a, b));
    hi = fmin(hi, fmax(a, b));
  } else if (fabs(p0x) > half) {
    return 0;
  }
  if (dy != 0.0) {
    double a = (-half - p0y) / dy, b = (half - p0y) / dy;
    lo = fmax(lo, fmin(a, b));
    hi = fmin(hi, fmax(a, b));
  } else if (fabs(p0y) > half) {
    return 0;
  }
  if (!(hi > lo)) return 0;

  int n = 0;
  lam[n++] = lo;
  lam[n++] = hi;
  for (int e = 0; e <= I; e++) {
    double edge = (e - 0.5 * I) * h;
    if (dx != 0.0) {
      double l = (edge - p0x) / dx;
      if (l > lo && l < hi) lam[n++] = l;
    }
    if (dy != 0.0) {
      double l = (edge - p0y) / dy;
      if (l > lo && l < hi) lam[n++] = l;
    }
  }
  qsort(lam, (size_t)n, sizeof(double), cmp_double);

  int m = 0;
  for (int k = 0; k + 1 < n; k++) {
    double seg = lam[k + 1] - lam[k];
    if (!(seg > 0.0)) continue;
    double lm = 0.5 * (lam[k] + lam[k + 1]);
    double xm = p0x + lm * dx, ym = p0y + lm * dy;
    int cols[2], rows[2];
    double wc[2], wr[2];
    int nc = locate(xm / h + 0.5 * I, I, cols, wc);
    int nr = locate(0.5 * I - ym / h, I, rows, wr);
    for (int a = 0; a < nr; a++)
      for (int b = 0; b < nc; b++) {
        idx[m] = rows[a] * I + cols[b];
        len[m] = seg * wr[a] * wc[b];
        m++;
      }
  }
  return m;
}

/* z_r = sum_j a_rj mu_j for every line r. */
void oracle_project(int I, double h, int64_t n_rays, const double *nx,
                    const double *ny, const double *s, const double *img,
                    double *sino) {
#pragma omp parallel
  {
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (8 * (size_t)I + 32));
    double *len = (double *)malloc(sizeof(double) * (8 * (size_t)I + 32));
    double *lam = (double *)malloc(sizeof(double) * (2 * (size_t)I + 8));
#pragma omp for schedule(dynamic, 64)
    for (int64_t r = 0; r < n_rays; r++) {
      int m = oracle_line_segments(I, h, nx[r], ny[r], s[r], idx, len, lam);
      double acc = 0.0;
      for (int k = 0; k < m; k++) acc += len[k] * img[idx[k]];
      sino[r] = acc;
    }
    free(idx);
    free(len);
    free(lam);
  }
}

/* g_j = sum_r a_rj s_r, using the same per-line weights as oracle_project. */
void oracle_backproject(int I, double h, int64_t n_rays, const double *nx,
                        const double *ny, const double *s, const double *sino,
                        double *img) {
  int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (8 * (size_t)I + 32));
  double *len = (double *)malloc(sizeof(double) * (8 * (size_t)I + 32));
  double *lam = (double *)malloc(sizeof(double) * (2 * (size_t)I + 8));
  memset(img, 0, sizeof(double) * (size_t)I * (size_t)I);
  for (int64_t r = 0; r < n_rays; r++) {
    int m = oracle_line_segments(I, h, nx[r], ny[r], s[r], idx, len, lam);
    for (int k = 0; k < m; k++) img[idx[k]] += len[k] * sino[r];
  }
  free(idx);
  free(len);
  free(lam);
}

/* Half-sample symmetric extension: -1 -> 0, -2 -> 1, I -> I-1, I+1 -> I-2. */
static int reflect(int k, int I) {
  while (k < 0 || k >= I) {
    if (k < 0) k = -k - 1;
    if (k >= I) k = 2 * I - k - 1;
  }
  return k;
}

/* Non-local means:  out_i = sum_o w_io r_{i+o} / sum_o w_io  over the
 * (2 sr + 1)^2 search offsets o, with
 *   d2_io = mean over the (2 pr + 1)^2 patch of (r_{i+q} - r_{i+o+q})^2
 *   w_io  = exp(-max(d2_io - 2 sigma^2, 0) / (hfac sigma)^2).
 * sigma <= 0 returns the input unchanged. */
void oracle_nlm(int I, const double *r, double sigma, int pr, int sr,
                double hfac, double *out) {
  if (!(sigma > 0.0)) {
    memcpy(out, r, sizeof(double) * (size_t)I * (size_t)I);
    return;
  }
  const double npatch = (double)((2 * pr + 1) * (2 * pr + 1));
  const double two_s2 = 2.0 * sigma * sigma;
  const double hh = (hfac * sigma) * (hfac * sigma);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < I; i++) {
    for (int j = 0; j < I; j++) {
      double wsum = 0.0, acc = 0.0;
      for (int oi = -sr; oi <= sr; oi++)
        for (int oj = -sr; oj <= sr; oj++) {
          double d2 = 0.0;
          for (int qi = -pr; qi <= pr; qi++)
            for (int qj = -pr; qj <= pr; qj++) {
              double a = r[reflect(i + qi, I) * I + reflect(j + qj, I)];
              double b = r[reflect(i + oi + qi, I) * I + reflect(j + oj + qj, I)];
              d2 += (a - b) * (a - b);
            }
          d2 /= npatch;
          double w = exp(-fmax(d2 - two_s2, 0.0) / hh);
          wsum += w;
          acc += w * r[reflect(i + oi, I) * I + reflect(j + oj, I)];
        }
      out[i * I + j] = acc / wsum;
    }
  }
}

/* Thread count of the OpenMP loops above (timing of the oracle only). */
#include <omp.h>
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }
