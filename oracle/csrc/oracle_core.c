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

/* ------------------------------------------------------------------ BM3D
 * The decisions of the two-stage block-matching collaborative filter (the
 * paper's plug-in denoiser, Dabov, Foi, Katkovnik & Egiazarian 2007): which
 * blocks join each reference block's group, and which coefficients of the
 * group's 3D transform survive the hard threshold.  They are taken on FP32
 * values, with every sum in the order written here (no contraction of a
 * multiply and an add), so that any implementation following the same order
 * takes the same decisions; everything continuous is left to FP64 code.
 */

/* Reference positions along one axis: 0, step, 2 step, ... <= I - n1, and
 * I - n1 itself if the grid misses it.  Returns the count. */
int oracle_bm3d_ref_axis(int I, int n1, int step, int32_t *pos) {
  int n = 0;
  for (int p = 0; p <= I - n1; p += step) pos[n++] = p;
  if (pos[n - 1] != I - n1) pos[n++] = I - n1;
  return n;
}

/* For every reference block (row-major over the reference grid): the
 * reference block itself first, then the other blocks (y, x) with
 * |y - y_r| <= ns, |x - x_r| <= ns, 0 <= y, x <= I - n1 whose distance
 * d = (sum over the block, row by row, of (a - b)^2) / n1^2 (the mean
 * squared difference) satisfies d <= thr, ordered by (d, y I + x); the first
 * min(count, n2) rounded down to a power of two form the group.
 * grp: n_ref * n2 raster indices (-1 past the group), gsize: n_ref. */
void oracle_bm3d_groups(int I, const float *r, int n1, int ns, int n2, float thr,
                        int n_axis, const int32_t *axis, int32_t *grp, int32_t *gsize) {
  const float inv = 1.0f / (float)(n1 * n1);
#pragma omp parallel
  {
    int cap = (2 * ns + 1) * (2 * ns + 1);
    float *dd = (float *)malloc(sizeof(float) * cap);
    int32_t *ii = (int32_t *)malloc(sizeof(int32_t) * cap);
#pragma omp for schedule(dynamic, 4)
    for (int q = 0; q < n_axis * n_axis; q++) {
      const int yr = axis[q / n_axis], xr = axis[q % n_axis];
      int m = 0;
      dd[m] = 0.0f; /* the reference block leads its group */
      ii[m] = yr * I + xr;
      m++;
      for (int y = yr - ns; y <= yr + ns; y++) {
        if (y < 0 || y > I - n1) continue;
        for (int x = xr - ns; x <= xr + ns; x++) {
          if (x < 0 || x > I - n1 || (y == yr && x == xr)) continue;
          float acc = 0.0f;
          for (int u = 0; u < n1; u++)
            for (int v = 0; v < n1; v++) {
              float t = r[(yr + u) * I + xr + v] - r[(y + u) * I + x + v];
              float t2 = t * t;
              acc = acc + t2;
            }
          float d = acc * inv;
          if (d <= thr) {
            dd[m] = d;
            ii[m] = y * I + x;
            m++;
          }
        }
      }
      /* the n2 smallest by (d, index), selection in order */
      int take = m < n2 ? m : n2;
      for (int k = 1; k < take; k++) {
        int best = k;
        for (int e = k + 1; e < m; e++)
          if (dd[e] < dd[best] || (dd[e] == dd[best] && ii[e] < ii[best])) best = e;
        float td = dd[k]; dd[k] = dd[best]; dd[best] = td;
        int32_t ti = ii[k]; ii[k] = ii[best]; ii[best] = ti;
      }
      int g = 1;
      while (2 * g <= take) g *= 2;
      gsize[q] = g;
      for (int k = 0; k < n2; k++) grp[(int64_t)q * n2 + k] = k < g ? ii[k] : -1;
    }
    free(dd);
    free(ii);
  }
}

/* Forward 3D transform of every group in FP32 -- per block the separable
 * 2D transform T1[u][v] = sum_k D[u][k] B[k][v], C[u][v] = sum_k T1[u][k]
 * D[v][k] (k ascending, each product rounded, then added), then along the
 * group the orthonormal Haar pyramid: at each level of length L the pairs
 * (2i, 2i+1) give ((a + b) c, (a - b) c), c = FP32(1/sqrt 2), sums first
 * then differences -- and the hard-threshold decision |coefficient| > thr.
 * keep: n_ref * n2 * n1 * n1 bytes (the group's first gsize blocks used),
 * nkeep: per group the number of surviving coefficients. */
void oracle_bm3d_keep(int I, const float *r, int n1, int n2, int n_ref, const int32_t *grp,
                      const int32_t *gsize, const float *D, float thr, uint8_t *keep,
                      int32_t *nkeep) {
  const float c = (float)0.70710678118654752440;
  const int bs = n1 * n1;
#pragma omp parallel
  {
    float *G = (float *)malloc(sizeof(float) * n2 * bs);
    float *T = (float *)malloc(sizeof(float) * n2 * bs);
    float *T1 = (float *)malloc(sizeof(float) * bs);
#pragma omp for schedule(dynamic, 4)
    for (int q = 0; q < n_ref; q++) {
      const int n = gsize[q];
      for (int b = 0; b < n; b++) {
        const int p = grp[(int64_t)q * n2 + b], y0 = p / I, x0 = p % I;
        for (int u = 0; u < n1; u++)
          for (int v = 0; v < n1; v++) {
            float acc = 0.0f;
            for (int k = 0; k < n1; k++) {
              float t = D[u * n1 + k] * r[(y0 + k) * I + x0 + v];
              acc = acc + t;
            }
            T1[u * n1 + v] = acc;
          }
        for (int u = 0; u < n1; u++)
          for (int v = 0; v < n1; v++) {
            float acc = 0.0f;
            for (int k = 0; k < n1; k++) {
              float t = T1[u * n1 + k] * D[v * n1 + k];
              acc = acc + t;
            }
            G[b * bs + u * n1 + v] = acc;
          }
      }
      for (int L = n; L > 1; L /= 2) {
        for (int i = 0; i < L / 2; i++)
          for (int e = 0; e < bs; e++) {
            float a = G[(2 * i) * bs + e], b = G[(2 * i + 1) * bs + e];
            float s = a + b, d = a - b;
            T[i * bs + e] = s * c;
            T[(L / 2 + i) * bs + e] = d * c;
          }
        memcpy(G, T, sizeof(float) * L * bs);
      }
      int cnt = 0;
      uint8_t *kq = keep + (int64_t)q * n2 * bs;
      for (int e = 0; e < n2 * bs; e++) kq[e] = 0;
      for (int e = 0; e < n * bs; e++) {
        uint8_t k = fabsf(G[e]) > thr;
        kq[e] = k;
        cnt += k;
      }
      nkeep[q] = cnt;
    }
    free(G);
    free(T);
    free(T1);
  }
}
