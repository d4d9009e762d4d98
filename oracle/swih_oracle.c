/*
 * Brute-force CPU oracle for spatially weighted local histograms (SWIH).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU path.
 *
 * What it computes is the plain quantity that the paper's method reaches
 * exactly (Sec. 3 states SWIH is exact against brute force; Sec. 5 repeats it):
 * for a window centred on (xc, yc), the b-bin histogram in which every pixel
 * adds its spatial weight k(dx, dy) to the bin of its quantised value
 * (Sec. 2, the convolution-style "brute-force approach", whose cost is linear
 * in the window area).  The oracle loops over every pixel of every window.
 *
 * Readings of the paper that this file fixes (the paper leaves them open):
 *  - Quantiser Q (Eq. 2 names it only): uniform bins over [0, 256),
 *    Q(v) = floor(v * nbins / 256).
 *  - Manhattan kernel (Eq. 1 is a distance; weights must fall toward the
 *    window border, Sec. 2): k = (rx + ry + 1) - |dx| - |dy|, which is 1 at the
 *    window corners and an integer everywhere.
 *  - Euclidean kernel (Fig. 1b, no formula): the squared-distance paraboloid
 *    k = (rx^2 + ry^2 + 1) - dx^2 - dy^2.
 *  - Gaussian kernel (Fig. 1c, no formula): the true Gaussian
 *    exp(-dx^2 / (2 sx^2) - dy^2 / (2 sy^2)).
 *  - Exponential kernel (named among the weighting functions of Sec. 2, no
 *    formula): the Laplacian of the city-block distance,
 *    exp(-|dx| / tx - |dy| / ty), widths tx = w / 4, ty = h / 4 as for the
 *    Gaussian.
 *  - Uniform kernel: k = 1, the plain local histogram (Sec. 1, integral
 *    histogram of Porikli).
 *  - Normalisation (Sec. 1 steps (4)-(5); Sec. 2.1): by the total kernel mass
 *    S, which does not depend on where the window sits.
 *  - Similarity behind the likelihood map (Sec. 2, Fig. 3; Sec. 4): the
 *    Bhattacharyya coefficient sum_b sqrt(p_b t_b).
 *  - Only windows lying wholly inside the image are evaluated.
 *
 * Integer kernels accumulate in int64, the Gaussian in double.  OpenMP
 * parallelises over window centres only; every centre is computed the same way.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_UNIFORM = 0, OR_MANHATTAN = 1, OR_EUCLIDEAN = 2, OR_GAUSSIAN = 3, OR_EXPONENTIAL = 5 };

/* Threads of the parallel loops below (n >= 1), and the current count: lets a
 * caller time the oracle on one core and on all of them in one process. */
void oracle_set_threads(int n) { omp_set_num_threads(n < 1 ? 1 : n); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Quantiser Q of Eq. 2: uniform bins over [0, 256). */
int oracle_quantise(int v, int nbins) { return (v * nbins) / 256; }

static int64_t iabs64(int64_t a) { return a < 0 ? -a : a; }

/*
 * Integer spatial kernel table k[(dy + ry) * w + (dx + rx)] for an odd w x h
 * window (Eq. 1 for Manhattan; readings above for the others).
 * Returns 0, or -1 for an unsupported kind / even size.
 */
int oracle_kernel_table_int(int kind, int w, int h, int64_t* out) {
  if (w < 1 || h < 1 || (w % 2) == 0 || (h % 2) == 0) return -1;
  const int64_t rx = (w - 1) / 2, ry = (h - 1) / 2;
  for (int64_t dy = -ry; dy <= ry; ++dy) {
    for (int64_t dx = -rx; dx <= rx; ++dx) {
      int64_t k;
      if (kind == OR_UNIFORM) {
        k = 1;
      } else if (kind == OR_MANHATTAN) {
        k = (rx + ry + 1) - iabs64(dx) - iabs64(dy);
      } else if (kind == OR_EUCLIDEAN) {
        k = (rx * rx + ry * ry + 1) - dx * dx - dy * dy;
      } else {
        return -1;
      }
      out[(dy + ry) * w + (dx + rx)] = k;
    }
  }
  return 0;
}

/* True Gaussian table, same indexing. */
int oracle_kernel_table_gauss(int w, int h, double sigma_x, double sigma_y, double* out) {
  if (w < 1 || h < 1 || (w % 2) == 0 || (h % 2) == 0) return -1;
  if (!(sigma_x > 0.0) || !(sigma_y > 0.0)) return -1;
  const int rx = (w - 1) / 2, ry = (h - 1) / 2;
  for (int dy = -ry; dy <= ry; ++dy) {
    for (int dx = -rx; dx <= rx; ++dx) {
      const double e = (double)dx * dx / (2.0 * sigma_x * sigma_x) +
                       (double)dy * dy / (2.0 * sigma_y * sigma_y);
      out[(dy + ry) * w + (dx + rx)] = exp(-e);
    }
  }
  return 0;
}

/* Exponential (Laplacian) table exp(-|dx| / tau_x - |dy| / tau_y), same indexing. */
int oracle_kernel_table_exp(int w, int h, double tau_x, double tau_y, double* out) {
  if (w < 1 || h < 1 || (w % 2) == 0 || (h % 2) == 0) return -1;
  if (!(tau_x > 0.0) || !(tau_y > 0.0)) return -1;
  const int rx = (w - 1) / 2, ry = (h - 1) / 2;
  for (int dy = -ry; dy <= ry; ++dy) {
    for (int dx = -rx; dx <= rx; ++dx) {
      const double e = fabs((double)dx) / tau_x + fabs((double)dy) / tau_y;
      out[(dy + ry) * w + (dx + rx)] = exp(-e);
    }
  }
  return 0;
}

/* Brute-force weighted histogram of one window, integer weights. */
static void hist_one_i64(const uint8_t* img, int pitch, int nbins, const int64_t* tab,
                         int w, int h, int xc, int yc, int64_t* out) {
  const int rx = (w - 1) / 2, ry = (h - 1) / 2;
  for (int b = 0; b < nbins; ++b) out[b] = 0;
  for (int dy = -ry; dy <= ry; ++dy) {
    const uint8_t* row = img + (size_t)(yc + dy) * pitch;
    for (int dx = -rx; dx <= rx; ++dx) {
      const int b = oracle_quantise(row[xc + dx], nbins);
      out[b] += tab[(dy + ry) * w + (dx + rx)];
    }
  }
}

static void hist_one_f64(const uint8_t* img, int pitch, int nbins, const double* tab,
                         int w, int h, int xc, int yc, double* out) {
  const int rx = (w - 1) / 2, ry = (h - 1) / 2;
  for (int b = 0; b < nbins; ++b) out[b] = 0.0;
  for (int dy = -ry; dy <= ry; ++dy) {
    const uint8_t* row = img + (size_t)(yc + dy) * pitch;
    for (int dx = -rx; dx <= rx; ++dx) {
      const int b = oracle_quantise(row[xc + dx], nbins);
      out[b] += tab[(dy + ry) * w + (dx + rx)];
    }
  }
}

static int centre_ok(int H, int W, int w, int h, int xc, int yc) {
  const int rx = (w - 1) / 2, ry = (h - 1) / 2;
  return xc >= rx && xc <= W - 1 - rx && yc >= ry && yc <= H - 1 - ry;
}

/*
 * Histograms at n listed centres ([n][2] = (xc, yc)), out [n][nbins].
 * Returns 0, or -1 if a centre puts the window outside the image.
 */
int oracle_hist_i64(const uint8_t* img, int H, int W, int pitch, int nbins, const int64_t* tab,
                    int w, int h, const int32_t* centres, int n, int64_t* out) {
  for (int k = 0; k < n; ++k)
    if (!centre_ok(H, W, w, h, centres[2 * k], centres[2 * k + 1])) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < n; ++k)
    hist_one_i64(img, pitch, nbins, tab, w, h, centres[2 * k], centres[2 * k + 1],
                 out + (size_t)k * nbins);
  return 0;
}

int oracle_hist_f64(const uint8_t* img, int H, int W, int pitch, int nbins, const double* tab,
                    int w, int h, const int32_t* centres, int n, double* out) {
  for (int k = 0; k < n; ++k)
    if (!centre_ok(H, W, w, h, centres[2 * k], centres[2 * k + 1])) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < n; ++k)
    hist_one_f64(img, pitch, nbins, tab, w, h, centres[2 * k], centres[2 * k + 1],
                 out + (size_t)k * nbins);
  return 0;
}

/*
 * Bhattacharyya likelihood at listed centres, integer kernels.
 * With p_b = H_b / S and t_b = T_b / S (S = kernel mass), the coefficient
 * sum_b sqrt(p_b t_b) equals (sum_b sqrt(H_b T_b)) / S; H_b T_b is an exact
 * integer below 2^53, so each term is one correctly rounded double sqrt,
 * added in bin order 0..nbins-1.
 */
int oracle_bc_i64(const uint8_t* img, int H, int W, int pitch, int nbins, const int64_t* tab,
                  int w, int h, const int64_t* tmpl_raw, const int32_t* centres, int n,
                  double* out) {
  for (int k = 0; k < n; ++k)
    if (!centre_ok(H, W, w, h, centres[2 * k], centres[2 * k + 1])) return -1;
  int64_t S = 0;
  for (int i = 0; i < w * h; ++i) S += tab[i];
#pragma omp parallel
  {
    int64_t* hb = (int64_t*)malloc(sizeof(int64_t) * (size_t)nbins);
#pragma omp for schedule(dynamic, 16)
    for (int k = 0; k < n; ++k) {
      hist_one_i64(img, pitch, nbins, tab, w, h, centres[2 * k], centres[2 * k + 1], hb);
      double acc = 0.0;
      for (int b = 0; b < nbins; ++b) acc += sqrt((double)(hb[b] * tmpl_raw[b]));
      out[k] = acc / (double)S;
    }
    free(hb);
  }
  return 0;
}

/*
 * Bhattacharyya likelihood at listed centres, real-valued kernels.
 * p_b = H_b / S with S the kernel mass; tmpl_p is the normalised template.
 */
int oracle_bc_f64(const uint8_t* img, int H, int W, int pitch, int nbins, const double* tab,
                  int w, int h, const double* tmpl_p, const int32_t* centres, int n,
                  double* out) {
  for (int k = 0; k < n; ++k)
    if (!centre_ok(H, W, w, h, centres[2 * k], centres[2 * k + 1])) return -1;
  double S = 0.0;
  for (int i = 0; i < w * h; ++i) S += tab[i];
#pragma omp parallel
  {
    double* hb = (double*)malloc(sizeof(double) * (size_t)nbins);
#pragma omp for schedule(dynamic, 16)
    for (int k = 0; k < n; ++k) {
      hist_one_f64(img, pitch, nbins, tab, w, h, centres[2 * k], centres[2 * k + 1], hb);
      double acc = 0.0;
      for (int b = 0; b < nbins; ++b) acc += sqrt((hb[b] / S) * tmpl_p[b]);
      out[k] = acc;
    }
    free(hb);
  }
  return 0;
}

/*
 * Dense map over the inclusive centre rectangle [x0, x1] x [y0, y1]
 * (row-major out[(yc - y0) * (x1 - x0 + 1) + (xc - x0)]).
 */
static int dense_centres(int H, int W, int w, int h, int x0, int y0, int x1, int y1,
                         int32_t** pts, int* n) {
  if (x1 < x0 || y1 < y0) { *pts = NULL; *n = 0; return 0; }
  if (!centre_ok(H, W, w, h, x0, y0) || !centre_ok(H, W, w, h, x1, y1)) return -1;
  const int nx = x1 - x0 + 1, ny = y1 - y0 + 1;
  int32_t* p = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)nx * ny);
  for (int yy = 0; yy < ny; ++yy)
    for (int xx = 0; xx < nx; ++xx) {
      p[2 * ((size_t)yy * nx + xx)] = x0 + xx;
      p[2 * ((size_t)yy * nx + xx) + 1] = y0 + yy;
    }
  *pts = p;
  *n = nx * ny;
  return 0;
}

int oracle_map_i64(const uint8_t* img, int H, int W, int pitch, int nbins, const int64_t* tab,
                   int w, int h, const int64_t* tmpl_raw, int x0, int y0, int x1, int y1,
                   double* out) {
  int32_t* pts; int n;
  if (dense_centres(H, W, w, h, x0, y0, x1, y1, &pts, &n)) return -1;
  int rc = n ? oracle_bc_i64(img, H, W, pitch, nbins, tab, w, h, tmpl_raw, pts, n, out) : 0;
  free(pts);
  return rc;
}

int oracle_map_f64(const uint8_t* img, int H, int W, int pitch, int nbins, const double* tab,
                   int w, int h, const double* tmpl_p, int x0, int y0, int x1, int y1,
                   double* out) {
  int32_t* pts; int n;
  if (dense_centres(H, W, w, h, x0, y0, x1, y1, &pts, &n)) return -1;
  int rc = n ? oracle_bc_f64(img, H, W, pitch, nbins, tab, w, h, tmpl_p, pts, n, out) : 0;
  free(pts);
  return rc;
}
