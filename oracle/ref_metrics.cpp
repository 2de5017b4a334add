/*
 * Oracle: quality metrics of Sec. III -- PSNR (Eq. 1) and SSIM (Eq. 2-3).
 * Test infrastructure only.  All sums in double, sequential.
 *
 * Readings for SSIM (Eq. 3 leaves the window open): uniform windows of
 * w^d points (w = 7), moved by one point, entirely inside the field (a
 * dimension shorter than w uses its full length); mean, variance and
 * covariance are population moments (divide by the window size);
 * c1 = (0.01 vrange)^2, c2 = (0.03 vrange)^2 with the range of X.
 */
#include <cmath>
#include <vector>
#include <cstring>
#include <limits>

#include "ref_internal.h"

using namespace qref;

namespace {

struct Sums {
  double x, y, xx, yy, xy;
};

inline double window_ssim(const Sums& s, double n, double c1, double c2) {
  double mx = s.x / n;
  double my = s.y / n;
  double vx = s.xx / n - mx * mx;
  double vy = s.yy / n - my * my;
  double cxy = s.xy / n - mx * my;
  double num = (2.0 * mx * my + c1) * (2.0 * cxy + c2);
  double den = (mx * mx + my * my + c1) * (vx + vy + c2);
  return num / den;
}

void window_extent(const Grid& g, int w, int64_t* we) {
  for (int i = 0; i < 3; ++i) we[i] = 1;
  for (int i = 0; i < g.d; ++i) we[i] = g.n[i] < w ? g.n[i] : w;
}

}  // namespace

namespace qref {

/* Separable window sums: along the last dimension, then the middle one,
 * then (3D) the first, each a sequential sum of w terms; planes along
 * dimension 0 are streamed through a ring of w0 planes. */
void ssim_separable_sums(const float* x, const float* y, const Grid& g,
                         int w, double vrange, double* sum, uint64_t* nwin) {
  double c1 = (0.01 * vrange) * (0.01 * vrange);
  double c2 = (0.03 * vrange) * (0.03 * vrange);
  /* view as [P][R][C]: 2D fields have one plane */
  int64_t P = g.d == 3 ? g.n[0] : 1;
  int64_t Rn = g.d == 3 ? g.n[1] : g.n[0];
  int64_t Cn = g.d == 3 ? g.n[2] : g.n[1];
  int64_t we[3];
  window_extent(g, w, we);
  int64_t wp = g.d == 3 ? we[0] : 1;
  int64_t wr = g.d == 3 ? we[1] : we[0];
  int64_t wc = g.d == 3 ? we[2] : we[1];
  int64_t oR = Rn - wr + 1, oC = Cn - wc + 1;
  double n = (double)(wp * wr * wc);
  std::vector<Sums> A((size_t)(Rn * oC));
  std::vector<Sums> ring((size_t)(wp * oR * oC));
  double total = 0.0;
  uint64_t count = 0;
  for (int64_t p = 0; p < P; ++p) {
    const float* xp = x + p * Rn * Cn;
    const float* yp = y + p * Rn * Cn;
    for (int64_t r = 0; r < Rn; ++r)
      for (int64_t c = 0; c < oC; ++c) {
        Sums s = {0, 0, 0, 0, 0};
        for (int64_t t = 0; t < wc; ++t) {
          double xv = xp[r * Cn + c + t], yv = yp[r * Cn + c + t];
          s.x += xv;
          s.y += yv;
          s.xx += xv * xv;
          s.yy += yv * yv;
          s.xy += xv * yv;
        }
        A[(size_t)(r * oC + c)] = s;
      }
    Sums* B = &ring[(size_t)((p % wp) * oR * oC)];
    for (int64_t r = 0; r < oR; ++r)
      for (int64_t c = 0; c < oC; ++c) {
        Sums s = {0, 0, 0, 0, 0};
        for (int64_t t = 0; t < wr; ++t) {
          const Sums& a = A[(size_t)((r + t) * oC + c)];
          s.x += a.x;
          s.y += a.y;
          s.xx += a.xx;
          s.yy += a.yy;
          s.xy += a.xy;
        }
        B[r * oC + c] = s;
      }
    if (p < wp - 1) continue;
    int64_t p0 = p - wp + 1;
    for (int64_t r = 0; r < oR; ++r)
      for (int64_t c = 0; c < oC; ++c) {
        Sums s = {0, 0, 0, 0, 0};
        for (int64_t t = 0; t < wp; ++t) {
          const Sums& b = ring[(size_t)((((p0 + t) % wp) * oR + r) * oC + c)];
          s.x += b.x;
          s.y += b.y;
          s.xx += b.xx;
          s.yy += b.yy;
          s.xy += b.xy;
        }
        total += window_ssim(s, n, c1, c2);
        ++count;
      }
  }
  *sum = total;
  *nwin = count;
}

}  // namespace qref

extern "C" int qref_ssim_direct(const float* x, const float* y,
                                qref_shape shape, uint32_t w, double vrange,
                                double* sum, uint64_t* nwin) {
  Grid g;
  if (!x || !y || !sum || !nwin || w < 1 || !shape_to_grid(shape, &g))
    return QREF_EINVAL;
  double c1 = (0.01 * vrange) * (0.01 * vrange);
  double c2 = (0.03 * vrange) * (0.03 * vrange);
  int64_t we[3];
  window_extent(g, (int)w, we);
  double n = (double)(we[0] * we[1] * we[2]);
  double total = 0.0;
  uint64_t count = 0;
  for (int64_t i0 = 0; i0 + we[0] <= g.n[0]; ++i0)
    for (int64_t i1 = 0; i1 + we[1] <= g.n[1]; ++i1)
      for (int64_t i2 = 0; i2 + we[2] <= g.n[2]; ++i2) {
        Sums s = {0, 0, 0, 0, 0};
        for (int64_t t0 = 0; t0 < we[0]; ++t0)
          for (int64_t t1 = 0; t1 < we[1]; ++t1)
            for (int64_t t2 = 0; t2 < we[2]; ++t2) {
              int64_t idx = (i0 + t0) * g.stride[0];
              if (g.d > 1) idx += (i1 + t1) * g.stride[1];
              if (g.d > 2) idx += (i2 + t2) * g.stride[2];
              double xv = x[idx], yv = y[idx];
              s.x += xv;
              s.y += yv;
              s.xx += xv * xv;
              s.yy += yv * yv;
              s.xy += xv * yv;
            }
        total += window_ssim(s, n, c1, c2);
        ++count;
      }
  *sum = total;
  *nwin = count;
  return QREF_OK;
}

extern "C" int qref_ssim_separable(const float* x, const float* y,
                                   qref_shape shape, uint32_t w,
                                   double vrange, double* sum,
                                   uint64_t* nwin) {
  Grid g;
  if (!x || !y || !sum || !nwin || w < 1 || !shape_to_grid(shape, &g))
    return QREF_EINVAL;
  ssim_separable_sums(x, y, g, (int)w, vrange, sum, nwin);
  return QREF_OK;
}

/* Eq. 1: PSNR = 20 log10(vrange / sqrt(mse)), vrange = max(X) - min(X). */
/* Eq. 4 with lag k = 1 along the fastest dimension: the mean and the
 * population variance of the errors over all points; the lagged moment
 * over every pair of neighbours in a row. */
double qref::ac_of_rows(const double* e, int64_t nrows, int64_t len) {
  const int64_t n = nrows * len;
  double mu = 0.0;
  for (int64_t i = 0; i < n; ++i) mu += e[i];
  mu /= (double)n;
  double var = 0.0;
  for (int64_t i = 0; i < n; ++i) var += (e[i] - mu) * (e[i] - mu);
  var /= (double)n;
  if (!(var > 0.0) || len < 2) return 0.0;
  double lag = 0.0;
  for (int64_t r = 0; r < nrows; ++r)
    for (int64_t k = 0; k + 1 < len; ++k)
      lag += (e[r * len + k] - mu) * (e[r * len + k + 1] - mu);
  lag /= (double)(nrows * (len - 1));
  return lag / var;
}

extern "C" int qref_error_ac(const float* x, const float* y, qref_shape shape,
                             double* ac) {
  Grid g;
  if (!x || !y || !ac || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  std::vector<double> e((size_t)g.N);
  for (int64_t i = 0; i < g.N; ++i) e[(size_t)i] = (double)x[i] - (double)y[i];
  const int64_t len = g.n[g.d - 1];
  *ac = ac_of_rows(e.data(), g.N / len, len);
  return QREF_OK;
}

extern "C" int qref_metrics(const float* x, const float* y, qref_shape shape,
                            uint32_t ssim_window, double* psnr, double* ssim,
                            double* max_abs_err) {
  Grid g;
  if (!x || !y || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  if (ssim_window == 0) ssim_window = 7;
  double vmin, vmax;
  value_range(x, g.N, &vmin, &vmax);
  double vrange = vmax - vmin;
  double sse = 0.0, mx = 0.0;
  for (int64_t i = 0; i < g.N; ++i) {
    double d = (double)x[i] - (double)y[i];
    sse += d * d;
    double a = std::fabs(d);
    if (a > mx) mx = a;
  }
  double mse = sse / (double)g.N;
  if (psnr)
    *psnr = mse == 0.0 ? std::numeric_limits<double>::infinity()
                       : 20.0 * std::log10(vrange / std::sqrt(mse));
  if (ssim) {
    double s;
    uint64_t nw;
    ssim_separable_sums(x, y, g, (int)ssim_window, vrange, &s, &nw);
    *ssim = s / (double)nw;
  }
  if (max_abs_err) *max_abs_err = mx;
  return QREF_OK;
}
