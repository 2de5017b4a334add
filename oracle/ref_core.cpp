/*
 * Oracle: multi-level interpolation predictor with level-wise error-bounded
 * linear quantization (Sec. V, Eq. 5).  Test infrastructure only.
 *
 * Readings of passages the paper leaves open (each listed in the design
 * notes) are marked "reading:" where they are taken.
 */
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>

#include "ref_internal.h"

namespace qref {

Grid make_grid(int d, const int64_t* n) {
  Grid g;
  g.d = d;
  for (int i = 0; i < 3; ++i) g.n[i] = 1;
  for (int i = 0; i < d; ++i) g.n[i] = n[i];
  int64_t st = 1;
  for (int i = d - 1; i >= 0; --i) {
    g.stride[i] = st;
    st *= g.n[i];
  }
  g.N = st;
  return g;
}

bool shape_to_grid(const qref_shape& s, Grid* g) {
  if (s.ndim != 2 && s.ndim != 3) return false;
  int64_t n[3];
  double total = 1.0;
  for (uint32_t i = 0; i < s.ndim; ++i) {
    if (s.dims[i] < 2 || s.dims[i] > (uint64_t)1 << 31) return false;
    n[i] = (int64_t)s.dims[i];
    total *= (double)s.dims[i];
  }
  /* element indices must fit 32 bits */
  if (total >= 4294967296.0) return false;
  *g = make_grid((int)s.ndim, n);
  return true;
}

/* Eq. 5: e_l = e / min(alpha^(l-1), beta), l = 1..L.  alpha^(l-1) is formed
 * by repeated multiplication.  Reading: the quantizer works in FP32 with a
 * bin width of 2 e_l, so each level also carries (float)(2 e_l) and
 * (float)(1 / (2 e_l)), both rounded once from double. */
void bounds_eq5(double e, double alpha, double beta, int L, LevelBounds* b) {
  double p = 1.0;
  for (int l = 1; l <= L; ++l) {
    if (l > 1) p = p * alpha;
    double m = p < beta ? p : beta;
    double el = e / m;
    b->eb[l - 1] = el;
    b->twoeb[l - 1] = (float)(2.0 * el);
    b->inv[l - 1] = (float)(1.0 / (2.0 * el));
  }
}

/* Algorithm 1 runs its trials at the user bound e on every level. */
void bounds_uniform(double e, int L, LevelBounds* b) {
  for (int l = 1; l <= L; ++l) {
    b->eb[l - 1] = e;
    b->twoeb[l - 1] = (float)(2.0 * e);
    b->inv[l - 1] = (float)(1.0 / (2.0 * e));
  }
}

/* Interpolation along one dimension at a midpoint (Sec. V-B: linear or cubic
 * spline).  a, b, c, d are the reconstructed values at -3h, -h, +h, +3h.
 * Reading: "cubic spline" is the 4-point midpoint rule (-1, 9, 9, -1)/16;
 * near an edge the available points give the one-sided quadratic
 * (3, 6, -1)/8 or (-1, 6, 3)/8, then the two-point mean; with no point at
 * +h, linear extrapolation (3b - a)/2, else a copy of b.  Every operation is
 * a separately rounded FP32 operation in the order written. */
float stencil(int cubic, float a, float b, float c, float d, bool has_a,
              bool has_c, bool has_d) {
  if (!has_c) {
    if (has_a) {
      float t = b * 3.0f;
      t = t - a;
      return t * 0.5f;
    }
    return b;
  }
  if (cubic) {
    if (has_a && has_d) {
      float s1 = b + c;
      float s2 = s1 * 9.0f;
      float s3 = a + d;
      float s4 = s2 - s3;
      return s4 * 0.0625f;
    }
    if (!has_a && has_d) {
      float t1 = b * 3.0f;
      float t2 = c * 6.0f;
      float t3 = t1 + t2;
      float t4 = t3 - d;
      return t4 * 0.125f;
    }
    if (has_a && !has_d) {
      float t1 = b * 6.0f;
      float t2 = c * 3.0f;
      float t3 = t1 + t2;
      float t4 = t3 - a;
      return t4 * 0.125f;
    }
  }
  float s = b + c;
  return s * 0.5f;
}

int64_t count_anchors(const Grid& g, int64_t s) {
  int64_t c = 1;
  for (int i = 0; i < g.d; ++i) c *= (g.n[i] - 1) / s + 1;
  return c;
}

/* Anchor points (Sec. V-B): every point whose coordinates are all multiples
 * of the stride s is known in advance and stored losslessly. */
void place_anchors(const float* x, const Grid& g, int64_t s, float* W,
                   std::vector<float>* anchors) {
  for (int64_t i0 = 0; i0 < g.n[0]; i0 += (g.d > 0 ? s : 1))
    for (int64_t i1 = 0; i1 < g.n[1]; i1 += (g.d > 1 ? s : 1))
      for (int64_t i2 = 0; i2 < g.n[2]; i2 += (g.d > 2 ? s : 1)) {
        int64_t idx = i0 * g.stride[0] + (g.d > 1 ? i1 * g.stride[1] : 0) +
                      (g.d > 2 ? i2 * g.stride[2] : 0);
        W[idx] = x[idx];
        if (anchors) anchors->push_back(x[idx]);
      }
}

namespace {

/* Target set of sweep j of level l (Sec. V-A, "along another dimension
 * alternatively"): along k = order[j] the coordinate is an odd multiple of
 * h; dimensions swept earlier in this level are multiples of h; dimensions
 * swept later are multiples of 2h.  Reading: every sweep covers the whole
 * field; targets are visited in row-major order of this sub-grid. */
void target_grid(const Grid& g, const int* order, int j, int64_t h,
                 int64_t* start, int64_t* step, int64_t* cnt) {
  for (int m = 0; m < 3; ++m) {
    start[m] = 0;
    step[m] = 1;
    cnt[m] = 1;
  }
  for (int pos = 0; pos < g.d; ++pos) {
    int m = order[pos];
    if (pos == j) {
      start[m] = h;
      step[m] = 2 * h;
    } else if (pos < j) {
      start[m] = 0;
      step[m] = h;
    } else {
      start[m] = 0;
      step[m] = 2 * h;
    }
    cnt[m] = start[m] <= g.n[m] - 1 ? (g.n[m] - 1 - start[m]) / step[m] + 1
                                     : 0;
  }
}

struct Neigh {
  float a, b, c, d;
  bool has_a, has_c, has_d;
};

inline Neigh gather(const float* W, const Grid& g, int64_t idx, int k,
                    int64_t pk, int64_t h) {
  Neigh r;
  int64_t sk = g.stride[k];
  int64_t nk = g.n[k];
  r.has_a = pk >= 3 * h;
  r.has_c = pk + h <= nk - 1;
  r.has_d = pk + 3 * h <= nk - 1;
  r.b = W[idx - h * sk];
  r.a = r.has_a ? W[idx - 3 * h * sk] : 0.0f;
  r.c = r.has_c ? W[idx + h * sk] : 0.0f;
  r.d = r.has_d ? W[idx + 3 * h * sk] : 0.0f;
  return r;
}

}  // namespace

/* Linear-scale quantization of one target (Sec. V-A).  Reading: bin width
 * 2 e_l, round half to even, R = 32768 bins on each side; a target whose bin
 * falls outside, or whose FP32 reconstruction misses x by more than e_l
 * (checked in double), is unpredictable: bin 0, the exact value is kept. */
static inline int32_t quantize(float x, float pred, float inv, float twoeb,
                               double eb, float* recon) {
  const float R = (float)QREF_RADIUS;
  float diff = x - pred;
  float qf = diff * inv;
  if (!(std::fabs(qf) < R)) {
    *recon = x;
    return 0;
  }
  float qr = std::rint(qf);
  int32_t q = (int32_t)qr;
  if (q >= QREF_RADIUS || q <= -QREF_RADIUS) {
    *recon = x;
    return 0;
  }
  float t = (float)q * twoeb;
  float r = pred + t;
  double err = std::fabs((double)r - (double)x);
  if (!(err <= eb)) {
    *recon = x;
    return 0;
  }
  *recon = r;
  return q + QREF_RADIUS;
}

void compress_levels(const float* x, const Grid& g, int l_hi, int l_lo,
                     const LevelPlan& plan, const LevelBounds& lb, float* W,
                     SweepSink* sink) {
  for (int l = l_hi; l >= l_lo; --l) {
    int64_t h = (int64_t)1 << (l - 1);
    const int* order = plan.order[l - 1];
    int cubic = plan.interp[l - 1];
    float inv = lb.inv[l - 1], twoeb = lb.twoeb[l - 1];
    double eb = lb.eb[l - 1];
    for (int j = 0; j < g.d; ++j) {
      int k = order[j];
      int64_t start[3], step[3], cnt[3];
      target_grid(g, order, j, h, start, step, cnt);
      for (int64_t a0 = 0; a0 < cnt[0]; ++a0)
        for (int64_t a1 = 0; a1 < cnt[1]; ++a1)
          for (int64_t a2 = 0; a2 < cnt[2]; ++a2) {
            int64_t p[3] = {start[0] + a0 * step[0], start[1] + a1 * step[1],
                            start[2] + a2 * step[2]};
            int64_t idx = 0;
            for (int m = 0; m < g.d; ++m) idx += p[m] * g.stride[m];
            Neigh nb = gather(W, g, idx, k, p[k], h);
            float pred = stencil(cubic, nb.a, nb.b, nb.c, nb.d, nb.has_a,
                                 nb.has_c, nb.has_d);
            float xv = x[idx];
            if (sink->l1_level == l) {
              sink->l1_sum += std::fabs((double)xv - (double)pred);
              sink->l1_count += 1;
            }
            float r;
            int32_t code = quantize(xv, pred, inv, twoeb, eb, &r);
            W[idx] = r;
            sink->n_codes += 1;
            if (code == 0) {
              sink->n_unpred += 1;
              if (sink->unpred) sink->unpred->push_back(xv);
            }
            if (sink->codes) sink->codes->push_back(code);
            if (sink->hist) sink->hist[code] += 1;
            if (sink->targets) sink->targets->push_back((uint32_t)idx);
            if (sink->preds) sink->preds->push_back(pred);
          }
    }
  }
}

bool decompress_levels(const Grid& g, int L, const LevelPlan& plan,
                       const LevelBounds& lb, const int32_t* codes,
                       uint64_t n_codes, const float* unpred,
                       uint64_t n_unpred, float* W) {
  uint64_t ci = 0, ui = 0;
  for (int l = L; l >= 1; --l) {
    int64_t h = (int64_t)1 << (l - 1);
    const int* order = plan.order[l - 1];
    int cubic = plan.interp[l - 1];
    float twoeb = lb.twoeb[l - 1];
    for (int j = 0; j < g.d; ++j) {
      int k = order[j];
      int64_t start[3], step[3], cnt[3];
      target_grid(g, order, j, h, start, step, cnt);
      for (int64_t a0 = 0; a0 < cnt[0]; ++a0)
        for (int64_t a1 = 0; a1 < cnt[1]; ++a1)
          for (int64_t a2 = 0; a2 < cnt[2]; ++a2) {
            int64_t p[3] = {start[0] + a0 * step[0], start[1] + a1 * step[1],
                            start[2] + a2 * step[2]};
            int64_t idx = 0;
            for (int m = 0; m < g.d; ++m) idx += p[m] * g.stride[m];
            if (ci >= n_codes) return false;
            int32_t code = codes[ci++];
            if (code == 0) {
              if (ui >= n_unpred) return false;
              W[idx] = unpred[ui++];
              continue;
            }
            Neigh nb = gather(W, g, idx, k, p[k], h);
            float pred = stencil(cubic, nb.a, nb.b, nb.c, nb.d, nb.has_a,
                                 nb.has_c, nb.has_d);
            float t = (float)(code - QREF_RADIUS) * twoeb;
            W[idx] = pred + t;
          }
    }
  }
  return ci == n_codes && ui == n_unpred;
}

bool validate_params(const qref_params& p, int d, int* L) {
  uint32_t s = p.anchor_stride;
  if (s < 2 || (s & (s - 1)) != 0) return false;
  int l = 0;
  while (((uint32_t)1 << l) < s) ++l;
  if (l > QREF_MAX_LEVELS) return false;
  for (int i = 0; i < l; ++i) {
    if (p.interp[i] > 1) return false;
    int seen = 0;
    for (int j = 0; j < d; ++j) {
      int m = p.order[i][j];
      if (m < 0 || m >= d || (seen >> m) & 1) return false;
      seen |= 1 << m;
    }
  }
  if (!(p.alpha >= 1.0) || !(p.beta >= 1.0)) return false;
  if (!std::isfinite(p.alpha) || !std::isfinite(p.beta)) return false;
  *L = l;
  return true;
}

bool all_finite(const float* x, int64_t N) {
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

void value_range(const float* x, int64_t N, double* vmin, double* vmax) {
  float lo = x[0], hi = x[0];
  for (int64_t i = 1; i < N; ++i) {
    if (x[i] < lo) lo = x[i];
    if (x[i] > hi) hi = x[i];
  }
  *vmin = lo;
  *vmax = hi;
}

}  // namespace qref

using namespace qref;

static void plan_from_params(const qref_params& p, int L, LevelPlan* plan) {
  for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
    plan->interp[l] = l < L ? p.interp[l] : 0;
    for (int j = 0; j < 3; ++j) plan->order[l][j] = l < L ? p.order[l][j] : j;
  }
}

extern "C" int qref_level_bounds(double e, double alpha, double beta,
                                 uint32_t L, double* e_l, float* twoeb,
                                 float* inv) {
  if (!(e > 0.0) || !std::isfinite(e) || !(alpha >= 1.0) || !(beta >= 1.0) ||
      L < 1 || L > QREF_MAX_LEVELS)
    return QREF_EINVAL;
  LevelBounds b;
  bounds_eq5(e, alpha, beta, (int)L, &b);
  for (uint32_t l = 0; l < L; ++l) {
    if (e_l) e_l[l] = b.eb[l];
    if (twoeb) twoeb[l] = b.twoeb[l];
    if (inv) inv[l] = b.inv[l];
  }
  return QREF_OK;
}

extern "C" float qref_stencil(int cubic, float a, float b, float c, float d,
                              int has_a, int has_c, int has_d) {
  return stencil(cubic, a, b, c, d, has_a != 0, has_c != 0, has_d != 0);
}

extern "C" int qref_predict_quantize(const float* x, qref_shape shape,
                                     double e, const qref_params* params,
                                     int32_t* codes, float* recon,
                                     float* unpred, float* anchors,
                                     uint64_t* n_codes, uint64_t* n_unpred,
                                     uint64_t* n_anchor) {
  Grid g;
  if (!x || !params || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  if (!(e > 0.0) || !std::isfinite(e)) return QREF_EINVAL;
  qref_params p = *params;
  if (p.anchor_stride == 0) p.anchor_stride = g.d == 2 ? 64 : 32;
  int L;
  if (!validate_params(p, g.d, &L)) return QREF_EINVAL;
  if (!all_finite(x, g.N)) return QREF_EINVAL;
  LevelPlan plan;
  plan_from_params(p, L, &plan);
  LevelBounds lb;
  bounds_eq5(e, p.alpha, p.beta, L, &lb);
  std::vector<float> W((size_t)g.N, std::numeric_limits<float>::quiet_NaN());
  std::vector<float> anc, un;
  std::vector<int32_t> cd;
  place_anchors(x, g, p.anchor_stride, W.data(), &anc);
  SweepSink sink;
  sink.codes = &cd;
  sink.unpred = &un;
  compress_levels(x, g, L, 1, plan, lb, W.data(), &sink);
  if (codes) copy_bytes(codes, cd.data(), cd.size() * sizeof(int32_t));
  if (recon) copy_bytes(recon, W.data(), W.size() * sizeof(float));
  if (unpred) copy_bytes(unpred, un.data(), un.size() * sizeof(float));
  if (anchors) copy_bytes(anchors, anc.data(), anc.size() * sizeof(float));
  *n_codes = cd.size();
  *n_unpred = un.size();
  *n_anchor = anc.size();
  return QREF_OK;
}

extern "C" int qref_reconstruct(const int32_t* codes, uint64_t n_codes,
                                const float* unpred, uint64_t n_unpred,
                                const float* anchors, uint64_t n_anchor,
                                qref_shape shape, double e,
                                const qref_params* params, float* y) {
  Grid g;
  if (!params || !y || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  qref_params p = *params;
  if (p.anchor_stride == 0) p.anchor_stride = g.d == 2 ? 64 : 32;
  int L;
  if (!validate_params(p, g.d, &L)) return QREF_EINVAL;
  int64_t s = p.anchor_stride;
  if ((int64_t)n_anchor != count_anchors(g, s)) return QREF_EINVAL;
  if (!(e > 0.0) || !std::isfinite(e)) return QREF_EINVAL;
  LevelPlan plan;
  plan_from_params(p, L, &plan);
  LevelBounds lb;
  bounds_eq5(e, p.alpha, p.beta, L, &lb);
  for (int64_t i = 0; i < g.N; ++i)
    y[i] = std::numeric_limits<float>::quiet_NaN();
  /* scatter anchors in row-major order */
  uint64_t ai = 0;
  for (int64_t i0 = 0; i0 < g.n[0]; i0 += s)
    for (int64_t i1 = 0; i1 < g.n[1]; i1 += (g.d > 1 ? s : 1))
      for (int64_t i2 = 0; i2 < g.n[2]; i2 += (g.d > 2 ? s : 1)) {
        int64_t idx = i0 * g.stride[0] + (g.d > 1 ? i1 * g.stride[1] : 0) +
                      (g.d > 2 ? i2 * g.stride[2] : 0);
        y[idx] = anchors[ai++];
      }
  if (!decompress_levels(g, L, plan, lb, codes, n_codes, unpred, n_unpred, y))
    return QREF_EFORMAT;
  return QREF_OK;
}

/* Stream-order trace of the compression sweeps: flat index, prediction and
 * bin of every target (for tests). */
extern "C" int qref_target_trace(const float* x, qref_shape shape, double e,
                                 const qref_params* params, uint32_t* idx,
                                 float* pred, int32_t* codes,
                                 uint64_t* n_codes) {
  Grid g;
  if (!x || !params || !n_codes || !shape_to_grid(shape, &g))
    return QREF_EINVAL;
  if (!(e > 0.0) || !std::isfinite(e)) return QREF_EINVAL;
  qref_params p = *params;
  if (p.anchor_stride == 0) p.anchor_stride = g.d == 2 ? 64 : 32;
  int L;
  if (!validate_params(p, g.d, &L)) return QREF_EINVAL;
  LevelPlan plan;
  plan_from_params(p, L, &plan);
  LevelBounds lb;
  bounds_eq5(e, p.alpha, p.beta, L, &lb);
  std::vector<float> W((size_t)g.N, std::numeric_limits<float>::quiet_NaN());
  place_anchors(x, g, p.anchor_stride, W.data(), nullptr);
  std::vector<uint32_t> ti;
  std::vector<float> pr;
  std::vector<int32_t> cd;
  SweepSink sink;
  sink.targets = &ti;
  sink.preds = &pr;
  sink.codes = &cd;
  compress_levels(x, g, L, 1, plan, lb, W.data(), &sink);
  if (idx) copy_bytes(idx, ti.data(), ti.size() * sizeof(uint32_t));
  if (pred) copy_bytes(pred, pr.data(), pr.size() * sizeof(float));
  if (codes) copy_bytes(codes, cd.data(), cd.size() * sizeof(int32_t));
  *n_codes = ti.size();
  return QREF_OK;
}
