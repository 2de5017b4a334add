/*
 * Oracle: the online tuner of Sec. VI -- uniform block sampling (Sec. VI-A),
 * level-adapted interpolator selection (Algorithm 1, Sec. VI-B) and the
 * (alpha, beta) search with the rate-quality comparison of Table I
 * (Sec. VI-C).  Test infrastructure only.
 *
 * Readings:
 *  - Sampling: block size b, stride S = round(b r^(-1/d)); origins at k*S
 *    along each dimension while k*S + b <= n-1; a block spans b+1 points per
 *    dimension and its points on the 2^Lt grid are known exactly.  If no
 *    block fits along some dimension, the whole field is the one block.
 *  - A trial on a block is the same predictor and quantizer applied to the
 *    block as a field of its own, with anchor stride 2^Lt and Lt levels.
 *  - Algorithm 1 compares candidates at the user bound e on every level,
 *    with the higher levels already fixed to their chosen interpolators;
 *    the L1 error is |x - prediction| before quantization; the first
 *    strictly smaller mean wins.
 *  - The bit rate of a trial is (Huffman bits of the bins aggregated over
 *    all blocks + 32 per unpredictable value) / points in the blocks; the
 *    dictionary stage is not part of the estimate.
 *  - Table I: the incumbent I starts as the first (alpha, beta) pair and is
 *    challenged by each later pair II in order (alpha outer, beta inner).
 *    Case 3 re-runs II at 0.8e and case 4 at 1.2e, as the table states (the
 *    prose states the opposite assignment; the table's choice is the one
 *    that brackets B_I between B_II and B'_II).  On the line or with a
 *    degenerate line I is kept.  In ratio mode M is 0 for every trial.
 *  - PSNR of a trial uses the global value range of X.
 *  - AC target (Eq. 4): lag 1 along the fastest dimension; a trial's AC
 *    takes the mean and variance over all block points and the lagged
 *    moment over the blocks' rows; M = -|AC| (the paper prefers errors as
 *    uncorrelated as possible).
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "ref_internal.h"

using namespace qref;

namespace {

const double kAlphas[5] = {1.0, 1.25, 1.5, 1.75, 2.0};
const double kBetas[4] = {1.5, 2.0, 3.0, 4.0};

struct Sample {
  uint32_t b = 0, S = 0, Lt = 0;
  Grid bg;                          /* block grid */
  std::vector<std::vector<float>> blocks;
  std::vector<int64_t> origins;     /* d per block */
};

int ilog2(uint32_t v) {
  int l = 0;
  while (((uint32_t)1 << (l + 1)) <= v) ++l;
  return l;
}

int make_plan(const Grid& g, uint32_t s, const qref_tune_config* cfg,
              Sample* sp, bool extract, const float* x) {
  uint32_t b = (cfg && cfg->block) ? cfg->block : (g.d == 2 ? 64u : 16u);
  if (b < 2 || (b & (b - 1)) != 0) return QREF_EINVAL;
  double r = (cfg && cfg->sample_rate > 0.0) ? cfg->sample_rate
                                             : (g.d == 2 ? 0.01 : 0.005);
  if (!(r > 0.0) || !(r <= 1.0)) return QREF_EINVAL;
  uint32_t S = (cfg && cfg->sample_stride)
                   ? cfg->sample_stride
                   : (uint32_t)std::llround((double)b *
                                            std::pow(r, -1.0 / g.d));
  if (S < 1) S = 1;
  sp->b = b;
  sp->S = S;
  sp->Lt = (uint32_t)ilog2(std::min(b, s));
  int64_t m[3] = {1, 1, 1};
  bool whole = false;
  for (int i = 0; i < g.d; ++i) {
    m[i] = 0;
    while ((int64_t)(m[i] * S + b) <= g.n[i] - 1) ++m[i];
    if (m[i] == 0) whole = true;
  }
  int64_t bn[3];
  if (whole) {
    for (int i = 0; i < g.d; ++i) bn[i] = g.n[i];
    for (int i = 0; i < 3; ++i) m[i] = 1;
  } else {
    for (int i = 0; i < g.d; ++i) bn[i] = (int64_t)b + 1;
  }
  sp->bg = make_grid(g.d, bn);
  sp->origins.clear();
  sp->blocks.clear();
  for (int64_t k0 = 0; k0 < m[0]; ++k0)
    for (int64_t k1 = 0; k1 < (g.d > 1 ? m[1] : 1); ++k1)
      for (int64_t k2 = 0; k2 < (g.d > 2 ? m[2] : 1); ++k2) {
        int64_t o[3] = {whole ? 0 : k0 * S, whole ? 0 : k1 * S,
                        whole ? 0 : k2 * S};
        for (int i = 0; i < g.d; ++i) sp->origins.push_back(o[i]);
        if (!extract) continue;
        std::vector<float> blk((size_t)sp->bg.N);
        for (int64_t i0 = 0; i0 < sp->bg.n[0]; ++i0)
          for (int64_t i1 = 0; i1 < sp->bg.n[1]; ++i1)
            for (int64_t i2 = 0; i2 < sp->bg.n[2]; ++i2) {
              int64_t src = (o[0] + i0) * g.stride[0];
              if (g.d > 1) src += (o[1] + i1) * g.stride[1];
              if (g.d > 2) src += (o[2] + i2) * g.stride[2];
              int64_t dst = i0 * sp->bg.stride[0];
              if (g.d > 1) dst += i1 * sp->bg.stride[1];
              if (g.d > 2) dst += i2 * sp->bg.stride[2];
              blk[(size_t)dst] = x[src];
            }
        sp->blocks.push_back(std::move(blk));
      }
  return QREF_OK;
}

struct Cand {
  int interp;
  int order[3];
};

std::vector<Cand> candidates(int d, bool all_orders) {
  std::vector<std::vector<int>> orders;
  if (all_orders) {
    std::vector<int> p(d);
    for (int i = 0; i < d; ++i) p[i] = i;
    do orders.push_back(p);
    while (std::next_permutation(p.begin(), p.end()));
  } else {
    std::vector<int> inc(d), dec(d);
    for (int i = 0; i < d; ++i) {
      inc[i] = i;
      dec[i] = d - 1 - i;
    }
    orders.push_back(inc);
    orders.push_back(dec);
  }
  std::vector<Cand> out;
  for (int t = 0; t < 2; ++t)
    for (auto& o : orders) {
      Cand c;
      c.interp = t;
      for (int i = 0; i < 3; ++i) c.order[i] = i < d ? o[i] : i;
      out.push_back(c);
    }
  return out;
}

/* Trial compression of every sampled block with one parameter set. */
void run_trial(const Sample& sp, const LevelPlan& plan, const LevelBounds& lb,
               double vrange, bool want_ssim, bool want_ac, int w,
               qref_trial_result* res) {
  const uint32_t nsym = 2 * QREF_RADIUS;
  std::vector<uint64_t> hist(nsym, 0);
  std::memset(res, 0, sizeof(*res));
  int64_t st = (int64_t)1 << sp.Lt;
  std::vector<float> W((size_t)sp.bg.N);
  std::vector<double> errs; /* every block's errors, block after block */
  for (const auto& blk : sp.blocks) {
    std::fill(W.begin(), W.end(), std::numeric_limits<float>::quiet_NaN());
    place_anchors(blk.data(), sp.bg, st, W.data(), nullptr);
    SweepSink sink;
    sink.hist = hist.data();
    compress_levels(blk.data(), sp.bg, (int)sp.Lt, 1, plan, lb, W.data(),
                    &sink);
    res->n_unpred += sink.n_unpred;
    res->n_codes += sink.n_codes;
    for (int64_t i = 0; i < sp.bg.N; ++i) {
      double d = (double)blk[(size_t)i] - (double)W[(size_t)i];
      res->sse += d * d;
      if (want_ac) errs.push_back(d);
    }
    res->n_points += (uint64_t)sp.bg.N;
    if (want_ssim) {
      double s;
      uint64_t nw;
      ssim_separable_sums(blk.data(), W.data(), sp.bg, w, vrange, &s, &nw);
      res->ssim_sum += s;
      res->n_windows += nw;
    }
  }
  if (want_ac) {
    /* the blocks' rows (along the fastest dimension) together */
    const int64_t rl = sp.bg.n[sp.bg.d - 1];
    res->ac = ac_of_rows(errs.data(), (int64_t)errs.size() / rl, rl);
  }
  std::vector<uint8_t> len(nsym);
  huffman_lengths(hist.data(), nsym, len.data());
  res->payload_bits = huffman_bits(hist.data(), len.data(), nsym);
  res->B = ((double)res->payload_bits + 32.0 * (double)res->n_unpred) /
           (double)res->n_points;
}

double metric_of(const qref_trial_result& r, int target, double vrange) {
  if (target == QREF_TARGET_PSNR) {
    if (r.sse == 0.0) return std::numeric_limits<double>::infinity();
    return 20.0 * std::log10(vrange / std::sqrt(r.sse / (double)r.n_points));
  }
  if (target == QREF_TARGET_SSIM) return r.ssim_sum / (double)r.n_windows;
  /* errors closest to uncorrelated are best (Eq. 4) */
  if (target == QREF_TARGET_AC) return -std::fabs(r.ac);
  return 0.0;
}

void plan_from(const qref_params& p, int L, LevelPlan* plan) {
  for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
    plan->interp[l] = l < L ? p.interp[l] : 0;
    for (int j = 0; j < 3; ++j) plan->order[l][j] = l < L ? p.order[l][j] : j;
  }
}

}  // namespace

extern "C" int qref_table1_case(double BI, double MI, double BII, double MII) {
  if (BI <= BII && MI >= MII) return 1;
  if (BI >= BII && MI <= MII) return 2;
  if (BI > BII && MI > MII) return 3;
  return 4;
}

extern "C" int qref_table1_line(double BI, double MI, double BII, double MII,
                                double BIIp, double MIIp) {
  if (BIIp == BII) return 0;
  double rise = (MIIp - MII) * (BI - BII);
  double Mline = MII + rise / (BIIp - BII);
  return MI < Mline ? 1 : 0;
}

extern "C" int qref_sample_plan(qref_shape shape, uint32_t anchor_stride,
                                const qref_tune_config* cfg, uint32_t* b,
                                uint32_t* S, uint32_t* Lt, uint64_t* nblocks,
                                uint64_t* block_dims, uint64_t* origins,
                                uint64_t origins_cap) {
  Grid g;
  if (!shape_to_grid(shape, &g)) return QREF_EINVAL;
  uint32_t s = anchor_stride ? anchor_stride : (g.d == 2 ? 64u : 32u);
  if (s < 2 || (s & (s - 1)) != 0) return QREF_EINVAL;
  Sample sp;
  int rc = make_plan(g, s, cfg, &sp, false, nullptr);
  if (rc != QREF_OK) return rc;
  if (b) *b = sp.b;
  if (S) *S = sp.S;
  if (Lt) *Lt = sp.Lt;
  if (nblocks) *nblocks = sp.origins.size() / g.d;
  if (block_dims)
    for (int i = 0; i < 3; ++i) block_dims[i] = (uint64_t)sp.bg.n[i];
  if (origins)
    for (size_t i = 0; i < sp.origins.size() && i < origins_cap; ++i)
      origins[i] = (uint64_t)sp.origins[i];
  return QREF_OK;
}

extern "C" int qref_trial(const float* x, qref_shape shape, double e_trial,
                          const qref_params* theta,
                          const qref_tune_config* cfg, double vrange,
                          uint32_t want, qref_trial_result* res) {
  Grid g;
  if (!x || !theta || !res || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  int L;
  if (!validate_params(*theta, g.d, &L)) return QREF_EINVAL;
  if (!(e_trial > 0.0)) return QREF_EINVAL;
  Sample sp;
  int rc = make_plan(g, theta->anchor_stride, cfg, &sp, true, x);
  if (rc != QREF_OK) return rc;
  LevelPlan plan;
  plan_from(*theta, L, &plan);
  LevelBounds lb;
  bounds_eq5(e_trial, theta->alpha, theta->beta, (int)sp.Lt, &lb);
  int w = (cfg && cfg->ssim_window) ? (int)cfg->ssim_window : 7;
  run_trial(sp, plan, lb, vrange, (want & 1u) != 0, (want & 2u) != 0, w,
            res);
  return QREF_OK;
}

extern "C" int qref_tune(const float* x, qref_shape shape, double e,
                         int target, const qref_tune_config* cfg,
                         qref_params* out, qref_tune_trace* trace) {
  Grid g;
  if (!x || !out || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  if (!(e > 0.0) || !std::isfinite(e)) return QREF_EINVAL;
  if (target < QREF_TARGET_CR || target > QREF_TARGET_AC) return QREF_EINVAL;
  if (cfg && (cfg->ablation & ~(QREF_ABLATE_AB | QREF_ABLATE_LEVELWISE)))
    return QREF_EINVAL;
  /* A ratio-target tuning reads only the sampled blocks (Sec. VI-A), so
   * only their values must be finite; the quality targets also use the
   * whole field's value range (Eq. 1-3) and check every value. */
  const bool ratio = target == QREF_TARGET_CR;
  if (!ratio && !all_finite(x, g.N)) return QREF_EINVAL;
  uint32_t s = out->anchor_stride ? out->anchor_stride : (g.d == 2 ? 64u : 32u);
  if (s < 2 || (s & (s - 1)) != 0) return QREF_EINVAL;
  int L = ilog2(s);
  if (L > QREF_MAX_LEVELS) return QREF_EINVAL;
  Sample sp;
  int rc = make_plan(g, s, cfg, &sp, true, x);
  if (rc != QREF_OK) return rc;
  if (ratio)
    for (const std::vector<float>& blk : sp.blocks)
      if (!all_finite(blk.data(), (int64_t)blk.size())) return QREF_EINVAL;
  int Lt = (int)sp.Lt;
  int w = (cfg && cfg->ssim_window) ? (int)cfg->ssim_window : 7;
  double vmin = 0.0, vmax = 0.0; /* unused by the ratio target */
  if (!ratio) value_range(x, g.N, &vmin, &vmax);
  double vrange = vmax - vmin;
  std::vector<Cand> cands = candidates(g.d, cfg && cfg->all_orders);
  if (trace) {
    std::memset(trace, 0, sizeof(*trace));
    trace->Lt = (uint32_t)Lt;
    trace->ncand = (uint32_t)cands.size();
    trace->nblocks = sp.blocks.size();
    trace->block_points = sp.blocks.size() * (uint64_t)sp.bg.N;
  }

  const uint32_t abl = cfg ? cfg->ablation : 0u;
  /* Algorithm 1 */
  LevelPlan Is;
  for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
    Is.interp[l] = 0;
    for (int j = 0; j < 3; ++j) Is.order[l][j] = j;
  }
  LevelBounds ub;
  bounds_uniform(e, Lt, &ub);
  int64_t st = (int64_t)1 << Lt;
  std::vector<float> W((size_t)sp.bg.N);
  if (abl & QREF_ABLATE_LEVELWISE) {
    /* one interpolator for the whole field: the candidate whose trial
     * compression of the sampled blocks (every level, uniform bound e)
     * has the lowest bit rate, the first on ties */
    double best = std::numeric_limits<double>::infinity();
    int ib = 0;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      LevelPlan pl;
      for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
        pl.interp[l] = cands[ci].interp;
        for (int j = 0; j < 3; ++j) pl.order[l][j] = cands[ci].order[j];
      }
      qref_trial_result r;
      run_trial(sp, pl, ub, vrange, false, false, w, &r);
      if (trace) trace->alg1_err[0][ci] = r.B;
      if (r.B < best) {
        best = r.B;
        ib = (int)ci;
      }
    }
    for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
      Is.interp[l] = cands[ib].interp;
      for (int j = 0; j < 3; ++j) Is.order[l][j] = cands[ib].order[j];
      if (trace && l < Lt) trace->alg1_choice[l] = (uint32_t)ib;
    }
  }
  for (int l = (abl & QREF_ABLATE_LEVELWISE) ? 0 : Lt; l >= 1; --l) {
    double best = std::numeric_limits<double>::infinity();
    int ib = 0;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      LevelPlan pl = Is;
      pl.interp[l - 1] = cands[ci].interp;
      for (int j = 0; j < 3; ++j) pl.order[l - 1][j] = cands[ci].order[j];
      double sum = 0.0;
      uint64_t cnt = 0;
      for (const auto& blk : sp.blocks) {
        std::fill(W.begin(), W.end(), std::numeric_limits<float>::quiet_NaN());
        place_anchors(blk.data(), sp.bg, st, W.data(), nullptr);
        SweepSink sink;
        sink.l1_level = l;
        compress_levels(blk.data(), sp.bg, Lt, l, pl, ub, W.data(), &sink);
        sum += sink.l1_sum;
        cnt += sink.l1_count;
      }
      double cur = cnt ? sum / (double)cnt : 0.0;
      if (trace) trace->alg1_err[l - 1][ci] = cur;
      if (cur < best) {
        best = cur;
        ib = (int)ci;
      }
    }
    Is.interp[l - 1] = cands[ib].interp;
    for (int j = 0; j < 3; ++j) Is.order[l - 1][j] = cands[ib].order[j];
    if (trace) trace->alg1_choice[l - 1] = (uint32_t)ib;
  }
  /* levels above the sampled blocks reuse the choice at Lt */
  for (int l = Lt + 1; l <= L; ++l) {
    Is.interp[l - 1] = Is.interp[Lt - 1];
    for (int j = 0; j < 3; ++j) Is.order[l - 1][j] = Is.order[Lt - 1][j];
  }

  /* (alpha, beta) search with Table I; without it the first pair, whose
   * alpha = 1 gives every level the bound e */
  const int npairs = (abl & QREF_ABLATE_AB) ? 1 : QREF_NPAIRS;
  bool want_ssim = target == QREF_TARGET_SSIM;
  bool want_ac = target == QREF_TARGET_AC;
  double B[QREF_NPAIRS], M[QREF_NPAIRS];
  for (int i = 0; i < npairs; ++i) {
    LevelBounds lb;
    bounds_eq5(e, kAlphas[i / 4], kBetas[i % 4], Lt, &lb);
    qref_trial_result r;
    run_trial(sp, Is, lb, vrange, want_ssim, want_ac, w, &r);
    B[i] = r.B;
    M[i] = metric_of(r, target, vrange);
    if (trace) {
      trace->B[i] = B[i];
      trace->M[i] = M[i];
      trace->Bp[i] = std::numeric_limits<double>::quiet_NaN();
      trace->Mp[i] = std::numeric_limits<double>::quiet_NaN();
      trace->eprime[i] = 0.0;
    }
  }
  int inc = 0;
  for (int i = 1; i < npairs; ++i) {
    int cs = qref_table1_case(B[inc], M[inc], B[i], M[i]);
    if (trace) trace->cmp_case[i] = cs;
    if (cs == 1) continue;
    if (cs == 2) {
      inc = i;
      continue;
    }
    double f = cs == 3 ? 0.8 : 1.2;
    double ep = e * f;
    LevelBounds lb;
    bounds_eq5(ep, kAlphas[i / 4], kBetas[i % 4], Lt, &lb);
    qref_trial_result r;
    run_trial(sp, Is, lb, vrange, want_ssim, want_ac, w, &r);
    double Bp = r.B, Mp = metric_of(r, target, vrange);
    if (trace) {
      trace->Bp[i] = Bp;
      trace->Mp[i] = Mp;
      trace->eprime[i] = f;
    }
    if (qref_table1_line(B[inc], M[inc], B[i], M[i], Bp, Mp)) inc = i;
  }
  if (trace) trace->best_pair = (uint32_t)inc;

  qref_params p;
  std::memset(&p, 0, sizeof(p));
  p.anchor_stride = s;
  p.levels = (uint32_t)L;
  for (int l = 0; l < L; ++l) {
    p.interp[l] = (uint8_t)Is.interp[l];
    for (int j = 0; j < 3; ++j)
      p.order[l][j] = (uint8_t)(j < g.d ? Is.order[l][j] : 0);
  }
  p.alpha = kAlphas[inc / 4];
  p.beta = kBetas[inc % 4];
  *out = p;
  return QREF_OK;
}
