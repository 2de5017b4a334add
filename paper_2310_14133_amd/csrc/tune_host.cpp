/*
 * Online tuner (Sec. VI): uniform block sampling (Sec. VI-A), level-adapted
 * interpolator selection (Algorithm 1, Sec. VI-B) and the (alpha, beta)
 * search with the rate-quality comparison of Table I (Sec. VI-C).
 *
 * GPU work per tuning: one gather of the sampled blocks, one launch per
 * level of Algorithm 1 covering every (candidate, block) pair, and a single
 * launch covering every distinct (alpha, beta, e') trial on every block.
 * The decisions (argmin, Table I) are taken on the host from per-block
 * partial sums read back after each launch.
 *
 * Choices where the paper is open: blocks of b+1 points per dimension at
 * origins k*S, S = round(b r^(-1/d)), their 2^Lt grid exact; the whole field
 * as one block when none fits; Algorithm 1 at bound e on every level over
 * committed higher levels, L1 of the prediction before quantization, first
 * strict minimum; bit rate = (Huffman bits of the aggregated bins + 32 per
 * unpredictable value) / points in the blocks; Table I with the incumbent
 * starting at the first pair, pairs in order alpha-major, case 3 re-run at
 * 0.8e and case 4 at 1.2e (as the table states), ties and degenerate lines
 * keep the incumbent; ratio mode compares bit rates only.
 */
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>

#include "qoz_internal.h"

namespace qoz {

static const double kAlpha[5] = {1.0, 1.25, 1.5, 1.75, 2.0};
static const double kBeta[4] = {1.5, 2.0, 3.0, 4.0};
constexpr size_t kPinTune = 2u << 20;

static int table1_case(double BI, double MI, double BII, double MII) {
  if (BI <= BII && MI >= MII) return 1;
  if (BI >= BII && MI <= MII) return 2;
  if (BI > BII && MI > MII) return 3;
  return 4;
}

/* II wins when (B_I, M_I) lies strictly below the line through II's two
 * results; a vertical line keeps I. */
static bool table1_line_prefers_II(double BI, double MI, double BII,
                                   double MII, double BIIp, double MIIp) {
  if (BIIp == BII) return false;
  double rise = (MIIp - MII) * (BI - BII);
  double Mline = MII + rise / (BIIp - BII);
  return MI < Mline;
}

struct Cand {
  uint8_t interp;
  uint8_t order[3]; /* real dimensions */
};

static uint32_t log2_floor(uint32_t v) {
  uint32_t l = 0;
  while ((2u << l) <= v) ++l;
  return l;
}

/* Huffman bits of the trials listed in `over`, whose used symbols
 * overflowed the first device sort: a second device sort of up to
 * kSortCapBig symbols, then whole histograms for any still larger.  May
 * move the pinned staging. */
static qoz_status overflow_bits(qoz_ctx* c, const std::vector<uint32_t>& over,
                                const uint32_t* dhist,
                                std::vector<uint64_t>& bits, hipStream_t s) {
  const uint32_t no = (uint32_t)over.size();
  std::vector<uint32_t> full;
  if (hist_sort_big_fits()) {
    const size_t kb = 8 * (size_t)(kSortCapBig + 1);
    QOZ_TRY(ensure(c->hsort, kb * no));
    QOZ_TRY(ensure(c->hsort_ids, 4 * (size_t)no));
    QOZ_TRY(ensure_pinned(c, kb * no + 4 * (size_t)no + 64));
    uint8_t* hp = (uint8_t*)c->pinned;
    std::memcpy(hp, over.data(), 4 * (size_t)no);
    QOZ_TRY(to_device(c, c->hsort_ids.p, hp, 4 * (size_t)no, s));
    launch_hist_sort_big(dhist, (const uint32_t*)c->hsort_ids.p, no,
                         (uint64_t*)c->hsort.p, s);
    uint64_t* hk = (uint64_t*)(hp + ((4 * (size_t)no + 63) / 64) * 64);
    QOZ_TRY(to_host(c, hk, c->hsort.p, kb * no, s));
    QOZ_HIP(hipGetLastError());
    QOZ_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < no; ++i) {
      const uint64_t* kt = hk + (size_t)i * (kSortCapBig + 1);
      if (kt[0] <= kSortCapBig)
        bits[over[i]] = huffman_cost_sorted(kt + 1, (uint32_t)kt[0]);
      else
        full.push_back(over[i]);
    }
  } else {
    full = over;
  }
  if (!full.empty()) {
    const size_t hb = 4 * (size_t)kNSym;
    QOZ_TRY(ensure_pinned(c, hb * full.size()));
    uint8_t* hp = (uint8_t*)c->pinned;
    for (size_t i = 0; i < full.size(); ++i)
      QOZ_TRY(to_host(c, hp + i * hb, dhist + (size_t)full[i] * kNSym, hb, s));
    QOZ_HIP(hipGetLastError());
    QOZ_HIP(hipStreamSynchronize(s));
    /* one host thread per histogram, at most 16 */
    std::atomic<size_t> next{0};
    auto work = [&]() {
      for (size_t i; (i = next.fetch_add(1)) < full.size();)
        bits[full[i]] =
            huffman_cost_hist((const uint32_t*)(hp + i * hb), kNSym);
    };
    const size_t nt = std::min<size_t>(full.size(), 16);
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
  }
  return QOZ_OK;
}

}  // namespace qoz

using namespace qoz;

static qoz_status tune_impl(qoz_ctx* c, const float* d_x, qoz_shape shape,
                            double e, qoz_target target,
                            const qoz_tune_config* cfg, qoz_params* out,
                            qoz_tune_trace* tr, hipStream_t s) {
  clear_error();
  if (!c || !d_x || !out) return fail(QOZ_EINVAL, "NULL argument");
  if (target < QOZ_TARGET_CR || target > QOZ_TARGET_AC)
    return fail(QOZ_EINVAL, "bad target");
  if (!(e > 0.0) || !std::isfinite(e))
    return fail(QOZ_EINVAL, "error bound must be finite and > 0");
  int d;
  uint64_t n[3] = {1, 1, 1};
  if (!shape_ok(shape, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  QOZ_TRY(set_device(c));
  const Geo g = make_geo(d, n);
  const uint64_t N = (uint64_t)g.n[0] * g.n[1] * g.n[2];
  const uint32_t sa = out->anchor_stride ? out->anchor_stride
                                         : (d == 2 ? 64u : 32u);
  if (sa < 2 || (sa & (sa - 1))) return fail(QOZ_EINVAL, "bad anchor stride");
  const uint32_t L = log2_floor(sa);
  if (L > QOZ_MAX_LEVELS) return fail(QOZ_EINVAL, "anchor stride too large");

  /* sampling plan (Sec. VI-A) */
  const uint32_t b = (cfg && cfg->block) ? cfg->block : (d == 2 ? 64u : 16u);
  if (b < 2 || (b & (b - 1))) return fail(QOZ_EINVAL, "bad block size");
  const double r = (cfg && cfg->sample_rate > 0.0) ? cfg->sample_rate
                                                   : (d == 2 ? 0.01 : 0.005);
  if (!(r > 0.0 && r <= 1.0)) return fail(QOZ_EINVAL, "bad sample rate");
  uint32_t S = (cfg && cfg->sample_stride)
                   ? cfg->sample_stride
                   : (uint32_t)std::llround((double)b * std::pow(r, -1.0 / d));
  if (S < 1) S = 1;
  const uint32_t Lt = log2_floor(b < sa ? b : sa);
  const bool all_orders = cfg && cfg->all_orders;
  const uint32_t abl = cfg ? cfg->ablation : 0u;
  if (abl & ~(QOZ_ABLATE_AB | QOZ_ABLATE_LEVELWISE))
    return fail(QOZ_EINVAL, "unknown ablation switch");
  const uint32_t w = (cfg && cfg->ssim_window) ? cfg->ssim_window : 7;
  if (w > 11) return fail(QOZ_EINVAL, "ssim_window must be <= 11");
  uint64_t m[3] = {1, 1, 1};
  bool whole = false;
  for (int i = 0; i < d; ++i) {
    m[i] = 0;
    while (m[i] * S + b <= n[i] - 1) ++m[i];
    whole |= m[i] == 0;
  }
  uint64_t bd[3];
  for (int i = 0; i < d; ++i) bd[i] = whole ? n[i] : (uint64_t)b + 1;
  if (whole)
    for (int i = 0; i < 3; ++i) m[i] = 1;
  BlockGeo bg;
  bg.g = make_geo(d, bd);
  bg.size = bg.g.n[0] * bg.g.n[1] * bg.g.n[2];
  bg.nb = (uint32_t)(m[0] * m[1] * (d == 3 ? m[2] : 1));
  bg.Lt = Lt;
  bg.d = (uint32_t)d;
  std::vector<uint32_t> origins;
  for (uint64_t k0 = 0; k0 < m[0]; ++k0)
    for (uint64_t k1 = 0; k1 < m[1]; ++k1)
      for (uint64_t k2 = 0; k2 < (d == 3 ? m[2] : 1); ++k2) {
        uint32_t o[3] = {(uint32_t)(k0 * S), (uint32_t)(k1 * S),
                         (uint32_t)(k2 * S)};
        if (whole) o[0] = o[1] = o[2] = 0;
        if (d == 2) {
          origins.push_back(0);
          origins.push_back(o[0]);
          origins.push_back(o[1]);
        } else {
          origins.insert(origins.end(), o, o + 3);
        }
      }

  /* candidates (Sec. V-B, VI-B): interpolation type outer, order inner */
  std::vector<Cand> cands;
  {
    std::vector<std::vector<uint8_t>> orders;
    std::vector<uint8_t> p(d);
    for (int i = 0; i < d; ++i) p[i] = (uint8_t)i;
    if (all_orders) {
      do orders.push_back(p);
      while (std::next_permutation(p.begin(), p.end()));
    } else {
      orders.push_back(p);
      std::reverse(p.begin(), p.end());
      orders.push_back(p);
    }
    for (uint8_t t = 0; t < 2; ++t)
      for (auto& o : orders) {
        Cand cd;
        cd.interp = t;
        for (int i = 0; i < 3; ++i) cd.order[i] = i < d ? o[i] : 0;
        cands.push_back(cd);
      }
  }
  const uint32_t ncand = (uint32_t)cands.size();
  if (tr) {
    std::memset(tr, 0, sizeof(*tr));
    tr->Lt = Lt;
    tr->ncand = ncand;
    tr->nblocks = bg.nb;
    tr->block_points = (uint64_t)bg.nb * bg.size;
  }
  const uint32_t shift = d == 2 ? 1 : 0;
  const uint32_t max_trials = 60;
  const uint32_t nslots = std::max(ncand, max_trials);

  /* scratch */
  const uint64_t bsz = (uint64_t)bg.nb * bg.size;
  const uint32_t rp = range_parts(N);
  QOZ_TRY(ensure(c->status, 256));
  QOZ_TRY(ensure(c->partial, 8 * (size_t)rp + 16 * (size_t)bg.nb + 64));
  QOZ_TRY(ensure(c->tune_x, 4 * bsz));
  QOZ_TRY(ensure(c->tune_wc, 4 * bsz));
  QOZ_TRY(ensure(c->tune_wt, 4 * bsz * nslots));
  const uint32_t adesc_n = QOZ_MAX_LEVELS * ncand;
  QOZ_TRY(ensure(c->tune_desc,
                 sizeof(TrialDesc) * (nslots + adesc_n) + 4 * QOZ_MAX_LEVELS));
  QOZ_TRY(ensure(c->tune_l1, 8 * (size_t)nslots * bg.nb));
  QOZ_TRY(ensure(c->tune_stats, 24 * (size_t)nslots * bg.nb));
  QOZ_TRY(ensure(c->tune_hist, 4 * (size_t)kNSym * max_trials));
  SsimJob sj;
  std::memset(&sj, 0, sizeof(sj));
  uint64_t ssim_np = 0;
  if (target == QOZ_TARGET_SSIM) {
    sj.P = bg.g.n[0];
    sj.Rn = bg.g.n[1];
    sj.Cn = bg.g.n[2];
    sj.wp = std::min(sj.P, w);
    sj.wr = std::min(sj.Rn, w);
    sj.wc = std::min(sj.Cn, w);
    sj.field_stride = bg.size;
    sj.batch = max_trials * bg.nb;
    sj.x_mod = bg.nb;
    ssim_np = ssim_parts(sj);
    QOZ_TRY(ensure(c->ssim_part, 8 * ssim_np));
  } else if (target == QOZ_TARGET_AC) {
    /* AC moments: one pass-0 and two pass-1 doubles per (trial, block) */
    ssim_np = 3 * (uint64_t)max_trials * bg.nb;
    QOZ_TRY(ensure(c->ssim_part, 8 * ssim_np));
  }
  const size_t pin_need = kPinTune + 4 * (size_t)kNSym * max_trials +
                          24 * (size_t)nslots * bg.nb +
                          8 * (size_t)nslots * bg.nb + 8 * ssim_np +
                          sizeof(TrialDesc) * (nslots + adesc_n) + 8 * rp +
                          12 * (size_t)bg.nb + 4096 +
                          (tr ? 8 * (size_t)QOZ_MAX_LEVELS * ncand * bg.nb
                              : 0);
  QOZ_TRY(ensure_pinned(c, pin_need));
  uint8_t* pbase;
  uint32_t *h_hist, *h_un, *h_status;
  double *h_sse, *h_l1, *h_ssim;
  TrialDesc *h_desc, *h_adesc;
  float* h_range;
  double* h_tl1; /* traced runs: Algorithm 1's per-block sums, per level */
  /* regions of the pinned staging (again after anything that may move it) */
  auto bind_pinned = [&]() {
    pbase = (uint8_t*)c->pinned + kPinTune;
    h_hist = (uint32_t*)pbase;
    h_sse = (double*)(pbase + 4 * (size_t)kNSym * max_trials);
    /* per (trial, block) item: two partials (levels above 1, level 1) */
    h_un = (uint32_t*)(h_sse + 2 * (size_t)nslots * bg.nb);
    h_l1 = (double*)(pbase + 4 * (size_t)kNSym * max_trials +
                     24 * (size_t)nslots * bg.nb);
    h_ssim = h_l1 + (size_t)nslots * bg.nb;
    h_desc = (TrialDesc*)(h_ssim + ssim_np);
    h_adesc = h_desc + nslots;
    h_range = (float*)(h_adesc + adesc_n);
    h_status = (uint32_t*)(h_range + 2 * rp);
    h_tl1 = (double*)(((uintptr_t)(h_status + 8 + 3 * (size_t)bg.nb +
                                   QOZ_MAX_LEVELS) +
                       7) &
                      ~(uintptr_t)7);
  };
  bind_pinned();

  float* xs = (float*)c->tune_x.p;
  float* wc = (float*)c->tune_wc.p;
  float* wt = (float*)c->tune_wt.p;
  TrialDesc* ddesc = (TrialDesc*)c->tune_desc.p;
  TrialDesc* dadesc = ddesc + nslots;
  uint32_t* dpick = (uint32_t*)(dadesc + adesc_n);
  double* dl1 = (double*)c->tune_l1.p;
  double* dsse = (double*)c->tune_stats.p;
  uint32_t* dun = (uint32_t*)(dsse + 2 * (size_t)nslots * bg.nb);
  uint32_t* dhist = (uint32_t*)c->tune_hist.p;
  uint32_t* st = (uint32_t*)c->status.p;
  float* pmin = (float*)c->partial.p;
  float* pmax = pmin + rp;
  uint32_t* dorig = (uint32_t*)(pmax + rp);

  /* The ratio target reads only the sampled blocks (Sec. VI-A), checked
   * for finiteness as they are gathered; the quality targets also need the
   * whole field's value range (Eq. 1-3) and check every value. */
  const bool need_range = target != QOZ_TARGET_CR;
  launch_init_status(st, s);
  if (need_range) {
    hipEvent_t ev = prof_begin(c, s, PK_CHECK);
    launch_range(d_x, N, pmin, pmax, st, rp, s);
    prof_end(c, s, ev, PK_CHECK, 4.0 * N);
    QOZ_TRY(to_host(c, h_range, pmin, 8 * (size_t)rp, s));
  }
  std::memcpy(h_status + 8, origins.data(), 4 * origins.size());
  QOZ_TRY(to_device(c, dorig, h_status + 8, 4 * origins.size(), s));
  {
    hipEvent_t ev = prof_begin(c, s, PK_TUNE_GATHER);
    launch_gather_blocks(d_x, g, bg, dorig, xs, wc, st, s);
    prof_end(c, s, ev, PK_TUNE_GATHER, 12.0 * bsz);
  }
  /* the status word (and range) arrive with Algorithm 1's first read-back:
   * the gather needs no wait of its own; they are taken right after that
   * wait, before anything can move the staging buffer */
  QOZ_TRY(to_host(c, h_status, st, 16, s));
  bool nonfinite = false;
  double vrange = 0.0; /* unused by the ratio target */
  auto take_status = [&]() {
    nonfinite = (h_status[0] & kStNonFinite) != 0;
    if (need_range) {
      float lo = h_range[0], hi = h_range[rp];
      for (uint32_t i = 1; i < rp; ++i) {
        lo = std::fmin(lo, h_range[i]);
        hi = std::fmax(hi, h_range[rp + i]);
      }
      vrange = (double)hi - (double)lo;
    }
  };

  /* ---- Algorithm 1 ---- */
  uint8_t Is_interp[QOZ_MAX_LEVELS] = {0};
  uint8_t Is_order[QOZ_MAX_LEVELS][3];
  for (int l = 0; l < QOZ_MAX_LEVELS; ++l)
    for (int j = 0; j < 3; ++j) Is_order[l][j] = (uint8_t)(j < d ? j : 0);
  double ueb[QOZ_MAX_LEVELS];
  float utw[QOZ_MAX_LEVELS], uiv[QOZ_MAX_LEVELS];
  level_bounds(e, 1.0, 1.0, Lt, ueb, utw, uiv);
  const double npts = (double)bg.size * bg.nb;

  /* the (alpha, beta) trials' level bounds, deduplicated by level-bound
   * vector (they do not depend on Algorithm 1's choices) */
  const int nf = target == QOZ_TARGET_CR ? 1 : 3;
  const double factors[3] = {1.0, 0.8, 1.2};
  struct Vec {
    double eb[QOZ_MAX_LEVELS];
    float tw[QOZ_MAX_LEVELS], iv[QOZ_MAX_LEVELS];
  };
  std::vector<Vec> vecs;
  int trial_of[3][20];
  if (!(abl & QOZ_ABLATE_AB)) {
    for (int f = 0; f < nf; ++f)
      for (int i = 0; i < 20; ++i) {
        Vec v;
        std::memset(&v, 0, sizeof(v));
        const double ef = f == 0 ? e : e * factors[f];
        level_bounds(ef, kAlpha[i / 4], kBeta[i % 4], Lt, v.eb, v.tw, v.iv);
        int found = -1;
        for (size_t k = 0; k < vecs.size(); ++k)
          if (std::memcmp(&vecs[k], &v, sizeof(Vec)) == 0) {
            found = (int)k;
            break;
          }
        if (found < 0) {
          found = (int)vecs.size();
          vecs.push_back(v);
        }
        trial_of[f][i] = found;
      }
  }
  const uint32_t ntrial = (uint32_t)vecs.size();
  /* the trials' descriptors: bounds here, interpolation types and orders
   * (Algorithm 1's choices) filled in on the device when both searches
   * run and the target needs no value range before the trials (then the
   * host waits once for Algorithm 1 and the trials together) */
  const bool dev_desc = !(abl & QOZ_ABLATE_LEVELWISE) &&
                        !(abl & QOZ_ABLATE_AB) && target != QOZ_TARGET_SSIM;
  auto fill_desc = [&]() {
    std::memset(h_desc, 0, sizeof(TrialDesc) * ntrial);
    for (uint32_t t = 0; t < ntrial; ++t)
      for (uint32_t l = 1; l <= Lt; ++l) {
        TrialLevel& lv = h_desc[t].lv[l - 1];
        lv.twoeb = vecs[t].tw[l - 1];
        lv.inv = vecs[t].iv[l - 1];
        lv.eb = vecs[t].eb[l - 1];
        lv.cubic = Is_interp[l - 1];
        for (int j = 0; j < 3; ++j)
          lv.order[j] = j < d ? Is_order[l - 1][j] + shift : 0;
      }
  };
  if (dev_desc) {
    fill_desc(); /* the choices are overwritten on the device */
    QOZ_TRY(to_device(c, ddesc, h_desc, sizeof(TrialDesc) * ntrial, s));
  }
  /* Algorithm 1's choices (read back to h_pick) into Is_interp/Is_order */
  uint32_t* const h_pick0 = h_status + 8 + 3 * (size_t)bg.nb;
  auto apply_picks = [&](const uint32_t* h_pick) -> qoz_status {
    for (uint32_t l = Lt; l >= 1; --l) {
      const uint32_t ib = h_pick[l - 1];
      if (ib >= ncand) return fail(QOZ_EDEVICE, "bad tuner choice");
      if (tr) {
        /* each candidate's mean as the device forms it: block sums in
         * block order over the level's target count */
        uint64_t on_fine = 1, on_coarse = 1;
        for (int i = 0; i < 3; ++i) {
          on_fine *= (bg.g.n[i] - 1) / (1u << (l - 1)) + 1;
          on_coarse *= (bg.g.n[i] - 1) / (1u << l) + 1;
        }
        const double count = (double)(on_fine - on_coarse) * bg.nb;
        const double* lp = h_tl1 + (size_t)(l - 1) * ncand * bg.nb;
        for (uint32_t ci = 0; ci < ncand; ++ci) {
          double sum = 0.0;
          for (uint32_t k = 0; k < bg.nb; ++k) sum += lp[(size_t)ci * bg.nb + k];
          tr->alg1_err[l - 1][ci] = count > 0 ? sum / count : 0.0;
        }
        tr->alg1_choice[l - 1] = ib;
      }
      Is_interp[l - 1] = cands[ib].interp;
      std::memcpy(Is_order[l - 1], cands[ib].order, 3);
    }
    for (uint32_t l = Lt + 1; l <= L; ++l) {
      Is_interp[l - 1] = Is_interp[Lt - 1];
      std::memcpy(Is_order[l - 1], Is_order[Lt - 1], 3);
    }
    return QOZ_OK;
  };

  if (abl & QOZ_ABLATE_LEVELWISE) {
    /* one interpolator for every level: each candidate trial-compresses
     * the sampled blocks at the uniform bound; the lowest bit rate wins,
     * the first on ties */
    std::memset(h_desc, 0, sizeof(TrialDesc) * ncand);
    for (uint32_t ci = 0; ci < ncand; ++ci)
      for (uint32_t l = 1; l <= Lt; ++l) {
        TrialLevel& lv = h_desc[ci].lv[l - 1];
        lv.twoeb = utw[l - 1];
        lv.inv = uiv[l - 1];
        lv.eb = ueb[l - 1];
        lv.cubic = cands[ci].interp;
        for (int j = 0; j < 3; ++j)
          lv.order[j] = j < d ? cands[ci].order[j] + shift : 0;
      }
    QOZ_TRY(to_device(c, ddesc, h_desc, sizeof(TrialDesc) * ncand, s));
    launch_zero_u32(dhist, (uint64_t)kNSym * ncand, s);
    {
      hipEvent_t ev = prof_begin(c, s, PK_TUNE_TRIAL);
      launch_trial(bg, xs, wt, ncand, ddesc, dhist, dsse, dun, false, s);
      prof_end(c, s, ev, PK_TUNE_TRIAL, 16.0 * bsz * ncand);
    }
    QOZ_TRY(ensure(c->hsort, 8 * (size_t)(kSortCap + 1) * ncand));
    launch_hist_sort(dhist, ncand, (uint64_t*)c->hsort.p, s);
    uint64_t* hk = (uint64_t*)h_hist;
    QOZ_TRY(to_host(c, hk, c->hsort.p, 8 * (size_t)(kSortCap + 1) * ncand,
                    s));
    QOZ_TRY(to_host(c, h_sse, dsse, 24 * (size_t)nslots * bg.nb, s));
    QOZ_HIP(hipGetLastError());
    QOZ_HIP(hipStreamSynchronize(s));
    take_status();
    std::vector<uint64_t> cbits(ncand, 0), cU(ncand, 0);
    std::vector<uint32_t> cover;
    for (uint32_t ci = 0; ci < ncand; ++ci) {
      const uint64_t* kt = hk + (size_t)ci * (kSortCap + 1);
      if (kt[0] <= kSortCap)
        cbits[ci] = huffman_cost_sorted(kt + 1, (uint32_t)kt[0]);
      else
        cover.push_back(ci);
      for (uint32_t k = 0; k < bg.nb; ++k) {
        const size_t it = 2 * ((size_t)ci * bg.nb + k);
        cU[ci] += h_un[it] + h_un[it + 1];
      }
    }
    if (!cover.empty()) QOZ_TRY(overflow_bits(c, cover, dhist, cbits, s));
    bind_pinned();
    double best = std::numeric_limits<double>::infinity();
    uint32_t ib = 0;
    for (uint32_t ci = 0; ci < ncand; ++ci) {
      const double Bc = ((double)cbits[ci] + 32.0 * (double)cU[ci]) / npts;
      if (tr) tr->alg1_err[0][ci] = Bc;
      if (Bc < best) {
        best = Bc;
        ib = ci;
      }
    }
    for (uint32_t l = 0; l < QOZ_MAX_LEVELS; ++l) {
      Is_interp[l] = cands[ib].interp;
      std::memcpy(Is_order[l], cands[ib].order, 3);
      if (tr && l < Lt) tr->alg1_choice[l] = ib;
    }
  }
  if (!(abl & QOZ_ABLATE_LEVELWISE)) {
    /* every level's candidates go up at once; each level's choice and the
     * commit of its working copy happen on the device, so the levels run
     * back to back and the host reads the choices once */
    std::memset(h_adesc, 0, sizeof(TrialDesc) * adesc_n);
    for (uint32_t l = Lt; l >= 1; --l)
      for (uint32_t ci = 0; ci < ncand; ++ci) {
        TrialLevel& lv = h_adesc[(l - 1) * ncand + ci].lv[l - 1];
        lv.twoeb = utw[l - 1];
        lv.inv = uiv[l - 1];
        lv.eb = ueb[l - 1];
        lv.cubic = cands[ci].interp;
        for (int j = 0; j < 3; ++j)
          lv.order[j] = j < d ? cands[ci].order[j] + shift : 0;
      }
    QOZ_TRY(
        to_device(c, dadesc, h_adesc, sizeof(TrialDesc) * Lt * ncand, s));
    for (uint32_t l = Lt; l >= 1; --l) {
      const bool in_lds = alg1_in_lds(bg, l);
      {
        hipEvent_t ev = prof_begin(c, s, PK_TUNE_ALG1);
        launch_alg1_level(bg, l, xs, wc, wt, ncand, dadesc + (l - 1) * ncand,
                          dl1, in_lds, l > 1, s);
        prof_end(c, s, ev, PK_TUNE_ALG1, 16.0 * bsz * ncand);
      }
      if (tr)
        QOZ_TRY(to_host(c, h_tl1 + (size_t)(l - 1) * ncand * bg.nb, dl1,
                        8 * (size_t)ncand * bg.nb, s));
      /* level-l targets: points of the 2^(l-1) grid off the 2^l grid */
      uint64_t on_fine = 1, on_coarse = 1;
      for (int i = 0; i < 3; ++i) {
        on_fine *= (bg.g.n[i] - 1) / (1u << (l - 1)) + 1;
        on_coarse *= (bg.g.n[i] - 1) / (1u << l) + 1;
      }
      const double count = (double)(on_fine - on_coarse) * bg.nb;
      launch_alg1_pick(bg, l, xs, dadesc + (l - 1) * ncand, dl1, ncand, count,
                       dpick + (l - 1), wt, wc, in_lds, l > 1, s);
    }
    /* the choices follow the origins in the staging buffer */
    QOZ_TRY(to_host(c, h_pick0, dpick, 4 * Lt, s));
    if (dev_desc) {
      launch_trial_fill(ddesc, ntrial, Lt, dadesc, ncand, dpick, s);
    } else {
      QOZ_HIP(hipGetLastError());
      QOZ_HIP(hipStreamSynchronize(s));
      take_status();
      QOZ_TRY(apply_picks(h_pick0));
    }
  }

  if (!dev_desc && nonfinite) {
    prof_collect(c);
    return fail(QOZ_EINVAL, "input contains NaN or Inf");
  }

  /* (alpha, beta); without the search the first pair, alpha = 1 */
  int inc = 0;
  if (!(abl & QOZ_ABLATE_AB)) {
    /* ---- (alpha, beta) trials ---- */
    if (!dev_desc) {
      fill_desc();
      QOZ_TRY(to_device(c, ddesc, h_desc, sizeof(TrialDesc) * ntrial, s));
    }
    launch_zero_u32(dhist, (uint64_t)kNSym * ntrial, s);
    {
      hipEvent_t ev = prof_begin(c, s, PK_TUNE_TRIAL);
      launch_trial(bg, xs, wt, ntrial, ddesc, dhist, dsse, dun,
                   target == QOZ_TARGET_SSIM || target == QOZ_TARGET_AC, s);
      prof_end(c, s, ev, PK_TUNE_TRIAL, 16.0 * bsz * ntrial);
    }
    if (target == QOZ_TARGET_SSIM) {
      sj.batch = ntrial * bg.nb;
      sj.c1 = (0.01 * vrange) * (0.01 * vrange);
      sj.c2 = (0.03 * vrange) * (0.03 * vrange);
      ssim_np = ssim_parts(sj);
      hipEvent_t ev = prof_begin(c, s, PK_SSIM);
      const bool launched =
          launch_ssim(sj, xs, wt, (double*)c->ssim_part.p, s);
      prof_end(c, s, ev, PK_SSIM, 8.0 * bsz * ntrial);
      if (!launched)
        return fail(QOZ_EDEVICE, "SSIM window ring does not fit LDS");
      QOZ_TRY(to_host(c, h_ssim, c->ssim_part.p, 8 * ssim_np, s));
    } else if (target == QOZ_TARGET_AC) {
      double* p0 = (double*)c->ssim_part.p;
      double* p1 = p0 + (size_t)ntrial * bg.nb;
      hipEvent_t ev = prof_begin(c, s, PK_REDUCE);
      launch_ac_items(xs, wt, ntrial, bg.nb, bg.size, bg.g.n[2], p0, p1, s);
      prof_end(c, s, ev, PK_REDUCE, 16.0 * bsz * ntrial);
      QOZ_TRY(to_host(c, h_ssim, p1, 16 * (size_t)ntrial * bg.nb, s));
    }
    /* used symbols of every trial histogram, sorted on the device */
    QOZ_TRY(ensure(c->hsort, 8 * (size_t)(kSortCap + 1) * ntrial));
    launch_hist_sort(dhist, ntrial, (uint64_t*)c->hsort.p, s);
    uint64_t* h_keys = (uint64_t*)h_hist;
    QOZ_TRY(to_host(c, h_keys, c->hsort.p,
                    8 * (size_t)(kSortCap + 1) * ntrial, s));
    QOZ_TRY(to_host(c, h_sse, dsse, 24 * (size_t)nslots * bg.nb, s));
    QOZ_HIP(hipGetLastError());
    QOZ_HIP(hipStreamSynchronize(s));
    prof_collect(c);
    if (dev_desc) {
      take_status();
      if (nonfinite) return fail(QOZ_EINVAL, "input contains NaN or Inf");
      QOZ_TRY(apply_picks(h_pick0));
    }

    const uint64_t per_item = sj.batch ? ssim_np / sj.batch : 0;
    const double nwin = (double)(sj.P - sj.wp + 1) *
                        (double)(sj.Rn - sj.wr + 1) *
                        (double)(sj.Cn - sj.wc + 1) * bg.nb;
    std::vector<double> B(ntrial), M(ntrial, 0.0);
    std::vector<uint64_t> bits(ntrial, 0), Us(ntrial, 0);
    std::vector<uint32_t> over; /* more used symbols than kSortCap */
    for (uint32_t t = 0; t < ntrial; ++t) {
      const uint64_t* kt = h_keys + (size_t)t * (kSortCap + 1);
      if (kt[0] <= kSortCap)
        bits[t] = huffman_cost_sorted(kt + 1, (uint32_t)kt[0]);
      else
        over.push_back(t);
      uint64_t U = 0;
      double sse = 0.0;
      for (uint32_t k = 0; k < bg.nb; ++k) {
        const size_t it = 2 * ((size_t)t * bg.nb + k);
        U += h_un[it] + h_un[it + 1];
        sse += h_sse[it] + h_sse[it + 1];
      }
      Us[t] = U;
      if (target == QOZ_TARGET_PSNR) {
        M[t] = sse == 0.0 ? std::numeric_limits<double>::infinity()
                          : 20.0 * std::log10(vrange / std::sqrt(sse / npts));
      } else if (target == QOZ_TARGET_SSIM) {
        double sum = 0.0;
        for (uint64_t q = 0; q < per_item * bg.nb; ++q)
          sum += h_ssim[(uint64_t)t * bg.nb * per_item + q];
        M[t] = sum / nwin;
      } else if (target == QOZ_TARGET_AC) {
        /* the blocks' rows together; errors nearest uncorrelated are best */
        double ss = 0.0, lag = 0.0;
        for (uint32_t k = 0; k < bg.nb; ++k) {
          const size_t it = 2 * ((size_t)t * bg.nb + k);
          ss += h_ssim[it];
          lag += h_ssim[it + 1];
        }
        const double len = (double)bg.g.n[2];
        M[t] = -std::fabs(ac_from_sums(ss, lag, npts, npts / len * (len - 1)));
      }
    }
    /* trials with many used symbols (may move the pinned staging: nothing
     * below reads it) */
    if (!over.empty()) QOZ_TRY(overflow_bits(c, over, dhist, bits, s));
    for (uint32_t t = 0; t < ntrial; ++t)
      B[t] = ((double)bits[t] + 32.0 * (double)Us[t]) / npts;

    if (tr)
      for (int i = 0; i < 20; ++i) {
        tr->B[i] = B[trial_of[0][i]];
        tr->M[i] = M[trial_of[0][i]];
        tr->Bp[i] = tr->Mp[i] = std::numeric_limits<double>::quiet_NaN();
      }
    for (int i = 1; i < 20; ++i) {
      const int tI = trial_of[0][inc], tII = trial_of[0][i];
      const int cs = table1_case(B[tI], M[tI], B[tII], M[tII]);
      if (tr) tr->cmp_case[i] = cs;
      if (cs == 1) continue;
      if (cs == 2) {
        inc = i;
        continue;
      }
      const int tp = trial_of[cs == 3 ? 1 : 2][i];
      if (tr) {
        tr->Bp[i] = B[tp];
        tr->Mp[i] = M[tp];
        tr->eprime[i] = factors[cs == 3 ? 1 : 2];
      }
      if (table1_line_prefers_II(B[tI], M[tI], B[tII], M[tII], B[tp], M[tp]))
        inc = i;
    }
  }
  if (tr) tr->best_pair = (uint32_t)inc;

  prof_collect(c);
  qoz_params p;
  std::memset(&p, 0, sizeof(p));
  p.anchor_stride = sa;
  p.levels = L;
  for (uint32_t l = 0; l < L; ++l) {
    p.interp[l] = Is_interp[l];
    for (int j = 0; j < 3; ++j) p.order[l][j] = j < d ? Is_order[l][j] : 0;
  }
  p.alpha = kAlpha[inc / 4];
  p.beta = kBeta[inc % 4];
  *out = p;
  return QOZ_OK;
}

extern "C" qoz_status qoz_tune(qoz_ctx* c, const float* d_x, qoz_shape shape,
                               double e, qoz_target target,
                               const qoz_tune_config* cfg, qoz_params* out,
                               hipStream_t s) {
  return tune_impl(c, d_x, shape, e, target, cfg, out, nullptr, s);
}

extern "C" qoz_status qoz_tune_traced(qoz_ctx* c, const float* d_x,
                                      qoz_shape shape, double e,
                                      qoz_target target,
                                      const qoz_tune_config* cfg,
                                      qoz_params* out, qoz_tune_trace* trace,
                                      hipStream_t s) {
  if (!trace) return fail(QOZ_EINVAL, "trace is NULL");
  return tune_impl(c, d_x, shape, e, target, cfg, out, trace, s);
}
