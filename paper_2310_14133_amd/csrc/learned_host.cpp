/*
 * Learned tuner entry points: block features, network forward pass,
 * gradient and Adam step, and learned tuning with the online tuner of
 * Sec. VI as the fallback.
 *
 * Sampling of the feature blocks follows Sec. VI-A with b = 32: blocks of
 * 33 points per dimension at origins k*S, S = round(32 r^(-1/d)), every
 * origin with k*S + 32 <= n - 1, for 2D (d = 2) and 3D (d = 3) fields.
 */
#include <cmath>
#include <cstring>
#include <vector>

#include <algorithm>

#include "qoz_internal.h"

namespace qoz {

static const double kAlphaL[5] = {1.0, 1.25, 1.5, 1.75, 2.0};
static const double kBetaL[4] = {1.5, 2.0, 3.0, 4.0};

static qoz_status learned_origins(int d, const uint64_t n[3],
                                  const qoz_tune_config* cfg,
                                  std::vector<uint32_t>* origins) {
  for (int i = 0; i < d; ++i)
    if (n[i] < 33)
      return fail(QOZ_EINVAL, "learned features need every dimension >= 33");
  const double r =
      (cfg && cfg->sample_rate > 0.0) ? cfg->sample_rate : 0.01;
  if (!(r > 0.0 && r <= 1.0)) return fail(QOZ_EINVAL, "bad sample rate");
  uint32_t S = (cfg && cfg->sample_stride)
                   ? cfg->sample_stride
                   : (uint32_t)std::llround(32.0 * std::pow(r, -1.0 / d));
  if (S < 1) S = 1;
  /* blocks per dimension; a 2D field is one plane of the 3D layout */
  uint64_t m[3] = {1, 1, 1};
  for (int i = 0; i < d; ++i) {
    uint64_t& mi = m[3 - d + i];
    mi = 0;
    while (mi * S + 32 <= n[i] - 1) ++mi;
  }
  origins->clear();
  for (uint64_t a = 0; a < m[0]; ++a)
    for (uint64_t b = 0; b < m[1]; ++b)
      for (uint64_t k = 0; k < m[2]; ++k) {
        origins->push_back((uint32_t)(a * S));
        origins->push_back((uint32_t)(b * S));
        origins->push_back((uint32_t)(k * S));
      }
  if (origins->size() / 3 > (1u << 20))
    return fail(QOZ_EINVAL, "too many sampled blocks");
  return QOZ_OK;
}

/* Enqueue the features; the status word is copied to the pinned staging
 * at *h_status (checked by the caller after a sync). */
static qoz_status enqueue_features(qoz_ctx* c, const float* d_x, int d,
                                   const uint64_t n[3], double e,
                                   const qoz_tune_config* cfg, float* d_mean,
                                   float* d_block, uint64_t block_cap,
                                   uint32_t* nb_out, uint32_t** h_status,
                                   hipStream_t s) {
  std::vector<uint32_t> org;
  QOZ_TRY(learned_origins(d, n, cfg, &org));
  const uint32_t nb = (uint32_t)(org.size() / 3);
  if (d_block && block_cap < nb)
    return fail(QOZ_EINVAL, "block feature buffer too small");
  if (!block_features_fit())
    return fail(QOZ_EDEVICE, "block features do not fit in LDS");
  const Geo g = make_geo(d, n);
  /* partial: origins (3 per block), then aux (3 per block) */
  QOZ_TRY(ensure(c->partial, 4 * 6 * (size_t)nb + 64));
  QOZ_TRY(ensure(c->status, 256));
  if (!d_block) QOZ_TRY(ensure(c->feat, 4 * (size_t)kMlpFeat * nb));
  /* pinned: status [0, 16), logits [16, 60), origins from 64 */
  QOZ_TRY(ensure_pinned(c, 4 * org.size() + 4096));
  uint32_t* dorig = (uint32_t*)c->partial.p;
  float* aux = (float*)(dorig + org.size());
  uint32_t* st = (uint32_t*)c->status.p;
  uint8_t* hp = (uint8_t*)c->pinned;
  std::memcpy(hp + 64, org.data(), 4 * org.size());
  QOZ_TRY(to_device(c, dorig, hp + 64, 4 * org.size(), s));
  {
    hipEvent_t ev = prof_begin(c, s, PK_LEARN_FEAT);
    launch_block_features(d_x, g, dorig, nb, e,
                          d_block ? d_block : (float*)c->feat.p, aux, d_mean,
                          st, s);
    prof_end(c, s, ev, PK_LEARN_FEAT,
             4.0 * (d == 2 ? 1089.0 : 35937.0) * nb);
  }
  QOZ_TRY(to_host(c, hp, st, 16, s));
  *nb_out = nb;
  *h_status = (uint32_t*)hp;
  return QOZ_OK;
}

}  // namespace qoz

using namespace qoz;

extern "C" qoz_status qoz_learned_features(qoz_ctx* c, const float* d_x,
                                           qoz_shape shape, double e,
                                           const qoz_tune_config* cfg,
                                           float* d_mean, float* d_block,
                                           uint64_t block_cap,
                                           uint64_t* nblocks, hipStream_t s) {
  clear_error();
  if (!c || !d_x || !d_mean) return fail(QOZ_EINVAL, "NULL argument");
  if (!(e > 0.0) || !std::isfinite(e))
    return fail(QOZ_EINVAL, "error bound must be finite and > 0");
  int d;
  uint64_t n[3] = {1, 1, 1};
  if (!shape_ok(shape, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  QOZ_TRY(set_device(c));
  uint32_t nb = 0;
  uint32_t* hst = nullptr;
  QOZ_TRY(enqueue_features(c, d_x, d, n, e, cfg, d_mean, d_block, block_cap,
                           &nb, &hst, s));
  QOZ_HIP(hipGetLastError());
  QOZ_HIP(hipStreamSynchronize(s));
  prof_collect(c);
  if (hst[0] & kStNonFinite)
    return fail(QOZ_EINVAL, "sampled blocks contain NaN or Inf");
  if (nblocks) *nblocks = nb;
  return QOZ_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

/* One row of logits: per head the first maximum; returns the smallest of
 * the heads' softmax probabilities of their picks (0 for NaN logits). */
static double decide(const float* hz, uint32_t pick[3]) {
  const uint32_t heads[3] = {kHeadInterp, kHeadAlpha, kHeadBeta};
  double conf = 1.0;
  uint32_t o = 0;
  for (int h = 0; h < 3; ++h) {
    uint32_t best = 0;
    for (uint32_t k = 1; k < heads[h]; ++k)
      if (hz[o + k] > hz[o + best]) best = k;
    double sum = 0.0;
    for (uint32_t k = 0; k < heads[h]; ++k)
      sum += std::exp((double)hz[o + k] - (double)hz[o + best]);
    const double p = 1.0 / sum;
    if (!(p >= 0.0)) conf = 0.0; /* NaN logits: untrusted */
    conf = std::fmin(conf, p);
    pick[h] = best;
    o += heads[h];
  }
  return conf;
}

/* The network's picks as parameters: one interpolation type for every
 * level, the identity dimension order. */
static qoz_params learned_params(const uint32_t pick[3], uint32_t sa,
                                 uint32_t L, int d) {
  qoz_params p;
  std::memset(&p, 0, sizeof(p));
  p.anchor_stride = sa;
  p.levels = L;
  for (uint32_t l = 0; l < L; ++l) {
    p.interp[l] = (uint8_t)pick[0];
    for (int j = 0; j < 3; ++j) p.order[l][j] = (uint8_t)(j < d ? j : 0);
  }
  p.alpha = kAlphaL[pick[1]];
  p.beta = kBetaL[pick[2]];
  return p;
}

/* Anchor stride (0 = the default of the dimensionality) and level count. */
static bool stride_levels(uint32_t want, int d, uint32_t* sa, uint32_t* L) {
  *sa = want ? want : (d == 2 ? 64u : 32u);
  if (*sa < 2 || (*sa & (*sa - 1))) return false;
  *L = 0;
  while ((2u << *L) <= *sa) ++*L;
  return *L <= QOZ_MAX_LEVELS;
}

extern "C" qoz_status qoz_mlp_forward(qoz_ctx* c, const float* d_params,
                                      const float* d_feat, uint32_t batch,
                                      float* d_logits, hipStream_t s) {
  clear_error();
  if (!c || !d_params || !d_feat || !d_logits)
    return fail(QOZ_EINVAL, "NULL argument");
  if (!aligned16(d_params))
    return fail(QOZ_EINVAL, "d_params must be 16-byte aligned");
  if (batch == 0) return fail(QOZ_EINVAL, "empty batch");
  QOZ_TRY(set_device(c));
  if (!mlp_fit()) return fail(QOZ_EDEVICE, "network does not fit in LDS");
  {
    hipEvent_t ev = prof_begin(c, s, PK_MLP);
    launch_mlp_forward(d_params, d_feat, batch, d_logits, s);
    prof_end(c, s, ev, PK_MLP, 4.0 * kMlpParams + 4.0 * 43 * batch);
  }
  QOZ_HIP(hipGetLastError());
  return QOZ_OK;
}

static qoz_status mlp_backward(qoz_ctx* c, float* P, float* m, float* v,
                               const float* X, const int32_t* labels,
                               const uint32_t* index, uint32_t n_rows,
                               uint32_t B, float* grad, float lr, uint32_t t,
                               bool adam, double* loss, hipStream_t s) {
  if (B == 0) return fail(QOZ_EINVAL, "empty batch");
  if (!aligned16(P)) return fail(QOZ_EINVAL, "d_params must be 16-byte aligned");
  if (!mlp_fit()) return fail(QOZ_EDEVICE, "network does not fit in LDS");
  const uint32_t nw = mlp_tiles(B);
  QOZ_TRY(ensure(c->mlp_part, 4 * (size_t)kMlpParams * nw));
  QOZ_TRY(ensure(c->mlp_loss, 8 * (size_t)nw));
  float* part = (float*)c->mlp_part.p;
  double* lp = (double*)c->mlp_loss.p;
  float bc1 = 1.0f, bc2 = 1.0f;
  if (adam) {
    bc1 = (float)(1.0 - std::pow((double)kAdamB1, (double)t));
    bc2 = (float)(1.0 - std::pow((double)kAdamB2, (double)t));
  }
  hipEvent_t ev = prof_begin(c, s, PK_MLP);
  launch_mlp_grad(P, X, labels, index, n_rows, B, part, lp, s);
  launch_mlp_reduce(part, nw, grad, P, m, v, lr, bc1, bc2, adam, lp, B, loss,
                    s);
  prof_end(c, s, ev, PK_MLP, 4.0 * kMlpParams * (2.0 * nw + 4.0));
  QOZ_HIP(hipGetLastError());
  return QOZ_OK;
}

extern "C" qoz_status qoz_mlp_grad(qoz_ctx* c, const float* d_params,
                                   const float* d_feat,
                                   const int32_t* d_labels,
                                   const uint32_t* d_index, uint32_t n_rows,
                                   uint32_t batch, float* d_grad,
                                   double* d_loss, hipStream_t s) {
  clear_error();
  if (!c || !d_params || !d_feat || !d_labels || !d_grad || !d_loss)
    return fail(QOZ_EINVAL, "NULL argument");
  QOZ_TRY(set_device(c));
  return mlp_backward(c, const_cast<float*>(d_params), nullptr, nullptr,
                      d_feat, d_labels, d_index, n_rows, batch, d_grad, 0.0f,
                      0, false, d_loss, s);
}

extern "C" qoz_status qoz_mlp_train_step(
    qoz_ctx* c, float* d_params, float* d_m, float* d_v, const float* d_feat,
    const int32_t* d_labels, const uint32_t* d_index, uint32_t n_rows,
    uint32_t batch, float lr, uint32_t t, double* d_loss, hipStream_t s) {
  clear_error();
  if (!c || !d_params || !d_m || !d_v || !d_feat || !d_labels)
    return fail(QOZ_EINVAL, "NULL argument");
  if (t < 1) return fail(QOZ_EINVAL, "Adam step must be >= 1");
  if (!(lr > 0.0f) || !std::isfinite(lr))
    return fail(QOZ_EINVAL, "learning rate must be finite and > 0");
  QOZ_TRY(set_device(c));
  return mlp_backward(c, d_params, d_m, d_v, d_feat, d_labels, d_index,
                      n_rows, batch, nullptr, lr, t, true, d_loss, s);
}

extern "C" qoz_status qoz_tune_learned(qoz_ctx* c, const float* d_x,
                                       qoz_shape shape, double e,
                                       const float* d_params,
                                       double min_confidence,
                                       qoz_target fallback_target,
                                       const qoz_tune_config* cfg,
                                       qoz_params* out, int* used_fallback,
                                       hipStream_t s) {
  clear_error();
  if (!c || !d_x || !d_params || !out) return fail(QOZ_EINVAL, "NULL argument");
  if (!aligned16(d_params))
    return fail(QOZ_EINVAL, "d_params must be 16-byte aligned");
  if (!(e > 0.0) || !std::isfinite(e))
    return fail(QOZ_EINVAL, "error bound must be finite and > 0");
  if (!(min_confidence >= 0.0 && min_confidence <= 1.0))
    return fail(QOZ_EINVAL, "min_confidence must be in [0, 1]");
  int d;
  uint64_t n[3] = {1, 1, 1};
  if (!shape_ok(shape, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  QOZ_TRY(set_device(c));
  uint32_t sa = 0, L = 0;
  if (!stride_levels(out->anchor_stride, d, &sa, &L))
    return fail(QOZ_EINVAL, "bad anchor stride");

  bool supported = n[0] >= 33 && n[1] >= 33 && (d == 2 || n[2] >= 33);
  double conf = 0.0;
  uint32_t pick[3] = {0, 0, 0};
  if (supported) {
    if (!mlp_fit()) return fail(QOZ_EDEVICE, "network does not fit in LDS");
    QOZ_TRY(ensure(c->mlp_io, 4 * 64));
    float* d_mean = (float*)c->mlp_io.p;
    float* d_logit = d_mean + kMlpFeat;
    uint32_t nb = 0;
    uint32_t* hst = nullptr;
    QOZ_TRY(enqueue_features(c, d_x, d, n, e, cfg, d_mean, nullptr, 0, &nb,
                             &hst, s));
    {
      hipEvent_t ev = prof_begin(c, s, PK_MLP);
      launch_mlp_forward(d_params, d_mean, 1, d_logit, s);
      prof_end(c, s, ev, PK_MLP, 4.0 * kMlpParams);
    }
    float* hz = (float*)((uint8_t*)hst + 16); /* status is 16 bytes */
    QOZ_TRY(to_host(c, hz, d_logit, 4 * kMlpOut, s));
    QOZ_HIP(hipGetLastError());
    QOZ_HIP(hipStreamSynchronize(s));
    prof_collect(c);
    if (hst[0] & kStNonFinite)
      return fail(QOZ_EINVAL, "sampled blocks contain NaN or Inf");
    conf = decide(hz, pick);
  }
  if (!supported || conf < min_confidence) {
    if (used_fallback) *used_fallback = 1;
    return qoz_tune(c, d_x, shape, e, fallback_target, cfg, out, s);
  }
  *out = learned_params(pick, sa, L, d);
  if (used_fallback) *used_fallback = 0;
  return QOZ_OK;
}

extern "C" qoz_status qoz_tune_learned_batch(
    qoz_ctx* c, qoz_learned_item* items, uint32_t n, const float* d_params,
    const float* d_params_2d, double min_confidence,
    qoz_target fallback_target, const qoz_tune_config* cfg, hipStream_t s) {
  clear_error();
  if (!c || (n && !items) || !d_params)
    return fail(QOZ_EINVAL, "NULL argument");
  if (!aligned16(d_params) || (d_params_2d && !aligned16(d_params_2d)))
    return fail(QOZ_EINVAL, "d_params must be 16-byte aligned");
  if (!(min_confidence >= 0.0 && min_confidence <= 1.0))
    return fail(QOZ_EINVAL, "min_confidence must be in [0, 1]");
  QOZ_TRY(set_device(c));
  if (!n) return QOZ_OK;
  if (!mlp_fit()) return fail(QOZ_EDEVICE, "network does not fit in LDS");
  if (!block_features_fit())
    return fail(QOZ_EDEVICE, "block features do not fit in LDS");
  struct Job {
    uint32_t item, nb;
    int d;
    uint64_t n[3];
    uint32_t sa, L;
    size_t org; /* first origin (in u32) */
    size_t blk; /* first block */
  };
  std::vector<Job> jobs;
  std::vector<uint32_t> fall; /* items for the online tuner */
  std::vector<uint32_t> org_all;
  size_t blocks = 0;
  for (uint32_t i = 0; i < n; ++i) {
    qoz_learned_item& it = items[i];
    it.status = QOZ_OK;
    it.used_fallback = 0;
    Job j{};
    j.item = i;
    if (!it.d_x || !(it.abs_eb > 0.0) || !std::isfinite(it.abs_eb) ||
        !shape_ok(it.shape, &j.d, j.n) ||
        !stride_levels(it.params.anchor_stride, j.d, &j.sa, &j.L)) {
      it.status = QOZ_EINVAL;
      continue;
    }
    const bool sup = j.n[0] >= 33 && j.n[1] >= 33 &&
                     (j.d == 3 ? j.n[2] >= 33 : d_params_2d != nullptr);
    if (!sup) {
      fall.push_back(i);
      continue;
    }
    std::vector<uint32_t> org;
    QOZ_TRY(learned_origins(j.d, j.n, cfg, &org));
    j.nb = (uint32_t)(org.size() / 3);
    j.org = org_all.size();
    j.blk = blocks;
    org_all.insert(org_all.end(), org.begin(), org.end());
    blocks += j.nb;
    jobs.push_back(j);
  }
  /* 3D fields first, then 2D ones: one forward pass per network */
  std::stable_partition(jobs.begin(), jobs.end(),
                        [](const Job& j) { return j.d == 3; });
  const uint32_t m = (uint32_t)jobs.size();
  uint32_t m3 = 0;
  while (m3 < m && jobs[m3].d == 3) ++m3;
  if (m) {
    /* device: origins, aux (3 per block), features (32 per block), means
     * (32 per field), logits (11 per field), status (4 words per field) */
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_org = 0;
    const size_t o_jobs = al(o_org + 4 * org_all.size());
    const size_t o_wg = o_jobs + sizeof(FeatJob) * (size_t)m;
    const size_t up = o_wg + 4 * (size_t)m; /* bytes uploaded */
    const size_t o_aux = al(up);
    const size_t o_feat = al(o_aux + 4 * 3 * blocks);
    const size_t o_mean = al(o_feat + 4 * (size_t)kMlpFeat * blocks);
    const size_t o_logit = al(o_mean + 4 * (size_t)kMlpFeat * m);
    const size_t o_st = al(o_logit + 4 * (size_t)kMlpOut * m);
    QOZ_TRY(ensure(c->lbatch, o_st + 16 * (size_t)m));
    uint8_t* D = (uint8_t*)c->lbatch.p;
    const size_t pin_org = kPinSingleBytes;
    const size_t pin_back = pin_org + al(up);
    QOZ_TRY(ensure_pinned(c, pin_back + 4 * (size_t)kMlpOut * m + 16 * m));
    uint8_t* hp = (uint8_t*)c->pinned;
    /* origins, one record per field (3D fields first) and each group's
     * first workgroups, uploaded in one copy */
    std::memcpy(hp + pin_org, org_all.data(), 4 * org_all.size());
    FeatJob* fj = (FeatJob*)(hp + pin_org + o_jobs);
    uint32_t* wg = (uint32_t*)(hp + pin_org + o_wg);
    uint32_t total3 = 0, total2 = 0;
    double bytes = 0.0;
    for (uint32_t k = 0; k < m; ++k) {
      const Job& j = jobs[k];
      uint32_t& total = k < m3 ? total3 : total2;
      wg[k] = total;
      total += j.nb;
      fj[k] = FeatJob{items[j.item].d_x,
                      make_geo(j.d, j.n),
                      (const uint32_t*)(D + o_org) + j.org,
                      j.nb,
                      items[j.item].abs_eb,
                      (float*)(D + o_feat) + (size_t)kMlpFeat * j.blk,
                      (float*)(D + o_aux) + 3 * j.blk,
                      (float*)(D + o_mean) + (size_t)kMlpFeat * k,
                      (uint32_t*)(D + o_st) + 4 * k};
      bytes += 4.0 * (j.d == 2 ? 1089.0 : 35937.0) * j.nb;
    }
    QOZ_TRY(to_device(c, D + o_org, hp + pin_org, up, s));
    {
      const FeatJob* dj = (const FeatJob*)(D + o_jobs);
      const uint32_t* dw = (const uint32_t*)(D + o_wg);
      hipEvent_t ev = prof_begin(c, s, PK_LEARN_FEAT);
      launch_block_features_q(dj, dw, m3, total3, dj + m3, dw + m3, m - m3,
                              total2, dj, m, s);
      prof_end(c, s, ev, PK_LEARN_FEAT, bytes);
    }
    if (m3) {
      hipEvent_t ev = prof_begin(c, s, PK_MLP);
      launch_mlp_forward(d_params, (const float*)(D + o_mean), m3,
                         (float*)(D + o_logit), s);
      prof_end(c, s, ev, PK_MLP, 4.0 * kMlpParams + 4.0 * 43 * m3);
    }
    if (m > m3) {
      hipEvent_t ev = prof_begin(c, s, PK_MLP);
      launch_mlp_forward(d_params_2d,
                         (const float*)(D + o_mean) + (size_t)kMlpFeat * m3,
                         m - m3,
                         (float*)(D + o_logit) + (size_t)kMlpOut * m3, s);
      prof_end(c, s, ev, PK_MLP, 4.0 * kMlpParams + 4.0 * 43 * (m - m3));
    }
    float* hz = (float*)(hp + pin_back);
    uint32_t* hs = (uint32_t*)(hz + (size_t)kMlpOut * m);
    QOZ_TRY(to_host(c, hz, D + o_logit, 4 * (size_t)kMlpOut * m, s));
    QOZ_TRY(to_host(c, hs, D + o_st, 16 * (size_t)m, s));
    QOZ_HIP(hipGetLastError());
    QOZ_HIP(hipStreamSynchronize(s));
    prof_collect(c);
    for (uint32_t k = 0; k < m; ++k) {
      const Job& j = jobs[k];
      qoz_learned_item& it = items[j.item];
      if (hs[4 * k] & kStNonFinite) {
        it.status = QOZ_EINVAL;
        continue;
      }
      uint32_t pick[3];
      if (decide(hz + (size_t)kMlpOut * k, pick) < min_confidence) {
        fall.push_back(j.item);
        continue;
      }
      it.params = learned_params(pick, j.sa, j.L, j.d);
    }
  }
  /* the online tuner for the rest, in item order */
  std::sort(fall.begin(), fall.end());
  for (uint32_t i : fall) {
    qoz_learned_item& it = items[i];
    it.used_fallback = 1;
    it.status = qoz_tune(c, it.d_x, it.shape, it.abs_eb, fallback_target, cfg,
                         &it.params, s);
  }
  for (uint32_t i = 0; i < n; ++i)
    if (items[i].status != QOZ_OK)
      return fail(items[i].status, "a field of the batch failed");
  return QOZ_OK;
}
