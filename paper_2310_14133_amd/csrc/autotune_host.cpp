/*
 * Launch-tile autotuning of the interpolation sweeps.  A sweep's targets
 * are rows of up to 64 consecutive points (lanes along the row); how many
 * rows a workgroup takes and how many a lane loops over trade parallelism
 * for the reuse of neighbour rows in cache, and the best choice depends on
 * the sweep's stride and extent.  Each sweep of a plan is timed with every
 * candidate on scratch data (the work per target does not depend on the
 * values) and the fastest is kept in the context for that plan's geometry.
 * The fused level-1 row kernels keep their own configuration.
 */
#include <vector>

#include "qoz_internal.h"

namespace qoz {

static const SweepTile kTileCands[] = {{1, 1}, {2, 1}, {4, 1}, {8, 1},
                                       {16, 1}, {4, 2}, {4, 4}, {8, 2},
                                       {16, 2}};
constexpr int kTileReps = 3;

/* Fastest candidate for one sweep: *out, its time *t_best and the default
 * tile's time *t_def (ms, the minimum over the repetitions). */
template <class Fn>
static qoz_status best_tile(hipStream_t s, hipEvent_t a, hipEvent_t b, Fn fn,
                            SweepTile* out, float* t_best, float* t_def) {
  const SweepTile dflt;
  float best = 0.0f;
  bool have = false;
  for (const SweepTile& t : kTileCands) {
    fn(t); /* warm-up */
    float tmin = 0.0f;
    for (int r = 0; r < kTileReps; ++r) {
      QOZ_HIP(hipEventRecord(a, s));
      fn(t);
      QOZ_HIP(hipEventRecord(b, s));
      QOZ_HIP(hipEventSynchronize(b));
      float ms = 0.0f;
      QOZ_HIP(hipEventElapsedTime(&ms, a, b));
      if (r == 0 || ms < tmin) tmin = ms;
    }
    if (t.ty == dflt.ty && t.rpt == dflt.rpt) *t_def = tmin;
    if (!have || tmin < best) {
      best = tmin;
      *out = t;
      have = true;
    }
  }
  *t_best = best;
  return QOZ_OK;
}

}  // namespace qoz

using namespace qoz;

extern "C" qoz_status qoz_autotune_tiles(qoz_ctx* c, qoz_shape shape,
                                         const qoz_params* params,
                                         uint32_t* n_sweeps,
                                         float* ms_default, float* ms_tuned,
                                         hipStream_t s) {
  clear_error();
  if (!c || !params) return fail(QOZ_EINVAL, "NULL argument");
  QOZ_TRY(set_device(c));
  Plan P;
  if (make_plan(shape, 1.0, *params, &P) != QOZ_OK)
    return fail(QOZ_EINVAL, "bad shape or parameters");
  const uint64_t N = (uint64_t)P.g.n[0] * P.g.n[1] * P.g.n[2];
  QOZ_TRY(ensure(c->W, 4 * N));
  QOZ_TRY(ensure(c->ptmp, 4 * N));
  QOZ_TRY(ensure(c->codes, 2 * (P.n_codes + 16)));
  QOZ_TRY(ensure(c->status, 256));
  float* x = (float*)c->ptmp.p;
  float* W = (float*)c->W.p;
  uint16_t* codes = (uint16_t*)c->codes.p;
  uint32_t* st = (uint32_t*)c->status.p;
  launch_zero_u32((uint32_t*)x, N, s);
  launch_zero_u32((uint32_t*)W, N, s);
  launch_zero_u32((uint32_t*)codes, (2 * (P.n_codes + 16)) / 4, s);
  launch_init_status(st, s);
  size_t fz = SIZE_MAX, fa = SIZE_MAX, fb = SIZE_MAX;
  RowJob rj;
  const bool fuse = level1_rows(P, &fz, &fa, &fb, &rj);
  hipEvent_t a = nullptr, b = nullptr;
  QOZ_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(QOZ_EDEVICE, "hipEventCreate failed");
  }
  const size_t ns = P.sweeps.size();
  std::vector<SweepTile> tc(ns), td(ns);
  uint32_t tuned = 0;
  float sum_def = 0.0f, sum_best = 0.0f, tb = 0.0f, tdf = 0.0f;
  qoz_status st_ = QOZ_OK;
  for (size_t i = 0; i < ns && st_ == QOZ_OK; ++i) {
    if (fuse && (i == fz || i == fa || i == fb)) continue;
    const Sweep& sw = P.sweeps[i];
    const bool last = i + 1 == ns;
    st_ = best_tile(s, a, b, [&](SweepTile t) {
      launch_sweep_comp(P.g, sw, x, W, codes, !last, st, s, t);
    }, &tc[i], &tb, &tdf);
    sum_def += tdf;
    sum_best += tb;
    if (st_ == QOZ_OK)
      st_ = best_tile(s, a, b, [&](SweepTile t) {
        launch_sweep_decomp(P.g, sw, W, codes, s, t);
      }, &td[i], &tb, &tdf);
    sum_def += tdf;
    sum_best += tb;
    ++tuned;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  QOZ_TRY(st_);
  QOZ_HIP(hipGetLastError());
  QOZ_HIP(hipStreamSynchronize(s));
  const std::vector<uint32_t> key = tile_key(P);
  c->tiles_comp[key] = tc;
  c->tiles_decomp[key] = td;
  if (n_sweeps) *n_sweeps = tuned;
  if (ms_default) *ms_default = sum_def;
  if (ms_tuned) *ms_tuned = sum_best;
  return QOZ_OK;
}
