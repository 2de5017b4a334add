/*
 * Online tuner kernels (Sec. VI) for gfx950.
 *
 * Uniformly sampled blocks (Sec. VI-A) are gathered into a compact buffer,
 * (b+1)^d points each.  A trial runs the same predictor and quantizer as
 * the full compression on each block, treated as a field of its own whose
 * points on the 2^Lt grid are known exactly.
 *
 * One workgroup owns one (candidate, block) pair and walks the block's
 * sweeps in order with a workgroup barrier between sweeps.  Its working
 * copy of the block lives in LDS when it fits (a 33^3 block takes 140 KB of
 * the CU's 160 KB; 1024 lanes per workgroup); Algorithm 1 keeps only the
 * level's sub-grid (stride 2^(l-1)) there, compacted, so a level-l sweep
 * becomes a stride-1 sweep of the compact grid.  Larger blocks use a
 * working copy in global memory.
 *  - k_alg1_level: Algorithm 1 -- the sweeps of level l for one candidate
 *    interpolator at the bound e, on top of the committed higher levels;
 *    reports the FP64 sum of |x - prediction| over the level's targets.
 *  - k_trial: one parameter set over all levels Lt..1; reports the bins'
 *    histogram (aggregated per trial), the unpredictable count and the FP64
 *    squared error.
 */
#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kTuneThreads = 256;

/* (candidate or trial, block) of a workgroup of a (gridDim.x, gridDim.y)
 * grid, ordered so that each of the 8 XCDs (dispatched round-robin, each
 * with its own L2) takes consecutive items: the candidates of one block
 * then read its samples from the same L2. */
struct Item {
  uint32_t c, blk;
};
__device__ __forceinline__ Item xcd_item() {
  const uint32_t total = gridDim.x * gridDim.y;
  uint32_t id = blockIdx.x + gridDim.x * blockIdx.y;
  if (total % 8 == 0) id = (id % 8) * (total / 8) + id / 8;
  return Item{id % gridDim.x, id / gridDim.x};
}

__device__ __forceinline__ void block_subgrid(const Geo& g,
                                              const uint32_t* order,
                                              uint32_t d, uint32_t j,
                                              uint32_t h, uint32_t* start,
                                              uint32_t* step, uint32_t* cnt) {
  for (int m = 0; m < 3; ++m) {
    start[m] = 0;
    step[m] = 1;
    cnt[m] = g.n[m];
  }
  for (uint32_t pos = 0; pos < d; ++pos) {
    uint32_t m = order[pos];
    start[m] = pos == j ? h : 0;
    step[m] = pos < j ? h : 2 * h;
    cnt[m] = start[m] < g.n[m] ? (g.n[m] - 1 - start[m]) / step[m] + 1 : 0;
  }
}

__device__ __forceinline__ double block_reduce_f64(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (uint32_t o = kTuneThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  return sh[0];
}

/* Copy the points of the 2^lg grid of a block from src to dst. */
__device__ __forceinline__ void copy_grid(const Geo& g, uint32_t lg,
                                          const float* src, float* dst) {
  const uint32_t st = 1u << lg;
  const uint32_t m0 = (g.n[0] - 1) / st + 1, m1 = (g.n[1] - 1) / st + 1,
                 m2 = (g.n[2] - 1) / st + 1;
  const uint32_t total = m0 * m1 * m2;
  const FastDiv f2(m2, total), f1(m1, total);
  for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) {
    const uint32_t r = f2.div(t), a2 = t - r * m2;
    const uint32_t a0 = f1.div(r), a1 = r - a0 * m1;
    uint32_t idx = a0 * st * g.st[0] + a1 * st * g.st[1] + a2 * st;
    dst[idx] = src[idx];
  }
}

/* The sampled blocks into xs and its committed copy wc: workgroup
 * (blockIdx.x, blockIdx.y) takes points [2048 blockIdx.x, +2048) of block
 * blockIdx.y in row-major order, eight per lane with all loads in flight;
 * the stores are contiguous, the loads rows of the field. */
constexpr uint32_t kGatherThreads = 256;
constexpr uint32_t kGatherPer = 8;

__global__ __launch_bounds__(kGatherThreads) void k_gather_blocks(
    const float* __restrict__ x, Geo g, BlockGeo bg,
    const uint32_t* __restrict__ origins, float* __restrict__ xs,
    float* __restrict__ wc, uint32_t* status) {
  const uint32_t blk = blockIdx.y;
  const uint32_t n1 = bg.g.n[1], n2 = bg.g.n[2], size = bg.size;
  const FastDiv f2(n2, size), f1(n1, size);
  const uint32_t* o = origins + 3 * blk;
  const uint32_t t0 = blockIdx.x * kGatherThreads * kGatherPer + threadIdx.x;
  float v[kGatherPer];
#pragma unroll
  for (uint32_t u = 0; u < kGatherPer; ++u) {
    const uint32_t t = t0 + u * kGatherThreads;
    if (t < size) {
      const uint32_t r = f2.div(t), i2 = t - r * n2;
      const uint32_t i0 = f1.div(r), i1 = r - i0 * n1;
      v[u] = x[(uint64_t)(o[0] + i0) * g.st[0] +
               (uint64_t)(o[1] + i1) * g.st[1] + o[2] + i2];
    }
  }
  const uint64_t base = (uint64_t)blk * size;
  bool bad = false;
#pragma unroll
  for (uint32_t u = 0; u < kGatherPer; ++u) {
    const uint32_t t = t0 + u * kGatherThreads;
    if (t < size) {
      xs[base + t] = v[u];
      wc[base + t] = v[u];
      bad |= !isfinite(v[u]);
    }
  }
  /* non-finite sampled values (the ratio target reads nothing else) */
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, kStNonFinite);
}

void launch_gather_blocks(const float* x, const Geo& g, const BlockGeo& bg,
                          const uint32_t* origins_dev, float* xs, float* wc,
                          uint32_t* status, hipStream_t s) {
  if (!bg.size || !bg.nb) return;
  const uint32_t per = kGatherThreads * kGatherPer;
  QOZ_LAUNCH(k_gather_blocks, dim3((bg.size + per - 1) / per, bg.nb),
                     dim3(kGatherThreads), 0, s, x, g, bg, origins_dev, xs,
                     wc, status);
}

__global__ __launch_bounds__(kTuneThreads) void k_alg1_level(
    BlockGeo bg, uint32_t l, const float* __restrict__ xs,
    const float* __restrict__ wc, float* wt, const TrialDesc* desc,
    double* l1_part) {
  __shared__ double red[kTuneThreads];
  const uint32_t c = blockIdx.x, blk = blockIdx.y;
  const Geo& g = bg.g;
  const float* X = xs + (uint64_t)blk * bg.size;
  float* Wt = wt + ((uint64_t)c * bg.nb + blk) * bg.size;
  copy_grid(g, l, wc + (uint64_t)blk * bg.size, Wt);
  __syncthreads();
  const TrialLevel lv = desc[c].lv[l - 1];
  const uint32_t h = 1u << (l - 1);
  double l1 = 0.0;
  for (uint32_t j = 0; j < bg.d; ++j) {
    uint32_t start[3], step[3], cnt[3];
    block_subgrid(g, lv.order, bg.d, j, h, start, step, cnt);
    const uint32_t k = lv.order[j];
    const uint32_t count = cnt[0] * cnt[1] * cnt[2];
    const FastDiv f2(cnt[2], count), f1(cnt[1], count);
    for (uint32_t t = threadIdx.x; t < count; t += blockDim.x) {
      const uint32_t r = f2.div(t), i2 = t - r * cnt[2];
      const uint32_t i0 = f1.div(r), i1 = r - i0 * cnt[1];
      uint32_t p[3] = {start[0] + i0 * step[0], start[1] + i1 * step[1],
                       start[2] + i2 * step[2]};
      uint32_t idx = p[0] * g.st[0] + p[1] * g.st[1] + p[2];
      float pred = predict_at(Wt, idx, p[k], g.st[k], g.n[k], h, lv.cubic);
      float xv = X[idx];
      l1 += fabs((double)xv - (double)pred);
      float rec;
      quantize_bin(xv, pred, lv.inv, lv.twoeb, lv.eb, &rec);
      Wt[idx] = rec;
    }
    __syncthreads();
  }
  double tot = block_reduce_f64(l1, red);
  if (threadIdx.x == 0) l1_part[(uint64_t)c * bg.nb + blk] = tot;
}

/* ---- LDS-resident variants ---- */
constexpr uint32_t kLdsThreads = 1024;
constexpr uint32_t kLdsBatch = 8; /* loads per lane in flight */

/* predict_at for a working copy in LDS, without branches: every operand is
 * read from an in-range index (the target itself stands in for a missing
 * neighbour, whose value is then not used) and the rule is selected; the
 * selected rule's arithmetic is that of interp_mid. */
__device__ __forceinline__ float predict_lds(const float* W, uint32_t idx,
                                             uint32_t pk, uint32_t sk,
                                             uint32_t nk, uint32_t h,
                                             uint32_t cubic) {
  const uint32_t hs = h * sk;
  const bool ha = pk >= 3 * h, hc = pk + h < nk, hd = pk + 3 * h < nk;
  const float b = W[idx - hs];
  const float c = W[hc ? idx + hs : idx];
  const float a = W[ha ? idx - 3 * hs : idx];
  const float ext = ha ? (b * 3.0f - a) * 0.5f : b;
  const float mid = (b + c) * 0.5f;
  float in = mid;
  if (cubic) {
    const float d = W[hd ? idx + 3 * hs : idx];
    const float c4 = ((b + c) * 9.0f - (a + d)) * 0.0625f;
    const float c3d = ((b * 3.0f + c * 6.0f) - d) * 0.125f;
    const float c3a = ((b * 6.0f + c * 3.0f) - a) * 0.125f;
    in = ha ? (hd ? c4 : c3a) : (hd ? c3d : mid);
  }
  return hc ? in : ext;
}

/* quantize_bin without branches (same arithmetic and outcomes) */
__device__ __forceinline__ int32_t quantize_sel(float x, float pred,
                                                float inv, float twoeb,
                                                double eb, float* rec) {
  const float qf = (x - pred) * inv;
  const bool in = fabsf(qf) < 32768.0f;
  const int32_t q = (int32_t)rintf(in ? qf : 0.0f);
  const float r = pred + (float)q * twoeb;
  const bool ok = in && q < 32768 && q > -32768 &&
                  fabs((double)r - (double)x) <= eb;
  *rec = ok ? r : x;
  return ok ? q + 32768 : 0;
}

template <uint32_t NT>
__device__ __forceinline__ double lds_block_sum_f64(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (uint32_t w = 0; w < NT / 64; ++w) t += red[w];
  return t;
}

/* The sub-grid of a block at stride h (points at multiples of h),
 * compacted: extents (n - 1) / h + 1, row-major. */
__device__ __forceinline__ Geo compact_geo(const Geo& g, uint32_t h) {
  Geo cg;
  for (int i = 0; i < 3; ++i) cg.n[i] = (g.n[i] - 1) / h + 1;
  cg.st[2] = 1;
  cg.st[1] = cg.n[2];
  cg.st[0] = cg.n[1] * cg.n[2];
  return cg;
}

/* flat block index of compact point t of cg (stride h) */
struct CompactMap {
  Geo cg;
  uint32_t h, st0, st1;
  FastDiv f2, f1;
  __device__ __forceinline__ CompactMap(const Geo& g, const Geo& c,
                                        uint32_t hh, uint32_t total)
      : cg(c), h(hh), st0(g.st[0]), st1(g.st[1]), f2(c.n[2], total),
        f1(c.n[1], total) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t t) const {
    const uint32_t r = f2.div(t), q2 = t - r * cg.n[2];
    const uint32_t q0 = f1.div(r), q1 = r - q0 * cg.n[1];
    return h * (q0 * st0 + q1 * st1 + q2);
  }
};

/* dst[t] = src[map(t)] (gather) or dst[map(t)] = src[t] (scatter) for
 * t < total, with kLdsBatch loads per lane in flight */
template <uint32_t NT, bool SCATTER>
__device__ __forceinline__ void copy_mapped(float* dst, const float* src,
                                            uint32_t total,
                                            const CompactMap& map) {
  for (uint32_t t0 = threadIdx.x; t0 < total; t0 += kLdsBatch * NT) {
    float v[kLdsBatch];
    uint32_t m[kLdsBatch];
#pragma unroll
    for (uint32_t u = 0; u < kLdsBatch; ++u) {
      const uint32_t t = t0 + u * NT;
      m[u] = t < total ? map(t) : 0u;
      v[u] = t < total ? src[SCATTER ? t : m[u]] : 0.0f;
    }
#pragma unroll
    for (uint32_t u = 0; u < kLdsBatch; ++u)
      if (t0 + u * NT < total) dst[SCATTER ? m[u] : t0 + u * NT] = v[u];
  }
}

/* One sweep over a working copy W in LDS: targets of sub-grid
 * (start, step, cnt) of geometry g, predicted along k at distance h;
 * x values from X (index scaled by xh), kLdsBatch loads per lane in
 * flight.  body(x, pred, idx) handles each target. */
template <uint32_t NT, typename Body>
__device__ __forceinline__ void lds_sweep(const Geo& g, const uint32_t* start,
                                          const uint32_t* step,
                                          const uint32_t* cnt, uint32_t k,
                                          uint32_t h, uint32_t cubic,
                                          const float* W, const float* X,
                                          const Geo& xg, uint32_t xh,
                                          Body body) {
  const uint32_t count = cnt[0] * cnt[1] * cnt[2];
  if (count == 0) return;
  const FastDiv f2(cnt[2], count), f1(cnt[1], count);
  /* NT = a2 cnt[2] + b2 and a2 = a1 cnt[1] + b1: with 256 threads the
   * coordinates of t + NT follow from those of t with one carry per
   * dimension (measured faster there; with 1024 threads, slower than the
   * two divisions per point) */
  constexpr bool kStep = NT <= 256;
  const uint32_t a2 = NT / cnt[2], b2 = NT - a2 * cnt[2];
  const uint32_t a1 = a2 / cnt[1], b1 = a2 - a1 * cnt[1];
  for (uint32_t t0 = threadIdx.x; t0 < count; t0 += kLdsBatch * NT) {
    uint32_t li[kLdsBatch], pk[kLdsBatch];
    float xv[kLdsBatch];
    uint32_t i0, i1, i2;
    {
      const uint32_t r = f2.div(t0);
      i2 = t0 - r * cnt[2];
      i0 = f1.div(r);
      i1 = r - i0 * cnt[1];
    }
#pragma unroll
    for (uint32_t u = 0; u < kLdsBatch; ++u) {
      const uint32_t t = t0 + u * NT;
      if (!kStep) {
        const uint32_t tt = t < count ? t : 0u;
        const uint32_t r = f2.div(tt);
        i2 = tt - r * cnt[2];
        i0 = f1.div(r);
        i1 = r - i0 * cnt[1];
      } else if (u) {
        i2 += b2;
        const uint32_t c2 = i2 >= cnt[2] ? 1u : 0u;
        i2 -= c2 ? cnt[2] : 0u;
        i1 += b1 + c2;
        i0 += a1;
        if (i1 >= cnt[1]) {
          i1 -= cnt[1];
          ++i0;
        }
      }
      /* past the end: any in-range point (nothing is read or written;
       * the divisions above already start from point 0 there) */
      const bool in = t < count;
      const bool clamp = kStep && !in;
      const uint32_t q[3] = {start[0] + (clamp ? 0u : i0) * step[0],
                             start[1] + (clamp ? 0u : i1) * step[1],
                             start[2] + (clamp ? 0u : i2) * step[2]};
      li[u] = q[0] * g.st[0] + q[1] * g.st[1] + q[2];
      pk[u] = q[k];
      xv[u] = in
                  ? X[xh * (q[0] * xg.st[0] + q[1] * xg.st[1] + q[2])]
                  : 0.0f;
    }
#pragma unroll
    for (uint32_t u = 0; u < kLdsBatch; ++u) {
      if (t0 + u * NT >= count) break;
      body(xv[u], predict_lds(W, li[u], pk[u], g.st[k], g.n[k], h, cubic),
           li[u]);
    }
  }
}

/* Algorithm 1 for one level in LDS: candidate blockIdx.x on block
 * blockIdx.y; the per-block sum of |x - prediction| goes to l1_part and,
 * when a finer level follows (keep), the compact reconstruction to the
 * candidate's slot in wt (its first `total` floats), from which the chosen
 * one is committed. */
template <uint32_t NT>
__global__ __launch_bounds__(NT) void k_alg1_lds(
    BlockGeo bg, uint32_t l, const float* __restrict__ xs,
    const float* __restrict__ wc, float* __restrict__ wt,
    const TrialDesc* __restrict__ desc, double* l1_part, uint32_t keep) {
  extern __shared__ float Ws[];
  __shared__ double red[NT / 64];
  const Item item = xcd_item();
  const uint32_t c = item.c, blk = item.blk;
  const uint32_t h = 1u << (l - 1);
  const Geo& g = bg.g;
  const Geo cg = compact_geo(g, h);
  const uint32_t total = cg.n[0] * cg.n[1] * cg.n[2];
  const float* X = xs + (uint64_t)blk * bg.size;
  const float* src = wc + (uint64_t)blk * bg.size;
  if (h == 1) {
    /* the whole block: a plain copy, no index map */
    for (uint32_t t0 = threadIdx.x; t0 < total; t0 += kLdsBatch * NT) {
      float v[kLdsBatch];
#pragma unroll
      for (uint32_t u = 0; u < kLdsBatch; ++u)
        v[u] = t0 + u * NT < total ? src[t0 + u * NT] : 0.0f;
#pragma unroll
      for (uint32_t u = 0; u < kLdsBatch; ++u)
        if (t0 + u * NT < total) Ws[t0 + u * NT] = v[u];
    }
  } else {
    copy_mapped<NT, false>(Ws, src, total, CompactMap(g, cg, h, total));
  }
  __syncthreads();
  const TrialLevel lv = desc[c].lv[l - 1];
  double l1 = 0.0;
  for (uint32_t j = 0; j < bg.d; ++j) {
    uint32_t start[3], step[3], cnt[3];
    block_subgrid(cg, lv.order, bg.d, j, 1, start, step, cnt);
    lds_sweep<NT>(cg, start, step, cnt, lv.order[j], 1, lv.cubic, Ws, X, g,
                  h, [&](float xv, float pred, uint32_t li) {
                    l1 += fabs((double)xv - (double)pred);
                    float rec;
                    quantize_sel(xv, pred, lv.inv, lv.twoeb, lv.eb, &rec);
                    Ws[li] = rec;
                  });
    __syncthreads();
  }
  if (keep) {
    float* Wo = wt + ((uint64_t)c * bg.nb + blk) * bg.size;
    for (uint32_t t = threadIdx.x; t < total; t += NT) Wo[t] = Ws[t];
  }
  const double tot = lds_block_sum_f64<NT>(l1, red);
  if (threadIdx.x == 0) l1_part[(uint64_t)c * bg.nb + blk] = tot;
}

/* wc's level-l sub-grid from the chosen candidate's compact copies */
__global__ void k_alg1_commit(BlockGeo bg, uint32_t l,
                              const float* __restrict__ wt,
                              const uint32_t* __restrict__ pick,
                              float* __restrict__ wc) {
  const uint32_t blk = blockIdx.y, h = 1u << (l - 1);
  const Geo& g = bg.g;
  const Geo cg = compact_geo(g, h);
  const uint32_t total = cg.n[0] * cg.n[1] * cg.n[2];
  const float* src = wt + ((uint64_t)(*pick) * bg.nb + blk) * bg.size;
  float* dst = wc + (uint64_t)blk * bg.size;
  const CompactMap map(g, cg, h, total);
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += gridDim.x * blockDim.x)
    dst[map(t)] = src[t];
}

/* Algorithm 1's choice and the commit of its reconstruction in one launch:
 * every workgroup forms the candidates' means itself (the same sums in the
 * same order as k_alg1_pick, a lane per candidate: at most 64) and takes
 * the first strict minimum; workgroup (0, 0) records it. */
__global__ __launch_bounds__(256) void k_alg1_pick_commit(
    BlockGeo bg, uint32_t l, const double* __restrict__ l1_part,
    uint32_t ncand, double count, uint32_t* pick,
    const float* __restrict__ wt, float* __restrict__ wc) {
  __shared__ uint32_t s_pick;
  if (threadIdx.x < 64) {
    const uint32_t ci = threadIdx.x;
    double cur = INFINITY;
    if (ci < ncand) {
      double sum = 0.0;
      for (uint32_t k = 0; k < bg.nb; ++k) sum += l1_part[(size_t)ci * bg.nb + k];
      cur = count > 0 ? sum / count : 0.0;
    }
    /* the first candidate whose mean is below every earlier one's and not
     * above any later one's: the smallest index among the minima (none
     * when every mean is NaN or infinite: candidate 0) */
    double m = cur;
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    const uint64_t at = __ballot(ci < ncand && cur == m && cur < INFINITY);
    if (ci == 0) s_pick = at ? (uint32_t)__ffsll((unsigned long long)at) - 1 : 0u;
  }
  __syncthreads();
  const uint32_t ib = s_pick;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *pick = ib;
  const uint32_t blk = blockIdx.y, h = 1u << (l - 1);
  const Geo& g = bg.g;
  const Geo cg = compact_geo(g, h);
  const uint32_t total = cg.n[0] * cg.n[1] * cg.n[2];
  const float* src = wt + ((uint64_t)ib * bg.nb + blk) * bg.size;
  float* dst = wc + (uint64_t)blk * bg.size;
  const CompactMap map(g, cg, h, total);
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += gridDim.x * blockDim.x)
    dst[map(t)] = src[t];
}

/* Dynamic LDS for `bytes` of working copy next to `static_bytes`, or false
 * when the device cannot give a workgroup that much. */
static bool lds_fits(const void* fn, size_t bytes, size_t static_bytes) {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            dev) != hipSuccess)
    return false;
  if (bytes + static_bytes > (size_t)max_lds) return false;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes) == hipSuccess;
}

static size_t alg1_lds_bytes(const BlockGeo& bg, uint32_t l) {
  const uint32_t h = 1u << (l - 1);
  size_t n = 1;
  for (int i = 0; i < 3; ++i) n *= (bg.g.n[i] - 1) / h + 1;
  return 4 * n;
}

/* small sub-grids take 256 lanes per workgroup, larger ones 1024 */
constexpr size_t kAlg1WideBytes = 4 * 8192;

bool alg1_in_lds(const BlockGeo& bg, uint32_t l) {
  const size_t bytes = alg1_lds_bytes(bg, l);
  return bytes <= kAlg1WideBytes
             ? lds_fits(reinterpret_cast<const void*>(&k_alg1_lds<256>),
                        bytes, sizeof(double) * 4)
             : lds_fits(reinterpret_cast<const void*>(&k_alg1_lds<kLdsThreads>),
                        bytes, sizeof(double) * (kLdsThreads / 64));
}

void launch_alg1_level(const BlockGeo& bg, uint32_t l, const float* xs,
                       const float* wc, float* wt, uint32_t ncand,
                       const TrialDesc* cand_desc, double* l1_part,
                       bool in_lds, bool keep, hipStream_t s) {
  if (in_lds) {
    const size_t bytes = alg1_lds_bytes(bg, l);
    if (bytes <= kAlg1WideBytes)
      QOZ_LAUNCH(k_alg1_lds<256>, dim3(ncand, bg.nb), dim3(256), bytes, s,
                 bg, l, xs, wc, wt, cand_desc, l1_part, keep ? 1u : 0u);
    else
      QOZ_LAUNCH(k_alg1_lds<kLdsThreads>, dim3(ncand, bg.nb),
                 dim3(kLdsThreads), bytes, s, bg, l, xs, wc, wt, cand_desc,
                 l1_part, keep ? 1u : 0u);
    return;
  }
  QOZ_LAUNCH(k_alg1_level, dim3(ncand, bg.nb), dim3(kTuneThreads), 0,
                     s, bg, l, xs, wc, wt, cand_desc, l1_part);
}

/* Algorithm 1's choice at one level, on the device: the mean absolute
 * prediction error of each candidate (its per-block sums added in block
 * order, then divided by the level's target count) and the first strict
 * minimum over candidates in order. */
constexpr uint32_t kPickThreads = 64;

__global__ __launch_bounds__(kPickThreads) void k_alg1_pick(
    const double* __restrict__ l1_part, uint32_t ncand, uint32_t nb,
    double count, uint32_t* pick) {
  __shared__ double cur[kPickThreads];
  for (uint32_t ci = threadIdx.x; ci < ncand; ci += kPickThreads) {
    double sum = 0.0;
    for (uint32_t k = 0; k < nb; ++k) sum += l1_part[(size_t)ci * nb + k];
    cur[ci] = count > 0 ? sum / count : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double best = INFINITY;
    uint32_t ib = 0;
    for (uint32_t ci = 0; ci < ncand; ++ci)
      if (cur[ci] < best) {
        best = cur[ci];
        ib = ci;
      }
    *pick = ib;
  }
}

/* The trials' interpolation types and orders from Algorithm 1's choices:
 * level l of every trial takes the chosen candidate's (a choice out of
 * range, which the host rejects afterwards, reads candidate 0). */
__global__ void k_trial_fill(TrialDesc* __restrict__ desc, uint32_t ntrial,
                             uint32_t Lt, const TrialDesc* __restrict__ cand,
                             uint32_t ncand,
                             const uint32_t* __restrict__ pick) {
  const uint32_t t = blockIdx.x, l = threadIdx.x;
  if (t >= ntrial || l >= Lt) return;
  const uint32_t ci = pick[l] < ncand ? pick[l] : 0u;
  const TrialLevel& src = cand[(size_t)l * ncand + ci].lv[l];
  TrialLevel& dst = desc[t].lv[l];
  dst.cubic = src.cubic;
  for (int j = 0; j < 3; ++j) dst.order[j] = src.order[j];
}

void launch_trial_fill(TrialDesc* desc, uint32_t ntrial, uint32_t Lt,
                       const TrialDesc* cand, uint32_t ncand,
                       const uint32_t* pick, hipStream_t s) {
  if (!ntrial || !Lt) return;
  QOZ_LAUNCH(k_trial_fill, dim3(ntrial), dim3(64), 0, s, desc, ntrial, Lt,
             cand, ncand, pick);
}

/* commit the chosen candidate's working copy: wc = wt[pick] */
__global__ void k_commit_copy(const float* __restrict__ wt,
                              const uint32_t* __restrict__ pick, uint64_t n,
                              float* __restrict__ wc) {
  const float* src = wt + (uint64_t)(*pick) * n;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    wc[i] = src[i];
}

void launch_alg1_pick(const BlockGeo& bg, uint32_t l, const float* xs,
                      const TrialDesc* cand_desc, const double* l1_part,
                      uint32_t ncand, double count, uint32_t* pick,
                      const float* wt, float* wc, bool in_lds, bool keep,
                      hipStream_t s) {
  const uint32_t nb = bg.nb;
  if (in_lds && keep && ncand <= 64) {
    const uint32_t total = (uint32_t)(alg1_lds_bytes(bg, l) / 4);
    QOZ_LAUNCH(k_alg1_pick_commit, dim3((total + 255) / 256, nb), dim3(256),
               0, s, bg, l, l1_part, ncand, count, pick, wt, wc);
    return;
  }
  QOZ_LAUNCH(k_alg1_pick, dim3(1), dim3(kPickThreads), 0, s, l1_part,
                     ncand, nb, count, pick);
  if (!keep && in_lds) return; /* no finer level reads the working copy */
  if (in_lds) {
    const uint32_t total = (uint32_t)(alg1_lds_bytes(bg, l) / 4);
    QOZ_LAUNCH(k_alg1_commit, dim3((total + 255) / 256, nb),
                       dim3(256), 0, s, bg, l, wt, pick, wc);
    return;
  }
  const uint64_t bsz = (uint64_t)nb * bg.size;
  uint64_t blocks = (bsz + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  QOZ_LAUNCH(k_commit_copy, dim3((uint32_t)blocks), dim3(256), 0, s,
                     wt, pick, bsz, wc);
}

__global__ __launch_bounds__(kTuneThreads) void k_trial(
    BlockGeo bg, const float* __restrict__ xs, float* wt,
    const TrialDesc* desc, uint32_t* hist, double* sse_part,
    uint32_t* unpred_part) {
  __shared__ uint32_t lh[kHistWin];
  __shared__ double red[kTuneThreads];
  __shared__ uint32_t ured[kTuneThreads / 64];
  const uint32_t tr = blockIdx.x, blk = blockIdx.y;
  const Geo& g = bg.g;
  const float* X = xs + (uint64_t)blk * bg.size;
  float* Wt = wt + ((uint64_t)tr * bg.nb + blk) * bg.size;
  uint32_t* H = hist + (uint64_t)tr * kNSym;
  for (uint32_t i = threadIdx.x; i < kHistWin; i += blockDim.x) lh[i] = 0;
  copy_grid(g, bg.Lt, X, Wt);
  __syncthreads();
  uint32_t center = 0, nun = 0;
  double sse = 0.0;
  for (uint32_t l = bg.Lt; l >= 1; --l) {
    const TrialLevel lv = desc[tr].lv[l - 1];
    const uint32_t h = 1u << (l - 1);
    for (uint32_t j = 0; j < bg.d; ++j) {
      uint32_t start[3], step[3], cnt[3];
      block_subgrid(g, lv.order, bg.d, j, h, start, step, cnt);
      const uint32_t k = lv.order[j];
      const uint32_t count = cnt[0] * cnt[1] * cnt[2];
      const FastDiv f2(cnt[2], count), f1(cnt[1], count);
      for (uint32_t t = threadIdx.x; t < count; t += blockDim.x) {
        const uint32_t r = f2.div(t), i2 = t - r * cnt[2];
        const uint32_t i0 = f1.div(r), i1 = r - i0 * cnt[1];
        uint32_t p[3] = {start[0] + i0 * step[0], start[1] + i1 * step[1],
                         start[2] + i2 * step[2]};
        uint32_t idx = p[0] * g.st[0] + p[1] * g.st[1] + p[2];
        float pred = predict_at(Wt, idx, p[k], g.st[k], g.n[k], h, lv.cubic);
        float xv = X[idx];
        float rec;
        int32_t code = quantize_bin(xv, pred, lv.inv, lv.twoeb, lv.eb, &rec);
        Wt[idx] = rec;
        hist_add(lh, H, code, center);
        nun += code == 0;
        double dd = (double)xv - (double)rec;
        sse += dd * dd;
      }
      __syncthreads();
    }
  }
  center = wave_sum_u32(center);
  uint32_t wn = wave_sum_u32(nun);
  if ((threadIdx.x & 63) == 0) {
    if (center) atomicAdd(&lh[32768 - kHistBase], center);
    ured[threadIdx.x >> 6] = wn;
  }
  double tot = block_reduce_f64(sse, red); /* contains a barrier */
  for (uint32_t i = threadIdx.x; i < kHistWin; i += blockDim.x) {
    uint32_t v = lh[i];
    if (v) atomicAdd(&H[kHistBase + (int32_t)i], v);
  }
  if (threadIdx.x == 0) {
    uint32_t u = 0;
    for (uint32_t w = 0; w < kTuneThreads / 64; ++w) u += ured[w];
    const uint64_t item = (uint64_t)tr * bg.nb + blk;
    sse_part[2 * item] = tot;
    sse_part[2 * item + 1] = 0.0;
    unpred_part[2 * item] = u;
    unpred_part[2 * item + 1] = 0;
  }
}

/* A trial in LDS, in two launches.  Levels Lt..2 touch only the block's
 * stride-2 sub-grid: k_trial_hi keeps that sub-grid, compacted, and its x
 * values in LDS (level l of the block is level l - 1 of the compact grid)
 * and leaves its reconstruction in the trial's wt slot.  k_trial_l1 puts
 * it back on the even points of a full working copy and runs level 1 with
 * x from global memory.  Each writes its own FP64 squared-error and
 * unpredictable-count partial (slot 2 i and 2 i + 1 of item i); with
 * `keep` the full reconstruction is left in wt (the SSIM target reads it). */
constexpr uint32_t kHiThreads = 256;

template <uint32_t NT>
__device__ __forceinline__ void trial_flush(uint32_t* lh, uint32_t* H,
                                            uint32_t center, uint32_t nun,
                                            double sse, double* red,
                                            uint32_t* ured, double* sse_out,
                                            uint32_t* un_out) {
  center = wave_sum_u32(center);
  const uint32_t wn = wave_sum_u32(nun);
  if ((threadIdx.x & 63) == 0) {
    if (center) atomicAdd(&lh[32768 - kHistBase], center);
    ured[threadIdx.x >> 6] = wn;
  }
  const double tot = lds_block_sum_f64<NT>(sse, red); /* has a barrier */
  for (uint32_t i = threadIdx.x; i < kHistWin; i += NT) {
    const uint32_t v = lh[i];
    if (v) atomicAdd(&H[kHistBase + (int32_t)i], v);
  }
  if (threadIdx.x == 0) {
    uint32_t u = 0;
    for (uint32_t w = 0; w < NT / 64; ++w) u += ured[w];
    *sse_out = tot;
    *un_out = u;
  }
}

__global__ __launch_bounds__(kHiThreads) void k_trial_hi(
    BlockGeo bg, const float* __restrict__ xs, float* __restrict__ wt,
    const TrialDesc* __restrict__ desc, uint32_t* hist, double* sse_part,
    uint32_t* unpred_part) {
  extern __shared__ float sm[];
  __shared__ uint32_t lh[kHistWin];
  __shared__ double red[kHiThreads / 64];
  __shared__ uint32_t ured[kHiThreads / 64];
  const Item xi = xcd_item();
  const uint32_t tr = xi.c, blk = xi.blk;
  const uint64_t item = (uint64_t)tr * bg.nb + blk;
  const Geo& g = bg.g;
  const Geo cg = compact_geo(g, 2);
  const uint32_t total = cg.n[0] * cg.n[1] * cg.n[2];
  float* Wq = sm;
  float* Xq = sm + total;
  for (uint32_t i = threadIdx.x; i < kHistWin; i += kHiThreads) lh[i] = 0;
  copy_mapped<kHiThreads, false>(Xq, xs + (uint64_t)blk * bg.size, total,
                                 CompactMap(g, cg, 2, total));
  __syncthreads();
  /* the 2^Lt grid of the block (2^(Lt-1) of the compact one) is exact */
  {
    const uint32_t m = (1u << (bg.Lt - 1)) - 1;
    const FastDiv f2(cg.n[2], total), f1(cg.n[1], total);
    for (uint32_t t = threadIdx.x; t < total; t += kHiThreads) {
      const uint32_t r = f2.div(t), q2 = t - r * cg.n[2];
      const uint32_t q0 = f1.div(r), q1 = r - q0 * cg.n[1];
      if (((q0 | q1 | q2) & m) == 0) Wq[t] = Xq[t];
    }
  }
  __syncthreads();
  uint32_t* H = hist + (uint64_t)tr * kNSym;
  uint32_t center = 0, nun = 0;
  double sse = 0.0;
  for (uint32_t l = bg.Lt; l >= 2; --l) {
    const TrialLevel lv = desc[tr].lv[l - 1];
    const uint32_t hc = 1u << (l - 2);
    for (uint32_t j = 0; j < bg.d; ++j) {
      uint32_t start[3], step[3], cnt[3];
      block_subgrid(cg, lv.order, bg.d, j, hc, start, step, cnt);
      lds_sweep<kHiThreads>(
          cg, start, step, cnt, lv.order[j], hc, lv.cubic, Wq, Xq, cg, 1,
          [&](float xv, float pred, uint32_t li) {
            float rec;
            const int32_t code =
                quantize_sel(xv, pred, lv.inv, lv.twoeb, lv.eb, &rec);
            Wq[li] = rec;
            hist_add(lh, H, code, center);
            nun += code == 0;
            const double dd = (double)xv - (double)rec;
            sse += dd * dd;
          });
      __syncthreads();
    }
  }
  float* Wo = wt + item * bg.size;
  for (uint32_t t = threadIdx.x; t < total; t += kHiThreads) Wo[t] = Wq[t];
  trial_flush<kHiThreads>(lh, H, center, nun, sse, red, ured,
                          sse_part + 2 * item, unpred_part + 2 * item);
}

__global__ __launch_bounds__(kLdsThreads) void k_trial_l1(
    BlockGeo bg, const float* __restrict__ xs, float* wt, uint32_t keep,
    const TrialDesc* __restrict__ desc, uint32_t* hist, double* sse_part,
    uint32_t* unpred_part) {
  extern __shared__ float Ws[];
  __shared__ uint32_t lh[kHistWin];
  __shared__ double red[kLdsThreads / 64];
  __shared__ uint32_t ured[kLdsThreads / 64];
  const Item xi = xcd_item();
  const uint32_t tr = xi.c, blk = xi.blk;
  const uint64_t item = (uint64_t)tr * bg.nb + blk;
  const Geo& g = bg.g;
  const float* X = xs + (uint64_t)blk * bg.size;
  float* Wt = wt + item * bg.size;
  for (uint32_t i = threadIdx.x; i < kHistWin; i += kLdsThreads) lh[i] = 0;
  {
    const Geo cg = compact_geo(g, 2);
    const uint32_t total = cg.n[0] * cg.n[1] * cg.n[2];
    copy_mapped<kLdsThreads, true>(Ws, Wt, total,
                                   CompactMap(g, cg, 2, total));
  }
  __syncthreads();
  uint32_t* H = hist + (uint64_t)tr * kNSym;
  uint32_t center = 0, nun = 0;
  double sse = 0.0;
  const TrialLevel lv = desc[tr].lv[0];
  for (uint32_t j = 0; j < bg.d; ++j) {
    uint32_t start[3], step[3], cnt[3];
    block_subgrid(g, lv.order, bg.d, j, 1, start, step, cnt);
    lds_sweep<kLdsThreads>(
        g, start, step, cnt, lv.order[j], 1, lv.cubic, Ws, X, g, 1,
        [&](float xv, float pred, uint32_t li) {
          float rec;
          const int32_t code =
              quantize_sel(xv, pred, lv.inv, lv.twoeb, lv.eb, &rec);
          Ws[li] = rec;
          hist_add(lh, H, code, center);
          nun += code == 0;
          const double dd = (double)xv - (double)rec;
          sse += dd * dd;
        });
    __syncthreads();
  }
  if (keep)
    for (uint32_t i = threadIdx.x; i < bg.size; i += kLdsThreads)
      Wt[i] = Ws[i];
  trial_flush<kLdsThreads>(lh, H, center, nun, sse, red, ured,
                           sse_part + 2 * item + 1,
                           unpred_part + 2 * item + 1);
}

void launch_trial(const BlockGeo& bg, const float* xs, float* wt,
                  uint32_t ntrial, const TrialDesc* desc, uint32_t* hist,
                  double* sse_part, uint32_t* unpred_part, bool keep_wt,
                  hipStream_t s) {
  size_t m2 = 1;
  for (int i = 0; i < 3; ++i) m2 *= (bg.g.n[i] - 1) / 2 + 1;
  const size_t hi_bytes = 8 * m2, l1_bytes = 4 * (size_t)bg.size;
  const size_t hi_stat = 4 * kHistWin + 12 * (kHiThreads / 64);
  const size_t l1_stat = 4 * kHistWin + 12 * (kLdsThreads / 64);
  if (lds_fits(reinterpret_cast<const void*>(&k_trial_hi), hi_bytes,
               hi_stat) &&
      lds_fits(reinterpret_cast<const void*>(&k_trial_l1), l1_bytes,
               l1_stat)) {
    QOZ_LAUNCH(k_trial_hi, dim3(ntrial, bg.nb), dim3(kHiThreads),
                       hi_bytes, s, bg, xs, wt, desc, hist, sse_part,
                       unpred_part);
    QOZ_LAUNCH(k_trial_l1, dim3(ntrial, bg.nb), dim3(kLdsThreads),
                       l1_bytes, s, bg, xs, wt, keep_wt ? 1u : 0u, desc,
                       hist, sse_part, unpred_part);
    return;
  }
  QOZ_LAUNCH(k_trial, dim3(ntrial, bg.nb), dim3(kTuneThreads), 0, s,
                     bg, xs, wt, desc, hist, sse_part, unpred_part);
}

}  // namespace qoz
