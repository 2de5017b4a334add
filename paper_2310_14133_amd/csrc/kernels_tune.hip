/*
 * Online tuner kernels (Sec. VI) for gfx950.
 *
 * Uniformly sampled blocks (Sec. VI-A) are gathered into a compact buffer,
 * (b+1)^d points each.  A trial runs the same predictor and quantizer as
 * the full compression on each block, treated as a field of its own whose
 * points on the 2^Lt grid are known exactly.
 *
 * One workgroup owns one (candidate, block) pair and walks the block's
 * sweeps in order with a workgroup barrier between sweeps; its working copy
 * of the block lives in global memory (L2-resident at the sampled sizes).
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
  for (uint32_t t = threadIdx.x; t < total; t += blockDim.x) {
    uint32_t a2 = t % m2, r = t / m2;
    uint32_t a1 = r % m1, a0 = r / m1;
    uint32_t idx = a0 * st * g.st[0] + a1 * st * g.st[1] + a2 * st;
    dst[idx] = src[idx];
  }
}

__global__ void k_gather_blocks(const float* __restrict__ x, Geo g,
                                BlockGeo bg, const uint32_t* origins,
                                float* __restrict__ xs) {
  const uint64_t total = (uint64_t)bg.nb * bg.size;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
       t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t blk = (uint32_t)(t / bg.size);
    uint32_t loc = (uint32_t)(t % bg.size);
    uint32_t i2 = loc % bg.g.n[2], r = loc / bg.g.n[2];
    uint32_t i1 = r % bg.g.n[1], i0 = r / bg.g.n[1];
    const uint32_t* o = origins + 3 * blk;
    uint32_t idx =
        (o[0] + i0) * g.st[0] + (o[1] + i1) * g.st[1] + (o[2] + i2);
    xs[t] = x[idx];
  }
}

void launch_gather_blocks(const float* x, const Geo& g, const BlockGeo& bg,
                          const uint32_t* origins_dev, float* xs,
                          hipStream_t s) {
  uint64_t total = (uint64_t)bg.nb * bg.size;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_gather_blocks, dim3((uint32_t)blocks), dim3(256), 0, s,
                     x, g, bg, origins_dev, xs);
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
    for (uint32_t t = threadIdx.x; t < count; t += blockDim.x) {
      uint32_t i2 = t % cnt[2], r = t / cnt[2];
      uint32_t i1 = r % cnt[1], i0 = r / cnt[1];
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

void launch_alg1_level(const BlockGeo& bg, uint32_t l, const float* xs,
                       const float* wc, float* wt, uint32_t ncand,
                       const TrialDesc* cand_desc, double* l1_part,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_alg1_level, dim3(ncand, bg.nb), dim3(kTuneThreads), 0,
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

/* commit the chosen candidate's working copy: wc = wt[pick] */
__global__ void k_commit_copy(const float* __restrict__ wt,
                              const uint32_t* __restrict__ pick, uint64_t n,
                              float* __restrict__ wc) {
  const float* src = wt + (uint64_t)(*pick) * n;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    wc[i] = src[i];
}

void launch_alg1_pick(const double* l1_part, uint32_t ncand, uint32_t nb,
                      double count, uint32_t* pick, const float* wt,
                      uint64_t bsz, float* wc, hipStream_t s) {
  hipLaunchKernelGGL(k_alg1_pick, dim3(1), dim3(kPickThreads), 0, s, l1_part,
                     ncand, nb, count, pick);
  uint64_t blocks = (bsz + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_commit_copy, dim3((uint32_t)blocks), dim3(256), 0, s,
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
      for (uint32_t t = threadIdx.x; t < count; t += blockDim.x) {
        uint32_t i2 = t % cnt[2], r = t / cnt[2];
        uint32_t i1 = r % cnt[1], i0 = r / cnt[1];
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
    sse_part[(uint64_t)tr * bg.nb + blk] = tot;
    unpred_part[(uint64_t)tr * bg.nb + blk] = u;
  }
}

void launch_trial(const BlockGeo& bg, const float* xs, float* wt,
                  uint32_t ntrial, const TrialDesc* desc, uint32_t* hist,
                  double* sse_part, uint32_t* unpred_part, hipStream_t s) {
  hipLaunchKernelGGL(k_trial, dim3(ntrial, bg.nb), dim3(kTuneThreads), 0, s,
                     bg, xs, wt, desc, hist, sse_part, unpred_part);
}

}  // namespace qoz
