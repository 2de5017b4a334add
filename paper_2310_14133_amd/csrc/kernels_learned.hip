/*
 * Learned tuner on gfx950: features of the sampled blocks and a small MLP
 * (32 -> 128 -> 128 -> 2 + 5 + 4) that predicts the choices of the online
 * tuner of Sec. VI (interpolation type, alpha and beta of Eq. 5).
 *
 * Features of one 33^3 block (b = 32 sampling of Sec. VI-A), e the bound:
 * for levels l = 1..5 (h = 2^(l-1)) and the linear / cubic stencils of
 * Sec. V-B applied to the original values along each dimension in turn,
 * log2(1 + mean|r| / e) and log2(1 + rms(r) / e) of the residuals r at the
 * points of the h-grid whose coordinate along that dimension is an odd
 * multiple of h (cubic only where p - 3h and p + 3h are inside the block,
 * else linear); the ten nearest-rank deciles of the squared forward-
 * difference gradient (dx*dx + dy*dy) + dz*dz over the 32^3 points with
 * every coordinate below 32, as log2(1 + sqrt(g2) / e); log2(1 + block
 * range / e) and log2(1 + range over all sampled blocks / e).  Residuals
 * and gradients are float32 in the order written; sums and logs are FP64.
 * Only the sampled blocks are read.
 *
 * Three workgroups of 1024 lanes per block, each with the block in LDS
 * (143.7 KB): level 1's residual sums; levels 2..5 and the value range;
 * the gradient deciles.  The residual sums are block reductions, and the
 * 32768 squared gradients stay in registers (32 per lane) while an exact
 * radix select
 * finds the ten deciles: four passes of 8 bits, each an LDS histogram per
 * distinct prefix still in play, a wave per decile scanning its histogram
 * to fix the next byte of its value and its rank below it.
 *
 * The network multiplies bfloat16 operands on the matrix cores
 * (v_mfma_f32_16x16x16_bf16, FP32 accumulate); biases, activations, the
 * softmax cross-entropy and Adam are FP32.  A workgroup of 4 waves takes 64
 * samples: all weights (bf16) and activations stay in LDS, and the
 * backward pass writes the workgroup's gradient to its own slot, summed in
 * slot order by the reduce kernel (deterministic).
 */
#include <hip/hip_runtime.h>

#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

/* ------------------------------------------------------------ features */
namespace {
constexpr uint32_t kFeatThreads = 1024;
constexpr uint32_t kB1 = 33;           /* block points per dimension */
constexpr uint32_t kPlane = kB1 * kB1; /* 1089 */
constexpr uint32_t kBlockPts = kB1 * kPlane;
constexpr uint32_t kNG = 32 * 32 * 32; /* gradient points */
constexpr uint32_t kGPer = kNG / kFeatThreads;
constexpr uint32_t kLoadBatch = 12;
constexpr uint32_t kLoadPer =
    (kBlockPts + kFeatThreads * kLoadBatch - 1) / (kFeatThreads * kLoadBatch) *
    kLoadBatch;
constexpr uint32_t kNone = 0xffffffffu;

template <int N>
__device__ void block_sum(double (&v)[N], double (*red)[kFeatThreads / 64]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = v[i];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) red[i][threadIdx.x >> 6] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = 0.0;
    for (uint32_t w = 0; w < kFeatThreads / 64; ++w) t += red[i][w];
    v[i] = t;
  }
  __syncthreads();
}
}  // namespace

/* feat[b][0..30] of block b (blockIdx.y picks the part); aux[b] = (min,
 * max, non-finite flag) for the pooling kernel, which fills feat[b][31] */
__device__ __forceinline__ void block_features_body(
    const float* __restrict__ x, const Geo& g,
    const uint32_t* __restrict__ origins, double e, float* __restrict__ feat,
    float* __restrict__ aux, uint32_t bx, uint32_t part_y) {
  extern __shared__ float blk[];
  __shared__ double red[4][kFeatThreads / 64];
  __shared__ float mred[3][kFeatThreads / 64];
  __shared__ double stat[20];
  __shared__ uint32_t rhist[10][256];
  __shared__ uint32_t rpre[10], rrank[10], dpre[10], dmap[10], ndist;
  const uint32_t tid = threadIdx.x, part = part_y;
  const uint32_t* o = origins + 3 * bx;
  const uint64_t base = (uint64_t)o[0] * g.st[0] + (uint64_t)o[1] * g.st[1] +
                        (uint64_t)o[2] * g.st[2];
  /* the block, 12 loads in flight per lane */
  for (uint32_t u0 = 0; u0 < kLoadPer; u0 += kLoadBatch) {
    float v[kLoadBatch];
#pragma unroll
    for (uint32_t u = 0; u < kLoadBatch; ++u) {
      const uint32_t t = tid + (u0 + u) * kFeatThreads;
      if (t < kBlockPts) {
        const uint32_t i = t / kPlane, r = t - i * kPlane, j = r / kB1,
                       k = r - j * kB1;
        v[u] = x[base + (uint64_t)i * g.st[0] + (uint64_t)j * g.st[1] + k];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kLoadBatch; ++u) {
      const uint32_t t = tid + (u0 + u) * kFeatThreads;
      if (t < kBlockPts) blk[t] = v[u];
    }
  }
  __syncthreads();
  /* block range and finiteness */
  if (part == 1) {
    float lo = blk[tid], hi = blk[tid];
    uint32_t bad = 0;
    for (uint32_t t = tid; t < kBlockPts; t += kFeatThreads) {
      const float v = blk[t];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
      bad |= (__float_as_uint(v) & 0x7f800000u) == 0x7f800000u;
    }
    for (int s = 32; s > 0; s >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, s, 64));
      hi = fmaxf(hi, __shfl_xor(hi, s, 64));
      bad |= __shfl_xor(bad, s, 64);
    }
    if ((tid & 63) == 0) {
      mred[0][tid >> 6] = lo;
      mred[1][tid >> 6] = hi;
      mred[2][tid >> 6] = bad ? 1.0f : 0.0f;
    }
  }
  /* level-wise residual sums: lin |r|, lin r^2, cubic |r|, cubic r^2 */
#pragma unroll
  for (uint32_t l = 1; l <= 5; ++l) {
    if (part == 2 || (part == 0) != (l == 1)) continue;
    const uint32_t h = 1u << (l - 1), m = 32 / h + 1, nodd = 16 / h;
    const uint32_t per_dim = nodd * m * m;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t t = tid; t < 3 * per_dim; t += kFeatThreads) {
      const uint32_t k = t / per_dim, q = t - k * per_dim;
      const uint32_t u = q / (m * m), vw = q - u * (m * m);
      const uint32_t v = vw / m, w = vw - v * m;
      const uint32_t ck = (2 * u + 1) * h; /* odd multiple along k */
      /* strides of k and of the two other dimensions, in order */
      const uint32_t s0 = k == 0 ? kPlane : (k == 1 ? kB1 : 1u);
      const uint32_t s1 = k == 0 ? kB1 : kPlane;
      const uint32_t s2 = k == 2 ? kB1 : 1u;
      const uint32_t p = ck * s0 + v * h * s1 + w * h * s2;
      const uint32_t sk = s0 * h;
      const float b = blk[p - sk], cc = blk[p + sk], xv = blk[p];
      const float lin = (b + cc) * 0.5f;
      float cub = lin;
      if (ck >= 3 * h && ck + 3 * h <= 32) {
        const float a = blk[p - 3 * sk], d = blk[p + 3 * sk];
        cub = ((b + cc) * 9.0f - (a + d)) * 0.0625f;
      }
      const double rl = (double)(xv - lin), rc = (double)(xv - cub);
      acc[0] += fabs(rl);
      acc[1] += rl * rl;
      acc[2] += fabs(rc);
      acc[3] += rc * rc;
    }
    block_sum<4>(acc, red);
    if (tid == 0) {
      const double n = 3.0 * per_dim;
      stat[4 * (l - 1) + 0] = log2(1.0 + (acc[0] / n) / e);
      stat[4 * (l - 1) + 1] = log2(1.0 + sqrt(acc[1] / n) / e);
      stat[4 * (l - 1) + 2] = log2(1.0 + (acc[2] / n) / e);
      stat[4 * (l - 1) + 3] = log2(1.0 + sqrt(acc[3] / n) / e);
    }
  }
  if (part != 2) {
    __syncthreads(); /* stat[] and mred[] complete */
    if (tid < 31 &&
        (part == 0 ? tid < 4 : (tid >= 4 && tid < 20) || tid == 30)) {
      double f;
      if (tid < 20) {
        f = stat[tid];
      } else {
        float l2 = mred[0][0], h2 = mred[1][0], b2 = mred[2][0];
        for (uint32_t w = 1; w < kFeatThreads / 64; ++w) {
          l2 = fminf(l2, mred[0][w]);
          h2 = fmaxf(h2, mred[1][w]);
          b2 = fmaxf(b2, mred[2][w]);
        }
        f = log2(1.0 + ((double)h2 - (double)l2) / e);
        aux[3 * (uint64_t)bx + 0] = l2;
        aux[3 * (uint64_t)bx + 1] = h2;
        aux[3 * (uint64_t)bx + 2] = b2;
      }
      feat[32 * (uint64_t)bx + tid] = (float)f;
    }
    return;
  }
  /* squared gradients, kept in registers */
  uint32_t g2[kGPer];
#pragma unroll
  for (uint32_t s = 0; s < kGPer; ++s) {
    const uint32_t t = tid + s * kFeatThreads;
    const uint32_t i = t >> 10, j = (t >> 5) & 31, k = t & 31;
    const uint32_t p = i * kPlane + j * kB1 + k;
    const float v = blk[p];
    const float dx = blk[p + kPlane] - v, dy = blk[p + kB1] - v,
                dz = blk[p + 1] - v;
    g2[s] = __float_as_uint((dx * dx + dy * dy) + dz * dz);
  }
  /* exact radix select of the deciles (non-negative floats order as their
   * bits): rank of decile q is ceil(q n / 10) - 1 */
  if (tid < 10) {
    rrank[tid] = ((tid + 1) * kNG + 9) / 10 - 1;
    rpre[tid] = 0;
    dmap[tid] = 0;
  }
  if (tid == 0) {
    dpre[0] = 0;
    ndist = 1;
  }
  __syncthreads();
  const uint32_t lane = tid & 63, wv = tid >> 6;
  uint32_t* flat = &rhist[0][0];
  for (uint32_t pass = 0; pass < 4; ++pass) {
    const uint32_t shift = 24 - 8 * pass;
    const uint32_t nd = ndist;
    for (uint32_t i = tid; i < nd * 256; i += kFeatThreads) flat[i] = 0;
    __syncthreads();
#pragma unroll 4
    for (uint32_t s = 0; s < kGPer; ++s) {
      const uint32_t key = g2[s];
      uint32_t d = pass == 0 ? 0u : kNone;
      if (pass != 0) {
        const uint32_t hi = key >> (shift + 8);
        for (uint32_t dd = 0; dd < nd; ++dd)
          if (dpre[dd] == hi) d = dd;
      }
      const uint32_t addr = d == kNone ? kNone : d * 256 + ((key >> shift) & 255);
      /* a wave whose lanes all hit one bin adds once */
      const uint32_t first = __builtin_amdgcn_readfirstlane(addr);
      if (__all(addr == first)) {
        if (lane == 0 && first != kNone) atomicAdd(&flat[first], 64u);
      } else if (addr != kNone) {
        atomicAdd(&flat[addr], 1u);
      }
    }
    __syncthreads();
    if (wv < 10) {
      const uint32_t* hq = rhist[dmap[wv]];
      const uint32_t c0 = hq[4 * lane], c1 = hq[4 * lane + 1],
                     c2 = hq[4 * lane + 2], c3 = hq[4 * lane + 3];
      const uint32_t sum = c0 + c1 + c2 + c3;
      uint32_t incl = sum;
      for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      const uint32_t excl = incl - sum, r = rrank[wv];
      if (r >= excl && r < incl) {
        uint32_t b = 4 * lane, before = excl;
        if (r >= before + c0) {
          before += c0;
          ++b;
          if (r >= before + c1) {
            before += c1;
            ++b;
            if (r >= before + c2) {
              before += c2;
              ++b;
            }
          }
        }
        rpre[wv] |= b << shift;
        rrank[wv] = r - before;
      }
    }
    __syncthreads();
    if (tid == 0) { /* distinct known prefixes for the next pass */
      uint32_t n = 0;
      for (uint32_t q = 0; q < 10; ++q) {
        const uint32_t hi = rpre[q] >> shift;
        uint32_t f = n;
        for (uint32_t dd = 0; dd < n; ++dd)
          if (dpre[dd] == hi) f = dd;
        if (f == n) dpre[n++] = hi;
        dmap[q] = f;
      }
      ndist = n;
    }
    __syncthreads();
  }
  if (tid >= 20 && tid < 30)
    feat[32 * (uint64_t)bx + tid] = (float)log2(
        1.0 + sqrt((double)__uint_as_float(rpre[tid - 20])) / e);
}

__global__ __launch_bounds__(kFeatThreads) void k_block_features(
    const float* __restrict__ x, Geo g, const uint32_t* __restrict__ origins,
    double e, float* __restrict__ feat, float* __restrict__ aux) {
  block_features_body(x, g, origins, e, feat, aux, blockIdx.x, blockIdx.y);
}

/* The same features of one 33 x 33 block of a 2D field (row stride
 * g.st[1]; origins hold (0, row, column) per block): residuals along the two
 * dimensions, g2 = dx*dx + dy*dy over the 32 x 32 points with both
 * coordinates below 32, whose deciles come from a bitonic sort of the 1024
 * values in LDS.  One 256-lane workgroup per block. */
namespace {
constexpr uint32_t kF2Threads = 256;
constexpr uint32_t kB2Pts = kB1 * kB1; /* 1089 */
constexpr uint32_t kNG2 = 32 * 32;     /* gradient points */
}  // namespace

__device__ __forceinline__ void block_features_2d_body(
    const float* __restrict__ x, const Geo& g,
    const uint32_t* __restrict__ origins, double e, float* __restrict__ feat,
    float* __restrict__ aux, uint32_t bx) {
  __shared__ float blk[kB2Pts];
  __shared__ uint32_t keys[kNG2];
  __shared__ double red[4][kF2Threads / 64];
  __shared__ float mred[3][kF2Threads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t* o = origins + 3 * bx;
  const uint64_t base = (uint64_t)o[1] * g.st[1] + o[2];
  float* out = feat + 32 * (uint64_t)bx;
  for (uint32_t t = tid; t < kB2Pts; t += kF2Threads) {
    const uint32_t i = t / kB1, j = t - i * kB1;
    blk[t] = x[base + (uint64_t)i * g.st[1] + j];
  }
  __syncthreads();
  /* block range and finiteness */
  {
    float lo = blk[tid], hi = blk[tid];
    uint32_t bad = 0;
    for (uint32_t t = tid; t < kB2Pts; t += kF2Threads) {
      const float v = blk[t];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
      bad |= (__float_as_uint(v) & 0x7f800000u) == 0x7f800000u;
    }
    for (int sh = 32; sh > 0; sh >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, sh, 64));
      hi = fmaxf(hi, __shfl_xor(hi, sh, 64));
      bad |= __shfl_xor(bad, sh, 64);
    }
    if (lane == 0) {
      mred[0][wv] = lo;
      mred[1][wv] = hi;
      mred[2][wv] = bad ? 1.0f : 0.0f;
    }
  }
  /* level-wise residual sums: lin |r|, lin r^2, cubic |r|, cubic r^2 */
  for (uint32_t l = 1; l <= 5; ++l) {
    const uint32_t h = 1u << (l - 1), m = 32 / h + 1, nodd = 16 / h;
    const uint32_t per_dim = nodd * m;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t t = tid; t < 2 * per_dim; t += kF2Threads) {
      const uint32_t k = t / per_dim, q = t - k * per_dim;
      const uint32_t u = q / m, v = q - u * m;
      const uint32_t ck = (2 * u + 1) * h; /* odd multiple along k */
      const uint32_t sk = (k == 0 ? kB1 : 1u) * h;
      const uint32_t p = k == 0 ? ck * kB1 + v * h : v * h * kB1 + ck;
      const float b = blk[p - sk], cc = blk[p + sk], xv = blk[p];
      const float lin = (b + cc) * 0.5f;
      float cub = lin;
      if (ck >= 3 * h && ck + 3 * h <= 32) {
        const float a = blk[p - 3 * sk], d = blk[p + 3 * sk];
        cub = ((b + cc) * 9.0f - (a + d)) * 0.0625f;
      }
      const double rl = (double)(xv - lin), rc = (double)(xv - cub);
      acc[0] += fabs(rl);
      acc[1] += rl * rl;
      acc[2] += fabs(rc);
      acc[3] += rc * rc;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double t = acc[i];
      for (int sh = 32; sh > 0; sh >>= 1) t += __shfl_xor(t, sh, 64);
      if (lane == 0) red[i][wv] = t;
    }
    __syncthreads();
    if (tid < 4) {
      double t = 0.0;
      for (uint32_t w = 0; w < kF2Threads / 64; ++w) t += red[tid][w];
      const double n = 2.0 * per_dim;
      out[4 * (l - 1) + tid] =
          (float)log2(1.0 + ((tid & 1) ? sqrt(t / n) : t / n) / e);
    }
    __syncthreads();
  }
  /* squared gradients (non-negative floats order as their bits) */
  for (uint32_t t = tid; t < kNG2; t += kF2Threads) {
    const uint32_t p = (t >> 5) * kB1 + (t & 31);
    const float v = blk[p];
    const float dx = blk[p + kB1] - v, dy = blk[p + 1] - v;
    keys[t] = __float_as_uint(dx * dx + dy * dy);
  }
  __syncthreads();
  for (uint32_t k = 2; k <= kNG2; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < kNG2; i += kF2Threads) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint32_t a = keys[i], b = keys[ixj];
          if ((a > b) == ((i & k) == 0)) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  if (tid < 10) {
    const uint32_t r = ((tid + 1) * kNG2 + 9) / 10 - 1;
    out[20 + tid] =
        (float)log2(1.0 + sqrt((double)__uint_as_float(keys[r])) / e);
  }
  if (tid == 0) {
    float l2 = mred[0][0], h2 = mred[1][0], b2 = mred[2][0];
    for (uint32_t w = 1; w < kF2Threads / 64; ++w) {
      l2 = fminf(l2, mred[0][w]);
      h2 = fmaxf(h2, mred[1][w]);
      b2 = fmaxf(b2, mred[2][w]);
    }
    out[30] = (float)log2(1.0 + ((double)h2 - (double)l2) / e);
    aux[3 * (uint64_t)bx + 0] = l2;
    aux[3 * (uint64_t)bx + 1] = h2;
    aux[3 * (uint64_t)bx + 2] = b2;
  }
}

__global__ __launch_bounds__(kF2Threads) void k_block_features_2d(
    const float* __restrict__ x, Geo g, const uint32_t* __restrict__ origins,
    double e, float* __restrict__ feat, float* __restrict__ aux) {
  block_features_2d_body(x, g, origins, e, feat, aux, blockIdx.x);
}

/* Range over all blocks into every row's feature 31, the mean of each
 * feature over the blocks into out[32], and the non-finite flag into
 * status[0]. */
__device__ __forceinline__ void feat_pool_body(float* __restrict__ feat,
                                               const float* __restrict__ aux,
                                               uint32_t nb, double e,
                                               float* __restrict__ out,
                                               uint32_t* __restrict__ status) {
  const uint32_t i = threadIdx.x;
  float lo = aux[0], hi = aux[1], bad = aux[2];
#pragma unroll 8
  for (uint32_t b = 1; b < nb; ++b) {
    lo = fminf(lo, aux[3 * (uint64_t)b]);
    hi = fmaxf(hi, aux[3 * (uint64_t)b + 1]);
    bad = fmaxf(bad, aux[3 * (uint64_t)b + 2]);
  }
  const float f31 = (float)log2(1.0 + ((double)hi - (double)lo) / e);
  if (i == 0) status[0] = bad != 0.0f ? kStNonFinite : 0u;
  if (i < 31) {
    double s = 0.0;
#pragma unroll 8
    for (uint32_t b = 0; b < nb; ++b) s += (double)feat[32 * (uint64_t)b + i];
    out[i] = (float)(s / (double)nb);
  } else if (i == 31) {
    out[31] = f31;
  }
  for (uint32_t b = i; b < nb; b += blockDim.x) feat[32 * (uint64_t)b + 31] = f31;
}

__global__ void k_feat_pool(float* __restrict__ feat,
                            const float* __restrict__ aux, uint32_t nb,
                            double e, float* __restrict__ out,
                            uint32_t* __restrict__ status) {
  feat_pool_body(feat, aux, nb, e, out, status);
}

size_t block_features_lds() { return 4 * (size_t)kBlockPts; }

/* The features of many fields in three launches: the 3D fields' blocks
 * (job j owns workgroups [wg0[j], wg0[j+1]) of x, three parts each in y),
 * the 2D fields' blocks, then one pooling workgroup per field.  Pointers
 * read from a record are made global (not flat). */
__global__ __launch_bounds__(kFeatThreads) void k_block_features_q(
    const FeatJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  const uint32_t j = find_job(wg0, n_jobs, blockIdx.x);
  const FeatJob& a = jobs[j];
  block_features_body((const float*)gptr(a.x), a.g,
                      (const uint32_t*)gptr(a.origins), a.e,
                      (float*)gptr(a.feat), (float*)gptr(a.aux),
                      blockIdx.x - wg0[j], blockIdx.y);
}

__global__ __launch_bounds__(kF2Threads) void k_block_features_2d_q(
    const FeatJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  const uint32_t j = find_job(wg0, n_jobs, blockIdx.x);
  const FeatJob& a = jobs[j];
  block_features_2d_body((const float*)gptr(a.x), a.g,
                         (const uint32_t*)gptr(a.origins), a.e,
                         (float*)gptr(a.feat), (float*)gptr(a.aux),
                         blockIdx.x - wg0[j]);
}

__global__ void k_feat_pool_q(const FeatJob* __restrict__ jobs) {
  const FeatJob& a = jobs[blockIdx.x];
  feat_pool_body((float*)gptr(a.feat), (const float*)gptr(a.aux), a.nb, a.e,
                 (float*)gptr(a.mean), (uint32_t*)gptr(a.status));
}

void launch_block_features_q(const FeatJob* jobs3, const uint32_t* wg3,
                             uint32_t n3, uint32_t total3,
                             const FeatJob* jobs2, const uint32_t* wg2,
                             uint32_t n2, uint32_t total2,
                             const FeatJob* all, uint32_t n, hipStream_t s) {
  if (n3 && total3)
    QOZ_LAUNCH(k_block_features_q, dim3(total3, 3), dim3(kFeatThreads),
               block_features_lds(), s, jobs3, wg3, n3);
  if (n2 && total2)
    QOZ_LAUNCH(k_block_features_2d_q, dim3(total2), dim3(kF2Threads), 0, s,
               jobs2, wg2, n2);
  if (n) QOZ_LAUNCH(k_feat_pool_q, dim3(n), dim3(64), 0, s, all);
}


bool block_features_fit() {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            dev) != hipSuccess)
    return false;
  const size_t stat_bytes = 8 * 4 * 16 + 4 * 3 * 16 + 8 * 20 + 4 * 10 * 256 +
                            4 * 41;
  if (block_features_lds() + stat_bytes > (size_t)max_lds) return false;
  return hipFuncSetAttribute(
             reinterpret_cast<const void*>(&k_block_features),
             hipFuncAttributeMaxDynamicSharedMemorySize,
             (int)block_features_lds()) == hipSuccess &&
         hipFuncSetAttribute(
             reinterpret_cast<const void*>(&k_block_features_q),
             hipFuncAttributeMaxDynamicSharedMemorySize,
             (int)block_features_lds()) == hipSuccess;
}

void launch_block_features(const float* x, const Geo& g,
                           const uint32_t* origins, uint32_t nb, double e,
                           float* feat, float* aux, float* mean,
                           uint32_t* status, hipStream_t s) {
  if (g.n[0] == 1) /* a 2D field: its geometry has a single plane */
    QOZ_LAUNCH(k_block_features_2d, dim3(nb), dim3(kF2Threads), 0, s,
                       x, g, origins, e, feat, aux);
  else
    QOZ_LAUNCH(k_block_features, dim3(nb, 3), dim3(kFeatThreads),
                       block_features_lds(), s, x, g, origins, e, feat, aux);
  QOZ_LAUNCH(k_feat_pool, dim3(1), dim3(64), 0, s, feat,
                     (const float*)aux, nb, e, mean, status);
}

/* ----------------------------------------------------------------- MLP */
namespace {
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kMlpThreads = 256;
constexpr uint32_t kTile = 64; /* samples per workgroup */
constexpr uint32_t NF = kMlpFeat, NH = kMlpHidden, NO = kMlpOut;
constexpr uint32_t NOP = 16; /* outputs padded to one MFMA tile */

/* LDS layout (bytes) */
constexpr uint32_t L_W1 = 0;
constexpr uint32_t L_W2 = L_W1 + 2 * NH * NF;
constexpr uint32_t L_W3 = L_W2 + 2 * NH * NH;
constexpr uint32_t L_BIAS = L_W3 + 2 * NOP * NH;
constexpr uint32_t L_X = L_BIAS + 4 * (2 * NH + NOP);
constexpr uint32_t L_H1 = L_X + 2 * kTile * NF;
constexpr uint32_t L_H2 = L_H1 + 2 * kTile * NH;
constexpr uint32_t L_Z = L_H2 + 2 * kTile * NH;
constexpr uint32_t L_FWD_END = L_Z + 4 * kTile * NOP;
constexpr uint32_t L_DZF = L_FWD_END;
constexpr uint32_t L_DZB = L_DZF + 4 * kTile * NOP;
constexpr uint32_t L_DHF = L_DZB + 2 * kTile * NOP;
constexpr uint32_t L_DH2 = L_DHF + 4 * kTile * NH;
constexpr uint32_t L_DH1 = L_DH2 + 2 * kTile * NH;
constexpr uint32_t L_END = L_DH1 + 2 * kTile * NH;

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

/* n4 float4 of a 16-byte aligned src to bf16 in dst, lane-strided, PER
 * per lane (PER * kMlpThreads >= n4) */
template <uint32_t PER>
__device__ __forceinline__ void stage_bf16(const float* __restrict__ src,
                                           uint32_t n4, uint16_t* dst) {
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4 v[PER];
#pragma unroll
  for (uint32_t u = 0; u < PER; ++u) {
    const uint32_t i = threadIdx.x + u * kMlpThreads;
    if (i < n4) v[u] = s4[i];
  }
#pragma unroll
  for (uint32_t u = 0; u < PER; ++u) {
    const uint32_t i = threadIdx.x + u * kMlpThreads;
    if (i < n4) {
      uint2 w;
      w.x = (uint32_t)to_bf16(v[u].x) | ((uint32_t)to_bf16(v[u].y) << 16);
      w.y = (uint32_t)to_bf16(v[u].z) | ((uint32_t)to_bf16(v[u].w) << 16);
      reinterpret_cast<uint2*>(dst)[i] = w;
    }
  }
}

/* Operand fragments of four consecutive k: from a matrix whose k runs
 * along a row (one 8-byte LDS read) or down a column (four reads). */
__device__ __forceinline__ bf16x4 frag_row(const uint16_t* base,
                                           uint32_t stride, uint32_t r,
                                           uint32_t k0) {
  return *reinterpret_cast<const bf16x4*>(base + r * stride + k0);
}
__device__ __forceinline__ bf16x4 frag_col(const uint16_t* base,
                                           uint32_t stride, uint32_t k0,
                                           uint32_t c) {
  bf16x4 v;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) v[j] = (short)base[(k0 + j) * stride + c];
  return v;
}

/* C[M x N] = sum_k A(m, k) B(k, n) on 16x16x16 bf16 MFMA tiles, tiles
 * spread over the workgroup's waves.  fa(m, k0) gives A(m, k0..k0+3),
 * fb(k0, n) gives B(k0..k0+3, n).  Lane layout: A row = lane % 16 and
 * k0 = 4 (lane / 16); B column = lane % 16, same k0; result row =
 * 4 (lane / 16) + j, column = lane % 16. */
template <class FA, class FB, class FC>
__device__ __forceinline__ void wave_mm(uint32_t M, uint32_t N, uint32_t K,
                                        FA fa, FB fb, FC c) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t r = lane & 15, q = lane >> 4;
  const uint32_t tn = N >> 4, tiles = (M >> 4) * tn;
  for (uint32_t t = wv; t < tiles; t += nw) {
    const uint32_t m0 = (t / tn) << 4, n0 = (t % tn) << 4;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t k0 = 0; k0 < K; k0 += 16) {
      const bf16x4 av = fa(m0 + r, k0 + 4 * q);
      const bf16x4 bv = fb(k0 + 4 * q, n0 + r);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) c(m0 + 4 * q + j, n0 + r, acc[j]);
  }
}
}  // namespace

/* TRAIN = false: logits of samples [64 blockIdx.x, +64) into `logits`.
 * TRAIN = true: the workgroup's summed loss into loss_part[blockIdx.x] and
 * its gradient of the mean loss into part[blockIdx.x][...]. */
template <bool TRAIN>
__global__ __launch_bounds__(kMlpThreads) void k_mlp(
    const float* __restrict__ P, const float* __restrict__ X,
    const int32_t* __restrict__ labels, const uint32_t* __restrict__ index,
    uint32_t n_rows, uint32_t B, float* __restrict__ logits,
    float* __restrict__ part, double* __restrict__ loss_part) {
  extern __shared__ uint8_t lds[];
  __shared__ double sloss[kTile];
  __shared__ int32_t rows[kTile];
  uint16_t* W1b = (uint16_t*)(lds + L_W1);
  uint16_t* W2b = (uint16_t*)(lds + L_W2);
  uint16_t* W3b = (uint16_t*)(lds + L_W3);
  float* b1 = (float*)(lds + L_BIAS);
  float* b2 = b1 + NH;
  float* b3 = b2 + NH;
  uint16_t* Xb = (uint16_t*)(lds + L_X);
  uint16_t* H1b = (uint16_t*)(lds + L_H1);
  uint16_t* H2b = (uint16_t*)(lds + L_H2);
  float* Zs = (float*)(lds + L_Z);
  const uint32_t tid = threadIdx.x;
  const uint32_t s0 = blockIdx.x * kTile;

  /* weights to bf16 in LDS: float4 loads, all of a matrix in flight */
  stage_bf16<NH * NF / 4 / kMlpThreads>(P + kOffW1, NH * NF / 4, W1b);
  stage_bf16<NH * NH / 4 / kMlpThreads>(P + kOffW2, NH * NH / 4, W2b);
  stage_bf16<(NOP * NH / 4 + kMlpThreads - 1) / kMlpThreads>(
      P + kOffW3, NO * NH / 4, W3b);
  for (uint32_t i = NO * NH + tid; i < NOP * NH; i += kMlpThreads) W3b[i] = 0;
  for (uint32_t i = tid; i < NH; i += kMlpThreads) {
    b1[i] = P[kOffB1 + i];
    b2[i] = P[kOffB2 + i];
  }
  if (tid < NOP) b3[tid] = tid < NO ? P[kOffB3 + tid] : 0.0f;
  if (tid < kTile) {
    const uint32_t s = s0 + tid;
    int32_t row = -1;
    if (s < B) {
      const uint32_t r = index ? index[s] : s;
      if (r < n_rows) row = (int32_t)r;
    }
    rows[tid] = row;
  }
  __syncthreads();
  for (uint32_t i = tid; i < kTile * NF; i += kMlpThreads) {
    const uint32_t s = i / NF, f = i - s * NF;
    const int32_t row = rows[s];
    float v = 0.0f;
    if (row >= 0)
      v = (X[(uint64_t)row * NF + f] - P[kOffMu + f]) / P[kOffSg + f];
    Xb[i] = to_bf16(v);
  }
  __syncthreads();

  /* forward rows: the whole tile when training, else the valid rows */
  const uint32_t live = B - s0 < kTile ? B - s0 : kTile;
  const uint32_t MF = TRAIN ? kTile : (live + 15) / 16 * 16;
  wave_mm(MF, NH, NF, [&](uint32_t m, uint32_t k) { return frag_row(Xb, NF, m, k); },
          [&](uint32_t k, uint32_t n) { return frag_row(W1b, NF, n, k); },
          [&](uint32_t m, uint32_t n, float v) {
            H1b[m * NH + n] = to_bf16(fmaxf(v + b1[n], 0.0f));
          });
  __syncthreads();
  wave_mm(MF, NH, NH, [&](uint32_t m, uint32_t k) { return frag_row(H1b, NH, m, k); },
          [&](uint32_t k, uint32_t n) { return frag_row(W2b, NH, n, k); },
          [&](uint32_t m, uint32_t n, float v) {
            H2b[m * NH + n] = to_bf16(fmaxf(v + b2[n], 0.0f));
          });
  __syncthreads();
  wave_mm(MF, NOP, NH,
          [&](uint32_t m, uint32_t k) { return frag_row(H2b, NH, m, k); },
          [&](uint32_t k, uint32_t n) { return frag_row(W3b, NH, n, k); },
          [&](uint32_t m, uint32_t n, float v) { Zs[m * NOP + n] = v + b3[n]; });
  __syncthreads();

  if (!TRAIN) {
    for (uint32_t i = tid; i < kTile * NO; i += kMlpThreads) {
      const uint32_t s = i / NO, o = i - s * NO;
      if (s0 + s < B) logits[(uint64_t)(s0 + s) * NO + o] = Zs[s * NOP + o];
    }
    return;
  }

  float* dZf = (float*)(lds + L_DZF);
  uint16_t* dZb = (uint16_t*)(lds + L_DZB);
  float* dHf = (float*)(lds + L_DHF);
  uint16_t* dH2b = (uint16_t*)(lds + L_DH2);
  uint16_t* dH1b = (uint16_t*)(lds + L_DH1);
  float* gp = part + (uint64_t)blockIdx.x * kMlpParams;

  /* softmax cross-entropy of the three heads, one lane per sample */
  if (tid < kTile) {
    const int32_t row = rows[tid];
    const float* z = Zs + tid * NOP;
    const float invB = 1.0f / (float)B;
    double ls = 0.0;
    uint32_t o = 0;
    const uint32_t heads[3] = {kHeadInterp, kHeadAlpha, kHeadBeta};
    for (uint32_t hd = 0; hd < 3; ++hd) {
      const uint32_t k = heads[hd];
      int32_t y = row >= 0 ? labels[(uint64_t)row * 3 + hd] : 0;
      y = y < 0 ? 0 : (y >= (int32_t)k ? (int32_t)k - 1 : y);
      float mx = z[o];
      for (uint32_t c = 1; c < k; ++c) mx = fmaxf(mx, z[o + c]);
      float sum = 0.0f;
      for (uint32_t c = 0; c < k; ++c) sum += expf(z[o + c] - mx);
      if (row >= 0) ls += (double)(mx + logf(sum)) - (double)z[o + y];
      for (uint32_t c = 0; c < k; ++c) {
        float d = expf(z[o + c] - mx) / sum - (c == (uint32_t)y ? 1.0f : 0.0f);
        d = row >= 0 ? d * invB : 0.0f;
        dZf[tid * NOP + o + c] = d;
        dZb[tid * NOP + o + c] = to_bf16(d);
      }
      o += k;
    }
    for (uint32_t c = NO; c < NOP; ++c) {
      dZf[tid * NOP + c] = 0.0f;
      dZb[tid * NOP + c] = 0;
    }
    sloss[tid] = ls;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (uint32_t s = 0; s < kTile; ++s) t += sloss[s];
    loss_part[blockIdx.x] = t;
  }
  if (tid < 2 * NF) gp[tid] = 0.0f; /* input shift and scale: not trained */
  /* output layer */
  wave_mm(NOP, NH, kTile,
          [&](uint32_t m, uint32_t k) { return frag_col(dZb, NOP, k, m); },
          [&](uint32_t k, uint32_t n) { return frag_col(H2b, NH, k, n); },
          [&](uint32_t m, uint32_t n, float v) {
            if (m < NO) gp[kOffW3 + m * NH + n] = v;
          });
  if (tid < NO) {
    float t = 0.0f;
    for (uint32_t s = 0; s < kTile; ++s) t += dZf[s * NOP + tid];
    gp[kOffB3 + tid] = t;
  }
  wave_mm(kTile, NH, NOP,
          [&](uint32_t m, uint32_t k) { return frag_row(dZb, NOP, m, k); },
          [&](uint32_t k, uint32_t n) { return frag_col(W3b, NH, k, n); },
          [&](uint32_t m, uint32_t n, float v) {
            const float d = from_bf16(H2b[m * NH + n]) > 0.0f ? v : 0.0f;
            dHf[m * NH + n] = d;
            dH2b[m * NH + n] = to_bf16(d);
          });
  __syncthreads();
  /* second layer */
  wave_mm(NH, NH, kTile,
          [&](uint32_t m, uint32_t k) { return frag_col(dH2b, NH, k, m); },
          [&](uint32_t k, uint32_t n) { return frag_col(H1b, NH, k, n); },
          [&](uint32_t m, uint32_t n, float v) { gp[kOffW2 + m * NH + n] = v; });
  if (tid < NH) {
    float t = 0.0f;
    for (uint32_t s = 0; s < kTile; ++s) t += dHf[s * NH + tid];
    gp[kOffB2 + tid] = t;
  }
  __syncthreads();
  wave_mm(kTile, NH, NH,
          [&](uint32_t m, uint32_t k) { return frag_row(dH2b, NH, m, k); },
          [&](uint32_t k, uint32_t n) { return frag_col(W2b, NH, k, n); },
          [&](uint32_t m, uint32_t n, float v) {
            const float d = from_bf16(H1b[m * NH + n]) > 0.0f ? v : 0.0f;
            dHf[m * NH + n] = d;
            dH1b[m * NH + n] = to_bf16(d);
          });
  __syncthreads();
  /* first layer */
  wave_mm(NH, NF, kTile,
          [&](uint32_t m, uint32_t k) { return frag_col(dH1b, NH, k, m); },
          [&](uint32_t k, uint32_t n) { return frag_col(Xb, NF, k, n); },
          [&](uint32_t m, uint32_t n, float v) { gp[kOffW1 + m * NF + n] = v; });
  if (tid < NH) {
    float t = 0.0f;
    for (uint32_t s = 0; s < kTile; ++s) t += dHf[s * NH + tid];
    gp[kOffB1 + tid] = t;
  }
}

/* Gradient = sum of the workgroups' slots in slot order; optionally one
 * Adam step (bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t) on
 * every trained entry; the mean loss into *loss. */
__global__ void k_mlp_reduce(const float* __restrict__ part, uint32_t nw,
                             float* __restrict__ grad, float* __restrict__ P,
                             float* __restrict__ m, float* __restrict__ v,
                             float lr, float bc1, float bc2, int adam,
                             const double* __restrict__ loss_part, uint32_t B,
                             double* __restrict__ loss) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && loss) {
    double t = 0.0;
    for (uint32_t w = 0; w < nw; ++w) t += loss_part[w];
    *loss = t / (double)B;
  }
  if (i >= kMlpParams) return;
  float g = 0.0f;
  for (uint32_t w = 0; w < nw; ++w) g += part[(uint64_t)w * kMlpParams + i];
  if (grad) grad[i] = g;
  if (adam && i >= kOffW1) {
    const float mi = kAdamB1 * m[i] + (1.0f - kAdamB1) * g;
    const float vi = kAdamB2 * v[i] + (1.0f - kAdamB2) * (g * g);
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    P[i] = P[i] - lr * (mh / (sqrtf(vh) + kAdamEps));
  }
}

uint32_t mlp_tiles(uint32_t B) { return (B + kTile - 1) / kTile; }

bool mlp_fit() {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            dev) != hipSuccess)
    return false;
  if (L_END + 8 * kTile + 4 * kTile > (uint32_t)max_lds) return false;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp<true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)L_END) == hipSuccess &&
         hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp<false>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)L_FWD_END) == hipSuccess;
}

void launch_mlp_forward(const float* P, const float* X, uint32_t B,
                        float* logits, hipStream_t s) {
  QOZ_LAUNCH(k_mlp<false>, dim3(mlp_tiles(B)), dim3(kMlpThreads),
                     L_FWD_END, s, P, X, (const int32_t*)nullptr,
                     (const uint32_t*)nullptr, B, B, logits, (float*)nullptr,
                     (double*)nullptr);
}

void launch_mlp_grad(const float* P, const float* X, const int32_t* labels,
                     const uint32_t* index, uint32_t n_rows, uint32_t B,
                     float* part, double* loss_part, hipStream_t s) {
  QOZ_LAUNCH(k_mlp<true>, dim3(mlp_tiles(B)), dim3(kMlpThreads),
                     L_END, s, P, X, labels, index, n_rows, B, (float*)nullptr,
                     part, loss_part);
}

void launch_mlp_reduce(const float* part, uint32_t nw, float* grad, float* P,
                       float* m, float* v, float lr, float bc1, float bc2,
                       bool adam, const double* loss_part, uint32_t B,
                       double* loss, hipStream_t s) {
  const uint32_t nt = 256, nb = (kMlpParams + nt - 1) / nt;
  QOZ_LAUNCH(k_mlp_reduce, dim3(nb), dim3(nt), 0, s, part, nw, grad,
                     P, m, v, lr, bc1, bc2, adam ? 1 : 0, loss_part, B, loss);
}

}  // namespace qoz
