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
 * One workgroup of 1024 lanes per block: the block sits in LDS (143.7 KB),
 * each level's residual sums are block reductions, and the 32768 squared
 * gradients, kept in registers while the block is still needed, are then
 * written over it and bitonic-sorted in LDS for the deciles.
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

/* feat[b][0..30] of block b; aux[b] = (min, max, non-finite flag) for the
 * pooling kernel, which fills feat[b][31] */
__global__ __launch_bounds__(kFeatThreads) void k_block_features(
    const float* __restrict__ x, Geo g, const uint32_t* __restrict__ origins,
    double e, float* __restrict__ feat, float* __restrict__ aux) {
  extern __shared__ float blk[];
  __shared__ double red[4][kFeatThreads / 64];
  __shared__ float mred[3][kFeatThreads / 64];
  __shared__ double stat[20];
  const uint32_t tid = threadIdx.x;
  const uint32_t* o = origins + 3 * blockIdx.x;
  const uint64_t base = (uint64_t)o[0] * g.st[0] + (uint64_t)o[1] * g.st[1] +
                        (uint64_t)o[2] * g.st[2];
  /* the block, row by row */
  for (uint32_t t = tid; t < kBlockPts; t += kFeatThreads) {
    const uint32_t i = t / kPlane, r = t - i * kPlane, j = r / kB1,
                   k = r - j * kB1;
    blk[t] = x[base + (uint64_t)i * g.st[0] + (uint64_t)j * g.st[1] + k];
  }
  __syncthreads();
  /* block range and finiteness */
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
  /* level-wise residual sums: lin |r|, lin r^2, cubic |r|, cubic r^2 */
  for (uint32_t l = 1; l <= 5; ++l) {
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
  /* squared gradients into registers, then over the block */
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
  __syncthreads();
  uint32_t* key = reinterpret_cast<uint32_t*>(blk);
#pragma unroll
  for (uint32_t s = 0; s < kGPer; ++s) key[tid + s * kFeatThreads] = g2[s];
  __syncthreads();
  /* bitonic sort, ascending (non-negative floats order as their bits) */
  for (uint32_t k = 2; k <= kNG; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t q = tid; q < kNG / 2; q += kFeatThreads) {
        const uint32_t i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
        const uint32_t a = key[i], b = key[i | j];
        const bool up = (i & k) == 0;
        if ((a > b) == up) {
          key[i] = b;
          key[i | j] = a;
        }
      }
      __syncthreads();
    }
  if (tid < 31) {
    double f;
    if (tid < 20) {
      f = stat[tid];
    } else if (tid < 30) {
      const uint32_t q = tid - 19;
      const uint32_t idx = (q * kNG + 9) / 10 - 1;
      f = log2(1.0 + sqrt((double)__uint_as_float(key[idx])) / e);
    } else {
      float l2 = mred[0][0], h2 = mred[1][0], b2 = mred[2][0];
      for (uint32_t w = 1; w < kFeatThreads / 64; ++w) {
        l2 = fminf(l2, mred[0][w]);
        h2 = fmaxf(h2, mred[1][w]);
        b2 = fmaxf(b2, mred[2][w]);
      }
      f = log2(1.0 + ((double)h2 - (double)l2) / e);
      if (tid == 30) {
        aux[3 * (uint64_t)blockIdx.x + 0] = l2;
        aux[3 * (uint64_t)blockIdx.x + 1] = h2;
        aux[3 * (uint64_t)blockIdx.x + 2] = b2;
      }
    }
    feat[32 * (uint64_t)blockIdx.x + tid] = (float)f;
  }
}

/* Range over all blocks into every row's feature 31, the mean of each
 * feature over the blocks into out[32], and the non-finite flag into
 * status[0]. */
__global__ void k_feat_pool(float* __restrict__ feat,
                            const float* __restrict__ aux, uint32_t nb,
                            double e, float* __restrict__ out,
                            uint32_t* __restrict__ status) {
  const uint32_t i = threadIdx.x;
  float lo = aux[0], hi = aux[1], bad = aux[2];
  for (uint32_t b = 1; b < nb; ++b) {
    lo = fminf(lo, aux[3 * (uint64_t)b]);
    hi = fmaxf(hi, aux[3 * (uint64_t)b + 1]);
    bad = fmaxf(bad, aux[3 * (uint64_t)b + 2]);
  }
  const float f31 = (float)log2(1.0 + ((double)hi - (double)lo) / e);
  for (uint32_t b = i; b < nb; b += blockDim.x) feat[32 * (uint64_t)b + 31] = f31;
  if (i == 0) status[0] = bad != 0.0f ? kStNonFinite : 0u;
  if (i < 31) {
    double s = 0.0;
    for (uint32_t b = 0; b < nb; ++b) s += (double)feat[32 * (uint64_t)b + i];
    out[i] = (float)(s / (double)nb);
  } else if (i == 31) {
    out[31] = f31;
  }
}

size_t block_features_lds() { return 4 * (size_t)kBlockPts; }

bool block_features_fit() {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            dev) != hipSuccess)
    return false;
  const size_t stat_bytes = 8 * 4 * 16 + 4 * 3 * 16 + 8 * 20;
  if (block_features_lds() + stat_bytes > (size_t)max_lds) return false;
  return hipFuncSetAttribute(
             reinterpret_cast<const void*>(&k_block_features),
             hipFuncAttributeMaxDynamicSharedMemorySize,
             (int)block_features_lds()) == hipSuccess;
}

void launch_block_features(const float* x, const Geo& g,
                           const uint32_t* origins, uint32_t nb, double e,
                           float* feat, float* aux, float* mean,
                           uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_block_features, dim3(nb), dim3(kFeatThreads),
                     block_features_lds(), s, x, g, origins, e, feat, aux);
  hipLaunchKernelGGL(k_feat_pool, dim3(1), dim3(64), 0, s, feat,
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

/* C[M x N] = sum_k A(m, k) B(k, n) on 16x16x16 bf16 MFMA tiles, tiles
 * spread over the workgroup's waves.  Operand lane layout: A row = lane %
 * 16, k = 4 (lane / 16) + j; B k = 4 (lane / 16) + j, column = lane % 16;
 * result row = 4 (lane / 16) + j, column = lane % 16. */
template <class FA, class FB, class FC>
__device__ __forceinline__ void wave_mm(uint32_t M, uint32_t N, uint32_t K,
                                        FA a, FB b, FC c) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t r = lane & 15, q = lane >> 4;
  const uint32_t tn = N >> 4, tiles = (M >> 4) * tn;
  for (uint32_t t = wv; t < tiles; t += nw) {
    const uint32_t m0 = (t / tn) << 4, n0 = (t % tn) << 4;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t k0 = 0; k0 < K; k0 += 16) {
      bf16x4 av, bv;
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        av[j] = (short)a(m0 + r, k0 + 4 * q + j);
        bv[j] = (short)b(k0 + 4 * q + j, n0 + r);
      }
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

  for (uint32_t i = tid; i < NH * NF; i += kMlpThreads)
    W1b[i] = to_bf16(P[kOffW1 + i]);
  for (uint32_t i = tid; i < NH * NH; i += kMlpThreads)
    W2b[i] = to_bf16(P[kOffW2 + i]);
  for (uint32_t i = tid; i < NOP * NH; i += kMlpThreads)
    W3b[i] = i < NO * NH ? to_bf16(P[kOffW3 + i]) : (uint16_t)0;
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

  wave_mm(kTile, NH, NF, [&](uint32_t m, uint32_t k) { return Xb[m * NF + k]; },
          [&](uint32_t k, uint32_t n) { return W1b[n * NF + k]; },
          [&](uint32_t m, uint32_t n, float v) {
            H1b[m * NH + n] = to_bf16(fmaxf(v + b1[n], 0.0f));
          });
  __syncthreads();
  wave_mm(kTile, NH, NH, [&](uint32_t m, uint32_t k) { return H1b[m * NH + k]; },
          [&](uint32_t k, uint32_t n) { return W2b[n * NH + k]; },
          [&](uint32_t m, uint32_t n, float v) {
            H2b[m * NH + n] = to_bf16(fmaxf(v + b2[n], 0.0f));
          });
  __syncthreads();
  wave_mm(kTile, NOP, NH,
          [&](uint32_t m, uint32_t k) { return H2b[m * NH + k]; },
          [&](uint32_t k, uint32_t n) { return W3b[n * NH + k]; },
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
          [&](uint32_t m, uint32_t k) { return dZb[k * NOP + m]; },
          [&](uint32_t k, uint32_t n) { return H2b[k * NH + n]; },
          [&](uint32_t m, uint32_t n, float v) {
            if (m < NO) gp[kOffW3 + m * NH + n] = v;
          });
  if (tid < NO) {
    float t = 0.0f;
    for (uint32_t s = 0; s < kTile; ++s) t += dZf[s * NOP + tid];
    gp[kOffB3 + tid] = t;
  }
  wave_mm(kTile, NH, NOP,
          [&](uint32_t m, uint32_t k) { return dZb[m * NOP + k]; },
          [&](uint32_t k, uint32_t n) { return W3b[k * NH + n]; },
          [&](uint32_t m, uint32_t n, float v) {
            const float d = from_bf16(H2b[m * NH + n]) > 0.0f ? v : 0.0f;
            dHf[m * NH + n] = d;
            dH2b[m * NH + n] = to_bf16(d);
          });
  __syncthreads();
  /* second layer */
  wave_mm(NH, NH, kTile,
          [&](uint32_t m, uint32_t k) { return dH2b[k * NH + m]; },
          [&](uint32_t k, uint32_t n) { return H1b[k * NH + n]; },
          [&](uint32_t m, uint32_t n, float v) { gp[kOffW2 + m * NH + n] = v; });
  if (tid < NH) {
    float t = 0.0f;
    for (uint32_t s = 0; s < kTile; ++s) t += dHf[s * NH + tid];
    gp[kOffB2 + tid] = t;
  }
  __syncthreads();
  wave_mm(kTile, NH, NH,
          [&](uint32_t m, uint32_t k) { return dH2b[m * NH + k]; },
          [&](uint32_t k, uint32_t n) { return W2b[k * NH + n]; },
          [&](uint32_t m, uint32_t n, float v) {
            const float d = from_bf16(H1b[m * NH + n]) > 0.0f ? v : 0.0f;
            dHf[m * NH + n] = d;
            dH1b[m * NH + n] = to_bf16(d);
          });
  __syncthreads();
  /* first layer */
  wave_mm(NH, NF, kTile,
          [&](uint32_t m, uint32_t k) { return dH1b[k * NH + m]; },
          [&](uint32_t k, uint32_t n) { return Xb[k * NF + n]; },
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
  hipLaunchKernelGGL(k_mlp<false>, dim3(mlp_tiles(B)), dim3(kMlpThreads),
                     L_FWD_END, s, P, X, (const int32_t*)nullptr,
                     (const uint32_t*)nullptr, B, B, logits, (float*)nullptr,
                     (double*)nullptr);
}

void launch_mlp_grad(const float* P, const float* X, const int32_t* labels,
                     const uint32_t* index, uint32_t n_rows, uint32_t B,
                     float* part, double* loss_part, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp<true>, dim3(mlp_tiles(B)), dim3(kMlpThreads),
                     L_END, s, P, X, labels, index, n_rows, B, (float*)nullptr,
                     part, loss_part);
}

void launch_mlp_reduce(const float* part, uint32_t nw, float* grad, float* P,
                       float* m, float* v, float lr, float bc1, float bc2,
                       bool adam, const double* loss_part, uint32_t B,
                       double* loss, hipStream_t s) {
  const uint32_t nt = 256, nb = (kMlpParams + nt - 1) / nt;
  hipLaunchKernelGGL(k_mlp_reduce, dim3(nb), dim3(nt), 0, s, part, nw, grad,
                     P, m, v, lr, bc1, bc2, adam ? 1 : 0, loss_part, B, loss);
}

}  // namespace qoz
