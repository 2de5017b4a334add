/*
 * Device functions shared by the compression, decompression and tuner
 * kernels: the 1D interpolation rules of the multi-level predictor
 * (Sec. V-B) and the linear-scale quantizer with level bound e_l (Eq. 5).
 *
 * The stencils are evaluated as separately rounded FP32 operations in the
 * order written; the library is built without FP contraction, so no FMA is
 * formed.
 */
#ifndef QOZ_DEVICE_H
#define QOZ_DEVICE_H
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qoz_internal.h"

namespace qoz {

/* Division of t < tmax by a divisor shared by all lanes, as a
 * multiply-high: m = ceil(2^32 / d) gives floor(t / d) exactly whenever
 * t * d <= 2^32 (t = q d + r: t m / 2^32 = q + (r + t e / 2^32) / d with
 * e = m d - 2^32 < d, and t e < 2^32 keeps the fraction below 1); larger
 * ranges take the plain division. */
struct FastDiv {
  uint32_t d, m;
  bool mul;
  __device__ __forceinline__ FastDiv(uint32_t dv, uint32_t tmax)
      : d(dv),
        m(dv > 1 ? 0xffffffffu / dv + 1u : 0u), /* = ceil(2^32 / d) */
        mul((uint64_t)tmax * dv <= (1ull << 32)) {}
  __device__ __forceinline__ uint32_t div(uint32_t t) const {
    if (d <= 1) return t;
    return mul ? __umulhi(t, m) : t / d;
  }
};

/* Interpolated value at a midpoint from a = f(-3h), b = f(-h), c = f(+h),
 * d = f(+3h).  Linear: mean of b and c.  Cubic: the 4-point midpoint rule
 * (-1, 9, 9, -1)/16, the one-sided 3-point rules (3, 6, -1)/8 and
 * (-1, 6, 3)/8 where a or d is outside the field, the mean where both are.
 * Without c: linear extrapolation (3b - a)/2, or b alone. */
__device__ __forceinline__ float interp_mid(uint32_t cubic, float a, float b,
                                            float c, float d, bool ha,
                                            bool hc, bool hd) {
  if (!hc) return ha ? (b * 3.0f - a) * 0.5f : b;
  if (cubic) {
    if (ha && hd) return ((b + c) * 9.0f - (a + d)) * 0.0625f;
    if (hd) return ((b * 3.0f + c * 6.0f) - d) * 0.125f;
    if (ha) return ((b * 6.0f + c * 3.0f) - a) * 0.125f;
  }
  return (b + c) * 0.5f;
}

/* Prediction of the point at flat index idx, coordinate pk along the swept
 * dimension (stride sk, extent nk), from reconstructed values in W. */
__device__ __forceinline__ float predict_at(const float* W, uint32_t idx,
                                            uint32_t pk, uint32_t sk,
                                            uint32_t nk, uint32_t h,
                                            uint32_t cubic) {
  const uint32_t hs = h * sk;
  const bool ha = pk >= 3 * h;
  const bool hc = pk + h < nk;
  const bool hd = pk + 3 * h < nk;
  const float b = W[idx - hs];
  const float c = hc ? W[idx + hs] : 0.0f;
  float a = 0.0f, d = 0.0f;
  if (cubic) {
    a = ha ? W[idx - 3 * hs] : 0.0f;
    d = hd ? W[idx + 3 * hs] : 0.0f;
  } else if (!hc && ha) {
    a = W[idx - 3 * hs];
  }
  return interp_mid(cubic, a, b, c, d, ha, hc, hd);
}

/* Linear-scale quantization with bin width 2 e_l (inv = 1 / (2 e_l)):
 * bin q = round-half-even((x - pred) / (2 e_l)) in (-R, R), stored as q + R.
 * A residual outside the bins, or a reconstruction pred + q * 2e_l whose
 * distance to x exceeds e_l (checked in FP64), makes the point
 * unpredictable: bin 0 and the exact value. */
__device__ __forceinline__ int32_t quantize_bin(float x, float pred,
                                                float inv, float twoeb,
                                                double eb, float* rec) {
  const float diff = x - pred;
  const float qf = diff * inv;
  if (!(fabsf(qf) < 32768.0f)) {
    *rec = x;
    return 0;
  }
  const int32_t q = (int32_t)rintf(qf);
  if (q >= 32768 || q <= -32768) {
    *rec = x;
    return 0;
  }
  const float t = (float)q * twoeb;
  const float r = pred + t;
  const double err = fabs((double)r - (double)x);
  if (!(err <= eb)) {
    *rec = x;
    return 0;
  }
  *rec = r;
  return q + 32768;
}

/* Windowed histogram of bins: a 4096-bin LDS window centred on the zero
 * bin (the zero bin itself counted per lane), global atomics outside. */
constexpr uint32_t kHistWin = 4096;
constexpr int32_t kHistBase = 32768 - (int32_t)(kHistWin / 2);

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void hist_add(uint32_t* lh, uint32_t* hist,
                                         int32_t c, uint32_t& center) {
  if (c == 32768) {
    ++center;
    return;
  }
  uint32_t o = (uint32_t)(c - kHistBase);
  if (o < kHistWin)
    atomicAdd(&lh[o], 1u);
  else
    atomicAdd(&hist[(uint32_t)c], 1u);
}

__device__ __forceinline__ float dequantize_bin(float pred, int32_t code,
                                                float twoeb) {
  const float t = (float)(code - 32768) * twoeb;
  return pred + t;
}

/* Flat index of the point whose bin sits at stream position pos. */
__device__ __forceinline__ uint32_t point_of(const SweepTable& t, const Geo& g, uint64_t pos) {
  uint32_t lo = 0, hi = t.n; /* find last sweep with off <= pos */
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (t.off[mid] <= pos) lo = mid;
    else hi = mid;
  }
  uint64_t local = pos - t.off[lo];
  uint32_t c2 = t.cnt[lo][2], c1 = t.cnt[lo][1];
  uint32_t i2 = (uint32_t)(local % c2);
  uint64_t r = local / c2;
  uint32_t i1 = (uint32_t)(r % c1);
  uint32_t i0 = (uint32_t)(r / c1);
  uint32_t p0 = t.start[lo][0] + i0 * t.step[lo][0];
  uint32_t p1 = t.start[lo][1] + i1 * t.step[lo][1];
  uint32_t p2 = t.start[lo][2] + i2 * t.step[lo][2];
  return p0 * g.st[0] + p1 * g.st[1] + p2;
}

/* Work queues of several fields in one launch: job j owns the launch's
 * workgroups [wg0[j], wg0[j + 1]) (wg0[0] = 0, nondecreasing).  Returns
 * the job of workgroup wg, the last j with wg0[j] <= wg, counted with one
 * ballot per 64 jobs; the same on every lane.  Every lane of the wave must
 * be active. */
/* A global-memory pointer read from memory (a field of a job record) is a
 * generic pointer to the compiler, which then emits flat accesses; flat
 * accesses count against the LDS wait counter too, so every LDS wait and
 * barrier after one also waits for it (a prefetch issued early is then
 * waited for at the next barrier).  gptr makes such a pointer a global one. */
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(
    const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
/* 16 bytes through a global pointer (uint4 has no assignment from a
 * global-address-space object) */
__device__ __forceinline__ uint4 gload16(const void* p) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = *gptr(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t find_job(const uint32_t* __restrict__ wg0,
                                             uint32_t n_jobs, uint32_t wg) {
  const uint32_t lane = __lane_id();
  uint32_t cnt = 0;
  for (uint32_t b = 0; b < n_jobs; b += 64) {
    const uint32_t i = b + lane;
    const bool le = i < n_jobs && wg0[i] <= wg;
    cnt += (uint32_t)__popcll(__ballot(le));
  }
  return __builtin_amdgcn_readfirstlane(cnt - 1);
}

}  // namespace qoz
#endif
