/*
 * Quality metrics of Sec. III on gfx950: value range (for Eq. 1 and the
 * value-range-relative bound), FP64 squared-error and max-error reductions
 * (Eq. 1), windowed SSIM (Eq. 2-3) and the error moments of the lag-1
 * autocorrelation (Eq. 4).
 *
 * Reductions write one partial per workgroup in a fixed assignment; the
 * host adds the partials in index order, so results are identical from run
 * to run.
 *
 * SSIM: w^d uniform windows, step 1, fully inside the field, population
 * moments.  Window sums are separable: along the contiguous dimension, then
 * the middle one, then (3D) the slowest one, each a sequential sum of w
 * terms in ascending order.  A workgroup owns 4 x 64 window origins of the
 * (row, column) plane and streams through a range of planes, keeping the
 * last w planes of 2D window sums in an LDS ring.
 */
#include <mutex>

#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

constexpr int kSsimLdsMax = 150 * 1024; /* largest dynamic LDS of k_ssim */

/* Scratch of the metrics call that allocates nothing (qoz_metrics_noalloc):
 * every device holds its own copy for the life of the process.  Host code
 * never passes this name to a kernel; it uses the address that
 * fixed_scratch_addr looks up on each device. */
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];
static_assert(kFixedPartialOff + 8 * 2048 + 16 * 2048 <= kFixedSsimOff,
              "range and SSE partial sums overlap the SSIM partial sums");

hipError_t fixed_scratch_addr(int dev, void** out) {
  constexpr int kMaxDev = 64;
  static std::once_flag once[kMaxDev];
  static void* addr[kMaxDev];
  static hipError_t err[kMaxDev];
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::call_once(once[dev], [dev] {
    err[dev] = hipGetSymbolAddress(&addr[dev], HIP_SYMBOL(scratch));
  });
  if (err[dev] != hipSuccess) return err[dev];
  *out = addr[dev];
  return hipSuccess;
}

constexpr uint32_t kRedThreads = 256;

uint32_t range_parts(uint64_t n) {
  uint64_t p = (n + kRedThreads * 64 - 1) / (kRedThreads * 64);
  if (p < 1) p = 1;
  if (p > 2048) p = 2048;
  return (uint32_t)p;
}
uint32_t sse_parts(uint64_t n) { return range_parts(n); }

/* four floats; a word-aligned 16-byte load */
struct __attribute__((aligned(4))) Q4 {
  float a, b, c, d;
};

/* Each workgroup reads a contiguous range of 4-float groups, four 16-byte
 * loads in flight per lane (contiguous ranges per workgroup stream better
 * than a grid-wide stride); the last n mod 4 values go to the first lanes
 * of the grid. */
template <class F>
__device__ __forceinline__ void for_each4(const float* __restrict__ x,
                                          uint64_t n, F&& f) {
  constexpr uint32_t kU = 4;
  const uint64_t n4 = n / 4;
  const uint64_t per = (n4 + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = b0 + per < n4 ? b0 + per : n4;
  const Q4* x4 = reinterpret_cast<const Q4*>(x);
  uint64_t i = b0 + threadIdx.x;
  for (; i + (kU - 1) * kRedThreads < b1; i += kU * kRedThreads) {
    Q4 v[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) v[u] = x4[i + u * kRedThreads];
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) f(i + u * kRedThreads, v[u]);
  }
  for (; i < b1; i += kRedThreads) f(i, x4[i]);
}

__global__ __launch_bounds__(kRedThreads) void k_range(
    const float* __restrict__ x, uint64_t n, float* pmin, float* pmax,
    uint32_t* status) {
  __shared__ float smin[kRedThreads], smax[kRedThreads];
  float lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  auto take = [&](float v) {
    bad |= !isfinite(v);
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  };
  for_each4(x, n, [&](uint64_t, const Q4& v) {
    take(v.a);
    take(v.b);
    take(v.c);
    take(v.d);
  });
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < n % 4) take(x[n / 4 * 4 + gid]);
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (uint32_t o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pmin[blockIdx.x] = smin[0];
    pmax[blockIdx.x] = smax[0];
  }
  if (bad) atomicOr(status, kStNonFinite);
}

void launch_range(const float* x, uint64_t n, float* part_min,
                  float* part_max, uint32_t* status, uint32_t nparts,
                  hipStream_t s) {
  QOZ_LAUNCH(k_range, dim3(nparts), dim3(kRedThreads), 0, s, x, n,
                     part_min, part_max, status);
}

/* Error moments of the lag-1 autocorrelation (Eq. 4) over cnt points of
 * rows of len values starting at x, y, in two passes as the definition
 * reads.  Pass 0: out[0] = sum e.  Pass 1, with the mean mu of e over the
 * whole set: out[0] = sum (e - mu)^2, out[1] = sum over the pairs of
 * neighbours in a row of (e_i - mu)(e_(i+1) - mu). */
__device__ void ac_moments(const float* __restrict__ x,
                           const float* __restrict__ y, uint32_t cnt,
                           uint32_t len, int pass, double mu, double* out) {
  __shared__ double red[2][kRedThreads / 64];
  const FastDiv fl(len, cnt);
  double m0 = 0.0, m1 = 0.0;
  for (uint32_t t = threadIdx.x; t < cnt; t += kRedThreads) {
    const double e = (double)x[t] - (double)y[t];
    if (pass == 0) {
      m0 += e;
      continue;
    }
    const double d = e - mu;
    m0 += d * d;
    const uint32_t col = t - fl.div(t) * len;
    if (col + 1 < len) m1 += d * (((double)x[t + 1] - (double)y[t + 1]) - mu);
  }
  for (int o = 32; o > 0; o >>= 1) {
    m0 += __shfl_xor(m0, o, 64);
    m1 += __shfl_xor(m1, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = m0;
    red[1][threadIdx.x >> 6] = m1;
  }
  __syncthreads();
  if (threadIdx.x < (pass == 0 ? 1u : 2u)) {
    double t = 0.0;
    for (uint32_t w = 0; w < kRedThreads / 64; ++w) t += red[threadIdx.x][w];
    out[threadIdx.x] = t;
  }
}

/* mean of a set from its pass-0 partials p[0..np) over n points */
__device__ __forceinline__ double ac_mean(const double* __restrict__ p,
                                          uint32_t np, double n) {
  double s = 0.0;
  for (uint32_t i = 0; i < np; ++i) s += p[i];
  return s / n;
}

/* the field: workgroup w takes rows [w rows_per_wg, +rows_per_wg); pass 1
 * reads the pass-0 partials p0 of all nparts workgroups */
__global__ __launch_bounds__(kRedThreads) void k_ac_field(
    const float* __restrict__ x, const float* __restrict__ y, uint64_t nrows,
    uint32_t len, uint64_t rows_per_wg, int pass, const double* p0,
    double* part) {
  const uint64_t r0 = (uint64_t)blockIdx.x * rows_per_wg;
  const uint64_t r1 = r0 + rows_per_wg < nrows ? r0 + rows_per_wg : nrows;
  const uint32_t cnt = r0 < r1 ? (uint32_t)((r1 - r0) * len) : 0u;
  const double mu =
      pass == 0 ? 0.0 : ac_mean(p0, gridDim.x, (double)nrows * (double)len);
  ac_moments(x + r0 * len, y + r0 * len, cnt, len, pass, mu,
             part + (pass == 0 ? 1 : 2) * (uint64_t)blockIdx.x);
}

uint32_t ac_parts(uint64_t nrows, uint32_t len, uint64_t* rows_per_wg) {
  uint64_t parts = nrows < 2048 ? nrows : 2048;
  if (parts < 1) parts = 1;
  uint64_t per = (nrows + parts - 1) / parts;
  /* a workgroup's points must index in 32 bits */
  const uint64_t cap = (1ull << 31) / (len ? len : 1);
  if (per > cap) per = cap;
  if (per < 1) per = 1;
  *rows_per_wg = per;
  return (uint32_t)((nrows + per - 1) / per);
}

void launch_ac_field(const float* x, const float* y, uint64_t nrows,
                     uint32_t len, double* p0, double* p1, hipStream_t s) {
  uint64_t per;
  const uint32_t parts = ac_parts(nrows, len, &per);
  QOZ_LAUNCH(k_ac_field, dim3(parts), dim3(kRedThreads), 0, s, x, y,
                     nrows, len, per, 0, (const double*)nullptr, p0);
  QOZ_LAUNCH(k_ac_field, dim3(parts), dim3(kRedThreads), 0, s, x, y,
                     nrows, len, per, 1, (const double*)p0, p1);
}

/* the tuner's items: block blockIdx.y of xs against trial blockIdx.x's
 * reconstruction in wt (stride `size` floats per item); the mean of pass 1
 * is that of the trial's nb blocks together */
__global__ __launch_bounds__(kRedThreads) void k_ac_items(
    const float* __restrict__ xs, const float* __restrict__ wt, uint32_t nb,
    uint32_t size, uint32_t len, int pass, const double* p0, double* part) {
  const uint64_t item = (uint64_t)blockIdx.x * nb + blockIdx.y;
  const double mu =
      pass == 0 ? 0.0
                : ac_mean(p0 + (uint64_t)blockIdx.x * nb, nb,
                          (double)nb * (double)size);
  ac_moments(xs + (uint64_t)blockIdx.y * size, wt + item * size, size, len,
             pass, mu, part + (pass == 0 ? 1 : 2) * item);
}

void launch_ac_items(const float* xs, const float* wt, uint32_t ntrial,
                     uint32_t nb, uint32_t size, uint32_t len, double* p0,
                     double* p1, hipStream_t s) {
  QOZ_LAUNCH(k_ac_items, dim3(ntrial, nb), dim3(kRedThreads), 0, s,
                     xs, wt, nb, size, len, 0, (const double*)nullptr, p0);
  QOZ_LAUNCH(k_ac_items, dim3(ntrial, nb), dim3(kRedThreads), 0, s,
                     xs, wt, nb, size, len, 1, (const double*)p0, p1);
}

__global__ __launch_bounds__(kRedThreads) void k_sse_max(
    const float* __restrict__ x, const float* __restrict__ y, uint64_t n,
    double* psse, double* pmax) {
  __shared__ double ss[kRedThreads], sm[kRedThreads];
  double acc = 0.0, mx = 0.0;
  const Q4* y4 = reinterpret_cast<const Q4*>(y);
  auto take = [&](float a, float b) {
    const double d = (double)a - (double)b;
    acc += d * d;
    mx = fmax(mx, fabs(d));
  };
  for_each4(x, n, [&](uint64_t i, const Q4& v) {
    const Q4 w = y4[i];
    take(v.a, w.a);
    take(v.b, w.b);
    take(v.c, w.c);
    take(v.d, w.d);
  });
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < n % 4) take(x[n / 4 * 4 + gid], y[n / 4 * 4 + gid]);
  ss[threadIdx.x] = acc;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (uint32_t o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    psse[blockIdx.x] = ss[0];
    pmax[blockIdx.x] = sm[0];
  }
}

void launch_sse_max(const float* x, const float* y, uint64_t n,
                    double* part_sse, double* part_max, uint32_t nparts,
                    hipStream_t s) {
  QOZ_LAUNCH(k_sse_max, dim3(nparts), dim3(kRedThreads), 0, s, x, y,
                     n, part_sse, part_max);
}

/* ---- SSIM ------------------------------------------------------------ */

constexpr uint32_t kSsTC = 64, kSsTR = 4, kSsThreads = kSsTC * kSsTR;
constexpr uint32_t kSsPlanes = 32; /* output planes per workgroup */

struct Mom {
  double x, y, xx, yy, xy;
};

__host__ __device__ static inline uint32_t ssim_chunks(const SsimJob& j) {
  uint32_t oP = j.P - j.wp + 1;
  return (oP + kSsPlanes - 1) / kSsPlanes;
}

static dim3 ssim_grid(const SsimJob& j) {
  uint32_t oR = j.Rn - j.wr + 1, oC = j.Cn - j.wc + 1;
  return dim3((oC + kSsTC - 1) / kSsTC, (oR + kSsTR - 1) / kSsTR,
              j.batch * ssim_chunks(j));
}

uint64_t ssim_parts(const SsimJob& j) {
  dim3 g = ssim_grid(j);
  return (uint64_t)g.x * g.y * g.z;
}

static size_t ssim_lds(const SsimJob& j) {
  return sizeof(Mom) * ((size_t)(kSsTR + j.wr - 1) * kSsTC +
                        (size_t)j.wp * kSsThreads);
}

__device__ __forceinline__ void mom_add(Mom& a, const Mom& b) {
  a.x += b.x;
  a.y += b.y;
  a.xx += b.xx;
  a.yy += b.yy;
  a.xy += b.xy;
}

__global__ __launch_bounds__(kSsThreads) void k_ssim(
    SsimJob j, const float* __restrict__ xb, const float* __restrict__ yb,
    double* parts) {
  extern __shared__ Mom lds[];
  Mom* A = lds;                                /* (TR + wr - 1) x TC */
  Mom* ring = lds + (kSsTR + j.wr - 1) * kSsTC; /* wp x threads */
  __shared__ double red[kSsThreads];
  const uint32_t nch = ssim_chunks(j);
  const uint32_t item = blockIdx.z / nch, chunk = blockIdx.z % nch;
  const uint32_t oP = j.P - j.wp + 1, oR = j.Rn - j.wr + 1,
                 oC = j.Cn - j.wc + 1;
  const uint32_t q0 = chunk * kSsPlanes;
  const uint32_t q1 = q0 + kSsPlanes < oP ? q0 + kSsPlanes : oP;
  const float* x = xb + (uint64_t)(item % j.x_mod) * j.field_stride;
  const float* y = yb + (uint64_t)item * j.field_stride;
  const uint32_t r0 = blockIdx.y * kSsTR, c0 = blockIdx.x * kSsTC;
  const uint32_t tr = threadIdx.x / kSsTC, tc = threadIdx.x % kSsTC;
  const bool mine = r0 + tr < oR && c0 + tc < oC;
  const double n = (double)j.wp * (double)j.wr * (double)j.wc;
  const uint64_t plane = (uint64_t)j.Rn * j.Cn;
  double acc = 0.0;
  for (uint32_t p = q0; p < q1 + j.wp - 1; ++p) {
    const float* xp = x + p * plane;
    const float* yp = y + p * plane;
    for (uint32_t e = threadIdx.x; e < (kSsTR + j.wr - 1) * kSsTC;
         e += kSsThreads) {
      uint32_t row = e / kSsTC, col = e % kSsTC;
      uint32_t rr = r0 + row, cc = c0 + col;
      Mom m = {0, 0, 0, 0, 0};
      if (rr < j.Rn && cc < oC) {
        const float* xr = xp + (uint64_t)rr * j.Cn + cc;
        const float* yr = yp + (uint64_t)rr * j.Cn + cc;
        for (uint32_t t = 0; t < j.wc; ++t) {
          double xv = xr[t], yv = yr[t];
          m.x += xv;
          m.y += yv;
          m.xx += xv * xv;
          m.yy += yv * yv;
          m.xy += xv * yv;
        }
      }
      A[e] = m;
    }
    __syncthreads();
    Mom b = {0, 0, 0, 0, 0};
    for (uint32_t t = 0; t < j.wr; ++t) mom_add(b, A[(tr + t) * kSsTC + tc]);
    ring[((p - q0) % j.wp) * kSsThreads + threadIdx.x] = b;
    if (p - q0 + 1 >= j.wp && mine) {
      uint32_t p0 = p + 1 - j.wp;
      Mom s = {0, 0, 0, 0, 0};
      for (uint32_t t = 0; t < j.wp; ++t)
        mom_add(s, ring[((p0 - q0 + t) % j.wp) * kSsThreads + threadIdx.x]);
      double mx = s.x / n;
      double my = s.y / n;
      double vx = s.xx / n - mx * mx;
      double vy = s.yy / n - my * my;
      double cxy = s.xy / n - mx * my;
      double num = (2.0 * mx * my + j.c1) * (2.0 * cxy + j.c2);
      double den = (mx * mx + my * my + j.c1) * (vx + vy + j.c2);
      acc += num / den;
    }
    __syncthreads();
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t o = kSsThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    uint64_t bid = ((uint64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x +
                   blockIdx.x;
    parts[bid] = red[0];
  }
}

/* The SSIM ring needs more dynamic LDS than the default limit.  The
 * attribute is set once per device under a per-device once-flag (batch
 * workers launch this from several threads) and its status is kept. */
bool launch_ssim(const SsimJob& j, const float* x, const float* y,
                 double* parts, hipStream_t s) {
  constexpr int kMaxDev = 64;
  static std::once_flag once[kMaxDev];
  static bool ok[kMaxDev];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev)
    return false;
  std::call_once(once[dev], [dev] {
    int max_lds = 0;
    ok[dev] = hipDeviceGetAttribute(&max_lds,
                                    hipDeviceAttributeMaxSharedMemoryPerBlock,
                                    dev) == hipSuccess &&
              max_lds >= kSsimLdsMax &&
              hipFuncSetAttribute((const void*)k_ssim,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kSsimLdsMax) == hipSuccess;
  });
  if (!ok[dev] || ssim_lds(j) > (size_t)kSsimLdsMax) return false;
  QOZ_LAUNCH(k_ssim, ssim_grid(j), dim3(kSsThreads), ssim_lds(j), s,
                     j, x, y, parts);
  return true;
}

}  // namespace qoz
