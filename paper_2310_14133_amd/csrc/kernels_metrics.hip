/*
 * Quality metrics of Sec. III on gfx950: value range (for Eq. 1 and the
 * value-range-relative bound), FP64 squared-error and max-error reductions
 * (Eq. 1), and windowed SSIM (Eq. 2-3).
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
#include "qoz_internal.h"

namespace qoz {

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
  hipLaunchKernelGGL(k_range, dim3(nparts), dim3(kRedThreads), 0, s, x, n,
                     part_min, part_max, status);
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
  hipLaunchKernelGGL(k_sse_max, dim3(nparts), dim3(kRedThreads), 0, s, x, y,
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

void launch_ssim(const SsimJob& j, const float* x, const float* y,
                 double* parts, hipStream_t s) {
  static bool attr_set = false;
  size_t lds = ssim_lds(j);
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_ssim,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              150 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(k_ssim, ssim_grid(j), dim3(kSsThreads), lds, s, j, x, y,
                     parts);
}

}  // namespace qoz
