/*
 * Interpolation sweeps of the multi-level predictor (Sec. V) with the
 * level-wise linear-scale quantizer (Eq. 5), for gfx950.
 *
 * One launch per (level, dimension) sweep.  Within a sweep every target is
 * predicted from points known before the sweep (coarser levels and earlier
 * sweeps of the level), so targets are independent: one lane per target,
 * 64 consecutive targets of a row per wavefront so that bin writes are
 * dense and reads along the contiguous dimension coalesce.
 *
 * FP32 evaluation order is fixed and FP contraction is disabled for the
 * whole library, so predictions, bins and reconstructions are reproducible
 * bit for bit on any IEEE FP32 implementation.
 */
#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

__global__ void k_init_status(uint32_t* st) {
  if (threadIdx.x < 8) st[threadIdx.x] = 0;
}

void launch_init_status(uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, s, status);
}

__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}

void launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s) {
  if (!n) return;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p,
                     n);
}

/* Anchor grid (Sec. V-B): every point whose coordinates are all multiples
 * of s is stored verbatim, in row-major order of the anchor grid. */
__global__ void k_anchor_copy(Geo g, uint32_t stride, uint32_t na0,
                              uint32_t na1, uint32_t na2,
                              const float* __restrict__ x,
                              float* __restrict__ W, float* __restrict__ out,
                              uint32_t* status) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t total = na0 * na1 * na2;
  if (t >= total) return;
  uint32_t a2 = t % na2;
  uint32_t r = t / na2;
  uint32_t a1 = r % na1;
  uint32_t a0 = r / na1;
  uint32_t idx = a0 * stride * g.st[0] + a1 * stride * g.st[1] + a2 * stride;
  float v = x[idx];
  W[idx] = v;
  out[t] = v;
  if (!isfinite(v)) atomicOr(status, kStNonFinite);
}

__global__ void k_anchor_scatter(Geo g, uint32_t stride, uint32_t na0,
                                 uint32_t na1, uint32_t na2,
                                 const float* __restrict__ in,
                                 float* __restrict__ W) {
  uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t total = na0 * na1 * na2;
  if (t >= total) return;
  uint32_t a2 = t % na2;
  uint32_t r = t / na2;
  uint32_t a1 = r % na1;
  uint32_t a0 = r / na1;
  uint32_t idx = a0 * stride * g.st[0] + a1 * stride * g.st[1] + a2 * stride;
  W[idx] = in[t];
}

void launch_anchor_copy(const Geo& g, uint32_t stride, const uint32_t na[3],
                        const float* x, float* W, float* out,
                        uint32_t* status, hipStream_t s) {
  uint32_t total = na[0] * na[1] * na[2];
  hipLaunchKernelGGL(k_anchor_copy, dim3((total + 255) / 256), dim3(256), 0,
                     s, g, stride, na[0], na[1], na[2], x, W, out, status);
}

void launch_anchor_scatter(const Geo& g, uint32_t stride, const uint32_t na[3],
                           const float* in, float* W, hipStream_t s) {
  uint32_t total = na[0] * na[1] * na[2];
  hipLaunchKernelGGL(k_anchor_scatter, dim3((total + 255) / 256), dim3(256),
                     0, s, g, stride, na[0], na[1], na[2], in, W);
}

/* Sweep launch shape: x covers 64 consecutive targets of a row, y covers
 * rows (flattened over the two outer sub-grid dimensions), 4 rows per
 * workgroup, grid-stride over rows beyond the y limit. */
constexpr uint32_t kSweepTX = 64;
constexpr uint32_t kSweepTY = 4;
constexpr uint32_t kMaxGridY = 65535;

struct SweepPoint {
  uint32_t idx;   /* flat index of the target */
  uint32_t pk;    /* its coordinate along the swept dimension */
  uint64_t pos;   /* its bin's stream position */
};

__device__ __forceinline__ SweepPoint sweep_point(const Geo& g,
                                                  const Sweep& s, uint32_t r,
                                                  uint32_t i2) {
  uint32_t i0 = r / s.cnt[1];
  uint32_t i1 = r - i0 * s.cnt[1];
  uint32_t p0 = s.start[0] + i0 * s.step[0];
  uint32_t p1 = s.start[1] + i1 * s.step[1];
  uint32_t p2 = s.start[2] + i2 * s.step[2];
  SweepPoint sp;
  sp.idx = p0 * g.st[0] + p1 * g.st[1] + p2;
  sp.pk = s.k == 0 ? p0 : (s.k == 1 ? p1 : p2);
  sp.pos = s.code_off + (uint64_t)r * s.cnt[2] + i2;
  return sp;
}

template <bool WRITE_W>
__global__ __launch_bounds__(kSweepTX * kSweepTY) void k_sweep_comp(
    Geo g, Sweep s, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status) {
  const uint32_t i2 = blockIdx.x * kSweepTX + threadIdx.x;
  if (i2 >= s.cnt[2]) return;
  const uint32_t rows = s.cnt[0] * s.cnt[1];
  const uint32_t sk = g.st[s.k];
  const uint32_t nk = g.n[s.k];
  bool bad = false;
  for (uint32_t r = blockIdx.y * kSweepTY + threadIdx.y; r < rows;
       r += gridDim.y * kSweepTY) {
    SweepPoint sp = sweep_point(g, s, r, i2);
    float pred = predict_at(W, sp.idx, sp.pk, sk, nk, s.h, s.cubic);
    float xv = x[sp.idx];
    float rec;
    int32_t code = quantize_bin(xv, pred, s.inv, s.twoeb, s.eb, &rec);
    if (WRITE_W) W[sp.idx] = rec;
    codes[sp.pos] = (uint16_t)code;
    bad |= !isfinite(xv);
  }
  if (bad) atomicOr(status, kStNonFinite);
}

/* Decompression: bins >= 1 reconstruct pred + (bin - R) * 2e_l with the
 * same two roundings as the compressor.  Bin 0 (unpredictable) is skipped:
 * its exact value was scattered into W before the sweeps. */
__global__ __launch_bounds__(kSweepTX * kSweepTY) void k_sweep_decomp(
    Geo g, Sweep s, float* W, const uint16_t* __restrict__ codes) {
  const uint32_t i2 = blockIdx.x * kSweepTX + threadIdx.x;
  if (i2 >= s.cnt[2]) return;
  const uint32_t rows = s.cnt[0] * s.cnt[1];
  const uint32_t sk = g.st[s.k];
  const uint32_t nk = g.n[s.k];
  for (uint32_t r = blockIdx.y * kSweepTY + threadIdx.y; r < rows;
       r += gridDim.y * kSweepTY) {
    SweepPoint sp = sweep_point(g, s, r, i2);
    const int32_t code = codes[sp.pos];
    if (code == 0) continue;
    float pred = predict_at(W, sp.idx, sp.pk, sk, nk, s.h, s.cubic);
    W[sp.idx] = dequantize_bin(pred, code, s.twoeb);
  }
}

/* Unpredictable values to their points: upos[r] is the stream position of
 * the r-th unpredictable bin (recorded by the decoder). */
__global__ void k_unpred_scatter(Geo g, SweepTable st,
                                 const uint32_t* __restrict__ upos,
                                 const float* __restrict__ vals,
                                 uint64_t n_unpred, uint64_t n_codes,
                                 float* __restrict__ W, uint32_t* status) {
  bool bad = false;
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
       r < n_unpred; r += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t pos = upos[r];
    if (pos >= n_codes) {
      bad = true;
      continue;
    }
    W[point_of(st, g, pos)] = vals[r];
  }
  if (bad) atomicOr(status, kStBadStream);
}

void launch_unpred_scatter(const Geo& g, const SweepTable& st,
                           const uint32_t* upos, const float* vals,
                           uint64_t n_unpred, uint64_t n_codes, float* W,
                           uint32_t* status, hipStream_t s) {
  if (!n_unpred) return;
  uint64_t blocks = (n_unpred + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_unpred_scatter, dim3((uint32_t)blocks), dim3(256), 0,
                     s, g, st, upos, vals, n_unpred, n_codes, W, status);
}

static dim3 sweep_grid_dim(const Sweep& sw) {
  uint32_t gx = (sw.cnt[2] + kSweepTX - 1) / kSweepTX;
  uint64_t rows = (uint64_t)sw.cnt[0] * sw.cnt[1];
  uint64_t gy = (rows + kSweepTY - 1) / kSweepTY;
  if (gy > kMaxGridY) gy = kMaxGridY;
  return dim3(gx, (uint32_t)gy);
}

void launch_sweep_comp(const Geo& g, const Sweep& sw, const float* x,
                       float* W, uint16_t* codes, bool write_w,
                       uint32_t* status, hipStream_t s) {
  if (sw.count == 0) return;
  dim3 grid = sweep_grid_dim(sw), block(kSweepTX, kSweepTY);
  if (write_w)
    hipLaunchKernelGGL(k_sweep_comp<true>, grid, block, 0, s, g, sw, x, W,
                       codes, status);
  else
    hipLaunchKernelGGL(k_sweep_comp<false>, grid, block, 0, s, g, sw, x, W,
                       codes, status);
}

void launch_sweep_decomp(const Geo& g, const Sweep& sw, float* W,
                         const uint16_t* codes, hipStream_t s) {
  if (sw.count == 0) return;
  dim3 grid = sweep_grid_dim(sw), block(kSweepTX, kSweepTY);
  hipLaunchKernelGGL(k_sweep_decomp, grid, block, 0, s, g, sw, W, codes);
}

}  // namespace qoz
