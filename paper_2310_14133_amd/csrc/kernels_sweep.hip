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
  QOZ_LAUNCH(k_init_status, dim3(1), dim3(64), 0, s, status);
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
  QOZ_LAUNCH(k_zero_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p,
                     n);
}

/* Copies between device memory and coherent host memory.  The host side
 * is accessed with system-scope (write-through, uncached) loads or stores,
 * 4 bytes at a time when both ends and the size allow, else bytewise; the
 * device side with plain accesses. */
template <bool TO_HOST, typename T>
__device__ __forceinline__ void copy_host_units(T* dst, const T* src,
                                                uint64_t n) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = tid; i < n; i += stride) {
    if (TO_HOST) {
      __hip_atomic_store(dst + i, src[i], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
      dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

template <bool TO_HOST>
__global__ void k_copy_host(uint8_t* dst, const uint8_t* src, uint64_t n) {
  if ((((uintptr_t)dst | (uintptr_t)src | n) & 3) == 0)
    copy_host_units<TO_HOST>(reinterpret_cast<uint32_t*>(dst),
                             reinterpret_cast<const uint32_t*>(src), n / 4);
  else
    copy_host_units<TO_HOST>(dst, src, n);
}

/* Up to four device-to-device copies in one launch (blockIdx.y picks
 * the region), 16 bytes per lane where both ends allow it; the runtime's
 * copy takes tens of microseconds per call for these small sections. */
struct CopyRegions {
  const uint8_t* src[4];
  uint8_t* dst[4];
  uint64_t bytes[4];
};

__global__ __launch_bounds__(256) void k_copy_regions(CopyRegions r) {
  const uint32_t k = blockIdx.y;
  const uint8_t* src = r.src[k];
  uint8_t* dst = r.dst[k];
  const uint64_t n = r.bytes[k];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((((uintptr_t)src | (uintptr_t)dst) & 15u) == 0) {
    const uint64_t n16 = n / 16;
    for (uint64_t i = t; i < n16; i += stride)
      reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    for (uint64_t i = n16 * 16 + t; i < n; i += stride) dst[i] = src[i];
  } else {
    for (uint64_t i = t; i < n; i += stride) dst[i] = src[i];
  }
}

void launch_copy_regions(void* const* dst, const void* const* src,
                         const uint64_t* bytes, uint32_t n, hipStream_t s) {
  CopyRegions r;
  uint64_t most = 0;
  uint32_t m = 0;
  for (uint32_t k = 0; k < n && m < 4; ++k) {
    if (!bytes[k]) continue;
    r.src[m] = (const uint8_t*)src[k];
    r.dst[m] = (uint8_t*)dst[k];
    r.bytes[m] = bytes[k];
    most = bytes[k] > most ? bytes[k] : most;
    ++m;
  }
  if (!m) return;
  uint64_t blocks = (most / 16 + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  QOZ_LAUNCH(k_copy_regions, dim3((uint32_t)blocks, m), dim3(256), 0,
                     s, r);
}

/* Many device-to-host copies in one launch, a workgroup per copy; the
 * copy list itself lies in coherent host memory. */
__global__ __launch_bounds__(256) void k_gather_host(
    const HostCopy* __restrict__ list) {
  const HostCopy* h = list + blockIdx.x;
  const uint8_t* src = (const uint8_t*)__hip_atomic_load(
      (const uint64_t*)&h->src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  uint8_t* dst = (uint8_t*)__hip_atomic_load(
      (const uint64_t*)&h->dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  const uint64_t n = __hip_atomic_load(&h->bytes, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
  if ((((uintptr_t)dst | (uintptr_t)src | n) & 3) == 0) {
    const uint32_t* s4 = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d4 = reinterpret_cast<uint32_t*>(dst);
    for (uint64_t i = threadIdx.x; i < n / 4; i += blockDim.x)
      __hip_atomic_store(d4 + i, s4[i], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  } else {
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x)
      __hip_atomic_store(dst + i, src[i], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

void launch_gather_host(const HostCopy* list, uint32_t n, hipStream_t s) {
  if (!n) return;
  QOZ_LAUNCH(k_gather_host, dim3(n), dim3(256), 0, s, list);
}

/* The exact values of a batch of streams: per job (one stream) the anchor
 * grid (first wg_anchor workgroups, one anchor per lane) and then the
 * unpredictable values (a grid-stride loop over the remaining ones). */
__global__ __launch_bounds__(256) void k_exact_q(
    const ExactJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  const uint32_t j = find_job(wg0, n_jobs, blockIdx.x);
  const ExactJob& a = jobs[j];
  const uint32_t lid = blockIdx.x - wg0[j];
  if (lid < a.wg_anchor) {
    const uint32_t t = lid * blockDim.x + threadIdx.x;
    const uint32_t total = a.na[0] * a.na[1] * a.na[2];
    if (t >= total) return;
    const uint32_t a2 = t % a.na[2];
    const uint32_t r = t / a.na[2];
    const uint32_t a1 = r % a.na[1];
    const uint32_t a0 = r / a.na[1];
    a.W[a0 * a.stride * a.g.st[0] + a1 * a.stride * a.g.st[1] +
        a2 * a.stride] = a.anchors[t];
    return;
  }
  const uint32_t wgu = wg0[j + 1] - wg0[j] - a.wg_anchor;
  bool bad = false;
  for (uint64_t r = (uint64_t)(lid - a.wg_anchor) * blockDim.x + threadIdx.x;
       r < a.n_unpred; r += (uint64_t)wgu * blockDim.x) {
    const uint32_t pos = a.upos[r];
    if (pos >= a.n_codes) {
      bad = true;
      continue;
    }
    a.W[point_of(*a.st, a.g, pos)] = a.vals[r];
  }
  if (bad) atomicOr(a.status, kStBadStream);
}

uint32_t exact_job_workgroups(ExactJob* j) {
  const uint64_t total = (uint64_t)j->na[0] * j->na[1] * j->na[2];
  j->wg_anchor = (uint32_t)((total + 255) / 256);
  /* the unpredictable values' grid-stride loop is sized by the number of
   * bins, not of unpredictable values, so that streams of the same shapes
   * give the same launch grid */
  uint64_t wu = (j->n_codes + 16383) / 16384;
  if (wu < 1) wu = 1;
  if (wu > 4096) wu = 4096;
  return j->wg_anchor + (uint32_t)wu;
}

void launch_exact_q(const ExactJob* jobs, const uint32_t* wg0,
                    uint32_t n_jobs, uint32_t total_wg, hipStream_t s) {
  if (!total_wg) return;
  QOZ_LAUNCH(k_exact_q, dim3(total_wg), dim3(256), 0, s, jobs, wg0,
                     n_jobs);
}

void launch_copy_host(void* dst, const void* src, size_t bytes, bool to_host,
                      hipStream_t s) {
  if (!bytes) return;
  uint64_t blocks = (bytes / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  if (to_host)
    QOZ_LAUNCH(k_copy_host<true>, dim3((uint32_t)blocks), dim3(256),
                       0, s, (uint8_t*)dst, (const uint8_t*)src,
                       (uint64_t)bytes);
  else
    QOZ_LAUNCH(k_copy_host<false>, dim3((uint32_t)blocks), dim3(256),
                       0, s, (uint8_t*)dst, (const uint8_t*)src,
                       (uint64_t)bytes);
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
  QOZ_LAUNCH(k_anchor_copy, dim3((total + 255) / 256), dim3(256), 0,
                     s, g, stride, na[0], na[1], na[2], x, W, out, status);
}

void launch_anchor_scatter(const Geo& g, uint32_t stride, const uint32_t na[3],
                           const float* in, float* W, hipStream_t s) {
  uint32_t total = na[0] * na[1] * na[2];
  QOZ_LAUNCH(k_anchor_scatter, dim3((total + 255) / 256), dim3(256),
                     0, s, g, stride, na[0], na[1], na[2], in, W);
}

/* Sweep launch shape: x covers 64 consecutive targets of a row, y covers
 * rows (flattened over the two outer sub-grid dimensions), 4 rows per
 * workgroup, grid-stride over rows beyond the y limit. */
/* Workgroups go to the 8 XCDs round-robin by dispatch id, each XCD with
 * its own L2.  xcd_block maps a dispatch id to a logical id so that every
 * XCD takes one contiguous range of logical workgroups (target rows that
 * read the same neighbour rows then share an L2); the identity when the
 * count is not a multiple of 8.  (The level-1 row kernels keep dispatch
 * order: their neighbour rows are mostly in the same workgroup, and the
 * remap measured slower there.) */
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t id, uint32_t total) {
  if (total % kXcds) return id;
  return (id % kXcds) * (total / kXcds) + id / kXcds;
}

constexpr uint32_t kSweepTX = 64;
constexpr uint32_t kSweepTYMax = 16; /* rows per workgroup: blockDim.y */
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

/* Workgroup (bx, by) of a sweep's gx x gy grid of ty-row tiles; this lane
 * is target tx of row tyi of the tile. */
template <bool WRITE_W>
__device__ __forceinline__ void sweep_comp_wg(
    const Geo& g, const Sweep& s, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status, uint32_t bx, uint32_t by,
    uint32_t gy, uint32_t tx, uint32_t tyi, uint32_t ty) {
  const uint32_t i2 = bx * kSweepTX + tx;
  if (i2 >= s.cnt[2]) return;
  const uint32_t rows = s.cnt[0] * s.cnt[1];
  const uint32_t sk = g.st[s.k];
  const uint32_t nk = g.n[s.k];
  bool bad = false;
  for (uint32_t r = by * ty + tyi; r < rows; r += gy * ty) {
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

template <bool WRITE_W>
__global__ __launch_bounds__(kSweepTX * kSweepTYMax) void k_sweep_comp(
    Geo g, Sweep s, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status) {
  const uint32_t lb = xcd_block(blockIdx.x + gridDim.x * blockIdx.y,
                                gridDim.x * gridDim.y);
  sweep_comp_wg<WRITE_W>(g, s, x, W, codes, status, lb % gridDim.x,
                         lb / gridDim.x, gridDim.y, threadIdx.x, threadIdx.y,
                         blockDim.y);
}

/* Decompression: bins >= 1 reconstruct pred + (bin - R) * 2e_l with the
 * same two roundings as the compressor.  Bin 0 (unpredictable) is skipped:
 * its exact value was scattered into W before the sweeps. */
/* Workgroup (bx, by) of a sweep's gx x gy grid of ty-row tiles; this lane
 * is target tx of row tyi of the tile. */
__device__ __forceinline__ void sweep_decomp_wg(
    const Geo& g, const Sweep& s, float* W, const uint16_t* __restrict__ codes,
    uint32_t bx, uint32_t by, uint32_t gy, uint32_t tx, uint32_t tyi,
    uint32_t ty) {
  const uint32_t i2 = bx * kSweepTX + tx;
  if (i2 >= s.cnt[2]) return;
  const uint32_t rows = s.cnt[0] * s.cnt[1];
  const uint32_t sk = g.st[s.k];
  const uint32_t nk = g.n[s.k];
  for (uint32_t r = by * ty + tyi; r < rows; r += gy * ty) {
    SweepPoint sp = sweep_point(g, s, r, i2);
    const int32_t code = codes[sp.pos];
    if (code == 0) continue;
    float pred = predict_at(W, sp.idx, sp.pk, sk, nk, s.h, s.cubic);
    W[sp.idx] = dequantize_bin(pred, code, s.twoeb);
  }
}

__global__ __launch_bounds__(kSweepTX * kSweepTYMax) void k_sweep_decomp(
    Geo g, Sweep s, float* W, const uint16_t* __restrict__ codes) {
  const uint32_t lb = xcd_block(blockIdx.x + gridDim.x * blockIdx.y,
                                gridDim.x * gridDim.y);
  sweep_decomp_wg(g, s, W, codes, lb % gridDim.x, lb / gridDim.x, gridDim.y,
                  threadIdx.x, threadIdx.y, blockDim.y);
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
  QOZ_LAUNCH(k_unpred_scatter, dim3((uint32_t)blocks), dim3(256), 0,
                     s, g, st, upos, vals, n_unpred, n_codes, W, status);
}

/* ---- level-1 row kernels ------------------------------------------------
 * The sweep along the contiguous dimension (targets at odd positions of a
 * row) reads only even positions of the same row, so it is fused with the
 * sweep just before it in the level's order (its targets sit at the even
 * positions of rows that are odd along that sweep's dimension, and are
 * predicted from neighbour rows).  A workgroup takes several rows; each
 * lane takes 8-point spans.  Phase 1 computes the even positions (sweep A,
 * or the known values) into LDS, phase 2 predicts and quantizes the odd
 * positions (sweep B).  Every target is computed exactly as the per-sweep
 * kernels compute it; only the schedule and the memory access change.
 * Rows are the (p0, p1) pairs of the row set (steps 1 or 2). */
constexpr uint32_t kRowThreads = 256;
constexpr uint32_t kSpan = 8;

__device__ __forceinline__ uint64_t stream_pos(const Sweep& s, uint32_t p0,
                                               uint32_t p1, uint32_t p2) {
  const uint32_t i0 = (p0 - s.start[0]) >> (s.step[0] >> 1);
  const uint32_t i1 = (p1 - s.start[1]) >> (s.step[1] >> 1);
  const uint32_t i2 = (p2 - s.start[2]) >> (s.step[2] >> 1);
  return s.code_off + ((uint64_t)i0 * s.cnt[1] + i1) * s.cnt[2] + i2;
}

/* a 4-byte-aligned 16-byte load */
struct __attribute__((aligned(4))) F4 {
  float x, y, z, w;
};

/* points p .. p + kSpan - 1 of a row (zero past n) */
__device__ __forceinline__ void load_span(const float* __restrict__ r,
                                          uint32_t p, uint32_t n, float* v) {
  if (p + kSpan <= n) {
    const F4 a = *reinterpret_cast<const F4*>(r + p);
    const F4 b = *reinterpret_cast<const F4*>(r + p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (uint32_t k = 0; k < kSpan; ++k) v[k] = p + k < n ? r[p + k] : 0.0f;
  }
}

/* the n (<= 4) bins of a span at pos; one 8-byte access when vec and the
 * span is full */
__device__ __forceinline__ void load_bins4(const uint16_t* __restrict__ c,
                                           uint64_t pos, bool vec,
                                           uint32_t n, int32_t* b) {
  if (vec && n == 4) {
    const uint2 v = *reinterpret_cast<const uint2*>(c + pos);
    b[0] = (int32_t)(v.x & 0xffffu);
    b[1] = (int32_t)(v.x >> 16);
    b[2] = (int32_t)(v.y & 0xffffu);
    b[3] = (int32_t)(v.y >> 16);
  } else {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) b[k] = k < n ? (int32_t)c[pos + k] : 0;
  }
}

__device__ __forceinline__ void store_bins4(uint16_t* __restrict__ c,
                                            uint64_t pos, bool vec,
                                            uint32_t n, const int32_t* b) {
  if (vec && n == 4) {
    *reinterpret_cast<uint2*>(c + pos) =
        make_uint2((uint32_t)b[0] | ((uint32_t)b[1] << 16),
                   (uint32_t)b[2] | ((uint32_t)b[3] << 16));
  } else {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
      if (k < n) c[pos + k] = (uint16_t)b[k];
  }
}

struct RowCtx {
  uint32_t p0, p1, row, pa;
  bool hasA;
};

/* item it of a workgroup: row it / spans, span it mod spans */
struct RowItems {
  uint32_t spans;
  FastDiv fs, fr;
  __device__ __forceinline__ RowItems(uint32_t sp, uint32_t items,
                                      uint32_t rows, uint32_t rcnt1)
      : spans(sp), fs(sp, items), fr(rcnt1, rows) {}
};

__device__ __forceinline__ RowCtx row_ctx(const Geo& g, const RowJob& rj,
                                          const FastDiv& fr, uint32_t r) {
  RowCtx c;
  const uint32_t i0 = fr.div(r);
  const uint32_t i1 = r - i0 * rj.rcnt[1];
  c.p0 = i0 * rj.rstep[0];
  c.p1 = i1 * rj.rstep[1];
  c.row = c.p0 * g.st[0] + c.p1 * g.st[1];
  c.pa = rj.a == 0 ? c.p0 : c.p1;
  c.hasA = rj.a >= 0 && (c.pa & 1u);
  return c;
}

/* Sweep-A predictions of the even points of span [p, p + kSpan): the
 * neighbour rows at -3, -1, +1, +3 along a (present ones only). */
__device__ __forceinline__ void predict_span_A(const Geo& g, const RowJob& rj,
                                               const float* W, const RowCtx& c,
                                               uint32_t p, float* pred) {
  const uint32_t sa = g.st[rj.a], na = g.n[rj.a], n2 = g.n[2];
  const bool ha = c.pa >= 3, hc = c.pa + 1 < na, hd = c.pa + 3 < na;
  const bool cub = rj.A.cubic != 0;
  /* the points each rule reads (see interp_mid); the rest stay unread */
  const bool la = ha && (cub || !hc), ld = hd && cub;
  float vb[kSpan], vc[kSpan], va[kSpan], vd[kSpan];
  load_span(W + c.row - sa, p, n2, vb);
  if (hc) load_span(W + c.row + sa, p, n2, vc);
  if (la) load_span(W + c.row - 3 * sa, p, n2, va);
  if (ld) load_span(W + c.row + 3 * sa, p, n2, vd);
#pragma unroll
  for (uint32_t k = 0; k < kSpan / 2; ++k)
    pred[k] = interp_mid(rj.A.cubic, la ? va[2 * k] : 0.0f, vb[2 * k],
                         hc ? vc[2 * k] : 0.0f, ld ? vd[2 * k] : 0.0f, ha, hc,
                         hd);
}

/* Workgroup blk of a fused level-1 row pair; E is the LDS row buffer. */
template <bool WRITE_W>
__device__ __forceinline__ void row_comp_wg(
    const Geo& g, const RowJob& rj, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status, uint32_t blk, float* E) {
  /* per row: E[t + 1] = value at 2t */
  const uint32_t n2 = g.n[2], ne = (n2 + 1) / 2, es = ne + 3;
  const uint32_t spans = (n2 + kSpan - 1) / kSpan;
  const uint32_t rows = rj.rcnt[0] * rj.rcnt[1];
  const uint32_t r0 = blk * rj.rows_per_wg;
  const uint32_t items = rj.rows_per_wg * spans;
  const RowItems ri(spans, items, rows, rj.rcnt[1]);
  /* one item per lane: the span's x values stay in registers between the
   * phases */
  const bool one = items <= kRowThreads;
  float xv[kSpan];
  bool bad = false;
  for (uint32_t it = threadIdx.x; it < items; it += kRowThreads) {
    const uint32_t rl = ri.fs.div(it), u = it - rl * spans;
    if (r0 + rl >= rows) break;
    const RowCtx c = row_ctx(g, rj, ri.fr, r0 + rl);
    const uint32_t p = u * kSpan;
    float* Er = E + rl * es;
    if (c.hasA || one) load_span(x + c.row, p, n2, xv);
    if (c.hasA) {
      float pred[kSpan / 2];
      predict_span_A(g, rj, W, c, p, pred);
      const uint64_t pos = stream_pos(rj.A, c.p0, c.p1, p);
      const uint32_t nA = p < n2 ? (n2 - p + 1) / 2 : 0u;
      int32_t bins[kSpan / 2];
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k) {
        bins[k] = 0;
        if (k >= nA) continue;
        float e;
        bins[k] =
            quantize_bin(xv[2 * k], pred[k], rj.A.inv, rj.A.twoeb, rj.A.eb, &e);
        bad |= !isfinite(xv[2 * k]);
        Er[p / 2 + k + 1] = e;
      }
      store_bins4(codes, pos, rj.vecA, nA < 4 ? nA : 4u, bins);
    } else {
      float wv[kSpan];
      load_span(W + c.row, p, n2, wv);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k)
        if (p + 2 * k < n2) Er[p / 2 + k + 1] = wv[2 * k];
    }
  }
  __syncthreads();
  for (uint32_t it = threadIdx.x; it < items; it += kRowThreads) {
    const uint32_t rl = ri.fs.div(it), u = it - rl * spans;
    if (r0 + rl >= rows) break;
    const RowCtx c = row_ctx(g, rj, ri.fr, r0 + rl);
    const uint32_t p = u * kSpan;
    const float* Er = E + rl * es;
    float out[kSpan];
    if (!one) load_span(x + c.row, p, n2, xv);
    const uint64_t pos = stream_pos(rj.B, c.p0, c.p1, p + 1);
    const uint32_t nB = p + 1 < n2 ? (n2 - p) / 2 : 0u;
    int32_t bins[kSpan / 2];
#pragma unroll
    for (uint32_t k = 0; k < kSpan / 2; ++k) {
      const uint32_t t = p / 2 + k, q = 2 * t + 1;
      out[2 * k] = Er[t + 1];
      out[2 * k + 1] = 0.0f;
      bins[k] = 0;
      if (q >= n2) continue;
      const bool ha = t >= 1, hc = q + 1 < n2, hd = q + 3 < n2;
      const float pred =
          interp_mid(rj.B.cubic, ha ? Er[t] : 0.0f, Er[t + 1],
                     hc ? Er[t + 2] : 0.0f, hd ? Er[t + 3] : 0.0f, ha, hc, hd);
      float rec;
      bins[k] =
          quantize_bin(xv[2 * k + 1], pred, rj.B.inv, rj.B.twoeb, rj.B.eb, &rec);
      bad |= !isfinite(xv[2 * k + 1]);
      out[2 * k + 1] = rec;
    }
    store_bins4(codes, pos, rj.vecB, nB < 4 ? nB : 4u, bins);
    if (WRITE_W) {
      float* wr = W + c.row;
      if (p + kSpan <= n2) {
        *reinterpret_cast<F4*>(wr + p) = F4{out[0], out[1], out[2], out[3]};
        *reinterpret_cast<F4*>(wr + p + 4) = F4{out[4], out[5], out[6], out[7]};
      } else {
        for (uint32_t k = 0; k < kSpan && p + k < n2; ++k) wr[p + k] = out[k];
      }
    }
  }
  if (bad) atomicOr(status, kStNonFinite);
}

template <bool WRITE_W>
__global__ __launch_bounds__(kRowThreads) void k_row_comp(
    Geo g, RowJob rj, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status) {
  extern __shared__ float E[];
  row_comp_wg<WRITE_W>(g, rj, x, W, codes, status, blockIdx.x, E);
}

/* Decompression: bin 0 keeps the exact value already scattered into W.
 * The single-stream kernel keeps its own copy of the body of row_decomp_wg
 * below: calling the shared inline body compiled to a schedule that ran
 * 6 % slower at 512^3. */
__global__ __launch_bounds__(kRowThreads) void k_row_decomp(
    Geo g, RowJob rj, float* W, const uint16_t* __restrict__ codes) {
  extern __shared__ float E[];
  const uint32_t n2 = g.n[2], ne = (n2 + 1) / 2, es = ne + 3;
  const uint32_t spans = (n2 + kSpan - 1) / kSpan;
  const uint32_t rows = rj.rcnt[0] * rj.rcnt[1];
  const uint32_t r0 = blockIdx.x * rj.rows_per_wg;
  const uint32_t items = rj.rows_per_wg * spans;
  const RowItems ri(spans, items, rows, rj.rcnt[1]);
  for (uint32_t it = threadIdx.x; it < items; it += kRowThreads) {
    const uint32_t rl = ri.fs.div(it), u = it - rl * spans;
    if (r0 + rl >= rows) break;
    const RowCtx c = row_ctx(g, rj, ri.fr, r0 + rl);
    const uint32_t p = u * kSpan;
    float* Er = E + rl * es;
    if (c.hasA) {
      const uint64_t pos = stream_pos(rj.A, c.p0, c.p1, p);
      const uint32_t nA = p < n2 ? (n2 - p + 1) / 2 : 0u;
      int32_t bins[kSpan / 2];
      load_bins4(codes, pos, rj.vecA, nA < 4 ? nA : 4u, bins);
      float pred[kSpan / 2];
      predict_span_A(g, rj, W, c, p, pred);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k) {
        if (k >= nA) break;
        const int32_t code = bins[k];
        Er[p / 2 + k + 1] = code ? dequantize_bin(pred[k], code, rj.A.twoeb)
                                 : W[c.row + p + 2 * k];
      }
    } else {
      float wv[kSpan];
      load_span(W + c.row, p, n2, wv);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k)
        if (p + 2 * k < n2) Er[p / 2 + k + 1] = wv[2 * k];
    }
  }
  __syncthreads();
  for (uint32_t it = threadIdx.x; it < items; it += kRowThreads) {
    const uint32_t rl = ri.fs.div(it), u = it - rl * spans;
    if (r0 + rl >= rows) break;
    const RowCtx c = row_ctx(g, rj, ri.fr, r0 + rl);
    const uint32_t p = u * kSpan;
    const float* Er = E + rl * es;
    float out[kSpan];
    const uint64_t pos = stream_pos(rj.B, c.p0, c.p1, p + 1);
    const uint32_t nB = p + 1 < n2 ? (n2 - p) / 2 : 0u;
    int32_t bins[kSpan / 2];
    load_bins4(codes, pos, rj.vecB, nB < 4 ? nB : 4u, bins);
#pragma unroll
    for (uint32_t k = 0; k < kSpan / 2; ++k) {
      const uint32_t t = p / 2 + k, q = 2 * t + 1;
      out[2 * k] = Er[t + 1];
      out[2 * k + 1] = 0.0f;
      if (q >= n2) continue;
      const int32_t code = bins[k];
      if (code) {
        const bool ha = t >= 1, hc = q + 1 < n2, hd = q + 3 < n2;
        const float pred = interp_mid(rj.B.cubic, ha ? Er[t] : 0.0f, Er[t + 1],
                                      hc ? Er[t + 2] : 0.0f,
                                      hd ? Er[t + 3] : 0.0f, ha, hc, hd);
        out[2 * k + 1] = dequantize_bin(pred, code, rj.B.twoeb);
      } else {
        out[2 * k + 1] = W[c.row + q];
      }
    }
    float* wr = W + c.row;
    if (p + kSpan <= n2) {
      *reinterpret_cast<F4*>(wr + p) = F4{out[0], out[1], out[2], out[3]};
      *reinterpret_cast<F4*>(wr + p + 4) = F4{out[4], out[5], out[6], out[7]};
    } else {
      for (uint32_t k = 0; k < kSpan && p + k < n2; ++k) wr[p + k] = out[k];
    }
  }
}

/* The same for workgroup wg of a queued job (kRowThreads lanes, E its
 * LDS rows). */
__device__ __forceinline__ void row_decomp_wg(
    const Geo& g, const RowJob& rj, float* W,
    const uint16_t* __restrict__ codes, uint32_t wg, float* E) {
  const uint32_t n2 = g.n[2], ne = (n2 + 1) / 2, es = ne + 3;
  const uint32_t spans = (n2 + kSpan - 1) / kSpan;
  const uint32_t rows = rj.rcnt[0] * rj.rcnt[1];
  const uint32_t r0 = wg * rj.rows_per_wg;
  const uint32_t items = rj.rows_per_wg * spans;
  const RowItems ri(spans, items, rows, rj.rcnt[1]);
  for (uint32_t it = threadIdx.x; it < items; it += kRowThreads) {
    const uint32_t rl = ri.fs.div(it), u = it - rl * spans;
    if (r0 + rl >= rows) break;
    const RowCtx c = row_ctx(g, rj, ri.fr, r0 + rl);
    const uint32_t p = u * kSpan;
    float* Er = E + rl * es;
    if (c.hasA) {
      const uint64_t pos = stream_pos(rj.A, c.p0, c.p1, p);
      const uint32_t nA = p < n2 ? (n2 - p + 1) / 2 : 0u;
      int32_t bins[kSpan / 2];
      load_bins4(codes, pos, rj.vecA, nA < 4 ? nA : 4u, bins);
      float pred[kSpan / 2];
      predict_span_A(g, rj, W, c, p, pred);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k) {
        if (k >= nA) break;
        const int32_t code = bins[k];
        Er[p / 2 + k + 1] = code ? dequantize_bin(pred[k], code, rj.A.twoeb)
                                 : W[c.row + p + 2 * k];
      }
    } else {
      float wv[kSpan];
      load_span(W + c.row, p, n2, wv);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k)
        if (p + 2 * k < n2) Er[p / 2 + k + 1] = wv[2 * k];
    }
  }
  __syncthreads();
  for (uint32_t it = threadIdx.x; it < items; it += kRowThreads) {
    const uint32_t rl = ri.fs.div(it), u = it - rl * spans;
    if (r0 + rl >= rows) break;
    const RowCtx c = row_ctx(g, rj, ri.fr, r0 + rl);
    const uint32_t p = u * kSpan;
    const float* Er = E + rl * es;
    float out[kSpan];
    const uint64_t pos = stream_pos(rj.B, c.p0, c.p1, p + 1);
    const uint32_t nB = p + 1 < n2 ? (n2 - p) / 2 : 0u;
    int32_t bins[kSpan / 2];
    load_bins4(codes, pos, rj.vecB, nB < 4 ? nB : 4u, bins);
#pragma unroll
    for (uint32_t k = 0; k < kSpan / 2; ++k) {
      const uint32_t t = p / 2 + k, q = 2 * t + 1;
      out[2 * k] = Er[t + 1];
      out[2 * k + 1] = 0.0f;
      if (q >= n2) continue;
      const int32_t code = bins[k];
      if (code) {
        const bool ha = t >= 1, hc = q + 1 < n2, hd = q + 3 < n2;
        const float pred = interp_mid(rj.B.cubic, ha ? Er[t] : 0.0f, Er[t + 1],
                                      hc ? Er[t + 2] : 0.0f,
                                      hd ? Er[t + 3] : 0.0f, ha, hc, hd);
        out[2 * k + 1] = dequantize_bin(pred, code, rj.B.twoeb);
      } else {
        out[2 * k + 1] = W[c.row + q];
      }
    }
    float* wr = W + c.row;
    if (p + kSpan <= n2) {
      *reinterpret_cast<F4*>(wr + p) = F4{out[0], out[1], out[2], out[3]};
      *reinterpret_cast<F4*>(wr + p + 4) = F4{out[4], out[5], out[6], out[7]};
    } else {
      for (uint32_t k = 0; k < kSpan && p + k < n2; ++k) wr[p + k] = out[k];
    }
  }
}


static uint32_t row_blocks(const Geo& g, RowJob* rj, size_t* lds) {
  const uint32_t rows = rj->rcnt[0] * rj->rcnt[1];
  const uint32_t spans = (g.n[2] + kSpan - 1) / kSpan;
  rj->rows_per_wg = spans >= kRowThreads ? 1u : kRowThreads / spans;
  if (rj->rows_per_wg > rows) rj->rows_per_wg = rows;
  *lds = 4 * (size_t)rj->rows_per_wg * ((g.n[2] + 1) / 2 + 3);
  return (rows + rj->rows_per_wg - 1) / rj->rows_per_wg;
}

void launch_row_comp(const Geo& g, const RowJob& rj_in, const float* x,
                     float* W, uint16_t* codes, bool write_w,
                     uint32_t* status, hipStream_t s) {
  if (!rj_in.rcnt[0] || !rj_in.rcnt[1]) return;
  RowJob rj = rj_in;
  size_t lds;
  const uint32_t blocks = row_blocks(g, &rj, &lds);
  if (write_w)
    QOZ_LAUNCH(k_row_comp<true>, dim3(blocks), dim3(kRowThreads), lds,
                       s, g, rj, x, W, codes, status);
  else
    QOZ_LAUNCH(k_row_comp<false>, dim3(blocks), dim3(kRowThreads),
                       lds, s, g, rj, x, W, codes, status);
}

void launch_row_decomp(const Geo& g, const RowJob& rj_in, float* W,
                       const uint16_t* codes, hipStream_t s) {
  if (!rj_in.rcnt[0] || !rj_in.rcnt[1]) return;
  RowJob rj = rj_in;
  size_t lds;
  const uint32_t blocks = row_blocks(g, &rj, &lds);
  QOZ_LAUNCH(k_row_decomp, dim3(blocks), dim3(kRowThreads), lds, s, g,
                     rj, W, codes);
}

/* One round of a batch's inverse sweeps: each job is one sweep (64 x 4
 * lane tiles) or one fused level-1 row pair of a different field, so the
 * jobs of a round are independent of each other. */
__global__ __launch_bounds__(kRowThreads) void k_sweep_round_q(
    const SweepJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  extern __shared__ float E[];
  const uint32_t gid = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t j = find_job(wg0, n_jobs, gid);
  const SweepJob& a = jobs[j];
  const uint32_t lid = gid - wg0[j];
  /* the record's pointers made global: flat accesses would also count
   * against the LDS counter */
  float* const W = (float*)gptr(a.W);
  const uint16_t* const codes = (const uint16_t*)gptr(a.codes);
  if (a.rows)
    row_decomp_wg(a.g, a.rj, W, codes, lid, E);
  else
    sweep_decomp_wg(a.g, a.s, W, codes, lid % a.gx, lid / a.gx, a.gy,
                    threadIdx.x % kSweepTX, threadIdx.x / kSweepTX,
                    kRowThreads / kSweepTX);
}

/* One round of a batch's compression sweeps, as k_sweep_round_q for the
 * inverse sweeps. */
__global__ __launch_bounds__(kRowThreads) void k_sweep_round_comp_q(
    const CompJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  extern __shared__ float E[];
  const uint32_t gid = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t j = find_job(wg0, n_jobs, gid);
  const CompJob& a = jobs[j];
  const uint32_t lid = gid - wg0[j];
  /* the record's pointers made global (not flat) */
  const float* const x = (const float*)gptr(a.x);
  float* const W = (float*)gptr(a.W);
  uint16_t* const codes = (uint16_t*)gptr(a.codes);
  uint32_t* const status = (uint32_t*)gptr(a.status);
  if (a.rows) {
    if (a.write_w)
      row_comp_wg<true>(a.g, a.rj, x, W, codes, status, lid, E);
    else
      row_comp_wg<false>(a.g, a.rj, x, W, codes, status, lid, E);
  } else {
    const uint32_t tx = threadIdx.x % kSweepTX, ty = threadIdx.x / kSweepTX;
    if (a.write_w)
      sweep_comp_wg<true>(a.g, a.s, x, W, codes, status, lid % a.gx,
                          lid / a.gx, a.gy, tx, ty, kRowThreads / kSweepTX);
    else
      sweep_comp_wg<false>(a.g, a.s, x, W, codes, status, lid % a.gx,
                           lid / a.gx, a.gy, tx, ty, kRowThreads / kSweepTX);
  }
}

/* The anchors of many fields in one launch. */
__global__ __launch_bounds__(256) void k_anchor_q(
    const AnchorJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  const uint32_t j = find_job(wg0, n_jobs, blockIdx.x);
  const AnchorJob& a = jobs[j];
  const uint32_t t = (blockIdx.x - wg0[j]) * blockDim.x + threadIdx.x;
  const uint32_t total = a.na[0] * a.na[1] * a.na[2];
  if (t >= total) return;
  const uint32_t a2 = t % a.na[2];
  const uint32_t r = t / a.na[2];
  const uint32_t a1 = r % a.na[1];
  const uint32_t a0 = r / a.na[1];
  const uint32_t idx = a0 * a.stride * a.g.st[0] + a1 * a.stride * a.g.st[1] +
                       a2 * a.stride;
  const float v = a.x[idx];
  a.W[idx] = v;
  a.out[t] = v;
  if (!isfinite(v)) atomicOr(a.status, kStNonFinite);
}

/* Copies (or zero fills) of a list, one workgroup per entry: 16-byte
 * accesses when both ends and the size allow, else 8-byte ones, else
 * bytes. */
__global__ __launch_bounds__(256) void k_copy_list(
    const DevCopy* __restrict__ list) {
  const DevCopy c = list[blockIdx.x];
  const uint64_t al = (uintptr_t)c.src | (uintptr_t)c.dst | c.bytes;
  if ((al & 15) == 0) {
    uint4* d = (uint4*)c.dst;
    const uint4* s = (const uint4*)c.src;
    for (uint64_t i = threadIdx.x; i < c.bytes / 16; i += blockDim.x)
      d[i] = s ? s[i] : make_uint4(0, 0, 0, 0);
  } else if ((al & 7) == 0) {
    uint2* d = (uint2*)c.dst;
    const uint2* s = (const uint2*)c.src;
    for (uint64_t i = threadIdx.x; i < c.bytes / 8; i += blockDim.x)
      d[i] = s ? s[i] : make_uint2(0, 0);
  } else {
    uint8_t* d = (uint8_t*)c.dst;
    const uint8_t* s = (const uint8_t*)c.src;
    for (uint64_t i = threadIdx.x; i < c.bytes; i += blockDim.x)
      d[i] = s ? s[i] : (uint8_t)0;
  }
}

uint32_t anchor_job_workgroups(const AnchorJob& j) {
  return (j.na[0] * j.na[1] * j.na[2] + 255) / 256;
}

void launch_anchor_q(const AnchorJob* jobs, const uint32_t* wg0,
                     uint32_t n_jobs, uint32_t total_wg, hipStream_t s) {
  if (!total_wg) return;
  QOZ_LAUNCH(k_anchor_q, dim3(total_wg), dim3(256), 0, s, jobs, wg0,
                     n_jobs);
}

void launch_copy_list(const DevCopy* list, uint32_t n, hipStream_t s) {
  if (!n) return;
  QOZ_LAUNCH(k_copy_list, dim3(n), dim3(256), 0, s, list);
}

static_assert(kRowThreads % kSweepTX == 0, "queued sweep tiles");

/* Launch shape of a sweep: x covers 64 consecutive targets of a row, y
 * covers rows (flattened over the two outer sub-grid dimensions), ty rows
 * per workgroup and rpt rows per lane (a grid-stride loop), the grid's y
 * extent capped at 65535. */
static dim3 sweep_grid_dim(const Sweep& sw, SweepTile t) {
  uint32_t gx = (sw.cnt[2] + kSweepTX - 1) / kSweepTX;
  uint64_t rows = (uint64_t)sw.cnt[0] * sw.cnt[1];
  uint64_t per = (uint64_t)t.ty * t.rpt;
  uint64_t gy = (rows + per - 1) / per;
  if (gy > kMaxGridY) gy = kMaxGridY;
  if (gy < 1) gy = 1;
  return dim3(gx, (uint32_t)gy);
}

bool sweep_tile_ok(SweepTile t) {
  return t.ty >= 1 && t.ty <= kSweepTYMax && (t.ty & (t.ty - 1)) == 0 &&
         t.rpt >= 1 && t.rpt <= 64;
}

void launch_sweep_comp(const Geo& g, const Sweep& sw, const float* x,
                       float* W, uint16_t* codes, bool write_w,
                       uint32_t* status, hipStream_t s, SweepTile t) {
  if (sw.count == 0) return;
  if (!sweep_tile_ok(t)) t = SweepTile();
  dim3 grid = sweep_grid_dim(sw, t), block(kSweepTX, t.ty);
  if (write_w)
    QOZ_LAUNCH(k_sweep_comp<true>, grid, block, 0, s, g, sw, x, W,
                       codes, status);
  else
    QOZ_LAUNCH(k_sweep_comp<false>, grid, block, 0, s, g, sw, x, W,
                       codes, status);
}

uint32_t sweep_job_prepare(SweepJob* j, size_t* lds) {
  *lds = 0;
  if (j->rows) {
    if (!j->rj.rcnt[0] || !j->rj.rcnt[1]) return 0;
    return row_blocks(j->g, &j->rj, lds);
  }
  if (j->s.count == 0) return 0;
  SweepTile t;
  t.ty = kRowThreads / kSweepTX;
  t.rpt = 1;
  const dim3 grid = sweep_grid_dim(j->s, t);
  j->gx = grid.x;
  j->gy = grid.y;
  return grid.x * grid.y;
}

uint32_t comp_job_prepare(CompJob* j, size_t* lds) {
  *lds = 0;
  if (j->rows) {
    if (!j->rj.rcnt[0] || !j->rj.rcnt[1]) return 0;
    return row_blocks(j->g, &j->rj, lds);
  }
  if (j->s.count == 0) return 0;
  SweepTile t;
  t.ty = kRowThreads / kSweepTX;
  t.rpt = 1;
  const dim3 grid = sweep_grid_dim(j->s, t);
  j->gx = grid.x;
  j->gy = grid.y;
  return grid.x * grid.y;
}

void launch_sweep_round_comp_q(const CompJob* jobs, const uint32_t* wg0,
                               uint32_t n_jobs, uint32_t total_wg, size_t lds,
                               hipStream_t s) {
  if (!total_wg) return;
  QOZ_LAUNCH(k_sweep_round_comp_q, dim3(total_wg), dim3(kRowThreads),
                     lds, s, jobs, wg0, n_jobs);
}

void launch_sweep_round_q(const SweepJob* jobs, const uint32_t* wg0,
                          uint32_t n_jobs, uint32_t total_wg, size_t lds,
                          hipStream_t s) {
  if (!total_wg) return;
  QOZ_LAUNCH(k_sweep_round_q, dim3(total_wg), dim3(kRowThreads), lds,
                     s, jobs, wg0, n_jobs);
}

void launch_sweep_decomp(const Geo& g, const Sweep& sw, float* W,
                         const uint16_t* codes, hipStream_t s, SweepTile t) {
  if (sw.count == 0) return;
  if (!sweep_tile_ok(t)) t = SweepTile();
  dim3 grid = sweep_grid_dim(sw, t), block(kSweepTX, t.ty);
  QOZ_LAUNCH(k_sweep_decomp, grid, block, 0, s, g, sw, W, codes);
}

}  // namespace qoz
