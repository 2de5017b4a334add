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
 * The sweep along the contiguous dimension (B: targets at odd points of a
 * row) reads only even points of the same row, so it is fused with the
 * sweep just before it in the level's order (A: its targets sit at the
 * even points of rows odd along a, predicted from the rows at -3 .. +3
 * along a) and, when the level's order is (f, a, 2), with the first sweep
 * too (F: targets at the even points of rows odd along f and even along a,
 * predicted from rows of the coarser levels).  A workgroup takes a tile of
 * rows along a (with two rows before and three after it, whose F values
 * it computes again, so that the A rows find their neighbours in LDS) by
 * up to 512 points; each lane takes 8-point spans.  Phase 1 computes the
 * even points of the even rows (sweep F, or the known values) into LDS,
 * phase 2 those of the odd rows (sweep A), phase 3 the odd points of the
 * tile's rows (sweep B).  Every target is computed exactly as the
 * per-sweep kernels compute it and coded by the one tile that owns it;
 * only the schedule and the memory access change. */
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
    /* streamed past the caches: the bins are read again only by the next
     * kernel, and the lines they would take are the rows' */
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    u32x2 w;
    w.x = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
    w.y = (uint32_t)b[2] | ((uint32_t)b[3] << 16);
    __builtin_nontemporal_store(w, reinterpret_cast<u32x2*>(c + pos));
  } else {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
      if (k < n) c[pos + k] = (uint16_t)b[k];
  }
}

/* A tile of the level-1 pass: T rows along the tile dimension td (A's
 * dimension when A exists, else dimension 1) at row index io of the other
 * dimension, by S points of the contiguous dimension from P0.  E holds the
 * values at the even points P0 - 2 .. P0 + S + 2 of the rows it0 - lo ..
 * it0 + T + hi - 1 (lo = 2, hi = 3 when A exists: the neighbour rows of
 * the tile's A rows; else the tile's rows only).  Entry e of a row (point
 * P0 + 2 (e - 1)) sits at index e + 3 of the row's es = S / 2 + 8 floats:
 * the four even points of a span are one aligned 16-byte word. */
struct L1Tile {
  uint32_t td, it0, io, P0, lo, nr, es, nt;
};

__device__ __forceinline__ L1Tile l1_tile(const RowJob& rj, uint32_t blk) {
  L1Tile t;
  t.td = rj.a >= 0 ? (uint32_t)rj.a : 1u;
  const uint32_t s2 = blk % rj.tiles2, r = blk / rj.tiles2;
  t.it0 = (r % rj.tilesT) * rj.T;
  t.io = r / rj.tilesT;
  t.P0 = s2 * rj.S;
  t.lo = rj.a >= 0 ? 2u : 0u;
  t.nr = rj.T + (rj.a >= 0 ? 5u : 0u);
  t.es = rj.S / 2 + 8;
  t.nt = rj.rcnt[t.td];
  return t;
}

/* E row l of a tile: its coordinates and flat offset; ok: inside the row
 * set; own: one of the tile's rows (its targets are this tile's to code). */
struct L1Row {
  uint32_t p0, p1, row, pt;
  bool ok, own;
};

__device__ __forceinline__ L1Row l1_row(const Geo& g, const RowJob& rj,
                                        const L1Tile& t, uint32_t l) {
  L1Row r;
  const int32_t it = (int32_t)t.it0 - (int32_t)t.lo + (int32_t)l;
  r.ok = it >= 0 && (uint32_t)it < t.nt;
  r.own = r.ok && l >= t.lo && l < t.lo + rj.T;
  r.pt = (r.ok ? (uint32_t)it : 0u) * rj.rstep[t.td];
  const uint32_t po = t.io * rj.rstep[1 - t.td];
  r.p0 = t.td == 0 ? r.pt : po;
  r.p1 = t.td == 0 ? po : r.pt;
  r.row = r.p0 * g.st[0] + r.p1 * g.st[1];
  return r;
}

/* Predictions of the even points of span [p, p + kSpan) of the row at
 * offset row (coordinate pk along the swept dimension: stride sk, extent
 * nk) from the rows at -3, -1, +1, +3 along it in W (present ones only). */
__device__ __forceinline__ void predict_span(const float* W, uint32_t row,
                                             uint32_t pk, uint32_t sk,
                                             uint32_t nk, uint32_t cubic,
                                             uint32_t p, uint32_t n2,
                                             float* pred) {
  const bool ha = pk >= 3, hc = pk + 1 < nk, hd = pk + 3 < nk;
  const bool cub = cubic != 0;
  /* the points each rule reads (see interp_mid); the rest stay unread */
  const bool la = ha && (cub || !hc), ld = hd && cub;
  float vb[kSpan], vc[kSpan], va[kSpan], vd[kSpan];
  load_span(W + row - sk, p, n2, vb);
  if (hc) load_span(W + row + sk, p, n2, vc);
  if (la) load_span(W + row - 3 * sk, p, n2, va);
  if (ld) load_span(W + row + 3 * sk, p, n2, vd);
#pragma unroll
  for (uint32_t k = 0; k < kSpan / 2; ++k)
    pred[k] = interp_mid(cubic, la ? va[2 * k] : 0.0f, vb[2 * k],
                         hc ? vc[2 * k] : 0.0f, ld ? vd[2 * k] : 0.0f, ha, hc,
                         hd);
}

/* The same along the tile dimension from the tile's E rows l - 3 .. l + 3
 * at the 16-byte word q of each (the entries of one span). */
__device__ __forceinline__ void predict_span_E(const float* E, uint32_t es,
                                               uint32_t l, uint32_t q,
                                               uint32_t pk, uint32_t nk,
                                               uint32_t cubic, float* pred) {
  const bool ha = pk >= 3, hc = pk + 1 < nk, hd = pk + 3 < nk;
  const bool cub = cubic != 0;
  const bool la = ha && (cub || !hc), ld = hd && cub;
  const float4 vb = reinterpret_cast<const float4*>(E + (l - 1) * es)[q];
  float4 va = make_float4(0.0f, 0.0f, 0.0f, 0.0f), vc = va, vd = va;
  if (hc) vc = reinterpret_cast<const float4*>(E + (l + 1) * es)[q];
  if (la) va = reinterpret_cast<const float4*>(E + (l - 3) * es)[q];
  if (ld) vd = reinterpret_cast<const float4*>(E + (l + 3) * es)[q];
  const float a4[4] = {va.x, va.y, va.z, va.w}, b4[4] = {vb.x, vb.y, vb.z, vb.w};
  const float c4[4] = {vc.x, vc.y, vc.z, vc.w}, d4[4] = {vd.x, vd.y, vd.z, vd.w};
#pragma unroll
  for (uint32_t k = 0; k < kSpan / 2; ++k)
    pred[k] = interp_mid(cubic, a4[k], b4[k], c4[k], d4[k], ha, hc, hd);
}

/* The even-point values v of span u into E row Er (word u: entries
 * 4u - 3 .. 4u; the left side span keeps only entry 0, the rest of the
 * word lies before the row; entries past the row's points are never
 * read). */
__device__ __forceinline__ void store_span_E(float* Er, uint32_t u,
                                             const float* v) {
  if (u == 0)
    Er[3] = v[3];
  else
    reinterpret_cast<float4*>(Er)[u] = make_float4(v[0], v[1], v[2], v[3]);
}

/* The entries 4u .. 4u + 6 of E row Er (the even points a phase-3 span's
 * odd points are predicted from). */
__device__ __forceinline__ void load_span_E(const float* Er, uint32_t u,
                                            float* v) {
  const float4 m = reinterpret_cast<const float4*>(Er)[u + 1];
  const float2 h = reinterpret_cast<const float2*>(Er)[2 * u + 4];
  v[0] = Er[4 * u + 3];
  v[1] = m.x; v[2] = m.y; v[3] = m.z; v[4] = m.w;
  v[5] = h.x; v[6] = h.y;
}

/* Phase items: rows of E and spans.  Phases 1 and 2 take the spans from
 * P0 - 8 to P0 + S (the tile's spans and one on each side, whose even
 * points P0 - 2, P0 + S and P0 + S + 2 the odd points of the tile's edge
 * spans are predicted from); phase 3 the tile's spans. */
struct L1Items {
  uint32_t spans, n;
  FastDiv fs;
  __device__ __forceinline__ L1Items(uint32_t sp, uint32_t rows)
      : spans(sp), n(sp * rows), fs(sp, sp * rows) {}
};

/* Workgroup blk of a level-1 pass (compression): sweep F (if fused) into
 * the even rows of E, then sweep A into its odd rows, then sweep B along
 * the rows; E is the LDS tile buffer. */
template <bool WRITE_W>
__device__ __forceinline__ void row_comp_wg(
    const Geo& g, const RowJob& rj, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status, uint32_t blk, float* E) {
  const L1Tile t = l1_tile(rj, blk);
  const uint32_t n2 = g.n[2];
  const bool hasA = rj.a >= 0;
  const uint32_t sp12 = rj.S / kSpan + 2, sp3 = rj.S / kSpan;
  bool bad = false;
  /* phase 1: even rows of E (all of them without A) */
  {
    const uint32_t rows = hasA ? (t.nr + 1) / 2 : rj.T;
    const L1Items ii(sp12, rows);
    for (uint32_t it = threadIdx.x; it < ii.n; it += kRowThreads) {
      const uint32_t rl = ii.fs.div(it), u = it - rl * sp12;
      const uint32_t l = hasA ? 2 * rl : rl;
      const L1Row r = l1_row(g, rj, t, l);
      if (!r.ok || t.P0 + kSpan * u < kSpan) continue;
      const uint32_t p = t.P0 + kSpan * u - kSpan;
      if (p >= n2) continue;
      float* Er = E + l * t.es;
      const bool isF = rj.f >= 0 && (((rj.f == 0 ? r.p0 : r.p1)) & 1u);
      float v[kSpan / 2];
      if (isF) {
        const uint32_t pf = rj.f == 0 ? r.p0 : r.p1;
        float pred[kSpan / 2], xv[kSpan];
        predict_span(W, r.row, pf, g.st[rj.f], g.n[rj.f], rj.F.cubic, p, n2,
                     pred);
        load_span(x + r.row, p, n2, xv);
        const bool coded = r.own && u >= 1 && u <= sp3;
        int32_t bins[kSpan / 2];
#pragma unroll
        for (uint32_t k = 0; k < kSpan / 2; ++k) {
          bins[k] = quantize_bin(xv[2 * k], pred[k], rj.F.inv, rj.F.twoeb,
                                 rj.F.eb, &v[k]);
          if (coded && p + 2 * k < n2) bad |= !isfinite(xv[2 * k]);
        }
        if (coded) {
          const uint32_t nF = (n2 - p + 1) / 2;
          store_bins4(codes, stream_pos(rj.F, r.p0, r.p1, p), rj.vecF,
                      nF < 4 ? nF : 4u, bins);
        }
      } else {
        float wv[kSpan];
        load_span(W + r.row, p, n2, wv);
#pragma unroll
        for (uint32_t k = 0; k < kSpan / 2; ++k) v[k] = wv[2 * k];
      }
      store_span_E(Er, u, v);
    }
  }
  __syncthreads();
  /* phase 2: the tile's A rows (odd along a) from the even rows of E */
  if (hasA) {
    const uint32_t na = g.n[rj.a];
    const L1Items ii(sp12, rj.T / 2);
    for (uint32_t it = threadIdx.x; it < ii.n; it += kRowThreads) {
      const uint32_t rl = ii.fs.div(it), u = it - rl * sp12;
      const uint32_t l = t.lo + 1 + 2 * rl;
      const L1Row r = l1_row(g, rj, t, l);
      if (!r.ok || t.P0 + kSpan * u < kSpan) continue;
      const uint32_t p = t.P0 + kSpan * u - kSpan;
      if (p >= n2) continue;
      float pred[kSpan / 2], xv[kSpan], v[kSpan / 2];
      predict_span_E(E, t.es, l, u, r.pt, na, rj.A.cubic, pred);
      load_span(x + r.row, p, n2, xv);
      const bool coded = u >= 1 && u <= sp3;
      int32_t bins[kSpan / 2];
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k) {
        bins[k] = quantize_bin(xv[2 * k], pred[k], rj.A.inv, rj.A.twoeb,
                               rj.A.eb, &v[k]);
        if (coded && p + 2 * k < n2) bad |= !isfinite(xv[2 * k]);
      }
      if (coded) {
        const uint32_t nA = (n2 - p + 1) / 2;
        store_bins4(codes, stream_pos(rj.A, r.p0, r.p1, p), rj.vecA,
                    nA < 4 ? nA : 4u, bins);
      }
      store_span_E(E + l * t.es, u, v);
    }
    __syncthreads();
  }
  /* phase 3: sweep B along the tile's rows */
  {
    const L1Items ii(sp3, rj.T);
    for (uint32_t it = threadIdx.x; it < ii.n; it += kRowThreads) {
      const uint32_t rl = ii.fs.div(it), u = it - rl * sp3;
      const uint32_t l = t.lo + rl;
      const L1Row r = l1_row(g, rj, t, l);
      const uint32_t p = t.P0 + kSpan * u;
      if (!r.ok || p >= n2) continue;
      const float* Er = E + l * t.es;
      float xv[kSpan], out[kSpan];
      load_span(x + r.row, p, n2, xv);
      const uint64_t pos = stream_pos(rj.B, r.p0, r.p1, p + 1);
      const uint32_t nB = p + 1 < n2 ? (n2 - p) / 2 : 0u;
      int32_t bins[kSpan / 2];
      float ev[7];
      load_span_E(Er, u, ev);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k) {
        const uint32_t q = p + 2 * k + 1;
        out[2 * k] = ev[k + 1];
        out[2 * k + 1] = 0.0f;
        bins[k] = 0;
        if (q >= n2) continue;
        const bool ha = q >= 3, hc = q + 1 < n2, hd = q + 3 < n2;
        const float pred =
            interp_mid(rj.B.cubic, ha ? ev[k] : 0.0f, ev[k + 1],
                       hc ? ev[k + 2] : 0.0f, hd ? ev[k + 3] : 0.0f, ha, hc,
                       hd);
        float rec;
        bins[k] = quantize_bin(xv[2 * k + 1], pred, rj.B.inv, rj.B.twoeb,
                               rj.B.eb, &rec);
        bad |= !isfinite(xv[2 * k + 1]);
        out[2 * k + 1] = rec;
      }
      store_bins4(codes, pos, rj.vecB, nB < 4 ? nB : 4u, bins);
      if (WRITE_W) {
        float* wr = W + r.row;
        if (p + kSpan <= n2) {
          *reinterpret_cast<F4*>(wr + p) = F4{out[0], out[1], out[2], out[3]};
          *reinterpret_cast<F4*>(wr + p + 4) =
              F4{out[4], out[5], out[6], out[7]};
        } else {
          for (uint32_t k = 0; k < kSpan && p + k < n2; ++k) wr[p + k] = out[k];
        }
      }
    }
  }
  if (bad) atomicOr(status, kStNonFinite);
}

template <bool WRITE_W>
__global__ __launch_bounds__(kRowThreads) void k_row_comp(
    Geo g, RowJob rj, const float* __restrict__ x, float* W,
    uint16_t* __restrict__ codes, uint32_t* status) {
  extern __shared__ __align__(16) float E[];
  row_comp_wg<WRITE_W>(g, rj, x, W, codes, status,
                       xcd_block(blockIdx.x, gridDim.x), E);
}

/* Decompression: the same phases; bin 0 keeps the exact value already
 * scattered into W. */
__device__ __forceinline__ void row_decomp_wg(
    const Geo& g, const RowJob& rj, float* W,
    const uint16_t* __restrict__ codes, uint32_t blk, float* E) {
  const L1Tile t = l1_tile(rj, blk);
  const uint32_t n2 = g.n[2];
  const bool hasA = rj.a >= 0;
  const uint32_t sp12 = rj.S / kSpan + 2, sp3 = rj.S / kSpan;
  {
    const uint32_t rows = hasA ? (t.nr + 1) / 2 : rj.T;
    const L1Items ii(sp12, rows);
    for (uint32_t it = threadIdx.x; it < ii.n; it += kRowThreads) {
      const uint32_t rl = ii.fs.div(it), u = it - rl * sp12;
      const uint32_t l = hasA ? 2 * rl : rl;
      const L1Row r = l1_row(g, rj, t, l);
      if (!r.ok || t.P0 + kSpan * u < kSpan) continue;
      const uint32_t p = t.P0 + kSpan * u - kSpan;
      if (p >= n2) continue;
      float* Er = E + l * t.es;
      const bool isF = rj.f >= 0 && (((rj.f == 0 ? r.p0 : r.p1)) & 1u);
      float v[kSpan / 2];
      if (isF) {
        const uint32_t pf = rj.f == 0 ? r.p0 : r.p1;
        float pred[kSpan / 2];
        predict_span(W, r.row, pf, g.st[rj.f], g.n[rj.f], rj.F.cubic, p, n2,
                     pred);
        const uint32_t nF = (n2 - p + 1) / 2;
        int32_t bins[kSpan / 2];
        load_bins4(codes, stream_pos(rj.F, r.p0, r.p1, p), rj.vecF,
                   nF < 4 ? nF : 4u, bins);
        /* bin 0 (and the points past the row): the exact value in W */
#pragma unroll
        for (uint32_t k = 0; k < kSpan / 2; ++k)
          v[k] = bins[k] ? dequantize_bin(pred[k], bins[k], rj.F.twoeb)
                 : p + 2 * k < n2 ? W[r.row + p + 2 * k]
                                  : 0.0f;
      } else {
        float wv[kSpan];
        load_span(W + r.row, p, n2, wv);
#pragma unroll
        for (uint32_t k = 0; k < kSpan / 2; ++k) v[k] = wv[2 * k];
      }
      store_span_E(Er, u, v);
    }
  }
  __syncthreads();
  if (hasA) {
    const uint32_t na = g.n[rj.a];
    const L1Items ii(sp12, rj.T / 2);
    for (uint32_t it = threadIdx.x; it < ii.n; it += kRowThreads) {
      const uint32_t rl = ii.fs.div(it), u = it - rl * sp12;
      const uint32_t l = t.lo + 1 + 2 * rl;
      const L1Row r = l1_row(g, rj, t, l);
      if (!r.ok || t.P0 + kSpan * u < kSpan) continue;
      const uint32_t p = t.P0 + kSpan * u - kSpan;
      if (p >= n2) continue;
      float pred[kSpan / 2], v[kSpan / 2];
      predict_span_E(E, t.es, l, u, r.pt, na, rj.A.cubic, pred);
      const uint32_t nA = (n2 - p + 1) / 2;
      int32_t bins[kSpan / 2];
      load_bins4(codes, stream_pos(rj.A, r.p0, r.p1, p), rj.vecA,
                 nA < 4 ? nA : 4u, bins);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k)
        v[k] = bins[k] ? dequantize_bin(pred[k], bins[k], rj.A.twoeb)
               : p + 2 * k < n2 ? W[r.row + p + 2 * k]
                                : 0.0f;
      store_span_E(E + l * t.es, u, v);
    }
    __syncthreads();
  }
  {
    const L1Items ii(sp3, rj.T);
    for (uint32_t it = threadIdx.x; it < ii.n; it += kRowThreads) {
      const uint32_t rl = ii.fs.div(it), u = it - rl * sp3;
      const uint32_t l = t.lo + rl;
      const L1Row r = l1_row(g, rj, t, l);
      const uint32_t p = t.P0 + kSpan * u;
      if (!r.ok || p >= n2) continue;
      const float* Er = E + l * t.es;
      float out[kSpan];
      const uint64_t pos = stream_pos(rj.B, r.p0, r.p1, p + 1);
      const uint32_t nB = p + 1 < n2 ? (n2 - p) / 2 : 0u;
      int32_t bins[kSpan / 2];
      load_bins4(codes, pos, rj.vecB, nB < 4 ? nB : 4u, bins);
      float ev[7];
      load_span_E(Er, u, ev);
#pragma unroll
      for (uint32_t k = 0; k < kSpan / 2; ++k) {
        const uint32_t q = p + 2 * k + 1;
        out[2 * k] = ev[k + 1];
        out[2 * k + 1] = 0.0f;
        if (q >= n2) continue;
        const int32_t code = bins[k];
        if (code) {
          const bool ha = q >= 3, hc = q + 1 < n2, hd = q + 3 < n2;
          const float pred =
              interp_mid(rj.B.cubic, ha ? ev[k] : 0.0f, ev[k + 1],
                         hc ? ev[k + 2] : 0.0f, hd ? ev[k + 3] : 0.0f, ha, hc,
                         hd);
          out[2 * k + 1] = dequantize_bin(pred, code, rj.B.twoeb);
        } else {
          out[2 * k + 1] = W[r.row + q];
        }
      }
      float* wr = W + r.row;
      if (p + kSpan <= n2) {
        /* the output field, streamed past the caches */
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        f32x4 o0, o1;
        o0.x = out[0]; o0.y = out[1]; o0.z = out[2]; o0.w = out[3];
        o1.x = out[4]; o1.y = out[5]; o1.z = out[6]; o1.w = out[7];
        __builtin_nontemporal_store(o0, reinterpret_cast<f32x4*>(wr + p));
        __builtin_nontemporal_store(o1, reinterpret_cast<f32x4*>(wr + p + 4));
      } else {
        for (uint32_t k = 0; k < kSpan && p + k < n2; ++k) wr[p + k] = out[k];
      }
    }
  }
}

__global__ __launch_bounds__(kRowThreads) void k_row_decomp(
    Geo g, RowJob rj, float* W, const uint16_t* __restrict__ codes) {
  extern __shared__ __align__(16) float E[];
  row_decomp_wg(g, rj, W, codes, xcd_block(blockIdx.x, gridDim.x), E);
}

/* Tile sizes: S points of the contiguous dimension (at most 512), T rows
 * (even, so that a tile's first row is even along a) for about 8 K points
 * per tile; E: T + 5 rows (T without A) of S / 2 + 8 values. */
static uint32_t row_blocks(const Geo& g, RowJob* rj, size_t* lds) {
  const uint32_t n2 = g.n[2];
  const uint32_t S = n2 >= 512 ? 512u : (n2 + kSpan - 1) / kSpan * kSpan;
  uint32_t T = (8192u / S) & ~1u;
  T = T < 2 ? 2u : T > 64 ? 64u : T;
  const uint32_t td = rj->a >= 0 ? (uint32_t)rj->a : 1u;
  const uint32_t nt = rj->rcnt[td], no = rj->rcnt[1 - td];
  if (T > nt + (nt & 1u)) T = nt + (nt & 1u); /* no more than the rows */
  if (T < 2) T = 2;
  rj->S = S;
  rj->T = T;
  rj->tiles2 = (n2 + S - 1) / S;
  rj->tilesT = (nt + T - 1) / T;
  const uint32_t nr = T + (rj->a >= 0 ? 5u : 0u);
  *lds = 4 * (size_t)nr * (S / 2 + 8);
  return rj->tiles2 * rj->tilesT * no;
}

void launch_row_comp(const Geo& g, const RowJob& rj_in, const float* x,
                     float* W, uint16_t* codes, bool write_w,
                     uint32_t* status, hipStream_t s) {
  if (!rj_in.rcnt[0] || !rj_in.rcnt[1]) return;
  RowJob rj = rj_in;
  size_t lds;
  const uint32_t blocks = row_blocks(g, &rj, &lds);
  if (write_w)
    QOZ_LAUNCH(k_row_comp<true>, dim3(blocks), dim3(kRowThreads), lds, s, g,
               rj, x, W, codes, status);
  else
    QOZ_LAUNCH(k_row_comp<false>, dim3(blocks), dim3(kRowThreads), lds, s, g,
               rj, x, W, codes, status);
}

void launch_row_decomp(const Geo& g, const RowJob& rj_in, float* W,
                       const uint16_t* codes, hipStream_t s) {
  if (!rj_in.rcnt[0] || !rj_in.rcnt[1]) return;
  RowJob rj = rj_in;
  size_t lds;
  const uint32_t blocks = row_blocks(g, &rj, &lds);
  QOZ_LAUNCH(k_row_decomp, dim3(blocks), dim3(kRowThreads), lds, s, g, rj, W,
             codes);
}

/* One round of a batch's inverse sweeps: each job is one sweep (64 x 4
 * lane tiles) or one fused level-1 row pair of a different field, so the
 * jobs of a round are independent of each other. */
__global__ __launch_bounds__(kRowThreads) void k_sweep_round_q(
    const SweepJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  extern __shared__ __align__(16) float E[];
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
  extern __shared__ __align__(16) float E[];
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
