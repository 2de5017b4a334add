/*
 * Huffman stage over the quantization bins (Sec. VI-A names Huffman as the
 * entropy coder of the pipeline), for gfx950.
 *
 *  - k_hist:       65536-bin histogram; a 4096-bin LDS window centred on
 *                  the zero bin plus a per-lane counter for the zero bin
 *                  itself absorb the concentrated traffic, the rest goes to
 *                  global atomics.
 *  - k_huff_count: code bits and symbol-0 bins per chunk (code lengths
 *                  in LDS).
 *  - k_scan_tiles / k_scan_apply: exclusive scans of per-chunk counts (one
 *                  workgroup per tile, then the tile offsets): the payload
 *                  offsets and unpredictable ranks of the chunks, and the
 *                  offsets of the zero-word packed payload.
 *  - k_huff_encode: workgroups take runs of chunks in a grid stride, code them with
 *                  the code table in LDS, pack the codes MSB-first into an LDS word
 *                  buffer (ds_or), store the words coalesced at the
 *                  chunk's scanned offset, and gather the exact values of
 *                  bin-0 lanes at their rank.
 * Decoding is in kernels_decode.hip.
 */
#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kHistPerBlock = 1u << 16;
constexpr uint32_t kHistThreads = 512;

/* Workgroup blk of a histogram: bins [blk * 65536, +65536) of codes. */
__device__ __forceinline__ void hist_wg(const uint16_t* __restrict__ codes,
                                        uint64_t n, uint32_t* hist,
                                        uint32_t blk) {
  __shared__ uint32_t lh[kHistWin];
  for (uint32_t i = threadIdx.x; i < kHistWin; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const uint64_t b0 = (uint64_t)blk * kHistPerBlock;
  const uint64_t b1 = b0 + kHistPerBlock < n ? b0 + kHistPerBlock : n;
  uint32_t center = 0;
  /* eight 16-bit bins per 16-byte load, four loads in flight per lane */
  constexpr uint32_t kU = 4;
  const uint64_t nvec = (b1 - b0) / 8;
  const uint4* v4 = reinterpret_cast<const uint4*>(codes + b0);
  for (uint64_t i0 = threadIdx.x; i0 < nvec; i0 += kU * kHistThreads) {
    uint4 q[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) {
      const uint64_t i = i0 + u * kHistThreads;
      q[u] = i < nvec ? v4[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) {
      if (i0 + u * kHistThreads >= nvec) break;
      const uint32_t w[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        hist_add(lh, hist, (int32_t)(w[k] & 0xffffu), center);
        hist_add(lh, hist, (int32_t)(w[k] >> 16), center);
      }
    }
  }
  for (uint64_t i = b0 + nvec * 8 + threadIdx.x; i < b1; i += blockDim.x)
    hist_add(lh, hist, codes[i], center);
  center = wave_sum_u32(center);
  if ((threadIdx.x & 63) == 0 && center)
    atomicAdd(&lh[kRadius - kHistBase], center);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kHistWin; i += blockDim.x) {
    uint32_t v = lh[i];
    if (v) atomicAdd(&hist[kHistBase + (int32_t)i], v);
  }
}

__global__ __launch_bounds__(kHistThreads) void k_hist(
    const uint16_t* __restrict__ codes, uint64_t n, uint32_t* hist) {
  hist_wg(codes, n, hist, blockIdx.x);
}

/* The histograms of many fields in one launch. */
__global__ __launch_bounds__(kHistThreads) void k_hist_q(
    const HistJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  const uint32_t j = find_job(wg0, n_jobs, blockIdx.x);
  /* the record's pointers made global (not flat) */
  hist_wg((const uint16_t*)gptr(jobs[j].codes), jobs[j].n,
          (uint32_t*)gptr(jobs[j].hist), blockIdx.x - wg0[j]);
}

uint32_t hist_job_workgroups(const HistJob& j) {
  return (uint32_t)((j.n + kHistPerBlock - 1) / kHistPerBlock);
}

void launch_hist_q(const HistJob* jobs, const uint32_t* wg0, uint32_t n_jobs,
                   uint32_t total_wg, hipStream_t s) {
  if (!total_wg) return;
  QOZ_LAUNCH(k_hist_q, dim3(total_wg), dim3(kHistThreads), 0, s, jobs,
                     wg0, n_jobs);
}

void launch_hist(const uint16_t* codes, uint64_t n, uint32_t* hist,
                 hipStream_t s) {
  if (!n) return;
  uint64_t blocks = (n + kHistPerBlock - 1) / kHistPerBlock;
  QOZ_LAUNCH(k_hist, dim3((uint32_t)blocks), dim3(kHistThreads), 0, s,
                     codes, n, hist);
}

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPer = 8;
constexpr uint32_t kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, 64);
    v += lane >= o ? t : 0ull;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T scan_block_sum(T v, T* ws) {
  for (uint32_t o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63u) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = 0;
  for (uint32_t w = 0; w < kScanThreads / 64; ++w) t += ws[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(
    const uint32_t* __restrict__ bits, const uint32_t* __restrict__ zeros,
    uint64_t n, uint64_t* __restrict__ tile_w, uint64_t* __restrict__ tile_z,
    uint64_t* __restrict__ tile_max) {
  __shared__ uint64_t ws[kScanThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t sw = 0, sz = 0, mx = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k) {
    const uint64_t i = base + threadIdx.x + k * kScanThreads;
    if (i < n) {
      const uint64_t w = (bits[i] + 31) / 32;
      sw += w;
      sz += zeros[i];
      mx = mx > w ? mx : w;
    }
  }
  for (uint32_t o = 32; o > 0; o >>= 1) {
    const uint64_t t = __shfl_xor(mx, o, 64);
    mx = mx > t ? mx : t;
  }
  __shared__ uint64_t wm[kScanThreads / 64];
  if ((threadIdx.x & 63u) == 0) wm[threadIdx.x >> 6] = mx;
  sw = scan_block_sum(sw, ws);
  sz = scan_block_sum(sz, ws);
  if (threadIdx.x == 0) {
    uint64_t m = 0;
    for (uint32_t w = 0; w < kScanThreads / 64; ++w) m = m > wm[w] ? m : wm[w];
    tile_w[blockIdx.x] = sw;
    tile_z[blockIdx.x] = sz;
    tile_max[blockIdx.x] = m;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(
    const uint32_t* __restrict__ bits, const uint32_t* __restrict__ zeros,
    uint64_t n, const uint64_t* __restrict__ tile_w,
    const uint64_t* __restrict__ tile_z, const uint64_t* __restrict__ tile_max,
    uint64_t* coff, uint64_t* upre, uint64_t* totals) {
  __shared__ uint64_t ws[kScanThreads / 64], wz[kScanThreads / 64];
  const uint32_t b = blockIdx.x, lane = threadIdx.x & 63u,
                 wave = threadIdx.x >> 6;
  /* sums of the tiles before this one */
  uint64_t ow = 0, oz = 0;
  for (uint32_t t = threadIdx.x; t < b; t += kScanThreads) {
    ow += tile_w[t];
    oz += tile_z[t];
  }
  ow = scan_block_sum(ow, ws);
  oz = scan_block_sum(oz, ws);
  /* this lane's 8 consecutive chunks */
  const uint64_t i0 = (uint64_t)b * kScanTile + (uint64_t)threadIdx.x * kScanPer;
  uint32_t w[kScanPer], z[kScanPer];
  uint64_t sw = 0, sz = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k) {
    const bool in = i0 + k < n;
    w[k] = in ? (bits[i0 + k] + 31) / 32 : 0u;
    z[k] = in ? zeros[i0 + k] : 0u;
    sw += w[k];
    sz += z[k];
  }
  const uint64_t iw = wave_incl_scan_u64(sw), iz = wave_incl_scan_u64(sz);
  if (lane == 63) {
    ws[wave] = iw;
    wz[wave] = iz;
  }
  __syncthreads();
  uint64_t pw = ow + iw - sw, pz = oz + iz - sz, tw = 0, tz = 0;
  for (uint32_t v = 0; v < kScanThreads / 64; ++v) {
    pw += v < wave ? ws[v] : 0ull;
    pz += v < wave ? wz[v] : 0ull;
    tw += ws[v];
    tz += wz[v];
  }
#pragma unroll
  for (uint32_t k = 0; k < kScanPer; ++k) {
    if (i0 + k < n) {
      coff[i0 + k] = pw;
      upre[i0 + k] = pz;
    }
    pw += w[k];
    pz += z[k];
  }
  if (b + 1 == gridDim.x && threadIdx.x == 0) {
    uint64_t m = 0;
    for (uint32_t t = 0; t < gridDim.x; ++t) m = m > tile_max[t] ? m : tile_max[t];
    coff[n] = ow + tw;
    upre[n] = oz + tz;
    totals[0] = ow + tw;
    totals[1] = oz + tz;
    totals[2] = m;
  }
}

/* Used symbols of each histogram as keys (count << 16) | symbol, sorted
 * ascending in LDS (bitonic), which is the (count, symbol) leaf order of
 * the two-queue Huffman construction.  out[h * (kSortCap + 1)] = number of
 * used symbols; the next min(that, kSortCap) entries are the sorted keys
 * (more used symbols than kSortCap: the caller falls back to the whole
 * histogram). */
constexpr uint32_t kSortThreads = 1024;

__global__ __launch_bounds__(kSortThreads) void k_hist_sort(
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ ids,
    uint32_t cap, uint64_t* __restrict__ out) {
  static_assert(kNSym % (4 * kSortThreads) == 0, "bins per lane");
  extern __shared__ uint64_t keys[]; /* cap entries, cap a power of two */
  __shared__ uint32_t n_used;
  const uint32_t hid = ids ? ids[blockIdx.x] : blockIdx.x;
  const uint32_t* hh = hist + (uint64_t)hid * kNSym;
  uint64_t* o = out + (uint64_t)blockIdx.x * (cap + 1);
  __shared__ uint32_t wcount[kSortThreads / 64];
  /* lane t holds bins [64 t, 64 t + 64): sixteen 16-byte loads in flight,
   * then the used ones are compacted in bin order by a block scan of the
   * per-lane counts */
  constexpr uint32_t kPer = kNSym / kSortThreads; /* 64 */
  uint32_t v[kPer];
  {
    const uint4* h4 =
        reinterpret_cast<const uint4*>(hh + (uint64_t)threadIdx.x * kPer);
#pragma unroll
    for (uint32_t q = 0; q < kPer / 4; ++q) {
      const uint4 w = h4[q];
      v[4 * q] = w.x;
      v[4 * q + 1] = w.y;
      v[4 * q + 2] = w.z;
      v[4 * q + 3] = w.w;
    }
  }
  uint32_t cnt = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) cnt += v[q] ? 1u : 0u;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint32_t incl = cnt;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    incl += lane >= o ? t : 0u;
  }
  if (lane == 63) wcount[wave] = incl;
  __syncthreads();
  uint32_t k = incl - cnt, total = 0;
  for (uint32_t w = 0; w < kSortThreads / 64; ++w) {
    k += w < wave ? wcount[w] : 0u;
    total += wcount[w];
  }
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q)
    if (v[q]) {
      if (k < cap)
        keys[k] = ((uint64_t)v[q] << 16) | (threadIdx.x * kPer + q);
      ++k;
    }
  if (threadIdx.x == 0) n_used = total;
  __syncthreads();
  const uint32_t n = n_used;
  const uint32_t m = n < cap ? n : cap;
  uint32_t p2 = 2;
  while (p2 < m) p2 <<= 1;
  for (uint32_t i = m + threadIdx.x; i < p2; i += kSortThreads)
    keys[i] = ~0ull;
  __syncthreads();
  for (uint32_t k = 2; k <= p2; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < p2; i += kSortThreads) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = keys[i], b = keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  if (threadIdx.x == 0) o[0] = n;
  for (uint32_t i = threadIdx.x; i < m; i += kSortThreads) o[1 + i] = keys[i];
}

void launch_hist_sort(const uint32_t* hist, uint32_t n_hist, uint64_t* out,
                      hipStream_t s) {
  if (!n_hist) return;
  QOZ_LAUNCH(k_hist_sort, dim3(n_hist), dim3(kSortThreads),
                     8 * kSortCap, s, hist, (const uint32_t*)nullptr,
                     kSortCap, out);
}

bool hist_sort_big_fits() {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                            dev) != hipSuccess)
    return false;
  if (8 * (size_t)kSortCapBig + 256 > (size_t)max_lds) return false;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hist_sort),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(8 * kSortCapBig)) == hipSuccess;
}

void launch_hist_sort_big(const uint32_t* hist, const uint32_t* ids,
                          uint32_t n, uint64_t* out, hipStream_t s) {
  if (!n) return;
  QOZ_LAUNCH(k_hist_sort, dim3(n), dim3(kSortThreads),
                     8 * kSortCapBig, s, hist, ids, kSortCapBig, out);
}

uint64_t chunk_scan_scratch(uint64_t n_chunks) {
  return 24 * ((n_chunks + kScanTile - 1) / kScanTile + 1);
}

void launch_chunk_scan(const uint32_t* chunk_bits,
                       const uint32_t* chunk_zeros, uint64_t n_chunks,
                       uint64_t* coff, uint64_t* upre, uint64_t* totals,
                       uint64_t* scratch, hipStream_t s) {
  /* at least one tile, so that the totals are written for no chunks too */
  const uint32_t tiles =
      n_chunks ? (uint32_t)((n_chunks + kScanTile - 1) / kScanTile) : 1u;
  uint64_t* tw = scratch;
  uint64_t* tz = tw + tiles;
  uint64_t* tm = tz + tiles;
  QOZ_LAUNCH(k_scan_tiles, dim3(tiles), dim3(kScanThreads), 0, s,
                     chunk_bits, chunk_zeros, n_chunks, tw, tz, tm);
  QOZ_LAUNCH(k_scan_apply, dim3(tiles), dim3(kScanThreads), 0, s,
                     chunk_bits, chunk_zeros, n_chunks, tw, tz, tm, coff,
                     upre, totals);
}

/* words of a chunk: at most 56 bits per bin (the encoder table's limit) */
constexpr uint32_t kEncMaxWords = kChunk * 56 / 32;
/* code table entries kept in LDS (a window of the field's table) */
constexpr uint32_t kEncTab = 4096;

/* First table index of the LDS window of a code table over symbols
 * [lo, lo + tn): the window of w entries is centred on the zero-residual
 * symbol R, where the bins concentrate, and kept inside the table. */
__device__ __forceinline__ uint32_t table_window(int32_t lo, uint32_t tn,
                                                 uint32_t w) {
  if (tn <= w) return 0;
  const int32_t want = kRadius - (int32_t)(w / 2) - lo;
  const int32_t top = (int32_t)(tn - w);
  return (uint32_t)(want < 0 ? 0 : want > top ? top : want);
}

/* Code bits and symbol-0 bins of every chunk, the counts the chunk scan
 * turns into payload offsets and unpredictable ranks before encoding.  A
 * workgroup takes kCountChunks consecutive chunks of one field (the
 * field's workgroups start at wg0[f]) with the field's code lengths in LDS
 * (a window of kCountLens symbols centred on the zero residual; the rest
 * from the global table); a wave counts one
 * chunk, each lane 8 groups of 8 bins read as 16-byte loads (chunks start
 * on a multiple of 64 bins).  Counts go to bits[chunk0[f] + c] and
 * zeros[chunk0[f] + c], the chunk's first bin and size to geo[..]. */
constexpr uint32_t kCountThreads = 256;
constexpr uint32_t kCountChunks = 8;
constexpr uint32_t kCountLens = 16384;

__global__ __launch_bounds__(kCountThreads) void k_huff_count(
    const EncField* __restrict__ fields, const uint64_t* __restrict__ chunk0,
    const uint32_t* __restrict__ wg0, uint32_t nf,
    uint32_t* __restrict__ bits_out, uint32_t* __restrict__ zeros_out,
    ChunkGeo* __restrict__ geo) {
  constexpr uint32_t kGroups = kChunk / (8 * 64); /* 8 per lane */
  __shared__ uint8_t lens[kCountLens];
  const uint32_t f = find_job(wg0, nf, blockIdx.x);
  const EncField& F = fields[f];
  /* pointers read from the record, made global (flat accesses would also
   * count against the LDS counter) */
  const __attribute__((address_space(1))) uint64_t* const tab = gptr(F.tab);
  const __attribute__((address_space(1))) uint16_t* const codes =
      gptr(F.codes);
  const uint32_t tn = F.tn;
  const uint32_t tl = tn < kCountLens ? tn : kCountLens;
  const int32_t lo = F.lo;
  const uint32_t wo = table_window(lo, tn, kCountLens);
  for (uint32_t i = threadIdx.x; i < tl; i += kCountThreads)
    lens[i] = (uint8_t)(tab[wo + i] & 0xff);
  __syncthreads();
  const uint32_t zlen = (uint32_t)(F.zero_entry & 0xff);
  const uint64_t c0 = (uint64_t)(blockIdx.x - wg0[f]) * kCountChunks;
  const uint64_t c1 = c0 + kCountChunks < F.nch ? c0 + kCountChunks : F.nch;
  const uint32_t lane = threadIdx.x & 63u;
  auto add = [&](uint32_t sym, uint32_t& bits, uint32_t& zeros) {
    const uint32_t o = sym - (uint32_t)lo;
    const uint32_t l = sym == 0 ? zlen
                       : o - wo < tl ? (uint32_t)lens[o - wo]
                       : o < tn ? (uint32_t)(tab[o] & 0xff)
                                : 0u;
    bits += l;
    zeros += sym == 0 ? 1u : 0u;
  };
  for (uint64_t c = c0 + (threadIdx.x >> 6); c < c1;
       c += kCountThreads / 64) {
    const uint64_t b = F.ch.begin(c);
    const uint32_t n = (uint32_t)(F.ch.end(c) - b);
    uint4 q[kGroups];
#pragma unroll
    for (uint32_t u = 0; u < kGroups; ++u) {
      const uint32_t m = lane + 64 * u;
      q[u] = 8 * m + 8 <= n
                 ? gload16((const uint16_t*)(codes + b + 8 * m))
                 : make_uint4(0, 0, 0, 0);
    }
    uint32_t bits = 0, zeros = 0;
#pragma unroll
    for (uint32_t u = 0; u < kGroups; ++u) {
      const uint32_t m = lane + 64 * u;
      if (8 * m + 8 <= n) {
        const uint32_t w[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k)
          add((w[k >> 1] >> (16 * (k & 1))) & 0xffffu, bits, zeros);
      } else {
        for (uint32_t i = 8 * m; i < n; ++i) add(codes[b + i], bits, zeros);
      }
    }
    bits = wave_sum_u32(bits);
    zeros = wave_sum_u32(zeros);
    if (lane == 0) {
      bits_out[chunk0[f] + c] = bits;
      zeros_out[chunk0[f] + c] = zeros;
      geo[chunk0[f] + c] = ChunkGeo{b, n, 0u};
    }
  }
}

uint32_t count_workgroups(uint64_t n_chunks) {
  return (uint32_t)((n_chunks + kCountChunks - 1) / kCountChunks);
}

void launch_huff_count(const EncField* fields, const uint64_t* chunk0,
                       const uint32_t* wg0, uint32_t nf, uint32_t total_wg,
                       uint32_t* bits, uint32_t* zeros, ChunkGeo* geo,
                       hipStream_t s) {
  if (!total_wg) return;
  QOZ_LAUNCH(k_huff_count, dim3(total_wg), dim3(kCountThreads), 0, s,
             fields, chunk0, wg0, nf, bits, zeros, geo);
}

/* Encoding of the chunks of one or more fields, after k_huff_count and the
 * chunk scan: gw and gz are the exclusive prefixes of the chunks' payload
 * words and symbol-0 bins over the global chunk order (a field's offsets
 * are differences of them).  Workgroup w codes runs of R global chunks
 * (field after field; R up to 8): runs w, w + G, w + 2G, ... for a grid of
 * G as large as the device holds at once, and loads the next chunk's bins
 * while it codes the current one.  Per chunk:
 *   - segment-major staging of the bins in LDS (segment j holds the
 *     chunk's bins j, j + 8, ...; bins past the chunk's end stage as 1);
 *   - thread t codes bins [16 (t mod 32), +16) of segment t / 32 (thread
 *     order is payload order) with the field's code table: a window of it
 *     in LDS, reloaded when the field changes; a symbol outside the window
 *     is read from the global table in a branch of its own;
 *   - block scans of the bit counts and of the bin-0 counts;
 *   - the codes packed MSB-first into an LDS word buffer: a completed word
 *     is a plain store, the two words a thread may share with its
 *     neighbours are ORed into the zeroed buffer;
 *   - the chunk's size under zero-word packing counted (and added to the
 *     field's packed total), the words stored at the chunk's offset, the
 *     chunk offset, unpredictable rank and segment lengths written to
 *     their stream sections, and the exact values of bin-0 bins gathered
 *     in bin order at their ranks.
 * A field's last chunk also writes its totals (payload words, symbol-0
 * bins).  No workgroup waits for another.  The field records are read
 * through the constant address space: they are not written while the
 * kernel runs, so the reads are scalar loads, which neither wait for nor
 * hold up the vector loads and stores in flight (a record read as a plain
 * load is a vector load, whose wait would also wait for the next chunk's
 * bins and for the stores). */
#define QOZ_CONST __attribute__((address_space(4)))

constexpr uint32_t kEncThreads = 256;
constexpr uint32_t kEncLaneBins = kChunk / kEncThreads;    /* 16 */
constexpr uint32_t kEncRounds = kChunk / (8 * kEncThreads); /* 2 */
constexpr uint32_t kEncLanesPerSeg = kSeg / kEncLaneBins;   /* 32 */
static_assert(kEncLanesPerSeg * kEncLaneBins == kSeg, "segment lanes");
static_assert(kEncRounds == 2 && kChunk / kSegPerChunk == kSeg,
              "chunk layout");

/* Inclusive scan over the wave by DPP: shifts by 1, 2, 4 and 8 lanes
 * within each row of 16, then the last lane of row 0 (and of row 2) added
 * to rows 1 and 3, and the last lane of row 1 to rows 2 and 3. */
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}

/* Exclusive scans of two values over the workgroup (one barrier); the
 * totals in *ta and *tb. */
__device__ __forceinline__ void block_excl_scan2(uint32_t a, uint32_t b,
                                                 uint32_t (*ws)[kEncThreads / 64],
                                                 uint32_t* ea, uint32_t* eb,
                                                 uint32_t* ta, uint32_t* tb) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  if (lane == 63) {
    ws[0][wave] = ia;
    ws[1][wave] = ib;
  }
  __syncthreads();
  uint32_t pa = 0, pb = 0, sa = 0, sb = 0;
#pragma unroll
  for (uint32_t w = 0; w < kEncThreads / 64; ++w) {
    pa += w < wave ? ws[0][w] : 0u;
    pb += w < wave ? ws[1][w] : 0u;
    sa += ws[0][w];
    sb += ws[1][w];
  }
  *ea = pa + ia - a;
  *eb = pb + ib - b;
  *ta = sa;
  *tb = sb;
}

template <bool kLong> /* kLong: some code is longer than 32 bits */
__global__ __launch_bounds__(kEncThreads, 4) void k_huff_encode(
    const EncField* __restrict__ fields, const uint64_t* __restrict__ chunk0,
    const ChunkGeo* __restrict__ geo, const uint64_t* __restrict__ gw,
    const uint64_t* __restrict__ gz, uint32_t nf, uint64_t n_total,
    uint32_t tcap, uint32_t max_words, uint32_t run) {
  extern __shared__ uint64_t lds64[];
  uint64_t* tabl = lds64; /* tcap entries, an empty one, symbol 0's */
  /* max_words + 1 words, then a dummy word per thread */
  uint32_t* words = reinterpret_cast<uint32_t*>(lds64 + tcap + 2);
  __shared__ __align__(16) uint16_t cbin[kChunk];
  __shared__ uint32_t ws[2][kEncThreads / 64];
  __shared__ uint32_t seg_end[kSegPerChunk];
  __shared__ uint32_t s_nz;
  const QOZ_CONST EncField* cfields = (const QOZ_CONST EncField*)fields;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  /* field of global chunk c2 (uniform, scalar) */
  const uint64_t c0_lane = lane < nf ? chunk0[lane] : ~0ull;
  auto field_of = [&](uint64_t c2) -> uint32_t {
    if (nf <= 64) /* chunk0 in registers, one entry per lane */
      return __builtin_amdgcn_readfirstlane(
          (uint32_t)__popcll(__ballot(c0_lane <= c2)) - 1);
    uint32_t cnt = 0;
    for (uint32_t b = 0; b < nf; b += 64) {
      const uint32_t i = b + lane;
      cnt += (uint32_t)__popcll(__ballot(i < nf && chunk0[i] <= c2));
    }
    return __builtin_amdgcn_readfirstlane(cnt - 1);
  };
  /* runs of `run` consecutive chunks, every grid-th run to a workgroup:
   * a run crosses few fields, so a batch of fields reloads few table
   * windows, and every workgroup still takes a share of every part of the
   * batch (the cost of a chunk varies much between fields) */
  uint64_t g = (uint64_t)blockIdx.x * run;
  const uint64_t g_end = n_total;
  const uint64_t hop = (uint64_t)(gridDim.x - 1) * run + 1;
  auto next_chunk = [&](uint64_t c2) -> uint64_t {
    return ((c2 + 1) & (run - 1)) ? c2 + 1 : c2 + hop; /* run: 2^k */
  };
  /* this thread's staging groups m = t + 256 r of a chunk */
  uint4 qr[kEncRounds];
  auto load_bins = [&](uint64_t c2, uint32_t f2) {
#pragma unroll
    for (uint32_t r = 0; r < kEncRounds; ++r) qr[r] = make_uint4(0, 0, 0, 0);
    if (c2 >= g_end) return;
    const uint16_t* codes2 = cfields[f2].codes;
    const uint64_t b2 = geo[c2].begin;
    const uint32_t n2 = geo[c2].n;
#pragma unroll
    for (uint32_t r = 0; r < kEncRounds; ++r) {
      const uint32_t m = tid + kEncThreads * r;
      /* a group the chunk ends in reads up to 7 bins past it: the bins of
       * the next chunk, or the 16 bins of padding after the last */
      if (8 * m < n2) qr[r] = gload16(codes2 + b2 + 8 * m);
    }
  };
  for (uint32_t i = tid; i <= max_words; i += kEncThreads) words[i] = 0;
  if (tid == 0) s_nz = 0;
  uint32_t fn = g < g_end ? field_of(g) : 0u;
  load_bins(g, fn);
  uint32_t loaded = ~0u; /* field whose table window is in LDS */
  uint32_t tw = 0, wo = 0;
  uint32_t dirty = 0;       /* words of the previous chunk (to zero again) */
  uint32_t pk_field = ~0u;  /* thread 0: packed words of pk_field so far */
  uint64_t pk_acc = 0;
  const uint32_t j = tid / kEncLanesPerSeg;
  const uint32_t k0 = (tid % kEncLanesPerSeg) * kEncLaneBins;
  while (g < g_end) {
    const uint32_t f = fn;
    const QOZ_CONST EncField& F = cfields[f];
    const int32_t lo = F.lo;
    const uint32_t tn = F.tn;
    const uint64_t zero_entry = F.zero_entry;
    if (f != loaded) { /* the last barrier ended every use of the old one */
      tw = tn < tcap ? tn : tcap;
      wo = table_window(lo, tn, tcap);
      for (uint32_t i = tid; i < tw; i += kEncThreads)
        tabl[i] = gptr(F.tab)[wo + i];
      /* slot tw: an empty entry (the padding symbol lo + tn of the fast
       * path), slot tw + 1: symbol 0, which min(symbol - lo, tw + 1)
       * reaches when the window starts at lo (symbol 0 is below every
       * other) */
      if (tid == 0) {
        tabl[tw] = 0;
        tabl[tw + 1] = zero_entry;
      }
      loaded = f;
    }
    const uint64_t c = g - chunk0[f]; /* chunk within the field */
    const uint64_t base = geo[g].begin;
    const uint32_t nsym = geo[g].n;
    /* the chunk's word and unpredictable offsets within its field */
    const uint64_t w0 = gw[g] - gw[chunk0[f]];
    const uint64_t u0 = gz[g] - gz[chunk0[f]];
    /* a chunk whose field's table lies whole in the LDS window needs no
     * check per bin (bins past a short chunk's end stage as the padding
     * symbol lo + tn, whose entry is empty) */
    const bool fast = tw == tn && f == loaded && (uint32_t)lo + tn <= 0xffffu;
    const uint32_t pad = fast ? (uint32_t)lo + tn : 1u;
    /* staging: bin 8 m + i to segment i, position m */
    uint32_t zpack = 0; /* bin-0 count of round r in bits [16 r, +16) */
    uint32_t zmask = 0; /* bit 8 r + i: bin 8 m + i of round r is 0 */
    if (fast && nsym == kChunk) {
      /* the halves of each word go straight to LDS; a zero half is
       * detected per word (exact: a borrow into the high half only follows
       * a zero low half) and counted only then */
      uint32_t hz = 0;
#pragma unroll
      for (uint32_t r = 0; r < kEncRounds; ++r) {
        const uint32_t m = tid + kEncThreads * r;
        const uint32_t w[4] = {qr[r].x, qr[r].y, qr[r].z, qr[r].w};
#pragma unroll
        for (uint32_t d = 0; d < 4; ++d) {
          cbin[(2 * d) * kSeg + m] = (uint16_t)w[d];
          cbin[(2 * d + 1) * kSeg + m] = (uint16_t)(w[d] >> 16);
          hz |= (w[d] - 0x00010001u) & ~w[d] & 0x80008000u;
        }
      }
      if (hz) {
#pragma unroll
        for (uint32_t r = 0; r < kEncRounds; ++r) {
          const uint32_t w[4] = {qr[r].x, qr[r].y, qr[r].z, qr[r].w};
          uint32_t z = 0;
#pragma unroll
          for (uint32_t i = 0; i < 8; ++i) {
            const bool zero = ((w[i / 2] >> (16 * (i & 1))) & 0xffffu) == 0;
            z += zero ? 1u : 0u;
            zmask |= (zero ? 1u : 0u) << (8 * r + i);
          }
          zpack |= z << (16 * r);
        }
      }
    } else {
#pragma unroll
      for (uint32_t r = 0; r < kEncRounds; ++r) {
        const uint32_t m = tid + kEncThreads * r;
        const uint32_t w[4] = {qr[r].x, qr[r].y, qr[r].z, qr[r].w};
        uint32_t z = 0;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
          const uint32_t v = 8 * m + i < nsym
                                 ? (w[i / 2] >> (16 * (i & 1))) & 0xffffu
                                 : pad;
          cbin[i * kSeg + m] = (uint16_t)v;
          z += v == 0 ? 1u : 0u;
          zmask |= (v == 0 ? 1u : 0u) << (8 * r + i);
        }
        zpack |= z << (16 * r);
      }
    }
    for (uint32_t i = tid; i < dirty; i += kEncThreads) words[i] = 0;
    __syncthreads();
    /* the next chunk's bins load while this one is coded */
    const uint64_t gn = next_chunk(g);
    fn = gn < g_end ? field_of(gn) : 0u;
    load_bins(gn, fn);
    /* the thread's 16 code table entries ((code << 8) | length; 0 past the
     * chunk's end); symbols outside the LDS window in a branch of their
     * own, so that its wait (which would also wait for the bins in flight)
     * stays off the common path */
    uint64_t ent[kEncLaneBins];
    uint32_t bits = 0;
    {
      const uint4* cb = reinterpret_cast<const uint4*>(cbin + j * kSeg + k0);
      const uint4 qa = cb[0], qb = cb[1];
      const uint32_t w[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
      if (fast) { /* the window is the whole table, from lo */
#pragma unroll
        for (uint32_t k = 0; k < kEncLaneBins; ++k) {
          const uint32_t o =
              ((w[k / 2] >> (16 * (k & 1))) & 0xffffu) - (uint32_t)lo;
          ent[k] = tabl[o < tw + 1 ? o : tw + 1];
          bits += (uint32_t)(ent[k] & 0xff);
        }
      } else {
        uint32_t far = 0;
#pragma unroll
        for (uint32_t k = 0; k < kEncLaneBins; ++k) {
          const uint32_t b = (k0 + k) * kSegPerChunk + j;
          const uint32_t sym = (w[k / 2] >> (16 * (k & 1))) & 0xffffu;
          const uint32_t o = sym - (uint32_t)lo;
          const uint32_t ow = o - wo;
          const bool in = b < nsym;
          const bool near = f == loaded && ow < tw;
          ent[k] = !in ? 0ull : sym == 0 ? zero_entry : near ? tabl[ow] : 0ull;
          far |= (in && sym != 0 && !near && o < tn ? 1u : 0u) << k;
        }
#pragma unroll
        for (uint32_t k = 0; k < kEncLaneBins; ++k)
          bits += (uint32_t)(ent[k] & 0xff);
        if (far) {
#pragma unroll
          for (uint32_t k = 0; k < kEncLaneBins; ++k)
            if ((far >> k) & 1u) {
              const uint32_t sym = (w[k / 2] >> (16 * (k & 1))) & 0xffffu;
              ent[k] = gptr(F.tab)[sym - (uint32_t)lo];
              bits += (uint32_t)(ent[k] & 0xff);
            }
        }
      }
    }
    uint32_t pos0, zex, tot_bits, tot_z;
    block_excl_scan2(bits, zpack, ws, &pos0, &zex, &tot_bits, &tot_z);
    const uint32_t nw = (tot_bits + 31) / 32;
    if (tid % kEncLanesPerSeg == kEncLanesPerSeg - 1) seg_end[j] = pos0 + bits;
    {
      /* acc holds the bits not yet written in its low nacc (< 32) bits.
       * Every code ends in one store without a branch: the word it
       * completes, or (when it completes none) a dummy slot of the thread.
       * A first word that starts before pos0 is shared with the threads
       * before: it is kept and ORed in at the end, as is the last partial
       * word (shared with the threads after). */
      uint64_t acc = 0;
      const uint32_t first = pos0 >> 5;
      const bool sfirst = (pos0 & 31u) != 0;
      const uint32_t dummy = max_words + 1 + tid;
      uint32_t nacc = pos0 & 31u, wi = first;
      uint32_t firstw = 0;
      auto put = [&](uint32_t code, uint32_t len) { /* len <= 32 */
        acc = (acc << len) | code;
        nacc += len;
        const bool full = nacc >= 32;
        nacc &= 31u;
        const uint32_t v = (uint32_t)(acc >> nacc);
        /* bitwise, so that no branch comes of it */
        const bool keep = full & sfirst & (wi == first);
        firstw = keep ? v : firstw;
        words[full & !keep ? wi : dummy] = v;
        wi += full ? 1u : 0u;
      };
#pragma unroll
      for (uint32_t k = 0; k < kEncLaneBins; ++k) {
        const uint32_t len = (uint32_t)(ent[k] & 0xff);
        const uint64_t code = ent[k] >> 8;
        if (kLong && len > 32) {
          put((uint32_t)(code >> 32), len - 32);
          put((uint32_t)code, 32);
        } else {
          put((uint32_t)code, len);
        }
      }
      const uint32_t tail = nacc ? (uint32_t)(acc << (32 - nacc)) : 0u;
      if (sfirst && wi == first)
        firstw |= tail; /* the thread's bits end in its shared first word */
      else if (nacc)
        atomicOr(&words[wi], tail);
      if (sfirst && bits) atomicOr(&words[first], firstw);
    }
    __syncthreads();
    if (tid < kSegPerChunk - 1)
      gptr(F.segs)[c * (kSegPerChunk - 1) + tid] =
          (uint16_t)(seg_end[tid] - (tid ? seg_end[tid - 1] : 0u));
    /* the chunk's size under zero-word packing (bitmap + nonzero words
     * when shorter, else raw), and the stores */
    {
      uint32_t nz = 0;
      bool over = false;
      for (uint32_t i = tid; i < nw; i += kEncThreads) {
        const uint32_t v = words[i];
        nz += v != 0u ? 1u : 0u;
        if (w0 + i < F.cap_words)
          __builtin_nontemporal_store(v, &gptr(F.payload)[w0 + i]);
        else
          over = true;
      }
      nz = wave_sum_u32(nz);
      if (lane == 0 && nz) atomicAdd(&s_nz, nz);
      if (__ballot(over) != 0 && lane == 0) atomicOr(F.status, kStOverflow);
    }
    /* bin-0 values in bin order (ascending bits of zmask within each
     * round), each round ranked from its own prefix */
    if (zmask) {
      uint64_t zr[kEncRounds] = {u0 + (zex & 0xffffu),
                                 u0 + (tot_z & 0xffffu) + (zex >> 16)};
      for (uint32_t zm = zmask; zm; zm &= zm - 1) {
        const uint32_t k = (uint32_t)__ffs(zm) - 1;
        const uint32_t r = k >> 3;
        const uint64_t rank = r ? zr[1]++ : zr[0]++;
        const uint32_t m = tid + kEncThreads * r;
        gptr(F.unpred)[rank] = gptr(F.x)[point_of(
            fields[f].st, fields[f].g, base + 8 * m + (k & 7))];
      }
    }
    __syncthreads();
    if (tid == 0) {
      const uint32_t zc = (tot_z & 0xffffu) + (tot_z >> 16);
      gptr(F.coff)[c] = w0;
      gptr(F.upre)[c] = (uint32_t)u0;
      if (c + 1 == F.nch) {
        gptr(F.coff)[F.nch] = w0 + nw;
        gptr(F.upre)[F.nch] = (uint32_t)(u0 + zc);
        gptr(F.totals)[0] = w0 + nw;
        gptr(F.totals)[1] = u0 + zc;
      }
      const uint32_t nbm = (nw + 31) / 32;
      const uint32_t pw = nbm + s_nz < nw ? nbm + s_nz : nw;
      s_nz = 0;
      gptr(F.pack_bits)[c] = 32 * pw;
      if (f != pk_field) {
        if (pk_field != ~0u)
          atomicAdd((unsigned long long*)&fields[pk_field].totals[2],
                    (unsigned long long)pk_acc);
        pk_field = f;
        pk_acc = 0;
      }
      pk_acc += pw;
    }
    dirty = nw + 1;
    g = gn;
  }
  if (tid == 0 && pk_field != ~0u)
    atomicAdd((unsigned long long*)&fields[pk_field].totals[2],
              (unsigned long long)pk_acc);
}

uint32_t encode_max_words(uint32_t max_len) {
  const uint64_t w = ((uint64_t)kChunk * max_len + 31) / 32;
  return (uint32_t)(w < kEncMaxWords ? w : kEncMaxWords);
}

void launch_huff_encode(const EncField* fields, const uint64_t* chunk0,
                        const ChunkGeo* geo, const uint64_t* gw,
                        const uint64_t* gz, uint32_t nf, uint64_t n_chunks,
                        uint32_t max_words, uint32_t max_tn, bool long_codes,
                        hipStream_t s) {
  if (!n_chunks || !nf) return;
  const uint32_t tcap = max_tn < kEncTab ? (max_tn ? max_tn : 1u) : kEncTab;
  /* LDS: the table window, an empty entry and symbol 0's, then the
   * chunk's words and a dummy word per thread */
  const size_t lds = 8 * ((size_t)tcap + 2) +
                     4 * ((size_t)max_words + 1 + kEncThreads);
  /* as many workgroups as can be resident at once (each takes every
   * grid-th run of chunks, so one that waits for a slot would finish
   * last) */
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu,
          long_codes ? reinterpret_cast<const void*>(k_huff_encode<true>)
                     : reinterpret_cast<const void*>(k_huff_encode<false>),
          kEncThreads, lds) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const uint64_t n_wg = (uint64_t)cus * (uint64_t)per_cu;
  /* runs of up to 8 chunks while every workgroup still takes 4 runs or
   * more */
  uint32_t run = 8;
  while (run > 1 && n_chunks < (uint64_t)run * 4 * n_wg) run /= 2;
  const uint64_t n_runs = (n_chunks + run - 1) / run;
  const uint32_t grid = (uint32_t)(n_runs < n_wg ? n_runs : n_wg);
  if (long_codes)
    QOZ_LAUNCH(k_huff_encode<true>, dim3(grid), dim3(kEncThreads), lds, s,
               fields, chunk0, geo, gw, gz, nf, n_chunks, tcap, max_words,
               run);
  else
    QOZ_LAUNCH(k_huff_encode<false>, dim3(grid), dim3(kEncThreads), lds, s,
               fields, chunk0, geo, gw, gz, nf, n_chunks, tcap, max_words,
               run);
}

}  // namespace qoz
