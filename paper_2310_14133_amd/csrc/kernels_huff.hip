/*
 * Huffman stage over the quantization bins (Sec. VI-A names Huffman as the
 * entropy coder of the pipeline), for gfx950.
 *
 *  - k_hist:       65536-bin histogram; a 4096-bin LDS window centred on
 *                  the zero bin plus a per-lane counter for the zero bin
 *                  itself absorb the concentrated traffic, the rest goes to
 *                  global atomics.
 *  - k_huff_len:   bits and unpredictable count per 4096-bin chunk.
 *  - k_chunk_scan: exclusive scans -> chunk word offsets and unpredictable
 *                  ranks (one workgroup).
 *  - k_huff_encode: one workgroup per chunk packs its codes MSB-first into
 *                  an LDS word buffer (ds_or), then stores the words
 *                  coalesced; lanes holding bin 0 gather their exact value
 *                  into the unpredictable list at their global rank.
 * Decoding is in kernels_decode.hip.
 */
#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kHistPerBlock = 1u << 16;
constexpr uint32_t kHistThreads = 512;

__global__ __launch_bounds__(kHistThreads) void k_hist(
    const uint16_t* __restrict__ codes, uint64_t n, uint32_t* hist) {
  __shared__ uint32_t lh[kHistWin];
  for (uint32_t i = threadIdx.x; i < kHistWin; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const uint64_t b0 = (uint64_t)blockIdx.x * kHistPerBlock;
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

void launch_hist(const uint16_t* codes, uint64_t n, uint32_t* hist,
                 hipStream_t s) {
  if (!n) return;
  uint64_t blocks = (n + kHistPerBlock - 1) / kHistPerBlock;
  hipLaunchKernelGGL(k_hist, dim3((uint32_t)blocks), dim3(kHistThreads), 0, s,
                     codes, n, hist);
}

/* Code table: entry = (code << 8) | length for symbols in [lo, lo + tn);
 * symbol 0 (unpredictable) has its own entry. */
__device__ __forceinline__ uint64_t code_entry(const uint64_t* tab,
                                               int32_t lo, uint32_t tn,
                                               uint64_t zero_entry,
                                               int32_t sym) {
  if (sym == 0) return zero_entry;
  uint32_t o = (uint32_t)(sym - lo);
  return o < tn ? tab[o] : 0;
}

constexpr uint32_t kEncThreads = 256;
constexpr uint32_t kEncPerThread = kChunk / kEncThreads; /* 16 */

__device__ __forceinline__ uint32_t block_reduce_u32(uint32_t v,
                                                     uint32_t* sh) {
  v = wave_sum_u32(v);
  const uint32_t wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  uint32_t r = 0;
  if (threadIdx.x == 0)
    for (uint32_t w = 0; w < blockDim.x / 64; ++w) r += sh[w];
  return r;
}

/* Bits and symbol-0 count per chunk.  Workgroups are persistent over
 * chunks; code lengths of the symbols [lo, lo + tn) sit in LDS as bytes
 * (from the code table in global memory when the range is wider than the
 * LDS copy).  A lane reads 16 bins as two 16-byte loads. */
constexpr uint32_t kLenLds = 16384;

__global__ __launch_bounds__(kEncThreads) void k_huff_len(
    const uint16_t* __restrict__ codes, Chunks ch,
    const uint64_t* __restrict__ tab, int32_t lo, uint32_t tn,
    uint64_t zero_entry, uint32_t* chunk_bits, uint32_t* chunk_zeros) {
  __shared__ uint8_t lens[kLenLds];
  const bool in_lds = tn <= kLenLds;
  if (in_lds)
    for (uint32_t i = threadIdx.x; i < tn; i += kEncThreads)
      lens[i] = (uint8_t)(tab[i] & 0xff);
  __syncthreads();
  const uint32_t zlen = (uint32_t)(zero_entry & 0xff);
  const uint64_t n_chunks = ch.count();
  const uint32_t lane = threadIdx.x & 63u;
  auto bin_len = [&](uint32_t s, uint32_t& bits, uint32_t& zeros) {
    if (s == 0) {
      bits += zlen;
      ++zeros;
      return;
    }
    const uint32_t o = s - (uint32_t)lo;
    bits += o < tn ? (in_lds ? lens[o] : (uint32_t)(tab[o] & 0xff)) : 0u;
  };
  /* one wave per chunk: lane t takes 8-bin groups t, t + 64, ...; chunks
   * start on a multiple of 64 bins, so full groups are 16-byte loads */
  constexpr uint32_t kU = 4;
  const uint64_t waves = (uint64_t)gridDim.x * (kEncThreads / 64);
  for (uint64_t c = (uint64_t)blockIdx.x * (kEncThreads / 64) + (threadIdx.x >> 6);
       c < n_chunks; c += waves) {
    const uint64_t b = ch.begin(c), e = ch.end(c);
    uint32_t bits = 0, zeros = 0;
    for (uint64_t g0 = b + 8 * (uint64_t)lane; g0 < e; g0 += 8 * 64 * kU) {
      uint4 q[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        const uint64_t g = g0 + 8 * 64 * u;
        q[u] = g + 8 <= e ? *reinterpret_cast<const uint4*>(codes + g)
                          : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        const uint64_t g = g0 + 8 * 64 * u;
        if (g >= e) break;
        if (g + 8 <= e) {
          const uint32_t w[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
          for (uint32_t k = 0; k < 8; ++k)
            bin_len((w[k >> 1] >> (16 * (k & 1))) & 0xffffu, bits, zeros);
        } else {
          for (uint64_t i = g; i < e; ++i) bin_len(codes[i], bits, zeros);
        }
      }
    }
    bits = wave_sum_u32(bits);
    zeros = wave_sum_u32(zeros);
    if (lane == 0) {
      chunk_bits[c] = bits;
      chunk_zeros[c] = zeros;
    }
  }
}

void launch_huff_len(const uint16_t* codes, const Chunks& chunks,
                     const uint64_t* table, int32_t tab_lo, uint32_t tab_n,
                     uint64_t zero_entry, uint32_t* chunk_bits,
                     uint32_t* chunk_zeros, hipStream_t s) {
  const uint64_t nch = chunks.count();
  if (!nch) return;
  const uint64_t per = kEncThreads / 64; /* chunks in flight per workgroup */
  const uint32_t blocks =
      (nch + per - 1) / per < 2048 ? (uint32_t)((nch + per - 1) / per) : 2048u;
  hipLaunchKernelGGL(k_huff_len, dim3(blocks), dim3(kEncThreads), 0, s,
                     codes, chunks, table, tab_lo, tab_n, zero_entry,
                     chunk_bits, chunk_zeros);
}

/* Exclusive scans over chunks (words = ceil(bits / 32), unpredictable
 * counts) in two launches: k_scan_tiles sums tiles of 2048 chunks (and
 * finds the largest chunk in words); k_scan_apply adds the sums of the
 * tiles before its own and scans its tile (8 consecutive chunks per lane,
 * lane sums scanned with wave shuffles).  The last tile also writes
 * coff[n], upre[n] and totals[0..2] = words, unpredictables, largest chunk
 * in words. */
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
    uint64_t* coff, uint32_t* upre, uint64_t* totals) {
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
      upre[i0 + k] = (uint32_t)pz;
    }
    pw += w[k];
    pz += z[k];
  }
  if (b + 1 == gridDim.x && threadIdx.x == 0) {
    uint64_t m = 0;
    for (uint32_t t = 0; t < gridDim.x; ++t) m = m > tile_max[t] ? m : tile_max[t];
    coff[n] = ow + tw;
    upre[n] = (uint32_t)(oz + tz);
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
  hipLaunchKernelGGL(k_hist_sort, dim3(n_hist), dim3(kSortThreads),
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
  hipLaunchKernelGGL(k_hist_sort, dim3(n), dim3(kSortThreads),
                     8 * kSortCapBig, s, hist, ids, kSortCapBig, out);
}

uint64_t chunk_scan_scratch(uint64_t n_chunks) {
  return 24 * ((n_chunks + kScanTile - 1) / kScanTile + 1);
}

void launch_chunk_scan(const uint32_t* chunk_bits,
                       const uint32_t* chunk_zeros, uint64_t n_chunks,
                       uint64_t* coff, uint32_t* upre, uint64_t* totals,
                       uint64_t* scratch, hipStream_t s) {
  /* at least one tile, so that the totals are written for no chunks too */
  const uint32_t tiles =
      n_chunks ? (uint32_t)((n_chunks + kScanTile - 1) / kScanTile) : 1u;
  uint64_t* tw = scratch;
  uint64_t* tz = tw + tiles;
  uint64_t* tm = tz + tiles;
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanThreads), 0, s,
                     chunk_bits, chunk_zeros, n_chunks, tw, tz, tm);
  hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kScanThreads), 0, s,
                     chunk_bits, chunk_zeros, n_chunks, tw, tz, tm, coff,
                     upre, totals);
}

/* words of a chunk: at most 56 bits per bin (the encoder table's limit) */
constexpr uint32_t kEncMaxWords = kChunk * 56 / 32;

/* Segment-major packing: segment j holds the chunk's bins j, j + 8, ....
 * The chunk's bins are staged in LDS by segment (cbin[j * 512 + k] = bin
 * 8k + j), lane t packs bins k in [16 (t mod 32), +16) of segment t / 32,
 * so the thread-order scan of bit counts is the payload order.  A lane
 * builds its bits in a register and writes whole words it alone covers
 * with plain LDS stores, the (at most two) words it shares with its
 * neighbours with atomic ORs.  Unpredictable values are gathered in bin
 * order: the staging lanes count the zero bins of their two 8-bin groups
 * (rounds 0 and 1, packed in one scan word) and rank them in bin order.
 * The word buffer is dynamic LDS sized for the largest chunk. */
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* ws,
                                                    uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, o, 64);
    x += lane >= o ? t : 0u;
  }
  if (lane == 63) ws[wave] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (uint32_t w = 0; w < kEncThreads / 64; ++w) {
    pre += w < wave ? ws[w] : 0u;
    tot += ws[w];
  }
  *total = tot;
  return pre + x - v;
}

/* at least 6 waves per SIMD (80 VGPRs): one register more costs a sixth
 * of the occupancy and about 15 % of the kernel's time */
template <bool kLong> /* kLong: some code is longer than 32 bits */
__global__ __launch_bounds__(kEncThreads, 6) void k_huff_encode(
    const uint16_t* __restrict__ codes, Chunks ch,
    const uint64_t* __restrict__ tab, int32_t lo, uint32_t tn,
    uint64_t zero_entry, const uint64_t* __restrict__ coff,
    const uint32_t* __restrict__ upre, uint16_t* __restrict__ segs,
    uint32_t* payload, uint64_t cap_words,
    float* unpred, const float* __restrict__ x, Geo g, SweepTable st,
    uint32_t* status, uint32_t* __restrict__ pack_bits) {
  constexpr uint32_t kRounds = kChunk / (8 * kEncThreads); /* 2 */
  constexpr uint32_t kSegBins = kChunk / kSegPerChunk;      /* 512 */
  extern __shared__ uint32_t words[];
  __shared__ __align__(16) uint16_t cbin[kChunk];
  __shared__ uint32_t ws[2][kEncThreads / 64];
  __shared__ uint32_t seg_end[kSegPerChunk];
  const uint32_t c = blockIdx.x;
  const uint64_t base = ch.begin(c);
  const uint32_t nsym = (uint32_t)(ch.end(c) - base);
  const uint64_t w0 = coff[c];
  const uint32_t nw = (uint32_t)(coff[c + 1] - w0);
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) words[i] = 0;
  /* staging: lane t takes the 8-bin groups m = t + 256 r; the full
   * groups' loads of both rounds are issued before either is used */
  uint32_t v[kRounds][8];
  uint32_t zpack = 0;
  uint4 qr[kRounds];
#pragma unroll
  for (uint32_t r = 0; r < kRounds; ++r) {
    const uint32_t m = threadIdx.x + r * kEncThreads;
    qr[r] = 8 * m + 8 <= nsym
                ? *reinterpret_cast<const uint4*>(codes + base + 8 * m)
                : make_uint4(0, 0, 0, 0);
  }
#pragma unroll
  for (uint32_t r = 0; r < kRounds; ++r) {
    const uint32_t m = threadIdx.x + r * kEncThreads;
    if (8 * m + 8 <= nsym) {
      const uint4 q = qr[r];
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i) v[r][i] = (w[i / 2] >> (16 * (i & 1))) & 0xffffu;
    } else {
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i)
        v[r][i] = 8 * m + i < nsym ? codes[base + 8 * m + i] : 1u;
    }
    uint32_t z = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) {
      cbin[i * kSegBins + m] = (uint16_t)v[r][i];
      z += v[r][i] == 0 ? 1u : 0u;
    }
    zpack |= z << (16 * r);
  }
  __syncthreads();
  constexpr uint32_t kLanesPerSeg = kSeg / kEncPerThread;
  static_assert(kLanesPerSeg * kEncPerThread == kSeg, "segment lanes");
  static_assert(kRounds == 2 && kSegBins == kSeg, "chunk layout");
  const uint32_t j = threadIdx.x / kLanesPerSeg;
  const uint32_t k0 = (threadIdx.x % kLanesPerSeg) * kEncPerThread;
  uint64_t ent[kEncPerThread];
  uint32_t bits = 0;
  {
    const uint4* cb = reinterpret_cast<const uint4*>(cbin + j * kSegBins + k0);
    const uint4 qa = cb[0], qb = cb[1];
    const uint32_t w[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
#pragma unroll
    for (uint32_t k = 0; k < kEncPerThread; ++k) {
      const uint32_t b = (k0 + k) * kSegPerChunk + j; /* bin in the chunk */
      const uint32_t sym = (w[k / 2] >> (16 * (k & 1))) & 0xffffu;
      ent[k] = b < nsym ? code_entry(tab, lo, tn, zero_entry, (int32_t)sym) : 0;
      bits += (uint32_t)(ent[k] & 0xff);
    }
  }
  uint32_t tot_bits, tot_z;
  const uint32_t pos0 = block_excl_scan(bits, ws[0], &tot_bits);
  const uint32_t zex = block_excl_scan(zpack, ws[1], &tot_z);
  /* payload bits of segments 0..6: the last lane of each segment knows
   * where the segment ends */
  if (threadIdx.x % kLanesPerSeg == kLanesPerSeg - 1) seg_end[j] = pos0 + bits;
  __syncthreads();
  if (threadIdx.x < kSegPerChunk - 1)
    segs[(uint64_t)c * (kSegPerChunk - 1) + threadIdx.x] = (uint16_t)(
        seg_end[threadIdx.x] - (threadIdx.x ? seg_end[threadIdx.x - 1] : 0u));
  /* This lane's bits [pos0, pos0 + bits), MSB-first.  acc holds the bits
   * not yet written in its low nacc (< 32) bits (above them: bits already
   * written, shifted out as codes come in); every complete word is ORed
   * into the zeroed chunk words (a lane's first and last words are shared
   * with its neighbours), and a code that completes no word ORs 0 into
   * the current word, so the stores need no branch. */
  {
    uint64_t acc = 0;
    uint32_t nacc = pos0 & 31u, wi = pos0 >> 5;
    auto put = [&](uint32_t code, uint32_t len) { /* len <= 32 */
      acc = (acc << len) | code;
      nacc += len;
      const bool full = nacc >= 32;
      nacc -= full ? 32u : 0u;
      atomicOr(&words[wi], full ? (uint32_t)(acc >> nacc) : 0u);
      wi += full ? 1u : 0u;
    };
#pragma unroll
    for (uint32_t k = 0; k < kEncPerThread; ++k) {
      const uint32_t len = (uint32_t)(ent[k] & 0xff);
      const uint64_t code = ent[k] >> 8;
      if (kLong && len > 32) {
        put((uint32_t)(code >> 32), len - 32);
        put((uint32_t)code, 32);
      } else {
        put((uint32_t)code, len);
      }
    }
    if (nacc) atomicOr(&words[wi], (uint32_t)(acc << (32 - nacc)));
  }
  uint32_t zr[kRounds] = {upre[c] + (zex & 0xffffu),
                          upre[c] + (tot_z & 0xffffu) + (zex >> 16)};
#pragma unroll
  for (uint32_t r = 0; r < kRounds; ++r) {
    const uint32_t m = threadIdx.x + r * kEncThreads;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i)
      if (v[r][i] == 0) {
        unpred[zr[r]] = x[point_of(st, g, base + 8 * m + i)];
        ++zr[r];
      }
  }
  __shared__ uint32_t nz_words;
  if (threadIdx.x == 0) nz_words = 0;
  __syncthreads();
  /* the chunk's size under zero-word packing (bitmap + nonzero words
   * when shorter, else raw), scanned afterwards for the packing decision
   * and the packed offsets; counted in LDS before the stores, so that no
   * barrier waits on them */
  uint32_t nz = 0;
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) nz += words[i] != 0u;
  for (uint32_t o = 32; o > 0; o >>= 1) nz += __shfl_xor(nz, o, 64);
  if ((threadIdx.x & 63u) == 0) atomicAdd(&nz_words, nz);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nbm = (nw + 31) / 32;
    pack_bits[c] = 32 * (nbm + nz_words < nw ? nbm + nz_words : nw);
  }
  bool over = false;
  for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) {
    if (w0 + i < cap_words)
      payload[w0 + i] = words[i];
    else
      over = true;
  }
  if (over) atomicOr(status, kStOverflow);
}

void launch_huff_encode(const uint16_t* codes, const Chunks& chunks,
                        const uint64_t* table, int32_t tab_lo, uint32_t tab_n,
                        uint64_t zero_entry, const uint64_t* coff,
                        const uint32_t* upre, uint16_t* segs,
                        uint32_t* payload,
                        uint64_t payload_cap_words, float* unpred,
                        const float* x, const Geo& g, const SweepTable& st,
                        uint32_t max_chunk_words, uint32_t max_len,
                        uint32_t* status, uint32_t* pack_bits, hipStream_t s) {
  const uint64_t nch = chunks.count();
  if (!nch) return;
  /* every chunk's word count is at most the largest one, which is at
   * most kEncMaxWords (codes of at most 56 bits) */
  const uint32_t mw = max_chunk_words < kEncMaxWords ? max_chunk_words
                                                     : kEncMaxWords;
  const size_t lds = 4 * ((size_t)mw + 1);
  if (max_len > 32)
    hipLaunchKernelGGL(k_huff_encode<true>, dim3((uint32_t)nch),
                       dim3(kEncThreads), lds, s, codes, chunks, table, tab_lo,
                       tab_n, zero_entry, coff, upre, segs, payload,
                       payload_cap_words, unpred, x, g, st, status, pack_bits);
  else
    hipLaunchKernelGGL(k_huff_encode<false>, dim3((uint32_t)nch),
                       dim3(kEncThreads), lds, s, codes, chunks, table, tab_lo,
                       tab_n, zero_entry, coff, upre, segs, payload,
                       payload_cap_words, unpred, x, g, st, status, pack_bits);
}

}  // namespace qoz
