/*
 * Zero-word packing of the Huffman payload (stream format 5), the
 * project's lossless stage after Huffman coding: runs of the zero bin,
 * whose canonical code is all zero bits, leave whole payload words at
 * zero.  A chunk of n raw words is stored, when shorter, as a bitmap of
 * ceil(n / 32) words (bit i of bitmap word k, least significant first,
 * set when raw word 32 k + i is nonzero) followed by its nonzero words.
 *
 * One wave per chunk, 64 words per step: a ballot of the nonzero flags is
 * two bitmap words, and each nonzero word's place is the count of set
 * bits below it plus those of the earlier steps.
 */
#include <hip/hip_runtime.h>

#include "qoz_internal.h"

namespace qoz {

namespace {
constexpr uint32_t kPackThreads = 256;
constexpr uint32_t kPackWaves = kPackThreads / 64;

__device__ __forceinline__ uint32_t lanes_below(uint64_t m, uint32_t lane) {
  return (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}
}  // namespace

__global__ __launch_bounds__(kPackThreads) void k_pack_write(
    const uint32_t* __restrict__ raw, const uint64_t* __restrict__ coff,
    const uint64_t* __restrict__ pcoff, uint64_t nch,
    uint32_t* __restrict__ dst) {
  const uint64_t c = (uint64_t)blockIdx.x * kPackWaves + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (c >= nch) return;
  const uint64_t r0 = coff[c], n = coff[c + 1] - r0;
  const uint64_t p0 = pcoff[c], p = pcoff[c + 1] - p0;
  if (p == n) {
    for (uint64_t i = lane; i < n; i += 64) dst[p0 + i] = raw[r0 + i];
    return;
  }
  const uint64_t nbm = (n + 31) / 32;
  uint64_t run = 0;
  for (uint64_t b = 0; b < n; b += 64) {
    const uint64_t i = b + lane;
    const uint32_t w = i < n ? raw[r0 + i] : 0u;
    const uint64_t m = __ballot(w != 0u);
    if (lane == 0) dst[p0 + b / 32] = (uint32_t)m;
    if (lane == 1 && b / 32 + 1 < nbm) dst[p0 + b / 32 + 1] = (uint32_t)(m >> 32);
    if (w) dst[p0 + nbm + run + lanes_below(m, lane)] = w;
    run += (uint64_t)__popcll(m);
  }
}

/* Expands the packed payload of every chunk into raw[coff[c]..coff[c+1]);
 * offsets or bitmaps that do not fit the stream set kStBadStream and the
 * chunk is left alone (every access stays inside src[0..n_packed) and
 * raw[0..n_words)). */
__global__ __launch_bounds__(kPackThreads) void k_unpack(
    const uint32_t* __restrict__ src, uint64_t n_packed,
    const uint64_t* __restrict__ coff, const uint64_t* __restrict__ pcoff,
    uint64_t nch, uint64_t n_words, uint32_t* __restrict__ raw,
    uint32_t* status) {
  const uint64_t c = (uint64_t)blockIdx.x * kPackWaves + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (c >= nch) return;
  const uint64_t r0 = coff[c], r1 = coff[c + 1];
  const uint64_t p0 = pcoff[c], p1 = pcoff[c + 1];
  bool bad = r1 < r0 || r1 > n_words || p1 < p0 || p1 > n_packed ||
             (c == 0 && (p0 != 0 || r0 != 0)) ||
             (c + 1 == nch && p1 != n_packed);
  const uint64_t n = bad ? 0 : r1 - r0, p = bad ? 0 : p1 - p0;
  bad = bad || p > n;
  const uint64_t nbm = (n + 31) / 32;
  bad = bad || (p < n && p < nbm);
  if (bad) {
    if (lane == 0) atomicOr(status, kStBadStream);
    return;
  }
  if (p == n) {
    for (uint64_t i = lane; i < n; i += 64) raw[r0 + i] = src[p0 + i];
    return;
  }
  const uint64_t nnz = p - nbm;
  uint64_t run = 0;
  bool err = false;
  for (uint64_t b = 0; b < n; b += 64) {
    const uint64_t k = b / 32 + (lane >= 32 ? 1 : 0);
    const uint32_t bw = k < nbm ? src[p0 + k] : 0u;
    const uint64_t i = b + lane;
    const bool bit = (bw >> (lane & 31u)) & 1u;
    const uint64_t m = __ballot(bit);
    const uint64_t at = run + lanes_below(m, lane);
    uint32_t w = 0;
    if (bit) {
      if (i >= n || at >= nnz)
        err = true;
      else
        w = src[p0 + nbm + at];
    }
    if (i < n) raw[r0 + i] = w;
    run += (uint64_t)__popcll(m);
  }
  err = err || run != nnz;
  if (err) atomicOr(status, kStBadStream);
}

void launch_pack_write(const uint32_t* raw, const uint64_t* coff,
                       const uint64_t* pcoff, uint64_t n_chunks,
                       uint32_t* dst, hipStream_t s) {
  if (!n_chunks) return;
  const uint64_t blocks = (n_chunks + kPackWaves - 1) / kPackWaves;
  QOZ_LAUNCH(k_pack_write, dim3((uint32_t)blocks), dim3(kPackThreads),
                     0, s, raw, coff, pcoff, n_chunks, dst);
}

void launch_unpack(const uint32_t* src, uint64_t n_packed,
                   const uint64_t* coff, const uint64_t* pcoff,
                   uint64_t n_chunks, uint64_t n_words, uint32_t* raw,
                   uint32_t* status, hipStream_t s) {
  if (!n_chunks) return;
  const uint64_t blocks = (n_chunks + kPackWaves - 1) / kPackWaves;
  QOZ_LAUNCH(k_unpack, dim3((uint32_t)blocks), dim3(kPackThreads), 0,
                     s, src, n_packed, coff, pcoff, n_chunks, n_words, raw,
                     status);
}

}  // namespace qoz
