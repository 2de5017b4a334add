/*
 * Huffman decoding of the chunked payload (the entropy stage of Sec. VI-A)
 * for gfx950, without any per-symbol index in the stream.
 *
 * One workgroup decodes one 4096-bin chunk at a time (persistent over
 * chunks); the chunk's words are staged in LDS and its bits are cut into
 * one subsequence per lane (at least 128 bits).  Huffman codes
 * resynchronise within a few codewords when decoding starts at an arbitrary
 * bit, which gives a parallel decoder:
 *  1. each lane walks its subsequence from the nominal first bit using code
 *     lengths only, counting codewords and symbol-0 codewords, and keeps a
 *     bitmap of the codeword starts (and symbol-0 starts) in its first 64
 *     bits;
 *  2. its true start is its predecessor's exit; walking from there stops at
 *     the first start in the bitmap (the walks coincide from then on),
 *     usually after two or three codewords, and the counts follow from
 *     population counts.  Starts are re-propagated until none changes
 *     (needed only when a subsequence did not resynchronise inside its
 *     window);
 *  3. an exclusive scan of the counts gives each lane its first bin index
 *     and unpredictable rank, and each lane decodes its codewords.
 * The walks read lengths from a 13-bit table (one byte per entry); the
 * final decode reads symbols from a 12-bit table; longer codes are sized by
 * comparing the window with the canonical code's per-length limits held in
 * registers.  Unpredictable bins also record their stream position, so the
 * exact values can be placed before the inverse sweeps.  Every read is
 * bounded by the chunk's words (zero beyond), and the stream is rejected if
 * a chunk does not end inside its words or its unpredictable count
 * disagrees with the chunk table.
 */
#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kDecWG = 256;
constexpr uint32_t kMinSubBits = 128;
constexpr uint32_t kLenBits = 13;  /* length table width */
constexpr uint32_t kSymBits = 12;  /* symbol table width */
constexpr uint32_t kRegMax = 27;   /* longest code sized from registers */
constexpr uint32_t kMaxChunkWords = kChunk * kMaxCodeLen / 32 + 2;
constexpr uint32_t kStageWords = 4096; /* chunks up to 32 bits/bin in LDS */
constexpr uint32_t kInvalidSym = 0xffffffffu;

struct DecShared {
  uint32_t words[kStageWords];
  uint8_t lz[1u << kLenBits];   /* length | 0x80 if symbol 0; 0 = longer */
  uint16_t sym[1u << kSymBits]; /* symbol of codes up to kSymBits bits */
  uint64_t first[kMaxCodeLen + 1];
  uint32_t off[kMaxCodeLen + 1];
  uint32_t start[kDecWG], exitp[kDecWG];
  uint32_t count[kDecWG], zeros[kDecWG];
  uint32_t scan_c[kDecWG], scan_z[kDecWG];
  uint32_t flag, bad;
};

/* MSB-first bit reader over words [0, nw); bits past the end read as 0. */
struct BitReader {
  const uint32_t* w;
  uint32_t nw, pos, wp;
  int nb;
  uint64_t buf;

  __device__ __forceinline__ void refill() {
    while (nb <= 32) {
      uint64_t v = wp < nw ? w[wp] : 0;
      buf |= v << (32 - nb);
      ++wp;
      nb += 32;
    }
  }
  __device__ __forceinline__ void seek(uint32_t p) {
    pos = p;
    wp = p >> 5;
    const uint32_t o = p & 31;
    uint64_t v = wp < nw ? w[wp] : 0;
    buf = (v << 32) << o;
    nb = 32 - (int)o;
    ++wp;
    refill();
  }
  __device__ __forceinline__ void advance(uint32_t len) {
    if ((int)len <= nb) {
      buf <<= len;
      nb -= (int)len;
      pos += len;
      refill();
    } else {
      seek(pos + len);
    }
  }
  /* the 64 bits at the current position, from memory */
  __device__ __forceinline__ uint64_t window() const {
    const uint32_t wi = pos >> 5, o = pos & 31;
    const uint64_t a = wi < nw ? w[wi] : 0;
    const uint64_t b = wi + 1 < nw ? w[wi + 1] : 0;
    const uint64_t c = wi + 2 < nw ? w[wi + 2] : 0;
    return (((a << 32) | b) << o) | (o ? c >> (32 - o) : 0);
  }
};

/* Top 32 bits of the canonical code's per-length limits: a window whose
 * top 32 bits are >= top[L] starts with a codeword longer than L (exact
 * for L <= 32; a limit of 2^64 is stored as 0xffffffff, which only the
 * exact fallback in long_len resolves). */
struct Limits {
  uint32_t top[kRegMax + 1];
};

/* Length of the codeword heading window V, known to be at least kFrom bits
 * long; 0 if invalid.  The register compares are exact below kRegMax; a
 * count that reaches kRegMax (a code that long, a saturated limit or an
 * invalid window) is decided again with the exact 64-bit limits. */
template <uint32_t kFrom>
__device__ __forceinline__ uint32_t long_len(uint64_t V, const Limits& lim,
                                             const DecTables* tabs,
                                             uint32_t maxlen) {
  const uint32_t top = (uint32_t)(V >> 32);
  uint32_t len = kFrom;
#pragma unroll
  for (uint32_t L = kFrom; L < kRegMax; ++L) len += top >= lim.top[L] ? 1u : 0u;
  if (len < kRegMax) return len <= maxlen ? len : maxlen;
  const uint64_t h = V >> 1;
  for (uint32_t L = kFrom; L <= maxlen; ++L)
    if (h < tabs->lim_half[L]) return tabs->cnt[L] ? L : 0;
  return 0;
}

/* Length and symbol-0 flag of the codeword at the reader.  The buffer holds
 * at least 33 valid bits: a prefix-free code decodes any length up to that
 * from it, and a longer or invalid result is decided again from memory. */
__device__ __forceinline__ uint32_t walk_len(const BitReader& br,
                                             const Limits& lim,
                                             const DecShared& sh,
                                             const DecTables* tabs,
                                             uint32_t maxlen, uint32_t zlen,
                                             uint64_t zcode, bool* zero) {
  const uint32_t e = sh.lz[(uint32_t)(br.buf >> (64 - kLenBits))];
  if (e & 0x3f) {
    *zero = (e & 0x80) != 0;
    return e & 0x3f;
  }
  uint64_t V = br.buf;
  uint32_t len = long_len<kLenBits + 1>(V, lim, tabs, maxlen);
  if (len == 0 || (int)len > br.nb) {
    V = br.window();
    len = long_len<kLenBits + 1>(V, lim, tabs, maxlen);
  }
  *zero = len && len == zlen && (V >> (64 - len)) == zcode;
  return len;
}

/* Symbol and length of the codeword at the reader. */
__device__ __forceinline__ uint32_t read_sym(const BitReader& br,
                                             const Limits& lim,
                                             const DecShared& sh,
                                             const DecTables* tabs,
                                             const uint32_t* syms,
                                             uint32_t maxlen,
                                             uint32_t* len_out) {
  const uint32_t e = sh.lz[(uint32_t)(br.buf >> (64 - kLenBits))];
  uint32_t len = e & 0x3f;
  if (len && len <= kSymBits) {
    *len_out = len;
    return sh.sym[(uint32_t)(br.buf >> (64 - kSymBits))];
  }
  uint64_t V = br.buf;
  if (!len) {
    len = long_len<kLenBits + 1>(V, lim, tabs, maxlen);
    if (len == 0 || (int)len > br.nb) {
      V = br.window();
      len = long_len<kLenBits + 1>(V, lim, tabs, maxlen);
    }
  }
  *len_out = len;
  if (!len) return kInvalidSym;
  const uint64_t r = (V >> (64 - len)) - sh.first[len];
  if (r >= tabs->cnt[len]) return kInvalidSym; /* past the last code */
  return syms[sh.off[len] + (uint32_t)r];
}

__device__ __forceinline__ void block_exclusive_scan2(uint32_t* a, uint32_t* b,
                                                      uint32_t va,
                                                      uint32_t vb,
                                                      uint32_t* ea,
                                                      uint32_t* eb,
                                                      uint32_t* ta) {
  a[threadIdx.x] = va;
  b[threadIdx.x] = vb;
  __syncthreads();
  for (uint32_t o = 1; o < kDecWG; o <<= 1) {
    uint32_t xa = threadIdx.x >= o ? a[threadIdx.x - o] : 0;
    uint32_t xb = threadIdx.x >= o ? b[threadIdx.x - o] : 0;
    __syncthreads();
    a[threadIdx.x] += xa;
    b[threadIdx.x] += xb;
    __syncthreads();
  }
  *ea = a[threadIdx.x] - va;
  *eb = b[threadIdx.x] - vb;
  *ta = a[kDecWG - 1];
  __syncthreads();
}

__global__ __launch_bounds__(kDecWG) void k_huff_decode(
    const uint32_t* __restrict__ payload, uint64_t n_words,
    const uint64_t* __restrict__ coff, const uint32_t* __restrict__ upre,
    uint64_t n_chunks, uint64_t n_codes, uint64_t n_unpred,
    const DecTables* __restrict__ tabs, const uint32_t* __restrict__ syms,
    uint16_t* __restrict__ codes, uint32_t* __restrict__ upos,
    uint32_t* status) {
  __shared__ DecShared sh;
  /* Length table from the canonical limits: for L <= kLenBits the limit is
   * a multiple of 2^(64 - kLenBits), so the first kLenBits bits decide it
   * exactly.  Symbol 0 is flagged from its own code. */
  const uint32_t zlen = tabs->zlen;
  const uint64_t zcode = tabs->zcode;
  for (uint32_t i = threadIdx.x; i < (1u << kLenBits); i += kDecWG) {
    const uint64_t h = (uint64_t)i << (63 - kLenBits);
    uint32_t len = 0;
    for (uint32_t L = 1; L <= kLenBits; ++L)
      if (h < tabs->lim_half[L]) {
        len = tabs->cnt[L] ? L : 0;
        break;
      }
    const bool z = len && len == zlen && (i >> (kLenBits - len)) == zcode;
    sh.lz[i] = (uint8_t)(len | (z ? 0x80u : 0u));
  }
  for (uint32_t i = threadIdx.x; i < (1u << kSymBits); i += kDecWG)
    sh.sym[i] = (uint16_t)(tabs->lut[i] >> 8);
  for (uint32_t i = threadIdx.x; i <= (uint32_t)kMaxCodeLen; i += kDecWG) {
    sh.first[i] = tabs->first[i];
    sh.off[i] = tabs->off[i];
  }
  const uint32_t maxlen = tabs->maxlen;
  Limits lim;
#pragma unroll
  for (uint32_t L = 0; L <= kRegMax; ++L) {
    const uint64_t h = tabs->lim_half[L];
    lim.top[L] = h >= (1ull << 63) ? 0xffffffffu : (uint32_t)(h >> 31);
  }
  if (threadIdx.x == 0) sh.bad = 0;
  __syncthreads();

  for (uint64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    /* chunk tables (uniform across the workgroup) */
    const uint64_t w0 = coff[c], w1 = coff[c + 1];
    const uint32_t u0 = upre[c], u1 = upre[c + 1];
    const bool last = c + 1 == n_chunks;
    if (w0 > w1 || w1 > n_words || (c == 0 && w0 != 0) || u0 > u1 ||
        u1 > n_unpred || w1 - w0 > kMaxChunkWords || w1 == w0 ||
        (last && (w1 != n_words || u1 != n_unpred))) {
      if (threadIdx.x == 0) sh.bad = 1;
      continue;
    }
    const uint32_t nw = (uint32_t)(w1 - w0);
    const uint64_t base = c * kChunk;
    const uint32_t nsym =
        (uint32_t)(n_codes - base < kChunk ? n_codes - base : kChunk);
    BitReader br;
    br.nw = nw;
    if (nw <= kStageWords) {
      for (uint32_t k = threadIdx.x; k < nw; k += kDecWG)
        sh.words[k] = payload[w0 + k];
      br.w = sh.words;
    } else {
      br.w = payload + w0;
    }
    const uint32_t nbits = nw * 32;
    uint32_t sub = (nbits + kDecWG - 1) / kDecWG;
    sub = sub < kMinSubBits ? kMinSubBits : sub;
    const uint32_t nsub = (nbits + sub - 1) / sub;
    const uint32_t i = threadIdx.x;
    const bool mine = i < nsub;
    const uint32_t s_lo = i * sub;
    const uint32_t s_hi = mine ? (s_lo + sub < nbits ? s_lo + sub : nbits) : 0;
    __syncthreads();

    /* 1: walk from the nominal start */
    uint64_t bmap = 0, zmap = 0;
    uint32_t spec_n = 0, spec_z = 0, spec_exit = 0;
    if (mine) {
      br.seek(s_lo);
      while (br.pos < s_hi) {
        const uint32_t rel = br.pos - s_lo;
        bool zero;
        uint32_t len =
            walk_len(br, lim, sh, tabs, maxlen, zlen, zcode, &zero);
        if (!len) len = 1;
        if (rel < 64) {
          bmap |= 1ull << rel;
          if (zero) zmap |= 1ull << rel;
        }
        spec_z += zero ? 1u : 0u;
        ++spec_n;
        br.advance(len);
      }
      spec_exit = br.pos;
      sh.start[i] = s_lo;
      sh.exitp[i] = spec_exit;
      sh.count[i] = spec_n;
      sh.zeros[i] = spec_z;
    }
    if (threadIdx.x == 0) sh.flag = 0;
    __syncthreads();

    /* 2: true starts from the predecessors' exits */
    for (uint32_t it = 0; it <= nsub; ++it) {
      const uint32_t want = i > 0 && mine ? sh.exitp[i - 1] : 0;
      __syncthreads();
      if (mine && want != sh.start[i]) {
        uint32_t n = 0, z = 0, ex = 0;
        bool synced = false;
        br.seek(want);
        while (br.pos < s_hi) {
          const uint32_t rel = br.pos - s_lo;
          if (rel < 64 && ((bmap >> rel) & 1)) {
            const uint64_t before = (1ull << rel) - 1;
            n += spec_n - (uint32_t)__popcll(bmap & before);
            z += spec_z - (uint32_t)__popcll(zmap & before);
            ex = spec_exit;
            synced = true;
            break;
          }
          bool zero;
          uint32_t len =
              walk_len(br, lim, sh, tabs, maxlen, zlen, zcode, &zero);
          if (!len) len = 1;
          z += zero ? 1u : 0u;
          ++n;
          br.advance(len);
        }
        if (!synced) ex = br.pos;
        sh.start[i] = want;
        sh.exitp[i] = ex;
        sh.count[i] = n;
        sh.zeros[i] = z;
        sh.flag = 1;
      }
      __syncthreads();
      const bool again = sh.flag != 0;
      __syncthreads();
      if (threadIdx.x == 0) sh.flag = 0;
      __syncthreads();
      if (!again) break;
    }

    /* 3: offsets, then the final decode straight to the bin array */
    uint32_t off_n, off_z, tot_n;
    block_exclusive_scan2(sh.scan_c, sh.scan_z, mine ? sh.count[i] : 0,
                          mine ? sh.zeros[i] : 0, &off_n, &off_z, &tot_n);
    bool bad = tot_n < nsym;
    uint32_t valid_zeros = 0;
    if (mine && !bad) {
      br.seek(sh.start[i]);
      const uint32_t n = sh.count[i];
      for (uint32_t k = 0; k < n && off_n < nsym; ++k, ++off_n) {
        uint32_t len;
        const uint32_t s = read_sym(br, lim, sh, tabs, syms, maxlen, &len);
        if (s == kInvalidSym) {
          bad = true;
          break;
        }
        codes[base + off_n] = (uint16_t)s;
        if (s == 0) {
          const uint32_t rank = u0 + off_z;
          if (rank < u1) upos[rank] = (uint32_t)(base + off_n);
          ++off_z;
          ++valid_zeros;
        }
        br.advance(len);
        if (off_n + 1 == nsym && br.pos > nbits) bad = true;
      }
    }
    if (bad) sh.bad = 1;
    sh.scan_c[threadIdx.x] = valid_zeros;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t z = 0;
      for (uint32_t t = 0; t < kDecWG; ++t) z += sh.scan_c[t];
      if (z != u1 - u0) sh.bad = 1;
    }
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0 && sh.bad) atomicOr(status, kStBadStream);
}

void launch_huff_decode(const uint32_t* payload, uint64_t n_words,
                        const uint64_t* coff, const uint32_t* upre,
                        uint64_t n_chunks, uint64_t n_codes,
                        uint64_t n_unpred, const DecTables* tabs,
                        const uint32_t* syms, uint16_t* codes,
                        uint32_t* upos, uint32_t* status, hipStream_t s) {
  if (!n_chunks) return;
  uint64_t blocks = n_chunks < 1024 ? n_chunks : 1024; /* 4 per CU */
  hipLaunchKernelGGL(k_huff_decode, dim3((uint32_t)blocks), dim3(kDecWG), 0,
                     s, payload, n_words, coff, upre, n_chunks, n_codes,
                     n_unpred, tabs, syms, codes, upos, status);
}

}  // namespace qoz
