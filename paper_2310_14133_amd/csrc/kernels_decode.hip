/*
 * Huffman decoding of the chunked payload (the entropy stage of Sec. VI-A)
 * for gfx950, without any per-symbol index in the stream.
 *
 * One workgroup decodes one 4096-bin chunk at a time (persistent over
 * chunks); the chunk's words are staged in LDS.  The chunk's bits are cut
 * into one subsequence per lane (at least 128 bits each).  Huffman codes
 * resynchronise within a few codewords when decoding starts at an arbitrary
 * bit, which gives a parallel decoder:
 *  1. every subsequence is decoded from its nominal first bit, counting the
 *     codewords that start inside it and recording which bit positions of
 *     its first 64 bits start a codeword (and which of those are symbol 0);
 *  2. its true start is its predecessor's exit; decoding from there stops
 *     at the first recorded boundary (the paths coincide from then on), so
 *     counts follow from population counts -- usually after two or three
 *     codewords.  Starts are re-propagated until none changes (only needed
 *     when a subsequence did not resynchronise inside its window);
 *  3. an exclusive scan of the counts gives each subsequence's first bin;
 *     a last decode writes the bins into LDS, which is stored coalesced.
 * Decoding uses a two-level table (11 bits, then up to 10 more); codes the
 * tables do not cover come from per-length limits of the canonical code.
 * Unpredictable bins (symbol 0) also record their stream position, so the
 * exact values can be placed before the inverse sweeps.  Every read is
 * bounded by the chunk's words (zero beyond), and the stream is rejected if
 * a chunk does not end inside its words or its unpredictable count
 * disagrees with the chunk table.
 */
#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kDecWG = 256;
constexpr uint32_t kMinSubBits = 128;
constexpr uint32_t kL1Bits = 11;
constexpr uint32_t kSubCap = 2048;
constexpr uint32_t kMaxChunkWords = kChunk * kMaxCodeLen / 32 + 2;
constexpr uint32_t kStageWords = 4096; /* chunks up to 32 bits/bin in LDS */
constexpr uint32_t kInvalidSym = 0xffffffffu;

struct DecShared {
  uint32_t words[kStageWords];
  uint32_t l1[1u << kL1Bits];
  uint32_t sub[kSubCap];
  uint16_t out[kChunk];
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
  /* the 64 bits at the current position, from memory */
  __device__ __forceinline__ uint64_t window64() const {
    const uint32_t wi = pos >> 5, o = pos & 31;
    const uint64_t a = wi < nw ? w[wi] : 0;
    const uint64_t b = wi + 1 < nw ? w[wi + 1] : 0;
    const uint64_t c = wi + 2 < nw ? w[wi + 2] : 0;
    return (((a << 32) | b) << o) | (o ? c >> (32 - o) : 0);
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
};

/* Codes the tables do not cover: the length is the smallest L whose
 * canonical limit exceeds the window.  Returns 0 if invalid. */
__device__ __noinline__ uint32_t slow_code(const BitReader& br,
                                           const DecTables* tabs,
                                           const uint32_t* syms,
                                           uint32_t* sym) {
  const uint64_t h = br.window64() >> 1;
  const uint32_t maxlen = tabs->maxlen;
  for (uint32_t L = 1; L <= maxlen; ++L) {
    if (h < tabs->lim_half[L]) {
      if (!tabs->cnt[L]) return 0;
      const uint64_t v = (h << 1) >> (64 - L);
      const uint64_t k = v - tabs->first[L];
      if (k >= tabs->cnt[L]) return 0;
      *sym = syms[tabs->off[L] + (uint32_t)k];
      return L;
    }
  }
  return 0;
}

/* Decode the codeword at the reader; returns its length (advancing) and
 * symbol (kInvalidSym for an invalid prefix, which advances one bit). */
__device__ __forceinline__ uint32_t decode_one(BitReader& br,
                                               const DecShared& sh,
                                               const DecTables* tabs,
                                               const uint32_t* syms) {
  const uint32_t e = sh.l1[(uint32_t)(br.buf >> (64 - kL1Bits))];
  const uint32_t lb = e & 0xff;
  uint32_t len = 0, sym = kInvalidSym;
  if (lb && !(lb & 0x80u)) {
    len = lb;
    sym = e >> 8;
  } else if (lb & 0x80u) {
    const uint32_t sb = lb & 0x7fu;
    const uint32_t e2 =
        sh.sub[(e >> 8) + (uint32_t)((br.buf << kL1Bits) >> (64 - sb))];
    if (e2) {
      len = kL1Bits + (e2 & 0xff);
      sym = e2 >> 8;
    }
  }
  if (!len) {
    len = slow_code(br, tabs, syms, &sym);
    if (!len) {
      len = 1;
      sym = kInvalidSym;
    }
  }
  br.advance(len);
  return sym;
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
  for (uint32_t i = threadIdx.x; i < (1u << kL1Bits); i += kDecWG)
    sh.l1[i] = tabs->l1[i];
  const uint32_t n_sub = tabs->n_sub;
  for (uint32_t i = threadIdx.x; i < n_sub; i += kDecWG) sh.sub[i] = tabs->sub[i];
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

    /* 1: speculative decode from the nominal start, with the boundary and
     * zero-symbol maps of the first 64 bits */
    uint64_t bmap = 0, zmap = 0;
    uint32_t spec_n = 0, spec_z = 0, spec_exit = 0;
    if (mine) {
      br.seek(s_lo);
      while (br.pos < s_hi) {
        const uint32_t rel = br.pos - s_lo;
        const uint32_t s = decode_one(br, sh, tabs, syms);
        if (rel < 64) {
          bmap |= 1ull << rel;
          if (s == 0) zmap |= 1ull << rel;
        }
        spec_z += s == 0 ? 1u : 0u;
        ++spec_n;
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
          const uint32_t s = decode_one(br, sh, tabs, syms);
          z += s == 0 ? 1u : 0u;
          ++n;
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

    /* 3: offsets, then the final decode into LDS */
    uint32_t off_n, off_z, tot_n;
    block_exclusive_scan2(sh.scan_c, sh.scan_z, mine ? sh.count[i] : 0,
                          mine ? sh.zeros[i] : 0, &off_n, &off_z, &tot_n);
    bool bad = tot_n < nsym;
    uint32_t valid_zeros = 0;
    if (mine && !bad) {
      br.seek(sh.start[i]);
      const uint32_t n = sh.count[i];
      for (uint32_t k = 0; k < n && off_n < nsym; ++k, ++off_n) {
        const uint32_t s = decode_one(br, sh, tabs, syms);
        if (s == kInvalidSym) {
          bad = true;
          break;
        }
        sh.out[off_n] = (uint16_t)s;
        if (s == 0) {
          const uint32_t rank = u0 + off_z;
          if (rank < u1) upos[rank] = (uint32_t)(base + off_n);
          ++off_z;
          ++valid_zeros;
        }
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
    for (uint32_t k = threadIdx.x; k < nsym; k += kDecWG)
      codes[base + k] = sh.out[k];
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
  uint64_t blocks = n_chunks < 768 ? n_chunks : 768; /* 3 per CU */
  hipLaunchKernelGGL(k_huff_decode, dim3((uint32_t)blocks), dim3(kDecWG), 0,
                     s, payload, n_words, coff, upre, n_chunks, n_codes,
                     n_unpred, tabs, syms, codes, upos, status);
}

}  // namespace qoz
