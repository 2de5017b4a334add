/*
 * Huffman decoding of the chunked payload (the entropy stage of Sec. VI-A)
 * for gfx950.
 *
 * A chunk of 4096 bins is stored as eight segments of 512 bins whose bit
 * lengths the stream keeps, so every segment decodes on its own: one lane
 * per segment, eight lanes per chunk, a wave covers eight consecutive
 * chunks.  Each lane keeps its next payload words in a 16-word ring in LDS
 * (word k of every lane's ring in one LDS row, so a wave's reads fall in
 * distinct banks) and the two words under its read position in registers:
 * the next 32 bits of the segment are one funnel shift of that pair.  Each
 * codeword costs one lookup in a 12-bit table in LDS that gives its length,
 * its symbol and whether it is symbol 0; when the position crosses a word,
 * the pair advances by the ring word read alongside the lookup.  Global
 * loads happen only at the ends of 8-bin groups, where a lane that has used
 * half its ring fetches the next eight words into registers and, one group
 * later, writes them over the used half.  Codes longer than 12 bits are
 * sized by comparing the 32-bit window with the canonical code's
 * per-length limits (held in registers) and mapped to their symbol through
 * the canonical order.  Bins are written eight at a time (16-byte stores).
 * Symbol-0 bins (unpredictable values) are ranked by a scan over the
 * chunk's eight lanes, only in groups where a lane of the wave met one, and
 * their stream positions go to `upos`, so the exact values can be placed
 * before the inverse sweeps.
 *
 * Every payload read is bounded by the chunk's words (zero beyond).  The
 * stream is rejected if a chunk table entry is inconsistent, a segment does
 * not end where the segment table says (the last one: inside the chunk's
 * words), a codeword is invalid, or a chunk's symbol-0 count disagrees with
 * the chunk table.
 */
#include <mutex>

#include "qoz_device.h"
#include "qoz_internal.h"

namespace qoz {

constexpr uint32_t kDecWG = 640; /* 10 waves: 80 chunks */
constexpr uint32_t kChunksPerWG = kDecWG / kSegPerChunk;
constexpr uint32_t kRegMax = 20; /* longest code sized from registers */
constexpr uint32_t kMaxChunkWords = kChunk * kMaxCodeLen / 32 + 2;
constexpr uint32_t kSortedLds = 1024; /* canonical symbols kept in LDS */
constexpr uint32_t kRing = 16;        /* payload words per lane in LDS */
constexpr uint32_t kHalf = kRing / 2;
constexpr uint32_t kInvalid = 0xffffffffu;
constexpr uint32_t kEntZero = 0x40u; /* DecTables::ent: symbol 0's code */

struct DecShared {
  uint32_t ring[kRing][kDecWG];
  /* per chunk, the 64 bins of the group being decoded, in bin order */
  __align__(16) uint16_t tb[kChunksPerWG][64];
  uint32_t ent[1u << kSymBits]; /* DecTables::ent */
  uint32_t ent2[kEnt2];         /* DecTables::ent2 */
  uint16_t sorted[kSortedLds];
  uint64_t first[kMaxCodeLen + 1];
  uint64_t lim_half[kMaxCodeLen + 1]; /* DecTables::lim_half */
  uint32_t off[kMaxCodeLen + 1];
  uint32_t cnt[kMaxCodeLen + 1];
};

/* Top 32 bits of the canonical code's per-length limits: a window whose
 * top 32 bits are >= top[L] starts with a codeword longer than L (exact
 * for L <= 32; a limit of 2^64 is stored as 0xffffffff, which only the
 * exact fallback in slow_symbol resolves). */
struct Limits {
  uint32_t top[kRegMax + 1];
};

/* four payload words; a word-aligned 16-byte load */
struct __attribute__((aligned(4))) Quad {
  uint32_t x, y, z, w;
};

/* The words of one chunk, zero past its end; `room` is the number of
 * payload words from the chunk start to the end of the payload, so a block
 * below it can be read with wide loads. */
struct Words {
  const uint32_t* w;
  uint32_t nw, room;
  __device__ __forceinline__ uint32_t operator()(uint32_t i) const {
    return i < nw ? w[i] : 0u;
  }
  /* words i .. i + 4n - 1 into v, unmasked: words at or past nw are
   * whatever follows the chunk (the caller masks them when it uses them,
   * so the loads stay in flight until then) */
  template <uint32_t n>
  __device__ __forceinline__ void raw_block(uint32_t i, uint32_t* v) const {
    if (i + 4 * n <= room) {
#pragma unroll
      for (uint32_t k = 0; k < n; ++k) {
        const Quad q = *reinterpret_cast<const Quad*>(w + i + 4 * k);
        v[4 * k] = q.x;
        v[4 * k + 1] = q.y;
        v[4 * k + 2] = q.z;
        v[4 * k + 3] = q.w;
      }
    } else {
#pragma unroll
      for (uint32_t k = 0; k < 4 * n; ++k) v[k] = (*this)(i + k);
    }
  }
  /* words i .. i + 4n - 1 into v */
  template <uint32_t n>
  __device__ __forceinline__ void block(uint32_t i, uint32_t* v) const {
    if (i + 4 * n <= room) {
#pragma unroll
      for (uint32_t k = 0; k < n; ++k) {
        const Quad q = *reinterpret_cast<const Quad*>(w + i + 4 * k);
        v[4 * k] = i + 4 * k < nw ? q.x : 0u;
        v[4 * k + 1] = i + 4 * k + 1 < nw ? q.y : 0u;
        v[4 * k + 2] = i + 4 * k + 2 < nw ? q.z : 0u;
        v[4 * k + 3] = i + 4 * k + 3 < nw ? q.w : 0u;
      }
    } else {
#pragma unroll
      for (uint32_t k = 0; k < 4 * n; ++k) v[k] = (*this)(i + k);
    }
  }
};

/* One lane's reader.  a and b are words wp - 2 and wp - 1 of the chunk;
 * the next 32 bits of the segment are ((a:b) >> so)[31:0] (so in [0, 31]),
 * i.e. the read position is 32 (wp - 1) - so.  The ring holds words
 * [B, B + kRing); pf holds words [B + kRing, B + kRing + kHalf), always in
 * flight.  Consuming up to 32 bits takes at most one word from the ring
 * (word wp), and the group end slides the ring whenever wp - B >= kHalf, so
 * wp - B <= 7 when a group starts and every ring read in its eight steps
 * is of a word the ring holds.  The prefetched words are masked to the
 * chunk only when they enter the ring, so their loads overlap the groups
 * decoded meanwhile instead of stalling the wave at issue. */
struct Reader {
  uint32_t a, b, so, wp, B;
  bool pending;
  uint32_t pf[kHalf];

  __device__ __forceinline__ uint32_t pos() const { return (wp - 1) * 32 - so; }
  __device__ __forceinline__ uint32_t window() const {
    return __builtin_amdgcn_alignbit(a, b, so);
  }
  __device__ __forceinline__ void seek(DecShared& sh, const Words& W,
                                       uint32_t p) {
    const uint32_t wi = p >> 5, o = p & 31;
    /* four words at a time (few registers: seeks are rare) */
    uint32_t v0 = 0, v1 = 0;
#pragma unroll 1
    for (uint32_t k = 0; k < kRing; k += 4) {
      uint32_t v[4];
      W.block<1>(wi + k, v);
      for (uint32_t i = 0; i < 4; ++i)
        sh.ring[(wi + k + i) % kRing][threadIdx.x] = v[i];
      if (k == 0) {
        v0 = v[0];
        v1 = v[1];
      }
    }
    W.raw_block<kHalf / 4>(wi + kRing, pf);
    if (o) { /* position o of word wi: the pair (wi, wi + 1) */
      a = v0;
      b = v1;
      wp = wi + 2;
      so = 32 - o;
    } else { /* the start of word wi: the pair (wi - 1, wi) */
      a = 0;
      b = v0;
      wp = wi + 1;
      so = 0;
    }
    B = wi;
    pending = true;
  }
  /* the 64 bits at the read position, from memory */
  /* the 64 bits from the read position: the window and the 32 bits after
   * it, from b and word wp (which the ring holds during a group) */
  __device__ __forceinline__ uint64_t window64(const DecShared& sh) const {
    const uint32_t c = sh.ring[wp % kRing][threadIdx.x];
    return ((uint64_t)__builtin_amdgcn_alignbit(a, b, so) << 32) |
           __builtin_amdgcn_alignbit(b, c, so);
  }
  /* move the read position by len <= 32 bits; nx is word wp */
  __device__ __forceinline__ void advance(uint32_t len, uint32_t nx) {
    const int t = (int)so - (int)len;
    const bool need = t < 0;
    a = need ? b : a;
    b = need ? nx : b;
    wp += need ? 1u : 0u;
    so = (uint32_t)t & 31u;
  }
  /* end of an 8-bin group: once the first half of the ring is used, move
   * the fetched words over it; keep the next half always in flight */
  __device__ __forceinline__ void group_end(DecShared& sh, const Words& W) {
    if (pending && wp >= B + kHalf) {
      /* pf holds words B + kRing + k, loaded unmasked: zero past the
       * chunk's words here, where the loads are first needed */
#pragma unroll
      for (uint32_t k = 0; k < kHalf; ++k)
        sh.ring[(B + k) % kRing][threadIdx.x] =
            B + kRing + k < W.nw ? pf[k] : 0u;
      B += kHalf;
      pending = false;
    }
    if (!pending) {
      W.raw_block<kHalf / 4>(B + kRing, pf);
      pending = true;
    }
  }
};

/* Symbol and length of a codeword the table does not resolve (longer than
 * kSymBits bits, or invalid): kInvalid if invalid.  top is the 32-bit
 * window at the read position. */
__device__ __forceinline__ uint32_t slow_symbol(
    const Reader& rd, const Words& W, uint32_t top, const Limits& lim,
    const DecShared& sh, const DecTables* __restrict__ tabs,
    const uint32_t* __restrict__ syms, uint32_t maxlen, uint32_t* len_out) {
  uint32_t len = kSymBits + 1;
#pragma unroll
  for (uint32_t L = kSymBits + 1; L < kRegMax; ++L)
    len += top >= lim.top[L] ? 1u : 0u;
  uint64_t r;
  if (len < kRegMax) {
    len = len <= maxlen ? len : maxlen;
    r = (uint64_t)(top >> (32 - len));
  } else { /* a code of kRegMax bits or more, or a saturated limit */
    const uint64_t V = rd.window64(sh);
    const uint64_t h = V >> 1;
    /* the number of lengths the code is longer than (the limits do not
     * decrease with L): independent loads, one LDS latency */
    len = kSymBits + 1;
    for (uint32_t L = kSymBits + 1; L < maxlen; ++L)
      len += h >= sh.lim_half[L] ? 1u : 0u;
    if (!sh.cnt[len]) return kInvalid;
    r = V >> (64 - len);
  }
  r -= sh.first[len];
  if (r >= sh.cnt[len]) return kInvalid; /* past the last code */
  const uint32_t k = sh.off[len] + (uint32_t)r;
  *len_out = len;
  return k < kSortedLds ? (uint32_t)sh.sorted[k] : syms[k];
}

__device__ __forceinline__ uint32_t group_or(uint32_t v) {
#pragma unroll
  for (uint32_t o = 1; o < kSegPerChunk; o <<= 1)
    v |= __shfl_xor(v, o, kSegPerChunk);
  return v;
}

__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v, uint32_t j) {
#pragma unroll
  for (uint32_t o = 1; o < kSegPerChunk; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, kSegPerChunk);
    v += j >= o ? t : 0u;
  }
  return v;
}

/* Workgroup wg of a stream's decoding: its chunks wg * kChunksPerWG on. */
__device__ __forceinline__ void decode_wg(
    DecShared& sh, const uint32_t* __restrict__ payload, uint64_t n_words,
    const uint64_t* __restrict__ coff, const uint32_t* __restrict__ upre,
    const uint16_t* __restrict__ segs, const Chunks& ch,
    uint64_t n_unpred, const DecTables* __restrict__ tabs,
    const uint32_t* __restrict__ syms, uint16_t* __restrict__ codes,
    uint32_t* __restrict__ upos, uint32_t* status, uint32_t wg) {
  {
    const uint4* src = reinterpret_cast<const uint4*>(tabs->ent);
    uint4* dst = reinterpret_cast<uint4*>(sh.ent);
    for (uint32_t i = threadIdx.x; i < sizeof(sh.ent) / 16; i += kDecWG)
      dst[i] = src[i];
    const uint4* src2 = reinterpret_cast<const uint4*>(tabs->ent2);
    uint4* dst2 = reinterpret_cast<uint4*>(sh.ent2);
    for (uint32_t i = threadIdx.x; i < sizeof(sh.ent2) / 16; i += kDecWG)
      dst2[i] = src2[i];
  }
  /* the canonical symbols a valid code can index (k < n_used) */
  const uint32_t n_used = tabs->n_used;
  const uint32_t n_sorted = n_used < kSortedLds ? n_used : kSortedLds;
  for (uint32_t i = threadIdx.x; i < n_sorted; i += kDecWG)
    sh.sorted[i] = (uint16_t)syms[i];
  for (uint32_t i = threadIdx.x; i <= (uint32_t)kMaxCodeLen; i += kDecWG) {
    sh.first[i] = tabs->first[i];
    sh.off[i] = tabs->off[i];
    sh.cnt[i] = tabs->cnt[i];
    sh.lim_half[i] = tabs->lim_half[i];
  }
  const uint32_t maxlen = tabs->maxlen;
  Limits lim;
#pragma unroll
  for (uint32_t L = 0; L <= kRegMax; ++L) {
    const uint64_t h = tabs->lim_half[L];
    lim.top[L] = h >= (1ull << 63) ? 0xffffffffu : (uint32_t)(h >> 31);
  }
  __syncthreads();

  /* this lane's chunk and segment */
  const uint32_t j = threadIdx.x % kSegPerChunk;
  const uint64_t c = (uint64_t)wg * kChunksPerWG + threadIdx.x / kSegPerChunk;
  const uint64_t n_chunks = ch.count();
  const bool have = c < n_chunks;
  bool bad = false;
  uint64_t w0 = 0, w1 = 0;
  uint32_t u0 = 0, u1 = 0, d = 0, nsym = 0;
  if (have) {
    w0 = coff[c];
    w1 = coff[c + 1];
    u0 = upre[c];
    u1 = upre[c + 1];
    const bool last = c + 1 == n_chunks;
    bad = w0 > w1 || w1 > n_words || (c == 0 && (w0 != 0 || u0 != 0)) ||
          u0 > u1 || u1 > n_unpred || w1 - w0 > kMaxChunkWords || w1 == w0 ||
          (last && (w1 != n_words || u1 != n_unpred));
    nsym = (uint32_t)(ch.end(c) - ch.begin(c));
    d = j + 1 < kSegPerChunk ? segs[c * (kSegPerChunk - 1) + j] : 0u;
  }
  /* segment starts: exclusive scan of the stored lengths over the chunk */
  const uint32_t start = group_incl_scan(d, j) - d;
  const uint32_t nw = bad ? 0u : (uint32_t)(w1 - w0);
  const uint32_t nbits = nw * 32;
  /* segment j holds the chunk's bins j, j + 8, ... */
  const uint32_t seg_n = j < nsym ? (nsym - j + 7) / 8 : 0u;
  if (have && (start > nbits || (seg_n == 0 && d != 0))) bad = true;
  const bool chunk_ok = have && group_or(bad ? 1u : 0u) == 0;

  /* decode */
  const Words W{payload + w0, chunk_ok ? nw : 0u,
                chunk_ok ? (uint32_t)(n_words - w0) : 0u};
  const uint64_t base = have ? ch.begin(c) : 0;
  bool inv = false;
  Reader rd;
  rd.seek(sh, W, start);
  /* symbol-0 flags of the group's steps (bit 6 of the table entries) */
  uint32_t zor = 0;
  /* one codeword; an invalid one is flagged and skipped as one bit */
  auto step = [&]() -> uint32_t {
    const uint32_t nx = sh.ring[rd.wp % kRing][threadIdx.x];
    const uint32_t top = rd.window();
    const uint32_t e = sh.ent[top >> (32 - kSymBits)];
    uint32_t len = e & 0x3fu;
    uint32_t s = e >> 16;
    zor |= e;
    /* one test on the common path: an entry of length 0 is either a
     * prefix with a second-level table or a code the tables do not hold */
    if (__builtin_expect(len == 0, 0)) {
      /* a code of up to kEnt2Depth bits beyond the prefix: one more lookup
       * with the bits after it */
      if (e & 0x80u) {
        const uint32_t d = (e >> 8) & 15u;
        const uint32_t e2 =
            sh.ent2[(e >> 12) + ((top << kSymBits) >> (32 - d))];
        len = e2 & 0x3fu;
        s = e2 >> 16;
        zor |= e2;
      }
      if (len == 0) {
        s = slow_symbol(rd, W, top, lim, sh, tabs, syms, maxlen, &len);
        if (s == kInvalid) {
          inv = true;
          s = 1;
          len = 1;
        }
        zor |= s == 0 ? kEntZero : 0u;
        /* a code longer than the pair's guaranteed bits: seek past it */
        if (len > 32) {
          rd.seek(sh, W, rd.pos() + len);
          len = 0;
        }
      }
    }
    rd.advance(len, nx);
    return s;
  };
  /* Group g: step u of lane j is bin 64 g + 8 u + j.  The chunk's eight
   * lanes (one wave) put their steps into the chunk's LDS block in bin
   * order, then lane j takes bins 64 g + 8 j .. + 7: one 16-byte store per
   * lane, a full 128-byte line per chunk.  Symbol-0 bins are ranked in bin
   * order: zeros of earlier groups, then of lower lanes, then within. */
  uint16_t* blk = sh.tb[threadIdx.x / kSegPerChunk];
  uint32_t zacc = 0;
  bool zbad = false;
  auto emit = [&](uint32_t g, const uint32_t* pk, uint32_t nsteps) {
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u)
      blk[8 * u + j] =
          u < nsteps ? (uint16_t)(pk[u >> 1] >> (16 * (u & 1))) : (uint16_t)1;
    __builtin_amdgcn_wave_barrier();
    const uint4 q = *reinterpret_cast<const uint4*>(blk + 8 * j);
    __builtin_amdgcn_wave_barrier();
    const uint32_t nat = 64 * g + 8 * j; /* first bin of this lane's run */
    const uint32_t nval = nat < nsym ? (nsym - nat < 8 ? nsym - nat : 8) : 0;
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
    if (__any((zor & kEntZero) != 0)) {
      uint32_t zm = 0;
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i)
        zm |= (i < nval && ((w[i >> 1] >> (16 * (i & 1))) & 0xffffu) == 0)
                  ? 1u << i
                  : 0u;
      const uint32_t zc = __popc(zm);
      const uint32_t zi = group_incl_scan(zc, j);
      uint32_t r = u0 + zacc + zi - zc;
      for (uint32_t m = zm; m; m &= m - 1) {
        if (r < u1)
          upos[r] = (uint32_t)(base + nat + (uint32_t)__ffs(m) - 1);
        else
          zbad = true;
        ++r;
      }
      zacc += __shfl(zi, kSegPerChunk - 1, kSegPerChunk);
    }
    zor = 0;
    if (nval == 8) {
      /* streamed past the caches, which keep the payload's lines */
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      u32x4 w;
      w.x = q.x; w.y = q.y; w.z = q.z; w.w = q.w;
      __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(codes + base + nat));
    } else {
      for (uint32_t i = 0; i < nval; ++i)
        codes[base + nat + i] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
    }
  };
  const uint32_t g_full = chunk_ok ? nsym / 64 : 0u;
  const uint32_t g_all = chunk_ok ? (nsym + 63) / 64 : 0u;
  for (uint32_t g = 0; g < g_full; ++g) {
    uint32_t pk[4];
#pragma unroll
    for (uint32_t u = 0; u < 8; u += 2) {
      const uint32_t lo = step();
      pk[u >> 1] = lo | (step() << 16);
    }
    rd.group_end(sh, W);
    emit(g, pk, 8);
  }
  if (g_all > g_full) { /* the last, partial group of the stream */
    const uint32_t have_steps = seg_n > 8 * g_full ? seg_n - 8 * g_full : 0u;
    uint32_t pk[4] = {0, 0, 0, 0};
    for (uint32_t u = 0; u < have_steps; ++u)
      pk[u >> 1] |= step() << (16 * (u & 1));
    emit(g_full, pk, have_steps);
  }
  if (chunk_ok) {
    const uint32_t end = j + 1 < kSegPerChunk ? start + d : nbits;
    const uint32_t pend = rd.pos();
    if (inv || zbad || (j + 1 < kSegPerChunk ? pend != end : pend > end))
      bad = true;
    if (zacc != u1 - u0) bad = true;
  }
  if (have && bad) atomicOr(status, kStBadStream);
}

static_assert(2 * sizeof(DecShared) <= 160 * 1024,
              "two decoding workgroups share a CU's LDS");

/* The decoding state lives in dynamic LDS (sizeof(DecShared), above the
 * default limit: the launchers raise it once per device).  With the size
 * unknown at compile time the compiler can be held to six waves per SIMD
 * (at most 80 VGPRs): two 10-wave workgroups then fit a CU however the
 * waves are spread over its SIMDs (with static LDS it assumes five, and a
 * second workgroup whose waves land unevenly waits for the first). */
__global__ __launch_bounds__(kDecWG) __attribute__((amdgpu_waves_per_eu(6, 8)))
void k_huff_decode(
    const uint32_t* __restrict__ payload, uint64_t n_words,
    const uint64_t* __restrict__ coff, const uint32_t* __restrict__ upre,
    const uint16_t* __restrict__ segs, Chunks ch,
    uint64_t n_unpred, const DecTables* __restrict__ tabs,
    const uint32_t* __restrict__ syms, uint16_t* __restrict__ codes,
    uint32_t* __restrict__ upos, uint32_t* status) {
  extern __shared__ DecShared dyn_sh[];
  DecShared& sh = dyn_sh[0];
  decode_wg(sh, payload, n_words, coff, upre, segs, ch, n_unpred, tabs, syms,
            codes, upos, status, blockIdx.x);
}

/* Every stream of a batch in one launch: a workgroup decodes chunks of the
 * stream its queue entry names. */
__global__ __launch_bounds__(kDecWG) __attribute__((amdgpu_waves_per_eu(6, 8)))
void k_huff_decode_q(
    const DecJob* __restrict__ jobs, const uint32_t* __restrict__ wg0,
    uint32_t n_jobs) {
  extern __shared__ DecShared dyn_sh[];
  DecShared& sh = dyn_sh[0];
  const uint32_t j = find_job(wg0, n_jobs, blockIdx.x);
  const DecJob& a = jobs[j];
  /* pointers read from a record are generic (flat accesses, which also
   * count against the LDS counter): made global again here */
  decode_wg(sh, (const uint32_t*)gptr(a.payload), a.n_words,
            (const uint64_t*)gptr(a.coff), (const uint32_t*)gptr(a.upre),
            (const uint16_t*)gptr(a.segs), a.ch, a.n_unpred,
            (const DecTables*)gptr(a.tabs), (const uint32_t*)gptr(a.syms),
            (uint16_t*)gptr(a.codes), (uint32_t*)gptr(a.upos),
            (uint32_t*)gptr(a.status), blockIdx.x - wg0[j]);
}

/* The decoders' dynamic LDS is above the default limit: raised once per
 * device (the launchers run on several host threads).  A launch whose
 * limit could not be raised fails, and its caller reports the error. */
static void dec_lds_limit() {
  constexpr int kMaxDev = 64;
  static std::once_flag once[kMaxDev];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return;
  std::call_once(once[dev], [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_huff_decode),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(DecShared));
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_huff_decode_q),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(DecShared));
  });
}

uint32_t decode_workgroups(uint64_t n_chunks) {
  return (uint32_t)((n_chunks + kChunksPerWG - 1) / kChunksPerWG);
}

void launch_huff_decode_q(const DecJob* jobs, const uint32_t* wg0,
                          uint32_t n_jobs, uint32_t total_wg, hipStream_t s) {
  if (!total_wg) return;
  dec_lds_limit();
  QOZ_LAUNCH(k_huff_decode_q, dim3(total_wg), dim3(kDecWG),
             sizeof(DecShared), s, jobs, wg0, n_jobs);
}

void launch_huff_decode(const uint32_t* payload, uint64_t n_words,
                        const uint64_t* coff, const uint32_t* upre,
                        const uint16_t* segs, const Chunks& chunks,
                        uint64_t n_unpred, const DecTables* tabs,
                        const uint32_t* syms, uint16_t* codes,
                        uint32_t* upos, uint32_t* status, hipStream_t s) {
  const uint64_t n_chunks = chunks.count();
  if (!n_chunks) return;
  const uint64_t blocks = (n_chunks + kChunksPerWG - 1) / kChunksPerWG;
  dec_lds_limit();
  QOZ_LAUNCH(k_huff_decode, dim3((uint32_t)blocks), dim3(kDecWG),
             sizeof(DecShared), s, payload, n_words, coff, upre, segs, chunks,
             n_unpred, tabs, syms, codes, upos, status);
}

}  // namespace qoz
