/*
 * Oracle: the compressed stream Z = C(X) and X' = D(Z) (Sec. III).
 * Test infrastructure only.
 *
 * Reading (the paper fixes no container): a 200-byte little-endian header,
 * then 8-byte-aligned sections: anchors f32[A]; codebook symbols u16[U_s]
 * (ascending) and lengths u8[U_s]; chunk word offsets u64[C+1]; number of
 * unpredictable values before each chunk u32[C+1]; segment bit lengths
 * u16[7 C]; unpredictable values f32[U]; Huffman payload u32[W], each chunk
 * starting on a word boundary and packed most-significant bit first.
 * Level l's bins form chunks of max(4096 >> (l - 1), 1024) bins (level
 * boundaries rounded up to 64 bins, a level's last chunk possibly
 * shorter).  A chunk is cut into eight interleaved segments: segment j holds
 * the chunk's bins j, j + 8, j + 16, ... and the payload stores segment 0,
 * then segment 1, and so on; the stream keeps the payload bits of segments
 * 0..6 (0 for an empty segment), so each segment can be decoded on its own.
 * Unpredictable values stay in bin order.  No dictionary (zstd) stage
 * follows the Huffman stage; a lossless zero-word packing may (below).
 *
 * Zero-word packing (format version 5; version 4 streams are unpacked):
 * runs of the zero bin, whose canonical code is all zero bits when it is
 * the most frequent symbol, leave whole payload words at zero.  Chunk c
 * of n_c raw words with z_c nonzero words is stored as a bitmap of
 * ceil(n_c / 32) words (bit i of bitmap word k, least significant first,
 * set when raw word 32 k + i is nonzero) followed by its nonzero words in
 * order, when that is shorter than n_c words; otherwise raw.  The stream
 * is packed only when the packed payload and its offset section together
 * take at most 97 % of the raw payload's bytes (the stage never grows a
 * stream);
 * byte 196 of the header then holds the packed word count W_p, the
 * payload section holds W_p words, and an 8-aligned section of packed
 * chunk word offsets u64[C+1] follows it (a chunk is raw exactly when its
 * packed and raw word counts agree).
 */
#include <cmath>
#include <cstring>
#include <limits>

#include "ref_internal.h"

using namespace qref;

namespace {

const size_t kHeader = 200;

struct Counts {
  uint64_t n_anchor, n_codes, n_unpred, n_used, n_chunks, n_words;
  uint64_t n_packed; /* packed payload words; 0 for an unpacked stream */
};

/* Chunking of the bin stream by level: level l (levels L..1 in stream
 * order) is cut into chunks of max(4096 >> (l - 1), 1024) bins (4096 on
 * level 1, 2048 on level 2, 1024 above: coarser levels' bins carry more
 * long codes); level boundaries are rounded up to a multiple of 64 bins (at
 * most all bins), and the last chunk of a level may be shorter. */
struct Regions {
  int n;                                 /* one per level, level L first */
  uint64_t start[QREF_MAX_LEVELS + 1];   /* first bin; start[n] = bins */
  uint64_t size[QREF_MAX_LEVELS];        /* chunk size */
  uint64_t first[QREF_MAX_LEVELS + 1];   /* first chunk; first[n] = all */
};

Regions regions_of(const Grid& g, int L, uint64_t n_codes) {
  Regions R;
  R.n = L;
  R.start[0] = 0;
  R.first[0] = 0;
  uint64_t t = 0;
  for (int r = 0; r < L; ++r) {
    const int l = L - r;
    t += (uint64_t)(count_anchors(g, (int64_t)1 << (l - 1)) -
                    count_anchors(g, (int64_t)1 << l));
    const uint64_t end = r + 1 == L ? n_codes : (t + 63) / 64 * 64;
    R.start[r + 1] = std::min<uint64_t>(end, n_codes);
    R.size[r] = std::max<uint64_t>((uint64_t)QREF_CHUNK >> (l - 1), 1024);
    const uint64_t bins = R.start[r + 1] - R.start[r];
    R.first[r + 1] = R.first[r] + (bins + R.size[r] - 1) / R.size[r];
  }
  return R;
}

void chunk_range(const Regions& R, uint64_t ch, uint64_t* lo, uint64_t* hi) {
  int r = 0;
  while (r + 1 < R.n && ch >= R.first[r + 1]) ++r;
  *lo = R.start[r] + (ch - R.first[r]) * R.size[r];
  *hi = std::min<uint64_t>(*lo + R.size[r], R.start[r + 1]);
}

struct Layout {
  size_t anchors, syms, lens, coff, upre, segs, unpred, payload, pcoff, total;
};

const uint32_t kSegPerChunk = QREF_CHUNK / QREF_SEG;
const uint32_t kSegLog2 = 9;
static_assert((1u << kSegLog2) == QREF_SEG, "segment size");

size_t al8(size_t v) { return (v + 7) & ~(size_t)7; }

Layout layout_of(const Counts& c) {
  Layout l;
  size_t off = kHeader;
  l.anchors = off;
  off = al8(off + 4 * c.n_anchor);
  l.syms = off;
  off = al8(off + 2 * c.n_used);
  l.lens = off;
  off = al8(off + c.n_used);
  l.coff = off;
  off = al8(off + 8 * (c.n_chunks + 1));
  l.upre = off;
  off = al8(off + 4 * (c.n_chunks + 1));
  l.segs = off;
  off = al8(off + 2 * (kSegPerChunk - 1) * c.n_chunks);
  l.unpred = off;
  off = al8(off + 4 * c.n_unpred);
  l.payload = off;
  if (c.n_packed) {
    off = al8(off + 4 * c.n_packed);
    l.pcoff = off;
    off = off + 8 * (c.n_chunks + 1);
  } else {
    off = off + 4 * c.n_words;
    l.pcoff = 0;
  }
  l.total = off;
  return l;
}

/* Zero-word packing of the chunked payload (raw word offsets coff):
 * packed words and packed offsets pcoff; returns whether the stream is
 * worth packing (packed words + offsets <= 97 % of the raw bytes). */
bool pack_payload(const std::vector<uint32_t>& words,
                  const std::vector<uint64_t>& coff, uint64_t n_chunks,
                  std::vector<uint32_t>* packed,
                  std::vector<uint64_t>* pcoff) {
  packed->clear();
  pcoff->assign(n_chunks + 1, 0);
  for (uint64_t ch = 0; ch < n_chunks; ++ch) {
    (*pcoff)[ch] = packed->size();
    const uint64_t w0 = coff[ch], n = coff[ch + 1] - coff[ch];
    uint64_t nz = 0;
    for (uint64_t i = 0; i < n; ++i) nz += words[w0 + i] != 0;
    const uint64_t nbm = (n + 31) / 32;
    if (nbm + nz < n) {
      std::vector<uint32_t> bm(nbm, 0);
      for (uint64_t i = 0; i < n; ++i)
        if (words[w0 + i]) bm[i / 32] |= 1u << (i % 32);
      packed->insert(packed->end(), bm.begin(), bm.end());
      for (uint64_t i = 0; i < n; ++i)
        if (words[w0 + i]) packed->push_back(words[w0 + i]);
    } else {
      packed->insert(packed->end(), words.begin() + w0,
                     words.begin() + w0 + n);
    }
  }
  (*pcoff)[n_chunks] = packed->size();
  return !words.empty() &&
         100 * (packed->size() + 2 * (n_chunks + 1)) <= 97 * words.size();
}

template <class T>
void put(uint8_t* base, size_t off, T v) {
  std::memcpy(base + off, &v, sizeof(T));
}
template <class T>
T get(const uint8_t* base, size_t off) {
  T v;
  std::memcpy(&v, base + off, sizeof(T));
  return v;
}

bool default_stride(const Grid& g, qref_params* p) {
  if (p->anchor_stride == 0) p->anchor_stride = g.d == 2 ? 64 : 32;
  return true;
}

}  // namespace

extern "C" int qref_compress_bound(qref_shape shape, uint32_t anchor_stride,
                                   size_t* bytes) {
  (void)anchor_stride;
  Grid g;
  if (!bytes || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  uint64_t N = (uint64_t)g.N;
  uint64_t cmax = (N + 1023) / 1024 + QREF_MAX_LEVELS;
  uint64_t wmax = (N + 1) / 2 + cmax;
  size_t b = kHeader + 4 * N + 8 + al8(2 * 65536) + al8(65536) +
             8 * (cmax + 1) + al8(4 * (cmax + 1)) +
             al8(2 * (kSegPerChunk - 1) * cmax) + 8 + 4 * wmax + 64;
  *bytes = b;
  return QREF_OK;
}

extern "C" int qref_compress(const float* x, qref_shape shape, double e,
                             const qref_params* params, int target,
                             const qref_tune_config* cfg, void* out,
                             size_t cap, size_t* out_bytes) {
  Grid g;
  if (!x || !out_bytes || !shape_to_grid(shape, &g)) return QREF_EINVAL;
  if (!(e > 0.0) || !std::isfinite(e)) return QREF_EINVAL;
  if (!all_finite(x, g.N)) return QREF_EINVAL;
  qref_params p;
  if (params) {
    p = *params;
    default_stride(g, &p);
  } else {
    std::memset(&p, 0, sizeof(p));
    int rc = qref_tune(x, shape, e, target, cfg, &p, nullptr);
    if (rc != QREF_OK) return rc;
  }
  int L;
  if (!validate_params(p, g.d, &L)) return QREF_EINVAL;

  /* prediction + quantization */
  std::vector<int32_t> codes((size_t)g.N);
  std::vector<float> unpred((size_t)g.N), anchors((size_t)g.N);
  uint64_t n_codes, n_unpred, n_anchor;
  int rc = qref_predict_quantize(x, shape, e, &p, codes.data(), nullptr,
                                 unpred.data(), anchors.data(), &n_codes,
                                 &n_unpred, &n_anchor);
  if (rc != QREF_OK) return rc;

  /* Huffman */
  const uint32_t nsym = 2 * QREF_RADIUS;
  std::vector<uint64_t> hist(nsym, 0);
  for (uint64_t i = 0; i < n_codes; ++i) hist[codes[i]] += 1;
  std::vector<uint8_t> len(nsym);
  std::vector<uint64_t> code(nsym);
  if (!huffman_lengths(hist.data(), nsym, len.data())) return QREF_EINVAL;
  canonical_codes(len.data(), nsym, code.data());

  Counts c;
  c.n_anchor = n_anchor;
  c.n_codes = n_codes;
  c.n_unpred = n_unpred;
  c.n_used = 0;
  for (uint32_t s = 0; s < nsym; ++s) c.n_used += len[s] ? 1 : 0;
  const Regions R = regions_of(g, L, n_codes);
  c.n_chunks = R.first[R.n];

  /* chunked MSB-first packing */
  std::vector<uint64_t> coff(c.n_chunks + 1);
  std::vector<uint32_t> upre(c.n_chunks + 1);
  std::vector<uint16_t> segs((kSegPerChunk - 1) * c.n_chunks, 0);
  std::vector<uint32_t> words;
  uint64_t zeros = 0;
  for (uint64_t ch = 0; ch < c.n_chunks; ++ch) {
    coff[ch] = words.size();
    upre[ch] = (uint32_t)zeros;
    uint64_t lo, hi;
    chunk_range(R, ch, &lo, &hi);
    uint64_t bitpos = 0;
    size_t base = words.size();
    for (uint64_t i = lo; i < hi; ++i)
      if (codes[i] == 0) ++zeros;
    /* segment j: the chunk's bins j, j + 8, ..., segments in order */
    for (uint32_t j = 0; j < kSegPerChunk; ++j) {
      for (uint64_t i = lo + j; i < hi; i += kSegPerChunk) {
        int32_t s = codes[i];
        if (j + 1 < kSegPerChunk)
          segs[ch * (kSegPerChunk - 1) + j] += (uint16_t)len[s];
        for (int b = len[s] - 1; b >= 0; --b) {
          uint32_t bit = (uint32_t)((code[s] >> b) & 1u);
          size_t wi = base + bitpos / 32;
          if (wi >= words.size()) words.push_back(0);
          words[wi] |= bit << (31 - (bitpos % 32));
          ++bitpos;
        }
      }
    }
  }
  coff[c.n_chunks] = words.size();
  upre[c.n_chunks] = (uint32_t)zeros;
  c.n_words = words.size();
  std::vector<uint32_t> pwords;
  std::vector<uint64_t> pcoff;
  const bool packed = pack_payload(words, coff, c.n_chunks, &pwords, &pcoff);
  c.n_packed = packed ? pwords.size() : 0;

  Layout lay = layout_of(c);
  if (cap < lay.total || !out) {
    *out_bytes = lay.total;
    return QREF_ENOSPACE;
  }
  uint8_t* o = (uint8_t*)out;
  std::memset(o, 0, lay.total);
  std::memcpy(o, "QOZ1", 4);
  put<uint16_t>(o, 4, packed ? 5 : 4);
  put<uint8_t>(o, 6, (uint8_t)g.d);
  put<uint8_t>(o, 7, (uint8_t)kSegLog2);
  for (int i = 0; i < 3; ++i)
    put<uint64_t>(o, 8 + 8 * i, (uint64_t)(i < g.d ? g.n[i] : 1));
  put<double>(o, 32, e);
  put<uint32_t>(o, 40, QREF_RADIUS);
  put<uint32_t>(o, 44, p.anchor_stride);
  put<uint32_t>(o, 48, (uint32_t)L);
  put<uint32_t>(o, 52, QREF_CHUNK);
  put<double>(o, 56, p.alpha);
  put<double>(o, 64, p.beta);
  for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
    put<uint8_t>(o, 72 + l, l < L ? p.interp[l] : 0);
    for (int j = 0; j < 3; ++j)
      put<uint8_t>(o, 88 + 3 * l + j,
                   (l < L && j < g.d) ? p.order[l][j] : 0);
  }
  put<uint64_t>(o, 136, c.n_anchor);
  put<uint64_t>(o, 144, c.n_codes);
  put<uint64_t>(o, 152, c.n_unpred);
  put<uint64_t>(o, 160, c.n_used);
  put<uint64_t>(o, 168, c.n_chunks);
  put<uint64_t>(o, 176, c.n_words);
  put<uint64_t>(o, 184, R.start[R.n - 1]); /* bins before level 1 */
  put<uint32_t>(o, 192, 1024);            /* smallest chunk size */
  put<uint32_t>(o, 196, (uint32_t)c.n_packed);
  copy_bytes(o + lay.anchors, anchors.data(), 4 * n_anchor);
  uint64_t k = 0;
  for (uint32_t s = 0; s < nsym; ++s)
    if (len[s]) {
      put<uint16_t>(o, lay.syms + 2 * k, (uint16_t)s);
      put<uint8_t>(o, lay.lens + k, len[s]);
      ++k;
    }
  for (uint64_t ch = 0; ch <= c.n_chunks; ++ch) {
    put<uint64_t>(o, lay.coff + 8 * ch, coff[ch]);
    put<uint32_t>(o, lay.upre + 4 * ch, upre[ch]);
  }
  for (size_t k = 0; k < segs.size(); ++k)
    put<uint16_t>(o, lay.segs + 2 * k, segs[k]);
  copy_bytes(o + lay.unpred, unpred.data(), 4 * n_unpred);
  if (packed) {
    copy_bytes(o + lay.payload, pwords.data(), 4 * c.n_packed);
    for (uint64_t ch = 0; ch <= c.n_chunks; ++ch)
      put<uint64_t>(o, lay.pcoff + 8 * ch, pcoff[ch]);
  } else {
    copy_bytes(o + lay.payload, words.data(), 4 * c.n_words);
  }
  *out_bytes = lay.total;
  return QREF_OK;
}

namespace {

struct Parsed {
  Grid g;
  qref_params p;
  int L;
  double e;
  Counts c;
  Regions R;
  Layout lay;
};

int parse(const uint8_t* in, size_t n, Parsed* P) {
  if (!in || n < kHeader) return QREF_EFORMAT;
  if (std::memcmp(in, "QOZ1", 4) != 0) return QREF_EFORMAT;
  const uint16_t ver = get<uint16_t>(in, 4);
  if (ver != 4 && ver != 5) return QREF_EFORMAT;
  if (get<uint8_t>(in, 7) != kSegLog2) return QREF_EFORMAT;
  qref_shape sh;
  std::memset(&sh, 0, sizeof(sh));
  sh.ndim = get<uint8_t>(in, 6);
  for (int i = 0; i < 3; ++i) sh.dims[i] = get<uint64_t>(in, 8 + 8 * i);
  if (!shape_to_grid(sh, &P->g)) return QREF_EFORMAT;
  for (uint32_t i = sh.ndim; i < 3; ++i)
    if (sh.dims[i] != 1) return QREF_EFORMAT;
  P->e = get<double>(in, 32);
  if (!(P->e > 0.0) || !std::isfinite(P->e)) return QREF_EFORMAT;
  if (get<uint32_t>(in, 40) != QREF_RADIUS) return QREF_EFORMAT;
  if (get<uint32_t>(in, 52) != QREF_CHUNK || get<uint32_t>(in, 192) != 1024)
    return QREF_EFORMAT;
  std::memset(&P->p, 0, sizeof(P->p));
  P->p.anchor_stride = get<uint32_t>(in, 44);
  P->p.alpha = get<double>(in, 56);
  P->p.beta = get<double>(in, 64);
  for (int l = 0; l < QREF_MAX_LEVELS; ++l) {
    P->p.interp[l] = get<uint8_t>(in, 72 + l);
    for (int j = 0; j < 3; ++j) P->p.order[l][j] = get<uint8_t>(in, 88 + 3 * l + j);
  }
  if (!validate_params(P->p, P->g.d, &P->L)) return QREF_EFORMAT;
  if (get<uint32_t>(in, 48) != (uint32_t)P->L) return QREF_EFORMAT;
  P->p.levels = (uint32_t)P->L;
  Counts& c = P->c;
  c.n_anchor = get<uint64_t>(in, 136);
  c.n_codes = get<uint64_t>(in, 144);
  c.n_unpred = get<uint64_t>(in, 152);
  c.n_used = get<uint64_t>(in, 160);
  c.n_chunks = get<uint64_t>(in, 168);
  c.n_words = get<uint64_t>(in, 176);
  c.n_packed = get<uint32_t>(in, 196);
  if ((ver == 5) != (c.n_packed != 0)) return QREF_EFORMAT;
  if (c.n_packed && 100 * (c.n_packed + 2 * (c.n_chunks + 1)) > 97 * c.n_words)
    return QREF_EFORMAT;
  int64_t A = count_anchors(P->g, P->p.anchor_stride);
  if (c.n_anchor != (uint64_t)A) return QREF_EFORMAT;
  if (c.n_codes != (uint64_t)P->g.N - (uint64_t)A) return QREF_EFORMAT;
  if (c.n_unpred > c.n_codes) return QREF_EFORMAT;
  if (c.n_used < 1 || c.n_used > 2 * QREF_RADIUS) return QREF_EFORMAT;
  P->R = regions_of(P->g, P->L, c.n_codes);
  if (get<uint64_t>(in, 184) != P->R.start[P->R.n - 1]) return QREF_EFORMAT;
  if (c.n_chunks != P->R.first[P->R.n]) return QREF_EFORMAT;
  if (c.n_words > 2 * c.n_codes + c.n_chunks) return QREF_EFORMAT;
  P->lay = layout_of(c);
  if (P->lay.total > n) return QREF_EFORMAT;
  return QREF_OK;
}

}  // namespace

extern "C" int qref_inspect(const void* in, size_t in_bytes,
                            qref_shape* shape, double* e,
                            qref_params* params) {
  Parsed P;
  int rc = parse((const uint8_t*)in, in_bytes, &P);
  if (rc != QREF_OK) return rc;
  if (shape) {
    std::memset(shape, 0, sizeof(*shape));
    shape->ndim = (uint32_t)P.g.d;
    for (int i = 0; i < 3; ++i) shape->dims[i] = (uint64_t)P.g.n[i];
  }
  if (e) *e = P.e;
  if (params) *params = P.p;
  return QREF_OK;
}

extern "C" int qref_decompress(const void* in_v, size_t in_bytes, float* y,
                               size_t y_cap_elems, qref_shape* out_shape) {
  const uint8_t* in = (const uint8_t*)in_v;
  Parsed P;
  int rc = parse(in, in_bytes, &P);
  if (rc != QREF_OK) return rc;
  const Counts& c = P.c;
  const Layout& lay = P.lay;
  if (!y || y_cap_elems < (size_t)P.g.N) return QREF_ENOSPACE;

  /* codebook */
  const uint32_t nsym = 2 * QREF_RADIUS;
  std::vector<uint8_t> len(nsym, 0);
  int64_t prev = -1;
  for (uint64_t k = 0; k < c.n_used; ++k) {
    uint16_t s = get<uint16_t>(in, lay.syms + 2 * k);
    uint8_t l = get<uint8_t>(in, lay.lens + k);
    if ((int64_t)s <= prev || l < 1 || l > 63) return QREF_EFORMAT;
    prev = s;
    len[s] = l;
  }
  /* Kraft: sum 2^-len <= 1 (exactly, in units of 2^-63) */
  {
    unsigned __int128 kraft = 0;
    for (uint32_t s = 0; s < nsym; ++s)
      if (len[s]) kraft += (unsigned __int128)1 << (63 - len[s]);
    if (kraft > ((unsigned __int128)1 << 63)) return QREF_EFORMAT;
  }
  std::vector<uint64_t> code(nsym);
  canonical_codes(len.data(), nsym, code.data());
  /* per length: first code, count, symbols in canonical order */
  std::vector<uint32_t> sorted;
  for (int l = 1; l <= 63; ++l)
    for (uint32_t s = 0; s < nsym; ++s)
      if (len[s] == l) sorted.push_back(s);
  uint64_t first[64] = {0}, cnt[64] = {0}, fidx[64] = {0};
  {
    uint64_t idx = 0;
    for (int l = 1; l <= 63; ++l) {
      fidx[l] = idx;
      for (uint64_t i = idx; i < sorted.size() && len[sorted[i]] == l; ++i)
        ++cnt[l];
      if (cnt[l]) first[l] = code[sorted[idx]];
      idx += cnt[l];
    }
  }

  /* the raw payload: as stored, or expanded from its zero-word packing */
  std::vector<uint32_t> raw((size_t)c.n_words, 0);
  if (!c.n_packed) {
    copy_bytes(raw.data(), in + lay.payload, 4 * c.n_words);
  } else {
    uint64_t prev_p = 0;
    for (uint64_t ch = 0; ch <= c.n_chunks; ++ch) {
      const uint64_t pc = get<uint64_t>(in, lay.pcoff + 8 * ch);
      if ((ch == 0 && pc != 0) || pc < prev_p) return QREF_EFORMAT;
      prev_p = pc;
    }
    if (prev_p != c.n_packed) return QREF_EFORMAT;
    for (uint64_t ch = 0; ch < c.n_chunks; ++ch) {
      const uint64_t w0 = get<uint64_t>(in, lay.coff + 8 * ch);
      const uint64_t w1 = get<uint64_t>(in, lay.coff + 8 * (ch + 1));
      const uint64_t p0 = get<uint64_t>(in, lay.pcoff + 8 * ch);
      const uint64_t p1 = get<uint64_t>(in, lay.pcoff + 8 * (ch + 1));
      if (w1 < w0 || w1 > c.n_words) return QREF_EFORMAT;
      const uint64_t n = w1 - w0, np = p1 - p0;
      if (np > n) return QREF_EFORMAT;
      const size_t pw = lay.payload + 4 * p0;
      if (np == n) {
        copy_bytes(raw.data() + w0, in + pw, 4 * n);
        continue;
      }
      const uint64_t nbm = (n + 31) / 32;
      if (np < nbm) return QREF_EFORMAT;
      uint64_t k = nbm;
      for (uint64_t i = 0; i < 32 * nbm; ++i) {
        const uint32_t bm = get<uint32_t>(in, pw + 4 * (i / 32));
        if (!((bm >> (i % 32)) & 1u)) continue;
        if (i >= n || k >= np) return QREF_EFORMAT;
        raw[w0 + i] = get<uint32_t>(in, pw + 4 * k);
        ++k;
      }
      if (k != np) return QREF_EFORMAT;
    }
  }

  /* decode each chunk bit by bit */
  std::vector<int32_t> codes((size_t)c.n_codes);
  uint64_t zeros = 0;
  for (uint64_t ch = 0; ch < c.n_chunks; ++ch) {
    uint64_t w0 = get<uint64_t>(in, lay.coff + 8 * ch);
    uint64_t w1 = get<uint64_t>(in, lay.coff + 8 * (ch + 1));
    if (get<uint32_t>(in, lay.upre + 4 * ch) != (uint32_t)zeros)
      return QREF_EFORMAT;
    if (w1 < w0 || w1 > c.n_words) return QREF_EFORMAT;
    if (ch == 0 && w0 != 0) return QREF_EFORMAT;
    uint64_t nbits = (w1 - w0) * 32;
    uint64_t bitpos = 0;
    uint64_t lo, hi;
    chunk_range(P.R, ch, &lo, &hi);
    /* segment j (bins j, j + 8, ...) must start where the bit lengths of
     * segments 0..j-1 say; an empty segment has length 0; a segment with a
     * stored length must end exactly there, the last one inside the
     * chunk's words */
    uint64_t seg_end = 0;
    for (uint32_t j = 0; j < kSegPerChunk; ++j) {
      const uint16_t b =
          j + 1 < kSegPerChunk
              ? get<uint16_t>(in, lay.segs + 2 * (ch * (kSegPerChunk - 1) + j))
              : 0;
      if (lo + j >= hi) {
        if (b != 0) return QREF_EFORMAT;
        continue;
      }
      if (bitpos != seg_end) return QREF_EFORMAT;
      seg_end = j + 1 < kSegPerChunk ? seg_end + b : nbits;
      for (uint64_t i = lo + j; i < hi; i += kSegPerChunk) {
        uint64_t v = 0;
        int l = 0;
        for (;;) {
          if (bitpos >= nbits) return QREF_EFORMAT;
          uint32_t word = raw[w0 + bitpos / 32];
          uint32_t bit = (word >> (31 - (bitpos % 32))) & 1u;
          ++bitpos;
          v = (v << 1) | bit;
          ++l;
          if (l > 63) return QREF_EFORMAT;
          if (cnt[l] && v >= first[l] && v - first[l] < cnt[l]) break;
        }
        int32_t s = (int32_t)sorted[fidx[l] + (v - first[l])];
        codes[i] = s;
        if (s == 0) ++zeros;
      }
      if (j + 1 < kSegPerChunk && bitpos != seg_end) return QREF_EFORMAT;
    }
  }
  if (get<uint64_t>(in, lay.coff + 8 * c.n_chunks) != c.n_words)
    return QREF_EFORMAT;
  if (get<uint32_t>(in, lay.upre + 4 * c.n_chunks) != (uint32_t)zeros ||
      zeros != c.n_unpred)
    return QREF_EFORMAT;

  std::vector<float> anchors(c.n_anchor), unpred(c.n_unpred);
  copy_bytes(anchors.data(), in + lay.anchors, 4 * c.n_anchor);
  copy_bytes(unpred.data(), in + lay.unpred, 4 * c.n_unpred);
  qref_shape sh;
  std::memset(&sh, 0, sizeof(sh));
  sh.ndim = (uint32_t)P.g.d;
  for (int i = 0; i < 3; ++i) sh.dims[i] = (uint64_t)P.g.n[i];
  rc = qref_reconstruct(codes.data(), c.n_codes, unpred.data(), c.n_unpred,
                        anchors.data(), c.n_anchor, sh, P.e, &P.p, y);
  if (rc != QREF_OK) return QREF_EFORMAT;
  if (out_shape) *out_shape = sh;
  return QREF_OK;
}
