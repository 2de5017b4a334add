/*
 * Entry points of the QoZ GPU library: compression C_theta, decompression
 * D_theta (Sec. III), stream inspection, and quality metrics (Eq. 1-3).
 * The tuner entry point is in tune_host.cpp.
 *
 * Host/device traffic per compression: one 256 KB histogram read-back to
 * build the Huffman code on the host, one read-back of the payload size,
 * and the small header and codebook uploads.
 */
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <limits>

#include "qoz_internal.h"

namespace qoz {

/* pinned staging regions */
constexpr size_t kPinHist = 0;                 /* 256 KB */
constexpr size_t kPinTable = 256u << 10;       /* 512 KB */
constexpr size_t kPinStage = 768u << 10;       /* 256 KB */
constexpr size_t kPinStatus = 1024u << 10;     /* 4 KB */
constexpr size_t kPinSmall = (1024u << 10) + 4096;
constexpr size_t kPinBase = kPinSingleBytes;

/* Algorithmic bytes per bin in the timing table: a bin counts as a 4-byte
 * quantization code (the width of the integer codes in the cost model of
 * the sweeps), although the kernels store bins as 2-byte values.  A
 * compression sweep target moves x, its neighbour line, its code and (except
 * in the last sweep) its reconstruction; a decompression target its code,
 * its neighbour line and its value. */
constexpr double kCodeBytes = 4.0;

static inline uint8_t* pin(qoz_ctx* c, size_t off) {
  return (uint8_t*)c->pinned + off;
}

#define PROF(kind, bytes, launch)                 \
  do {                                            \
    hipEvent_t ev_ = prof_begin(c, s, (kind));    \
    launch;                                       \
    prof_end(c, s, ev_, (kind), (double)(bytes)); \
  } while (0)

static qoz_status sync_checked(hipStream_t s) {
  QOZ_HIP(hipGetLastError());
  QOZ_HIP(hipStreamSynchronize(s));
  return QOZ_OK;
}

qoz_status compress_with_plan(qoz_ctx* c, const float* d_x, const Plan& P,
                              void* d_out, size_t cap, size_t* out_bytes,
                              hipStream_t s) {
  const uint64_t N = (uint64_t)P.g.n[0] * P.g.n[1] * P.g.n[2];
  const uint64_t nch = P.n_chunks;
  QOZ_TRY(ensure_pinned(c, kPinBase));
  QOZ_TRY(ensure(c->W, 4 * N));
  QOZ_TRY(ensure(c->codes, 2 * (P.n_codes + 16)));
  QOZ_TRY(ensure(c->hist, 4 * kNSym));
  QOZ_TRY(ensure(c->status, 256));
  QOZ_TRY(ensure(c->anchors, 4 * P.n_anchor));
  QOZ_TRY(ensure(c->chunk_bits, 4 * nch));
  QOZ_TRY(ensure(c->chunk_zeros, 4 * nch));
  QOZ_TRY(ensure(c->coff, 8 * (nch + 1)));
  QOZ_TRY(ensure(c->scan, chunk_scan_scratch(nch)));
  QOZ_TRY(ensure(c->upre, 8 * (nch + 1)));
  QOZ_TRY(ensure(c->pcoff, 8 * (nch + 1)));
  QOZ_TRY(ensure(c->chunk_geo, sizeof(ChunkGeo) * (nch ? nch : 1)));
  /* the code table, then the encoder's field record and chunk range */
  QOZ_TRY(ensure(c->enc_table, 8 * kNSym + 4096));
  float* W = (float*)c->W.p;
  uint16_t* codes = (uint16_t*)c->codes.p;
  uint32_t* hist = (uint32_t*)c->hist.p;
  uint32_t* st = (uint32_t*)c->status.p;
  uint64_t* totals = (uint64_t*)((uint8_t*)c->status.p + 64);

  launch_init_status(st, s);
  launch_zero_u32(hist, kNSym, s);
  PROF(PK_ANCHOR, 8.0 * P.n_anchor,
       launch_anchor_copy(P.g, P.s, P.na, d_x, W, (float*)c->anchors.p, st,
                          s));
  size_t fz = SIZE_MAX, fa = SIZE_MAX, fb = SIZE_MAX;
  RowJob rj;
  const bool fuse = level1_rows(P, &fz, &fa, &fb, &rj);
  const std::vector<SweepTile>* tiles = nullptr;
  {
    auto it = c->tiles_comp.find(tile_key(P));
    if (it != c->tiles_comp.end()) tiles = &it->second;
  }
  for (size_t i = 0; i < P.sweeps.size(); ++i) {
    const Sweep& sw = P.sweeps[i];
    if (fuse && (i == fz || i == fa || i == fb)) {
      if (i == fb) { /* sweeps F and A (if fused) and B as one pass */
        const bool write_w = fb + 1 < P.sweeps.size();
        const double tg = (double)rj.B.count +
                          (fa != SIZE_MAX ? rj.A.count : 0) +
                          (fz != SIZE_MAX ? rj.F.count : 0);
        PROF(PK_ROW_COMP_L1, tg * ((write_w ? 12.0 : 8.0) + kCodeBytes),
             launch_row_comp(P.g, rj, d_x, W, codes, write_w, st, s));
      }
      continue;
    }
    const bool last = i + 1 == P.sweeps.size();
    PROF(sw.level == 1 ? PK_SWEEP_COMP_L1 : PK_SWEEP_COMP,
         (double)sw.count * ((last ? 8.0 : 12.0) + kCodeBytes),
         launch_sweep_comp(P.g, sw, d_x, W, codes, !last, st, s,
                           tiles ? (*tiles)[i] : SweepTile()));
  }
  PROF(PK_HIST, kCodeBytes * P.n_codes, launch_hist(codes, P.n_codes, hist, s));
  /* used symbols sorted on the device; the tree is built on the host */
  QOZ_TRY(ensure(c->hsort, 8 * (kSortCap + 1)));
  launch_hist_sort(hist, 1, (uint64_t*)c->hsort.p, s);
  uint64_t* hk = (uint64_t*)pin(c, kPinHist);
  QOZ_TRY(to_host(c, hk, c->hsort.p, 8 * (kSortCap + 1), s));
  QOZ_TRY(to_host(c, pin(c, kPinStatus), st, 32, s));
  QOZ_TRY(sync_checked(s));
  if (((uint32_t*)pin(c, kPinStatus))[0] & kStNonFinite)
    return fail(QOZ_EINVAL, "input contains NaN or Inf");

  /* Huffman code on the host: lengths of the used symbols (in key order),
   * then canonical codes in ascending symbol order */
  std::vector<uint16_t> usym;
  std::vector<uint8_t> ulen;
  uint64_t n_unpred = 0; /* symbol 0's count: the unpredictable values */
  uint64_t payload_bits = 0;
  uint32_t words_bound = 0; /* payload words of the longest chunk, at most */
  {
    const uint64_t n_keys = hk[0];
    std::vector<uint8_t> klen;
    std::vector<uint64_t> keys;
    bool have = false;
    if (n_keys <= kSortCap) {
      keys.assign(hk + 1, hk + 1 + n_keys);
      have = true;
    } else if (n_keys <= kSortCapBig && hist_sort_big_fits()) {
      /* a second device sort with room for kSortCapBig symbols; its keys
       * (128 KB) land in the table region of the pinned staging */
      QOZ_TRY(ensure(c->hsort, 8 * (kSortCapBig + 1)));
      launch_hist_sort_big(hist, nullptr, 1, (uint64_t*)c->hsort.p, s);
      uint64_t* hb = (uint64_t*)pin(c, kPinTable);
      QOZ_TRY(to_host(c, hb, c->hsort.p, 8 * (n_keys + 1), s));
      QOZ_TRY(sync_checked(s));
      keys.assign(hb + 1, hb + 1 + n_keys);
      have = true;
    }
    if (!have) { /* too many used symbols for the device sort */
      uint32_t* h = (uint32_t*)pin(c, kPinTable);
      QOZ_TRY(to_host(c, h, hist, 4 * kNSym, s));
      QOZ_TRY(sync_checked(s));
      for (uint32_t sy = 0; sy < kNSym; ++sy)
        if (h[sy]) keys.push_back(((uint64_t)h[sy] << 16) | sy);
      std::sort(keys.begin(), keys.end());
    }
    klen.resize(keys.size());
    if (!huffman_lengths_sorted(keys.data(), (uint32_t)keys.size(),
                                klen.data()))
      return fail(QOZ_EINVAL, "Huffman code longer than 63 bits");
    words_bound = chunk_words_bound(keys.data(), klen.data(),
                                    (uint32_t)keys.size(), kChunk);
    std::vector<uint32_t> idx(keys.size());
    for (uint32_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
      return (keys[a] & 0xffffu) < (keys[b] & 0xffffu);
    });
    usym.resize(keys.size());
    ulen.resize(keys.size());
    for (uint32_t i = 0; i < idx.size(); ++i) {
      usym[i] = (uint16_t)(keys[idx[i]] & 0xffffu);
      ulen[i] = klen[idx[i]];
      if (usym[i] == 0) n_unpred = keys[idx[i]] >> 16;
      payload_bits += (keys[idx[i]] >> 16) * klen[idx[i]];
    }
  }
  const uint64_t n_used = usym.size();
  /* an encoder table entry holds the code above an 8-bit length; a code
   * longer than 56 bits needs more than Fib(58) ~ 5.9e11 coded points */
  uint32_t max_len = 0;
  for (uint64_t i = 0; i < n_used; ++i) {
    if (ulen[i] > 56) return fail(QOZ_EINVAL, "Huffman code longer than 56 bits");
    max_len = std::max<uint32_t>(max_len, ulen[i]);
  }
  std::vector<uint64_t> ucode(n_used);
  canonical_codes_sparse(usym.data(), ulen.data(), (uint32_t)n_used,
                         ucode.data());
  uint64_t zero_entry = 0;
  int32_t lo = -1, hi = -1;
  for (uint64_t i = 0; i < n_used; ++i) {
    if (usym[i] == 0) {
      zero_entry = (ucode[i] << 8) | ulen[i];
      continue;
    }
    if (lo < 0) lo = usym[i];
    hi = usym[i];
  }
  const uint32_t tab_n = lo < 0 ? 0 : (uint32_t)(hi - lo + 1);
  /* Every section before the payload has a size known now (the payload's
   * start depends on the unpredictable count, symbol 0's count); the
   * encoder writes the chunk offsets, unpredictable ranks, segment lengths
   * and unpredictable values into them and finds the payload size.  When
   * the caller's buffer cannot hold even those sections, the encoder runs
   * into scratch to learn the size needed. */
  const Layout lay0 = layout_of(P.n_anchor, n_used, nch, n_unpred, 0);
  const bool room = d_out && cap >= lay0.payload;
  if (!room) QOZ_TRY(ensure(c->ptmp, lay0.payload));
  uint8_t* out = room ? (uint8_t*)d_out : (uint8_t*)c->ptmp.p;
  const uint64_t cap_words = room ? (cap - lay0.payload) / 4 : 0;
  /* the chunks' exclusive prefixes of payload words and symbol-0 bins
   * (from the count and the chunk scan) and the encoder's totals (zero on
   * entry) */
  uint64_t* gw = (uint64_t*)c->coff.p;
  uint64_t* gz = (uint64_t*)c->upre.p;
  uint64_t* etot = totals + 3;
  /* the code table, then the encoder's field record, its chunk range and
   * the count's workgroup range (after the largest table) */
  uint64_t* tab = (uint64_t*)pin(c, kPinTable);
  std::memset(tab, 0, 8ull * tab_n);
  for (uint64_t i = 0; i < n_used; ++i)
    if (usym[i]) tab[usym[i] - lo] = (ucode[i] << 8) | ulen[i];
  if (tab_n)
    QOZ_TRY(to_device(c, c->enc_table.p, tab, 8ull * tab_n, s));
  uint8_t* hp = pin(c, kPinSmall);
  const size_t f_off = 8ull * kNSym;
  EncField* ef = (EncField*)hp;
  std::memset(ef, 0, sizeof(EncField));
  ef->codes = codes;
  ef->ch = P.chunks;
  ef->nch = nch;
  ef->tab = (const uint64_t*)c->enc_table.p;
  ef->lo = lo;
  ef->tn = tab_n;
  ef->zero_entry = zero_entry;
  ef->coff = (uint64_t*)(out + lay0.coff);
  ef->upre = (uint32_t*)(out + lay0.upre);
  ef->segs = (uint16_t*)(out + lay0.segs);
  ef->payload = (uint32_t*)(out + lay0.payload);
  ef->cap_words = cap_words;
  ef->unpred = (float*)(out + lay0.unpred);
  ef->x = d_x;
  ef->g = P.g;
  ef->totals = etot;
  ef->status = st;
  ef->pack_bits = (uint32_t*)c->chunk_bits.p;
  fill_sweep_table(P, &ef->st);
  const size_t c0_off = (sizeof(EncField) + 255) / 256 * 256;
  static_assert((sizeof(EncField) + 255) / 256 * 256 + 24 <= 4096,
                "encoder record larger than its scratch");
  uint64_t* c0 = (uint64_t*)(hp + c0_off);
  c0[0] = 0;
  c0[1] = nch;
  uint32_t* wg0 = (uint32_t*)(hp + c0_off + 16);
  const uint32_t count_wg = count_workgroups(nch);
  wg0[0] = 0;
  wg0[1] = count_wg;
  uint8_t* dtab = (uint8_t*)c->enc_table.p;
  QOZ_TRY(to_device(c, dtab + f_off, hp, c0_off + 24, s));
  /* section padding must read as zero */
  launch_zero_u32((uint32_t*)out, lay0.payload / 4, s);
  uint8_t* cb = pin(c, kPinStage + 256);
  const size_t cb_bytes = lay0.coff - lay0.syms;
  std::memset(cb, 0, cb_bytes);
  std::memcpy(cb, usym.data(), 2 * n_used);
  std::memcpy(cb + (lay0.lens - lay0.syms), ulen.data(), n_used);
  QOZ_TRY(to_device(c, out + lay0.syms, cb, cb_bytes, s));
  {
    void* dst[1] = {out + lay0.anchors};
    const void* src[1] = {c->anchors.p};
    const uint64_t bytes[1] = {4 * P.n_anchor};
    launch_copy_regions(dst, src, bytes, 1, s);
  }
  launch_zero_u32((uint32_t*)etot, 6, s);
  const EncField* d_ef = (const EncField*)(dtab + f_off);
  const uint64_t* d_c0 = (const uint64_t*)(dtab + f_off + c0_off);
  /* per chunk its code bits and symbol-0 bins, scanned into the chunks'
   * payload offsets and unpredictable ranks (the scan's totals are
   * rewritten by the packing scan below) */
  PROF(PK_HUFF_COUNT, kCodeBytes * P.n_codes + 8.0 * nch,
       launch_huff_count(d_ef, d_c0,
                         (const uint32_t*)(dtab + f_off + c0_off + 16), 1,
                         count_wg, (uint32_t*)c->chunk_bits.p,
                         (uint32_t*)c->chunk_zeros.p, (ChunkGeo*)c->chunk_geo.p,
                         s));
  launch_chunk_scan((uint32_t*)c->chunk_bits.p, (uint32_t*)c->chunk_zeros.p,
                    nch, gw, gz, totals, (uint64_t*)c->scan.p, s);
  /* algorithmic bytes: the bins (as 4-byte codes), the payload (its Huffman
   * bits), the unpredictable values read and written, and per chunk its
   * offsets (read and written), rank, segment lengths and packed size */
  PROF(PK_HUFF_ENC,
       kCodeBytes * P.n_codes + (double)payload_bits / 8.0 + 8.0 * n_unpred +
           46.0 * nch,
       launch_huff_encode(d_ef, d_c0, (const ChunkGeo*)c->chunk_geo.p, gw, gz,
                          1, nch,
                          std::min(encode_max_words(max_len), words_bound),
                          tab_n, max_len > 32, s));
  /* each chunk's size under zero-word packing (from the encoder, in
   * chunk_bits, free again after the first scan), scanned into the packed
   * offsets and total; upre and chunk_zeros are spent by now */
  uint64_t* pcoff = (uint64_t*)c->pcoff.p;
  PROF(PK_PACK, 8.0 * nch,
       launch_chunk_scan((uint32_t*)c->chunk_bits.p,
                         (uint32_t*)c->chunk_zeros.p, nch, pcoff,
                         (uint64_t*)c->upre.p, totals, (uint64_t*)c->scan.p,
                         s));
  QOZ_TRY(to_host(c, pin(c, kPinStatus), st, 32, s));
  QOZ_TRY(to_host(c, pin(c, kPinStatus + 64), totals, 48, s));
  QOZ_TRY(sync_checked(s));
  /* the encoder's totals (words, symbol-0 bins) follow the packing scan's
   * three totals */
  const uint64_t n_words = ((const uint64_t*)pin(c, kPinStatus + 64))[3];
  if (((const uint64_t*)pin(c, kPinStatus + 64))[4] != n_unpred)
    return fail(QOZ_EDEVICE, "internal: unpredictable count mismatch");
  const Layout lay = layout_of(P.n_anchor, n_used, nch, n_unpred, n_words);
  if (!room || lay.total > cap ||
      (((uint32_t*)pin(c, kPinStatus))[0] & kStOverflow)) {
    prof_collect(c);
    *out_bytes = lay.total;
    return fail(QOZ_ENOSPACE, "output capacity too small");
  }
  uint8_t* hs = pin(c, kPinStage);
  write_header(hs, P, n_unpred, n_used, n_words);
  QOZ_TRY(to_device(c, out, hs, kHeaderBytes, s));
  /* zero-word packing, when the packed payload and its offsets take at
   * most kPackPercent % of the raw payload's bytes */
  const uint64_t n_packed = ((const uint64_t*)pin(c, kPinStatus + 64))[0];
  if (n_words &&
      100 * (n_packed + 2 * (nch + 1)) <= (uint64_t)kPackPercent * n_words) {
    const Layout lp =
        layout_of(P.n_anchor, n_used, nch, n_unpred, n_words, n_packed);
    QOZ_TRY(ensure(c->ptmp, 4 * n_packed + 4));
    uint32_t* raw = (uint32_t*)(out + lay.payload);
    PROF(PK_PACK, 4.0 * n_words + 4.0 * n_packed + 8.0 * nch,
         launch_pack_write(raw, (const uint64_t*)(out + lay.coff), pcoff,
                           nch, (uint32_t*)c->ptmp.p, s));
    {
      void* dst[2] = {raw, out + lp.pcoff};
      const void* src[2] = {c->ptmp.p, pcoff};
      const uint64_t bytes[2] = {4 * n_packed, 8 * (nch + 1)};
      launch_copy_regions(dst, src, bytes, 2, s);
    }
    /* the padding word before the offsets reads as zero */
    if (lp.pcoff > lay.payload + 4 * n_packed)
      launch_zero_u32((uint32_t*)(out + lay.payload + 4 * n_packed),
                      (lp.pcoff - lay.payload - 4 * n_packed) / 4, s);
    const uint16_t ver = kStreamVersionPacked;
    const uint32_t npk = (uint32_t)n_packed;
    std::memcpy(hs + 4, &ver, 2);
    std::memcpy(hs + 196, &npk, 4);
    QOZ_TRY(to_device(c, out, hs, kHeaderBytes, s));
    QOZ_TRY(sync_checked(s));
    prof_collect(c);
    *out_bytes = lp.total;
    return QOZ_OK;
  }
  prof_collect(c);
  *out_bytes = lay.total;
  return QOZ_OK;
}

}  // namespace qoz

using namespace qoz;

extern "C" {

qoz_status qoz_compress_bound(qoz_shape shape, size_t* bytes) {
  clear_error();
  int d;
  uint64_t n[3];
  if (!bytes || !shape_ok(shape, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  uint64_t N = 1;
  for (int i = 0; i < d; ++i) N *= n[i];
  /* every point a bin (no anchors): <= 16 bits each plus a padding word per
   * chunk, every bin possibly unpredictable, all 65536 symbols used */
  uint64_t chunks = (N + kMinChunk - 1) / kMinChunk + QOZ_MAX_LEVELS;
  Layout lay = layout_of(0, kNSym, chunks, N, (N + 1) / 2 + chunks);
  *bytes = lay.total + 64;
  return QOZ_OK;
}

qoz_status qoz_compress(qoz_ctx* c, const float* d_x, qoz_shape shape,
                        double abs_eb, const qoz_params* params,
                        qoz_target target, const qoz_tune_config* cfg,
                        void* d_out, size_t cap, size_t* out_bytes,
                        hipStream_t s) {
  clear_error();
  if (!c || !d_x || !out_bytes) return fail(QOZ_EINVAL, "NULL argument");
  if (((uintptr_t)d_out & 7) != 0)
    return fail(QOZ_EINVAL, "output must be 8-byte aligned");
  QOZ_TRY(set_device(c));
  qoz_params p;
  if (params) {
    p = *params;
  } else {
    std::memset(&p, 0, sizeof(p));
    QOZ_TRY(qoz_tune(c, d_x, shape, abs_eb, target, cfg, &p, s));
  }
  Plan P;
  QOZ_TRY(make_plan(shape, abs_eb, p, &P));
  return compress_with_plan(c, d_x, P, d_out, cap, out_bytes, s);
}

qoz_status qoz_inspect(const void* h_in, size_t in_bytes, qoz_shape* shape,
                       double* abs_eb, qoz_params* params) {
  clear_error();
  if (!h_in) return fail(QOZ_EFORMAT, "NULL stream");
  Plan P;
  uint64_t nu, nused, nw;
  uint64_t npk_unused;
  QOZ_TRY(parse_header((const uint8_t*)h_in, in_bytes, false, &P, &nu, &nused,
                       &nw, &npk_unused));
  if (shape) {
    std::memset(shape, 0, sizeof(*shape));
    shape->ndim = (uint32_t)P.d;
    if (P.d == 2) {
      shape->dims[0] = P.g.n[1];
      shape->dims[1] = P.g.n[2];
      shape->dims[2] = 1;
    } else {
      for (int i = 0; i < 3; ++i) shape->dims[i] = P.g.n[i];
    }
  }
  if (abs_eb) *abs_eb = P.e;
  if (params) {
    std::memset(params, 0, sizeof(*params));
    params->anchor_stride = P.s;
    params->levels = P.L;
    std::memcpy(params->interp, P.interp, sizeof(P.interp));
    std::memcpy(params->order, P.order, sizeof(P.order));
    params->alpha = P.alpha;
    params->beta = P.beta;
  }
  return QOZ_OK;
}

qoz_status qoz_decompress(qoz_ctx* c, const void* d_in, size_t in_bytes,
                          float* d_y, size_t y_cap_elems,
                          qoz_shape* out_shape, hipStream_t s) {
  clear_error();
  if (!c || !d_in) return fail(QOZ_EINVAL, "NULL argument");
  if (((uintptr_t)d_in & 7) != 0)
    return fail(QOZ_EINVAL, "stream must be 8-byte aligned");
  QOZ_TRY(set_device(c));
  QOZ_TRY(ensure_pinned(c, kPinBase));
  if (in_bytes < kHeaderBytes) return fail(QOZ_EFORMAT, "stream too short");
  /* the header and the bytes after it in one read: the codebook usually
   * lies within them (else a second read fetches it) */
  constexpr size_t kSpecBytes = 64u << 10;
  const size_t spec = in_bytes < kSpecBytes ? in_bytes : kSpecBytes;
  uint8_t* hs = pin(c, kPinStage);
  QOZ_TRY(to_host(c, hs, d_in, spec, s));
  QOZ_TRY(sync_checked(s));
  Plan P;
  uint64_t nu, nused, nw;
  uint64_t npk;
  QOZ_TRY(parse_header(hs, in_bytes, true, &P, &nu, &nused, &nw, &npk));
  const uint64_t N = (uint64_t)P.g.n[0] * P.g.n[1] * P.g.n[2];
  if (!d_y || y_cap_elems < N)
    return fail(QOZ_ENOSPACE, "output field too small");
  const uint64_t nch = P.n_chunks;
  const Layout lay = layout_of(P.n_anchor, nused, nch, nu, nw, npk);
  const uint8_t* in = (const uint8_t*)d_in;
  const uint8_t* cb = hs + lay.syms;
  if (lay.coff > spec) {
    uint8_t* cbr = pin(c, kPinStage + 256);
    QOZ_TRY(to_host(c, cbr, in + lay.syms, lay.coff - lay.syms, s));
    QOZ_TRY(sync_checked(s));
    cb = cbr;
  }
  DecTables* dt = (DecTables*)pin(c, kPinTable);
  std::vector<uint32_t> sorted;
  if (!build_dec_tables((const uint16_t*)cb, cb + (lay.lens - lay.syms),
                        (uint32_t)nused, dt, &sorted))
    return fail(QOZ_EFORMAT, "bad Huffman codebook");
  const size_t syms_off = (sizeof(DecTables) + 255) / 256 * 256;
  std::memcpy(pin(c, kPinTable + syms_off), sorted.data(),
              4 * sorted.size());
  QOZ_TRY(ensure(c->dec_tables, sizeof(DecTables)));
  QOZ_TRY(ensure(c->dec_syms, 4 * kNSym));
  QOZ_TRY(ensure(c->codes, 2 * (P.n_codes + 16)));
  QOZ_TRY(ensure(c->status, 256));
  QOZ_TRY(to_device(c, c->dec_tables.p, dt, sizeof(DecTables), s));
  QOZ_TRY(to_device(c, c->dec_syms.p, pin(c, kPinTable + syms_off),
                    4 * sorted.size(), s));
  QOZ_TRY(ensure(c->upos, 4 * (nu + 1)));
  uint32_t* st = (uint32_t*)c->status.p;
  uint16_t* codes = (uint16_t*)c->codes.p;
  uint32_t* upos = (uint32_t*)c->upos.p;
  launch_init_status(st, s);
  /* a packed payload is expanded into scratch first */
  const uint32_t* payload = (const uint32_t*)(in + lay.payload);
  if (npk) {
    QOZ_TRY(ensure(c->ptmp, 4 * nw + 4));
    PROF(PK_PACK, 4.0 * npk + 4.0 * nw + 16.0 * nch,
         launch_unpack(payload, npk, (const uint64_t*)(in + lay.coff),
                       (const uint64_t*)(in + lay.pcoff), nch, nw,
                       (uint32_t*)c->ptmp.p, st, s));
    payload = (const uint32_t*)c->ptmp.p;
  }
  PROF(PK_HUFF_DEC, 4.0 * nw + kCodeBytes * P.n_codes + 4.0 * nu + 26.0 * nch,
       launch_huff_decode(payload, nw,
                          (const uint64_t*)(in + lay.coff),
                          (const uint32_t*)(in + lay.upre),
                          (const uint16_t*)(in + lay.segs), P.chunks, nu,
                          (const DecTables*)c->dec_tables.p,
                          (const uint32_t*)c->dec_syms.p, codes, upos, st, s));
  SweepTable tbl;
  fill_sweep_table(P, &tbl);
  launch_unpred_scatter(P.g, tbl, upos, (const float*)(in + lay.unpred), nu,
                        P.n_codes, d_y, st, s);
  PROF(PK_ANCHOR, 8.0 * P.n_anchor,
       launch_anchor_scatter(P.g, P.s, P.na, (const float*)(in + lay.anchors),
                             d_y, s));
  size_t fz = SIZE_MAX, fa = SIZE_MAX, fb = SIZE_MAX;
  RowJob rj;
  const bool fuse = level1_rows(P, &fz, &fa, &fb, &rj);
  const std::vector<SweepTile>* tiles = nullptr;
  {
    auto it = c->tiles_decomp.find(tile_key(P));
    if (it != c->tiles_decomp.end()) tiles = &it->second;
  }
  for (size_t i = 0; i < P.sweeps.size(); ++i) {
    const Sweep& sw = P.sweeps[i];
    if (fuse && (i == fz || i == fa || i == fb)) {
      if (i == fb) {
        const double tg = (double)rj.B.count +
                          (fa != SIZE_MAX ? rj.A.count : 0) +
                          (fz != SIZE_MAX ? rj.F.count : 0);
        PROF(PK_ROW_DEC_L1, tg * (8.0 + kCodeBytes),
             launch_row_decomp(P.g, rj, d_y, codes, s));
      }
      continue;
    }
    PROF(sw.level == 1 ? PK_SWEEP_DEC_L1 : PK_SWEEP_DEC,
         (double)sw.count * (8.0 + kCodeBytes),
         launch_sweep_decomp(P.g, sw, d_y, codes, s,
                             tiles ? (*tiles)[i] : SweepTile()));
  }
  QOZ_TRY(to_host(c, pin(c, kPinStatus), st, 32, s));
  QOZ_TRY(sync_checked(s));
  prof_collect(c);
  if (((uint32_t*)pin(c, kPinStatus))[0] & kStBadStream)
    return fail(QOZ_EFORMAT, "corrupt Huffman payload or chunk tables");
  if (out_shape) {
    std::memset(out_shape, 0, sizeof(*out_shape));
    out_shape->ndim = (uint32_t)P.d;
    if (P.d == 2) {
      out_shape->dims[0] = P.g.n[1];
      out_shape->dims[1] = P.g.n[2];
      out_shape->dims[2] = 1;
    } else {
      for (int i = 0; i < 3; ++i) out_shape->dims[i] = P.g.n[i];
    }
  }
  return QOZ_OK;
}

}  // extern "C"

namespace qoz {

/* Device scratch of one metrics call: status words, the range and SSE
 * partials, and the SSIM partials (at most ssim_cap of them).  `prof` says
 * whether launches may be bracketed with timing events. */
struct MetricsScratch {
  uint32_t* status;
  uint8_t* partial;
  double* ssim;
  uint64_t ssim_cap;
  bool prof;
};

/* Partials go to the host through the context's pinned staging buffer in
 * pieces of at most this many bytes. */
constexpr size_t kMetricsPiece = 512u << 10;

static qoz_status metrics_impl(qoz_ctx* c, const float* d_x,
                               const float* d_y, const Geo& g,
                               const SsimJob& j0, double* psnr, double* ssim,
                               double* max_abs_err, const MetricsScratch& m,
                               hipStream_t s) {
  SsimJob j = j0;
  const uint64_t N = (uint64_t)g.n[0] * g.n[1] * g.n[2];
  const uint32_t rp = range_parts(N), sp = sse_parts(N);
  const uint64_t qp = ssim ? ssim_parts(j) : 0;
  if (qp > m.ssim_cap) return fail(QOZ_EINVAL, "too many SSIM partial sums");
  if (c->pinned_bytes < kPinSmall + kMetricsPiece)
    return fail(QOZ_EDEVICE, "staging buffer smaller than its minimum");
  float* pmin = (float*)m.partial;
  float* pmax = pmin + rp;
  double* psse = (double*)(m.partial + 8 * (size_t)rp);
  double* pmx = psse + sp;
  launch_init_status(m.status, s);
  if (m.prof) {
    PROF(PK_CHECK, 4.0 * N, launch_range(d_x, N, pmin, pmax, m.status, rp, s));
    PROF(PK_REDUCE, 8.0 * N,
         launch_sse_max(d_x, d_y, N, psse, pmx, sp, s));
  } else {
    launch_range(d_x, N, pmin, pmax, m.status, rp, s);
    launch_sse_max(d_x, d_y, N, psse, pmx, sp, s);
  }
  const size_t part_bytes = 8 * (size_t)rp + 16 * (size_t)sp;
  QOZ_TRY(to_host(c, pin(c, kPinSmall), m.partial, part_bytes, s));
  QOZ_TRY(to_host(c, pin(c, kPinStatus), m.status, 32, s));
  QOZ_TRY(sync_checked(s));
  const float* hmin = (const float*)pin(c, kPinSmall);
  const float* hmax = hmin + rp;
  float lo = hmin[0], hi = hmax[0];
  for (uint32_t i = 1; i < rp; ++i) {
    lo = std::fmin(lo, hmin[i]);
    hi = std::fmax(hi, hmax[i]);
  }
  const double vrange = (double)hi - (double)lo;
  const double* hsse = (const double*)(pin(c, kPinSmall) + 8 * (size_t)rp);
  double sse = 0.0, mx = 0.0;
  for (uint32_t i = 0; i < sp; ++i) {
    sse += hsse[i];
    mx = std::fmax(mx, hsse[sp + i]);
  }
  if (psnr) {
    double mse = sse / (double)N;
    *psnr = mse == 0.0 ? std::numeric_limits<double>::infinity()
                       : 20.0 * std::log10(vrange / std::sqrt(mse));
  }
  if (max_abs_err) *max_abs_err = mx;
  if (ssim) {
    j.c1 = (0.01 * vrange) * (0.01 * vrange);
    j.c2 = (0.03 * vrange) * (0.03 * vrange);
    bool launched = false;
    if (m.prof) {
      PROF(PK_SSIM, 8.0 * N, launched = launch_ssim(j, d_x, d_y, m.ssim, s));
    } else {
      launched = launch_ssim(j, d_x, d_y, m.ssim, s);
    }
    if (!launched)
      return fail(QOZ_EDEVICE, "SSIM window ring does not fit LDS");
    /* sequential sum in partial index order, piece by piece */
    double tot = 0.0;
    const uint64_t per = kMetricsPiece / 8;
    for (uint64_t i0 = 0; i0 < qp; i0 += per) {
      const uint64_t k = std::min<uint64_t>(per, qp - i0);
      QOZ_TRY(to_host(c, pin(c, kPinSmall), m.ssim + i0, 8 * k, s));
      QOZ_TRY(sync_checked(s));
      const double* hp = (const double*)pin(c, kPinSmall);
      for (uint64_t i = 0; i < k; ++i) tot += hp[i];
    }
    const double nwin = (double)(j.P - j.wp + 1) * (double)(j.Rn - j.wr + 1) *
                        (double)(j.Cn - j.wc + 1);
    *ssim = tot / nwin;
  }
  if (m.prof) prof_collect(c);
  return QOZ_OK;
}

/* Shape checks and the SSIM window job shared by both metrics calls. */
static qoz_status metrics_setup(qoz_ctx* c, const float* d_x,
                                const float* d_y, qoz_shape shape,
                                uint32_t ssim_window, Geo* g, SsimJob* j) {
  if (!c || !d_x || !d_y) return fail(QOZ_EINVAL, "NULL argument");
  int d;
  uint64_t n[3] = {1, 1, 1};
  if (!shape_ok(shape, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  if (ssim_window == 0) ssim_window = 7;
  if (ssim_window > 11) return fail(QOZ_EINVAL, "ssim_window must be <= 11");
  *g = make_geo(d, n);
  j->P = g->n[0];
  j->Rn = g->n[1];
  j->Cn = g->n[2];
  j->wp = g->n[0] < ssim_window ? g->n[0] : ssim_window;
  j->wr = g->n[1] < ssim_window ? g->n[1] : ssim_window;
  j->wc = g->n[2] < ssim_window ? g->n[2] : ssim_window;
  j->field_stride = (uint64_t)g->n[0] * g->n[1] * g->n[2];
  j->batch = 1;
  j->x_mod = 1;
  j->c1 = j->c2 = 0.0;
  return QOZ_OK;
}

}  // namespace qoz

extern "C" {

qoz_status qoz_metrics(qoz_ctx* c, const float* d_x, const float* d_y,
                       qoz_shape shape, uint32_t ssim_window, double* psnr,
                       double* ssim, double* max_abs_err, hipStream_t s) {
  clear_error();
  Geo g;
  SsimJob j;
  QOZ_TRY(metrics_setup(c, d_x, d_y, shape, ssim_window, &g, &j));
  QOZ_TRY(set_device(c));
  const uint64_t N = (uint64_t)g.n[0] * g.n[1] * g.n[2];
  const uint32_t rp = range_parts(N), sp = sse_parts(N);
  const uint64_t qp = ssim ? ssim_parts(j) : 0;
  const size_t small = 8 * (2 * (size_t)rp + 2 * (size_t)sp) + 1024;
  QOZ_TRY(ensure_pinned(c, kPinSmall + std::max(small, kMetricsPiece)));
  QOZ_TRY(ensure(c->partial, small));
  QOZ_TRY(ensure(c->ssim_part, 8 * (qp + 1)));
  QOZ_TRY(ensure(c->status, 256));
  MetricsScratch m{(uint32_t*)c->status.p, (uint8_t*)c->partial.p,
                   (double*)c->ssim_part.p, qp, true};
  return metrics_impl(c, d_x, d_y, g, j, psnr, ssim, max_abs_err, m, s);
}

qoz_status qoz_metrics_noalloc(qoz_ctx* c, const float* d_x,
                               const float* d_y, qoz_shape shape,
                               uint32_t ssim_window, double* psnr,
                               double* ssim, double* max_abs_err,
                               hipStream_t s) {
  clear_error();
  Geo g;
  SsimJob j;
  QOZ_TRY(metrics_setup(c, d_x, d_y, shape, ssim_window, &g, &j));
  if (!c->fixed_scratch)
    return fail(QOZ_EDEVICE, "fixed device scratch was not resolved");
  QOZ_TRY(set_device(c));
  uint8_t* base = (uint8_t*)c->fixed_scratch;
  MetricsScratch m{(uint32_t*)(base + kFixedStatusOff),
                   base + kFixedPartialOff,
                   (double*)(base + kFixedSsimOff),
                   (kFixedScratchBytes - kFixedSsimOff) / 8, false};
  return metrics_impl(c, d_x, d_y, g, j, psnr, ssim, max_abs_err, m, s);
}

qoz_status qoz_error_ac(qoz_ctx* c, const float* d_x, const float* d_y,
                        qoz_shape shape, double* ac, hipStream_t s) {
  clear_error();
  if (!c || !d_x || !d_y || !ac) return fail(QOZ_EINVAL, "NULL argument");
  int d;
  uint64_t n[3] = {1, 1, 1};
  if (!shape_ok(shape, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  QOZ_TRY(set_device(c));
  const Geo g = make_geo(d, n);
  const uint32_t len = g.n[2];
  const uint64_t nrows = (uint64_t)g.n[0] * g.n[1];
  uint64_t per;
  const uint32_t np = ac_parts(nrows, len, &per);
  const size_t bytes = 24 * (size_t)np;
  QOZ_TRY(ensure_pinned(c, kPinSmall + bytes));
  QOZ_TRY(ensure(c->partial, bytes));
  double* p0 = (double*)c->partial.p;
  double* p1 = p0 + np;
  PROF(PK_REDUCE, 8.0 * nrows * len,
       launch_ac_field(d_x, d_y, nrows, len, p0, p1, s));
  QOZ_TRY(to_host(c, pin(c, kPinSmall), p1, 16 * (size_t)np, s));
  QOZ_TRY(sync_checked(s));
  const double* hp = (const double*)pin(c, kPinSmall);
  double ss = 0.0, lag = 0.0;
  for (uint32_t i = 0; i < np; ++i) {
    ss += hp[2 * i];
    lag += hp[2 * i + 1];
  }
  *ac = ac_from_sums(ss, lag, (double)nrows * len,
                     (double)nrows * (len > 0 ? len - 1 : 0));
  prof_collect(c);
  return QOZ_OK;
}

}  // extern "C"
