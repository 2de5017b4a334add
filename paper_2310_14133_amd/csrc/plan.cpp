/*
 * Host planning for the QoZ GPU library: shape and parameter checks, the
 * level bounds of Eq. 5, the per-level sweep schedule of the multi-level
 * interpolation (Sec. V), and the byte layout of the compressed stream.
 */
#include <cmath>
#include <cstring>

#include "qoz_internal.h"

namespace qoz {

bool shape_ok(const qoz_shape& sh, int* d, uint64_t n[3]) {
  if (sh.ndim != 2 && sh.ndim != 3) return false;
  uint64_t total = 1;
  for (uint32_t i = 0; i < sh.ndim; ++i) {
    if (sh.dims[i] < 2 || sh.dims[i] > (1ull << 31)) return false;
    total *= sh.dims[i];
    if (total >= (1ull << 32)) return false;
    n[i] = sh.dims[i];
  }
  *d = (int)sh.ndim;
  return true;
}

Geo make_geo(int d, const uint64_t* n) {
  Geo g;
  if (d == 2) {
    g.n[0] = 1;
    g.n[1] = (uint32_t)n[0];
    g.n[2] = (uint32_t)n[1];
  } else {
    for (int i = 0; i < 3; ++i) g.n[i] = (uint32_t)n[i];
  }
  g.st[2] = 1;
  g.st[1] = g.n[2];
  g.st[0] = g.n[1] * g.n[2];
  return g;
}

bool params_ok(const qoz_params& p, int d, uint32_t* L) {
  uint32_t s = p.anchor_stride;
  if (s < 2 || (s & (s - 1))) return false;
  uint32_t levels = 0;
  while ((1u << levels) < s) ++levels;
  if (levels > QOZ_MAX_LEVELS) return false;
  for (uint32_t l = 0; l < levels; ++l) {
    if (p.interp[l] > 1) return false;
    unsigned mask = 0;
    for (int j = 0; j < d; ++j) {
      unsigned m = p.order[l][j];
      if (m >= (unsigned)d || (mask & (1u << m))) return false;
      mask |= 1u << m;
    }
  }
  if (!(p.alpha >= 1.0) || !std::isfinite(p.alpha)) return false;
  if (!(p.beta >= 1.0) || !std::isfinite(p.beta)) return false;
  *L = levels;
  return true;
}

/* Eq. 5: e_l = e / min(alpha^(l-1), beta); the quantizer takes the bin
 * width 2 e_l and its reciprocal, each rounded once to FP32. */
void level_bounds(double e, double alpha, double beta, uint32_t L,
                  double* eb, float* twoeb, float* inv) {
  double a = 1.0;
  for (uint32_t l = 0; l < L; ++l) {
    if (l) a *= alpha;
    double den = beta < a ? beta : a;
    double v = e / den;
    eb[l] = v;
    twoeb[l] = (float)(v * 2.0);
    inv[l] = (float)(1.0 / (v * 2.0));
  }
}

/* Targets of sweep j in a level of half-stride h: along the swept dimension
 * the odd multiples of h; dimensions swept before it in this level step by
 * h; those swept after it step by 2h. */
void sweep_grid(const Geo& g, const uint32_t* order_grid, int d, int j,
                uint32_t h, uint32_t* start, uint32_t* step, uint32_t* cnt) {
  for (int m = 0; m < 3; ++m) {
    start[m] = 0;
    step[m] = 1;
    cnt[m] = g.n[m];
  }
  for (int pos = 0; pos < d; ++pos) {
    uint32_t m = order_grid[pos];
    uint32_t st = pos == j ? h : 0;
    uint32_t sp = pos < j ? h : 2 * h;
    start[m] = st;
    step[m] = sp;
    cnt[m] = st < g.n[m] ? (g.n[m] - 1 - st) / sp + 1 : 0;
  }
}

qoz_status make_plan(const qoz_shape& sh, double e, const qoz_params& p_in,
                     Plan* plan) {
  int d;
  uint64_t n[3] = {1, 1, 1};
  if (!shape_ok(sh, &d, n)) return fail(QOZ_EINVAL, "bad shape");
  if (!(e > 0.0) || !std::isfinite(e))
    return fail(QOZ_EINVAL, "error bound must be finite and > 0");
  qoz_params p = p_in;
  if (p.anchor_stride == 0) p.anchor_stride = d == 2 ? 64 : 32;
  uint32_t L;
  if (!params_ok(p, d, &L)) return fail(QOZ_EINVAL, "bad parameters");
  Plan& P = *plan;
  P.g = make_geo(d, n);
  P.d = d;
  P.s = p.anchor_stride;
  P.L = L;
  P.e = e;
  P.alpha = p.alpha;
  P.beta = p.beta;
  std::memcpy(P.interp, p.interp, sizeof(P.interp));
  std::memcpy(P.order, p.order, sizeof(P.order));
  for (int m = 0; m < 3; ++m) P.na[m] = (P.g.n[m] - 1) / P.s + 1;
  if (d == 2) P.na[0] = 1;
  P.n_anchor = (uint64_t)P.na[0] * P.na[1] * P.na[2];
  double eb[QOZ_MAX_LEVELS];
  float tw[QOZ_MAX_LEVELS], iv[QOZ_MAX_LEVELS];
  level_bounds(e, p.alpha, p.beta, L, eb, tw, iv);
  P.sweeps.clear();
  uint64_t off = 0;
  const uint32_t shift = d == 2 ? 1 : 0;
  for (uint32_t l = L; l >= 1; --l) {
    uint32_t og[3];
    for (int j = 0; j < d; ++j) og[j] = p.order[l - 1][j] + shift;
    for (int j = 0; j < d; ++j) {
      Sweep sw;
      sweep_grid(P.g, og, d, j, 1u << (l - 1), sw.start, sw.step, sw.cnt);
      sw.k = og[j];
      sw.h = 1u << (l - 1);
      sw.cubic = p.interp[l - 1];
      sw.level = l;
      sw.code_off = off;
      sw.count = (uint64_t)sw.cnt[0] * sw.cnt[1] * sw.cnt[2];
      sw.twoeb = tw[l - 1];
      sw.inv = iv[l - 1];
      sw.eb = eb[l - 1];
      off += sw.count;
      P.sweeps.push_back(sw);
    }
  }
  P.n_codes = off;
  /* chunking by level, level L first (as in the stream) */
  {
    Chunks& C = P.chunks;
    C = Chunks();
    C.n = L;
    C.start[0] = 0;
    C.first[0] = 0;
    uint64_t t = 0;
    for (uint32_t r = 0; r < L; ++r) {
      const uint32_t l = L - r;
      for (const Sweep& sw : P.sweeps)
        if (sw.level == l) t += sw.count;
      const uint64_t e = r + 1 == L ? off : (t + 63) / 64 * 64;
      C.start[r + 1] = e < off ? e : off;
      const uint32_t sz = kChunk >> (l - 1);
      C.size[r] = sz > kMinChunk ? sz : kMinChunk;
      C.first[r + 1] =
          C.first[r] + (C.start[r + 1] - C.start[r] + C.size[r] - 1) / C.size[r];
    }
  }
  P.n_chunks = P.chunks.count();
  if (P.n_codes + P.n_anchor != (uint64_t)P.g.n[0] * P.g.n[1] * P.g.n[2])
    return fail(QOZ_EINVAL, "internal: sweep schedule does not cover field");
  return QOZ_OK;
}

bool level1_rows(const Plan& P, size_t* iz, size_t* ia, size_t* ib,
                 RowJob* rj) {
  const size_t ns = P.sweeps.size(), d = (size_t)P.d;
  *iz = *ia = *ib = SIZE_MAX;
  if (ns < d || P.g.n[2] > 2 * kRowMaxEven) return false;
  const size_t first = ns - d; /* the level-1 sweeps close the schedule */
  size_t jb = d;
  for (size_t j = 0; j < d; ++j)
    if (P.sweeps[first + j].k == 2) jb = j;
  if (jb == d) return false;
  std::memset(rj, 0, sizeof(*rj));
  *ib = first + jb;
  *ia = jb > 0 ? first + jb - 1 : SIZE_MAX;
  rj->B = P.sweeps[*ib];
  rj->a = -1;
  rj->f = -1;
  if (jb > 0) {
    rj->A = P.sweeps[*ia];
    rj->a = (int32_t)rj->A.k;
  }
  /* order (f, a, 2): F's targets are the even points of rows odd along f
   * and even along a */
  if (jb == 2 && d == 3) {
    *iz = first;
    rj->F = P.sweeps[first];
    rj->f = (int32_t)rj->F.k;
  }
  /* B's targets fill rows of its (p0, p1) sub-grid; A's are those rows
   * that are odd along a */
  for (int m = 0; m < 2; ++m) {
    rj->rstep[m] = rj->B.step[m];
    rj->rcnt[m] = rj->B.cnt[m];
  }
  rj->vecA = jb > 0 && rj->A.code_off % 4 == 0 && rj->A.cnt[2] % 4 == 0;
  rj->vecB = rj->B.code_off % 4 == 0 && rj->B.cnt[2] % 4 == 0;
  rj->vecF = rj->f >= 0 && rj->F.code_off % 4 == 0 && rj->F.cnt[2] % 4 == 0;
  return true;
}

void fill_sweep_table(const Plan& p, SweepTable* t) {
  std::memset(t, 0, sizeof(*t));
  t->n = (uint32_t)p.sweeps.size();
  for (uint32_t i = 0; i < t->n; ++i) {
    const Sweep& s = p.sweeps[i];
    t->off[i] = s.code_off;
    for (int m = 0; m < 3; ++m) {
      t->start[i][m] = s.start[m];
      t->step[i][m] = s.step[m];
      t->cnt[i][m] = s.cnt[m];
    }
  }
  t->off[t->n] = p.n_codes;
}

/* Stream layout: header, then 8-byte-aligned sections in this order:
 * anchors f32, codebook symbols u16, codebook lengths u8, chunk word
 * offsets u64[chunks+1], unpredictable counts before each chunk
 * u32[chunks+1], payload bits of the first seven 512-bin segments of each
 * chunk u16[7 chunks] (0 past the last bin), unpredictable values f32,
 * Huffman payload u32. */
static uint64_t up8(uint64_t v) { return (v + 7) / 8 * 8; }

Layout layout_of(uint64_t n_anchor, uint64_t n_used, uint64_t n_chunks,
                 uint64_t n_unpred, uint64_t n_words, uint64_t n_packed) {
  Layout L;
  uint64_t o = kHeaderBytes;
  L.anchors = o;
  o = up8(o + 4 * n_anchor);
  L.syms = o;
  o = up8(o + 2 * n_used);
  L.lens = o;
  o = up8(o + n_used);
  L.coff = o;
  o = up8(o + 8 * (n_chunks + 1));
  L.upre = o;
  o = up8(o + 4 * (n_chunks + 1));
  L.segs = o;
  o = up8(o + 2 * (kSegPerChunk - 1) * n_chunks);
  L.unpred = o;
  o = up8(o + 4 * n_unpred);
  L.payload = o;
  if (n_packed) { /* packed payload, then the packed chunk offsets */
    L.pcoff = up8(o + 4 * n_packed);
    L.total = L.pcoff + 8 * (n_chunks + 1);
  } else {
    L.pcoff = 0;
    L.total = o + 4 * n_words;
  }
  return L;
}

template <class T>
static void wr(uint8_t* b, size_t o, T v) {
  std::memcpy(b + o, &v, sizeof(T));
}
template <class T>
static T rd(const uint8_t* b, size_t o) {
  T v;
  std::memcpy(&v, b + o, sizeof(T));
  return v;
}

std::vector<uint32_t> tile_key(const Plan& p) {
  std::vector<uint32_t> k = {p.g.n[0], p.g.n[1], p.g.n[2],
                             (uint32_t)p.sweeps.size()};
  for (const Sweep& sw : p.sweeps) {
    k.push_back(sw.k);
    k.push_back(sw.h);
    for (int i = 0; i < 3; ++i) {
      k.push_back(sw.start[i]);
      k.push_back(sw.step[i]);
      k.push_back(sw.cnt[i]);
    }
  }
  return k;
}

void write_header(uint8_t* h, const Plan& p, uint64_t n_unpred,
                  uint64_t n_used, uint64_t n_words) {
  std::memset(h, 0, kHeaderBytes);
  std::memcpy(h, "QOZ1", 4);
  wr<uint16_t>(h, 4, kStreamVersion);
  wr<uint8_t>(h, 6, (uint8_t)p.d);
  wr<uint8_t>(h, 7, (uint8_t)kSegLog2);
  uint64_t dims[3] = {1, 1, 1};
  if (p.d == 2) {
    dims[0] = p.g.n[1];
    dims[1] = p.g.n[2];
  } else {
    for (int i = 0; i < 3; ++i) dims[i] = p.g.n[i];
  }
  for (int i = 0; i < 3; ++i) wr<uint64_t>(h, 8 + 8 * i, dims[i]);
  wr<double>(h, 32, p.e);
  wr<uint32_t>(h, 40, (uint32_t)kRadius);
  wr<uint32_t>(h, 44, p.s);
  wr<uint32_t>(h, 48, p.L);
  wr<uint32_t>(h, 52, kChunk);
  wr<double>(h, 56, p.alpha);
  wr<double>(h, 64, p.beta);
  for (uint32_t l = 0; l < p.L; ++l) {
    h[72 + l] = p.interp[l];
    for (int j = 0; j < p.d; ++j) h[88 + 3 * l + j] = p.order[l][j];
  }
  wr<uint64_t>(h, 136, p.n_anchor);
  wr<uint64_t>(h, 144, p.n_codes);
  wr<uint64_t>(h, 152, n_unpred);
  wr<uint64_t>(h, 160, n_used);
  wr<uint64_t>(h, 168, p.n_chunks);
  wr<uint64_t>(h, 176, n_words);
  wr<uint64_t>(h, 184, p.chunks.start[p.chunks.n - 1]); /* before level 1 */
  wr<uint32_t>(h, 192, kMinChunk);
}

qoz_status parse_header(const uint8_t* h, size_t in_bytes, bool need_all, Plan* plan,
                        uint64_t* n_unpred, uint64_t* n_used,
                        uint64_t* n_words, uint64_t* n_packed) {
  if (in_bytes < kHeaderBytes) return fail(QOZ_EFORMAT, "stream too short");
  if (std::memcmp(h, "QOZ1", 4) != 0) return fail(QOZ_EFORMAT, "bad magic");
  const uint16_t ver = rd<uint16_t>(h, 4);
  if (ver != kStreamVersion && ver != kStreamVersionPacked)
    return fail(QOZ_EFORMAT, "bad version");
  if (h[7] != kSegLog2) return fail(QOZ_EFORMAT, "unsupported segment size");
  qoz_shape sh;
  std::memset(&sh, 0, sizeof(sh));
  sh.ndim = h[6];
  for (int i = 0; i < 3; ++i) sh.dims[i] = rd<uint64_t>(h, 8 + 8 * i);
  if (sh.ndim == 2 && sh.dims[2] != 1) return fail(QOZ_EFORMAT, "bad dims");
  if (rd<uint32_t>(h, 40) != (uint32_t)kRadius ||
      rd<uint32_t>(h, 52) != kChunk || rd<uint32_t>(h, 192) != kMinChunk)
    return fail(QOZ_EFORMAT, "unsupported radius or chunk size");
  qoz_params p;
  std::memset(&p, 0, sizeof(p));
  p.anchor_stride = rd<uint32_t>(h, 44);
  p.alpha = rd<double>(h, 56);
  p.beta = rd<double>(h, 64);
  for (int l = 0; l < QOZ_MAX_LEVELS; ++l) {
    p.interp[l] = h[72 + l];
    for (int j = 0; j < 3; ++j) p.order[l][j] = h[88 + 3 * l + j];
  }
  double e = rd<double>(h, 32);
  int d;
  uint64_t n[3];
  uint32_t L;
  if (!shape_ok(sh, &d, n) || !params_ok(p, d, &L) || !(e > 0.0) ||
      !std::isfinite(e) || p.anchor_stride == 0)
    return fail(QOZ_EFORMAT, "bad header fields");
  if (rd<uint32_t>(h, 48) != L) return fail(QOZ_EFORMAT, "bad level count");
  qoz_status st = make_plan(sh, e, p, plan);
  if (st != QOZ_OK) return fail(QOZ_EFORMAT, "bad header fields");
  uint64_t na = rd<uint64_t>(h, 136), nc = rd<uint64_t>(h, 144);
  uint64_t nu = rd<uint64_t>(h, 152), nused = rd<uint64_t>(h, 160);
  uint64_t nch = rd<uint64_t>(h, 168), nw = rd<uint64_t>(h, 176);
  if (na != plan->n_anchor || nc != plan->n_codes || nch != plan->n_chunks ||
      rd<uint64_t>(h, 184) != plan->chunks.start[plan->chunks.n - 1] ||
      nu > nc || nused < 1 || nused > kNSym ||
      nw > 2 * nc + nch)
    return fail(QOZ_EFORMAT, "inconsistent counts in header");
  const uint64_t npk = rd<uint32_t>(h, 196);
  if ((ver == kStreamVersionPacked) != (npk != 0) ||
      100 * npk > (uint64_t)kPackPercent * nw)
    return fail(QOZ_EFORMAT, "inconsistent packed payload size");
  Layout lay = layout_of(na, nused, nch, nu, nw, npk);
  if (need_all && lay.total > in_bytes)
    return fail(QOZ_EFORMAT, "stream truncated");
  *n_unpred = nu;
  *n_used = nused;
  *n_words = nw;
  *n_packed = npk;
  return QOZ_OK;
}

}  // namespace qoz
