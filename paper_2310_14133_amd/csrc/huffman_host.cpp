/*
 * Host side of the Huffman stage (the entropy coder named in Sec. VI-A):
 * code lengths by the two-queue construction, canonical code values, and the
 * decoder's lookup tables.
 *
 * Tie rules (shared by encoder and decoder so streams are reproducible):
 * leaves are ordered by (count, symbol); when a leaf and a merged node have
 * equal weight the leaf is taken first; a single used symbol gets length 1;
 * canonical codes are assigned in (length, symbol) order.
 */
#include <algorithm>
#include <cstring>

#include "qoz_internal.h"

namespace qoz {

bool huffman_lengths(const uint32_t* hist, uint32_t nsym, uint8_t* len) {
  std::memset(len, 0, nsym);
  std::vector<uint32_t> sym;
  for (uint32_t s = 0; s < nsym; ++s)
    if (hist[s]) sym.push_back(s);
  const size_t n = sym.size();
  if (n == 0) return true;
  if (n == 1) {
    len[sym[0]] = 1;
    return true;
  }
  std::stable_sort(sym.begin(), sym.end(), [&](uint32_t a, uint32_t b) {
    return hist[a] < hist[b];
  });
  /* nodes [0, n) are leaves in queue order, [n, 2n-1) merged nodes in
   * creation order; up[] links each node to its parent */
  std::vector<uint64_t> w(2 * n - 1);
  std::vector<uint32_t> up(2 * n - 1, 0);
  for (size_t i = 0; i < n; ++i) w[i] = hist[sym[i]];
  size_t leaf = 0, merged = n, made = n;
  for (; made < 2 * n - 1; ++made) {
    size_t pick[2];
    for (int t = 0; t < 2; ++t) {
      bool use_leaf =
          leaf < n && (merged >= made || w[leaf] <= w[merged]);
      pick[t] = use_leaf ? leaf++ : merged++;
    }
    w[made] = w[pick[0]] + w[pick[1]];
    up[pick[0]] = (uint32_t)made;
    up[pick[1]] = (uint32_t)made;
  }
  /* depth of each node, root (last made) at 0, parents made after
   * children so one backward pass suffices */
  std::vector<uint8_t> depth(2 * n - 1, 0);
  for (size_t v = 2 * n - 2; v-- > 0;) {
    unsigned dp = depth[up[v]] + 1u;
    if (dp > (unsigned)kMaxCodeLen) return false;
    depth[v] = (uint8_t)dp;
  }
  for (size_t i = 0; i < n; ++i) len[sym[i]] = depth[i];
  return true;
}

/* Two-queue construction over leaves already in (count, symbol) order,
 * with the same tie rule as huffman_lengths (leaf first on equal weight). */
bool huffman_lengths_sorted(const uint64_t* keys, uint32_t n, uint8_t* len) {
  if (n == 0) return true;
  if (n == 1) {
    len[0] = 1;
    return true;
  }
  std::vector<uint64_t> w(2 * (size_t)n - 1);
  std::vector<uint32_t> up(2 * (size_t)n - 1, 0);
  for (uint32_t i = 0; i < n; ++i) w[i] = keys[i] >> 16;
  size_t leaf = 0, merged = n, made = n;
  for (; made < 2 * (size_t)n - 1; ++made) {
    size_t pick[2];
    for (int t = 0; t < 2; ++t) {
      const bool use_leaf = leaf < n && (merged >= made || w[leaf] <= w[merged]);
      pick[t] = use_leaf ? leaf++ : merged++;
    }
    w[made] = w[pick[0]] + w[pick[1]];
    up[pick[0]] = (uint32_t)made;
    up[pick[1]] = (uint32_t)made;
  }
  std::vector<uint8_t> depth(2 * (size_t)n - 1, 0);
  for (size_t v = 2 * (size_t)n - 2; v-- > 0;) {
    const unsigned dp = depth[up[v]] + 1u;
    if (dp > (unsigned)kMaxCodeLen) return false;
    depth[v] = (uint8_t)dp;
  }
  for (uint32_t i = 0; i < n; ++i) len[i] = depth[i];
  return true;
}

/* Total code bits = sum of the merged weights (any optimal merge order has
 * the same total). */
uint64_t huffman_cost_sorted(const uint64_t* keys, uint32_t n) {
  if (n == 0) return 0;
  if (n == 1) return keys[0] >> 16;
  std::vector<uint64_t> q(n);
  size_t leaf = 0, qh = 0, qt = 0;
  uint64_t cost = 0;
  for (uint32_t made = 0; made + 1 < n; ++made) {
    uint64_t s = 0;
    for (int t = 0; t < 2; ++t) {
      const bool use_leaf =
          leaf < n && (qh >= qt || (keys[leaf] >> 16) <= q[qh]);
      s += use_leaf ? keys[leaf++] >> 16 : q[qh++];
    }
    q[qt++] = s;
    cost += s;
  }
  return cost;
}

uint32_t chunk_words_bound(const uint64_t* keys, const uint8_t* lens,
                           uint32_t n, uint32_t chunk) {
  /* the longest codes first, each as often as it occurs in the field,
   * until a chunk's bins are used up */
  uint64_t by_len[kMaxCodeLen + 1] = {0};
  for (uint32_t i = 0; i < n; ++i) by_len[lens[i]] += keys[i] >> 16;
  uint64_t left = chunk, bits = 0;
  for (int l = kMaxCodeLen; l > 0 && left; --l) {
    const uint64_t take = by_len[l] < left ? by_len[l] : left;
    bits += take * (uint64_t)l;
    left -= take;
  }
  return (uint32_t)((bits + 31) / 32);
}

void canonical_codes_sparse(const uint16_t* syms, const uint8_t* lens,
                            uint32_t n, uint64_t* codes) {
  uint64_t count[kMaxCodeLen + 2] = {0};
  for (uint32_t i = 0; i < n; ++i) count[lens[i]]++;
  uint64_t next[kMaxCodeLen + 2] = {0};
  uint64_t c = 0;
  for (int l = 1; l <= kMaxCodeLen; ++l) {
    c = (c + (l > 1 ? count[l - 1] : 0)) << 1;
    next[l] = c;
  }
  /* ascending symbols: codes of one length are handed out in symbol order */
  for (uint32_t i = 0; i < n; ++i) codes[i] = next[lens[i]]++;
}

void canonical_codes(const uint8_t* len, uint32_t nsym, uint64_t* code) {
  uint32_t count[kMaxCodeLen + 2] = {0};
  for (uint32_t s = 0; s < nsym; ++s) count[len[s]]++;
  count[0] = 0;
  uint64_t next[kMaxCodeLen + 2] = {0};
  uint64_t c = 0;
  for (int l = 1; l <= kMaxCodeLen; ++l) {
    c = (c + count[l - 1]) << 1;
    next[l] = c;
  }
  /* with the DEFLATE rule the first code of length l is
   * (first(l-1) + count(l-1)) << 1, starting from first(1) = 0 */
  for (uint32_t s = 0; s < nsym; ++s) {
    code[s] = 0;
    if (len[s]) code[s] = next[len[s]]++;
  }
}

void hist_keys_sorted(const uint32_t* hist, uint32_t nsym,
                      std::vector<uint64_t>* keys) {
  /* the used symbols in ascending order, then two stable 16-bit radix
   * passes over the count: ascending (count, symbol) */
  std::vector<uint64_t>& a = *keys;
  a.clear();
  a.reserve(4096);
  for (uint32_t s = 0; s < nsym; ++s)
    if (hist[s]) a.push_back(((uint64_t)hist[s] << 16) | s);
  std::vector<uint64_t> b(a.size());
  std::vector<uint32_t> cnt(65537);
  for (int shift = 16; shift < 48; shift += 16) {
    std::fill(cnt.begin(), cnt.end(), 0u);
    for (uint64_t k : a) cnt[((k >> shift) & 0xffffu) + 1]++;
    for (uint32_t d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
    for (uint64_t k : a) b[cnt[(k >> shift) & 0xffffu]++] = k;
    a.swap(b);
  }
}

/* Total code bits of a whole histogram: the used symbols' counts sorted
 * by two 16-bit radix passes, then the two-queue merge above. */
uint64_t huffman_cost_hist(const uint32_t* hist, uint32_t nsym) {
  std::vector<uint64_t> a;
  hist_keys_sorted(hist, nsym, &a);
  return huffman_cost_sorted(a.data(), (uint32_t)a.size());
}

uint64_t huffman_cost(const uint32_t* hist, uint32_t nsym) {
  std::vector<uint8_t> len(nsym);
  if (!huffman_lengths(hist, nsym, len.data())) return ~0ull;
  uint64_t bits = 0;
  for (uint32_t s = 0; s < nsym; ++s) bits += (uint64_t)hist[s] * len[s];
  return bits;
}

bool build_dec_tables(const uint16_t* syms, const uint8_t* lens,
                      uint32_t n_used, DecTables* t,
                      std::vector<uint32_t>* sorted) {
  std::memset(t, 0, sizeof(*t));
  uint64_t per_len[kMaxCodeLen + 2] = {0};
  int prev = -1;
  for (uint32_t i = 0; i < n_used; ++i) {
    if ((int)syms[i] <= prev) return false;
    if (lens[i] < 1 || lens[i] > kMaxCodeLen) return false;
    prev = syms[i];
    per_len[lens[i]]++;
  }
  /* Kraft sum must not exceed one */
  unsigned __int128 kraft = 0;
  for (uint32_t i = 0; i < n_used; ++i)
    kraft += (unsigned __int128)1 << (kMaxCodeLen - lens[i]);
  if (kraft > ((unsigned __int128)1 << kMaxCodeLen)) return false;
  /* code[i] of symbol syms[i] (ascending symbols) */
  std::vector<uint64_t> code(n_used ? n_used : 1);
  canonical_codes_sparse(syms, lens, n_used, code.data());
  t->n_used = n_used;
  t->zlen = n_used && syms[0] == 0 ? lens[0] : 0;
  t->zcode = t->zlen ? code[0] : 0;
  {
    uint64_t c = 0; /* first canonical code of length L */
    t->lim_half[0] = 0;
    for (int L = 1; L <= kMaxCodeLen; ++L) {
      c = (c + per_len[L - 1]) << 1;
      t->lim_half[L] = (c + per_len[L]) << (63 - L);
    }
  }
  /* symbols in canonical order (length, then symbol): a counting sort */
  sorted->assign(n_used, 0u);
  uint32_t pos[kMaxCodeLen + 2] = {0};
  uint32_t acc = 0;
  for (int l = 1; l <= kMaxCodeLen; ++l) {
    t->off[l] = acc;
    pos[l] = acc;
    t->cnt[l] = (uint32_t)per_len[l];
    acc += (uint32_t)per_len[l];
    if (per_len[l]) t->maxlen = (uint32_t)l;
  }
  for (uint32_t i = 0; i < n_used; ++i) {
    const uint32_t l = lens[i];
    if (pos[l] == t->off[l]) t->first[l] = code[i];
    (*sorted)[pos[l]++] = syms[i];
  }
  /* Fast table: a code of length l <= kSymBits fills the 2^(kSymBits - l)
   * entries that start with it; entries of longer (or invalid) codes stay
   * 0. */
  for (uint32_t i = 0; i < n_used; ++i) {
    const uint32_t l = lens[i];
    if (l > (uint32_t)kSymBits) continue;
    const uint32_t e = l | (syms[i] == 0 ? 0x40u : 0u) |
                       ((uint32_t)syms[i] << 16);
    const uint32_t base = (uint32_t)(code[i] << (kSymBits - l));
    for (uint32_t k = 0; k < (1u << (kSymBits - l)); ++k) t->ent[base + k] = e;
  }
  /* Second level: a kSymBits-bit prefix of longer codes gets a table of
   * 2^d entries indexed by the next d bits, d the depth of its deepest code
   * beyond the prefix, at most kEnt2Depth, while kEnt2 entries last (a
   * prefix without one, and codes deeper than its d, take the search by
   * length).  A code of length l fills the 2^(d - (l - kSymBits)) entries
   * that start with its last l - kSymBits bits. */
  {
    std::vector<uint32_t> depth(1u << kSymBits, 0), base2(1u << kSymBits, 0);
    for (uint32_t i = 0; i < n_used; ++i) {
      const uint32_t l = lens[i];
      if (l <= (uint32_t)kSymBits) continue;
      const uint32_t p = (uint32_t)(code[i] >> (l - kSymBits));
      depth[p] = std::max<uint32_t>(depth[p], l - kSymBits);
    }
    uint32_t used2 = 0;
    for (uint32_t p = 0; p < (1u << kSymBits); ++p) {
      if (!depth[p]) continue;
      const uint32_t d = std::min<uint32_t>(depth[p], kEnt2Depth);
      if (used2 + (1u << d) > kEnt2) {
        depth[p] = 0;
        continue;
      }
      depth[p] = d;
      base2[p] = used2;
      t->ent[p] = 0x80u | (d << 8) | (used2 << 12);
      used2 += 1u << d;
    }
    for (uint32_t i = 0; i < n_used; ++i) {
      const uint32_t l = lens[i];
      if (l <= (uint32_t)kSymBits) continue;
      const uint32_t p = (uint32_t)(code[i] >> (l - kSymBits));
      const uint32_t d = depth[p], x = l - kSymBits;
      if (!d || x > d) continue;
      const uint32_t e = l | (syms[i] == 0 ? 0x40u : 0u) |
                         ((uint32_t)syms[i] << 16);
      const uint32_t suffix = (uint32_t)(code[i] & ((1ull << x) - 1));
      const uint32_t b = base2[p] + (suffix << (d - x));
      for (uint32_t k = 0; k < (1u << (d - x)); ++k) t->ent2[b + k] = e;
    }
  }
  return true;
}

}  // namespace qoz
