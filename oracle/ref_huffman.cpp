/*
 * Oracle: Huffman coding of the quantization bins (Sec. VI-A names Huffman
 * as the entropy stage of the pipeline).  Test infrastructure only.
 *
 * Reading: code lengths come from the two-queue Huffman construction over
 * the used symbols sorted by (count, symbol); on equal weights the leaf
 * queue is taken before the internal-node queue.  A lone used symbol gets
 * length 1.  Codes are canonical: symbols sorted by (length, symbol) receive
 * consecutive code values, shifted left whenever the length grows.
 */
#include <algorithm>
#include <cstring>

#include "ref_internal.h"

namespace qref {

bool huffman_lengths(const uint64_t* hist, uint32_t nsym, uint8_t* len) {
  std::memset(len, 0, nsym);
  struct Leaf {
    uint64_t w;
    uint32_t sym;
  };
  std::vector<Leaf> leaves;
  for (uint32_t s = 0; s < nsym; ++s)
    if (hist[s] > 0) leaves.push_back({hist[s], s});
  if (leaves.empty()) return true;
  if (leaves.size() == 1) {
    len[leaves[0].sym] = 1;
    return true;
  }
  std::sort(leaves.begin(), leaves.end(), [](const Leaf& a, const Leaf& b) {
    return a.w != b.w ? a.w < b.w : a.sym < b.sym;
  });
  /* node ids: 0..n-1 leaves (in sorted order), n.. internal nodes */
  size_t n = leaves.size();
  std::vector<uint64_t> weight(2 * n - 1);
  std::vector<int64_t> parent(2 * n - 1, -1);
  for (size_t i = 0; i < n; ++i) weight[i] = leaves[i].w;
  size_t li = 0;         /* front of the leaf queue */
  size_t qi = n;         /* front of the internal queue */
  size_t next = n;       /* next internal node id (= back of that queue) */
  auto take = [&]() -> size_t {
    bool leaf_ok = li < n;
    bool int_ok = qi < next;
    if (leaf_ok && (!int_ok || weight[li] <= weight[qi])) return li++;
    return qi++;
  };
  while (next < 2 * n - 1) {
    size_t first = take();
    size_t second = take();
    weight[next] = weight[first] + weight[second];
    parent[first] = (int64_t)next;
    parent[second] = (int64_t)next;
    ++next;
  }
  for (size_t i = 0; i < n; ++i) {
    int depth = 0;
    for (int64_t v = (int64_t)i; parent[v] >= 0; v = parent[v]) ++depth;
    if (depth > 63) return false;
    len[leaves[i].sym] = (uint8_t)depth;
  }
  return true;
}

void canonical_codes(const uint8_t* len, uint32_t nsym, uint64_t* code) {
  std::vector<uint32_t> syms;
  for (uint32_t s = 0; s < nsym; ++s) {
    code[s] = 0;
    if (len[s]) syms.push_back(s);
  }
  std::sort(syms.begin(), syms.end(), [&](uint32_t a, uint32_t b) {
    return len[a] != len[b] ? len[a] < len[b] : a < b;
  });
  uint64_t c = 0;
  for (size_t i = 0; i < syms.size(); ++i) {
    if (i > 0) c = (c + 1) << (len[syms[i]] - len[syms[i - 1]]);
    code[syms[i]] = c;
  }
}

uint64_t huffman_bits(const uint64_t* hist, const uint8_t* len,
                      uint32_t nsym) {
  uint64_t bits = 0;
  for (uint32_t s = 0; s < nsym; ++s) bits += hist[s] * len[s];
  return bits;
}

}  // namespace qref

using namespace qref;

extern "C" int qref_huffman_lengths(const uint64_t* hist, uint32_t nsym,
                                    uint8_t* len) {
  if (!hist || !len || nsym == 0) return QREF_EINVAL;
  return huffman_lengths(hist, nsym, len) ? QREF_OK : QREF_EINVAL;
}

extern "C" int qref_huffman_codes(const uint8_t* len, uint32_t nsym,
                                  uint64_t* code) {
  if (!len || !code || nsym == 0) return QREF_EINVAL;
  canonical_codes(len, nsym, code);
  return QREF_OK;
}
