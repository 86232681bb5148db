// huffman.h -- Huffman code lengths and canonical codewords (host side).
//
// The code is built over the histogram of the quantization codes of the
// whole field (the Huffman stage of the SZ pipeline, Sec. 3.1; Algorithm 1).
// The tree merges the used symbols in (count, symbol) order with two queues,
// the sorted leaves and the internal nodes in creation order, a tie going to
// the leaf; one used symbol gets length 1.  A tree deeper than the length
// limit halves every count (keeping at least 1) and is built again; ties
// among halved counts go by symbol.
// Codewords are canonical: consecutive in symbol order within a length, the
// first code of length l being (first code of length l-1 + count of length
// l-1) << 1.
//
// Cost: one radix sort of the leaves.  Halving keeps the count order, so
// every rebuild reuses it: a build links parents only and reads the deepest
// leaf's depth off its path; the depths of all leaves are taken once, from
// the last tree, and only runs of tied halved counts whose depths differ are
// put in symbol order (at most one run per depth boundary).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace sdcsz {

struct HuffmanBuilder {
  std::vector<uint64_t> key, tmp;  // count << 16 | leaf index (index order = symbol order), sorted
  std::vector<uint64_t> lw, iw;    // leaf / internal weights, each followed by a +inf sentinel
  std::vector<uint32_t> up;        // parent (internal index) of leaf i at [i], of internal t at [S + t]
  std::vector<uint32_t> idep;      // depth of internal t
  std::vector<uint64_t> mark;      // one bit per leaf index
  uint32_t rebuilds = 0;

  // stable LSD radix sort by count; the digit width follows the largest
  // count and the number of keys (at most 16 bits, so that the buckets of a
  // pass stay in cache); the keys start in index order, so ties stay in it
  void sort_keys() {
    const size_t S = key.size();
    tmp.resize(S);
    uint64_t top = 1;
    for (uint64_t k : key) top = std::max(top, k >> 16);
    const int bits = 64 - __builtin_clzll(top);
    const int lg = 64 - __builtin_clzll((uint64_t)S);
    const int width = std::min(16, std::max(8, lg + 1));
    const int passes = (bits + width - 1) / width;
    const int db = (bits + passes - 1) / passes;
    const uint64_t mask = (1ull << db) - 1;
    std::vector<uint32_t> c(1u << db);
    for (int p = 0; p < passes; p++) {
      const int sh = 16 + db * p;
      std::fill(c.begin(), c.end(), 0);
      for (uint64_t k : key) c[(k >> sh) & mask]++;
      uint32_t acc = 0;
      for (uint32_t &x : c) {
        const uint32_t t = x;
        x = acc;
        acc += t;
      }
      for (uint64_t k : key) tmp[c[(k >> sh) & mask]++] = k;
      key.swap(tmp);
    }
  }

  // the two-queue tree over the weights max(1, count >> k) of the sorted
  // keys (a tie goes to the leaf); returns the depth of the first leaf,
  // which is the largest: leaves and internal nodes leave their queues in
  // order, so a node taken earlier never sits higher than one taken later.
  // The shape depends on the weights alone, and halving keeps their order.
  uint32_t build(uint32_t k) {
    const size_t S = key.size();
    constexpr uint64_t kInf = ~0ull;
    lw.resize(S + 1);
    iw.resize(S);
    up.resize(2 * S);
    for (size_t i = 0; i < S; i++) lw[i] = std::max<uint64_t>(1, (key[i] >> 16) >> k);
    lw[S] = kInf;
    iw[0] = kInf;
    size_t li = 0, ii = 0;
    for (size_t t = 0; t + 1 < S; t++) {
      uint64_t w = 0;
      for (int r = 0; r < 2; r++) {
        if (lw[li] <= iw[ii]) {
          w += lw[li];
          up[li++] = (uint32_t)t;
        } else {
          w += iw[ii];
          up[S + ii++] = (uint32_t)t;
        }
      }
      iw[t] = w;
      iw[t + 1] = kInf;
    }
    uint32_t d = 1;
    for (uint32_t v = up[0]; v + 2 < S; v = up[S + v]) d++;
    return d;
  }

  // lengths from the last tree.  With the counts halved k times the leaves
  // are ordered by (halved count, symbol); the keys here are ordered by
  // (count, symbol), which differs only inside runs of equal halved count.
  // Depths do not increase along the leaf order, so inside a run whose
  // depths differ, the run's depths go to its symbols in ascending order.
  void assign_lengths(std::vector<uint8_t> &len) {
    const size_t S = key.size();
    idep.resize(S - 1);
    idep[S - 2] = 0;
    for (size_t t = S - 2; t-- > 0;) idep[t] = idep[up[S + t]] + 1;
    mark.assign((S + 63) / 64, 0);
    size_t a = 0;
    while (a < S) {
      size_t b = a + 1;
      while (b < S && lw[b] == lw[a]) b++;
      const uint32_t da = idep[up[a]] + 1, db = idep[up[b - 1]] + 1;
      if (da == db) {
        for (size_t p = a; p < b; p++) len[key[p] & 0xFFFFu] = (uint8_t)da;
      } else {
        for (size_t p = a; p < b; p++) mark[(key[p] & 0xFFFFu) >> 6] |= 1ull << (key[p] & 63);
        size_t q = a;
        for (size_t w = 0; w < mark.size(); w++)
          for (uint64_t x = mark[w]; x; x &= x - 1) len[64 * w + __builtin_ctzll(x)] = (uint8_t)(idep[up[q++]] + 1);
        std::fill(mark.begin(), mark.end(), 0);
      }
      a = b;
    }
  }

  // lengths of the used symbols (ascending) with counts `cnt` (> 0, < 2^32)
  void lengths(const std::vector<uint64_t> &cnt, uint32_t max_len, std::vector<uint8_t> &len) {
    const size_t S = cnt.size();
    len.assign(S, 0);
    rebuilds = 0;
    if (S == 0) return;
    if (S == 1) {
      len[0] = 1;
      return;
    }
    key.resize(S);
    for (size_t i = 0; i < S; i++) key[i] = (cnt[i] << 16) | i;
    sort_keys();
    while (build(rebuilds) > max_len) rebuilds++;
    assign_lengths(len);
  }
};

// Canonical codewords of the used symbols (lengths in ascending symbol order).
inline void canonical_codes(const std::vector<uint8_t> &len, uint32_t max_len, std::vector<uint32_t> &code) {
  std::vector<uint32_t> count(max_len + 2, 0), next(max_len + 2, 0);
  for (auto l : len) count[l]++;
  uint32_t c = 0;
  for (uint32_t l = 1; l <= max_len; l++) {
    c = (c + count[l - 1]) << 1;
    next[l] = c;
  }
  code.resize(len.size());
  for (size_t i = 0; i < len.size(); i++) code[i] = next[len[i]]++;
}

}  // namespace sdcsz
