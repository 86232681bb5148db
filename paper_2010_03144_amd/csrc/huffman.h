// huffman.h -- Huffman code lengths and canonical codewords (host side).
//
// The code is built over the histogram of the quantization codes of the
// whole field (the Huffman stage of the SZ pipeline, Sec. 3.1; Algorithm 1).
// The tree merges the used symbols in (count, symbol) order with two queues,
// the sorted leaves and the internal nodes in creation order, a tie going to
// the leaf; one used symbol gets length 1.  A tree deeper than the length
// limit halves every count (keeping at least 1) and is built again.
// Codewords are canonical: consecutive in symbol order within a length, the
// first code of length l being (first code of length l-1 + count of length
// l-1) << 1.
//
// Cost: one radix sort of the leaves; each rebuild after halving keeps the
// order (halving is monotonic) except among leaves whose halved counts tie,
// which are re-merged by symbol in linear time.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace sdcsz {

struct HuffmanBuilder {
  std::vector<uint64_t> key, tmp;  // count << 16 | leaf index (index order = symbol order), sorted
  std::vector<uint64_t> wgt;
  std::vector<uint32_t> up, dep;
  uint32_t rebuilds = 0;

  // stable LSD radix sort by count, 8 bits per pass, skipping digits that
  // every key shares; the keys start in index order, so ties stay in it
  void sort_keys() {
    const size_t S = key.size();
    tmp.resize(S);
    uint32_t cnt[256];
    for (int sh = 16; sh < 48; sh += 8) {
      for (uint32_t &c : cnt) c = 0;
      for (uint64_t k : key) cnt[(k >> sh) & 0xFFu]++;
      if (cnt[(key[0] >> sh) & 0xFFu] == S) continue;
      uint32_t acc = 0;
      for (uint32_t &c : cnt) {
        const uint32_t t = c;
        c = acc;
        acc += t;
      }
      for (uint64_t k : key) tmp[cnt[(k >> sh) & 0xFFu]++] = k;
      key.swap(tmp);
    }
  }

  // halve the counts (at least 1) keeping the keys sorted: halving keeps the
  // count order, so only runs of equal halved counts need re-merging by
  // symbol (each run is at most three symbol-sorted pieces)
  void halve() {
    const size_t S = key.size();
    for (uint64_t &k : key) {
      const uint64_t c = std::max<uint64_t>(1, (k >> 16) >> 1);
      k = (c << 16) | (k & 0xFFFFu);
    }
    size_t a = 0;
    while (a < S) {
      size_t b = a + 1;
      while (b < S && (key[b] >> 16) == (key[a] >> 16)) b++;
      size_t m = a + 1;
      while (m < b && key[m - 1] <= key[m]) m++;
      while (m < b) {  // merge the next ascending piece into [a, m)
        size_t e = m + 1;
        while (e < b && key[e - 1] <= key[e]) e++;
        std::inplace_merge(key.begin() + a, key.begin() + m, key.begin() + e);
        m = e;
      }
      a = b;
    }
  }

  // depth of every leaf (in key order) of the two-queue tree; returns the largest
  uint32_t depths() {
    const size_t S = key.size();
    wgt.resize(2 * S - 1);
    up.resize(2 * S - 1);
    dep.resize(2 * S - 1);
    for (size_t i = 0; i < S; i++) wgt[i] = key[i] >> 16;
    size_t li = 0, ii = S, top = S;
    for (size_t m = 0; m + 1 < S; m++) {
      size_t pick[2];
      for (int r = 0; r < 2; r++) {
        const bool leaf = li < S && (ii >= top || wgt[li] <= wgt[ii]);
        pick[r] = leaf ? li++ : ii++;
      }
      wgt[top] = wgt[pick[0]] + wgt[pick[1]];
      up[pick[0]] = up[pick[1]] = (uint32_t)top;
      top++;
    }
    dep[2 * S - 2] = 0;
    uint32_t deepest = 0;
    for (size_t v = 2 * S - 2; v-- > 0;) {
      dep[v] = dep[up[v]] + 1;
      if (v < S) deepest = std::max(deepest, dep[v]);
    }
    return deepest;
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
    while (depths() > max_len) {
      halve();
      rebuilds++;
    }
    for (size_t i = 0; i < S; i++) len[key[i] & 0xFFFFu] = (uint8_t)dep[i];
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
