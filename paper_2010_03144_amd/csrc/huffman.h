// huffman.h -- Huffman code lengths and canonical codewords (host side).
//
// The code is built over the histogram of the quantization codes of the
// whole field (the Huffman stage of the SZ pipeline, Sec. 3.1; Algorithm 1).  The tree
// merges the used symbols in (count, symbol) order with two queues, the
// sorted leaves and the internal nodes in creation order, a tie going to the
// leaf; one used symbol gets length 1.  A tree deeper than the length limit
// halves every count (keeping at least 1) and is built again.  Codewords are
// canonical: consecutive in symbol order within a length, the first code of
// length l being (first code of length l-1 + count of length l-1) << 1.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace sdcsz {

// Lengths of the used symbols from their counts (both in ascending symbol
// order, every count > 0).
inline void huffman_lengths(std::vector<uint64_t> cnt, uint32_t max_len, std::vector<uint8_t> &len) {
  const size_t S = cnt.size();
  len.assign(S, 0);
  if (S == 0) return;
  if (S == 1) {
    len[0] = 1;
    return;
  }
  std::vector<uint32_t> ord(S), up(2 * S - 1), dep(2 * S - 1);
  std::vector<uint64_t> wgt(2 * S - 1);
  for (;;) {
    for (size_t i = 0; i < S; i++) ord[i] = (uint32_t)i;
    std::sort(ord.begin(), ord.end(),
              [&](uint32_t a, uint32_t b) { return cnt[a] != cnt[b] ? cnt[a] < cnt[b] : a < b; });
    for (size_t i = 0; i < S; i++) wgt[i] = cnt[ord[i]];
    // nodes 0..S-1: leaves in sorted order; S..2S-2: internal, in creation order
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
    // parents come after their children: depths from the root downwards
    dep[2 * S - 2] = 0;
    for (size_t v = 2 * S - 2; v-- > 0;) dep[v] = dep[up[v]] + 1;
    uint32_t deepest = 0;
    for (size_t i = 0; i < S; i++) deepest = std::max(deepest, dep[i]);
    if (deepest <= max_len) {
      for (size_t i = 0; i < S; i++) len[ord[i]] = (uint8_t)dep[i];
      return;
    }
    for (auto &c : cnt) c = std::max<uint64_t>(1, c >> 1);
  }
}

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
