// Reads histograms (65536 u64 counts each) from stdin and writes, per
// histogram, the code lengths (65536 bytes) and canonical codewords (65536
// u32, 0 for unused symbols) that the library's host-side codebook builder
// gives, for comparison with the oracle.
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "huffman.h"

int main() {
  std::vector<uint64_t> hist(65536);
  sdcsz::HuffmanBuilder b;
  std::vector<uint64_t> cnt;
  std::vector<uint8_t> len;
  std::vector<uint32_t> code;
  while (fread(hist.data(), 8, 65536, stdin) == 65536) {
    cnt.clear();
    std::vector<uint32_t> sym;
    for (uint32_t s = 0; s < 65536; s++)
      if (hist[s]) {
        cnt.push_back(hist[s]);
        sym.push_back(s);
      }
    b.lengths(cnt, 24, len);
    sdcsz::canonical_codes(len, 24, code);
    std::vector<uint8_t> out_len(65536, 0);
    std::vector<uint32_t> out_code(65536, 0);
    for (size_t i = 0; i < sym.size(); i++) {
      out_len[sym[i]] = len[i];
      out_code[sym[i]] = code[i];
    }
    fwrite(out_len.data(), 1, 65536, stdout);
    fwrite(out_code.data(), 4, 65536, stdout);
  }
  return 0;
}
