// common.h -- definitions shared by the library's kernels and its host code.
//
// Stream format, block geometry and the per-call device work areas of the
// SDC-resilient independent-block compressor (arXiv 2010.03144).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sdcsz.h"

namespace sdcsz {

constexpr uint32_t kRadius = 32768;  // code of a zero residual; 0 marks an outlier
constexpr uint32_t kMaxLen = 24;     // longest Huffman codeword
constexpr uint64_t kHeader = 192;    // fixed stream header bytes
static_assert(kHeader == SDCSZ_HEADER_BYTES, "header size");
constexpr uint32_t kMaxBlockPts = 8192;
constexpr uint32_t kMaxPatches = 8;  // fault-plan entries per block and call
constexpr uint32_t kMaxRedo = 4096;  // blocks re-run after a detected mismatch

// Result slots (u64) of a compression call, next to the counters.
enum { R_SIZE = 0, R_OUTLIERS, R_REGRESSION, R_WORDS, R_WRITTEN, R_EB, R_N = 8 };

// Counter slots (u64) in the device report area.
enum {
  C_INJ = 0,
  C_DET = SDCSZ_N_TARGETS,
  C_COR = 2 * SDCSZ_N_TARGETS,
  C_UNC = 3 * SDCSZ_N_TARGETS,
  C_MISSING = 4 * SDCSZ_N_TARGETS,  // a code without codeword was met while encoding
  C_HIST_DONE,                       // histogram chunks finished (the call's first job only)
  C_LIST,                            // fault-plan blocks run by the generic per-block routine
  C_REDO2,                           // decompression: blocks the fault-applying decoder queued
  C_SPIN,                            // compression: a look-back that gave up waiting (never expected)
  C_N = 42
};
static_assert(C_SPIN < C_N, "counter layout");

// Block grid of a field normalised to three axes (leading axes of extent 1).
struct Geo {
  uint64_t d[3];
  uint32_t b[3];
  uint32_t nb[3];
  uint32_t rem[3];  // extent of the last block along each axis
  uint32_t ndim;    // dimensionality of the block as configured (1..3)
  uint32_t bpts;    // points of a full block
  uint32_t groups;  // 4-code groups per block in the code staging layout
  uint64_t n_blocks;
  uint64_t n_values;
};

// Error-bound constants, written on the device by the constants kernel.
struct EbDev {
  double eb_abs;
  double q, inv, inv_e;    // 2eb, 1/(2eb), 1/eb
  float qf, invf, inv_ef;  // the same rounded to FP32
  float lo, hi;            // FP32 |x - r| <= lo passes, > hi fails the bound;
                           // in between the double comparison decides
};

// Regression constants per partial-block pattern (bit a set: axis a partial).
template <typename T> struct RegTab {
  T K[8][3];     // 12 / (n (n_a^2 - 1)), 0 when n_a == 1
  T inv_pts[8];  // 1 / n
  T c[8][3];     // (n_a - 1) / 2
};

// Fault plan on the device: entries sorted by block and one bit per block
// with entries (bits).  On a field of the lane-per-block kernels, list holds
// the plan blocks the wave-per-block routine takes and flist those the
// lane-per-block kernels' fault-applying instantiation takes (both
// ascending); the production instantiation leaves every plan block.
struct PlanDev {
  const sdcsz_fault *f;
  uint32_t n;
  const uint32_t *bits;
  const uint64_t *list, *flist;
  uint32_t nlist, nflist;
};

// Per-call device areas of compression (inside the caller's workspace).
struct CompWork {
  uint16_t *codes;     // interleaved staging layout (see code_index)
  void *vals;          // bpts values per block: outliers, packed in order
  void *recon;         // bpts values per block (generic kernels only)
  uint32_t *meta;      // per block: n_outliers << 1 | is_regression
  uint32_t *words;     // per block: payload words
  void *coef;          // 4 values per block
  uint64_t *sum_dc;    // per block
  uint64_t *sum_q;     // per block
  uint64_t *isum_q;    // per block
  uint32_t *hist;      // 65536
  uint32_t *enc;       // 65536: codeword << 8 | length
  unsigned long long *cnt;  // C_N counters
  uint64_t *off_pay;   // n_blocks + 1
  uint32_t *off_out;   // n_blocks + 1
  uint32_t *off_coef;  // n_blocks + 1
  uint64_t *scan_part; // 3 per scan chunk
  void *range_part;    // 2 doubles + flag per range work-group
  EbDev *eb;
  uint32_t *redo_n;    // blocks queued for a re-run
  uint64_t *redo;      // kMaxRedo entries of 3 words: block | reason << 56, first-pass S and Q
  uint64_t *tiles;     // one-pass code check and encoding: a status word per tile of 256 blocks
  uint32_t *ticket;    // and the next tile to hand out (both cleared at the start of a call)
  struct Header *hdr;  // stream header, filled on the device
  uint64_t *res;       // R_* results of the call, read back once at its end
  uint8_t *hdr_bytes;  // the stream's kHeader header bytes, read back with the results
  uint32_t *cb;        // n_sym pairs (symbol << 8 | length, codeword), ascending symbols
  uint64_t *tot;       // scanned totals: payload words, outliers, regression blocks
};

// Decoder tables built from the stream's codebook (canonical code).
struct DecTab {
  uint32_t first[kMaxLen + 2];
  uint32_t count[kMaxLen + 2];
  uint32_t start[kMaxLen + 2];
  uint32_t min_len, max_len;
  uint32_t sub_n;  // entries of the second-level table (0: not built, lut2 falls back to the search)
};

struct DecWork {
  uint16_t *symbols;   // 65536: symbols ordered by (length, symbol)
  DecTab *tab;
  void *recon;         // bpts values per block (generic kernels only)
  uint64_t *off_pay;   // n_blocks + 1
  uint32_t *off_out;
  uint32_t *off_coef;
  uint64_t *scan_part;
  unsigned long long *cnt;
  uint32_t *lut;       // 2^kLutBits entries: symbol << 8 | length (0: longer code)
  uint32_t *lut2;      // the same prefixes for the specialised decoder (two-level, see kLut2Sub)
  uint32_t *sub;       // kSubMax entries: second level of lut2, symbol << 8 | length
  uint32_t *redo_n;    // blocks queued for re-execution
  uint64_t *redo;      // 2 kMaxRedo entries, block | reason << 56: the production decoder's
                       // queue, then the fault-applying decoder's (count cnt[C_REDO2])
  uint32_t *err;       // non-zero: the codebook or the block table is not valid
  uint64_t *tot;       // scanned totals: payload words, outliers, regression blocks
};

constexpr uint32_t kLutBits = 11;  // codeword prefix resolved by one table lookup
// lut2 entries: symbol << 8 | length for a codeword of at most kLutBits bits;
// for a prefix that only longer codewords (lengths lmin..lmax) start with,
// off << 12 | w << 8 when its second level was built (2^w entries from
// sub[off], indexed by the next w = min(lmax - kLutBits, kSubBits) bits),
// else kLut2Search | lmax << 16 | lmin << 8; 0 if no codeword starts with
// the prefix.  A second-level entry is symbol << 8 | length, or, for bits
// that only codewords longer than kLutBits + w start with, kLut2Search |
// lmax << 16 | (kLutBits + w + 1) << 8 (the lengths left to search), or 0.
constexpr uint32_t kLut2Search = 0x80000000u;
constexpr uint32_t kSubBits = 8;
constexpr uint32_t kSubMax = 65536;  // second-level entries of one codebook at most

// Stream header fields (byte offsets inside the 192-byte header).
struct Header {
  uint32_t dtype, ndim;
  uint64_t d[3];
  uint32_t b[3];
  uint32_t eb_mode;
  double eb, eb_abs;
  uint32_t abft, n_sym;
  uint64_t n_blocks, n_outliers, n_regression, payload_words;
  uint64_t off_codebook, off_table, off_coef, off_sumdc, off_outliers, off_payload, total;
  uint32_t predictor;
};

__host__ __device__ inline uint64_t align8(uint64_t v) { return (v + 7) & ~7ull; }

// Section offsets from the counts in the header: codebook, block table,
// coefficients, sum_dc (ABFT only), outliers, payload; each 8-byte aligned.
__host__ __device__ inline void section_offsets(Header &h) {
  const uint64_t vb = h.dtype == SDCSZ_F32 ? 4 : 8;
  h.off_codebook = kHeader;
  h.off_table = align8(h.off_codebook + 4ull * h.n_sym);
  h.off_coef = h.off_table + 8ull * h.n_blocks;
  h.off_sumdc = align8(h.off_coef + 4ull * vb * h.n_regression);
  h.off_outliers = h.off_sumdc + (h.abft ? 8ull * h.n_blocks : 0);
  h.off_payload = align8(h.off_outliers + vb * h.n_outliers);
  h.total = align8(h.off_payload + 4ull * h.payload_words);
}

}  // namespace sdcsz
