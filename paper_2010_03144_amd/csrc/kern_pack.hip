// kern_pack.hip -- the lossless stage behind the Huffman coder (the last
// pass of Algorithm 1, undone first by Algorithm 2).
//
// The payload of Huffman codewords holds almost no redundancy a byte coder
// could take out; the per-block metadata does: each block's payload length,
// its outlier count and predictor flag, and with ABFT its 64-bit checksum
// sum_dc.  These columns are cut into chunks of kPackChunk blocks and each
// chunk column is stored by frame of reference:
//   u32 base (low), u32 base (high), u32 width w (0..64), then ceil(n w / 32)
//   words; value i - base takes bits [i w, (i + 1) w) of the column's bit
//   string, whose bit t is bit t % 32 of word t / 32.
// A section is u32 offsets of its chunks (nch + 1, in words after the
// offsets, the first 0) and then the chunks: the table section holds the two
// table columns of every chunk, the sum_dc section (ABFT streams) the sum_dc
// column.  One block's entries are found from its chunk alone, so random
// access to blocks survives.  A packed stream keeps the header (magic "v2")
// and puts codebook, coefficients, outliers and payload first, unchanged,
// then the table section and the sum_dc section, each 8-byte aligned.
//
// Packing: k_pack_sizes (one work-group per chunk: minima, widths, chunk
// words), k_pack_scan (one work-group: offsets and section sizes), then
// k_pack_write (one work-group per chunk: offsets, columns, header, pads).
// Unpacking: k_unpack_check (section extents, header, pads) and
// k_unpack_chunks (one work-group per chunk, every read bounded by the
// extents checked before it).
#include "kern.h"

namespace sdcsz {

namespace {

constexpr uint32_t kPackThreads = 256;
static_assert(kPackThreads == kPackChunk, "one thread per block of a chunk");
constexpr uint32_t kScanT = 1024;

__device__ inline uint32_t width_of(uint64_t v) { return v ? 64u - (uint32_t)__clzll((long long)v) : 0u; }
__device__ inline uint32_t col_words(uint32_t n, uint32_t w) { return (uint32_t)(((uint64_t)n * w + 31) / 32); }
__device__ inline uint32_t chunk_n(uint64_t nb, uint64_t c) {
  const uint64_t left = nb - c * kPackChunk;
  return left < kPackChunk ? (uint32_t)left : kPackChunk;
}

// block b0 + i's table entry (payload words, outliers << 1 | regression) and sum_dc
__device__ inline void load_entry(const PackArgs &a, uint64_t b, uint64_t v[3]) {
  const uint2 e = *(const uint2 *)(a.src + a.src_table + 8 * b);
  v[0] = e.x;
  v[1] = e.y;
  v[2] = a.abft ? *(const uint64_t *)(a.src + a.src_sumdc + 8 * b) : 0;
}

// minimum and maximum over the 256 threads (lanes outside the chunk pass lo = ~0, hi = 0)
__device__ inline void wg_minmax(uint64_t &lo, uint64_t &hi, uint64_t *sl, uint64_t *sh) {
  for (int m = 32; m; m >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, m), h2 = __shfl_xor(hi, m);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  const uint32_t wv = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    sl[wv] = lo;
    sh[wv] = hi;
  }
  __syncthreads();
  lo = sl[0];
  hi = sh[0];
  for (uint32_t k = 1; k < kPackThreads / 64; k++) {
    lo = sl[k] < lo ? sl[k] : lo;
    hi = sh[k] > hi ? sh[k] : hi;
  }
  __syncthreads();
}

// ORs difference d of value i into the column's packed words
__device__ inline void put_bits(uint32_t *pk, uint32_t i, uint32_t w, uint64_t d) {
  if (w == 0) return;
  const uint32_t bit = i * w, q = bit >> 5, s = bit & 31;
  atomicOr(&pk[q], (uint32_t)(d << s));
  if (s + w > 32) atomicOr(&pk[q + 1], (uint32_t)(d >> (32 - s)));
  if (s + w > 64) atomicOr(&pk[q + 2], (uint32_t)(d >> (64 - s)));
}

// value i's difference from packed words pk (two zero words past the column)
__device__ inline uint64_t get_bits(const uint32_t *pk, uint32_t i, uint32_t w) {
  if (w == 0) return 0;
  const uint32_t bit = i * w, q = bit >> 5, s = bit & 31;
  uint64_t d = ((uint64_t)pk[q] | ((uint64_t)pk[q + 1] << 32)) >> s;
  if (s && s + w > 64) d |= (uint64_t)pk[q + 2] << (64 - s);
  return w < 64 ? d & ((1ull << w) - 1) : d;
}

// one chunk column: base, width, packed words
__device__ inline void write_column(uint32_t *o, const uint32_t *pk, uint64_t base, uint32_t w, uint32_t n) {
  const uint32_t nw = 3 + col_words(n, w);
  for (uint32_t j = threadIdx.x; j < nw; j += kPackThreads)
    o[j] = j == 0 ? (uint32_t)base : j == 1 ? (uint32_t)(base >> 32) : j == 2 ? w : pk[j - 3];
}

}  // namespace

__global__ __launch_bounds__(kPackThreads) void k_pack_sizes(PackArgs a) {
  __shared__ uint64_t sl[4], sh[4];
  const uint64_t c = blockIdx.x, b0 = c * kPackChunk;
  const uint32_t n = chunk_n(a.nb, c), i = threadIdx.x;
  uint64_t v[3] = {0, 0, 0};
  if (i < n) load_entry(a, b0 + i, v);
  PackChunk ci;
  const int ncol = a.abft ? 3 : 2;
  for (int k = 0; k < 3; k++) {
    uint64_t lo = i < n ? v[k] : ~0ull, hi = i < n ? v[k] : 0;
    if (k < ncol) wg_minmax(lo, hi, sl, sh);
    else lo = hi = 0;
    ci.base[k] = lo;
    ci.width[k] = width_of(hi - lo);
  }
  if (i == 0) {
    ci.words_t = 6 + col_words(n, ci.width[0]) + col_words(n, ci.width[1]);
    ci.words_s = a.abft ? 3 + col_words(n, ci.width[2]) : 0;
    ci.off_t = ci.off_s = 0;
    a.info[c] = ci;
  }
}

// Exclusive offsets of the chunks in both sections and the sections' sizes
// (one work-group; each thread takes a run of consecutive chunks).
__global__ __launch_bounds__(kScanT) void k_pack_scan(PackArgs a) {
  __shared__ uint32_t part[2][kScanT];
  const uint32_t t = threadIdx.x;
  const uint64_t per = (a.nch + kScanT - 1) / kScanT;
  const uint64_t c0 = min(a.nch, t * per), c1 = min(a.nch, c0 + per);
  uint32_t st = 0, ss = 0;
  for (uint64_t c = c0; c < c1; c++) {
    st += a.info[c].words_t;
    ss += a.info[c].words_s;
  }
  part[0][t] = st;
  part[1][t] = ss;
  __syncthreads();
  for (uint32_t d = 1; d < kScanT; d <<= 1) {
    const uint32_t pt = t >= d ? part[0][t - d] : 0, ps = t >= d ? part[1][t - d] : 0;
    __syncthreads();
    part[0][t] += pt;
    part[1][t] += ps;
    __syncthreads();
  }
  uint32_t rt = part[0][t] - st, rs = part[1][t] - ss;
  for (uint64_t c = c0; c < c1; c++) {
    a.info[c].off_t = rt;
    a.info[c].off_s = rs;
    rt += a.info[c].words_t;
    rs += a.info[c].words_s;
  }
  if (t == kScanT - 1) {
    a.res[0] = part[0][t];
    a.res[1] = part[1][t];
  }
}

// Chunk c's columns and its entry in the sections' offsets; work-group 0
// also writes the leading offsets, the header and the alignment pads.
__global__ __launch_bounds__(kPackThreads) void k_pack_write(PackArgs a) {
  __shared__ uint32_t pk[3][kPackColWords];
  const uint64_t c = blockIdx.x, b0 = c * kPackChunk;
  const uint32_t n = chunk_n(a.nb, c), i = threadIdx.x;
  uint32_t *d = (uint32_t *)a.dst;
  if (c == 0) {
    for (uint32_t j = i; j < kHeader / 4; j += kPackThreads) d[j] = a.hdr[j];
    if (i < a.n_pads) d[a.pads[i] / 4] = 0;
    if (i == 0) {
      d[a.dst_table / 4] = 0;
      if (a.abft) d[a.dst_sumdc / 4] = 0;
    }
  }
  if (c >= a.nch) return;  // a stream without blocks: the header work only
  const PackChunk ci = a.info[c];
  for (uint32_t j = i; j < 3 * kPackColWords; j += kPackThreads) (&pk[0][0])[j] = 0;
  __syncthreads();
  if (i < n) {
    uint64_t v[3];
    load_entry(a, b0 + i, v);
    put_bits(pk[0], i, ci.width[0], v[0] - ci.base[0]);
    put_bits(pk[1], i, ci.width[1], v[1] - ci.base[1]);
    if (a.abft) put_bits(pk[2], i, ci.width[2], v[2] - ci.base[2]);
  }
  __syncthreads();
  uint32_t *tsec = d + a.dst_table / 4;
  if (i == 0) tsec[c + 1] = ci.off_t + ci.words_t;
  uint32_t *o = tsec + a.nch + 1 + ci.off_t;
  write_column(o, pk[0], ci.base[0], ci.width[0], n);
  write_column(o + 3 + col_words(n, ci.width[0]), pk[1], ci.base[1], ci.width[1], n);
  if (a.abft) {
    uint32_t *ssec = d + a.dst_sumdc / 4;
    if (i == 0) ssec[c + 1] = ci.off_s + ci.words_s;
    write_column(ssec + a.nch + 1 + ci.off_s, pk[2], ci.base[2], ci.width[2], n);
  }
}

// A section [off, end) of nch chunks: its offsets fit, the first is 0, the
// last one's data ends where the 8-byte aligned section ends.
__device__ inline bool section_ok(const uint8_t *s, uint64_t off, uint64_t end, uint64_t nch) {
  if (end < off || end - off < 4 * (nch + 1)) return false;
  const uint32_t *w = (const uint32_t *)(s + off);
  const uint64_t used = 4 * (nch + 1 + (uint64_t)w[nch]);
  return w[0] == 0 && used <= end - off && align8(off + used) == end;
}

__global__ void k_unpack_check(UnpackArgs a) {
  uint32_t *d = (uint32_t *)a.dst;
  if (a.write) {
    for (uint32_t j = threadIdx.x; j < kHeader / 4; j += blockDim.x) d[j] = a.hdr[j];
    if (threadIdx.x < a.n_pads) d[a.pads[threadIdx.x] / 4] = 0;
  }
  if (threadIdx.x == 0) {
    bool ok = section_ok(a.src, a.src_table, a.src_sumdc, a.nch);
    if (a.abft) ok = ok && section_ok(a.src, a.src_sumdc, a.src_total, a.nch);
    *a.err = ok ? 0u : 1u;
  }
}

__global__ __launch_bounds__(kPackThreads) void k_unpack_chunks(UnpackArgs a) {
  __shared__ uint32_t pk[kPackColWords + 2];
  if (*(volatile uint32_t *)a.err) return;
  const uint64_t c = blockIdx.x, b0 = c * kPackChunk;
  const uint32_t n = chunk_n(a.nb, c), i = threadIdx.x;
  uint64_t v[3] = {0, 0, 0};
  const int nsec = a.abft ? 2 : 1;
  for (int sec = 0, k = 0; sec < nsec; sec++) {
    // every thread reads the same words and takes the same branches
    const uint32_t *w = (const uint32_t *)(a.src + (sec ? a.src_sumdc : a.src_table));
    const uint32_t *data = w + a.nch + 1;
    const uint64_t nwords = w[a.nch];
    const uint64_t w0 = w[c], w1 = w[c + 1];
    if (w1 < w0 || w1 > nwords) {
      if (i == 0) atomicOr(a.err, 1u);
      return;
    }
    uint64_t at = w0;
    const int ncol = sec ? 1 : 2;
    const uint32_t maxw = sec ? 64 : 32;
    for (int col = 0; col < ncol; col++, k++) {
      if (at + 3 > w1 || data[at + 2] > maxw) {
        if (i == 0) atomicOr(a.err, 1u);
        return;
      }
      const uint64_t base = (uint64_t)data[at] | ((uint64_t)data[at + 1] << 32);
      const uint32_t wd = data[at + 2];
      at += 3;
      const uint32_t nw = col_words(n, wd);
      if (at + nw > w1) {
        if (i == 0) atomicOr(a.err, 1u);
        return;
      }
      __syncthreads();  // the previous column's reads of pk are done
      for (uint32_t j = i; j < nw + 2; j += kPackThreads) pk[j] = j < nw ? data[at + j] : 0u;
      __syncthreads();
      if (i < n) v[k] = base + get_bits(pk, i, wd);
      at += nw;
    }
    if (at != w1) {
      if (i == 0) atomicOr(a.err, 1u);
      return;
    }
  }
  if (i >= n) return;
  if (v[0] > 0xFFFFFFFFull || v[1] > 0xFFFFFFFFull) atomicOr(a.err, 1u);
  if (!a.write) return;
  *(uint2 *)(a.dst + a.dst_table + 8 * (b0 + i)) = make_uint2((uint32_t)v[0], (uint32_t)v[1]);
  if (a.abft) *(uint64_t *)(a.dst + a.dst_sumdc + 8 * (b0 + i)) = v[2];
}

}  // namespace sdcsz
