// kern_stream.hip -- stream assembly and decoder tables on the device.
//
// Compression: the codeword table is scattered from the host's compact
// codebook list; once the scans are done, k_header derives the section
// offsets from the scanned totals and writes the header, the codebook
// section and the alignment pads, but only when the call met no
// uncorrectable error and the stream fits the caller's buffer (the encoder
// kernels read the same decision).  Decompression: k_dectab validates the
// codebook section and builds the canonical decoding tables; k_dec_check
// compares the scanned block table with the header's counts.  The host reads
// the outcome once, at the end of the call.
#include "dev.h"
#include "kern.h"

namespace sdcsz {

// enc[symbol] = codeword << 8 | length for each codebook entry.
__global__ void __launch_bounds__(256) k_put_codes(JobTab t) {
  const JobWg jw = job_of(t);
  const Job &J = *jw.J;
  const uint32_t i = jw.b * blockDim.x + threadIdx.x;
  if (i >= J.n_sym) return;
  const uint32_t e = J.cw.cb[2 * i], code = J.cw.cb[2 * i + 1];
  J.cw.enc[e >> 8] = (code << 8) | (e & 0xFFu);
}

// Histogram of each job compacted to (symbol << 32 | count) for the used
// symbols, in symbol order, all jobs one after another.  The 65536 symbols
// of a job are cut into kHistChunks chunks: k_hist_count counts the used
// symbols of every chunk (one work-group per chunk), k_hist_scan (one
// work-group) turns the counts into offsets and per-job totals, k_hist_pack
// writes every chunk's entries at its offset.  (Letting the count kernel's
// last work-group do the scan costs a device-scope fence per work-group,
// which on a batch's 12,288 work-groups took far longer than the launch it
// saves.)
constexpr uint32_t kHistChunks = 64, kHistChunk = 65536 / kHistChunks;
static_assert(kHistChunks == 64, "a job's chunk counts are one wave's lanes");

namespace {
// exclusive scan of one value per thread over a 256-thread work-group;
// *total: the sum over the work-group, *wave_total: over the thread's wave
__device__ inline uint32_t wg_exclusive_u32(uint32_t v, uint32_t *total, uint32_t *wave_total) {
  __shared__ uint32_t ws[4];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) ws[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, all = 0;
#pragma unroll
  for (uint32_t q = 0; q < 4; q++) {
    pre += q < wave ? ws[q] : 0u;
    all += ws[q];
  }
  *wave_total = ws[wave];
  __syncthreads();  // ws is free for the next call
  *total = all;
  return pre + inc - v;
}
}  // namespace

__global__ void __launch_bounds__(256) k_hist_count(JobTab t, uint32_t *chunk_cnt) {
  const JobWg jw = job_of(t);
  const uint32_t *hist = jw.J->cw.hist + jw.b * kHistChunk;
  uint32_t c = 0;
  for (uint32_t s = threadIdx.x; s < kHistChunk; s += blockDim.x) c += hist[s] ? 1u : 0u;
  for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off);
  __shared__ uint32_t wsum[4];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) chunk_cnt[jw.slot * kHistChunks + jw.b] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// one work-group: exclusive scan of the n * kHistChunks chunk counts in
// place, and each job's total into counts[] (a job's chunks are one wave)
// counts: per job, in device memory and (hcounts) in the caller's pinned staging.
__global__ void __launch_bounds__(256) k_hist_scan(uint32_t n, uint32_t *chunk_cnt, uint32_t *counts,
                                                   uint32_t *hcounts) {
  const uint32_t total = n * kHistChunks;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < total; base += 256) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < total ? chunk_cnt[i] : 0u;
    uint32_t all, job_total;
    const uint32_t ex = wg_exclusive_u32(v, &all, &job_total);
    if (i < total) chunk_cnt[i] = carry + ex;
    if (i < total && (threadIdx.x & 63) == 63) {
      counts[i / kHistChunks] = job_total;
      hcounts[i / kHistChunks] = job_total;
    }
    carry += all;
  }
}

// The pairs go to dst (device memory), and the first hn of them also to hdst
// (the caller's pinned staging, read after the synchronisation).
__global__ void __launch_bounds__(256) k_hist_pack(JobTab t, const uint32_t *chunk_off, uint64_t *dst, uint64_t *hdst,
                                                   uint64_t hn) {
  const JobWg jw = job_of(t);
  const uint32_t s0 = jw.b * kHistChunk;
  const uint32_t *hist = jw.J->cw.hist;
  constexpr uint32_t per = kHistChunk / 256;
  uint32_t mine = 0;
  for (uint32_t q = 0; q < per; q++) mine += hist[s0 + threadIdx.x * per + q] ? 1u : 0u;
  uint32_t all, wt;
  uint64_t at = chunk_off[jw.slot * kHistChunks + jw.b] + wg_exclusive_u32(mine, &all, &wt);
  for (uint32_t q = 0; q < per; q++) {
    const uint32_t s = s0 + threadIdx.x * per + q;
    const uint32_t c = hist[s];
    if (c) {
      const uint64_t v = ((uint64_t)s << 32) | c;
      dst[at] = v;
      if (at < hn) hdst[at] = v;
      at++;
    }
  }
}

// Each job's counters and results, one after another (per words each).
__global__ void __launch_bounds__(64) k_results(JobTab t, uint64_t *dst, uint32_t per) {
  const JobWg jw = job_of(t);
  for (uint32_t i = threadIdx.x; i < per; i += blockDim.x) dst[(uint64_t)jw.slot * per + i] = jw.J->stat[i];
}

// Each job's stream header, one after another.
__global__ void __launch_bounds__(64) k_headers(JobTab t, uint8_t *dst) {
  const JobWg jw = job_of(t);
  const uint32_t *src = (const uint32_t *)jw.J->src;
  uint32_t *d = (uint32_t *)(dst + (uint64_t)jw.slot * kHeader);
  for (uint32_t i = threadIdx.x; i < kHeader / 4; i += blockDim.x) d[i] = src[i];
}

namespace {

__device__ inline void put32(uint8_t *o, uint32_t off, uint32_t v) { *(uint32_t *)(o + off) = v; }
__device__ inline void put64(uint8_t *o, uint32_t off, uint64_t v) {
  put32(o, off, (uint32_t)v);
  put32(o, off + 4, (uint32_t)(v >> 32));
}

// The 192-byte header: magic "SDCSZ\0v1", then the fields at fixed offsets
// (unused bytes zero).
__device__ void write_header(const Header &h, uint8_t *o) {
  for (uint32_t off = 0; off < kHeader; off += 4) put32(o, off, 0u);
  put32(o, 0, 0x53434453u);  // 'S' 'D' 'C' 'S'
  put32(o, 4, 0x3176005Au);  // 'Z' 0 'v' '1'
  put32(o, 8, h.dtype);
  put32(o, 12, h.ndim);
  for (uint32_t a = 0; a < 3; a++) put64(o, 16 + 8 * a, h.d[a]);
  for (uint32_t a = 0; a < 3; a++) put32(o, 40 + 4 * a, h.b[a]);
  put32(o, 52, h.eb_mode);
  put64(o, 56, (uint64_t)__double_as_longlong(h.eb));
  put64(o, 64, (uint64_t)__double_as_longlong(h.eb_abs));
  put32(o, 72, h.abft);
  put32(o, 76, h.n_sym);
  put64(o, 80, h.n_blocks);
  put64(o, 88, h.n_outliers);
  put64(o, 96, h.n_regression);
  put64(o, 104, h.payload_words);
  put64(o, 112, h.off_codebook);
  put64(o, 120, h.off_table);
  put64(o, 128, h.off_coef);
  put64(o, 136, h.off_sumdc);
  put64(o, 144, h.off_outliers);
  put64(o, 152, h.off_payload);
  put64(o, 160, h.total);
  put32(o, 168, h.predictor);
}

}  // namespace

// Completes the header (fixed fields set by the host) from the device
// results and decides whether the stream is written: no uncorrectable error
// in the input, coefficient or code stages, no code without a codeword, and
// the stream fits the caller's buffer.  One thread per codebook entry (>= 1).
__global__ void __launch_bounds__(256) k_header(JobTab tb) {
  const JobWg jw = job_of(tb);
  Header h = jw.J->h;
  const CompWork &w = jw.J->cw;
  uint8_t *out = jw.J->dst;
  const uint64_t out_cap = jw.J->dst_cap;
  h.eb_abs = w.eb->eb_abs;
  const uint64_t *tot = w.tot;  // left by the scan (zero without blocks)
  h.payload_words = tot[0];
  h.n_outliers = tot[1];
  h.n_regression = tot[2];
  section_offsets(h);
  const unsigned long long *c = w.cnt;
  const bool unc = c[C_UNC + SDCSZ_T_INPUT] || c[C_UNC + SDCSZ_T_COEF] || c[C_UNC + SDCSZ_T_CODE] ||
                   c[C_UNC + SDCSZ_T_PREP_INPUT] || c[C_MISSING];
  const bool ok = !unc && out != nullptr && h.total <= out_cap;
  const uint32_t t = jw.b * blockDim.x + threadIdx.x;
  if (t == 0) {
    w.res[R_SIZE] = h.total;
    w.res[R_OUTLIERS] = h.n_outliers;
    w.res[R_REGRESSION] = h.n_regression;
    w.res[R_WORDS] = h.payload_words;
    w.res[R_WRITTEN] = ok ? 1u : 0u;
    w.res[R_EB] = (uint64_t)__double_as_longlong(h.eb_abs);
    *w.hdr = h;
  }
  if (!ok) return;
  if (t < h.n_sym) put32(out, (uint32_t)(kHeader + 4 * t), w.cb[2 * t]);
  if (t == 0) {
    write_header(h, out);
    write_header(h, w.hdr_bytes);  // the caller's copy
    const uint64_t vb = h.dtype == SDCSZ_F32 ? 4 : 8;
    // 4-byte alignment pads after the codebook, the outliers and the payload
    if (h.off_table > kHeader + 4ull * h.n_sym) put32(out + kHeader, 4 * h.n_sym, 0u);
    const uint64_t out_end = h.off_outliers + vb * h.n_outliers;
    if (h.off_payload > out_end) *(uint32_t *)(out + out_end) = 0u;
    const uint64_t pay_end = h.off_payload + 4ull * h.payload_words;
    if (h.total > pay_end) *(uint32_t *)(out + pay_end) = 0u;
  }
}

// Canonical decoding tables from the codebook section (one u32 per used
// symbol: symbol << 8 | length).  The entries must name distinct symbols
// with lengths 1..kMaxLen; codes follow (length, symbol) order.  Writes
// w.symbols (symbols by (length, symbol)), w.tab (first code, count and
// first position per length) and w.lut (for each kLutBits-bit prefix the
// shortest codeword it starts with, symbol << 8 | length; for a prefix that
// only longer codewords start with, the range of their lengths,
// lmax << 16 | lmin << 8; 0 if none); sets *w.err on an invalid codebook.
// One work-group of kDecTabThreads threads (the serial parts of a thread's
// work shrink with more threads, and four waves per SIMD hide the LDS
// latency).  Up to 4096 entries in ascending symbol order (as the
// compressor writes them) are ranked per length with wave ballots; more
// entries, or any other order, go through a table of the lengths of all
// 65536 symbols.
__global__ void __launch_bounds__(kDecTabThreads) k_dectab(JobTab tb) {
  const Job &J = *job_of(tb).J;
  const uint32_t *cbk = (const uint32_t *)(J.src + kHeader);
  const uint32_t n_sym = J.h.n_sym;
  const DecWork &w = J.dw;
  __shared__ uint32_t lens4[65536 / 4];       // code length of each symbol, one byte each
  __shared__ uint16_t part[kMaxLen + 1][kDecTabThreads];  // per length: symbols before each thread's range, in its wave
  __shared__ uint32_t wsum[kMaxLen + 1][kDecTabWaves];    // per length: symbols in each wave's part
  __shared__ uint32_t run[kMaxLen + 1];        // per length: symbols placed so far
  __shared__ uint16_t short_sym[1u << kLutBits];  // symbols at positions < 2^kLutBits
  __shared__ uint32_t first[kMaxLen + 2], cnt[kMaxLen + 2], start[kMaxLen + 2];
  __shared__ uint32_t smin, smax, bad, unordered, hmis;
  __shared__ uint32_t pe[1u << kLutBits];       // lut entry of each prefix
  __shared__ uint32_t poff[(1u << kLutBits) + 1];  // second-level offset of each prefix
  __shared__ uint32_t ptot[kDecTabWaves];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool small = n_sym <= 4096;
  // a header the caller supplied (the host sized everything from it) must be
  // the stream's own, word for word
  if (J.hdr_expect) {
    if (tid == 0) hmis = 0;
    __syncthreads();
    if (tid < kHeader / 4 && ((const uint32_t *)J.src)[tid] != J.hdr_expect[tid]) atomicOr(&hmis, 1u);
    __syncthreads();
    if (hmis) {
      if (tid == 0) *w.err = 1;
      return;
    }
  }
  if (tid <= kMaxLen) {
    cnt[tid] = 0;
    run[tid] = 0;
  }
  if (tid == 0) {
    smin = 0xFFFFFFFFu;
    smax = 0;
    bad = 0;
    unordered = 0;
  }
  auto len_of = [&](uint32_t s) { return (lens4[s >> 2] >> (8 * (s & 3))) & 0xFFu; };
  if (!small)
    for (uint32_t i = tid; i < 65536 / 4; i += kDecTabThreads) lens4[i] = 0;
  __syncthreads();
  // one pass over the entries, kU at a time per thread (their loads in
  // flight together): validity and order; few entries are counted per
  // length here, many go into the table of lengths by symbol (a symbol
  // listed twice is an error)
  constexpr uint32_t kU = 8;
  uint32_t elo = 0xFFFFFFFFu, ehi = 0;
  for (uint32_t base = tid; base < n_sym; base += kDecTabThreads * kU) {
    uint32_t ev[kU], pv[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint32_t t = base + u * kDecTabThreads;
      ev[u] = t < n_sym ? cbk[t] : 0u;
      pv[u] = t > 0 && t < n_sym ? cbk[t - 1] : 0u;
    }
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint32_t t = base + u * kDecTabThreads;
      if (t >= n_sym) continue;
      const uint32_t s = ev[u] >> 8, l = ev[u] & 0xFFu;
      if (s > 65535 || l == 0 || l > kMaxLen) {
        atomicOr(&bad, 1u);
        continue;
      }
      if (t > 0 && (pv[u] >> 8) >= s) atomicOr(&unordered, 1u);
      if (small) {
        atomicAdd(&cnt[l], 1u);
      } else {
        const uint32_t sh = 8 * (s & 3);
        const uint32_t old = atomicOr(&lens4[s >> 2], l << sh);
        if ((old >> sh) & 0xFFu) atomicOr(&bad, 1u);
        elo = min(elo, s);
        ehi = max(ehi, s);
      }
    }
  }
  if (!small) {
    for (int off = 32; off > 0; off >>= 1) {
      elo = min(elo, (uint32_t)__shfl_xor((int)elo, off));
      ehi = max(ehi, (uint32_t)__shfl_xor((int)ehi, off));
    }
    if (lane == 0) {
      atomicMin(&smin, elo);
      atomicMax(&smax, ehi);
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) *w.err = 1;
    return;
  }
  // entries in ascending symbol order are ranked with ballots, a chunk of
  // kDecTabThreads at a time; many entries (or any other order) go through the table of
  // the lengths of all symbols, which ranks a thread's range of symbols at
  // once (the ballot loop took 0.24 ms for 65,536 entries)
  const bool ordered = !unordered && small;
  uint32_t a = 0, b = 0;  // unordered case: this thread's range of the symbol span
  if (!ordered && small) {
    // few entries out of order: their lengths by symbol (a symbol listed
    // twice is an error)
    for (uint32_t i = tid; i < 65536 / 4; i += kDecTabThreads) lens4[i] = 0;
    __syncthreads();
    uint32_t lo = 0xFFFFFFFFu, hi = 0;  // this thread's extremes, then one atomic per wave
    for (uint32_t t = tid; t < n_sym; t += kDecTabThreads) {
      const uint32_t e = cbk[t], s = e >> 8, l = e & 0xFFu;
      const uint32_t sh = 8 * (s & 3);
      const uint32_t old = atomicOr(&lens4[s >> 2], l << sh);
      if ((old >> sh) & 0xFFu) atomicOr(&bad, 1u);
      lo = min(lo, s);
      hi = max(hi, s);
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
      hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
    }
    if (lane == 0) {
      atomicMin(&smin, lo);
      atomicMax(&smax, hi);
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) *w.err = 1;
      return;
    }
  }
  if (!ordered) {
    // counts per length over contiguous symbol ranges, one per thread
    const uint32_t span = smax >= smin ? smax - smin + 1 : 0;
    const uint32_t per = (span + kDecTabThreads - 1) / kDecTabThreads;
    a = smin + tid * per;
    b = min(a + per, smin + span);
    uint32_t mine[kMaxLen + 1];
#pragma unroll
    for (uint32_t l = 0; l <= kMaxLen; l++) mine[l] = 0;
    for (uint32_t s = a; s < b; s++) {
      const uint32_t l = len_of(s);
#pragma unroll
      for (uint32_t m = 1; m <= kMaxLen; m++) mine[m] += l == m ? 1u : 0u;
    }
#pragma unroll
    for (uint32_t l = 1; l <= kMaxLen; l++) {
      uint32_t v = mine[l];
#pragma unroll
      for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)v, d);
        if (lane >= d) v += u;
      }
      part[l][tid] = (uint16_t)(v - mine[l]);
      if (lane == 63) wsum[l][wave] = v;
    }
    __syncthreads();
    if (tid <= kMaxLen) {
      uint32_t acc = 0;
      for (uint32_t q = 0; q < kDecTabWaves; q++) {
        const uint32_t c = tid ? wsum[tid][q] : 0u;
        wsum[tid][q] = acc;
        acc += c;
      }
      if (!small && tid > 0) cnt[tid] = acc;  // symbols of length tid
    }
  }
  __syncthreads();
  if (tid == 0) {
    // first code of length l: (first code + count of length l - 1) << 1, in
    // 32-bit arithmetic (one past the last code of the previous used length,
    // extended to l bits)
    uint32_t code = 0, acc = 0, lo = kMaxLen + 1, hi = 0;
    first[0] = start[0] = 0;
    cnt[0] = 0;
    for (uint32_t l = 1; l <= kMaxLen; l++) {
      code = (code + cnt[l - 1]) << 1;
      first[l] = code;
      start[l] = acc;
      acc += cnt[l];
      if (cnt[l]) {
        lo = min(lo, l);
        hi = max(hi, l);
      }
    }
    DecTab *tb = w.tab;
    for (uint32_t l = 0; l < kMaxLen + 2; l++) {
      tb->first[l] = l <= kMaxLen ? first[l] : 0u;
      tb->count[l] = l <= kMaxLen ? cnt[l] : 0u;
      tb->start[l] = l <= kMaxLen ? start[l] : 0u;
    }
    tb->min_len = hi ? lo : 1u;
    tb->max_len = hi;
  }
  __syncthreads();
  auto place = [&](uint32_t pos, uint32_t s) {
    w.symbols[pos] = (uint16_t)s;
    if (pos < (1u << kLutBits)) short_sym[pos] = (uint16_t)s;
  };
  if (ordered) {
    // rank of each entry among the earlier entries of its length
    const uint64_t below = (1ull << lane) - 1;
    for (uint32_t base = 0; base < n_sym; base += kDecTabThreads) {
      const uint32_t t = base + tid;
      const uint32_t e = t < n_sym ? cbk[t] : 0u, l = e & 0xFFu;
      uint32_t rank = 0;
      for (uint32_t m = 1; m <= kMaxLen; m++) {
        const uint64_t mask = __ballot(l == m);
        if (l == m) rank = (uint32_t)__popcll(mask & below);
        if (lane == 0) wsum[m][wave] = (uint32_t)__popcll(mask);
      }
      __syncthreads();
      if (l) {
        uint32_t off = run[l];
        for (uint32_t q = 0; q < wave; q++) off += wsum[l][q];
        place(start[l] + off + rank, e >> 8);
      }
      __syncthreads();
      if (tid >= 1 && tid <= kMaxLen)
        for (uint32_t q = 0; q < kDecTabWaves; q++) run[tid] += wsum[tid][q];
      __syncthreads();
    }
  } else {
    for (uint32_t s = a; s < b; s++) {
      const uint32_t l = len_of(s);
      if (!l) continue;
      place(start[l] + wsum[l][wave] + part[l][tid]++, s);
    }
  }
  __syncthreads();
  // prefix table: for each kLutBits-bit prefix the first length whose top
  // bits fall among that length's codes (the rule of bit-by-bit decoding)
  for (uint32_t v = tid; v < (1u << kLutBits); v += kDecTabThreads) {
    uint32_t e = 0;
    for (uint32_t l = 1; l <= kLutBits; l++) {
      const uint32_t c = v >> (kLutBits - l);
      if (cnt[l] && c >= first[l] && c - first[l] < cnt[l]) {
        const uint32_t pos = start[l] + c - first[l];
        const uint32_t s = pos < (1u << kLutBits) ? (uint32_t)short_sym[pos] : (uint32_t)w.symbols[pos];
        e = (s << 8) | l;
        break;
      }
    }
    if (e == 0) {
      uint32_t lmin = 0, lmax = 0;
      for (uint32_t l = kLutBits + 1; l <= kMaxLen; l++) {
        if (!cnt[l]) continue;
        // 11-bit prefixes of the readable codes of length l (codes < 2^l)
        const uint64_t c0 = first[l], c1 = min((uint64_t)first[l] + cnt[l], 1ull << l);
        if (c0 >= c1) continue;
        const uint64_t p0 = c0 >> (l - kLutBits), p1 = (c1 - 1) >> (l - kLutBits);
        if (v >= p0 && v <= p1) {
          if (!lmin) lmin = l;
          lmax = l;
        }
      }
      if (lmin) e = (lmax << 16) | (lmin << 8);
    }
    w.lut[v] = e;
    pe[v] = e;
  }
  __syncthreads();
  // The specialised decoder's two-level table (lut2, sub): a prefix that
  // only codewords longer than kLutBits start with gets 2^(lmax - kLutBits)
  // second-level entries, one per value of the bits after it, each holding
  // the first length lmin..lmax whose codes take those bits (the rule of
  // bit-by-bit decoding again).  Offsets come from an exclusive scan over the
  // prefixes; beyond kSubMax entries in all the long prefixes keep the search.
  constexpr uint32_t kNP = 1u << kLutBits, kPer = kNP / kDecTabThreads;
  static_assert(kPer * kDecTabThreads == kNP, "prefixes per thread");
  uint32_t np[kPer], mine = 0;
#pragma unroll
  for (uint32_t u = 0; u < kPer; u++) {
    const uint32_t e = pe[tid * kPer + u];
    np[u] = (e && !(e & 0xFFu)) ? 1u << min((e >> 16) - kLutBits, kSubBits) : 0u;
    mine += np[u];
  }
  uint32_t inc = mine;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)inc, d);
    if (lane >= d) inc += u;
  }
  if (lane == 63) ptot[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, total = 0;
  for (uint32_t q = 0; q < kDecTabWaves; q++) {
    pre += q < wave ? ptot[q] : 0u;
    total += ptot[q];
  }
  uint32_t o = pre + inc - mine;
#pragma unroll
  for (uint32_t u = 0; u < kPer; u++) {
    poff[tid * kPer + u] = o;
    o += np[u];
  }
  if (tid == 0) poff[kNP] = total;
  __syncthreads();
  const bool build = total <= kSubMax;
#pragma unroll
  for (uint32_t u = 0; u < kPer; u++) {
    const uint32_t v = tid * kPer + u, e = pe[v];
    uint32_t e2 = e;
    if (e && !(e & 0xFFu))
      e2 = build ? (poff[v] << 12) | (min((e >> 16) - kLutBits, kSubBits) << 8) : (kLut2Search | e);
    w.lut2[v] = e2;
  }
  if (tid == 0) w.tab->sub_n = build ? total : 0u;
  if (!build) return;
  // each thread fills a contiguous run of entries: one search for the
  // prefix of its first entry, then forward; a codeword shorter than lmax
  // covers consecutive entries, so the last match is tried first
  const uint32_t per = (total + kDecTabThreads - 1) / kDecTabThreads;
  const uint32_t i0 = min(total, tid * per), i1 = min(total, i0 + per);
  if (i0 < i1) {
    uint32_t lo = 0, hi = kNP;  // the prefix whose entries hold i0: the last with poff[p] <= i0
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (poff[mid] <= i0) lo = mid;
      else hi = mid;
    }
    uint32_t p = lo;
    uint32_t hit_l = 0, hit_lo = 0, hit_hi = 0, hit_e = 0;  // last match: length, range of c, entry
    for (uint32_t idx = i0; idx < i1; idx++) {
      while (poff[p + 1] <= idx) {
        p++;
        hit_l = 0;
      }
      const uint32_t e = pe[p], lmin = (e >> 8) & 0xFFu, lmax = e >> 16;
      const uint32_t wb = min(lmax - kLutBits, kSubBits), cb = kLutBits + wb;
      const uint32_t c = (p << wb) | (idx - poff[p]);  // the first cb bits
      uint32_t se = 0;
      if (hit_l && c >= hit_lo && c < hit_hi) {
        se = hit_e;
      } else {
        hit_l = 0;
        for (uint32_t l = lmin; l <= cb; l++) {
          const uint32_t cl = c >> (cb - l);
          if (cnt[l] && cl >= first[l] && cl - first[l] < cnt[l]) {
            const uint32_t pos = start[l] + cl - first[l];
            const uint32_t sy = pos < kNP ? (uint32_t)short_sym[pos] : (uint32_t)w.symbols[pos];
            se = (sy << 8) | l;
            hit_l = l;
            hit_lo = cl << (cb - l);
            hit_hi = (cl + 1) << (cb - l);
            hit_e = se;
            break;
          }
        }
        // longer codewords only: the decoder searches lengths cb + 1 .. lmax
        if (!hit_l && lmax > cb) se = kLut2Search | (lmax << 16) | ((cb + 1) << 8);
      }
      w.sub[idx] = se;
    }
  }
}

// Region decoding state kept in a workspace across calls: mode 1 stores the
// stream's header beside the tables and offsets built from it; mode 2, a
// later call that reuses them, first checks that the stream still has that
// header (and the caller's copy, when given): a mismatch sets the error
// flag, so that no decoder reads the tables.
__global__ void __launch_bounds__(64) k_hdr_keep(JobTab t, uint32_t mode) {
  const Job &J = *job_of(t).J;
  const uint32_t *src = (const uint32_t *)J.src;
  __shared__ uint32_t mis;
  if (threadIdx.x == 0) mis = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kHeader / 4; i += blockDim.x) {
    const uint32_t v = src[i];
    if (mode == 1) J.hdr_keep[i] = v;
    else if (v != J.hdr_keep[i] || (J.hdr_expect && v != J.hdr_expect[i])) atomicOr(&mis, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0 && mis) *J.dw.err = 1;
}

// The block table must add up to the header's counts (u64 totals of the scan).
__global__ void __launch_bounds__(64) k_dec_check(JobTab t) {
  const Job &J = *job_of(t).J;
  const uint64_t *tot = J.dw.tot;
  if (threadIdx.x == 0 && (tot[0] != J.h.payload_words || tot[1] != J.h.n_outliers || tot[2] != J.h.n_regression))
    *J.dw.err = 1;
}

}  // namespace sdcsz
