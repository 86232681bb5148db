// kern_util.hip -- range/constant kernels, code check and sizing, scans and
// stream assembly.
#include "dev.h"
#include "kern.h"

namespace sdcsz {

__global__ void k_zero_u64(unsigned long long *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_zero_u32(uint32_t *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// each job's area that must start at zero (counters, results, histogram, ...)
__global__ void __launch_bounds__(256) k_zero_jobs(JobTab t) {
  const JobWg jw = job_of(t);
  const Job &J = *jw.J;
  for (uint64_t i = (uint64_t)jw.b * blockDim.x + threadIdx.x; i < J.zero_words; i += (uint64_t)jw.nb * blockDim.x)
    J.zero[i] = 0;
}

// each job's fault-plan bitmap (cleared by k_zero_jobs): one bit per block
// with entries
__global__ void __launch_bounds__(256) k_plan_bits(JobTab t) {
  const JobWg jw = job_of(t);
  const PlanDev &P = jw.J->plan;
  const uint32_t i = jw.b * blockDim.x + threadIdx.x;
  if (i < P.n) {
    const uint64_t b = P.f[i].block;
    atomicOr((uint32_t *)P.bits + (b >> 5), 1u << (b & 31));
  }
}

// ---- value range of the finite values (value-range relative bound) ----------
template <typename T> __device__ inline void minmax_finite(T v, T &lo, T &hi) {
  const bool f = isfinite(v);
  lo = (f && v < lo) ? v : lo;
  hi = (f && v > hi) ? v : hi;
}

namespace {

// eb_abs and its derived constants, computed in double then rounded once
__device__ void write_consts(uint32_t mode, double eb, double lo, double hi, EbDev *out) {
  double eb_abs = eb;
  if (mode == SDCSZ_REL) eb_abs = lo <= hi ? eb * (hi - lo) : 0.0;
  EbDev e;
  e.eb_abs = eb_abs;
  e.q = 2.0 * eb_abs;
  e.inv = 1.0 / (2.0 * eb_abs);
  e.inv_e = 1.0 / eb_abs;
  e.qf = (float)e.q;
  e.invf = (float)e.inv;
  e.inv_ef = (float)e.inv_e;
  // FP32 rounding of |x - r| has relative error below 2^-24 (exact when the
  // result is subnormal), so a margin of 1e-6 on either side of eb leaves the
  // double comparison the only judge inside the band
  const double dlo = eb_abs * (1.0 - 1e-6), dhi = eb_abs * (1.0 + 1e-6);
  float flo = (float)dlo, fhi = (float)dhi;
  if ((double)flo > dlo) flo = nextafterf(flo, 0.0f);
  if ((double)fhi < dhi) fhi = nextafterf(fhi, INFINITY);
  e.lo = flo;
  e.hi = fhi;
  *out = e;
}

// min and max over the work-group (order-free, so exact)
__device__ void wg_minmax(double &lo, double &hi) {
  __shared__ double slo[kRangeThreads], shi[kRangeThreads];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (uint32_t s = kRangeThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  lo = slo[0];
  hi = shi[0];
  __syncthreads();
}

}  // namespace

// Value range of the finite values (value-range-relative bound): each job
// takes J.nparts work-groups, each writing its partial extremes.
template <typename T> __global__ void __launch_bounds__(kRangeThreads) k_range(JobTab t) {
  const JobWg jw = job_of(t);
  const Job &J = *jw.J;
  const T *in = (const T *)J.src;
  const uint64_t n = J.eb_mode == SDCSZ_REL ? J.g.n_values : 0;
  double *part = (double *)J.cw.range_part;
  T lo = (T)INFINITY, hi = (T)-INFINITY;
  // 16-byte vector loads over the aligned body, scalar loads for the rest
  constexpr uint32_t V = 16 / sizeof(T);
  const uint64_t head = (((uintptr_t)in & 15) ? (16 - ((uintptr_t)in & 15)) / sizeof(T) : 0);
  const uint64_t h = head < n ? head : n;
  const uint64_t nv = (n - h) / V;
  const uint64_t tid = (uint64_t)jw.b * blockDim.x + threadIdx.x, nth = (uint64_t)jw.nb * blockDim.x;
  typedef T vec_t __attribute__((ext_vector_type(V)));
  const vec_t *vin = (const vec_t *)(in + h);
  // non-temporal: the pass streams at close to HBM rate instead of also
  // filling the caches (which saves the compression kernel less than it costs)
  for (uint64_t i = tid; i < nv; i += nth) {
    const vec_t v = __builtin_nontemporal_load(vin + i);
#pragma unroll
    for (uint32_t c = 0; c < V; c++) minmax_finite<T>(v[c], lo, hi);
  }
  for (uint64_t i = tid; i < h; i += nth) minmax_finite<T>(in[i], lo, hi);
  for (uint64_t i = h + nv * V + tid; i < n; i += nth) minmax_finite<T>(in[i], lo, hi);
  double dlo = (double)lo, dhi = (double)hi;
  wg_minmax(dlo, dhi);
  if (threadIdx.x == 0) {
    part[2 * jw.b] = dlo;
    part[2 * jw.b + 1] = dhi;
  }
}
template __global__ void k_range<float>(JobTab);
template __global__ void k_range<double>(JobTab);

// The error-bound constants of each job (one work-group per job) from the
// partial extremes of its range work-groups (none with an absolute bound).
__global__ void __launch_bounds__(kRangeThreads) k_consts(JobTab t) {
  const Job &J = *job_of(t).J;
  const double *part = (const double *)J.cw.range_part;
  const uint32_t np = J.eb_mode == SDCSZ_REL && J.g.n_values ? J.nparts : 0u;
  double dlo = INFINITY, dhi = -INFINITY;
  for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) {
    dlo = fmin(dlo, part[2 * i]);
    dhi = fmax(dhi, part[2 * i + 1]);
  }
  wg_minmax(dlo, dhi);
  if (threadIdx.x == 0) write_consts(J.eb_mode, J.eb, dlo, dhi, J.cw.eb);
}

// ---- codes at rest: fault injection, then detection/correction + sizing ----
__global__ void k_code_faults(PlanDev plan, Geo g, uint16_t *codes, unsigned long long *cnt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (uint32_t t = 0; t < plan.n; t++) {
    const sdcsz_fault f = plan.f[t];
    if (f.target != SDCSZ_T_CODE) continue;
    const Box b = box_of(g, f.block);
    const uint32_t p = (uint32_t)f.word;
    const uint32_t k = p % b.n[2], j = (p / b.n[2]) % b.n[1], i = p / (b.n[2] * b.n[1]);
    codes[code_index(f.block, padded_index(g, i, j, k), g.groups)] ^= (uint16_t)(1u << (f.bit & 15));
    cnt[C_INJ + SDCSZ_T_CODE]++;
  }
}

// One thread per block: verify/correct the block's codes with sum_q/isum_q
// (Algorithm 1, before encoding) and size its Huffman payload in words.
__global__ void __launch_bounds__(256) k_codes_check(JobTab t) {
  const JobWg jw = job_of(t);
  const Geo &g = jw.J->g;
  const CompWork &w = jw.J->cw;
  const uint32_t abft = jw.J->abft;
  const uint64_t blk = (uint64_t)jw.b * blockDim.x + threadIdx.x;
  if (blk >= g.n_blocks) return;
  const Box b = box_of(g, blk);
  uint16_t *codes = w.codes;
  // position in the staging layout of the block's p-th point (C order)
  auto at = [&](uint32_t p) -> uint64_t {
    uint32_t k = p % b.n[2], j = (p / b.n[2]) % b.n[1], i = p / (b.n[2] * b.n[1]);
    return code_index(blk, padded_index(g, i, j, k), g.groups);
  };
  if (abft) {
    uint64_t s2 = 0, i2 = 0;
    for (uint32_t p = 0; p < b.pts; p++) {
      uint32_t c = codes[at(p)];
      s2 += c;
      i2 += (uint64_t)p * c;
    }
    uint64_t j;
    uint32_t v;
    int st = locate_repair(s2, i2, w.sum_q[blk], w.isum_q[blk], b.pts, 16,
                           [&](uint64_t jj) { return (uint32_t)codes[at((uint32_t)jj)]; }, &j, &v);
    if (st != 0) count(w.cnt, C_DET + SDCSZ_T_CODE);
    if (st == 1) {
      codes[at((uint32_t)j)] = (uint16_t)v;
      count(w.cnt, C_COR + SDCSZ_T_CODE);
    }
    if (st < 0) count(w.cnt, C_UNC + SDCSZ_T_CODE);
  }
  uint64_t bits = 0;
  bool missing = false;
  for (uint32_t p = 0; p < b.pts; p++) {
    uint32_t len = w.enc[codes[at(p)]] & 0xFFu;
    missing |= len == 0;
    bits += len;
  }
  if (missing) count(w.cnt, C_MISSING);
  w.words[blk] = (uint32_t)((bits + 31) / 32);
}

// ---- scans of per-block counts ----------------------------------------------
namespace {
struct Tri {
  uint64_t a;
  uint64_t b;
  uint64_t c;
};

// (no words: a scan of the outliers and regression blocks only)
__device__ inline Tri item(const ScanSrc &s, uint64_t i) {
  uint32_t m = s.meta[i * s.stride];
  return Tri{s.words ? s.words[i * s.stride] : 0u, m >> 1, m & 1u};
}

__device__ inline uint64_t wave_inclusive(uint64_t v) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint64_t u = __shfl_up(v, d);
    if (lane >= d) v += u;
  }
  return v;
}

// exclusive scan of one Tri per thread across the work-group (wave scans,
// then the wave totals); returns the exclusive prefix and sets *total.
__device__ Tri block_exclusive(Tri v, Tri *total) {
  constexpr uint32_t kWaves = kScanThreads / 64;
  __shared__ uint64_t wsum[3][kWaves];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const Tri inc{wave_inclusive(v.a), wave_inclusive(v.b), wave_inclusive(v.c)};
  if (lane == 63) {
    wsum[0][wave] = inc.a;
    wsum[1][wave] = inc.b;
    wsum[2][wave] = inc.c;
  }
  __syncthreads();
  Tri pre{0, 0, 0}, all{0, 0, 0};
#pragma unroll
  for (uint32_t q = 0; q < kWaves; q++) {
    const Tri w{wsum[0][q], wsum[1][q], wsum[2][q]};
    if (q < wave) {
      pre.a += w.a;
      pre.b += w.b;
      pre.c += w.c;
    }
    all.a += w.a;
    all.b += w.b;
    all.c += w.c;
  }
  __syncthreads();  // wsum is free for the next call
  *total = all;
  return Tri{pre.a + inc.a - v.a, pre.b + inc.b - v.b, pre.c + inc.c - v.c};
}
}  // namespace

// Exclusive scans of (payload words, outliers, regression flag) per block:
// k_scan1 totals per chunk of scan_chunk(n) blocks; k_scan3 adds up the
// totals of the chunks before its own and writes the offsets, and the 64-bit
// totals after the last block.  k_scan2 gives a job without blocks its zero
// offset and totals (launched only when a call has such a job).
__global__ void __launch_bounds__(kScanThreads) k_scan1(JobTab t) {
  const JobWg jw = job_of(t);
  const ScanSrc src = jw.J->ss;
  const uint64_t n = jw.J->g.n_blocks;
  const uint32_t items = scan_items(n);
  uint64_t *part = jw.J->sc_part;
  const uint32_t bid = jw.b;
  const uint64_t base = (uint64_t)bid * scan_chunk(n) + (uint64_t)threadIdx.x * items;
  Tri s{0, 0, 0};
  for (uint32_t u = 0; u < items; u++)
    if (base + u < n) {
      Tri v = item(src, base + u);
      s.a += v.a;
      s.b += v.b;
      s.c += v.c;
    }
  Tri tot;
  block_exclusive(s, &tot);
  if (threadIdx.x == 0) {
    part[3 * bid] = tot.a;
    part[3 * bid + 1] = tot.b;
    part[3 * bid + 2] = tot.c;
  }
}

// one work-group per job: zero offset and totals of a job without blocks
__global__ void __launch_bounds__(kScanThreads) k_scan2(JobTab t) {
  const Job &J = *job_of(t).J;
  if (J.g.n_blocks == 0 && threadIdx.x == 0) {
    J.sc_off_pay[0] = 0;
    J.sc_off_out[0] = 0;
    J.sc_off_coef[0] = 0;
    J.sc_tot[0] = J.sc_tot[1] = J.sc_tot[2] = 0;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan3(JobTab t) {
  const JobWg jw = job_of(t);
  const Job &J = *jw.J;
  const ScanSrc src = J.ss;
  const uint64_t n = J.g.n_blocks;
  const uint32_t items = scan_items(n);
  const uint64_t *part = J.sc_part;
  uint64_t *off_pay = J.sc_off_pay, *total = J.sc_tot;
  uint32_t *off_out = J.sc_off_out, *off_coef = J.sc_off_coef;
  const uint32_t bid = jw.b;
  // totals of the chunks before this one
  Tri before{0, 0, 0};
  for (uint32_t i = threadIdx.x; i < bid; i += kScanThreads) {
    before.a += part[3 * i];
    before.b += part[3 * i + 1];
    before.c += part[3 * i + 2];
  }
  Tri chunk;
  block_exclusive(before, &chunk);
  const uint64_t base = (uint64_t)bid * scan_chunk(n) + (uint64_t)threadIdx.x * items;
  Tri s{0, 0, 0};
  for (uint32_t u = 0; u < items; u++)
    if (base + u < n) {
      const Tri v = item(src, base + u);
      s.a += v.a;
      s.b += v.b;
      s.c += v.c;
    }
  Tri tot;
  const Tri ex = block_exclusive(s, &tot);
  Tri run{chunk.a + ex.a, chunk.b + ex.b, chunk.c + ex.c};
  for (uint32_t u = 0; u < items && base + u < n; u++) {  // the items again (cache hits)
    off_pay[base + u] = run.a;
    off_out[base + u] = (uint32_t)run.b;
    off_coef[base + u] = (uint32_t)run.c;
    const Tri v = item(src, base + u);
    run.a += v.a;
    run.b += v.b;
    run.c += v.c;
    if (base + u + 1 == n) {
      off_pay[n] = run.a;
      off_out[n] = (uint32_t)run.b;
      off_coef[n] = (uint32_t)run.c;
      total[0] = run.a;  // 64-bit totals: a table whose counts wrap 32 bits cannot match a header
      total[1] = run.b;
      total[2] = run.c;
    }
  }
}

// ---- stream assembly: one thread per block ----------------------------------
template <typename T> __global__ void __launch_bounds__(256) k_encode(JobTab t) {
  const JobWg jw = job_of(t);
  const Geo &g = jw.J->g;
  const CompWork &w = jw.J->cw;
  uint8_t *out = jw.J->dst;
  if (!w.res[R_WRITTEN]) return;  // the stream is not written (see k_header)
  const Header h = *w.hdr;
  const uint64_t blk = (uint64_t)jw.b * blockDim.x + threadIdx.x;
  if (blk >= g.n_blocks) return;
  const Box b = box_of(g, blk);
  uint32_t *dst = (uint32_t *)(out + h.off_payload) + w.off_pay[blk];
  uint64_t acc = 0;
  uint32_t nacc = 0;
  for (uint32_t i = 0; i < b.n[0]; i++)
    for (uint32_t j = 0; j < b.n[1]; j++)
      for (uint32_t k = 0; k < b.n[2]; k++) {
    uint32_t e = w.enc[w.codes[code_index(blk, padded_index(g, i, j, k), g.groups)]];
    uint32_t len = e & 0xFFu;
    acc = (acc << len) | (e >> 8);
    nacc += len;
    if (nacc >= 32) {
      nacc -= 32;
      *dst++ = (uint32_t)(acc >> nacc);
      acc &= (1ull << nacc) - 1;
    }
      }
  if (nacc > 0) *dst++ = (uint32_t)(acc << (32 - nacc));
  const uint32_t meta = w.meta[blk];
  uint32_t *tab = (uint32_t *)(out + h.off_table) + 2 * blk;
  tab[0] = w.words[blk];
  tab[1] = meta;
  const T *src = (const T *)w.vals + blk * (uint64_t)g.bpts;
  T *od = (T *)(out + h.off_outliers) + w.off_out[blk];
  for (uint32_t t = 0; t < (meta >> 1); t++) od[t] = src[t];
  if (meta & 1u) {
    const T *cf = (const T *)w.coef + 4 * blk;
    T *cd = (T *)(out + h.off_coef) + 4ull * w.off_coef[blk];
    for (int a = 0; a < 4; a++) cd[a] = cf[a];
  }
  if (h.abft) ((uint64_t *)(out + h.off_sumdc))[blk] = w.sum_dc[blk];
}
template __global__ void k_encode<float>(JobTab);
template __global__ void k_encode<double>(JobTab);

}  // namespace sdcsz
