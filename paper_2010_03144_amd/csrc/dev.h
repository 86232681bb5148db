// dev.h -- device helpers: value words, block boxes, fault-plan lookup.
#pragma once

#include "common.h"

namespace sdcsz {

// ---- global-memory views of device pointers -------------------------------
// A pointer read out of a job table has no known address space, so accesses
// through it compile to flat instructions, and a flat access counts on the
// LDS counter too: the wait for the next LDS result then also waits for it
// (a prefetch, a store).  Accesses through these views are global ones.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline gptr<T> gbl(T *p) { return (gptr<T>)p; }
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));  // 16- and 8-byte accesses without a class copy
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));

// ---- words of a value (integer reinterpretation, Sec. 5.4) ---------------
template <typename T> struct Wd;
template <> struct Wd<float> {
  static constexpr uint32_t per = 1;
  __device__ static inline void split(float v, uint32_t *w) { w[0] = __float_as_uint(v); }
  __device__ static inline float join(const uint32_t *w) { return __uint_as_float(w[0]); }
  __device__ static inline uint32_t sum(float v) { return __float_as_uint(v); }
  __device__ static inline bool same(float a, float b) { return __float_as_uint(a) == __float_as_uint(b); }
  // non-zero iff the bit patterns differ
  __device__ static inline uint32_t diff(float a, float b) { return __float_as_uint(a) ^ __float_as_uint(b); }
  __device__ static inline float flip(float v, uint32_t bit) {
    return __uint_as_float(__float_as_uint(v) ^ (1u << (bit & 31)));
  }
};
template <> struct Wd<double> {
  static constexpr uint32_t per = 2;
  __device__ static inline void split(double v, uint32_t *w) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    w[0] = (uint32_t)u;
    w[1] = (uint32_t)(u >> 32);
  }
  __device__ static inline double join(const uint32_t *w) {
    return __longlong_as_double((long long)((uint64_t)w[0] | ((uint64_t)w[1] << 32)));
  }
  // sum of the two words, widened
  __device__ static inline uint64_t sum(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u & 0xFFFFFFFFull) + (u >> 32);
  }
  __device__ static inline uint32_t diff(double a, double b) {
    uint64_t x = (uint64_t)__double_as_longlong(a) ^ (uint64_t)__double_as_longlong(b);
    return (uint32_t)x | (uint32_t)(x >> 32);
  }
  __device__ static inline bool same(double a, double b) {
    return __double_as_longlong(a) == __double_as_longlong(b);
  }
  __device__ static inline double flip(double v, uint32_t bit) {
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)(1ull << (bit & 63)));
  }
};

template <typename T> struct EbSel;
template <> struct EbSel<float> {
  __device__ static inline float q(const EbDev &e) { return e.qf; }
  __device__ static inline float inv(const EbDev &e) { return e.invf; }
  __device__ static inline float inv_e(const EbDev &e) { return e.inv_ef; }
};
template <> struct EbSel<double> {
  __device__ static inline double q(const EbDev &e) { return e.q; }
  __device__ static inline double inv(const EbDev &e) { return e.inv; }
  __device__ static inline double inv_e(const EbDev &e) { return e.inv_e; }
};

// ---- block box ------------------------------------------------------------
struct Box {
  uint64_t o[3];
  uint32_t n[3];
  uint32_t pts;
  uint32_t pat;  // partial pattern: bit (2 - a) ... see pattern()
};

__device__ inline Box box_of(const Geo &g, uint64_t blk) {
  Box b;
  uint64_t t = blk;
  uint32_t c2 = (uint32_t)(t % g.nb[2]);
  t /= g.nb[2];
  uint32_t c1 = (uint32_t)(t % g.nb[1]);
  uint32_t c0 = (uint32_t)(t / g.nb[1]);
  uint32_t c[3] = {c0, c1, c2};
  b.pat = 0;
  for (int a = 0; a < 3; a++) {
    b.o[a] = (uint64_t)c[a] * g.b[a];
    bool last = c[a] + 1 == g.nb[a];
    b.n[a] = last ? g.rem[a] : g.b[a];
    if (b.n[a] != g.b[a]) b.pat |= 1u << a;
  }
  b.pts = b.n[0] * b.n[1] * b.n[2];
  return b;
}

__device__ inline uint64_t fidx(const Geo &g, const Box &b, uint32_t i, uint32_t j, uint32_t k) {
  return ((b.o[0] + i) * g.d[1] + (b.o[1] + j)) * g.d[2] + (b.o[2] + k);
}

// ---- fault plan -----------------------------------------------------------
__device__ inline bool plan_hit(const PlanDev &P, uint64_t blk) {
  return P.n != 0 && ((P.bits[blk >> 5] >> (blk & 31)) & 1u);
}

// index of the first plan entry of block blk (entries sorted by block)
__device__ inline uint32_t plan_first(const PlanDev &P, uint64_t blk) {
  uint32_t lo = 0, hi = P.n;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (P.f[mid].block < blk) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---- checksum repair (Sec. 3.2) -----------------------------------------
// Given the recomputed sums (s2, i2) and the stored ones, locate the single
// corrupted word and return its repaired value.  Returns 0 clean, 1 repaired
// (*j, *val set), -1 uncorrectable.  `word_of(j)` reads the current word j.
template <typename F>
__device__ inline int locate_repair(uint64_t s2, uint64_t i2, uint64_t s, uint64_t is,
                                    uint64_t n, uint32_t width, F word_of, uint64_t *jout,
                                    uint32_t *val) {
  if (s2 == s && i2 == is) return 0;
  int64_t ds = (int64_t)(s2 - s);
  int64_t di = (int64_t)(i2 - is);
  if (ds == 0) return -1;
  if (di % ds != 0) return -1;
  int64_t j = di / ds;
  if (j < 0 || (uint64_t)j >= n) return -1;
  int64_t rep = (int64_t)word_of((uint64_t)j) - ds;
  int64_t top = width == 16 ? 0xFFFF : 0xFFFFFFFFll;
  if (rep < 0 || rep > top) return -1;
  *jout = (uint64_t)j;
  *val = (uint32_t)rep;
  return 1;
}

// ---- code staging layout --------------------------------------------------
// Codes of 64 consecutive blocks are interleaved in groups of 4: the 4 codes
// q..q+3 (q a multiple of 4, q the point's index in the block padded to the
// configured block shape) of block blk sit in one 8-byte vector, and the 64
// blocks of a tile store their vectors for group q/4 contiguously (512 B).
__device__ inline uint64_t code_index(uint64_t blk, uint32_t q, uint32_t groups) {
  return (((blk >> 6) * groups + (q >> 2)) * 64 + (blk & 63)) * 4 + (q & 3);
}
__device__ inline uint32_t padded_index(const Geo &g, uint32_t i, uint32_t j, uint32_t k) {
  return (i * g.b[1] + j) * g.b[2] + k;
}

// A block's slot of the generic kernels' recon scratch, interleaved across
// 64 consecutive blocks: point p of block blk sits at
// ((blk / 64) * bpts + p) * 64 + blk % 64, so the lanes of a wave (one block
// each) touch consecutive values.  The area holds bpts values for every
// block of the block count rounded up to 64.
template <typename T> struct Slot {
  T *p;
  __device__ T &operator[](uint32_t i) const { return p[(uint64_t)i * 64]; }
};
template <typename T> __device__ inline Slot<T> slot_of(void *base, uint64_t blk, uint32_t bpts) {
  return Slot<T>{(T *)base + (blk >> 6) * (uint64_t)bpts * 64 + (blk & 63)};
}

__device__ inline void count(unsigned long long *cnt, int slot, unsigned long long v = 1) {
  atomicAdd(cnt + slot, v);
}

}  // namespace sdcsz
