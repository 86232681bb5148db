// kern_fast_dec.hip -- block-shape-specialised decompression: one lane per block.
//
// Algorithm 2 for one block per lane: canonical Huffman decoding through a
// lookup table in LDS (the first kLutBits bits of a codeword; longer codes
// take a short search over the lengths their prefix allows) from a window
// of the block's payload staged in LDS with 16-byte loads, reconstruction
// with the arithmetic of compression (previous reconstructed plane in
// registers), the checksum of the block against sum_dc, and coalesced row
// stores.  A checksum mismatch or an undecodable block queues the block for
// k_decode_wave_redo (kern_wave.hip), which re-executes it from the
// compressed bytes.  The production instantiation leaves the blocks a fault
// plan names; the one that applies the plan's RECON flips to the
// decompressed words (FAULTS) runs them, a lane per block of the plan's list,
// and blocks with more than one flip run in k_decode_wave_list.
#include "dev.h"
#include "kern.h"

namespace sdcsz {

namespace {

__device__ inline uint64_t dmap_block(const Geo &g, const Launch &L, uint32_t mode, uint64_t idx) {
  uint64_t c0, c1, c2;
  if (mode == 0) {
    c2 = idx % L.nf[2];
    uint64_t t = idx / L.nf[2];
    c1 = t % L.nf[1];
    c0 = t / L.nf[1];
  } else if (idx < L.s2) {
    c2 = g.nb[2] - 1;
    c1 = idx % g.nb[1];
    c0 = idx / g.nb[1];
  } else if (idx < L.s2 + L.s1) {
    uint64_t t = idx - L.s2;
    c1 = g.nb[1] - 1;
    c2 = t % L.nf[2];
    c0 = t / L.nf[2];
  } else {
    uint64_t t = idx - L.s2 - L.s1;
    c0 = g.nb[0] - 1;
    c2 = t % L.nf[2];
    c1 = t / L.nf[2];
  }
  return (c0 * g.nb[1] + c1) * g.nb[2] + c2;
}

// Block of a region launch: lane idx walks, in C order, the box of blocks
// the region touches (block coordinates rb.lo .. rb.hi).
__device__ inline uint64_t rmap_block(const Geo &g, const Region &rb, uint64_t idx) {
  const uint64_t e1 = rb.hi[1] - rb.lo[1], e2 = rb.hi[2] - rb.lo[2];
  const uint64_t c2 = rb.lo[2] + idx % e2, t = idx / e2;
  const uint64_t c1 = rb.lo[1] + t % e1, c0 = rb.lo[0] + t / e1;
  return (c0 * g.nb[1] + c1) * g.nb[2] + c2;
}

// The output row of a region that holds field row (z, y), or null when the
// row lies outside the region; a store through it must still check its
// column x against [r.lo[2], r.hi[2]) and write at x - r.lo[2].
template <typename T> __device__ inline T *region_row(T *out, const Region &r, uint64_t z, uint64_t y) {
  if (z < r.lo[0] || z >= r.hi[0] || y < r.lo[1] || y >= r.hi[1]) return nullptr;
  return out + ((z - r.lo[0]) * (r.hi[1] - r.lo[1]) + (y - r.lo[1])) * (r.hi[2] - r.lo[2]);
}

template <typename V> __device__ inline void dpin(V &v) { __asm__ volatile("" : "+v"(v)); }
template <typename... V> __device__ inline void drow_fence(V &...v) {
  (dpin(v), ...);
  __asm__ volatile("" ::: "memory");
}

constexpr uint32_t kDecThreads = 256;
constexpr uint32_t kRing = 16;                 // payload words per lane in LDS
constexpr uint32_t kRingGroups = kRing / 4;    // 16-byte groups of the ring

// The payload bits of one lane's block, read through a ring of kRing words
// in LDS (word r of thread t at win[r * kDecThreads + t], so a wave's
// accesses to one word index fall in distinct banks).  The ring fills with
// the stream's 16-byte groups as decoding reaches them, each group fetched
// once: group k, counted from the group that holds the block's first payload
// bit, sits in slot k % kRingGroups.  stage<N>() makes the ring hold the next
// N codewords of at most kMaxLen bits and the 64 bits a lookup reads past
// them; with the current position's offset inside its group (< 128 bits)
// that is at most kRingGroups groups, the oldest of which it may overwrite
// (none of their words is read again).  The 64 bits from the current word
// on sit in a register pair, refilled with one LDS read per 32 bits consumed.
struct Window {
  const uint8_t *g0;   // the 16-byte group holding the block's first payload bit
  const uint8_t *end;  // end of the readable stream bytes
  uint32_t *win;       // this thread's column of the ring
  uint32_t skew;       // bits from g0 to the block's first payload bit
  uint32_t ap;         // current bit position, from g0
  uint32_t ng;         // groups fetched so far
  uint64_t bb;         // stream bits [32 * (ap >> 5), 32 * (ap >> 5) + 64)
  uint4 pf;            // group ng, fetched ahead

  __device__ inline void init(const uint8_t *pay, const uint8_t *e, uint32_t *w) {
    g0 = pay - ((uintptr_t)pay & 15);
    skew = (uint32_t)(pay - g0) * 8;
    ap = skew;
    ng = 0;
    end = e;
    win = w;
    bb = 0;
  }
  __device__ inline uint32_t word(uint32_t i) const { return win[(i % kRing) * kDecThreads]; }
  __device__ inline uint4 fetch(uint32_t gi) const {
    const uint8_t *ga = g0 + 16ull * gi;
    uint4 v;
    if (__builtin_expect(ga + 16 <= end, 1)) {
      v = *(const uint4 *)ga;
    } else {  // the group reaches past the stream: word by word, zeros beyond
      const uint32_t *gw = (const uint32_t *)ga;
      v.x = ga + 4 <= end ? gw[0] : 0u;
      v.y = ga + 8 <= end ? gw[1] : 0u;
      v.z = ga + 12 <= end ? gw[2] : 0u;
      v.w = 0u;
    }
    return v;
  }
  __device__ inline void put(uint32_t gi, const uint4 &v) {
    uint32_t *d = win + (gi % kRingGroups) * 4 * kDecThreads;
    d[0] = v.x;
    d[kDecThreads] = v.y;
    d[2 * kDecThreads] = v.z;
    d[3 * kDecThreads] = v.w;
  }
  // Every stage after the first holds group ng in registers (pf), fetched
  // one stage earlier so that its latency hides behind that stage's
  // decoding; a stage that needs more than that group waits for the rest.
  template <uint32_t N> __device__ inline void stage() {
    static_assert(((127 + N * kMaxLen + 63) >> 7) + 1 <= kRingGroups, "N codewords fit the ring");
    const uint32_t last = (ap + N * kMaxLen + 63) >> 7;  // last group the next N codewords may touch
    const bool first = ng == 0;
    bool have = !first;
    if (have && ng <= last) {
      put(ng, pf);
      ng++;
      have = false;
    }
#pragma unroll 1
    for (; ng <= last; ng++) put(ng, fetch(ng));
    if (!have) pf = fetch(ng);
    if (first) bb = ((uint64_t)word(ap >> 5) << 32) | word((ap >> 5) + 1);
  }
  // the next 32 bits of the block (most significant first)
  __device__ inline uint32_t peek() const { return (uint32_t)((bb << (ap & 31)) >> 32); }
  // the word that follows bb, read before the codeword's length is known
  // (the read overlaps the table lookup; it is used only when the codeword
  // ends past bb's first word, and then it lies inside the staged groups)
  __device__ inline uint32_t ahead() const { return word((ap >> 5) + 2); }
  __device__ inline void skip(uint32_t n, uint32_t nx) {  // n < 32; nx: ahead() at the codeword's start
    const uint32_t na = ap + n;
    if ((na >> 5) != (ap >> 5)) bb = (bb << 32) | nx;
    ap = na;
  }
  __device__ inline uint32_t pos() const { return ap - skew; }
};

// Canonical decoding tables in LDS: the two-level prefix table (lut2), the
// first kSubLds entries of its second level, and first code, count and first
// position per length for prefixes that keep the search.
constexpr uint32_t kSubLds = 2048;
struct DecLds {
  uint32_t lut[1u << kLutBits];
  uint32_t first[kMaxLen + 2], count[kMaxLen + 2], start[kMaxLen + 2];
  uint32_t sub_lds;  // second-level entries held in sub
  uint32_t sub[kSubLds];
};

// Decode one symbol.  The prefix table resolves codewords of up to kLutBits
// bits; a longer one takes one second-level lookup indexed by the next (at
// most kSubBits) bits (from LDS, or from the global table past kSubLds
// entries, waiting for that load inside its own branch).  Codewords longer
// than the second level resolves, and prefixes without one, search the
// lengths left, the first length whose codes hold the top bits winning.  Sets *bad when no codeword matches.  Reading
// past the block's words is checked once, at the end of the block.
__device__ inline uint32_t decode_sym(Window &br, const DecLds &t, const uint32_t *gsub, const uint16_t *gsym,
                                      bool *bad) {
  const uint32_t v = br.peek();
  const uint32_t nx = br.ahead();
  const uint32_t e = t.lut[v >> (32 - kLutBits)];
  uint32_t len = e & 0xFFu, sym = e >> 8;
  if (__builtin_expect(len == 0, 0)) {
    sym = 0;
    uint32_t f = e;  // a second-level entry, or the lengths to search
    if (e != 0 && !(e & kLut2Search)) {
      const uint32_t wb = (e >> 8) & 0xFu;  // 1..kSubBits
      const uint32_t idx = (e >> 12) + ((v << kLutBits) >> (32 - wb));
      if (idx < t.sub_lds) {
        f = t.sub[idx];
      } else {
        f = gsub[idx];
        __asm__ volatile("" : "+v"(f));
      }
      len = f & 0xFFu;
      sym = f >> 8;
    }
    if (len == 0 && (f & kLut2Search)) {
      const uint32_t lmin = (f >> 8) & 0xFFu, lmax = (f >> 16) & 0xFFu;
#pragma unroll 1
      for (uint32_t l = lmin; l <= lmax; l++) {
        const uint32_t c = v >> (32 - l);
        const uint32_t fc = t.first[l], n = t.count[l];
        if (c >= fc && c - fc < n) {
          uint32_t gs = gsym[t.start[l] + c - fc];
          __asm__ volatile("" : "+v"(gs));
          sym = gs;
          len = l;
          break;
        }
      }
    }
    if (len == 0) {
      *bad = true;
      len = 1;
    }
  }
  br.skip(len, nx);
  return sym;
}

// per-lane routine instantiations
enum { kDProd = 0, kDFaults = 1 };

// A lane's RECON flip (at most one: the host sends blocks with more to the
// generic routine): point index in C order over the block's extents, word
// half, xor mask; the wave flag is uniform.
struct LaneRecon {
  uint32_t p = ~0u, half = 0, m = 0;
  bool wave = false;
};
__device__ inline LaneRecon lane_recon(const PlanDev &plan, uint64_t blk, bool active, uint32_t per) {
  LaneRecon f;
  if (active && plan_hit(plan, blk))
    for (uint32_t t = plan_first(plan, blk); t < plan.n && plan.f[t].block == blk; t++)
      if (plan.f[t].target == SDCSZ_T_RECON) {
        f.p = (uint32_t)(plan.f[t].word / per);
        f.half = (uint32_t)(plan.f[t].word % per);
        f.m = 1u << (plan.f[t].bit & 31);
      }
  f.wave = __ballot(f.p != ~0u) != 0;
  return f;
}

template <typename T> __device__ inline T word_xor(T v, uint32_t half, uint32_t m) {
  uint32_t wv[2] = {0, 0};
  Wd<T>::split(v, wv);
  wv[0] ^= half == 0 ? m : 0u;
  if (Wd<T>::per == 2) wv[1] ^= half == 1 ? m : 0u;
  return Wd<T>::join(wv);
}

// The wave's lowest block origin (every lane takes part).
__device__ inline uint64_t dwave_min(uint64_t org) {
  uint64_t omin = org;
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)omin, off);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(omin >> 32), off);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    omin = o < omin ? o : omin;
  }
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(omin >> 32)) << 32) |
         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)omin);
}

// What a lane's decoding found.
struct DecOut {
  bool bad;      // no codeword matched, the payload overran, or the outliers disagree
  uint64_t sum;  // checksum of the decompressed words
};

}  // namespace

// One lane's block (every lane of the wave calls it; inactive lanes with a
// valid block id).  MODE: kDProd, or kDFaults (the plan's RECON flips).
template <typename T, int ND, int B0, int B1, int B2, bool FULL, bool REG, bool WIDE, int MODE>
__device__ __forceinline__ DecOut decode_lanes(const uint8_t *__restrict__ s, const Header &h, const Geo &g,
                                               const DecWork &w, const PlanDev &plan, T *out, const DecLds &tl,
                                               uint32_t *win, uint64_t blk, bool active, const Region &reg,
                                               T *stg, uint32_t *lof) {
  static_assert(!(REG && FULL), "a region launch takes the masked path");
  const Box bx = box_of(g, blk);
  const uint64_t org = fidx(g, bx, 0, 0, 0);
  const uint64_t org0 = WIDE ? 0 : dwave_min(org);
  // below 2 GiB: a wave-uniform base and 32-bit per-lane offsets; wider
  // fields: a per-lane base at the block's origin (32-bit offsets inside it)
  char *wbase = WIDE ? (char *)(out + org) : (char *)(out + org0);
  const uint32_t loff = WIDE ? 0u : (uint32_t)((org - org0) * sizeof(T));
  // plan blocks: the fault-applying launch over the plan's list, or k_decode_wave_list
  if (MODE == kDProd && active && plan_hit(plan, blk)) active = false;
  const LaneRecon lf = MODE == kDFaults ? lane_recon(plan, blk, active, Wd<T>::per) : LaneRecon{};
  // A wave of full blocks with every lane active stores its rows through
  // LDS (stg: 64 rows of B2 values; lof: the lanes' offsets): B2 passes of 64
  // consecutive values, so that each store instruction covers whole cache
  // lines.  Stored lane by lane, the rows leave partial lines (24 bytes per
  // lane in FP32), which non-temporal stores write out slowly.
  constexpr bool CAN_COOP = FULL && !REG && MODE == kDProd && !WIDE;
  uint32_t soff[CAN_COOP ? B2 : 1];  // byte offset (before the row's) of the value each pass stores
  bool coop = false;
  const uint32_t lane = threadIdx.x & 63;
  if constexpr (CAN_COOP) {
    coop = __ballot(active) == ~0ull;
    if (coop) {
      lof[lane] = loff;
      __asm__ volatile("" ::: "memory");  // the wave's LDS accesses run in order
#pragma unroll
      for (int p = 0; p < B2; p++) {
        const uint32_t f = lane + 64u * (uint32_t)p;
        soff[p] = lof[f / B2] + (f % B2) * (uint32_t)sizeof(T);
      }
    }
  }
  DecOut res{false, 0};
  if (!active) return res;

  const uint32_t n0 = FULL ? B0 : bx.n[0], n1 = FULL ? B1 : bx.n[1], n2 = FULL ? B2 : bx.n[2];
  const uint32_t PSB = (uint32_t)(g.d[1] * g.d[2] * sizeof(T)), RSB = (uint32_t)(g.d[2] * sizeof(T));
  const T q = (T)(2.0 * h.eb_abs);
  const T c0 = (T)(n0 - 1) * (T)0.5, c1 = (T)(n1 - 1) * (T)0.5, c2 = (T)(n2 - 1) * (T)0.5;
  const uint32_t meta = *(const uint32_t *)(s + h.off_table + 8 * blk + 4);
  const bool is_reg = meta & 1u;
  const uint32_t nout = meta >> 1;
  const T *outl = (const T *)(s + h.off_outliers) + w.off_out[blk];
  T beta0 = 0, beta1 = 0, beta2 = 0, mu = 0;
  if (is_reg) {
    const T *cp = (const T *)(s + h.off_coef) + 4ull * w.off_coef[blk];
    beta0 = cp[0];
    beta1 = cp[1];
    beta2 = cp[2];
    mu = cp[3];
  }
  const uint32_t nw = (uint32_t)(w.off_pay[blk + 1] - w.off_pay[blk]);
  Window br;
  br.init(s + h.off_payload + 4ull * w.off_pay[blk], s + h.total, win);
  bool bad = false;
  uint32_t used_out = 0;
  uint64_t sum = 0;

  T Pw[B1][B2];
#pragma unroll
  for (int j = 0; j < B1; j++)
#pragma unroll
    for (int k = 0; k < B2; k++) Pw[j][k] = 0;
  T Bk[B2];
#pragma unroll
  for (int k = 0; k < B2; k++) Bk[k] = beta2 * ((T)k - c2);

#pragma unroll 1
  for (int i = 0; i < B0; i++) {
    if (!FULL && (uint32_t)i >= n0) break;
    const T A0 = beta0 * ((T)i - c0);
    T Sv[B2];
#pragma unroll
    for (int k = 0; k < B2; k++) Sv[k] = 0;
#pragma unroll
    for (int j = 0; j < B1; j++) {
      if (!FULL && (uint32_t)j >= n1) break;
      if (j % 2 == 0) br.stage<2 * B2>();
      T Aj = A0 + beta1 * ((T)j - c1);
      dpin(Aj);
      T rowold[B2], rv[B2];
      T cprev = 0, Up = 0;
      const uint32_t prow = ((uint32_t)i * n1 + (uint32_t)j) * n2;  // point index of the row's start
#pragma unroll
      for (int k = 0; k < B2; k++) {
        const bool v = FULL || (uint32_t)k < n2;
        const uint32_t sym = v ? decode_sym(br, tl, w.sub, w.symbols, &bad) : kRadius;
        const T a = Pw[j][k];
        rowold[k] = a;
        const T b = j > 0 ? Pw[j - 1][k] : (T)0;
        const T d = j > 0 ? Sv[k] : (T)0;
        T lor, U1 = 0;
        if (ND == 2) {
          const T f = (j > 0 && k > 0) ? Pw[j - 1][k - 1] : (T)0;
          lor = (b + cprev) - f;
        } else {
          U1 = (a + b) - d;
          lor = cprev + (U1 - Up);
        }
        const T reg = (Aj + Bk[k]) + mu;
        const T pred = is_reg ? reg : lor;
        T r = pred + (T)((int)sym - (int)kRadius) * q;
        const bool z = v && sym == 0;
        if (__builtin_expect(__ballot(z) != 0, 0)) {
          if (z) {
            if (used_out < nout) {
              T o = outl[used_out];
              dpin(o);  // wait for the load here, not at every later use of r
              r = o;
            } else {
              bad = true;
            }
            used_out++;
          }
        }
        Pw[j][k] = r;
        T rs = r;  // the decompressed word as stored and checked
        if (MODE == kDFaults && lf.wave) {
          if (v && lf.p == prow + k) {
            rs = word_xor(r, lf.half, lf.m);
            count(w.cnt, C_INJ + SDCSZ_T_RECON);
          }
        }
        rv[k] = rs;
        cprev = r;
        Up = U1;
        if (v) sum += Wd<T>::sum(rs);
      }
      if constexpr (REG) {
        // the part of the row inside the region
        T *row = region_row(out, reg, bx.o[0] + (uint64_t)i, bx.o[1] + (uint64_t)j);
        if (row) {
#pragma unroll
          for (int k = 0; k < B2; k++) {
            const uint64_t x = bx.o[2] + (uint64_t)k;
            if ((uint32_t)k < n2 && x >= reg.lo[2] && x < reg.hi[2]) row[x - reg.lo[2]] = rv[k];
          }
        }
      } else {
        // store the row (non-temporal: the output is not read again here, and
        // keeping it out of the caches leaves them to the payload windows)
        bool stored = false;
        if constexpr (CAN_COOP) {
          if (coop) {  // wave-uniform
            __asm__ volatile("" ::: "memory");  // the last row's reads of stg come first
#pragma unroll
            for (int k = 0; k < B2; k++) stg[lane * B2 + k] = rv[k];
            __asm__ volatile("" ::: "memory");
            const uint32_t rowoff = (uint32_t)i * PSB + (uint32_t)j * RSB;
#pragma unroll
            for (int p = 0; p < B2; p++)
              __builtin_nontemporal_store(stg[lane + 64u * (uint32_t)p], gbl((T *)(wbase + (soff[p] + rowoff))));
            stored = true;
          }
        }
        if (!stored) {
          char *dst = wbase + (loff + (uint32_t)i * PSB + (uint32_t)j * RSB);
#pragma unroll
          for (int k = 0; k < B2; k++)
            if (FULL || (uint32_t)k < n2) __builtin_nontemporal_store(rv[k], (T *)(dst + k * sizeof(T)));
        }
      }
#pragma unroll
      for (int k = 0; k < B2; k++) Sv[k] = rowold[k];
      drow_fence(cprev, sum, br.ap, br.bb);
    }
  }
  if (used_out != nout || br.pos() > nw * 32u) bad = true;
  res.bad = bad;
  res.sum = sum;
  const uint64_t *sumdc = (const uint64_t *)(s + h.off_sumdc);
  uint64_t why = 0;
  if (bad) why = 2;
  else if (h.abft && sum != sumdc[blk]) {
    why = 1;
    count(w.cnt, C_DET + SDCSZ_T_RECON);
  }
  if (__builtin_expect(why != 0, 0)) {
    if (MODE == kDFaults) {  // the fault-applying launch: its own queue, re-executed on its stream
      const uint64_t slot = atomicAdd(w.cnt + C_REDO2, 1ull);
      if (slot < kMaxRedo) w.redo[kMaxRedo + slot] = blk | (why << 56);
    } else {
      const uint32_t slot = atomicAdd(w.redo_n, 1u);
      if (slot < kMaxRedo) w.redo[slot] = blk | (why << 56);
    }
  }
  return res;
}

// One lane's 2D block of B1 rows by B2 columns, a row per iteration with the
// previous reconstructed row in registers; the ring is staged every 8
// codewords (every row when B2 is not a multiple of 8).
template <typename T, int B1, int B2, bool FULL, bool REG, bool WIDE, int MODE>
__device__ __forceinline__ DecOut decode_rows(const uint8_t *__restrict__ s, const Header &h, const Geo &g,
                                              const DecWork &w, const PlanDev &plan, T *out, const DecLds &tl,
                                              uint32_t *win, uint64_t blk, bool active, const Region &reg) {
  constexpr uint32_t kRowStage = B2 % 8 == 0 ? 8 : B2;  // codewords per ring stage
  static_assert(!(REG && FULL), "a region launch takes the masked path");
  const Box bx = box_of(g, blk);
  const uint64_t org = fidx(g, bx, 0, 0, 0);
  const uint64_t org0 = WIDE ? 0 : dwave_min(org);
  // below 2 GiB: a wave-uniform base and 32-bit per-lane offsets; wider
  // fields: a per-lane base at the block's origin (32-bit offsets inside it)
  char *wbase = WIDE ? (char *)(out + org) : (char *)(out + org0);
  const uint32_t loff = WIDE ? 0u : (uint32_t)((org - org0) * sizeof(T));
  // plan blocks: the fault-applying launch over the plan's list, or k_decode_wave_list
  if (MODE == kDProd && active && plan_hit(plan, blk)) active = false;
  const LaneRecon lf = MODE == kDFaults ? lane_recon(plan, blk, active, Wd<T>::per) : LaneRecon{};
  DecOut res{false, 0};
  if (!active) return res;

  const uint32_t n0 = bx.n[0], n1 = FULL ? B1 : bx.n[1], n2 = FULL ? B2 : bx.n[2];
  const uint32_t RSB = (uint32_t)(g.d[2] * sizeof(T));
  const T q = (T)(2.0 * h.eb_abs);
  const T c0 = (T)(n0 - 1) * (T)0.5, c1 = (T)(n1 - 1) * (T)0.5, c2 = (T)(n2 - 1) * (T)0.5;
  const uint32_t meta = *(const uint32_t *)(s + h.off_table + 8 * blk + 4);
  const bool is_reg = meta & 1u;
  const uint32_t nout = meta >> 1;
  const T *outl = (const T *)(s + h.off_outliers) + w.off_out[blk];
  T beta0 = 0, beta1 = 0, beta2 = 0, mu = 0;
  if (is_reg) {
    const T *cp = (const T *)(s + h.off_coef) + 4ull * w.off_coef[blk];
    beta0 = cp[0];
    beta1 = cp[1];
    beta2 = cp[2];
    mu = cp[3];
  }
  const uint32_t nw = (uint32_t)(w.off_pay[blk + 1] - w.off_pay[blk]);
  Window br;
  br.init(s + h.off_payload + 4ull * w.off_pay[blk], s + h.total, win);
  bool bad = false;
  uint32_t used_out = 0;
  uint64_t sum = 0;
  const T A0 = beta0 * ((T)0 - c0);
  T Bk[B2], Pr[B2];  // Pr: reconstructed row j - 1
#pragma unroll
  for (int k = 0; k < B2; k++) {
    Bk[k] = beta2 * ((T)k - c2);
    Pr[k] = 0;
  }
#pragma unroll 1
  for (int j = 0; j < B1; j++) {
    if (!FULL && (uint32_t)j >= n1) break;
    T Aj = A0 + beta1 * ((T)j - c1);
    dpin(Aj);
    T cprev = 0, fold = 0;
    T rv[B2];
    const uint32_t prow = (uint32_t)j * n2;  // point index of the row's start
#pragma unroll
    for (int k = 0; k < B2; k++) {
      if (k % kRowStage == 0) br.stage<kRowStage>();
      const bool v = FULL || (uint32_t)k < n2;
      const uint32_t sym = v ? decode_sym(br, tl, w.sub, w.symbols, &bad) : kRadius;
      const T b = Pr[k], f = fold;  // r(j-1,k), r(j-1,k-1)
      fold = b;
      const T lor = (b + cprev) - f;
      const T reg = (Aj + Bk[k]) + mu;
      const T pred = is_reg ? reg : lor;
      T r = pred + (T)((int)sym - (int)kRadius) * q;
      const bool z = v && sym == 0;
      if (__builtin_expect(__ballot(z) != 0, 0)) {
        if (z) {
          if (used_out < nout) {
            T o = outl[used_out];
            dpin(o);  // wait for the load here, not at every later use of r
            r = o;
          } else {
            bad = true;
          }
          used_out++;
        }
      }
      Pr[k] = r;
      T rs = r;  // the decompressed word as stored and checked
      if (MODE == kDFaults && lf.wave) {
        if (v && lf.p == prow + k) {
          rs = word_xor(r, lf.half, lf.m);
          count(w.cnt, C_INJ + SDCSZ_T_RECON);
        }
      }
      rv[k] = rs;
      cprev = r;
      if (v) sum += Wd<T>::sum(rs);
    }
    if constexpr (REG) {
      T *row = region_row(out, reg, bx.o[0], bx.o[1] + (uint64_t)j);
      if (row) {
#pragma unroll
        for (int k = 0; k < B2; k++) {
          const uint64_t x = bx.o[2] + (uint64_t)k;
          if ((uint32_t)k < n2 && x >= reg.lo[2] && x < reg.hi[2]) row[x - reg.lo[2]] = rv[k];
        }
      }
    } else {
      // plain row stores: non-temporal ones (as in 3D) made the decoding of a
      // mixed batch's 2D fields much slower
      char *dst = wbase + (loff + (uint32_t)j * RSB);
#pragma unroll
      for (int k = 0; k < B2; k++)
        if (FULL || (uint32_t)k < n2) *(T *)(dst + k * sizeof(T)) = rv[k];
    }
    drow_fence(sum, br.ap, br.bb);
  }
  if (used_out != nout || br.pos() > nw * 32u) bad = true;
  res.bad = bad;
  res.sum = sum;
  const uint64_t *sumdc = (const uint64_t *)(s + h.off_sumdc);
  uint64_t why = 0;
  if (bad) why = 2;
  else if (h.abft && sum != sumdc[blk]) {
    why = 1;
    count(w.cnt, C_DET + SDCSZ_T_RECON);
  }
  if (__builtin_expect(why != 0, 0)) {
    if (MODE == kDFaults) {  // the fault-applying launch: its own queue, re-executed on its stream
      const uint64_t slot = atomicAdd(w.cnt + C_REDO2, 1ull);
      if (slot < kMaxRedo) w.redo[kMaxRedo + slot] = blk | (why << 56);
    } else {
      const uint32_t slot = atomicAdd(w.redo_n, 1u);
      if (slot < kMaxRedo) w.redo[slot] = blk | (why << 56);
    }
  }
  return res;
}

// The decoding tables in LDS (every thread of the work-group takes part).
__device__ inline void load_tables(DecLds &tl, const DecWork &w) {
  for (uint32_t t = threadIdx.x; t < (1u << kLutBits); t += blockDim.x) tl.lut[t] = w.lut2[t];
  if (threadIdx.x < kMaxLen + 2) {
    tl.first[threadIdx.x] = w.tab->first[threadIdx.x];
    tl.count[threadIdx.x] = w.tab->count[threadIdx.x];
    tl.start[threadIdx.x] = w.tab->start[threadIdx.x];
  }
  const uint32_t n = min(w.tab->sub_n, kSubLds);
  for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) tl.sub[t] = w.sub[t];
  if (threadIdx.x == 0) tl.sub_lds = n;
  __syncthreads();
}

// Work-groups [0, L.full_wgs) take full blocks, the rest the partial shell.
// FAULTS: the instantiation that applies the plan's RECON flips, one lane
// per block of the plan's list (plan.flist) on the masked path.
template <typename T, int ND, int B0, int B1, int B2, bool WIDE, bool FAULTS>
__global__ void __launch_bounds__(kDecThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_decode_fast(JobTab tab) {
  const JobWg jw = job_of(tab);
  const uint8_t *__restrict__ s = jw.J->src;
  const Header h = jw.J->h;
  const Geo g = jw.J->g;
  const DecWork w = jw.J->dw;
  const PlanDev plan = jw.J->plan;
  T *out = (T *)jw.J->dst;
  const Launch L = jw.J->L;
  if (*w.err) return;  // invalid codebook or block table: nothing is read
  __shared__ DecLds tl;
  __shared__ uint32_t win[kRing * kDecThreads];
  // 3D full blocks: each wave's rows on their way out, and its lanes' offsets
  __shared__ T stage[ND == 3 ? B2 * kDecThreads : 1];
  __shared__ uint32_t lofs[ND == 3 ? kDecThreads : 1];
  T *stg = stage + (ND == 3 ? (threadIdx.x >> 6) * 64u * B2 : 0u);
  uint32_t *lof = lofs + (ND == 3 ? (threadIdx.x & ~63u) : 0u);
  load_tables(tl, w);
  constexpr int M = FAULTS ? kDFaults : kDProd;
  const Region &reg = jw.J->reg, &rb = jw.J->rblk;
  if constexpr (FAULTS) {
    __builtin_amdgcn_s_setprio(3);  // a few blocks beside the production launch
    const uint32_t idx = jw.b * blockDim.x + threadIdx.x, nl = plan.nflist;
    const bool act = idx < nl;
    const uint64_t blk = plan.flist[act ? idx : nl - 1];
    if constexpr (ND == 2)
      decode_rows<T, B1, B2, false, false, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act, reg);
    else
      decode_lanes<T, ND, B0, B1, B2, false, false, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act,
                                                             reg, stg, lof);
  } else {
  if (jw.J->mode == 2) {
    // region decompression: one lane per block of the box of blocks the
    // region touches (L.shell_count of them), each storing only its part of
    // the region, at region-relative offsets
    const uint64_t idx = (uint64_t)jw.b * blockDim.x + threadIdx.x;
    const bool act = idx < L.shell_count;
    const uint64_t blk = rmap_block(g, rb, act ? idx : L.shell_count - 1);
    if constexpr (ND == 2)
      decode_rows<T, B1, B2, false, true, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act, reg);
    else
      decode_lanes<T, ND, B0, B1, B2, false, true, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act,
                                                            reg, stg, lof);
    return;
  }
  const bool full = jw.b < L.full_wgs;
  const uint64_t idx = (uint64_t)(full ? jw.b : jw.b - L.full_wgs) * blockDim.x + threadIdx.x;
  const uint64_t nl = full ? L.full_count : L.shell_count;
  const bool act = idx < nl;
  const uint64_t blk = dmap_block(g, L, full ? 0u : 1u, act ? idx : nl - 1);
  if constexpr (ND == 2) {
    static_assert(B0 == 1, "2D blocks have one plane");
    if (full)
      decode_rows<T, B1, B2, true, false, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act, reg);
    else
      decode_rows<T, B1, B2, false, false, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act, reg);
  } else {
    if (full)
      decode_lanes<T, ND, B0, B1, B2, true, false, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act,
                                                            reg, stg, lof);
    else
      decode_lanes<T, ND, B0, B1, B2, false, false, WIDE, M>(s, h, g, w, plan, out, tl, win + threadIdx.x, blk, act,
                                                             reg, stg, lof);
  }
}
}

#define SDCSZ_INST_DEC(T, ND, B0, B1, B2)                                           \
  template __global__ void k_decode_fast<T, ND, B0, B1, B2, false, false>(JobTab); \
  template __global__ void k_decode_fast<T, ND, B0, B1, B2, true, false>(JobTab);  \
  template __global__ void k_decode_fast<T, ND, B0, B1, B2, false, true>(JobTab);
SDCSZ_INST_DEC(float, 3, 6, 6, 6)
SDCSZ_INST_DEC(double, 3, 6, 6, 6)
SDCSZ_INST_DEC(float, 2, 1, 16, 16)
SDCSZ_INST_DEC(double, 2, 1, 16, 16)

}  // namespace sdcsz
