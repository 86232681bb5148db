// kern_fast_enc.hip -- block-shape-specialised code check and Huffman encoding.
//
// One lane per block over consecutive block ids, so the interleaved code
// staging layout gives fully coalesced 8-byte-per-lane reads.  The codeword
// table is held in LDS for the codes around the zero residual (where almost
// all codes fall) and read from global memory outside that window.
#include "dev.h"
#include "kern.h"

namespace sdcsz {

namespace {

// Codeword entries of the codes around the zero residual held in LDS: 3584
// (14 KiB) leaves k_checkenc_fast 30 KiB of LDS per work-group, five
// work-groups per CU (4096 entries allowed four; fewer entries send more
// codes to the global table at small bounds)
constexpr uint32_t kEncWin = 3584;
constexpr uint32_t kEncLo = kRadius - kEncWin / 2;

// Codeword table entry of a code: from the LDS window, or (rarely) from the
// global table, waiting for that load inside its own branch.
__device__ inline uint32_t enc_of(uint32_t code, const uint32_t *encw, const uint32_t *enc) {
  const uint32_t c = code - kEncLo;
  uint32_t e = encw[c < kEncWin ? c : 0u];
  if (__builtin_expect(c >= kEncWin, 0)) {
    uint32_t f = gbl(enc)[code];
    __asm__ volatile("" : "+v"(f));
    e = f;
  }
  return e;
}

// Code length of a code: from a byte table in LDS for the codes around the
// zero residual (the check only needs lengths; nearby codes share LDS words,
// so a wave's lookups mostly broadcast instead of meeting bank conflicts),
// else from the global table inside its own branch.
constexpr uint32_t kLenWin = 4096;
constexpr uint32_t kLenLo = kRadius - kLenWin / 2;
__device__ inline uint32_t len_of(uint32_t code, const uint8_t *lenw, const uint32_t *enc) {
  const uint32_t c = code - kLenLo;
  uint32_t l = lenw[c < kLenWin ? c : 0u];
  if (__builtin_expect(c >= kLenWin, 0)) {
    uint32_t f = enc[code] & 0xFFu;
    __asm__ volatile("" : "+v"(f));
    l = f;
  }
  return l;
}

__device__ inline void load_lengths(uint8_t *lenw, const uint32_t *enc) {
  for (uint32_t t = threadIdx.x; t < kLenWin / 4; t += blockDim.x) {
    const uint32_t *e = enc + kLenLo + 4 * t;
    ((uint32_t *)lenw)[t] = (e[0] & 0xFFu) | (e[1] & 0xFFu) << 8 | (e[2] & 0xFFu) << 16 | (e[3] & 0xFFu) << 24;
  }
  __syncthreads();
}

__device__ inline void load_window(uint32_t *encw, const uint32_t *enc) {
  for (uint32_t t = threadIdx.x; t < kEncWin; t += blockDim.x) encw[t] = enc[kEncLo + t];
  __syncthreads();
}

// The codes of one lane's block, one plane at a time: plane i sits in
// buffer i & 1 while plane i + 1 loads into the other (8 bytes per lane per
// access, coalesced across the wave in the interleaved staging layout).
template <int B0, int B1, int B2, bool LAST = true> struct PlaneCodes {
  static constexpr int PG = B1 * B2 / 4;  // 4-code groups per plane
  static_assert((B1 * B2) % 4 == 0, "a plane fills whole groups");
  const uint2 *cb;
  uint32_t v[2][2 * PG];  // two codes per word
  __device__ void init(const uint16_t *codes, uint64_t blk, uint32_t groups) {
    cb = (const uint2 *)(codes + code_index(blk, 0, groups));
  }
  __device__ void load(int i) {
#pragma unroll
    for (int gi = 0; gi < PG; gi++) {
      // the last read of the codes is non-temporal, so they do not displace
      // the output in the caches; an earlier one keeps them there
      const gptr<const uint64_t> a = gbl((const uint64_t *)(cb + (uint64_t)(i * PG + gi) * 64));
      const uint64_t u64 = LAST ? __builtin_nontemporal_load(a) : *a;
      const uint2 u = make_uint2((uint32_t)u64, (uint32_t)(u64 >> 32));
      v[i & 1][2 * gi] = u.x;
      v[i & 1][2 * gi + 1] = u.y;
    }
  }
  // code q (= j * B2 + k) of plane i
  __device__ uint32_t at(int i, int q) const { return (v[i & 1][q >> 1] >> (16 * (q & 1))) & 0xFFFFu; }
};

}  // namespace

// The codes of a block are walked in units of whole 4-code groups: planes of
// a 3D block (U0 planes of U1 x U2 codes), rows of a 2D block (U0 = B1 rows
// of one row of B2 codes).  Ext gives a block's actual extents in that view.
template <int ND, int B0, int B1, int B2> struct Units {
  static constexpr int U0 = ND == 2 ? B1 : B0, U1 = ND == 2 ? 1 : B1, U2 = B2;
  __device__ static void ext(const Box &b, uint32_t &e0, uint32_t &e1, uint32_t &e2) {
    e0 = ND == 2 ? b.n[1] : b.n[0];
    e1 = ND == 2 ? 1u : b.n[1];
    e2 = b.n[2];
  }
};

// Verify/correct the codes of each block with sum_q/isum_q (Algorithm 1,
// before encoding) and size its payload in 32-bit words.
template <int ND, int B0, int B1, int B2> __global__ void __launch_bounds__(256) k_check_fast(JobTab jt) {
  using U = Units<ND, B0, B1, B2>;
  const JobWg jw = job_of(jt);
  const Geo g = jw.J->g;
  const CompWork w = jw.J->cw;
  const uint32_t abft = jw.J->abft;
  __shared__ __align__(16) uint8_t lenw[kLenWin];
  load_lengths(lenw, w.enc);
  const uint64_t blk = (uint64_t)jw.b * blockDim.x + threadIdx.x;
  if (blk >= g.n_blocks) return;
  const Box b = box_of(g, blk);
  uint32_t e0, n1, n2;
  U::ext(b, e0, n1, n2);
  // units in a rolled loop (one unit of code groups live, the next in flight)
  const uint2 *cb = (const uint2 *)(w.codes + code_index(blk, 0, g.groups));
  constexpr int PG = U::U1 * U::U2 / 4;
  static_assert((U::U1 * U::U2) % 4 == 0, "a unit fills whole groups");
  uint2 cur[PG], nxt[PG];
#pragma unroll
  for (int t = 0; t < PG; t++) cur[t] = cb[(uint64_t)t * 64];
  uint64_t s = 0, is = 0, bits = 0;
  uint32_t missing = 0;  // codes without a codeword
#pragma unroll 1
  for (int i = 0; i < U::U0; i++) {
    if (i + 1 < U::U0) {
#pragma unroll
      for (int t = 0; t < PG; t++) nxt[t] = cb[(uint64_t)((i + 1) * PG + t) * 64];
    }
#pragma unroll
    for (int j = 0; j < U::U1; j++) {
      const uint32_t rowbase = ((uint32_t)i * n1 + (uint32_t)j) * n2;
      uint32_t rs = 0, rk = 0;
#pragma unroll
      for (int k = 0; k < U::U2; k++) {
        const int q = j * U::U2 + k;
        const uint32_t word = (q & 2) ? cur[q >> 2].y : cur[q >> 2].x;
        const bool v = (uint32_t)i < e0 && (uint32_t)j < n1 && (uint32_t)k < n2;
        const uint32_t c = v ? ((word >> (16 * (q & 1))) & 0xFFFFu) : 0u;
        const uint32_t len = len_of(c, lenw, w.enc);
        if (v) {
          rs += c;
          rk += (uint32_t)k * c;
          bits += len;
          missing += len == 0 ? 1u : 0u;
        }
      }
      s += rs;
      is += (uint64_t)rowbase * rs + rk;
    }
#pragma unroll
    for (int t = 0; t < PG; t++) cur[t] = nxt[t];
  }
  if (abft && (s != w.sum_q[blk] || is != w.isum_q[blk])) {
    // detected: locate and repair one code, then size the block again
    auto pos = [&](uint64_t p) -> uint64_t {  // in the geometry's own axes
      const uint32_t m1 = b.n[1], m2 = b.n[2];
      const uint32_t k = (uint32_t)(p % m2), j = (uint32_t)((p / m2) % m1), i = (uint32_t)(p / ((uint64_t)m2 * m1));
      return code_index(blk, padded_index(g, i, j, k), g.groups);
    };
    uint64_t jf;
    uint32_t vf;
    const int st = locate_repair(s, is, w.sum_q[blk], w.isum_q[blk], b.pts, 16,
                                 [&](uint64_t jj) { return (uint32_t)w.codes[pos(jj)]; }, &jf, &vf);
    count(w.cnt, C_DET + SDCSZ_T_CODE);
    if (st == 1) {
      // one code changed: the block's size changes by its lengths' difference
      const uint32_t l_old = len_of(w.codes[pos(jf)], lenw, w.enc), l_new = len_of(vf, lenw, w.enc);
      w.codes[pos(jf)] = (uint16_t)vf;
      count(w.cnt, C_COR + SDCSZ_T_CODE);
      bits = bits - l_old + l_new;
      missing = missing - (l_old == 0 ? 1u : 0u) + (l_new == 0 ? 1u : 0u);
    } else {
      count(w.cnt, C_UNC + SDCSZ_T_CODE);
    }
  }
  if (missing) count(w.cnt, C_MISSING);
  w.words[blk] = (uint32_t)((bits + 31) / 32);
}

// Per-block Huffman encoding (MSB first into 32-bit words) and the block's
// table entry, coefficients, sum_dc and outliers at their scanned offsets.
// Finished words go to a per-lane ring of 16 words in LDS; at the end of
// each row the lane writes out what is complete, whole aligned 32-byte
// chunks as two 16-byte stores, so HBM sees full sectors instead of one
// partial write per word (only a block's first and last chunk are partial).
template <typename T, int ND, int B0, int B1, int B2> __global__ void __launch_bounds__(256) k_encode_fast(JobTab jt) {
  using U = Units<ND, B0, B1, B2>;
  const JobWg jw = job_of(jt);
  const Geo g = jw.J->g;
  const CompWork w = jw.J->cw;
  uint8_t *out = jw.J->dst;
  if (!w.res[R_WRITTEN]) return;  // the stream is not written (see k_header)
  const Header h = *w.hdr;
  __shared__ uint32_t encw[kEncWin];
  __shared__ uint32_t ring_all[16 * 256];
  load_window(encw, w.enc);
  const uint64_t blk = (uint64_t)jw.b * blockDim.x + threadIdx.x;
  if (blk >= g.n_blocks) return;
  const Box b = box_of(g, blk);
  uint32_t e0, e1, e2;
  U::ext(b, e0, e1, e2);
  PlaneCodes<U::U0, U::U1, U::U2> bc;
  bc.init(w.codes, blk, g.groups);
  bc.load(0);
  uint32_t *ring = ring_all + threadIdx.x;  // word with absolute index a at ring[(a & 15) * 256]
  const gptr<uint32_t> pay = gbl((uint32_t *)(out + h.off_payload));
  uint64_t wabs = w.off_pay[blk];  // absolute index of the next word produced
  uint64_t fl = wabs;              // first word not yet written out
  auto flush = [&]() {
    if (fl & 7) {  // block head: single words up to the first chunk boundary
      const uint64_t hb = (fl + 7) & ~7ull;
      if (wabs >= hb)
        for (; fl < hb; fl++) pay[fl] = ring[(fl & 15) * 256];
    }
    if (!(fl & 7) && fl + 8 <= wabs) {
      const uint32_t s0 = (uint32_t)(fl & 8);
      uint4 u0, u1;
      u0.x = ring[(s0 + 0) * 256];
      u0.y = ring[(s0 + 1) * 256];
      u0.z = ring[(s0 + 2) * 256];
      u0.w = ring[(s0 + 3) * 256];
      u1.x = ring[(s0 + 4) * 256];
      u1.y = ring[(s0 + 5) * 256];
      u1.z = ring[(s0 + 6) * 256];
      u1.w = ring[(s0 + 7) * 256];
      const gptr<v4u32> d = (gptr<v4u32>)(pay + fl);
      d[0] = v4u32{u0.x, u0.y, u0.z, u0.w};
      d[1] = v4u32{u1.x, u1.y, u1.z, u1.w};
      fl += 8;
    }
  };
  uint64_t acc = 0;
  uint32_t nacc = 0;
  // at most 8 codes (<= 6 words) between flushes: with <= 7 words left
  // after a flush, the 16-word ring never overruns
  constexpr int FE = U::U2 < 8 ? U::U2 : 8;
#pragma unroll
  for (int i = 0; i < U::U0; i++) {
    if (i + 1 < U::U0) bc.load(i + 1);
#pragma unroll
    for (int j = 0; j < U::U1; j++) {
#pragma unroll
      for (int k = 0; k < U::U2; k++) {
        const bool v = (uint32_t)i < e0 && (uint32_t)j < e1 && (uint32_t)k < e2;
        const uint32_t e = enc_of(v ? bc.at(i, j * U::U2 + k) : kRadius, encw, w.enc);
        const uint32_t len = v ? (e & 0xFFu) : 0u;
        acc = (acc << len) | (e >> 8 & ((1u << len) - 1u));
        nacc += len;
        if (nacc >= 32) {
          nacc -= 32;
          ring[(wabs & 15) * 256] = (uint32_t)(acc >> nacc);
          wabs++;
          acc &= (1ull << nacc) - 1;
        }
        if ((k + 1) % FE == 0 || k + 1 == U::U2) flush();
      }
    }
  }
  if (nacc > 0) {
    ring[(wabs & 15) * 256] = (uint32_t)(acc << (32 - nacc));
    wabs++;
  }
  flush();
  for (; fl < wabs; fl++) pay[fl] = ring[(fl & 15) * 256];  // block tail
  const uint32_t meta = w.meta[blk];
  uint32_t *tab = (uint32_t *)(out + h.off_table) + 2 * blk;
  tab[0] = w.words[blk];
  tab[1] = meta;
  if (__builtin_expect((meta >> 1) != 0, 0)) {
    const T *src = (const T *)w.vals + blk * (uint64_t)g.bpts;
    T *od = (T *)(out + h.off_outliers) + w.off_out[blk];
    for (uint32_t t = 0; t < (meta >> 1); t++) od[t] = src[t];
  }
  if (meta & 1u) {
    const T *cf = (const T *)w.coef + 4 * blk;
    T *cd = (T *)(out + h.off_coef) + 4ull * w.off_coef[blk];
    for (int a = 0; a < 4; a++) cd[a] = cf[a];
  }
  if (h.abft) ((uint64_t *)(out + h.off_sumdc))[blk] = w.sum_dc[blk];
}

// Code check and encoding in one kernel (Algorithm 1 before and at the
// encoding) for 3D blocks, one lane per block: a lane checks its block's
// codes a plane at a time (sums and codeword lengths), takes its payload
// offset, then reads the codes again, now mostly from the caches, and encodes
// them.  The offsets come from a scan across work-groups with a
// decoupled look-back: a work-group takes the next tile of 256 blocks of its
// field from a ticket counter (so every tile it waits for belongs to a
// work-group already running), publishes its tile's payload words, and adds
// the published counts of the tiles before it until it meets a published
// prefix, which it then extends.  The outlier and coefficient offsets and
// their totals were scanned before (they depend on the prediction pass
// only); the last tile leaves the field's payload total for k_header.  The
// payload, table, coefficients, sum_dc and outliers are written before the
// call knows whether another block ends uncorrectable (the caller is told
// by the return code; the host takes this path only when the output holds
// the largest stream).
constexpr uint32_t kTileSpin = 1u << 24;  // polls of an unpublished tile before giving up

template <typename T, int B0, int B1, int B2>
__global__ void __launch_bounds__(256) k_checkenc_fast(JobTab jt) {
  static_assert((B1 * B2) % 4 == 0, "a plane fills whole groups");
  const JobWg jw = job_of(jt);
  const Geo g = jw.J->g;
  const CompWork w = jw.J->cw;
  const uint32_t abft = jw.J->abft;
  uint8_t *out = jw.J->dst;
  __shared__ uint32_t encw[kEncWin];
  __shared__ uint32_t ring_all[16 * 256];
  __shared__ uint32_t s_tile, s_wsum[4];
  __shared__ uint64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(w.ticket, 1u);
  load_window(encw, w.enc);  // synchronises the work-group
  const uint32_t tile = s_tile;
  // tickets past the field's tiles would mean a counter not cleared for this
  // call: touch nothing then (the tile states hold one word per tile)
  if ((uint64_t)tile * 256 >= g.n_blocks) return;
  const uint64_t blk = (uint64_t)tile * 256 + threadIdx.x;
  const bool active = blk < g.n_blocks;
  // section offsets of the stream (the payload offset does not depend on the payload's size)
  Header h = jw.J->h;
  h.payload_words = 0;
  h.n_outliers = w.tot[1];
  h.n_regression = w.tot[2];
  section_offsets(h);

  // ---- check: the codes into registers, sums, sizes, repair ----------------
  uint64_t bits = 0;
  uint32_t e0 = 0, n1 = 0, n2 = 0;
  Box b;
  if (active) {
    b = box_of(g, blk);
    e0 = b.n[0];
    n1 = b.n[1];
    n2 = b.n[2];
    // one plane of codes in registers, the next in flight (kept in the
    // caches for the encoding's second read)
    PlaneCodes<B0, B1, B2, false> pc;
    pc.init(w.codes, blk, g.groups);
    pc.load(0);
    uint64_t s = 0, is = 0;
    uint32_t missing = 0;
#pragma unroll
    for (int i = 0; i < B0; i++) {
      if (i + 1 < B0) pc.load(i + 1);
#pragma unroll
      for (int j = 0; j < B1; j++) {
        const uint32_t rowbase = ((uint32_t)i * n1 + (uint32_t)j) * n2;
        uint32_t rs = 0, rk = 0;
#pragma unroll
        for (int k = 0; k < B2; k++) {
          const int q = j * B2 + k;
          const bool v = (uint32_t)i < e0 && (uint32_t)j < n1 && (uint32_t)k < n2;
          const uint32_t c = v ? pc.at(i, q) : kRadius;
          const uint32_t len = enc_of(c, encw, w.enc) & 0xFFu;
          if (v) {
            rs += c;
            rk += (uint32_t)k * c;
            bits += len;
            missing += len == 0 ? 1u : 0u;
          }
        }
        s += rs;
        is += (uint64_t)rowbase * rs + rk;
      }
      // one plane's lookups at a time (the compiler would otherwise hold
      // the whole block's table entries at once)
      __asm__ volatile("" : "+v"(bits), "+v"(s), "+v"(is), "+v"(missing)::"memory");
    }
    if (abft && (s != w.sum_q[blk] || is != w.isum_q[blk])) {
      // detected: locate and repair one code (the encoding reads it back)
      // and size the block again
      auto pos = [&](uint64_t p) -> uint64_t {
        const uint32_t m1 = b.n[1], m2 = b.n[2];
        const uint32_t k = (uint32_t)(p % m2), j = (uint32_t)((p / m2) % m1), i = (uint32_t)(p / ((uint64_t)m2 * m1));
        return code_index(blk, padded_index(g, i, j, k), g.groups);
      };
      uint64_t jf;
      uint32_t vf;
      const int st = locate_repair(s, is, w.sum_q[blk], w.isum_q[blk], b.pts, 16,
                                   [&](uint64_t jj) { return (uint32_t)w.codes[pos(jj)]; }, &jf, &vf);
      count(w.cnt, C_DET + SDCSZ_T_CODE);
      if (st == 1) {
        const uint32_t l_old = enc_of(w.codes[pos(jf)], encw, w.enc) & 0xFFu;
        const uint32_t l_new = enc_of(vf, encw, w.enc) & 0xFFu;
        w.codes[pos(jf)] = (uint16_t)vf;
        count(w.cnt, C_COR + SDCSZ_T_CODE);
        bits = bits - l_old + l_new;
        missing = missing - (l_old == 0 ? 1u : 0u) + (l_new == 0 ? 1u : 0u);
      } else {
        count(w.cnt, C_UNC + SDCSZ_T_CODE);
      }
    }
    if (missing) count(w.cnt, C_MISSING);
  }
  const uint32_t words = active ? (uint32_t)((bits + 31) / 32) : 0u;

  // ---- offsets: scan inside the tile, look-back across tiles ---------------
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = words;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)incl, d);
    if (lane >= d) incl += u;
  }
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, agg = 0;
#pragma unroll
  for (uint32_t q = 0; q < 4; q++) {
    before += q < wave ? s_wsum[q] : 0u;
    agg += s_wsum[q];
  }
  // A tile's state is one 64-bit word (count << 2 | flag), written and read
  // with relaxed device-scope atomics: nothing else is ordered by it, and
  // release/acquire at that scope would write back and invalidate the L2 of
  // the work-group's XCD at every step.
  if (threadIdx.x == 0) {
    uint64_t *st = w.tiles;
    uint64_t excl = 0;
    if (tile == 0) {
      __hip_atomic_store(st, ((uint64_t)agg << 2) | 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(st + tile, ((uint64_t)agg << 2) | 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int64_t p = (int64_t)tile - 1;
      uint32_t spins = 0;
      while (p >= 0) {
        const uint64_t v = __hip_atomic_load(st + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t f = (uint32_t)(v & 3u);
        if (f == 0) {
          if (++spins > kTileSpin) {  // never expected: report it and go on
            count(w.cnt, C_SPIN);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += v >> 2;
        if (f == 2) break;
        p--;
      }
      __hip_atomic_store(st + tile, ((excl + agg) << 2) | 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_excl = excl;
    if ((uint64_t)(tile + 1) * 256 >= g.n_blocks) w.tot[0] = excl + agg;  // the field's payload words
  }
  __syncthreads();
  if (!active) return;

  // ---- encoding: the codes again, a plane at a time --------------------------
  PlaneCodes<B0, B1, B2> bc;
  bc.init(w.codes, blk, g.groups);
  bc.load(0);
  uint32_t *ring = ring_all + threadIdx.x;  // word with absolute index a at ring[(a & 15) * 256]
  const gptr<uint32_t> pay = gbl((uint32_t *)(out + h.off_payload));
  uint64_t wabs = s_excl + before + (incl - words);  // absolute index of the next word produced
  uint64_t fl = wabs;                       // first word not yet written out
  auto flush = [&]() {
    if (fl & 7) {  // block head: single words up to the first chunk boundary
      const uint64_t hb = (fl + 7) & ~7ull;
      if (wabs >= hb)
        for (; fl < hb; fl++) pay[fl] = ring[(fl & 15) * 256];
    }
    if (!(fl & 7) && fl + 8 <= wabs) {
      const uint32_t s0 = (uint32_t)(fl & 8);
      uint4 u0, u1;
      u0.x = ring[(s0 + 0) * 256];
      u0.y = ring[(s0 + 1) * 256];
      u0.z = ring[(s0 + 2) * 256];
      u0.w = ring[(s0 + 3) * 256];
      u1.x = ring[(s0 + 4) * 256];
      u1.y = ring[(s0 + 5) * 256];
      u1.z = ring[(s0 + 6) * 256];
      u1.w = ring[(s0 + 7) * 256];
      const gptr<v4u32> d = (gptr<v4u32>)(pay + fl);
      d[0] = v4u32{u0.x, u0.y, u0.z, u0.w};
      d[1] = v4u32{u1.x, u1.y, u1.z, u1.w};
      fl += 8;
    }
  };
  uint64_t acc = 0;
  uint32_t nacc = 0;
  constexpr int FE = B2 < 8 ? B2 : 8;  // codes between flushes (<= 6 words), as in k_encode_fast
#pragma unroll
  for (int i = 0; i < B0; i++) {
    if (i + 1 < B0) bc.load(i + 1);
#pragma unroll
    for (int j = 0; j < B1; j++) {
#pragma unroll
      for (int k = 0; k < B2; k++) {
        const int q = j * B2 + k;
        const bool v = (uint32_t)i < e0 && (uint32_t)j < n1 && (uint32_t)k < n2;
        const uint32_t e = enc_of(v ? bc.at(i, q) : kRadius, encw, w.enc);
        const uint32_t len = v ? (e & 0xFFu) : 0u;
        acc = (acc << len) | (e >> 8 & ((1u << len) - 1u));
        nacc += len;
        if (nacc >= 32) {
          nacc -= 32;
          ring[(wabs & 15) * 256] = (uint32_t)(acc >> nacc);
          wabs++;
          acc &= (1ull << nacc) - 1;
        }
        if ((k + 1) % FE == 0 || k + 1 == B2) flush();
      }
      __asm__ volatile("" : "+v"(acc), "+v"(nacc), "+v"(wabs), "+v"(fl)::"memory");
    }
  }
  if (nacc > 0) {
    ring[(wabs & 15) * 256] = (uint32_t)(acc << (32 - nacc));
    wabs++;
  }
  flush();
  for (; fl < wabs; fl++) pay[fl] = ring[(fl & 15) * 256];  // block tail
  const uint32_t meta = w.meta[blk];
  uint32_t *tab = (uint32_t *)(out + h.off_table) + 2 * blk;
  tab[0] = words;
  tab[1] = meta;
  if (__builtin_expect((meta >> 1) != 0, 0)) {
    const T *src = (const T *)w.vals + blk * (uint64_t)g.bpts;
    T *od = (T *)(out + h.off_outliers) + w.off_out[blk];
    for (uint32_t t = 0; t < (meta >> 1); t++) od[t] = src[t];
  }
  if (meta & 1u) {
    const T *cf = (const T *)w.coef + 4 * blk;
    T *cd = (T *)(out + h.off_coef) + 4ull * w.off_coef[blk];
    for (int a = 0; a < 4; a++) cd[a] = cf[a];
  }
  if (h.abft) ((uint64_t *)(out + h.off_sumdc))[blk] = w.sum_dc[blk];
}

template __global__ void k_checkenc_fast<float, 6, 6, 6>(JobTab);
template __global__ void k_checkenc_fast<double, 6, 6, 6>(JobTab);
template __global__ void k_check_fast<3, 6, 6, 6>(JobTab);
template __global__ void k_check_fast<2, 1, 16, 16>(JobTab);
template __global__ void k_encode_fast<float, 3, 6, 6, 6>(JobTab);
template __global__ void k_encode_fast<double, 3, 6, 6, 6>(JobTab);
template __global__ void k_encode_fast<float, 2, 1, 16, 16>(JobTab);
template __global__ void k_encode_fast<double, 2, 1, 16, 16>(JobTab);

}  // namespace sdcsz
