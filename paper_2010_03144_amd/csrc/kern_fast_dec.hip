// kern_fast_dec.hip -- block-shape-specialised decompression: one lane per block.
//
// Algorithm 2 for one block per lane: canonical Huffman decoding through a
// lookup table in LDS (the first kLutBits bits of a codeword; longer codes
// take a short search by length), reconstruction with the arithmetic of
// compression (previous reconstructed plane in registers), the checksum of
// the block against sum_dc, and coalesced row stores.  A checksum mismatch
// or an undecodable block is queued for k_decode_redo (re-execution from the
// compressed bytes); blocks named in a fault plan run in k_decode_list.
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

template <typename V> __device__ inline void dpin(V &v) { __asm__ volatile("" : "+v"(v)); }
template <typename... V> __device__ inline void drow_fence(V &...v) {
  (dpin(v), ...);
  __asm__ volatile("" ::: "memory");
}

// Bit reader over one block's payload words (most significant bit first).
struct Bits {
  const uint32_t *pay;
  uint32_t nw;    // payload words of the block
  uint32_t wi;    // next word to fetch into `nxt`
  uint32_t nxt;   // prefetched word
  uint64_t buf;   // left-aligned unread bits
  uint32_t nb;    // valid bits in buf
  uint32_t used;  // bits consumed
  __device__ void init(const uint32_t *p, uint32_t n) {
    pay = p;
    nw = n;
    const uint32_t w0 = n > 0 ? p[0] : 0u, w1 = n > 1 ? p[1] : 0u;
    buf = ((uint64_t)w0 << 32) | w1;
    nb = 64;
    wi = 2;
    nxt = n > 2 ? p[2] : 0u;
    used = 0;
  }
  // top bits available for the next codeword (>= 32 valid bits after refill)
  __device__ inline void refill() {
    if (nb < 32) {
      buf |= (uint64_t)nxt << (32 - nb);
      nb += 32;
      wi++;
      nxt = wi < nw ? pay[wi] : 0u;
    }
  }
  __device__ inline void skip(uint32_t len) {
    buf <<= len;
    nb -= len;
    used += len;
  }
};

// Decode one symbol; sets *bad on an invalid code or a read past the block.
__device__ inline uint32_t decode_sym(Bits &br, const uint32_t *lut, const DecTab *tab, const uint16_t *symbols,
                                      bool *bad) {
  br.refill();
  const uint32_t e = lut[(uint32_t)(br.buf >> (64 - kLutBits))];
  uint32_t len = e & 0xFFu, sym = e >> 8;
  if (__builtin_expect(len == 0, 0)) {
    sym = 0;
    for (uint32_t l = kLutBits + 1; l <= kMaxLen; l++) {
      const uint32_t c = (uint32_t)(br.buf >> (64 - l));
      const uint32_t f = tab->first[l], n = tab->count[l];
      if (n && c >= f && c - f < n) {
        sym = symbols[tab->start[l] + c - f];
        len = l;
        break;
      }
    }
    if (len == 0) {
      *bad = true;
      len = 1;
    }
  }
  if (br.used + len > br.nw * 32u) *bad = true;
  br.skip(len);
  return sym;
}

}  // namespace

template <typename T, int ND, int B0, int B1, int B2, bool FULL>
__device__ __forceinline__ void decode_lanes(const uint8_t *__restrict__ s, const Header &h, const Geo &g,
                                             const DecWork &w, const PlanDev &plan, T *out, const Launch &L,
                                             const uint32_t *lut, uint64_t idx, uint64_t nlanes) {
  bool active = idx < nlanes;
  const uint64_t blk = dmap_block(g, L, FULL ? 0u : 1u, active ? idx : nlanes - 1);
  const Box bx = box_of(g, blk);
  const uint64_t org = fidx(g, bx, 0, 0, 0);
  uint64_t omin = org;
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)omin, off);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(omin >> 32), off);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    omin = o < omin ? o : omin;
  }
  const uint64_t org0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(omin >> 32)) << 32) |
                        (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)omin);
  char *wbase = (char *)(out + org0);
  const uint32_t loff = (uint32_t)((org - org0) * sizeof(T));
  if (active && plan_hit(plan, blk)) active = false;  // done by k_decode_list
  if (!active) return;

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
  Bits br;
  br.init((const uint32_t *)(s + h.off_payload) + w.off_pay[blk], (uint32_t)(w.off_pay[blk + 1] - w.off_pay[blk]));
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
      T Aj = A0 + beta1 * ((T)j - c1);
      dpin(Aj);
      T rowold[B2], rv[B2];
      T cprev = 0, Up = 0;
#pragma unroll
      for (int k = 0; k < B2; k++) {
        const bool v = FULL || (uint32_t)k < n2;
        const uint32_t sym = v ? decode_sym(br, lut, w.tab, w.symbols, &bad) : kRadius;
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
            if (used_out < nout) r = outl[used_out];
            else bad = true;
            used_out++;
          }
        }
        Pw[j][k] = r;
        rv[k] = r;
        cprev = r;
        Up = U1;
        if (v) sum += Wd<T>::sum(r);
      }
      // store the row
      char *dst = wbase + (loff + (uint32_t)i * PSB + (uint32_t)j * RSB);
#pragma unroll
      for (int k = 0; k < B2; k++)
        if (FULL || (uint32_t)k < n2) *(T *)(dst + k * sizeof(T)) = rv[k];
#pragma unroll
      for (int k = 0; k < B2; k++) Sv[k] = rowold[k];
      drow_fence(cprev, sum, br.buf, br.nb);
    }
  }
  if (used_out != nout) bad = true;
  const uint64_t *sumdc = (const uint64_t *)(s + h.off_sumdc);
  uint64_t why = 0;
  if (bad) why = 2;
  else if (h.abft && sum != sumdc[blk]) {
    why = 1;
    count(w.cnt, C_DET + SDCSZ_T_RECON);
  }
  if (__builtin_expect(why != 0, 0)) {
    const uint32_t slot = atomicAdd(w.redo_n, 1u);
    if (slot < kMaxRedo) w.redo[slot] = blk | (why << 56);
  }
}

// Work-groups [0, L.full_wgs) take full blocks, the rest the partial shell.
template <typename T, int ND, int B0, int B1, int B2>
__global__ void __launch_bounds__(256)
k_decode_fast(const uint8_t *__restrict__ s, Header h, Geo g, DecWork w, PlanDev plan, T *out, Launch L) {
  if (*w.err) return;  // invalid codebook or block table: nothing is read
  __shared__ uint32_t lut[1u << kLutBits];
  for (uint32_t t = threadIdx.x; t < (1u << kLutBits); t += blockDim.x) lut[t] = w.lut[t];
  __syncthreads();
  if (blockIdx.x < L.full_wgs)
    decode_lanes<T, ND, B0, B1, B2, true>(s, h, g, w, plan, out, L, lut,
                                          (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, L.full_count);
  else
    decode_lanes<T, ND, B0, B1, B2, false>(s, h, g, w, plan, out, L, lut,
                                           (uint64_t)(blockIdx.x - L.full_wgs) * blockDim.x + threadIdx.x,
                                           L.shell_count);
}

#define SDCSZ_INST_DEC(T, ND, B0, B1, B2) \
  template __global__ void k_decode_fast<T, ND, B0, B1, B2>(const uint8_t *, Header, Geo, DecWork, PlanDev, T *, Launch);
SDCSZ_INST_DEC(float, 3, 6, 6, 6)
SDCSZ_INST_DEC(double, 3, 6, 6, 6)

}  // namespace sdcsz
