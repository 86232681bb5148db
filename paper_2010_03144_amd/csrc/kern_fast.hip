// kern_fast.hip -- block-shape-specialised compression: one lane per block.
//
// Block edges are template parameters, so the block's values sit in
// registers with compile-time indexing: a fully unrolled first pass (input
// checksums, regression sums, costs at the diagonal samples) and a plane loop
// that keeps the previous reconstructed plane in registers for the Lorenzo
// recursion.  The input is read twice (first pass, prediction pass); the
// first pass takes the exact 64-bit input checksums of Algorithm 1, the
// prediction pass recomputes them (modulo 2^32) over exactly the words it
// predicts from, which detects a word changed in between.  The coefficient
// checksums are taken when the coefficients are computed and verified (a
// corrupted word located and repaired in place) before the prediction pass.
// A block whose input checksums or duplicated computations disagree is
// queued with its first-pass checksums; k_redo_wave (kern_wave.hip) locates
// and repairs the input word against them and runs the block again.
//
// Two instantiations of the per-lane routine share this source: the
// production one, which leaves the blocks a fault plan names, and one that
// runs those blocks (a launch over the plan's list of blocks) and applies the
// flips at the program points of evaluation mode A (input and coefficient
// memory errors after their checksums, flips of the first copy of a
// duplicated prediction or reconstruction).  Blocks whose plan that
// instantiation does not model take the wave-per-block routine
// (k_compress_wave_list).
#include "block_generic.h"
#include "kern.h"

namespace sdcsz {

namespace {

// reasons a block is queued for a re-run (high byte of the queue entry)
constexpr uint64_t kWhyInput = 1, kWhyPred = 4, kWhyRecon = 8;

__device__ inline uint64_t map_block(const Geo &g, const Launch &L, uint32_t mode, uint64_t idx) {
  uint64_t c0, c1, c2;
  if (mode == 0) {
    c2 = idx % L.nf[2];
    uint64_t t = idx / L.nf[2];
    c1 = t % L.nf[1];
    c0 = t / L.nf[1];
  } else if (idx < L.s2) {  // slab of blocks partial along the fastest axis
    c2 = g.nb[2] - 1;
    c1 = idx % g.nb[1];
    c0 = idx / g.nb[1];
  } else if (idx < L.s2 + L.s1) {  // partial along the middle axis
    uint64_t t = idx - L.s2;
    c1 = g.nb[1] - 1;
    c2 = t % L.nf[2];
    c0 = t / L.nf[2];
  } else {  // partial along the slowest axis
    uint64_t t = idx - L.s2 - L.s1;
    c0 = g.nb[0] - 1;
    c2 = t % L.nf[2];
    c1 = t / L.nf[2];
  }
  return (c0 * g.nb[1] + c1) * g.nb[2] + c2;
}

// an opaque copy: the compiler must assume a different value, so a
// computation on it is carried out again rather than reused
template <typename T> __device__ inline T launder(T v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}

// Compiler-only barrier that consumes a row's results: the row's work stays
// before it and the next row's loads after it, so loads run one row ahead of
// their use instead of all at once (which would hold the whole block).
template <typename V> __device__ inline void pin(V &v) { __asm__ volatile("" : "+v"(v)); }
template <typename... V> __device__ inline void row_fence(V &...v) {
  (pin(v), ...);
  __asm__ volatile("" ::: "memory");
}

// point (i,j,k) lies on a diagonal of the configured block (3D: the four
// space diagonals; 2D: the two diagonals)
template <int ND, int B0, int B1, int B2> constexpr bool is_sample(int i, int j, int k) {
  if (ND == 2) {
    constexpr int m = B1 < B2 ? B1 : B2;
    return j < m && (k == j || k == B2 - 1 - j);
  }
  constexpr int m = B0 < B1 ? (B0 < B2 ? B0 : B2) : (B1 < B2 ? B1 : B2);
  return (i < m && j == i && k == i) || (i < m && j == i && k == B2 - 1 - i) ||
         (i < m && k == i && j == B1 - 1 - i) || (j < m && k == j && i == B0 - 1 - j);
}

// slot of a sample point among the samples in C order
template <int ND, int B0, int B1, int B2> constexpr int sample_slot(int i0, int j0, int k0) {
  int n = 0;
  for (int i = 0; i < B0; i++)
    for (int j = 0; j < B1; j++)
      for (int k = 0; k < B2; k++) {
        if (i == i0 && j == j0 && k == k0) return n;
        if (is_sample<ND, B0, B1, B2>(i, j, k)) n++;
      }
  return n;
}

// Checksum-word accumulation of the prediction pass: S = sum of the words,
// Q = sum of the running sums (the paper's isum = sum_j j * w_j, 0-based j,
// is n_words*S - Q).  This pair only detects, so it is kept modulo 2^32: a
// corrupted word changes S by a non-zero amount below 2^32 in magnitude,
// which no 32-bit wrap can hide.  Locating the word takes the exact
// first-pass pair (Ck64), which k_redo_wave compares with the memory as it
// is.
template <typename T> struct Ck;
template <> struct Ck<float> {
  __device__ static inline void add(float v, uint32_t &S, uint32_t &Q) {
    S += __float_as_uint(v);
    Q += S;
  }
};
template <> struct Ck<double> {
  __device__ static inline void add(double v, uint32_t &S, uint32_t &Q) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    S += (uint32_t)u;
    Q += S;
    S += (uint32_t)(u >> 32);
    Q += S;
  }
};

// The double-precision check of the bound, with an FP32 shortcut taken only
// where it provably agrees with the double comparison.
template <typename T> struct Bound;
template <> struct Bound<float> {
  __device__ static inline bool ok(float x, float r, const EbDev &e) {
    const float d = fabsf(x - r);
    const bool fast = d <= e.lo;
    const bool maybe = !fast && !(d > e.hi);  // NaN and the thin band around eb
    if (__builtin_expect(__ballot(maybe) != 0, 0)) {
      const bool exact = fabs((double)x - (double)r) <= e.eb_abs;
      return fast || (maybe && exact);
    }
    return fast;
  }
};
template <> struct Bound<double> {
  __device__ static inline bool ok(double x, double r, const EbDev &e) { return fabs(x - r) <= e.eb_abs; }
};

// Exact (64-bit) input checksums of the first pass: S = sum of the words,
// Q = sum of the running sums, so isum = n_words * S - Q (mod 2^64).  The
// low 32 bits equal the prediction pass's Ck pair over the same words.
template <typename T> struct Ck64;
template <> struct Ck64<float> {
  __device__ static inline void add(float v, uint64_t &S, uint64_t &Q) {
    S += __float_as_uint(v);
    Q += S;
  }
};
template <> struct Ck64<double> {
  __device__ static inline void add(double v, uint64_t &S, uint64_t &Q) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    S += (uint32_t)u;
    Q += S;
    S += u >> 32;
    Q += S;
  }
};

// value v with word `half` (0 low, 1 high for FP64) xor-ed with m
template <typename T> __device__ inline T word_xor(T v, uint32_t half, uint32_t m) {
  uint32_t wv[2] = {0, 0};
  Wd<T>::split(v, wv);
  wv[0] ^= half == 0 ? m : 0u;
  if (Wd<T>::per == 2) wv[1] ^= half == 1 ? m : 0u;
  return Wd<T>::join(wv);
}

// Checksums of the coefficient words (Sec. 3.2 algebra: sum, and sum of
// index times word, 0-based).
template <typename T> __device__ inline void coef_sums(T b0, T b1, T b2, T m, uint64_t &s, uint64_t &is) {
  constexpr uint32_t per = Wd<T>::per;
  uint32_t cw[4 * per];
  Wd<T>::split(b0, cw);
  Wd<T>::split(b1, cw + per);
  Wd<T>::split(b2, cw + 2 * per);
  Wd<T>::split(m, cw + 3 * per);
  s = 0;
  is = 0;
#pragma unroll
  for (uint32_t a = 0; a < 4 * per; a++) {
    s += cw[a];
    is += (uint64_t)a * cw[a];
  }
}

// Verify the coefficients against their checksums; a single corrupted word
// is located and repaired in place (Algorithm 1, third loop).  Returns 0
// clean, 1 repaired, -1 uncorrectable.
template <typename T> __device__ inline int coef_check(T &b0, T &b1, T &b2, T &m, uint64_t s, uint64_t is) {
  constexpr uint32_t per = Wd<T>::per;
  uint64_t s2, i2;
  coef_sums<T>(b0, b1, b2, m, s2, i2);
  if (s2 == s && i2 == is) return 0;
  uint32_t cw[4 * per];
  Wd<T>::split(b0, cw);
  Wd<T>::split(b1, cw + per);
  Wd<T>::split(b2, cw + 2 * per);
  Wd<T>::split(m, cw + 3 * per);
  uint64_t jf = 0;
  uint32_t vf = 0;
  const int st = locate_repair(s2, i2, s, is, 4 * per, 32, [&](uint64_t j) {
    uint32_t x = 0;
#pragma unroll
    for (uint32_t a = 0; a < 4 * per; a++) x = a == j ? cw[a] : x;
    return x;
  }, &jf, &vf);
  if (st != 1) return st;
#pragma unroll
  for (uint32_t a = 0; a < 4 * per; a++) cw[a] = a == jf ? vf : cw[a];
  b0 = Wd<T>::join(cw);
  b1 = Wd<T>::join(cw + per);
  b2 = Wd<T>::join(cw + 2 * per);
  m = Wd<T>::join(cw + 3 * per);
  return 1;
}

// per-lane routine instantiations
enum { kProd = 0, kFaults = 1 };

// A lane's flips of a fault plan (at most one of each kind: the host sends
// blocks with more to the generic routine).  Words and points index the
// block in C order over its actual extents.  The wave flags are uniform:
// some lane of the wave has a flip of that kind.
struct LaneFaults {
  uint32_t in = ~0u;            // INPUT: 32-bit word | bit << 16
  uint32_t cf = ~0u;            // COEF: coefficient word | bit << 16
  uint32_t dp = ~0u, dr = ~0u;  // DUP_PRED / DUP_RECON: point | bit << 16
  bool wave_in = false, wave_dp = false, wave_dr = false;
  __device__ uint32_t in_w() const { return in & 0xFFFFu; }
  __device__ uint32_t in_m() const { return 1u << ((in >> 16) & 31); }
};

// All lanes of the wave call this (the flags are ballots).
__device__ inline LaneFaults lane_faults(const PlanDev &plan, uint64_t blk, bool active) {
  LaneFaults f;
  if (active && plan_hit(plan, blk)) {
    for (uint32_t t = plan_first(plan, blk); t < plan.n && plan.f[t].block == blk; t++) {
      const sdcsz_fault e = plan.f[t];
      if (e.target == SDCSZ_T_INPUT) {
        f.in = (uint32_t)e.word | (e.bit << 16);
      } else if (e.target == SDCSZ_T_COEF) {
        f.cf = (uint32_t)e.word | (e.bit << 16);
      } else if (e.target == SDCSZ_T_DUP_PRED) {
        f.dp = (uint32_t)e.word | (e.bit << 16);
      } else if (e.target == SDCSZ_T_DUP_RECON) {
        f.dr = (uint32_t)e.word | (e.bit << 16);
      }
    }
  }
  f.wave_in = __ballot(f.in != ~0u) != 0;
  f.wave_dp = __ballot(f.dp != ~0u) != 0;
  f.wave_dr = __ballot(f.dr != ~0u) != 0;
  return f;
}

// Flip the coefficient word w of (b0, b1, b2, m) by mask mk.  Selects, not
// branches: hipcc laid out an if-else chain over the four coefficients of the
// FP64 instantiation so that a flip of the last one took the first one's
// value (the chain's last branch lost its input in the structured control
// flow), which made such flips uncorrectable.
template <typename T> __device__ inline void coef_flip(T &b0, T &b1, T &b2, T &m, uint32_t w, uint32_t mk) {
  constexpr uint32_t per = Wd<T>::per;
  const uint32_t a = w / per, half = w % per;
  b0 = a == 0 ? word_xor(b0, half, mk) : b0;
  b1 = a == 1 ? word_xor(b1, half, mk) : b1;
  b2 = a == 2 ? word_xor(b2, half, mk) : b2;
  m = a == 3 ? word_xor(m, half, mk) : m;
}

// What a lane's pass found: mismatch reasons and the first-pass checksums.
struct LaneOut {
  uint64_t why, S1, Q1;
};

// The wave's lowest block origin (every lane takes part; inactive lanes pass
// a valid block's origin).
__device__ inline uint64_t wave_min(uint64_t org) {
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

}  // namespace

// One lane's block: full blocks (FULL) have compile-time extents, blocks of
// the partial shell mask every point by their actual extents.  MODE selects
// the instantiation (kProd, kFaults).  Every lane of the wave calls it
// (inactive lanes with a valid block id).  Returns the lane's mismatch
// reasons and first-pass checksums; the checksums wait in `stash` (two
// words of LDS per lane) through the prediction pass, which keeps only
// their low halves in registers.
template <typename T, int ND, int B0, int B1, int B2, bool FULL, bool ABFT, bool WIDE, int MODE>
__device__ __forceinline__ LaneOut compress_lanes(const T *__restrict__ in, const Geo &g, const RegTab<T> &rt,
                                                  const PlanDev &plan, const CompWork &w, uint32_t predictor,
                                                  uint32_t *hist, uint32_t hlo, uint32_t hw, uint32_t &hot,
                                                  uint64_t blk, bool active, uint64_t *stash) {
  constexpr int PL = B1 * B2;  // points per plane
  static_assert(PL % 4 == 0, "a plane must fill whole 4-code groups");
  constexpr int NS = sample_slot<ND, B0, B1, B2>(B0, 0, 0);
  constexpr uint32_t per = Wd<T>::per;
  // wave-uniform base of the input (the wave's lowest block origin); lanes
  // address it with 32-bit byte offsets (fields below 2 GiB, so every offset
  // fits; wider fields take the WIDE instantiation)
  const Box bx = box_of(g, blk);
  const uint64_t org = fidx(g, bx, 0, 0, 0);
  const uint64_t org0 = WIDE ? 0 : wave_min(org);
  // below 2 GiB: a wave-uniform base and 32-bit per-lane offsets; wider
  // fields: a per-lane base at the block's origin (32-bit offsets inside it)
  const char *wbase = WIDE ? (const char *)(in + org) : (const char *)(in + org0);
  const uint32_t loff = WIDE ? 0u : (uint32_t)((org - org0) * sizeof(T));
  // plan blocks: the fault-applying launch over the plan's list, or k_compress_wave_list
  if (MODE == kProd && active && plan_hit(plan, blk)) active = false;
  const LaneFaults lf = MODE == kFaults ? lane_faults(plan, blk, active) : LaneFaults{};
  LaneOut out{0, 0, 0};
  if (active) {
    const EbDev eb = *w.eb;
    const T q = EbSel<T>::q(eb), inv = EbSel<T>::inv(eb), inv_e = EbSel<T>::inv_e(eb);
    const uint32_t n0 = FULL ? B0 : bx.n[0], n1 = FULL ? B1 : bx.n[1], n2 = FULL ? B2 : bx.n[2];
    const uint32_t pat = FULL ? 0 : bx.pat;
    const T c0 = rt.c[pat][0], c1 = rt.c[pat][1], c2 = rt.c[pat][2];
    const uint32_t PSB = (uint32_t)(g.d[1] * g.d[2] * sizeof(T)), RSB = (uint32_t)(g.d[2] * sizeof(T));
    auto valid = [&](int i, int j, int k) -> bool {
      return FULL || ((uint32_t)i < n0 && (uint32_t)j < n1 && (uint32_t)k < n2);
    };
    auto ld = [&](int i, int j, int k) -> T {
      if (FULL) return *gbl((const T *)(wbase + (loff + (uint32_t)i * PSB + (uint32_t)j * RSB) + k * sizeof(T)));
      const uint32_t ii = min((uint32_t)i, n0 - 1), jj = min((uint32_t)j, n1 - 1), kk = min((uint32_t)k, n2 - 1);
      const T v = *gbl((const T *)(wbase + (loff + ii * PSB + jj * RSB + kk * (uint32_t)sizeof(T))));
      return valid(i, j, k) ? v : (T)0;
    };

    // ---- first pass: input checksums, regression sums, Lorenzo costs ------
    T x[B0][B1][B2];
    T sx[NS > 0 ? NS : 1];
    uint64_t S1 = 0, Q1 = 0;
    uint32_t e_lor = 0;
    T S0 = 0, Sa0 = 0, Sa1 = 0, Sa2 = 0;
#pragma unroll
    for (int j = 0; j < B1; j++)
#pragma unroll
      for (int k = 0; k < B2; k++) x[0][j][k] = ld(0, j, k);
#pragma unroll
    for (int i = 0; i < B0; i++) {
      T P = 0, A = 0, Bv = 0;
      T D[B2];
#pragma unroll
      for (int k = 0; k < B2; k++) D[k] = 0;
      // loads run one plane ahead of the work (a row's work is far shorter
      // than the memory latency)
      if (i + 1 < B0) {
#pragma unroll
        for (int j = 0; j < B1; j++)
#pragma unroll
          for (int k = 0; k < B2; k++) x[i + 1][j][k] = ld(i + 1, j, k);
      }
#pragma unroll
      for (int j = 0; j < B1; j++) {
        T R = 0;
#pragma unroll
        for (int k = 0; k < B2; k++) {
          if (valid(i, j, k)) {
            if (ABFT) Ck64<T>::add(x[i][j][k], S1, Q1);
            R = R + x[i][j][k];
            D[k] = D[k] + x[i][j][k];
          }
          if (is_sample<ND, B0, B1, B2>(i, j, k)) {
            // Lorenzo on the original values (zero outside the block)
            auto X = [&](int a, int b, int c) -> T { return (a < 0 || b < 0 || c < 0) ? (T)0 : x[a][b][c]; };
            T pl;
            if (ND == 2) {
              pl = (X(i, j - 1, k) + X(i, j, k - 1)) - X(i, j - 1, k - 1);
            } else {
              const T u = (X(i - 1, j, k) + X(i, j - 1, k)) - X(i - 1, j - 1, k);
              const T up = (X(i - 1, j, k - 1) + X(i, j - 1, k - 1)) - X(i - 1, j - 1, k - 1);
              pl = X(i, j, k - 1) + (u - up);
            }
            sx[sample_slot<ND, B0, B1, B2>(i, j, k)] = x[i][j][k];
            if (valid(i, j, k)) e_lor += cost<T>(x[i][j][k] - pl, inv_e) + 1u;
          }
        }
        if (valid(i, j, 0)) {
          P = P + R;
          A = A + ((T)j - c1) * R;
        }
        row_fence(P, A, S1, Q1, e_lor);
#pragma unroll
        for (int k = 0; k < B2; k++) pin(D[k]);
      }
#pragma unroll
      for (int k = 0; k < B2; k++)
        if (valid(i, 0, k)) Bv = Bv + ((T)k - c2) * D[k];
      if (valid(i, 0, 0)) {
        S0 = S0 + P;
        Sa0 = Sa0 + ((T)i - c0) * P;
        Sa1 = Sa1 + A;
        Sa2 = Sa2 + Bv;
      }
    }
    uint32_t S1l = 0, Q1l = 0;  // what the prediction pass compares with
    if (ABFT) {
      stash[0] = S1;
      stash[1] = Q1;
      S1l = (uint32_t)S1;
      Q1l = (uint32_t)Q1;
    }
    T beta0 = n0 > 1 ? Sa0 * rt.K[pat][0] : (T)0;
    T beta1 = n1 > 1 ? Sa1 * rt.K[pat][1] : (T)0;
    T beta2 = n2 > 1 ? Sa2 * rt.K[pat][2] : (T)0;
    T mu = S0 * rt.inv_pts[pat];
    uint64_t s_c = 0, i_c = 0;  // coefficient checksums, taken as they are computed
    if (ABFT) coef_sums<T>(beta0, beta1, beta2, mu, s_c, i_c);

    bool is_reg;
    if (predictor == SDCSZ_PRED_LORENZO) is_reg = false;
    else if (predictor == SDCSZ_PRED_REGRESSION) is_reg = true;
    else {
      uint32_t e_reg = 0;
#pragma unroll
      for (int i = 0; i < B0; i++)
#pragma unroll
        for (int j = 0; j < B1; j++)
#pragma unroll
          for (int k = 0; k < B2; k++) {
            if (!is_sample<ND, B0, B1, B2>(i, j, k)) continue;
            const T pr = ((beta0 * ((T)i - c0) + beta1 * ((T)j - c1)) + beta2 * ((T)k - c2)) + mu;
            if (valid(i, j, k)) e_reg += cost<T>(sx[sample_slot<ND, B0, B1, B2>(i, j, k)] - pr, inv_e);
          }
      is_reg = e_reg <= e_lor;
    }

    uint64_t why = 0;
    if (MODE == kFaults && lf.cf != ~0u) {  // memory error in a coefficient after its checksums
      coef_flip<T>(beta0, beta1, beta2, mu, lf.cf & 0xFFFFu, 1u << ((lf.cf >> 16) & 31));
      count(w.cnt, C_INJ + SDCSZ_T_COEF);
    }
    if (ABFT) {  // verify (and repair) the coefficients as they are held now
      beta0 = launder(beta0);
      beta1 = launder(beta1);
      beta2 = launder(beta2);
      mu = launder(mu);
      const int st = coef_check<T>(beta0, beta1, beta2, mu, s_c, i_c);
      if (__builtin_expect(st != 0, 0)) {
        count(w.cnt, C_DET + SDCSZ_T_COEF);
        count(w.cnt, (st > 0 ? C_COR : C_UNC) + SDCSZ_T_COEF);
      }
    }

    // ---- prediction pass ------------------------------------------------
    T Pw[B1][B2];  // reconstructed plane i-1, overwritten row by row with plane i
#pragma unroll
    for (int j = 0; j < B1; j++)
#pragma unroll
      for (int k = 0; k < B2; k++) Pw[j][k] = 0;
    const T beta0d = ABFT ? launder(beta0) : beta0, beta1d = ABFT ? launder(beta1) : beta1;
    const T beta2d = ABFT ? launder(beta2) : beta2;
    T Bk[B2], Bk2[B2];
#pragma unroll
    for (int k = 0; k < B2; k++) {
      Bk[k] = beta2 * ((T)k - c2);
      Bk2[k] = beta2d * ((T)k - c2);
    }
    uint32_t S2 = 0, Q2 = 0;
    uint64_t s_dc = 0, is_q = 0;
    uint32_t s_q = 0, nout = 0;
    uint32_t mis_p = 0, mis_r = 0;  // OR of bit differences between the duplicated results
    T *outl = (T *)w.vals + blk * (uint64_t)g.bpts;
    const gptr<v2u32> cbase = gbl((v2u32 *)(w.codes + code_index(blk, 0, g.groups)));  // next group is 64 vectors on
    T xn[B2], xn2[B2];  // the next two rows, loaded two rows ahead of their use
#pragma unroll
    for (int k = 0; k < B2; k++) {
      xn[k] = ld(0, 0, k);
      xn2[k] = ld(0, 1, k);
    }
#pragma unroll 1
    for (int i = 0; i < B0; i++) {
      if (!FULL && (uint32_t)i >= n0) break;
      const T A0 = beta0 * ((T)i - c0), A0d = beta0d * ((T)i - c0);
      T Sv[B2];  // row j-1 of plane i-1
#pragma unroll
      for (int k = 0; k < B2; k++) Sv[k] = 0;
      uint32_t pk0 = 0, pk1 = 0;
#pragma unroll
      for (int j = 0; j < B1; j++) {
        T Aj = A0 + beta1 * ((T)j - c1), Ajd = A0d + beta1d * ((T)j - c1);
        pin(Aj);  // keeps this row's regression predictions inside the row
        if (ABFT) pin(Ajd);
        T xr[B2];
#pragma unroll
        for (int k = 0; k < B2; k++) {
          xr[k] = xn[k];
          xn[k] = xn2[k];
        }
        if (j + 2 < B1) {
#pragma unroll
          for (int k = 0; k < B2; k++) xn2[k] = ld(i, j + 2, k);
        } else if (i + 1 < B0) {
#pragma unroll
          for (int k = 0; k < B2; k++) xn2[k] = ld(i + 1, j + 2 - B1, k);
        }
        T rowold[B2];
        T cprev = 0, Up = 0, Up2 = 0;
        uint32_t rs = 0, rk = 0;
        const uint32_t prow = ((uint32_t)i * n1 + (uint32_t)j) * n2;  // point index of the row's start
#pragma unroll
        for (int k = 0; k < B2; k++) {
          const bool v = valid(i, j, k);
          T xv = xr[k];
          if (MODE == kFaults && lf.wave_in) {  // the memory error the first pass did not see
            if (v && lf.in_w() / per == prow + k) {
              xv = word_xor(xv, lf.in_w() % per, lf.in_m());
              count(w.cnt, C_INJ + SDCSZ_T_INPUT);
            }
          }
          if (ABFT && v) Ck<T>::add(xv, S2, Q2);
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
          T pred = is_reg ? reg : lor;
          if (MODE == kFaults && lf.wave_dp) {  // flip of the first copy
            if (v && (lf.dp & 0xFFFFu) == prow + k) {
              pred = Wd<T>::flip(pred, lf.dp >> 16);
              count(w.cnt, C_INJ + SDCSZ_T_DUP_PRED);
            }
          }
          if (ABFT) {  // pred' <- f_dup()
            const T bl = launder(b);
            T lor2, U2 = 0;
            if (ND == 2) {
              const T f = (j > 0 && k > 0) ? Pw[j - 1][k - 1] : (T)0;
              lor2 = (bl + cprev) - f;
            } else {
              U2 = (a + bl) - d;
              lor2 = cprev + (U2 - Up2);
            }
            const T reg2 = (Ajd + Bk2[k]) + mu;
            mis_p |= Wd<T>::diff(pred, is_reg ? reg2 : lor2);
            Up2 = U2;
          }
          const T diff = xv - pred;
          const T t = fabs(diff) * inv + (T)0.5;
          const bool inr = t < (T)32768;
          // m = trunc(t) with the sign of the difference; truncating the
          // signed value gives the same integer (-0.0 gives 0 either way)
          const int sm = (int)copysign(t, diff);
          T r1 = pred + (T)sm * q;
          if (MODE == kFaults && lf.wave_dr) {  // flip of the first copy (codes in range only)
            if (v && inr && (lf.dr & 0xFFFFu) == prow + k) {
              r1 = Wd<T>::flip(r1, lf.dr >> 16);
              count(w.cnt, C_INJ + SDCSZ_T_DUP_RECON);
            }
          }
          if (ABFT) mis_r |= Wd<T>::diff(r1, pred + (T)launder(sm) * q);  // dec_dup()
          const bool bok = Bound<T>::ok(xv, r1, eb);
          const bool ok = inr && bok;
          const uint32_t code = (ok && v) ? (uint32_t)(sm + (int)kRadius) : 0u;
          const T r_out = ok ? r1 : xv;
          Pw[j][k] = r_out;
          cprev = r_out;
          Up = U1;
          const bool is_out = v && !ok;
          if (__builtin_expect(__ballot(is_out) != 0, 0)) {
            if (is_out) gbl(outl)[nout] = xv;
            nout += is_out ? 1u : 0u;
          }
          const bool z = v && code == kRadius;
          hot += (uint32_t)__popcll(__ballot(z));  // the same in every lane running the pass
          if (v) {
            if (ABFT) {
              s_dc += Wd<T>::sum(r_out);
              rs += code;
              rk += (uint32_t)k * code;
            }
            if (!z) {
              const uint32_t cb = code - hlo;
              if (cb < hw) atomicAdd(&hist[cb], 1u);
              else atomicAdd(w.hist + code, 1u);
            }
          }
          // pack the codes of 4 consecutive padded indices into 8 bytes
          constexpr int dummy_unused = 0;
          (void)dummy_unused;
          const int qp = j * B2 + k;  // index inside the plane (planes fill whole groups)
          if ((qp & 1) == 0) {
            if ((qp & 2) == 0) pk0 = code;
            else pk1 = code;
          } else {
            if ((qp & 2) == 0) pk0 |= code << 16;
            else pk1 |= code << 16;
          }
          if ((qp & 3) == 3) cbase[(uint64_t)((i * PL + qp) >> 2) * 64] = v2u32{pk0, pk1};
        }
        if (ABFT) {
          const uint32_t rowbase = ((uint32_t)i * n1 + (uint32_t)j) * n2;
          is_q += (uint64_t)rowbase * rs + rk;
          s_q += rs;
        }
#pragma unroll
        for (int k = 0; k < B2; k++) Sv[k] = rowold[k];
        row_fence(cprev, S2, Q2, s_dc, is_q, s_q, nout, mis_p, mis_r);
      }
    }
    w.meta[blk] = (nout << 1) | (is_reg ? 1u : 0u);
    T *cf = (T *)w.coef + 4 * blk;
    cf[0] = beta0;
    cf[1] = beta1;
    cf[2] = beta2;
    cf[3] = mu;
    if (ABFT) {
      w.sum_dc[blk] = s_dc;
      w.sum_q[blk] = s_q;
      w.isum_q[blk] = is_q;
      if (S1l != S2 || Q1l != Q2) why |= kWhyInput;
      if (mis_p) why |= kWhyPred;
      if (mis_r) why |= kWhyRecon;
      out.why = why;
      if (why) {
        out.S1 = stash[0];
        out.Q1 = stash[1];
      }
    }
  }
  return out;
}

// One lane's 2D block of B1 rows by B2 columns (the geometry's slowest axis
// has extent 1).  The same arithmetic as compress_lanes with ND == 2, but the
// block streams through registers a row at a time: rows are loaded one ahead
// in the first pass and two ahead in the prediction pass, which keeps the
// previous reconstructed row only, so a 16x16 block needs no more registers
// than a 6x6x6 one.
template <typename T, int B1, int B2, bool FULL, bool ABFT, bool WIDE, int MODE>
__device__ __forceinline__ LaneOut compress_rows(const T *__restrict__ in, const Geo &g, const RegTab<T> &rt,
                                                 const PlanDev &plan, const CompWork &w, uint32_t predictor,
                                                 uint32_t *hist, uint32_t hlo, uint32_t hw, uint32_t &hot,
                                                 uint64_t blk, bool active, uint64_t *stash) {
  static_assert(B2 % 4 == 0, "a row must fill whole 4-code groups");
  // FP32 keeps the sampled values in registers; FP64 reads them again
  // (from cache) for the regression cost
  constexpr int NS = sizeof(T) == 4 ? sample_slot<2, 1, B1, B2>(1, 0, 0) : 0;
  constexpr uint32_t per = Wd<T>::per;
  const Box bx = box_of(g, blk);
  const uint64_t org = fidx(g, bx, 0, 0, 0);
  const uint64_t org0 = WIDE ? 0 : wave_min(org);
  // below 2 GiB: a wave-uniform base and 32-bit per-lane offsets; wider
  // fields: a per-lane base at the block's origin (32-bit offsets inside it)
  const char *wbase = WIDE ? (const char *)(in + org) : (const char *)(in + org0);
  const uint32_t loff = WIDE ? 0u : (uint32_t)((org - org0) * sizeof(T));
  // plan blocks: the fault-applying launch over the plan's list, or k_compress_wave_list
  if (MODE == kProd && active && plan_hit(plan, blk)) active = false;
  const LaneFaults lf = MODE == kFaults ? lane_faults(plan, blk, active) : LaneFaults{};
  LaneOut out{0, 0, 0};
  if (!active) return out;
  const EbDev eb = *w.eb;
  const T q = EbSel<T>::q(eb), inv = EbSel<T>::inv(eb), inv_e = EbSel<T>::inv_e(eb);
  const uint32_t n1 = FULL ? B1 : bx.n[1], n2 = FULL ? B2 : bx.n[2];
  const uint32_t pat = FULL ? 0 : bx.pat;
  const T c0 = rt.c[pat][0], c1 = rt.c[pat][1], c2 = rt.c[pat][2];
  const uint32_t RSB = (uint32_t)(g.d[2] * sizeof(T));
  auto valid = [&](int j, int k) -> bool { return FULL || ((uint32_t)j < n1 && (uint32_t)k < n2); };
  auto ld = [&](int j, int k) -> T {
    if (FULL) return *gbl((const T *)(wbase + (loff + (uint32_t)j * RSB) + k * sizeof(T)));
    const uint32_t jj = min((uint32_t)j, n1 - 1), kk = min((uint32_t)k, n2 - 1);
    const T v = *gbl((const T *)(wbase + (loff + jj * RSB + kk * (uint32_t)sizeof(T))));
    return valid(j, k) ? v : (T)0;
  };

  // ---- first pass: input checksums, regression sums, Lorenzo costs --------
  T xc[B2], xn[B2], xp[B2];  // rows j, j + 1 (in flight) and j - 1
  T sx[NS > 0 ? NS : 1];
  T D[B2];
  uint64_t S1 = 0, Q1 = 0;
  uint32_t e_lor = 0;
  T P = 0, A = 0;
#pragma unroll
  for (int k = 0; k < B2; k++) {
    xc[k] = ld(0, k);
    xp[k] = 0;
    D[k] = 0;
  }
#pragma unroll
  for (int j = 0; j < B1; j++) {
    if (j + 1 < B1) {
#pragma unroll
      for (int k = 0; k < B2; k++) xn[k] = ld(j + 1, k);
    }
    T R = 0;
#pragma unroll
    for (int k = 0; k < B2; k++) {
      if (valid(j, k)) {
        if (ABFT) Ck64<T>::add(xc[k], S1, Q1);
        R = R + xc[k];
        D[k] = D[k] + xc[k];
      }
      if (is_sample<2, 1, B1, B2>(0, j, k)) {
        // Lorenzo on the original values (zero outside the block)
        const T up = j > 0 ? xp[k] : (T)0, left = k > 0 ? xc[k - 1] : (T)0;
        const T diag = (j > 0 && k > 0) ? xp[k - 1] : (T)0;
        const T pl = (up + left) - diag;
        if (NS > 0) sx[sample_slot<2, 1, B1, B2>(0, j, k)] = xc[k];
        if (valid(j, k)) e_lor += cost<T>(xc[k] - pl, inv_e) + 1u;
      }
    }
    if (valid(j, 0)) {
      P = P + R;
      A = A + ((T)j - c1) * R;
    }
    row_fence(P, A, S1, Q1, e_lor);
#pragma unroll
    for (int k = 0; k < B2; k++) {
      pin(D[k]);
      xp[k] = xc[k];
      xc[k] = xn[k];
    }
  }
  T Bv = 0;
#pragma unroll
  for (int k = 0; k < B2; k++)
    if (valid(0, k)) Bv = Bv + ((T)k - c2) * D[k];
  // the slowest axis has one plane: its sums start from zero like the
  // paper-order routine's
  const T S0 = (T)0 + P, Sa1 = (T)0 + A, Sa2 = (T)0 + Bv;
  uint32_t S1l = 0, Q1l = 0;  // what the prediction pass compares with
  if (ABFT) {
    stash[0] = S1;
    stash[1] = Q1;
    S1l = (uint32_t)S1;
    Q1l = (uint32_t)Q1;
  }
  T beta0 = 0;
  T beta1 = n1 > 1 ? Sa1 * rt.K[pat][1] : (T)0;
  T beta2 = n2 > 1 ? Sa2 * rt.K[pat][2] : (T)0;
  T mu = S0 * rt.inv_pts[pat];
  uint64_t s_c = 0, i_c = 0;  // coefficient checksums, taken as they are computed
  if (ABFT) coef_sums<T>(beta0, beta1, beta2, mu, s_c, i_c);

  bool is_reg;
  if (predictor == SDCSZ_PRED_LORENZO) is_reg = false;
  else if (predictor == SDCSZ_PRED_REGRESSION) is_reg = true;
  else {
    uint32_t e_reg = 0;
#pragma unroll
    for (int j = 0; j < B1; j++)
#pragma unroll
      for (int k = 0; k < B2; k++) {
        if (!is_sample<2, 1, B1, B2>(0, j, k)) continue;
        const T pr = ((beta0 * ((T)0 - c0) + beta1 * ((T)j - c1)) + beta2 * ((T)k - c2)) + mu;
        const T xs = NS > 0 ? sx[NS > 0 ? sample_slot<2, 1, B1, B2>(0, j, k) : 0] : ld(j, k);
        if (valid(j, k)) e_reg += cost<T>(xs - pr, inv_e);
      }
    is_reg = e_reg <= e_lor;
  }

  uint64_t why = 0;
  if (MODE == kFaults && lf.cf != ~0u) {  // memory error in a coefficient after its checksums
    coef_flip<T>(beta0, beta1, beta2, mu, lf.cf & 0xFFFFu, 1u << ((lf.cf >> 16) & 31));
    count(w.cnt, C_INJ + SDCSZ_T_COEF);
  }
  if (ABFT) {  // verify (and repair) the coefficients as they are held now
    beta0 = launder(beta0);
    beta1 = launder(beta1);
    beta2 = launder(beta2);
    mu = launder(mu);
    const int st = coef_check<T>(beta0, beta1, beta2, mu, s_c, i_c);
    if (__builtin_expect(st != 0, 0)) {
      count(w.cnt, C_DET + SDCSZ_T_COEF);
      count(w.cnt, (st > 0 ? C_COR : C_UNC) + SDCSZ_T_COEF);
    }
  }

  // ---- prediction pass, a row per iteration --------------------------------
  const T beta0d = ABFT ? launder(beta0) : beta0, beta1d = ABFT ? launder(beta1) : beta1;
  const T beta2d = ABFT ? launder(beta2) : beta2;
  const T A0 = beta0 * ((T)0 - c0), A0d = beta0d * ((T)0 - c0);
  T Bk[B2], Bk2[B2], Pr[B2];  // Pr: reconstructed row j - 1
#pragma unroll
  for (int k = 0; k < B2; k++) {
    Bk[k] = beta2 * ((T)k - c2);
    Bk2[k] = beta2d * ((T)k - c2);
    Pr[k] = 0;
  }
  uint32_t S2 = 0, Q2 = 0;
  uint64_t s_dc = 0, is_q = 0;
  uint32_t s_q = 0, nout = 0;
  uint32_t mis_p = 0, mis_r = 0;
  T *outl = (T *)w.vals + blk * (uint64_t)g.bpts;
  const gptr<v2u32> cbase = gbl((v2u32 *)(w.codes + code_index(blk, 0, g.groups)));
  T xn1[B2], xn2[B2];  // the next two rows, loaded two rows ahead of their use
#pragma unroll
  for (int k = 0; k < B2; k++) {
    xn1[k] = ld(0, k);
    xn2[k] = ld(1, k);
  }
#pragma unroll 1
  for (int j = 0; j < B1; j++) {
    if (!FULL && (uint32_t)j >= n1) break;
    T Aj = A0 + beta1 * ((T)j - c1), Ajd = A0d + beta1d * ((T)j - c1);
    pin(Aj);
    if (ABFT) pin(Ajd);
    T xr[B2];
#pragma unroll
    for (int k = 0; k < B2; k++) {
      xr[k] = xn1[k];
      xn1[k] = xn2[k];
    }
    if (j + 2 < B1) {
#pragma unroll
      for (int k = 0; k < B2; k++) xn2[k] = ld(j + 2, k);
    }
    T cprev = 0, fold = 0;
    uint32_t rs = 0, rk = 0, pk0 = 0, pk1 = 0;
    const uint32_t prow = (uint32_t)j * n2;  // point index of the row's start
#pragma unroll
    for (int k = 0; k < B2; k++) {
      const bool v = valid(j, k);
      T xv = xr[k];
      if (MODE == kFaults && lf.wave_in) {  // the memory error the first pass did not see
        if (v && lf.in_w() / per == prow + k) {
          xv = word_xor(xv, lf.in_w() % per, lf.in_m());
          count(w.cnt, C_INJ + SDCSZ_T_INPUT);
        }
      }
      if (ABFT && v) Ck<T>::add(xv, S2, Q2);
      const T b = Pr[k], f = fold;  // r(j-1,k), r(j-1,k-1)
      fold = b;
      const T lor = (b + cprev) - f;
      const T reg = (Aj + Bk[k]) + mu;
      T pred = is_reg ? reg : lor;
      if (MODE == kFaults && lf.wave_dp) {  // flip of the first copy
        if (v && (lf.dp & 0xFFFFu) == prow + k) {
          pred = Wd<T>::flip(pred, lf.dp >> 16);
          count(w.cnt, C_INJ + SDCSZ_T_DUP_PRED);
        }
      }
      if (ABFT) {  // pred' <- f_dup()
        const T lor2 = (launder(b) + cprev) - f;
        const T reg2 = (Ajd + Bk2[k]) + mu;
        mis_p |= Wd<T>::diff(pred, is_reg ? reg2 : lor2);
      }
      const T diff = xv - pred;
      const T t = fabs(diff) * inv + (T)0.5;
      const bool inr = t < (T)32768;
      const int sm = (int)copysign(t, diff);
      T r1 = pred + (T)sm * q;
      if (MODE == kFaults && lf.wave_dr) {  // flip of the first copy (codes in range only)
        if (v && inr && (lf.dr & 0xFFFFu) == prow + k) {
          r1 = Wd<T>::flip(r1, lf.dr >> 16);
          count(w.cnt, C_INJ + SDCSZ_T_DUP_RECON);
        }
      }
      if (ABFT) mis_r |= Wd<T>::diff(r1, pred + (T)launder(sm) * q);  // dec_dup()
      const bool bok = Bound<T>::ok(xv, r1, eb);
      const bool ok = inr && bok;
      const uint32_t code = (ok && v) ? (uint32_t)(sm + (int)kRadius) : 0u;
      const T r_out = ok ? r1 : xv;
      Pr[k] = r_out;
      cprev = r_out;
      const bool is_out = v && !ok;
      if (__builtin_expect(__ballot(is_out) != 0, 0)) {
        if (is_out) gbl(outl)[nout] = xv;
        nout += is_out ? 1u : 0u;
      }
      const bool z = v && code == kRadius;
      hot += (uint32_t)__popcll(__ballot(z));
      if (v) {
        if (ABFT) {
          s_dc += Wd<T>::sum(r_out);
          rs += code;
          rk += (uint32_t)k * code;
        }
        if (!z) {
          const uint32_t cb = code - hlo;
          if (cb < hw) atomicAdd(&hist[cb], 1u);
          else atomicAdd(w.hist + code, 1u);
        }
      }
      if ((k & 1) == 0) {
        if ((k & 2) == 0) pk0 = code;
        else pk1 = code;
      } else {
        if ((k & 2) == 0) pk0 |= code << 16;
        else pk1 |= code << 16;
      }
      if ((k & 3) == 3) cbase[(uint64_t)((j * B2 + k) >> 2) * 64] = v2u32{pk0, pk1};
      // work in steps of 4 points (the duplicated computations of a whole
      // row at once would need twice the registers)
      if ((k & 3) == 3 && k + 1 < B2) row_fence(cprev, fold, S2, Q2, s_dc, rs, rk, nout, mis_p, mis_r);
    }
    if (ABFT) {
      is_q += (uint64_t)((uint32_t)j * n2) * rs + rk;
      s_q += rs;
    }
    row_fence(S2, Q2, s_dc, is_q, s_q, nout, mis_p, mis_r);
  }
  w.meta[blk] = (nout << 1) | (is_reg ? 1u : 0u);
  T *cf = (T *)w.coef + 4 * blk;
  cf[0] = beta0;
  cf[1] = beta1;
  cf[2] = beta2;
  cf[3] = mu;
  if (ABFT) {
    w.sum_dc[blk] = s_dc;
    w.sum_q[blk] = s_q;
    w.isum_q[blk] = is_q;
    if (S1l != S2 || Q1l != Q2) why |= kWhyInput;
    if (mis_p) why |= kWhyPred;
    if (mis_r) why |= kWhyRecon;
    out.why = why;
    if (why) {
      out.S1 = stash[0];
      out.Q1 = stash[1];
    }
  }
  return out;
}

// Queue a block whose checks disagreed, with its first-pass checksums.
__device__ inline void queue_redo(const CompWork &w, uint64_t blk, const LaneOut &o) {
  if (o.why & kWhyInput) count(w.cnt, C_DET + SDCSZ_T_INPUT);
  if (o.why & kWhyPred) count(w.cnt, C_DET + SDCSZ_T_DUP_PRED);
  if (o.why & kWhyRecon) count(w.cnt, C_DET + SDCSZ_T_DUP_RECON);
  const uint32_t slot = atomicAdd(w.redo_n, 1u);
  if (slot < kMaxRedo) {
    w.redo[3 * slot] = blk | (o.why << 56);
    w.redo[3 * slot + 1] = o.S1;
    w.redo[3 * slot + 2] = o.Q1;
  }
}

// Work-groups [0, L.full_wgs) of a job take its full blocks, the rest the
// partial shell.  PART 1 launches the full blocks' work-groups and PART 2 the
// shell's, numbered from 0 (the host runs them on two streams at once): in
// one kernel the two paths would share one register allocation, and the
// masked path's needs made the full-block path spill.
// FAULTS: the instantiation that applies the fault plan's flips, one lane
// per block of the plan's list (plan.flist) on the masked path.
template <typename T, int ND, int B0, int B1, int B2, bool ABFT, bool WIDE, bool FAULTS, int PART>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(ND == 3 && sizeof(T) == 4 ? (FAULTS ? 2 : 3) : 1)))
k_compress_fast(JobTab tab) {
  static_assert(FAULTS ? PART == 0 : (PART == 1 || PART == 2), "production launches take one part");
  const JobWg jw = job_of(tab);
  const T *__restrict__ in = (const T *)jw.J->src;
  const Geo g = jw.J->g;
  const RegTab<T> &rt = rt_of<T>(*jw.J);  // stays in memory: indexed by each block's pattern
  const PlanDev plan = jw.J->plan;
  const CompWork w = jw.J->cw;
  const uint32_t predictor = jw.J->predictor;
  const Launch L = jw.J->L;
  // LDS window of the histogram: hw codes centred on the zero residual
  // (wider for small bounds, whose codes spread further; the launch sizes
  // the dynamic LDS for the widest window of its jobs); the rest go to the
  // global histogram
  const uint32_t hw = jw.J->hist_win, hlo = kRadius - hw / 2;
  extern __shared__ uint32_t hist[];
  __shared__ uint64_t stash[2 * 256];  // first-pass input checksums, per lane
  for (uint32_t t = threadIdx.x; t < hw; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  uint32_t hot = 0;
  uint64_t *st = ABFT ? stash + 2 * threadIdx.x : nullptr;
  LaneOut o;
  uint64_t blk;
  if constexpr (FAULTS) {
    // a few blocks beside the production launch: their waves go first on
    // the SIMDs they share, so the launch ends with the production one
    __builtin_amdgcn_s_setprio(3);
    const uint32_t idx = jw.b * blockDim.x + threadIdx.x, nl = plan.nflist;
    const bool act = idx < nl;
    blk = plan.flist[act ? idx : nl - 1];
    if constexpr (ND == 2)
      o = compress_rows<T, B1, B2, false, ABFT, WIDE, kFaults>(in, g, rt, plan, w, predictor, hist, hlo, hw, hot, blk,
                                                               act, st);
    else
      o = compress_lanes<T, ND, B0, B1, B2, false, ABFT, WIDE, kFaults>(in, g, rt, plan, w, predictor, hist, hlo, hw,
                                                                        hot, blk, act, st);
  } else {
  constexpr bool full = PART == 1;
  const uint64_t idx = (uint64_t)jw.b * blockDim.x + threadIdx.x;
  const uint64_t nl = full ? L.full_count : L.shell_count;
  const bool act = idx < nl;
  blk = map_block(g, L, full ? 0u : 1u, act ? idx : nl - 1);
  constexpr int M = kProd;
  if constexpr (ND == 2) {
    static_assert(B0 == 1, "2D blocks have one plane");
    o = compress_rows<T, B1, B2, full, ABFT, WIDE, M>(in, g, rt, plan, w, predictor, hist, hlo, hw, hot, blk, act, st);
  } else {
    o = compress_lanes<T, ND, B0, B1, B2, full, ABFT, WIDE, M>(in, g, rt, plan, w, predictor, hist, hlo, hw, hot, blk,
                                                               act, st);
  }
  }
  if (ABFT && __builtin_expect(o.why != 0, 0)) queue_redo(w, blk, o);
  // wave total of the zero-residual bin (lanes that ran the pass agree; the
  // others hold 0), then flush the window
  for (int off = 32; off > 0; off >>= 1) hot = max(hot, (uint32_t)__shfl_xor((int)hot, off));
  if ((threadIdx.x & 63) == 0 && hot) atomicAdd(&hist[kRadius - hlo], hot);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < hw; t += blockDim.x)
    if (hist[t]) atomicAdd(w.hist + hlo + t, hist[t]);
}

#define SDCSZ_INST_FAST(T, ND, B0, B1, B2, ABFT, WIDE, FAULTS, PART) \
  template __global__ void k_compress_fast<T, ND, B0, B1, B2, ABFT, WIDE, FAULTS, PART>(JobTab);
#define SDCSZ_INST_PROD(T, ND, B0, B1, B2, ABFT, WIDE)        \
  SDCSZ_INST_FAST(T, ND, B0, B1, B2, ABFT, WIDE, false, 1) \
  SDCSZ_INST_FAST(T, ND, B0, B1, B2, ABFT, WIDE, false, 2)
#define SDCSZ_INST_SHAPE(T, ND, B0, B1, B2)          \
  SDCSZ_INST_PROD(T, ND, B0, B1, B2, true, false)   \
  SDCSZ_INST_PROD(T, ND, B0, B1, B2, false, false)  \
  SDCSZ_INST_PROD(T, ND, B0, B1, B2, true, true)    \
  SDCSZ_INST_PROD(T, ND, B0, B1, B2, false, true)   \
  SDCSZ_INST_FAST(T, ND, B0, B1, B2, true, false, true, 0) \
  SDCSZ_INST_FAST(T, ND, B0, B1, B2, false, false, true, 0)
SDCSZ_INST_SHAPE(float, 3, 6, 6, 6)
SDCSZ_INST_SHAPE(double, 3, 6, 6, 6)
SDCSZ_INST_SHAPE(float, 2, 1, 16, 16)
SDCSZ_INST_SHAPE(double, 2, 1, 16, 16)

}  // namespace sdcsz
