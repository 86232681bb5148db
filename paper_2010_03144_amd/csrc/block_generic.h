// block_generic.h -- Algorithm 1 for one block of any shape, one thread.
//
// Used by the shape-generic kernel and, for blocks named in a fault plan or
// after a detected mismatch, by the specialised kernels.
#pragma once

#include "dev.h"

namespace sdcsz {

// Value of point (i,j,k) of the block as the predictor reads it, with the
// block's fault patches (xor masks on words) and the ABFT repair applied.
template <typename T> struct BlockReader {
  const T *in;
  const Geo *g;
  const Box *b;
  uint32_t np;
  uint64_t pj[kMaxPatches];
  uint32_t pm[kMaxPatches];
  bool fixed;
  uint64_t fj;
  uint32_t fv;

  __device__ T raw(uint32_t i, uint32_t j, uint32_t k) const { return in[fidx(*g, *b, i, j, k)]; }
  __device__ T get(uint32_t p, uint32_t i, uint32_t j, uint32_t k) const {
    T x = raw(i, j, k);
    if (np == 0 && !fixed) return x;
    uint32_t w[2] = {0, 0};
    Wd<T>::split(x, w);
    for (uint32_t t = 0; t < np; t++)
      if (pj[t] / Wd<T>::per == p) w[pj[t] % Wd<T>::per] ^= pm[t];
    if (fixed && fj / Wd<T>::per == p) w[fj % Wd<T>::per] = fv;
    return Wd<T>::join(w);
  }
  __device__ uint32_t word(uint64_t jw) const {
    uint32_t p = (uint32_t)(jw / Wd<T>::per);
    uint32_t k = p % b->n[2], j = (p / b->n[2]) % b->n[1], i = p / (b->n[2] * b->n[1]);
    uint32_t w[2] = {0, 0};
    Wd<T>::split(get(p, i, j, k), w);
    return w[jw % Wd<T>::per];
  }
};

// The block's values as the regression and the sampling read them (through
// the reader: prediction-preparation input faults are visible there).
template <typename T> __device__ inline T prep_at(const BlockReader<T> &rd, const Box &b, uint32_t i, uint32_t j,
                                                  uint32_t k) {
  return rd.get((i * b.n[1] + j) * b.n[2] + k, i, j, k);
}

template <typename T>
__device__ void regression_generic(const BlockReader<T> &rd, const Box &b, const RegTab<T> &rt, T coef[4]) {
  const T *c = rt.c[b.pat];
  T S0 = 0, Sa0 = 0, Sa1 = 0, Sa2 = 0;
  for (uint32_t i = 0; i < b.n[0]; i++) {
    T P = 0, A = 0, B = 0;
    for (uint32_t j = 0; j < b.n[1]; j++) {
      T R = 0;
      for (uint32_t k = 0; k < b.n[2]; k++) R = R + prep_at(rd, b, i, j, k);
      P = P + R;
      A = A + ((T)j - c[1]) * R;
    }
    for (uint32_t k = 0; k < b.n[2]; k++) {
      T D = 0;
      for (uint32_t j = 0; j < b.n[1]; j++) D = D + prep_at(rd, b, i, j, k);
      B = B + ((T)k - c[2]) * D;
    }
    S0 = S0 + P;
    Sa0 = Sa0 + ((T)i - c[0]) * P;
    Sa1 = Sa1 + A;
    Sa2 = Sa2 + B;
  }
  coef[0] = b.n[0] > 1 ? Sa0 * rt.K[b.pat][0] : (T)0;
  coef[1] = b.n[1] > 1 ? Sa1 * rt.K[b.pat][1] : (T)0;
  coef[2] = b.n[2] > 1 ? Sa2 * rt.K[b.pat][2] : (T)0;
  coef[3] = S0 * rt.inv_pts[b.pat];
}

template <typename T>
__device__ inline T reg_pred(const T coef[4], const T *c, uint32_t i, uint32_t j, uint32_t k) {
  T w0 = (T)i - c[0], w1 = (T)j - c[1], w2 = (T)k - c[2];
  return ((coef[0] * w0 + coef[1] * w1) + coef[2] * w2) + coef[3];
}

// Lorenzo on values v (C order over the block's extents), zero outside.
template <typename T, typename F>
__device__ inline T lorenzo_gen(F at, uint32_t ndim, int i, int j, int k) {
  if (ndim == 1) return at(i, j, k - 1);
  if (ndim == 2) return (at(i, j - 1, k) + at(i, j, k - 1)) - at(i, j - 1, k - 1);
  T a = at(i - 1, j, k), b = at(i, j - 1, k), c = at(i, j, k - 1);
  T d = at(i - 1, j - 1, k), e = at(i - 1, j, k - 1), f = at(i, j - 1, k - 1);
  T g = at(i - 1, j - 1, k - 1);
  T u = (a + b) - d;
  T u_prev = (e + f) - g;
  return c + (u - u_prev);
}

template <typename T> __device__ inline uint32_t cost(T diff, T inv_e) {
  T t = fabs(diff) * inv_e;
  return t < (T)65536 ? (uint32_t)t : 65536u;
}


// One block of Algorithm 1 in the paper's order, for any block shape: first
// loop (coefficients, checksums), sampling, fault plan, detection and
// correction, then the per-point loop.  Reconstructed values go to the
// block's slot of the recon scratch area.
template <typename T>
__device__ __noinline__ void compress_block_generic(const T *__restrict__ in, const Geo &g, const RegTab<T> &rt,
                                                    const PlanDev &plan, const CompWork &w, uint32_t abft,
                                                    uint32_t predictor, uint64_t blk) {
  const Box b = box_of(g, blk);
  const EbDev eb = *w.eb;
  const T q = EbSel<T>::q(eb), inv = EbSel<T>::inv(eb), inv_e = EbSel<T>::inv_e(eb);
  const T *c = rt.c[b.pat];
  BlockReader<T> rd;
  rd.in = in;
  rd.g = &g;
  rd.b = &b;
  rd.np = 0;
  rd.fixed = false;
  const uint64_t nw = (uint64_t)b.pts * Wd<T>::per;

  // ---- prediction-preparation faults: input words flipped after the input
  // checksums (taken below from the memory as it was) but before the
  // regression and the sampling read them
  const bool hit = plan_hit(plan, blk);
  const uint32_t pfirst = hit ? plan_first(plan, blk) : 0;
  bool prep_in = false;
  if (hit)
    for (uint32_t t = pfirst; t < plan.n && plan.f[t].block == blk; t++)
      if (plan.f[t].target == SDCSZ_T_PREP_INPUT && rd.np < kMaxPatches) {
        rd.pj[rd.np] = plan.f[t].word;
        rd.pm[rd.np] = 1u << (plan.f[t].bit & 31);
        rd.np++;
        prep_in = true;
        count(w.cnt, C_INJ + SDCSZ_T_PREP_INPUT);
      }
  const int t_in = prep_in ? SDCSZ_T_PREP_INPUT : SDCSZ_T_INPUT;  // where a detection is counted

  // ---- first loop: regression coefficients + input/coefficient checksums
  T coef[4];
  regression_generic<T>(rd, b, rt, coef);
  if (hit)  // computation errors in the regression, before its checksums
    for (uint32_t t = pfirst; t < plan.n && plan.f[t].block == blk; t++)
      if (plan.f[t].target == SDCSZ_T_PREP_COEF) {
        uint32_t cw[8];
        for (int a = 0; a < 4; a++) Wd<T>::split(coef[a], cw + a * Wd<T>::per);
        cw[plan.f[t].word] ^= 1u << (plan.f[t].bit & 31);
        for (int a = 0; a < 4; a++) coef[a] = Wd<T>::join(cw + a * Wd<T>::per);
        count(w.cnt, C_INJ + SDCSZ_T_PREP_COEF);
      }
  uint64_t s_in = 0, is_in = 0, s_c = 0, is_c = 0;
  if (abft) {
    for (uint32_t i = 0, p = 0; i < b.n[0]; i++)
      for (uint32_t j = 0; j < b.n[1]; j++)
        for (uint32_t k = 0; k < b.n[2]; k++, p++) {
          uint32_t wv[2] = {0, 0};
          Wd<T>::split(rd.raw(i, j, k), wv);
          for (uint32_t t = 0; t < Wd<T>::per; t++) {
            uint64_t jw = (uint64_t)p * Wd<T>::per + t;
            s_in += wv[t];
            is_in += jw * wv[t];
          }
        }
    for (int a = 0; a < 4; a++) {
      uint32_t wv[2] = {0, 0};
      Wd<T>::split(coef[a], wv);
      for (uint32_t t = 0; t < Wd<T>::per; t++) {
        uint64_t jw = (uint64_t)a * Wd<T>::per + t;
        s_c += wv[t];
        is_c += jw * wv[t];
      }
    }
  }

  // ---- second loop: sampled selection
  bool is_reg;
  if (predictor == SDCSZ_PRED_LORENZO) is_reg = false;
  else if (predictor == SDCSZ_PRED_REGRESSION) is_reg = true;
  else {
    uint64_t e_lor = 0, e_reg = 0, ns = 0;
    auto orig = [&](int i, int j, int k) -> T {
      return (i < 0 || j < 0 || k < 0) ? (T)0 : prep_at(rd, b, (uint32_t)i, (uint32_t)j, (uint32_t)k);
    };
    auto sample = [&](uint32_t i, uint32_t j, uint32_t k) {
      T x = prep_at(rd, b, i, j, k);
      T pl = lorenzo_gen<T>(orig, g.ndim, (int)i, (int)j, (int)k);
      T pr = reg_pred<T>(coef, c, i, j, k);
      e_lor += cost<T>(x - pl, inv_e);
      e_reg += cost<T>(x - pr, inv_e);
      ns++;
    };
    // diagonals of the configured block, clipped to the block's extents
    auto inside = [&](uint32_t i, uint32_t j, uint32_t k) { return i < b.n[0] && j < b.n[1] && k < b.n[2]; };
    if (g.ndim == 1) {
      for (uint32_t k = 0; k < b.n[2]; k++) sample(0, 0, k);
    } else if (g.ndim == 2) {
      uint32_t m = min(g.b[1], g.b[2]);
      for (uint32_t t = 0; t < m; t++) {
        if (inside(0, t, t)) sample(0, t, t);
        uint32_t k2 = g.b[2] - 1 - t;
        if (k2 != t && inside(0, t, k2)) sample(0, t, k2);
      }
    } else {
      uint32_t m = min(g.b[0], min(g.b[1], g.b[2]));
      for (uint32_t t = 0; t < m; t++) {
        uint32_t P[4][3] = {{t, t, t}, {t, t, g.b[2] - 1 - t}, {t, g.b[1] - 1 - t, t},
                            {g.b[0] - 1 - t, t, t}};
        for (int u = 0; u < 4; u++) {
          bool dup = !inside(P[u][0], P[u][1], P[u][2]);
          for (int v = 0; v < u; v++)
            if (P[u][0] == P[v][0] && P[u][1] == P[v][1] && P[u][2] == P[v][2]) dup = true;
          if (!dup) sample(P[u][0], P[u][1], P[u][2]);
        }
      }
    }
    e_lor += ns;
    if (hit)  // computation errors in the sampled estimates
      for (uint32_t t = pfirst; t < plan.n && plan.f[t].block == blk; t++)
        if (plan.f[t].target == SDCSZ_T_PREP_SAMPLE) {
          uint64_t &e = plan.f[t].word == 0 ? e_lor : e_reg;
          e ^= 1ull << (plan.f[t].bit & 63);
          count(w.cnt, C_INJ + SDCSZ_T_PREP_SAMPLE);
        }
    is_reg = e_reg <= e_lor;
  }

  // ---- mode-A memory errors after the checksums: input and coefficients
  bool dp = false, dr = false;
  if (plan_hit(plan, blk)) {
    for (uint32_t t = plan_first(plan, blk); t < plan.n && plan.f[t].block == blk; t++) {
      const sdcsz_fault f = plan.f[t];
      if (f.target == SDCSZ_T_INPUT) {
        if (rd.np < kMaxPatches) {
          rd.pj[rd.np] = f.word;
          rd.pm[rd.np] = 1u << (f.bit & 31);
          rd.np++;
        }
        count(w.cnt, C_INJ + SDCSZ_T_INPUT);
      } else if (f.target == SDCSZ_T_COEF) {
        uint32_t cw[8];
        for (int a = 0; a < 4; a++) Wd<T>::split(coef[a], cw + a * Wd<T>::per);
        cw[f.word] ^= 1u << (f.bit & 31);
        for (int a = 0; a < 4; a++) coef[a] = Wd<T>::join(cw + a * Wd<T>::per);
        count(w.cnt, C_INJ + SDCSZ_T_COEF);
      } else if (f.target == SDCSZ_T_DUP_PRED) {
        dp = true;
      } else if (f.target == SDCSZ_T_DUP_RECON) {
        dr = true;
      }
    }
  }

  // ---- third loop: detect/correct input and coefficients
  bool bad = false;
  if (abft) {
    uint64_t s2 = 0, i2 = 0;
    for (uint64_t jw = 0; jw < nw; jw++) {
      uint32_t v = rd.word(jw);
      s2 += v;
      i2 += jw * v;
    }
    uint64_t jf;
    uint32_t vf;
    int st = locate_repair(s2, i2, s_in, is_in, nw, 32, [&](uint64_t j) { return rd.word(j); }, &jf, &vf);
    if (st != 0) count(w.cnt, C_DET + t_in);
    if (st == 1) {
      rd.fixed = true;
      rd.fj = jf;
      rd.fv = vf;
      count(w.cnt, C_COR + t_in);
    }
    if (st < 0) {
      count(w.cnt, C_UNC + t_in);
      bad = true;
    }
    uint32_t cw[8];
    for (int a = 0; a < 4; a++) Wd<T>::split(coef[a], cw + a * Wd<T>::per);
    s2 = 0;
    i2 = 0;
    for (uint32_t jw = 0; jw < 4 * Wd<T>::per; jw++) {
      s2 += cw[jw];
      i2 += (uint64_t)jw * cw[jw];
    }
    st = locate_repair(s2, i2, s_c, is_c, 4 * Wd<T>::per, 32, [&](uint64_t j) { return cw[j]; }, &jf, &vf);
    if (st != 0) count(w.cnt, C_DET + SDCSZ_T_COEF);
    if (st == 1) {
      cw[jf] = vf;
      for (int a = 0; a < 4; a++) coef[a] = Wd<T>::join(cw + a * Wd<T>::per);
      count(w.cnt, C_COR + SDCSZ_T_COEF);
    }
    if (st < 0) {
      count(w.cnt, C_UNC + SDCSZ_T_COEF);
      bad = true;
    }
  }
  (void)bad;

  // ---- per-point prediction, quantization, reconstruction, double check
  const uint64_t base = blk * (uint64_t)g.bpts;
  const Slot<T> rec = slot_of<T>(w.recon, blk, g.bpts);
  T *outl = (T *)w.vals + base;
  auto rat = [&](int i, int j, int k) -> T {
    return (i < 0 || j < 0 || k < 0) ? (T)0 : rec[((uint32_t)i * b.n[1] + (uint32_t)j) * b.n[2] + (uint32_t)k];
  };
  uint64_t s_dc = 0, s_q = 0, is_q = 0;
  uint32_t nout = 0;
  uint32_t fbeg = (dp || dr) ? plan_first(plan, blk) : 0;
  for (uint32_t i = 0, p = 0; i < b.n[0]; i++)
    for (uint32_t j = 0; j < b.n[1]; j++)
      for (uint32_t k = 0; k < b.n[2]; k++, p++) {
        const T x = rd.get(p, i, j, k);
        T pred = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
        if (dp)
          for (uint32_t t = fbeg; t < plan.n && plan.f[t].block == blk; t++)
            if (plan.f[t].target == SDCSZ_T_DUP_PRED && plan.f[t].word == p) {
              pred = Wd<T>::flip(pred, plan.f[t].bit);
              count(w.cnt, C_INJ + SDCSZ_T_DUP_PRED);
            }
        if (abft) {
          __asm__ volatile("" ::: "memory");
          T pred2 = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
          if (!Wd<T>::same(pred, pred2)) {
            count(w.cnt, C_DET + SDCSZ_T_DUP_PRED);
            __asm__ volatile("" ::: "memory");
            T pred3 = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
            if (Wd<T>::same(pred3, pred2)) count(w.cnt, C_COR + SDCSZ_T_DUP_PRED);
            else count(w.cnt, C_UNC + SDCSZ_T_DUP_PRED);
            pred = Wd<T>::same(pred3, pred) ? pred : pred2;
          }
        }
        const T diff = x - pred;
        const T t = fabs(diff) * inv + (T)0.5;
        uint16_t code = 0;
        T r_out = x;
        if (t < (T)32768) {
          int m = (int)t;
          int sm = diff < (T)0 ? -m : m;
          T r = pred + (T)sm * q;
          if (dr)
            for (uint32_t u = fbeg; u < plan.n && plan.f[u].block == blk; u++)
              if (plan.f[u].target == SDCSZ_T_DUP_RECON && plan.f[u].word == p) {
                r = Wd<T>::flip(r, plan.f[u].bit);
                count(w.cnt, C_INJ + SDCSZ_T_DUP_RECON);
              }
          if (abft) {
            T smf = (T)sm, qq = q, pp = pred;
            __asm__ volatile("" : "+v"(smf), "+v"(qq), "+v"(pp));
            T r2 = pp + smf * qq;
            if (!Wd<T>::same(r, r2)) {
              count(w.cnt, C_DET + SDCSZ_T_DUP_RECON);
              __asm__ volatile("" : "+v"(smf), "+v"(qq), "+v"(pp));
              T r3 = pp + smf * qq;
              if (Wd<T>::same(r3, r2)) count(w.cnt, C_COR + SDCSZ_T_DUP_RECON);
              else count(w.cnt, C_UNC + SDCSZ_T_DUP_RECON);
              r = Wd<T>::same(r3, r) ? r : r2;
            }
          }
          if (fabs((double)x - (double)r) <= eb.eb_abs) {
            code = (uint16_t)(sm + (int)kRadius);
            r_out = r;
          }
        }
        w.codes[code_index(blk, padded_index(g, i, j, k), g.groups)] = code;
        rec[p] = r_out;
        if (code == 0) outl[nout++] = x;
        s_dc += Wd<T>::sum(r_out);
        s_q += code;
        is_q += (uint64_t)p * code;
        atomicAdd(w.hist + code, 1u);
      }
  w.meta[blk] = (nout << 1) | (is_reg ? 1u : 0u);
  T *cf = (T *)w.coef + 4 * blk;
  for (int a = 0; a < 4; a++) cf[a] = coef[a];
  w.sum_dc[blk] = s_dc;
  w.sum_q[blk] = s_q;
  w.isum_q[blk] = is_q;
}

}  // namespace sdcsz
