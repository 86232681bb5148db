// kern_wave.hip -- one wave per block: Algorithm 1 in the paper's order for
// any block shape, with the block staged in LDS.
//
// The 64 lanes of a wave share one block.  Work that is independent
// across points (loads, checksums, samples, regression prediction,
// quantization, stores) is spread over the lanes; the Lorenzo recursion runs
// along anti-diagonal fronts (points with i + j + k = s depend only on
// smaller s), so the lanes take a front's points together.  Every
// floating-point value is computed with the operations, operands and order
// of the one-thread-per-block routine (compress_block_generic): the
// regression's row, column and plane sums are sequential chains, each run by
// one lane; integer sums (checksums, costs) are reduced across the wave.
//
// It serves block shapes without a lane-per-block kernel, the fault-plan
// blocks those kernels leave, and the re-execution of the blocks they queue
// (the input verified and repaired against their first-pass checksums).
#include "block_generic.h"
#include "kern.h"

namespace sdcsz {

namespace {

constexpr uint32_t kWL = 64;  // lanes of a wave

// The wave's LDS writes are seen by its later LDS reads (the waves of a
// work-group work on different blocks, so they never wait for each other).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint64_t wave_sum(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, off);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), off);
    v += ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// plan entries of a block that strike its points during prediction
struct DupEntry {
  uint32_t target, point, bit;
};

}  // namespace

// LDS of one block: values (C order over the block's extents), reconstructed
// values (the regression's partial sums before that) and one outlier bit per
// point.  rsz: max(points, rows + columns + 3 planes) of the configured block.
template <typename T> struct WaveLds {
  T *x, *r;
  uint32_t *ob;
  DupEntry *dup;  // kMaxPatches entries
};

// What one block's pass found: the state of the input after verification
// (0 clean, 1 repaired, -1 uncorrectable).
struct WaveRes {
  int st_in;
};

// One block through Algorithm 1 by one wave.  redo: the block was queued by
// a lane-per-block kernel; `pre` holds its first-pass input checksums (sum,
// isum), the plan's INPUT flips (memory errors, which persist) are applied
// to the values read, and the input is verified and repaired against `pre`
// before the regression; no other flip is applied and nothing is counted
// (the caller counts).  Every lane of the wave calls it with the same block.
// Codes within [hlo, hlo + hw) are counted in the LDS histogram `hist` (the
// work-group flushes it), the others in the global one (hist null: all).
template <typename T>
__device__ WaveRes compress_block_wave(const T *__restrict__ in, const Geo &g, const RegTab<T> &rt,
                                       const PlanDev &plan, const CompWork &w, uint32_t abft, uint32_t predictor,
                                       uint64_t blk, const WaveLds<T> &L, bool redo, const uint64_t *pre,
                                       uint32_t *hist, uint32_t hlo, uint32_t hw) {
  constexpr uint32_t per = Wd<T>::per;
  const uint32_t l = threadIdx.x & (kWL - 1);
  const Box b = box_of(g, blk);
  const uint32_t n0 = b.n[0], n1 = b.n[1], n2 = b.n[2], pts = b.pts;
  const uint64_t nw = (uint64_t)pts * per;
  const EbDev eb = *w.eb;
  const T q = EbSel<T>::q(eb), inv = EbSel<T>::inv(eb), inv_e = EbSel<T>::inv_e(eb);
  const T *c = rt.c[b.pat];
  T *x = L.x, *r = L.r;
  const bool lead = l == 0;
  WaveRes res{0};

  // ---- the block's plan entries (the same in every lane)
  const bool hit = plan_hit(plan, blk);
  const uint32_t pf = hit ? plan_first(plan, blk) : 0;
  uint32_t ndup = 0;
  bool prep_in = false;
  if (hit && !redo)
    for (uint32_t t = pf; t < plan.n && plan.f[t].block == blk; t++) {
      const sdcsz_fault f = plan.f[t];
      if ((f.target == SDCSZ_T_DUP_PRED || f.target == SDCSZ_T_DUP_RECON) && ndup < kMaxPatches) {
        if (lead) L.dup[ndup] = DupEntry{f.target, (uint32_t)f.word, f.bit};
        ndup++;
      }
      prep_in |= f.target == SDCSZ_T_PREP_INPUT;
    }
  const int t_in = prep_in ? SDCSZ_T_PREP_INPUT : SDCSZ_T_INPUT;  // where an input detection is counted

  // ---- load, input checksums (the first loop's, from memory as it is)
  uint64_t s = 0, is = 0;
  for (uint32_t p = l; p < pts; p += kWL) {
    const uint32_t k = p % n2, j = (p / n2) % n1, i = p / (n2 * n1);
    const T v = in[fidx(g, b, i, j, k)];
    x[p] = v;
    if (abft && !redo) {
      uint32_t wv[2] = {0, 0};
      Wd<T>::split(v, wv);
      for (uint32_t h = 0; h < per; h++) {
        s += wv[h];
        is += ((uint64_t)p * per + h) * wv[h];
      }
    }
  }
  for (uint32_t t = l; t < (pts + 31) / 32; t += kWL) L.ob[t] = 0;
  const uint64_t s_in = redo ? pre[0] : wave_sum(s), is_in = redo ? pre[1] : wave_sum(is);
  wave_sync();

  // flips of input words that persist in memory until the input is checked
  auto flip_x = [&](uint32_t tgt) {
    if (!hit) return;
    for (uint32_t t = pf; t < plan.n && plan.f[t].block == blk; t++) {
      const sdcsz_fault f = plan.f[t];
      if (f.target != tgt) continue;
      if (lead) {
        uint32_t wv[2] = {0, 0};
        Wd<T>::split(x[f.word / per], wv);
        wv[f.word % per] ^= 1u << (f.bit & 31);
        x[f.word / per] = Wd<T>::join(wv);
        if (!redo) count(w.cnt, C_INJ + tgt);
      }
    }
    wave_sync();
  };
  // verification and repair of the input against (s_in, is_in)
  auto verify_input = [&]() -> int {
    uint64_t s2 = 0, i2 = 0;
    for (uint32_t p = l; p < pts; p += kWL) {
      uint32_t wv[2] = {0, 0};
      Wd<T>::split(x[p], wv);
      for (uint32_t h = 0; h < per; h++) {
        s2 += wv[h];
        i2 += ((uint64_t)p * per + h) * wv[h];
      }
    }
    s2 = wave_sum(s2);
    i2 = wave_sum(i2);
    uint64_t jf = 0;
    uint32_t vf = 0;
    const int st = locate_repair(s2, i2, s_in, is_in, nw, 32, [&](uint64_t jw) {
      uint32_t wv[2] = {0, 0};
      Wd<T>::split(x[jw / per], wv);
      return wv[jw % per];
    }, &jf, &vf);
    wave_sync();  // every lane has read the word before it is repaired
    if (st == 1 && lead) {
      uint32_t wv[2] = {0, 0};
      Wd<T>::split(x[jf / per], wv);
      wv[jf % per] = vf;
      x[jf / per] = Wd<T>::join(wv);
    }
    wave_sync();
    return st;
  };

  if (redo) {
    flip_x(SDCSZ_T_INPUT);
    res.st_in = verify_input();
    if (res.st_in < 0) return res;  // the block keeps the queued pass's results
    // the codes the queued pass counted leave the histogram
    for (uint32_t p = l; p < pts; p += kWL) {
      const uint32_t k = p % n2, j = (p / n2) % n1, i = p / (n2 * n1);
      atomicSub(w.hist + w.codes[code_index(blk, padded_index(g, i, j, k), g.groups)], 1u);
    }
  } else {
    flip_x(SDCSZ_T_PREP_INPUT);  // errors in the prediction preparation
  }

  // ---- regression: row sums, column sums and plane sums, each a
  // sequential chain in the paper-order routine's order
  T *R = r, *D = r + n0 * n1, *PAB = D + n0 * n2;
  for (uint32_t u = l; u < n0 * n1; u += kWL) {
    const uint32_t i = u / n1, j = u % n1;
    T sr = 0;
    for (uint32_t k = 0; k < n2; k++) sr = sr + x[(i * n1 + j) * n2 + k];
    R[u] = sr;
  }
  for (uint32_t u = l; u < n0 * n2; u += kWL) {
    const uint32_t i = u / n2, k = u % n2;
    T sd = 0;
    for (uint32_t j = 0; j < n1; j++) sd = sd + x[(i * n1 + j) * n2 + k];
    D[u] = sd;
  }
  wave_sync();
  for (uint32_t i = l; i < n0; i += kWL) {
    T P = 0, A = 0, Bv = 0;
    for (uint32_t j = 0; j < n1; j++) {
      const T Rv = R[i * n1 + j];
      P = P + Rv;
      A = A + ((T)j - c[1]) * Rv;
    }
    for (uint32_t k = 0; k < n2; k++) Bv = Bv + ((T)k - c[2]) * D[i * n2 + k];
    PAB[3 * i] = P;
    PAB[3 * i + 1] = A;
    PAB[3 * i + 2] = Bv;
  }
  wave_sync();
  T S0 = 0, Sa0 = 0, Sa1 = 0, Sa2 = 0;
  for (uint32_t i = 0; i < n0; i++) {
    const T P = PAB[3 * i];
    S0 = S0 + P;
    Sa0 = Sa0 + ((T)i - c[0]) * P;
    Sa1 = Sa1 + PAB[3 * i + 1];
    Sa2 = Sa2 + PAB[3 * i + 2];
  }
  T coef[4];
  coef[0] = n0 > 1 ? Sa0 * rt.K[b.pat][0] : (T)0;
  coef[1] = n1 > 1 ? Sa1 * rt.K[b.pat][1] : (T)0;
  coef[2] = n2 > 1 ? Sa2 * rt.K[b.pat][2] : (T)0;
  coef[3] = S0 * rt.inv_pts[b.pat];
  wave_sync();  // the partial sums' area becomes the reconstruction
  auto flip_coef = [&](uint32_t tgt) {
    if (!hit || redo) return;
    for (uint32_t t = pf; t < plan.n && plan.f[t].block == blk; t++) {
      const sdcsz_fault f = plan.f[t];
      if (f.target != tgt) continue;
      uint32_t cw[8];
      for (int a = 0; a < 4; a++) Wd<T>::split(coef[a], cw + a * per);
      cw[f.word] ^= 1u << (f.bit & 31);
      for (int a = 0; a < 4; a++) coef[a] = Wd<T>::join(cw + a * per);
      if (lead) count(w.cnt, C_INJ + tgt);
    }
  };
  flip_coef(SDCSZ_T_PREP_COEF);  // computation errors before the checksums
  uint64_t s_c = 0, is_c = 0;
  if (abft) {
    uint32_t cw[8];
    for (int a = 0; a < 4; a++) Wd<T>::split(coef[a], cw + a * per);
    for (uint32_t jw = 0; jw < 4 * per; jw++) {
      s_c += cw[jw];
      is_c += (uint64_t)jw * cw[jw];
    }
  }

  // ---- sampled selection (diagonals of the configured block, clipped)
  bool is_reg;
  if (predictor == SDCSZ_PRED_LORENZO) is_reg = false;
  else if (predictor == SDCSZ_PRED_REGRESSION) is_reg = true;
  else {
    auto orig = [&](int i, int j, int k) -> T {
      return (i < 0 || j < 0 || k < 0) ? (T)0 : x[((uint32_t)i * n1 + (uint32_t)j) * n2 + (uint32_t)k];
    };
    auto inside = [&](uint32_t i, uint32_t j, uint32_t k) { return i < n0 && j < n1 && k < n2; };
    uint64_t e_lor = 0, e_reg = 0, ns = 0;
    uint32_t ncand;
    if (g.ndim == 1) ncand = n2;
    else if (g.ndim == 2) ncand = 2 * min(g.b[1], g.b[2]);
    else ncand = 4 * min(g.b[0], min(g.b[1], g.b[2]));
    for (uint32_t u = l; u < ncand; u += kWL) {
      uint32_t i = 0, j = 0, k = 0;
      bool use;
      if (g.ndim == 1) {
        k = u;
        use = true;
      } else if (g.ndim == 2) {
        const uint32_t t = u / 2;
        j = t;
        k = (u & 1) ? g.b[2] - 1 - t : t;
        use = ((u & 1) == 0 || k != t) && inside(0, j, k);
      } else {
        const uint32_t t = u / 4, a = u % 4;
        const uint32_t P[4][3] = {{t, t, t}, {t, t, g.b[2] - 1 - t}, {t, g.b[1] - 1 - t, t}, {g.b[0] - 1 - t, t, t}};
        i = P[a][0];
        j = P[a][1];
        k = P[a][2];
        use = inside(i, j, k);
        for (uint32_t v = 0; v < a; v++)
          if (P[v][0] == i && P[v][1] == j && P[v][2] == k) use = false;
      }
      if (use) {
        const T xs = x[(i * n1 + j) * n2 + k];
        const T pl = lorenzo_gen<T>(orig, g.ndim, (int)i, (int)j, (int)k);
        const T pr = reg_pred<T>(coef, c, i, j, k);
        e_lor += cost<T>(xs - pl, inv_e);
        e_reg += cost<T>(xs - pr, inv_e);
        ns++;
      }
    }
    e_lor = wave_sum(e_lor) + wave_sum(ns);
    e_reg = wave_sum(e_reg);
    if (hit && !redo)  // computation errors in the sampled estimates
      for (uint32_t t = pf; t < plan.n && plan.f[t].block == blk; t++)
        if (plan.f[t].target == SDCSZ_T_PREP_SAMPLE) {
          uint64_t &e = plan.f[t].word == 0 ? e_lor : e_reg;
          e ^= 1ull << (plan.f[t].bit & 63);
          if (lead) count(w.cnt, C_INJ + SDCSZ_T_PREP_SAMPLE);
        }
    is_reg = e_reg <= e_lor;
  }

  // ---- mode-A memory errors after the checksums, then detection and
  // correction of the input and the coefficients
  if (!redo) {
    flip_x(SDCSZ_T_INPUT);
    flip_coef(SDCSZ_T_COEF);
    if (abft) {
      const int st = verify_input();
      if (lead) {
        if (st != 0) count(w.cnt, C_DET + t_in);
        if (st == 1) count(w.cnt, C_COR + t_in);
        if (st < 0) count(w.cnt, C_UNC + t_in);
      }
      res.st_in = st;
    }
  }
  if (abft) {
    uint32_t cw[8];
    for (int a = 0; a < 4; a++) Wd<T>::split(coef[a], cw + a * per);
    uint64_t s2 = 0, i2 = 0;
    for (uint32_t jw = 0; jw < 4 * per; jw++) {
      s2 += cw[jw];
      i2 += (uint64_t)jw * cw[jw];
    }
    uint64_t jf;
    uint32_t vf;
    const int st = locate_repair(s2, i2, s_c, is_c, 4 * per, 32, [&](uint64_t j) { return cw[j]; }, &jf, &vf);
    if (lead && !redo) {
      if (st != 0) count(w.cnt, C_DET + SDCSZ_T_COEF);
      if (st == 1) count(w.cnt, C_COR + SDCSZ_T_COEF);
      if (st < 0) count(w.cnt, C_UNC + SDCSZ_T_COEF);
    }
    if (st == 1) {
      cw[jf] = vf;
      for (int a = 0; a < 4; a++) coef[a] = Wd<T>::join(cw + a * per);
    }
  }

  // ---- per-point prediction, quantization, reconstruction, double check
  const uint64_t base = blk * (uint64_t)g.bpts;
  T *outl = (T *)w.vals + base;
  auto rat = [&](int i, int j, int k) -> T {
    return (i < 0 || j < 0 || k < 0) ? (T)0 : r[((uint32_t)i * n1 + (uint32_t)j) * n2 + (uint32_t)k];
  };
  uint64_t s_dc = 0, s_q = 0, is_q = 0;
  auto point = [&](uint32_t i, uint32_t j, uint32_t k, bool on) {
    const uint32_t p = (i * n1 + j) * n2 + k;
    uint32_t code = 0;
    if (on) {
      const T xv = x[p];
      T pred = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
      for (uint32_t e = 0; e < ndup; e++)
        if (L.dup[e].target == SDCSZ_T_DUP_PRED && L.dup[e].point == p) {
          pred = Wd<T>::flip(pred, L.dup[e].bit);
          count(w.cnt, C_INJ + SDCSZ_T_DUP_PRED);
        }
      if (abft) {
        __asm__ volatile("" ::: "memory");
        T pred2 = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
        if (!Wd<T>::same(pred, pred2)) {
          count(w.cnt, C_DET + SDCSZ_T_DUP_PRED);
          __asm__ volatile("" ::: "memory");
          T pred3 = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
          count(w.cnt, (Wd<T>::same(pred3, pred2) ? C_COR : C_UNC) + SDCSZ_T_DUP_PRED);
          pred = Wd<T>::same(pred3, pred) ? pred : pred2;
        }
      }
      const T diff = xv - pred;
      const T t = fabs(diff) * inv + (T)0.5;
      T r_out = xv;
      if (t < (T)32768) {
        const int m = (int)t;
        const int sm = diff < (T)0 ? -m : m;
        T rr = pred + (T)sm * q;
        for (uint32_t e = 0; e < ndup; e++)
          if (L.dup[e].target == SDCSZ_T_DUP_RECON && L.dup[e].point == p) {
            rr = Wd<T>::flip(rr, L.dup[e].bit);
            count(w.cnt, C_INJ + SDCSZ_T_DUP_RECON);
          }
        if (abft) {
          T smf = (T)sm, qq = q, pp = pred;
          __asm__ volatile("" : "+v"(smf), "+v"(qq), "+v"(pp));
          const T r2 = pp + smf * qq;
          if (!Wd<T>::same(rr, r2)) {
            count(w.cnt, C_DET + SDCSZ_T_DUP_RECON);
            __asm__ volatile("" : "+v"(smf), "+v"(qq), "+v"(pp));
            const T r3 = pp + smf * qq;
            count(w.cnt, (Wd<T>::same(r3, r2) ? C_COR : C_UNC) + SDCSZ_T_DUP_RECON);
            rr = Wd<T>::same(r3, rr) ? rr : r2;
          }
        }
        if (fabs((double)xv - (double)rr) <= eb.eb_abs) {
          code = (uint32_t)(sm + (int)kRadius);
          r_out = rr;
        }
      }
      r[p] = r_out;
      w.codes[code_index(blk, padded_index(g, i, j, k), g.groups)] = (uint16_t)code;
      if (code == 0) atomicOr(&L.ob[p >> 5], 1u << (p & 31));
      s_dc += Wd<T>::sum(r_out);
      s_q += code;
      is_q += (uint64_t)p * code;
    }
    // the zero residual's bin once per wave, the others per point
    const bool z = on && code == kRadius;
    const uint32_t nz = (uint32_t)__popcll(__ballot(z));
    if (lead && nz) {
      if (hist && kRadius - hlo < hw) atomicAdd(&hist[kRadius - hlo], nz);
      else atomicAdd(w.hist + kRadius, nz);
    }
    if (on && !z) {
      if (hist && code - hlo < hw) atomicAdd(&hist[code - hlo], 1u);
      else atomicAdd(w.hist + code, 1u);
    }
  };
  if (is_reg) {
    for (uint32_t p0 = 0; p0 < pts; p0 += kWL) {
      const uint32_t p = p0 + l;
      const uint32_t k = p % n2, j = (p / n2) % n1, i = p / (n2 * n1);
      point(i, j, k, p < pts);
    }
  } else {
    // anti-diagonal fronts: every neighbour of a point lies on an earlier one
    const uint32_t fronts = n0 + n1 + n2 - 2;
    for (uint32_t s = 0; s < fronts; s++) {
      for (uint32_t u0 = 0; u0 < n0 * n1; u0 += kWL) {
        const uint32_t u = u0 + l, i = u / n1, j = u % n1;
        const int k = (int)s - (int)i - (int)j;
        point(i, j, (uint32_t)k, u < n0 * n1 && k >= 0 && k < (int)n2);
      }
      wave_sync();
    }
  }
  wave_sync();
  s_dc = wave_sum(s_dc);
  s_q = wave_sum(s_q);
  is_q = wave_sum(is_q);

  // ---- outliers in C order, the block's table entry, coefficients, sums
  uint32_t nout = 0;
  for (uint32_t p0 = 0; p0 < pts; p0 += kWL) {
    const uint32_t p = p0 + l;
    const bool o = p < pts && ((L.ob[p >> 5] >> (p & 31)) & 1u);
    const uint64_t m = __ballot(o);
    if (o) outl[nout + (uint32_t)__popcll(m & ((1ull << l) - 1))] = x[p];
    nout += (uint32_t)__popcll(m);
  }
  if (lead) {
    w.meta[blk] = (nout << 1) | (is_reg ? 1u : 0u);
    T *cf = (T *)w.coef + 4 * blk;
    for (int a = 0; a < 4; a++) cf[a] = coef[a];
    w.sum_dc[blk] = s_dc;
    w.sum_q[blk] = s_q;
    w.isum_q[blk] = is_q;
  }
  wave_sync();
  return res;
}

// LDS slice of a wave's block (wave_lds_bytes() of dynamic LDS each: 2 * rsz
// values, the outlier bits, the plan's duplicated-computation entries).
template <typename T> __device__ inline WaveLds<T> wave_lds(uint8_t *lds, uint32_t rsz) {
  WaveLds<T> L;
  L.x = (T *)lds;
  L.r = L.x + rsz;
  L.ob = (uint32_t *)(L.r + rsz);
  L.dup = (DupEntry *)(L.ob + (rsz + 31) / 32);
  static_assert(sizeof(DupEntry) <= kWaveDupBytes, "LDS of the plan entries");
  return L;
}

// Every block of a field (block shapes without a lane-per-block kernel),
// fault plans applied: blockDim.x / 64 waves per work-group, each taking
// blocks in turn, and the work-group's LDS histogram window (hist_win codes
// around the zero residual) flushed once at its end.  Dynamic LDS: the
// waves' block slices (slice bytes each, at least wave_slice_bytes), then
// the window.
template <typename T> __global__ void __launch_bounds__(256) k_compress_wave(JobTab tab, uint32_t slice) {
  const JobWg jw = job_of(tab);
  const Job &J = *jw.J;
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t nwv = blockDim.x >> 6, wv = threadIdx.x >> 6;
  const WaveLds<T> L = wave_lds<T>(lds + wv * slice, wave_rsz(J.g));
  uint32_t *hist = (uint32_t *)(lds + nwv * slice);
  const uint32_t hw = J.hist_win, hlo = kRadius - hw / 2;
  for (uint32_t t = threadIdx.x; t < hw; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const uint64_t step = (uint64_t)jw.nb * nwv;
  for (uint64_t blk = (uint64_t)jw.b * nwv + wv; blk < J.g.n_blocks; blk += step)
    compress_block_wave<T>((const T *)J.src, J.g, rt_of<T>(J), J.plan, J.cw, J.abft, J.predictor, blk, L, false,
                           nullptr, hist, hlo, hw);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < hw; t += blockDim.x)
    if (hist[t]) atomicAdd(J.cw.hist + hlo + t, hist[t]);
}

// The fault-plan blocks a lane-per-block kernel leaves (its list).
template <typename T> __global__ void __launch_bounds__(64) k_compress_wave_list(JobTab tab) {
  const JobWg jw = job_of(tab);
  const Job &J = *jw.J;
  extern __shared__ __align__(16) uint8_t lds[];
  const WaveLds<T> L = wave_lds<T>(lds, wave_rsz(J.g));
  compress_block_wave<T>((const T *)J.src, J.g, rt_of<T>(J), J.plan, J.cw, J.abft, J.predictor,
                         J.plan.list[jw.b], L, false, nullptr, nullptr, 0, 0);
  if (threadIdx.x == 0) count(J.cw.cnt, C_LIST);
}

// Re-execution of the blocks a lane-per-block kernel queued (Algorithm 1's
// correction at block granularity): the block's codes leave the histogram,
// then it runs again with its input verified and repaired against the
// first-pass checksums of the queue entry (an input word that cannot be
// located is uncorrectable, and the block keeps its first results).  One
// work-group per entry at a time.
template <typename T> __global__ void __launch_bounds__(64) k_redo_wave(JobTab tab) {
  const JobWg jw = job_of(tab);
  const Job &J = *jw.J;
  const CompWork &w = J.cw;
  if (!J.abft) return;
  const uint32_t n = min(*w.redo_n, kMaxRedo);
  if (jw.b >= n) return;
  extern __shared__ __align__(16) uint8_t lds[];
  const WaveLds<T> L = wave_lds<T>(lds, wave_rsz(J.g));
  constexpr uint32_t per = Wd<T>::per;
  for (uint32_t e = jw.b; e < n; e += jw.nb) {
    const uint64_t ent = w.redo[3 * e];
    const uint64_t blk = ent & ((1ull << 56) - 1), why = ent >> 56;
    const Box b = box_of(J.g, blk);
    const uint64_t nw = (uint64_t)b.pts * per, S1 = w.redo[3 * e + 1], Q1 = w.redo[3 * e + 2];
    const uint64_t pre[2] = {S1, nw * S1 - Q1};  // sum and isum of the first pass
    const WaveRes r0 = compress_block_wave<T>((const T *)J.src, J.g, rt_of<T>(J), J.plan, w, 1, J.predictor, blk, L,
                                              true, pre, nullptr, 0, 0);
    if (threadIdx.x == 0) {
      const int slot = r0.st_in < 0 ? C_UNC : C_COR;  // reasons: 1 input, 4 prediction, 8 reconstruction
      if (why & 1) count(w.cnt, slot + SDCSZ_T_INPUT);
      if (why & 4) count(w.cnt, slot + SDCSZ_T_DUP_PRED);
      if (why & 8) count(w.cnt, slot + SDCSZ_T_DUP_RECON);
    }
  }
}

// ---------------------------------------------------------------------------
// Decompression of one block by one wave (Algorithm 2): the first lane
// decodes the block's codewords in order (the symbols go to LDS; outliers
// take their stored values at once), then the wave reconstructs by fronts
// (Lorenzo) or all points at once (regression) with the arithmetic of
// compression, stores, and compares the checksum with sum_dc; a mismatch
// decodes the block again from the stream.
// ---------------------------------------------------------------------------

// Decoding tables in LDS: the prefix table (a codeword's length and symbol
// from its first kLutBits bits, or the range of lengths of longer codes with
// that prefix) and the canonical first code, count and position per length;
// and a staging area for a block's payload words (a block of kMaxBlockPts
// points of 24-bit codewords fits; words beyond it are read from memory).
constexpr uint32_t kWavePayWords = kMaxBlockPts * kMaxLen / 32 + 2;
struct WaveDecTab {
  alignas(16) uint32_t lut[1u << kLutBits];
  uint32_t first[kMaxLen + 2], count[kMaxLen + 2], start[kMaxLen + 2];
  uint32_t pay[kWavePayWords];
};
__device__ inline void load_wave_tab(WaveDecTab &t, const DecWork &w) {
  // the prefix table 16 bytes per load, all of a lane's loads in flight together
  constexpr uint32_t kQ = (1u << kLutBits) / 4, kPerLane = kQ / kWL;
  static_assert(kPerLane * kWL == kQ, "prefix table quarter-words per lane");
  uint4 q[kPerLane];
#pragma unroll
  for (uint32_t u = 0; u < kPerLane; u++) q[u] = ((const uint4 *)w.lut)[threadIdx.x + u * kWL];
#pragma unroll
  for (uint32_t u = 0; u < kPerLane; u++) ((uint4 *)t.lut)[threadIdx.x + u * kWL] = q[u];
  for (uint32_t v = threadIdx.x; v < kMaxLen + 2; v += blockDim.x) {
    t.first[v] = w.tab->first[v];
    t.count[v] = w.tab->count[v];
    t.start[v] = w.tab->start[v];
  }
  __syncthreads();
}

// Decode and reconstruct into L.r; false on an invalid code, a payload
// overrun or an outlier-count mismatch (the same in every lane).  Codewords
// are resolved as by bit-by-bit decoding: the shortest length whose codes
// hold the next bits.
template <typename T>
__device__ bool decode_block_wave(const uint8_t *__restrict__ s, const Header &h, const Geo &g, const DecWork &w,
                                  WaveDecTab &tab, uint64_t blk, const Box &b, const WaveLds<T> &L) {
  const uint32_t l = threadIdx.x;
  const uint32_t n0 = b.n[0], n1 = b.n[1], n2 = b.n[2], pts = b.pts;
  uint16_t *sym = (uint16_t *)L.x;  // the block's symbols
  T *r = L.r;
  const uint32_t meta = *(const uint32_t *)(s + h.off_table + 8 * blk + 4);
  const bool is_reg = meta & 1u;
  const uint32_t nout = meta >> 1;
  __shared__ uint32_t ok_s;
  const uint32_t *words = (const uint32_t *)(s + h.off_payload) + w.off_pay[blk];
  const uint64_t nwords = w.off_pay[blk + 1] - w.off_pay[blk], nbits = nwords * 32ull;
  // the payload into LDS, all lanes at once (the decoding is serial)
  const uint32_t nst = (uint32_t)min(nwords, (uint64_t)kWavePayWords);
  uint32_t *pay = tab.pay;
  for (uint32_t i = l; i < nst; i += kWL) pay[i] = words[i];
  __syncthreads();
  // a block's codewords take at most kMaxBlockPts * kMaxLen bits, so the
  // staged words hold every bit the decoding can reach; words past them
  // read as zeros (an LDS read, never a generic one)
  auto word = [&](uint64_t i) -> uint32_t { return i < nst ? pay[i] : 0u; };
  if (l == 0) {
    const T *outl = (const T *)(s + h.off_outliers) + w.off_out[blk];
    uint64_t pos = 0;
    uint32_t used = 0;
    bool ok = true;
    // 64 bits of the payload in a register, refilled a word at a time (zeros
    // past the block's words): the next 32 bits are buf's top after `sh`
    auto wd = [&](uint64_t i) -> uint64_t { return i < nwords ? word(i) : 0u; };
    uint64_t buf = (wd(0) << 32) | wd(1), nextw = 2;
    uint32_t sh = 0;
    for (uint32_t p = 0; p < pts && ok; p++) {
      const uint32_t win = (uint32_t)((buf << sh) >> 32);
      const uint32_t e = tab.lut[win >> (32 - kLutBits)];
      int sy = -1;
      uint32_t len = e & 0xFFu;
      if (len) {
        sy = (int)(e >> 8);
      } else {
        const uint32_t lmin = (e >> 8) & 0xFFu, lmax = e >> 16;
        for (uint32_t ln = lmin; ln && ln <= lmax; ln++) {
          const uint32_t cw = win >> (32 - ln);
          if (tab.count[ln] && cw >= tab.first[ln] && cw - tab.first[ln] < tab.count[ln]) {
            sy = w.symbols[tab.start[ln] + cw - tab.first[ln]];
            len = ln;
            break;
          }
        }
      }
      if (sy < 0 || pos + len > nbits) {
        ok = false;
        break;
      }
      pos += len;
      sh += len;
      if (sh >= 32) {
        buf = (buf << 32) | wd(nextw++);
        sh -= 32;
      }
      sym[p] = (uint16_t)sy;
      if (sy == 0) {
        if (used >= nout) {
          ok = false;
          break;
        }
        r[p] = outl[used++];
      }
    }
    ok_s = ok && used == nout;
  }
  __syncthreads();
  if (!ok_s) return false;
  const T q = (T)(2.0 * h.eb_abs);
  T coef[4] = {0, 0, 0, 0};
  if (is_reg) {
    const T *cp = (const T *)(s + h.off_coef) + 4ull * w.off_coef[blk];
    for (int a = 0; a < 4; a++) coef[a] = cp[a];
  }
  T c[3];
  for (int a = 0; a < 3; a++) c[a] = (T)(b.n[a] - 1) * (T)0.5;
  auto rat = [&](int i, int j, int k) -> T {
    return (i < 0 || j < 0 || k < 0) ? (T)0 : r[((uint32_t)i * n1 + (uint32_t)j) * n2 + (uint32_t)k];
  };
  auto point = [&](uint32_t i, uint32_t j, uint32_t k) {
    const uint32_t p = (i * n1 + j) * n2 + k;
    const uint32_t sy = sym[p];
    if (sy == 0) return;  // an outlier, already in place
    const T pred = is_reg ? reg_pred<T>(coef, c, i, j, k) : lorenzo_gen<T>(rat, g.ndim, (int)i, (int)j, (int)k);
    r[p] = pred + (T)((int)sy - (int)kRadius) * q;
  };
  if (is_reg) {
    for (uint32_t p = l; p < pts; p += kWL) point(p / (n2 * n1), (p / n2) % n1, p % n2);
  } else {
    const uint32_t fronts = n0 + n1 + n2 - 2;
    for (uint32_t st = 0; st < fronts; st++) {
      for (uint32_t u = l; u < n0 * n1; u += kWL) {
        const uint32_t i = u / n1, j = u % n1;
        const int k = (int)st - (int)i - (int)j;
        if (k >= 0 && k < (int)n2) point(i, j, (uint32_t)k);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  return true;
}

// Store the block's values (mode 2: the part inside the region, at
// region-relative offsets) and return the checksum of the stored words.
template <typename T>
__device__ uint64_t store_block_wave(const Geo &g, const Box &b, const T *r, T *out, uint32_t mode, const Region &reg) {
  uint64_t sum = 0;
  for (uint32_t p = threadIdx.x; p < b.pts; p += kWL) {
    const uint32_t k = p % b.n[2], j = (p / b.n[2]) % b.n[1], i = p / (b.n[2] * b.n[1]);
    const T v = r[p];
    sum += Wd<T>::sum(v);
    if (mode == 2) {
      const uint64_t z = b.o[0] + i, y = b.o[1] + j, x = b.o[2] + k;
      if (z < reg.lo[0] || z >= reg.hi[0] || y < reg.lo[1] || y >= reg.hi[1] || x < reg.lo[2] || x >= reg.hi[2])
        continue;
      out[((z - reg.lo[0]) * (reg.hi[1] - reg.lo[1]) + (y - reg.lo[1])) * (reg.hi[2] - reg.lo[2]) + (x - reg.lo[2])] = v;
    } else {
      out[fidx(g, b, i, j, k)] = v;
    }
  }
  return wave_sum(sum);
}

// Algorithm 2 for one block: decode, reconstruct, the plan's RECON flips on
// the decompressed words, store, checksum against sum_dc and, on a mismatch,
// decode again from the compressed bytes (corrected when the new checksum
// matches).  A block that cannot be decoded is zeroed and uncorrectable.
// first: false when the block was queued by the lane-per-block decoder,
// which stored it and counted the detection already (why: its reason).
template <typename T>
__device__ void decode_one_wave(const uint8_t *__restrict__ s, const Header &h, const Geo &g, const DecWork &w,
                                const PlanDev &plan, T *out, uint32_t mode, const Region &reg, uint64_t blk,
                                const WaveLds<T> &L, WaveDecTab &tab, bool first, uint64_t why) {
  const Box b = box_of(g, blk);
  const bool lead = threadIdx.x == 0;
  const uint64_t *sumdc = (const uint64_t *)(s + h.off_sumdc);
  auto zero = [&]() {
    for (uint32_t p = threadIdx.x; p < b.pts; p += kWL) L.r[p] = (T)0;
    __syncthreads();
    store_block_wave<T>(g, b, L.r, out, mode, reg);
    if (lead) count(w.cnt, C_UNC + SDCSZ_T_RECON);
  };
  if (!first) {
    if (why != 1) {  // undecodable in the first pass: so it stays
      zero();
      return;
    }
  } else {
    if (!decode_block_wave<T>(s, h, g, w, tab, blk, b, L)) {
      zero();
      return;
    }
    if (plan_hit(plan, blk)) {  // flips of decompressed words, before the checksum
      for (uint32_t t = plan_first(plan, blk); t < plan.n && plan.f[t].block == blk; t++)
        if (plan.f[t].target == SDCSZ_T_RECON && lead) {
          const uint32_t p = (uint32_t)(plan.f[t].word / Wd<T>::per);
          uint32_t wv[2] = {0, 0};
          Wd<T>::split(L.r[p], wv);
          wv[plan.f[t].word % Wd<T>::per] ^= 1u << (plan.f[t].bit & 31);
          L.r[p] = Wd<T>::join(wv);
          count(w.cnt, C_INJ + SDCSZ_T_RECON);
        }
      __syncthreads();
    }
    const uint64_t sum = store_block_wave<T>(g, b, L.r, out, mode, reg);
    if (!h.abft || sum == sumdc[blk]) return;
    if (lead) count(w.cnt, C_DET + SDCSZ_T_RECON);
  }
  // re-execution from the compressed bytes
  __syncthreads();
  bool ok = decode_block_wave<T>(s, h, g, w, tab, blk, b, L);
  if (ok) {
    uint64_t sum = 0;
    for (uint32_t p = threadIdx.x; p < b.pts; p += kWL) sum += Wd<T>::sum(L.r[p]);
    ok = wave_sum(sum) == sumdc[blk];
  }
  if (ok) store_block_wave<T>(g, b, L.r, out, mode, reg);
  if (lead) count(w.cnt, (ok ? C_COR : C_UNC) + SDCSZ_T_RECON);
}

// The fault-plan blocks the lane-per-block decoder leaves (full
// decompression).
template <typename T> __global__ void __launch_bounds__(64) k_decode_wave_list(JobTab tab) {
  const JobWg jw = job_of(tab);
  const Job &J = *jw.J;
  if (*J.dw.err) return;
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ WaveDecTab dt;
  load_wave_tab(dt, J.dw);
  const WaveLds<T> L = wave_lds<T>(lds, wave_rsz(J.g));
  const Region none{};
  decode_one_wave<T>(J.src, J.h, J.g, J.dw, J.plan, (T *)J.dst, 0, none, J.plan.list[jw.b], L, dt, true, 0);
  if (threadIdx.x == 0) count(J.dw.cnt, C_LIST);
}

// The blocks the lane-per-block decoder queued: a checksum mismatch is
// decoded again from the stream; an undecodable block is zeroed.  One
// work-group per entry at a time.
template <typename T> __global__ void __launch_bounds__(64) k_decode_wave_redo(JobTab tab, uint32_t queue) {
  const JobWg jw = job_of(tab);
  const Job &J = *jw.J;
  const DecWork &w = J.dw;
  if (*w.err) return;
  // queue 0: the production decoder's entries; 1: the fault-applying decoder's
  const uint32_t n = queue ? (uint32_t)min((uint64_t)w.cnt[C_REDO2], (uint64_t)kMaxRedo) : min(*w.redo_n, kMaxRedo);
  const uint64_t *q = w.redo + (queue ? kMaxRedo : 0u);
  if (jw.b >= n) return;
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ WaveDecTab dt;
  load_wave_tab(dt, w);
  const WaveLds<T> L = wave_lds<T>(lds, wave_rsz(J.g));
  const uint32_t mode = J.mode == 2 ? 2u : 0u;
  for (uint32_t e = jw.b; e < n; e += jw.nb) {
    const uint64_t ent = q[e];
    decode_one_wave<T>(J.src, J.h, J.g, w, J.plan, (T *)J.dst, mode, J.reg, ent & ((1ull << 56) - 1), L, dt, false,
                       ent >> 56);
    __syncthreads();
  }
}

// Region decompression of few blocks: a wave per block of the box of
// blocks the region touches, each decoded by one lane (the serial part) and
// reconstructed by the wave, storing its part of the region; the checksum
// and the re-execution follow at once.  Small regions finish in about one
// block's decoding time, where a lane per block would take a whole lane's
// serial chain at one wave per SIMD.
template <typename T> __global__ void __launch_bounds__(64) k_decode_wave_region(JobTab tab) {
  const JobWg jw = job_of(tab);
  const Job &J = *jw.J;
  if (*J.dw.err) return;
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ WaveDecTab dt;
  load_wave_tab(dt, J.dw);
  const WaveLds<T> L = wave_lds<T>(lds, wave_rsz(J.g));
  const Region &rb = J.rblk;
  const uint64_t e1 = rb.hi[1] - rb.lo[1], e2 = rb.hi[2] - rb.lo[2];
  for (uint64_t idx = jw.b; idx < J.L.shell_count; idx += jw.nb) {
    const uint64_t c2 = rb.lo[2] + idx % e2, t = idx / e2;
    const uint64_t c1 = rb.lo[1] + t % e1, c0 = rb.lo[0] + t / e1;
    const uint64_t blk = (c0 * J.g.nb[1] + c1) * J.g.nb[2] + c2;
    decode_one_wave<T>(J.src, J.h, J.g, J.dw, J.plan, (T *)J.dst, 2, J.reg, blk, L, dt, true, 0);
    __syncthreads();
  }
}

template __global__ void k_decode_wave_region<float>(JobTab);
template __global__ void k_decode_wave_region<double>(JobTab);
template __global__ void k_decode_wave_list<float>(JobTab);
template __global__ void k_decode_wave_list<double>(JobTab);
template __global__ void k_decode_wave_redo<float>(JobTab, uint32_t);
template __global__ void k_decode_wave_redo<double>(JobTab, uint32_t);
template __global__ void k_compress_wave<float>(JobTab, uint32_t);
template __global__ void k_compress_wave<double>(JobTab, uint32_t);
template __global__ void k_compress_wave_list<float>(JobTab);
template __global__ void k_compress_wave_list<double>(JobTab);
template __global__ void k_redo_wave<float>(JobTab);
template __global__ void k_redo_wave<double>(JobTab);

}  // namespace sdcsz
