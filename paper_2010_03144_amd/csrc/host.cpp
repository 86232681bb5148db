// host.cpp -- C ABI, parameter validation, workspace layout, Huffman codebook
// construction, stream header handling and kernel orchestration.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "huffman.h"
#include "kern.h"

using namespace sdcsz;

namespace {

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return SDCSZ_EHIP; \
  } while (0)

// ---------------------------------------------------------------------------
// kernel-phase timing: with timing on, a phase's first and last kernel
// dispatches record its start and stop events themselves
// (hipExtLaunchKernelGGL), so timing adds no packets to the stream
// ---------------------------------------------------------------------------
enum { PH_RANGE, PH_PREDICT, PH_CODEFAULT, PH_CHECK, PH_SCAN_C, PH_ENCODE, PH_SCAN_D, PH_DECODE, PH_NONE = -1 };
const char *kPhaseNames[SDCSZ_N_PHASES] = {"range",      "predict_quantize", "code_faults", "code_check",
                                           "scan_compress", "encode",        "scan_decompress", "decode"};

struct PhaseTimer {
  bool on = false;
  bool made = false;
  hipEvent_t ev[SDCSZ_N_PHASES][2];
  bool pending[SDCSZ_N_PHASES] = {};
  double ms[SDCSZ_N_PHASES] = {};
  uint64_t launches[SDCSZ_N_PHASES] = {};
  bool ready() {
    if (!on) return false;
    if (!made) {
      for (int i = 0; i < SDCSZ_N_PHASES; i++)
        for (int j = 0; j < 2; j++)
          if (hipEventCreate(&ev[i][j]) != hipSuccess) {
            on = false;
            return false;
          }
      made = true;
    }
    return true;
  }
  void resolve() {
    for (int i = 0; i < SDCSZ_N_PHASES; i++)
      if (pending[i]) {
        float t = 0;
        (void)hipEventSynchronize(ev[i][1]);
        if (hipEventElapsedTime(&t, ev[i][0], ev[i][1]) == hipSuccess) {
          ms[i] += t;
          launches[i]++;
        }
        pending[i] = false;
      }
  }
};
PhaseTimer g_timer;

// Launch one kernel of phase `ph` (PH_NONE: untimed); `first`/`last` mark the
// phase's first and last kernel.
template <typename F, typename... Args>
void launch(int ph, bool first, bool last, F kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ph >= 0 && g_timer.ready()) {
    if (first) a = g_timer.ev[ph][0];
    if (last) {
      b = g_timer.ev[ph][1];
      g_timer.pending[ph] = true;
    }
  }
  hipExtLaunchKernelGGL(kernel, grid, block, 0, st, a, b, 0, args...);
}

uint32_t grid_for(uint64_t n, uint32_t per) { return (uint32_t)std::max<uint64_t>(1, (n + per - 1) / per); }
uint64_t a256(uint64_t v) { return (v + 255) & ~255ull; }
uint32_t vbytes(uint32_t dtype) { return dtype == SDCSZ_F32 ? 4u : 8u; }

// ---------------------------------------------------------------------------
// geometry and validation
// ---------------------------------------------------------------------------
bool geometry(uint32_t ndim, const uint64_t *dims, const uint32_t *block, Geo *g) {
  if (ndim < 1 || ndim > 3) return false;
  std::memset(g, 0, sizeof(*g));
  for (int a = 0; a < 3; a++) {
    g->d[a] = 1;
    g->b[a] = 1;
  }
  const uint32_t off = 3 - ndim;
  for (uint32_t a = 0; a < ndim; a++) {
    if (block[a] < 1 || block[a] > 4096) return false;
    g->d[off + a] = dims[a];
    g->b[off + a] = block[a];
  }
  uint64_t bp = (uint64_t)g->b[0] * g->b[1] * g->b[2];
  if (bp > kMaxBlockPts) return false;
  g->bpts = (uint32_t)bp;
  g->groups = (uint32_t)((bp + 3) / 4);
  g->ndim = ndim;
  g->n_values = g->d[0] * g->d[1] * g->d[2];
  if (g->n_values >= (1ull << 32)) return false;
  uint64_t nb = 1;
  for (int a = 0; a < 3; a++) {
    uint64_t n = (g->d[a] + g->b[a] - 1) / g->b[a];
    g->nb[a] = (uint32_t)n;
    g->rem[a] = n ? (uint32_t)(g->d[a] - (n - 1) * g->b[a]) : 0;
    nb *= n;
  }
  g->n_blocks = nb;
  return true;
}

uint64_t block_pts(const Geo &g, uint64_t blk) {
  uint64_t t = blk;
  uint64_t c2 = t % g.nb[2];
  t /= g.nb[2];
  uint64_t c1 = t % g.nb[1], c0 = t / g.nb[1];
  uint64_t c[3] = {c0, c1, c2}, pts = 1;
  for (int a = 0; a < 3; a++) pts *= (c[a] + 1 == g.nb[a]) ? g.rem[a] : g.b[a];
  return pts;
}

// fault entries of the targets a call uses; EINVAL on out-of-range entries
int check_plan(const Geo &g, uint32_t dtype, const sdcsz_fault *f, uint32_t n, bool decomp,
               std::vector<sdcsz_fault> &out) {
  out.clear();
  if (n && !f) return SDCSZ_EINVAL;
  const uint32_t per = dtype == SDCSZ_F32 ? 1 : 2;
  for (uint32_t t = 0; t < n; t++) {
    const sdcsz_fault &e = f[t];
    if (e.target >= SDCSZ_N_TARGETS || e.block >= g.n_blocks) return SDCSZ_EINVAL;
    const uint64_t pts = block_pts(g, e.block);
    switch (e.target) {
      case SDCSZ_T_INPUT:
      case SDCSZ_T_RECON:
        if (e.word >= pts * per || e.bit >= 32) return SDCSZ_EINVAL;
        break;
      case SDCSZ_T_COEF:
        if (e.word >= 4ull * per || e.bit >= 32) return SDCSZ_EINVAL;
        break;
      case SDCSZ_T_CODE:
        if (e.word >= pts || e.bit >= 32) return SDCSZ_EINVAL;
        break;
      default:
        if (e.word >= pts || e.bit >= 32 * per) return SDCSZ_EINVAL;
        break;
    }
    if ((e.target == SDCSZ_T_RECON) == decomp) out.push_back(e);
  }
  std::stable_sort(out.begin(), out.end(),
                   [](const sdcsz_fault &a, const sdcsz_fault &b) { return a.block < b.block; });
  // the kernels keep at most kMaxPatches plan entries per block
  for (size_t i = 0, run = 0; i < out.size(); i++) {
    run = (i > 0 && out[i].block == out[i - 1].block) ? run + 1 : 1;
    if (run > kMaxPatches) return SDCSZ_EINVAL;
  }
  return SDCSZ_OK;
}

int check_params(const sdcsz_params *p, Geo *g) {
  if (!p || p->dtype > 1 || p->eb_mode > 1 || p->predictor > 2 || p->abft > 1) return SDCSZ_EINVAL;
  if (!(p->eb > 0) || !std::isfinite(p->eb)) return SDCSZ_EINVAL;
  if (!geometry(p->ndim, p->dims, p->block, g)) return SDCSZ_EINVAL;
  return SDCSZ_OK;
}

template <typename T> RegTab<T> reg_table(const Geo &g) {
  RegTab<T> rt;
  for (uint32_t pat = 0; pat < 8; pat++) {
    uint64_t n[3], pts = 1;
    for (int a = 0; a < 3; a++) {
      n[a] = (pat >> a) & 1 ? g.rem[a] : g.b[a];
      pts *= n[a];
    }
    for (int a = 0; a < 3; a++) {
      rt.c[pat][a] = (T)(0.5 * (double)(n[a] - 1));
      rt.K[pat][a] = n[a] > 1 ? (T)(12.0 / ((double)pts * ((double)n[a] * (double)n[a] - 1.0))) : (T)0;
    }
    rt.inv_pts[pat] = pts ? (T)(1.0 / (double)pts) : (T)0;
  }
  return rt;
}

// ---------------------------------------------------------------------------
// workspace layouts
// ---------------------------------------------------------------------------
struct CompLayout {
  uint64_t cnt, res, redo_n, hist, enc, zero_end;
  uint64_t eb, range, codes, vals, recon, meta, words, coef, sum_dc, sum_q, isum_q;
  uint64_t off_pay, off_out, off_coef, scan, tot, plan, bits, redo, plan_blocks, hdr, cb, total;
};

CompLayout comp_layout(const Geo &g, uint32_t dtype, uint32_t nfaults) {
  CompLayout L;
  const uint64_t nb = g.n_blocks, vb = vbytes(dtype), slots = nb * g.bpts;
  const uint64_t chunks = (nb + kScanChunk - 1) / kScanChunk + 1;
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = at;
    at = a256(at + bytes);
    return o;
  };
  // cleared by one launch at the start of a call: counters, results, redo
  // count, histogram and codeword table
  L.cnt = take(8 * C_N + 8 * R_N + 8);
  L.res = L.cnt + 8 * C_N;
  L.redo_n = L.res + 8 * R_N;
  L.hist = take(4 * 65536);
  L.enc = take(4 * 65536);
  L.zero_end = at;
  L.eb = take(sizeof(EbDev));
  L.range = take(16ull * kRangeBlocks);
  L.codes = take(2ull * 256 * g.groups * ((nb + 63) / 64));
  L.vals = take(vb * slots);
  L.recon = take(vb * slots);
  L.meta = take(4 * nb);
  L.words = take(4 * nb);
  L.coef = take(4 * vb * nb);
  L.sum_dc = take(8 * nb);
  L.sum_q = take(8 * nb);
  L.isum_q = take(8 * nb);
  L.off_pay = take(8 * (nb + 1));
  L.off_out = take(4 * (nb + 1));
  L.off_coef = take(4 * (nb + 1));
  L.scan = take(24 * chunks);
  L.tot = take(24);
  L.plan = take(sizeof(sdcsz_fault) * (uint64_t)std::max<uint32_t>(nfaults, 1));
  L.bits = take(4 * (nb / 32 + 1));
  L.redo = take(8ull * kMaxRedo);
  L.plan_blocks = take(8ull * std::max<uint32_t>(nfaults, 1));
  L.hdr = take(sizeof(Header));
  L.cb = take(8ull * 65536);
  L.total = at;
  return L;
}

// Specialised kernel for this block shape, if there is one.  Its lanes
// address the input with 32-bit byte offsets from the wave's lowest block,
// so it takes fields below 2 GiB.
bool fast_shape(const Geo &g, uint32_t vb) {
  if (!(g.ndim == 3 && g.b[0] == 6 && g.b[1] == 6 && g.b[2] == 6)) return false;
  return g.n_values * vb < (1ull << 31);
}

// One launch of a specialised kernel: the first work-groups take the
// sub-grid of full blocks, the others the shell of partial blocks along the
// upper faces.  Returns the number of work-groups of 256 lanes.
uint32_t fast_launch(const Geo &g, Launch *L) {
  bool part[3];
  std::memset(L, 0, sizeof(*L));
  for (int a = 0; a < 3; a++) {
    part[a] = g.rem[a] != g.b[a];
    L->nf[a] = g.nb[a] - (part[a] ? 1 : 0);
  }
  L->full_count = (uint64_t)L->nf[0] * L->nf[1] * L->nf[2];
  L->s2 = part[2] ? (uint64_t)g.nb[0] * g.nb[1] : 0;
  L->s1 = part[1] ? (uint64_t)g.nb[0] * L->nf[2] : 0;
  const uint64_t s0 = part[0] ? (uint64_t)L->nf[1] * L->nf[2] : 0;
  L->shell_count = L->s2 + L->s1 + s0;
  L->full_wgs = (uint32_t)((L->full_count + 255) / 256);
  return L->full_wgs + (uint32_t)((L->shell_count + 255) / 256);
}

template <typename T, bool ABFT>
void launch_fast(const T *in, const Geo &g, const RegTab<T> &rt, const PlanDev &pd, const CompWork &w,
                 uint32_t predictor, const uint64_t *plan_blocks, uint32_t n_plan_blocks, hipStream_t st) {
  if (n_plan_blocks)
    hipLaunchKernelGGL(k_compress_list<T>, dim3(grid_for(n_plan_blocks, 64)), dim3(64), 0, st, in, g, rt, pd, w,
                       ABFT ? 1u : 0u, predictor, plan_blocks, n_plan_blocks);
  Launch L;
  const uint32_t wgs = fast_launch(g, &L);
  if (wgs)
    launch(PH_PREDICT, true, true, k_compress_fast<T, 3, 6, 6, 6, ABFT>, dim3(wgs), dim3(256), st, in, g, rt, pd, w,
           predictor, L);
  hipLaunchKernelGGL(k_redo<T>, dim3(1), dim3(64), 0, st, in, g, rt, pd, w, ABFT ? 1u : 0u, predictor);
}

struct DecLayout {
  uint64_t cnt, redo_n, err, zero_end;
  uint64_t symbols, tab, recon, off_pay, off_out, off_coef, scan, tot, plan, bits, lut, redo, plan_blocks;
  uint64_t total;
};

DecLayout dec_layout(const Geo &g, uint32_t dtype, uint32_t nfaults) {
  DecLayout L;
  const uint64_t nb = g.n_blocks, vb = vbytes(dtype), slots = nb * g.bpts;
  const uint64_t chunks = (nb + kScanChunk - 1) / kScanChunk + 1;
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = at;
    at = a256(at + bytes);
    return o;
  };
  // counters, redo count and error flag: cleared together, read back together
  L.cnt = take(8 * C_N + 8);
  L.redo_n = L.cnt + 8 * C_N;
  L.err = L.redo_n + 4;
  L.zero_end = at;
  L.symbols = take(2 * 65536);
  L.tab = take(sizeof(DecTab));
  L.recon = take(vb * slots);
  L.off_pay = take(8 * (nb + 1));
  L.off_out = take(4 * (nb + 1));
  L.off_coef = take(4 * (nb + 1));
  L.scan = take(24 * chunks);
  L.tot = take(24);
  L.plan = take(sizeof(sdcsz_fault) * (uint64_t)std::max<uint32_t>(nfaults, 1));
  L.bits = take(4 * (nb / 32 + 1));
  L.lut = take(4ull << kLutBits);
  L.redo = take(8ull * kMaxRedo);
  L.plan_blocks = take(8ull * std::max<uint32_t>(nfaults, 1));
  L.total = at;
  return L;
}

// ---------------------------------------------------------------------------
// pinned host staging of the calling thread: the code histogram, the
// codebook list and each call's results cross PCIe through it.  Allocated
// on first use and kept until the process ends.
// ---------------------------------------------------------------------------
constexpr size_t kStageHist = 0;                             // 65536 u32 counts
constexpr size_t kStageCb = kStageHist + 4 * 65536;         // 65536 pairs of u32
constexpr size_t kStageRes = kStageCb + 8 * 65536;          // results of the call
constexpr size_t kStageBytes = kStageRes + 8 * (C_N + R_N + 2);

struct Staging {
  uint8_t *p = nullptr;
  uint8_t *get() {
    if (!p && hipHostMalloc((void **)&p, kStageBytes, hipHostMallocDefault) != hipSuccess) p = nullptr;
    return p;
  }
};
thread_local Staging t_stage;

// Huffman construction buffers of the calling thread, reused across calls
struct HuffmanScratch {
  HuffmanBuilder b;
  std::vector<uint32_t> sym, code;
  std::vector<uint64_t> cnt;
  std::vector<uint8_t> len;
};
thread_local HuffmanScratch t_huff;

// ---------------------------------------------------------------------------
// header
// ---------------------------------------------------------------------------
const uint8_t kMagic[8] = {'S', 'D', 'C', 'S', 'Z', 0, 'v', '1'};

template <typename V> V get(const uint8_t *b, uint64_t off) {
  V v;
  std::memcpy(&v, b + off, sizeof(V));
  return v;
}

// parse + validate the header (and its geometry) from host bytes
int unpack_header(const uint8_t *o, uint64_t stream_size, Header &h, Geo &g) {
  if (stream_size < kHeader || std::memcmp(o, kMagic, 8) != 0) return SDCSZ_EFORMAT;
  h.dtype = get<uint32_t>(o, 8);
  h.ndim = get<uint32_t>(o, 12);
  for (int a = 0; a < 3; a++) h.d[a] = get<uint64_t>(o, 16 + 8 * a);
  for (int a = 0; a < 3; a++) h.b[a] = get<uint32_t>(o, 40 + 4 * a);
  h.eb_mode = get<uint32_t>(o, 52);
  h.eb = get<double>(o, 56);
  h.eb_abs = get<double>(o, 64);
  h.abft = get<uint32_t>(o, 72);
  h.n_sym = get<uint32_t>(o, 76);
  h.n_blocks = get<uint64_t>(o, 80);
  h.n_outliers = get<uint64_t>(o, 88);
  h.n_regression = get<uint64_t>(o, 96);
  h.payload_words = get<uint64_t>(o, 104);
  h.predictor = get<uint32_t>(o, 168);
  if (h.dtype > 1 || h.abft > 1 || h.n_sym > 65536 || h.ndim < 1 || h.ndim > 3) return SDCSZ_EFORMAT;
  Header chk = h;
  section_offsets(chk);
  if (chk.off_table != get<uint64_t>(o, 120) || chk.off_coef != get<uint64_t>(o, 128) ||
      chk.off_sumdc != get<uint64_t>(o, 136) || chk.off_outliers != get<uint64_t>(o, 144) ||
      chk.off_payload != get<uint64_t>(o, 152) || chk.total != get<uint64_t>(o, 160) ||
      get<uint64_t>(o, 112) != kHeader)
    return SDCSZ_EFORMAT;
  h = chk;
  if (h.total > stream_size) return SDCSZ_EFORMAT;
  uint64_t dims[3];
  uint32_t blk[3];
  for (uint32_t a = 0; a < 3 - h.ndim; a++)
    if (h.d[a] != 1 || h.b[a] != 1) return SDCSZ_EFORMAT;
  for (uint32_t a = 0; a < h.ndim; a++) {
    dims[a] = h.d[3 - h.ndim + a];
    blk[a] = h.b[3 - h.ndim + a];
  }
  if (!geometry(h.ndim, dims, blk, &g) || g.n_blocks != h.n_blocks) return SDCSZ_EFORMAT;
  if (h.n_outliers > g.n_values || h.n_regression > g.n_blocks) return SDCSZ_EFORMAT;
  return SDCSZ_OK;
}

void fill_report(sdcsz_report *r, const unsigned long long *cnt, uint64_t nb) {
  std::memset(r, 0, sizeof(*r));
  r->n_blocks = nb;
  for (int t = 0; t < SDCSZ_N_TARGETS; t++) {
    r->injected[t] = cnt[C_INJ + t];
    r->detected[t] = cnt[C_DET + t];
    r->corrected[t] = cnt[C_COR + t];
    r->uncorrectable[t] = cnt[C_UNC + t];
  }
}

// upload a sorted plan and its per-block bitmap (from pageable memory: the
// vectors must live until the stream has passed the copies)
int upload_plan(const std::vector<sdcsz_fault> &pl, uint64_t nb, uint8_t *ws, uint64_t off_plan,
                uint64_t off_bits, std::vector<uint32_t> &bits_host, hipStream_t st, PlanDev *pd) {
  pd->n = (uint32_t)pl.size();
  pd->f = (const sdcsz_fault *)(ws + off_plan);
  pd->bits = (const uint32_t *)(ws + off_bits);
  if (pl.empty()) return SDCSZ_OK;
  bits_host.assign(nb / 32 + 1, 0);
  for (auto &f : pl) bits_host[f.block >> 5] |= 1u << (f.block & 31);
  HIPCHK(hipMemcpyAsync(ws + off_plan, pl.data(), pl.size() * sizeof(sdcsz_fault), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ws + off_bits, bits_host.data(), bits_host.size() * 4, hipMemcpyHostToDevice, st));
  return SDCSZ_OK;
}

// exclusive scans of payload words, outliers and regression flags per block,
// with the 64-bit totals in tot[0..2]
int launch_scan(ScanSrc src, uint64_t n, uint64_t *part, uint64_t *off_pay, uint32_t *off_out,
                uint32_t *off_coef, uint64_t *tot, int ph, hipStream_t st) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long *)off_pay, 1);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, off_out, 1);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, off_coef, 1);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long *)tot, 3);
    return hipGetLastError() == hipSuccess ? SDCSZ_OK : SDCSZ_EHIP;
  }
  uint32_t chunks = (uint32_t)((n + kScanChunk - 1) / kScanChunk);
  launch(ph, true, false, k_scan1, dim3(chunks), dim3(kScanThreads), st, src, n, part);
  launch(ph, false, false, k_scan2, dim3(1), dim3(kScanThreads), st, part, chunks);
  launch(ph, false, true, k_scan3, dim3(chunks), dim3(kScanThreads), st, src, n, (const uint64_t *)part, off_pay,
         off_out, off_coef, tot);
  return hipGetLastError() == hipSuccess ? SDCSZ_OK : SDCSZ_EHIP;
}

// distinct blocks of a sorted plan
std::vector<uint64_t> plan_block_list(const std::vector<sdcsz_fault> &plan) {
  std::vector<uint64_t> pb;
  for (auto &f : plan)
    if (pb.empty() || pb.back() != f.block) pb.push_back(f.block);
  return pb;
}

// ---------------------------------------------------------------------------
// compression: two host synchronisations, one for the code histogram (the
// Huffman code is built on the host) and one for the results at the end
// ---------------------------------------------------------------------------
template <typename T>
int compress_t(const void *d_in, const sdcsz_params *p, const Geo &g, uint8_t *d_out, uint64_t out_cap,
               uint64_t *h_out_size, sdcsz_report *h_rep, uint8_t *ws, uint64_t ws_size, hipStream_t st) {
  std::vector<sdcsz_fault> plan;
  int rc = check_plan(g, p->dtype, p->faults, p->n_faults, false, plan);
  if (rc) return rc;
  const CompLayout L = comp_layout(g, p->dtype, p->n_faults);
  if (!ws || ws_size < L.total) return SDCSZ_ENOSPC;
  uint8_t *hs = t_stage.get();
  if (!hs) return SDCSZ_EHIP;
  CompWork w;
  w.codes = (uint16_t *)(ws + L.codes);
  w.vals = ws + L.vals;
  w.recon = ws + L.recon;
  w.meta = (uint32_t *)(ws + L.meta);
  w.words = (uint32_t *)(ws + L.words);
  w.coef = ws + L.coef;
  w.sum_dc = (uint64_t *)(ws + L.sum_dc);
  w.sum_q = (uint64_t *)(ws + L.sum_q);
  w.isum_q = (uint64_t *)(ws + L.isum_q);
  w.hist = (uint32_t *)(ws + L.hist);
  w.enc = (uint32_t *)(ws + L.enc);
  w.cnt = (unsigned long long *)(ws + L.cnt);
  w.off_pay = (uint64_t *)(ws + L.off_pay);
  w.off_out = (uint32_t *)(ws + L.off_out);
  w.off_coef = (uint32_t *)(ws + L.off_coef);
  w.scan_part = (uint64_t *)(ws + L.scan);
  w.range_part = ws + L.range;
  w.eb = (EbDev *)(ws + L.eb);
  w.redo_n = (uint32_t *)(ws + L.redo_n);
  w.redo = (uint64_t *)(ws + L.redo);
  w.hdr = (Header *)(ws + L.hdr);
  w.res = (uint64_t *)(ws + L.res);
  w.cb = (uint32_t *)(ws + L.cb);
  w.tot = (uint64_t *)(ws + L.tot);

  // host vectors read by asynchronous copies live until the histogram sync
  std::vector<uint32_t> bits_host;
  PlanDev pd;
  rc = upload_plan(plan, g.n_blocks, ws, L.plan, L.bits, bits_host, st, &pd);
  if (rc) return rc;
  const std::vector<uint64_t> pb = plan_block_list(plan);

  hipLaunchKernelGGL(k_zero_u32, dim3(256), dim3(256), 0, st, (uint32_t *)ws, L.zero_end / 4);
  uint32_t nparts = 0;
  if (p->eb_mode == SDCSZ_REL && g.n_values) {
    nparts = (uint32_t)std::min<uint64_t>(kRangeBlocks, grid_for(g.n_values, kRangeThreads * 8));
    launch(PH_RANGE, true, true, k_range<T>, dim3(nparts), dim3(kRangeThreads), st, (const T *)d_in, g.n_values,
           (double *)w.range_part);
  }
  hipLaunchKernelGGL(k_consts, dim3(1), dim3(256), 0, st, (const double *)w.range_part, nparts, p->eb_mode,
                     p->eb, w.eb);
  HIPCHK(hipGetLastError());

  const bool fast = g.n_blocks && fast_shape(g, sizeof(T));
  if (g.n_blocks) {
    const RegTab<T> rt = reg_table<T>(g);
    if (fast) {
      // the distinct blocks the plan names run through the generic routine
      const uint64_t *d_pb = (const uint64_t *)(ws + L.plan_blocks);
      if (!pb.empty())
        HIPCHK(hipMemcpyAsync(ws + L.plan_blocks, pb.data(), 8 * pb.size(), hipMemcpyHostToDevice, st));
      if (p->abft) launch_fast<T, true>((const T *)d_in, g, rt, pd, w, p->predictor, d_pb, (uint32_t)pb.size(), st);
      else launch_fast<T, false>((const T *)d_in, g, rt, pd, w, p->predictor, d_pb, (uint32_t)pb.size(), st);
    } else {
      launch(PH_PREDICT, true, true, k_compress_generic<T>, dim3(grid_for(g.n_blocks, 64)), dim3(64), st,
             (const T *)d_in, g, rt, pd, w, p->abft, p->predictor);
    }
    HIPCHK(hipGetLastError());
    bool any_code = false;
    for (auto &f : plan) any_code |= f.target == SDCSZ_T_CODE;
    if (any_code) {
      launch(PH_CODEFAULT, true, true, k_code_faults, dim3(1), dim3(64), st, pd, g, w.codes, w.cnt);
    }
  }

  // Huffman code over the whole field's codes (host)
  const uint32_t *hist = (const uint32_t *)(hs + kStageHist);
  HIPCHK(hipMemcpyAsync(hs + kStageHist, w.hist, 4 * 65536, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<uint32_t> &used = t_huff.sym;
  std::vector<uint64_t> &counts = t_huff.cnt;
  used.clear();
  counts.clear();
  const uint64_t *h64 = (const uint64_t *)hist;
  for (uint32_t q = 0; q < 32768; q++) {
    const uint64_t v = h64[q];
    if (!v) continue;
    if ((uint32_t)v) {
      used.push_back(2 * q);
      counts.push_back((uint32_t)v);
    }
    if (v >> 32) {
      used.push_back(2 * q + 1);
      counts.push_back(v >> 32);
    }
  }
  std::vector<uint8_t> &len = t_huff.len;
  std::vector<uint32_t> &codes = t_huff.code;
  t_huff.b.lengths(counts, kMaxLen, len);
  canonical_codes(len, kMaxLen, codes);
  const uint32_t n_sym = (uint32_t)used.size();
  uint32_t *cb = (uint32_t *)(hs + kStageCb);
  for (uint32_t t = 0; t < n_sym; t++) {
    cb[2 * t] = (used[t] << 8) | len[t];
    cb[2 * t + 1] = codes[t];
  }
  if (n_sym) {
    HIPCHK(hipMemcpyAsync(w.cb, cb, 8ull * n_sym, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_put_codes, dim3(grid_for(n_sym, 256)), dim3(256), 0, st, w.cb, n_sym, w.enc);
  }

  if (g.n_blocks) {
    if (fast)
      launch(PH_CHECK, true, true, k_check_fast<6, 6, 6>, dim3(grid_for(g.n_blocks, 256)), dim3(256), st, g, w,
             p->abft);
    else
      launch(PH_CHECK, true, true, k_codes_check, dim3(grid_for(g.n_blocks, 256)), dim3(256), st, g, w, p->abft);
  }
  ScanSrc src{w.words, w.meta, 1};
  rc = launch_scan(src, g.n_blocks, w.scan_part, w.off_pay, w.off_out, w.off_coef, w.tot, PH_SCAN_C, st);
  if (rc) return rc;

  // header, codebook and pads on the device; the encoder follows its decision
  Header h;
  std::memset(&h, 0, sizeof(h));
  h.dtype = p->dtype;
  h.ndim = p->ndim;
  for (int a = 0; a < 3; a++) {
    h.d[a] = g.d[a];
    h.b[a] = g.b[a];
  }
  h.eb_mode = p->eb_mode;
  h.eb = p->eb;
  h.abft = p->abft;
  h.n_sym = n_sym;
  h.n_blocks = g.n_blocks;
  h.predictor = p->predictor;
  hipLaunchKernelGGL(k_header, dim3(grid_for(n_sym, 256)), dim3(256), 0, st, h, w, d_out, d_out ? out_cap : 0);
  if (fast)
    launch(PH_ENCODE, true, true, k_encode_fast<T, 6, 6, 6>, dim3(grid_for(g.n_blocks, 256)), dim3(256), st, g, w,
           d_out);
  else if (g.n_blocks)
    launch(PH_ENCODE, true, true, k_encode<T>, dim3(grid_for(g.n_blocks, 256)), dim3(256), st, g, w, d_out);
  HIPCHK(hipGetLastError());

  // counters and results: one copy, one synchronisation
  unsigned long long *cnt = (unsigned long long *)(hs + kStageRes);
  const uint64_t *res = (const uint64_t *)(hs + kStageRes + 8 * C_N);
  HIPCHK(hipMemcpyAsync(hs + kStageRes, ws + L.cnt, 8 * (C_N + R_N), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  g_timer.resolve();

  sdcsz_report rep;
  fill_report(&rep, cnt, g.n_blocks);
  double eb_abs;
  std::memcpy(&eb_abs, &res[R_EB], 8);
  rep.eb_abs = eb_abs;
  const bool unc = cnt[C_UNC + SDCSZ_T_INPUT] || cnt[C_UNC + SDCSZ_T_COEF] || cnt[C_UNC + SDCSZ_T_CODE] ||
                   cnt[C_MISSING];
  if (unc) {
    *h_out_size = 0;
    if (h_rep) *h_rep = rep;
    return SDCSZ_ESDC;
  }
  rep.n_outliers = res[R_OUTLIERS];
  rep.n_regression = res[R_REGRESSION];
  rep.payload_words = res[R_WORDS];
  rep.stream_size = res[R_SIZE];
  *h_out_size = res[R_SIZE];
  if (h_rep) *h_rep = rep;
  return res[R_WRITTEN] ? SDCSZ_OK : SDCSZ_ENOSPC;
}

// ---------------------------------------------------------------------------
// decompression / verification / region: one synchronisation for the header
// (the host sizes the launches from it) and one for the results
// ---------------------------------------------------------------------------
struct Opened {
  Header h;
  Geo g;
};

int open_stream(const void *d_stream, uint64_t size, hipStream_t st, Opened &o) {
  if (!d_stream) return SDCSZ_EINVAL;
  if (size < kHeader) return SDCSZ_EFORMAT;
  uint8_t *hs = t_stage.get();
  if (!hs) return SDCSZ_EHIP;
  HIPCHK(hipMemcpyAsync(hs + kStageRes, d_stream, kHeader, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return unpack_header(hs + kStageRes, size, o.h, o.g);
}

template <typename T>
int decode_t(const uint8_t *d_s, Opened &o, T *d_out, uint32_t mode, const Region &reg,
             const sdcsz_fault *faults, uint32_t n_faults, sdcsz_report *h_rep, uint8_t *ws, uint64_t ws_size,
             hipStream_t st) {
  const Header &h = o.h;
  const Geo &g = o.g;
  std::vector<sdcsz_fault> plan;
  int rc = check_plan(g, h.dtype, faults, n_faults, true, plan);
  if (rc) return rc;
  const DecLayout L = dec_layout(g, h.dtype, n_faults);
  if (!ws || ws_size < L.total) return SDCSZ_ENOSPC;
  uint8_t *hs = t_stage.get();
  if (!hs) return SDCSZ_EHIP;
  DecWork w;
  w.cnt = (unsigned long long *)(ws + L.cnt);
  w.symbols = (uint16_t *)(ws + L.symbols);
  w.tab = (DecTab *)(ws + L.tab);
  w.recon = ws + L.recon;
  w.off_pay = (uint64_t *)(ws + L.off_pay);
  w.off_out = (uint32_t *)(ws + L.off_out);
  w.off_coef = (uint32_t *)(ws + L.off_coef);
  w.scan_part = (uint64_t *)(ws + L.scan);
  w.lut = (uint32_t *)(ws + L.lut);
  w.redo_n = (uint32_t *)(ws + L.redo_n);
  w.redo = (uint64_t *)(ws + L.redo);
  w.err = (uint32_t *)(ws + L.err);
  w.tot = (uint64_t *)(ws + L.tot);
  std::vector<uint32_t> bits_host;
  PlanDev pd;
  rc = upload_plan(plan, g.n_blocks, ws, L.plan, L.bits, bits_host, st, &pd);
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, (uint32_t *)ws, L.zero_end / 4);
  // decoder tables from the codebook section, then the block table's scans
  hipLaunchKernelGGL(k_dectab, dim3(1), dim3(256), 0, st, (const uint32_t *)(d_s + kHeader), h.n_sym, w);
  const uint32_t *table = (const uint32_t *)(d_s + h.off_table);
  ScanSrc src{table, table + 1, 2};
  rc = launch_scan(src, g.n_blocks, w.scan_part, w.off_pay, w.off_out, w.off_coef, w.tot, PH_SCAN_D, st);
  hipLaunchKernelGGL(k_dec_check, dim3(1), dim3(64), 0, st, (const uint64_t *)w.tot, h.payload_words, h.n_outliers,
                     h.n_regression, w.err);
  if (rc) return rc;
  const bool fast = mode == 0 && fast_shape(g, sizeof(T));
  const std::vector<uint64_t> pb = plan_block_list(plan);
  if (g.n_blocks && fast) {
    const uint64_t *d_pb = (const uint64_t *)(ws + L.plan_blocks);
    if (!pb.empty()) HIPCHK(hipMemcpyAsync(ws + L.plan_blocks, pb.data(), 8 * pb.size(), hipMemcpyHostToDevice, st));
    if (!pb.empty())
      hipLaunchKernelGGL(k_decode_list<T>, dim3(grid_for(pb.size(), 64)), dim3(64), 0, st, d_s, h, g, w, pd, d_out,
                         d_pb, (uint32_t)pb.size());
    Launch FL;
    const uint32_t wgs = fast_launch(g, &FL);
    if (wgs)
      launch(PH_DECODE, true, true, k_decode_fast<T, 3, 6, 6, 6>, dim3(wgs), dim3(256), st, d_s, h, g, w, pd, d_out,
             FL);
    hipLaunchKernelGGL(k_decode_redo<T>, dim3(kMaxRedo / 64), dim3(64), 0, st, d_s, h, g, w, d_out);
    HIPCHK(hipGetLastError());
  } else if (g.n_blocks) {
    launch(PH_DECODE, true, true, k_decode_generic<T>, dim3(grid_for(g.n_blocks, 64)), dim3(64), st, d_s, h, g, w,
           pd, d_out, mode, reg);
    HIPCHK(hipGetLastError());
  }
  // counters, redo count and error flag: one copy, one synchronisation
  const unsigned long long *cnt = (const unsigned long long *)(hs + kStageRes);
  const uint32_t *tail = (const uint32_t *)(hs + kStageRes + 8 * C_N);
  HIPCHK(hipMemcpyAsync(hs + kStageRes, ws + L.cnt, 8 * C_N + 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  g_timer.resolve();
  if (tail[1]) return SDCSZ_EFORMAT;
  if (fast && tail[0] > kMaxRedo) {
    // more blocks to re-execute than the queue holds: decode everything again
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, w.cnt, (uint64_t)C_N);
    hipLaunchKernelGGL(k_decode_generic<T>, dim3(grid_for(g.n_blocks, 64)), dim3(64), 0, st, d_s, h, g, w, pd,
                       d_out, mode, reg);
    HIPCHK(hipMemcpyAsync(hs + kStageRes, w.cnt, 8 * C_N, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  sdcsz_report rep;
  fill_report(&rep, cnt, g.n_blocks);
  rep.eb_abs = h.eb_abs;
  rep.n_outliers = h.n_outliers;
  rep.n_regression = h.n_regression;
  rep.payload_words = h.payload_words;
  rep.stream_size = h.total;
  if (h_rep) *h_rep = rep;
  return cnt[C_UNC + SDCSZ_T_RECON] ? SDCSZ_ESDC : SDCSZ_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *sdcsz_strerror(int code) {
  switch (code) {
    case SDCSZ_OK: return "ok";
    case SDCSZ_EINVAL: return "invalid argument";
    case SDCSZ_ENOSPC: return "output or workspace too small";
    case SDCSZ_EFORMAT: return "not a valid sdcsz stream";
    case SDCSZ_ESDC: return "uncorrectable silent data corruption";
    case SDCSZ_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

void sdcsz_timing_enable(int on) {
  for (int i = 0; i < SDCSZ_N_PHASES; i++) {
    g_timer.ms[i] = 0;
    g_timer.launches[i] = 0;
    g_timer.pending[i] = false;
  }
  g_timer.on = on != 0;
}

void sdcsz_timing_read(sdcsz_timing *h_out) {
  if (!h_out) return;
  for (int i = 0; i < SDCSZ_N_PHASES; i++) {
    h_out->ms[i] = g_timer.ms[i];
    h_out->launches[i] = g_timer.launches[i];
  }
}

const char *sdcsz_phase_name(int phase) {
  return phase >= 0 && phase < SDCSZ_N_PHASES ? kPhaseNames[phase] : "unknown";
}

uint64_t sdcsz_max_compressed_size(const sdcsz_params *p) {
  Geo g;
  if (check_params(p, &g)) return 0;
  Header h;
  std::memset(&h, 0, sizeof(h));
  h.dtype = p->dtype;
  h.abft = 1;
  h.n_sym = 65536;
  h.n_blocks = g.n_blocks;
  h.n_regression = g.n_blocks;
  h.n_outliers = g.n_values;
  h.payload_words = (g.n_values * kMaxLen + 31) / 32 + g.n_blocks;
  section_offsets(h);
  return h.total;
}

uint64_t sdcsz_compress_workspace_size(const sdcsz_params *p) {
  Geo g;
  if (check_params(p, &g)) return 0;
  return comp_layout(g, p->dtype, p->n_faults).total;
}

int sdcsz_compress(const void *d_in, const sdcsz_params *p, void *d_out, uint64_t out_cap, uint64_t *h_out_size,
                   sdcsz_report *h_rep, void *d_ws, uint64_t ws_size, void *stream) {
  Geo g;
  int rc = check_params(p, &g);
  if (rc) return rc;
  if (!h_out_size || (g.n_values && !d_in)) return SDCSZ_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (p->dtype == SDCSZ_F32)
    return compress_t<float>(d_in, p, g, (uint8_t *)d_out, out_cap, h_out_size, h_rep, (uint8_t *)d_ws, ws_size, st);
  return compress_t<double>(d_in, p, g, (uint8_t *)d_out, out_cap, h_out_size, h_rep, (uint8_t *)d_ws, ws_size, st);
}

int sdcsz_stream_info(const void *d_stream, uint64_t stream_size, sdcsz_params *h_p, uint64_t *h_n_blocks,
                      double *h_eb_abs, void *stream) {
  Opened o;
  int rc = open_stream(d_stream, stream_size, (hipStream_t)stream, o);
  if (rc) return rc;
  if (h_p) {
    std::memset(h_p, 0, sizeof(*h_p));
    h_p->dtype = o.h.dtype;
    h_p->ndim = o.h.ndim;
    for (uint32_t a = 0; a < o.h.ndim; a++) {
      h_p->dims[a] = o.h.d[3 - o.h.ndim + a];
      h_p->block[a] = o.h.b[3 - o.h.ndim + a];
    }
    h_p->eb_mode = o.h.eb_mode;
    h_p->predictor = o.h.predictor;
    h_p->eb = o.h.eb;
    h_p->abft = o.h.abft;
  }
  if (h_n_blocks) *h_n_blocks = o.h.n_blocks;
  if (h_eb_abs) *h_eb_abs = o.h.eb_abs;
  return SDCSZ_OK;
}

uint64_t sdcsz_decompress_workspace_size(const sdcsz_params *p) {
  Geo g;
  if (!p || p->dtype > 1 || !geometry(p->ndim, p->dims, p->block, &g)) return 0;
  return dec_layout(g, p->dtype, p->n_faults).total;
}

int sdcsz_decompress(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap,
                     const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                     void *stream) {
  hipStream_t st = (hipStream_t)stream;
  Opened o;
  int rc = open_stream(d_stream, stream_size, st, o);
  if (rc) return rc;
  if (out_cap < o.g.n_values * vbytes(o.h.dtype) || (o.g.n_values && !d_out)) return SDCSZ_ENOSPC;
  Region reg{};
  if (o.h.dtype == SDCSZ_F32)
    return decode_t<float>((const uint8_t *)d_stream, o, (float *)d_out, 0, reg, h_faults, n_faults, h_rep,
                           (uint8_t *)d_ws, ws_size, st);
  return decode_t<double>((const uint8_t *)d_stream, o, (double *)d_out, 0, reg, h_faults, n_faults, h_rep,
                          (uint8_t *)d_ws, ws_size, st);
}

int sdcsz_verify(const void *d_stream, uint64_t stream_size, void *d_data, uint64_t data_size,
                 const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                 void *stream) {
  hipStream_t st = (hipStream_t)stream;
  Opened o;
  int rc = open_stream(d_stream, stream_size, st, o);
  if (rc) return rc;
  if (!o.h.abft) return SDCSZ_EINVAL;
  if (data_size < o.g.n_values * vbytes(o.h.dtype) || (o.g.n_values && !d_data)) return SDCSZ_ENOSPC;
  Region reg{};
  if (o.h.dtype == SDCSZ_F32)
    return decode_t<float>((const uint8_t *)d_stream, o, (float *)d_data, 1, reg, h_faults, n_faults, h_rep,
                           (uint8_t *)d_ws, ws_size, st);
  return decode_t<double>((const uint8_t *)d_stream, o, (double *)d_data, 1, reg, h_faults, n_faults, h_rep,
                          (uint8_t *)d_ws, ws_size, st);
}

int sdcsz_decompress_region(const void *d_stream, uint64_t stream_size, const uint64_t *h_lo, const uint64_t *h_hi,
                            void *d_out, uint64_t out_cap, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                            void *stream) {
  hipStream_t st = (hipStream_t)stream;
  Opened o;
  int rc = open_stream(d_stream, stream_size, st, o);
  if (rc) return rc;
  if (!h_lo || !h_hi) return SDCSZ_EINVAL;
  Region reg;
  uint64_t cnt = 1;
  const uint32_t off = 3 - o.h.ndim;
  for (int a = 0; a < 3; a++) {
    reg.lo[a] = 0;
    reg.hi[a] = 1;
  }
  for (uint32_t a = 0; a < o.h.ndim; a++) {
    reg.lo[off + a] = h_lo[a];
    reg.hi[off + a] = h_hi[a];
  }
  for (int a = 0; a < 3; a++) {
    if (reg.lo[a] >= reg.hi[a] || reg.hi[a] > o.g.d[a]) return SDCSZ_EINVAL;
    cnt *= reg.hi[a] - reg.lo[a];
  }
  if (out_cap < cnt * vbytes(o.h.dtype) || !d_out) return SDCSZ_ENOSPC;
  if (o.h.dtype == SDCSZ_F32)
    return decode_t<float>((const uint8_t *)d_stream, o, (float *)d_out, 2, reg, nullptr, 0, h_rep, (uint8_t *)d_ws,
                           ws_size, st);
  return decode_t<double>((const uint8_t *)d_stream, o, (double *)d_out, 2, reg, nullptr, 0, h_rep, (uint8_t *)d_ws,
                          ws_size, st);
}

}  // extern "C"
