// host.cpp -- C ABI, parameter validation, workspace layout, Huffman codebook
// construction, stream header handling and kernel orchestration.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"
#include "huffman.h"
#include "kern.h"

using namespace sdcsz;

// Device scratch of sdcsz_decompress_noalloc: one array per GPU, held from the
// library's load until the process ends.  Host code must not pass this name
// to a kernel or a copy: it only stands in for the device array, whose
// address hipGetSymbolAddress gives per device.
static __device__ __align__(256) uint8_t scratch[SDCSZ_NOALLOC_SCRATCH_BYTES];

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
enum { PH_RANGE, PH_PREDICT, PH_CODEFAULT, PH_CHECK, PH_SCAN_C, PH_ENCODE, PH_SCAN_D, PH_DECODE,
       PH_HOST_CODEBOOK, PH_HOST_WAIT, PH_HOST_CALL, PH_NONE = -1 };
constexpr int kDevicePhases = PH_HOST_CODEBOOK;
const char *kPhaseNames[SDCSZ_N_PHASES] = {"range",         "predict_quantize", "code_faults",    "code_check",
                                           "scan_compress", "encode",           "scan_decompress", "decode",
                                           "host_codebooks", "host_wait",       "host_call"};

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
      for (int i = 0; i < kDevicePhases; i++)
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
    for (int i = 0; i < kDevicePhases; i++)
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

// Host wall time of a scope, added to a host phase while timing is on.
struct HostSpan {
  int ph;
  std::chrono::steady_clock::time_point t0;
  explicit HostSpan(int p) : ph(p), t0(std::chrono::steady_clock::now()) {}
  ~HostSpan() {
    if (!g_timer.on) return;
    g_timer.ms[ph] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    g_timer.launches[ph]++;
  }
};

hipError_t sync_wait(hipStream_t st) {
  HostSpan h(PH_HOST_WAIT);
  return hipStreamSynchronize(st);
}

// Launch one kernel of phase `ph` (PH_NONE: untimed); `first`/`last` mark the
// phase's first and last kernel.
template <typename F, typename... Args>
void launch_shm(int ph, bool first, bool last, F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st,
                Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ph >= 0 && g_timer.ready()) {
    if (first) a = g_timer.ev[ph][0];
    if (last) {
      b = g_timer.ev[ph][1];
      g_timer.pending[ph] = true;
    }
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shm, st, a, b, 0, args...);
}
template <typename F, typename... Args>
void launch(int ph, bool first, bool last, F kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
  launch_shm(ph, first, last, kernel, grid, block, 0, st, args...);
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
      case SDCSZ_T_PREP_INPUT:
      case SDCSZ_T_RECON:
        if (e.word >= pts * per || e.bit >= 32) return SDCSZ_EINVAL;
        break;
      case SDCSZ_T_COEF:
      case SDCSZ_T_PREP_COEF:
        if (e.word >= 4ull * per || e.bit >= 32) return SDCSZ_EINVAL;
        break;
      case SDCSZ_T_PREP_SAMPLE:
        if (e.word >= 2 || e.bit >= 64) return SDCSZ_EINVAL;
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
// per-field workspace layouts
// ---------------------------------------------------------------------------
struct CompLayout {
  uint64_t cnt, res, redo_n, hist, enc, tiles, zero_end, bits, bits_end;
  uint64_t eb, range, codes, vals, recon, meta, words, coef, sum_dc, sum_q, isum_q;
  uint64_t off_pay, off_out, off_coef, scan, tot, plan, redo, hdr, total;
};

// A fault plan's device area: the entries, then the blocks of the wave
// routine's list and of the fault-applying instantiation's list (one copy).
uint64_t plan_bytes(uint32_t nfaults) { return (sizeof(sdcsz_fault) + 16ull) * std::max<uint32_t>(nfaults, 1); }

uint64_t tiles_of(uint64_t nb) { return (nb + kEncTile - 1) / kEncTile; }

// The largest stream of a field: every value an outlier and a codeword of
// the longest length, every block a regression block, all 65,536 symbols.
uint64_t max_stream_size(const Geo &g, uint32_t dtype) {
  Header h;
  std::memset(&h, 0, sizeof(h));
  h.dtype = dtype;
  h.abft = 1;
  h.n_sym = 65536;
  h.n_blocks = g.n_blocks;
  h.n_regression = g.n_blocks;
  h.n_outliers = g.n_values;
  h.payload_words = (g.n_values * kMaxLen + 31) / 32 + g.n_blocks;
  section_offsets(h);
  return h.total;
}

CompLayout comp_layout(const Geo &g, uint32_t dtype, uint32_t nfaults) {
  CompLayout L;
  const uint64_t nb = g.n_blocks, vb = vbytes(dtype), slots = nb * g.bpts;
  const uint64_t chunks = (nb + scan_chunk(nb) - 1) / scan_chunk(nb) + 1;
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = at;
    at = a256(at + bytes);
    return o;
  };
  // cleared by one launch at the start of a call: counters, results, redo
  // count, histogram and codeword table
  // counters, results, redo count and the header bytes are adjacent: the
  // end of a call reads them back with one copy
  L.cnt = take(8 * C_N + 8 * R_N + 8 + kHeader);
  L.res = L.cnt + 8 * C_N;
  L.redo_n = L.res + 8 * R_N;
  L.hist = take(4 * 65536);
  L.enc = take(4 * 65536);
  L.tiles = take(8 * (tiles_of(nb) + 1));  // one-pass check and encoding: tile states, then the ticket
  L.zero_end = at;
  L.bits = take(4 * (nb / 32 + 1));  // a plan's blocks: cleared too when there is a plan
  L.bits_end = at;
  L.eb = take(sizeof(EbDev));
  L.range = take(16ull * kRangeBlocks);
  L.codes = take(2ull * 256 * g.groups * ((nb + 63) / 64));
  L.vals = take(vb * slots);
  L.recon = take(vb * ((nb + 63) / 64) * 64 * g.bpts);  // interleaved across 64 blocks
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
  L.plan = take(plan_bytes(nfaults));
  L.redo = take(24ull * kMaxRedo);  // block | reason, first-pass checksums
  L.hdr = take(sizeof(Header));
  L.total = at;
  return L;
}

struct DecLayout {
  uint64_t cnt, redo_n, err, zero_end, bits, bits_end;
  uint64_t symbols, tab, recon, off_pay, off_out, off_coef, scan, tot, plan, lut, lut2, sub, redo, hdr;
  uint64_t total;
};

// small_recon: no recon scratch (the specialised decoder and its
// re-execution keep blocks in registers; only the generic kernels stage
// values there, one slot per block, including the fallback that decodes a
// whole field again when more blocks fail than the re-execution queue holds).
DecLayout dec_layout(const Geo &g, uint32_t dtype, uint32_t nfaults, bool small_recon = false) {
  DecLayout L;
  const uint64_t nb = g.n_blocks, vb = vbytes(dtype);
  const uint64_t slots = small_recon ? 0 : (nb + 63) / 64 * 64;
  const uint64_t chunks = (nb + scan_chunk(nb) - 1) / scan_chunk(nb) + 1;
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
  L.bits = take(4 * (nb / 32 + 1));  // a plan's blocks: cleared too when there is a plan
  L.bits_end = at;
  L.symbols = take(2 * 65536);
  L.tab = take(sizeof(DecTab));
  L.recon = take(vb * slots * g.bpts);  // interleaved across 64 slots
  L.off_pay = take(8 * (nb + 1));
  L.off_out = take(4 * (nb + 1));
  L.off_coef = take(4 * (nb + 1));
  L.scan = take(24 * chunks);
  L.tot = take(24);
  L.plan = take(plan_bytes(nfaults));
  L.lut = take(4ull << kLutBits);
  L.lut2 = take(4ull << kLutBits);
  L.sub = take(4ull * kSubMax);
  L.redo = take(16ull * kMaxRedo);  // the production decoder's queue, then the fault-applying one's
  L.hdr = take(kHeader);
  L.total = at;
  return L;
}

// Block shapes with specialised kernels (one lane per block): class 0 is
// 6x6x6 in 3D, class 1 is 16x16 in 2D; -1 means the generic kernels.
constexpr int kClasses = 2;
// The specialised kernels address a field below 2 GiB from a wave-uniform
// base with 32-bit offsets; a wider field takes their "wide" instantiation
// (a base per lane at the block's origin), which needs the offsets inside a
// block to stay below 2^31 bytes.
bool wide_field(const Geo &g, uint32_t vb) { return g.n_values * vb >= (1ull << 31); }

int fast_class(const Geo &g, uint32_t vb) {
  if (!g.n_blocks) return -1;
  const uint64_t in_block =
      ((uint64_t)(g.b[0] - 1) * g.d[1] * g.d[2] + (uint64_t)(g.b[1] - 1) * g.d[2] + g.b[2]) * vb;
  if (in_block >= (1ull << 31)) return -1;
  if (g.ndim == 3 && g.b[0] == 6 && g.b[1] == 6 && g.b[2] == 6) return 0;
  if (g.ndim == 2 && g.b[1] == 16 && g.b[2] == 16) return 1;
  return -1;
}

using JobKernel = void (*)(JobTab);
// [class][dtype][abft][variant]: variant 0 narrow, 1 wide (fields of 2 GiB
// or more), 2 narrow with fault plans applied; 0 and 1 take the full blocks,
// 3 (narrow) and 4 (wide) the partial shell
#define SDCSZ_CF(T, ND, B0, B1, B2, A)                                                                       \
  {                                                                                                          \
    k_compress_fast<T, ND, B0, B1, B2, A, false, false, 1>, k_compress_fast<T, ND, B0, B1, B2, A, true, false, 1>, \
        k_compress_fast<T, ND, B0, B1, B2, A, false, true, 0>,                                               \
        k_compress_fast<T, ND, B0, B1, B2, A, false, false, 2>,                                              \
        k_compress_fast<T, ND, B0, B1, B2, A, true, false, 2>                                                \
  }
const JobKernel kCompFast[kClasses][2][2][5] = {
    {{SDCSZ_CF(float, 3, 6, 6, 6, false), SDCSZ_CF(float, 3, 6, 6, 6, true)},
     {SDCSZ_CF(double, 3, 6, 6, 6, false), SDCSZ_CF(double, 3, 6, 6, 6, true)}},
    {{SDCSZ_CF(float, 2, 1, 16, 16, false), SDCSZ_CF(float, 2, 1, 16, 16, true)},
     {SDCSZ_CF(double, 2, 1, 16, 16, false), SDCSZ_CF(double, 2, 1, 16, 16, true)}}};
#undef SDCSZ_CF
const JobKernel kCheckFast[kClasses] = {k_check_fast<3, 6, 6, 6>, k_check_fast<2, 1, 16, 16>};
// [class][dtype]
const JobKernel kEncFast[kClasses][2] = {{k_encode_fast<float, 3, 6, 6, 6>, k_encode_fast<double, 3, 6, 6, 6>},
                                         {k_encode_fast<float, 2, 1, 16, 16>, k_encode_fast<double, 2, 1, 16, 16>}};
// [class][dtype][variant]: 0 narrow, 1 wide, 2 narrow with fault plans applied
const JobKernel kDecFast[kClasses][2][3] = {
    {{k_decode_fast<float, 3, 6, 6, 6, false, false>, k_decode_fast<float, 3, 6, 6, 6, true, false>,
      k_decode_fast<float, 3, 6, 6, 6, false, true>},
     {k_decode_fast<double, 3, 6, 6, 6, false, false>, k_decode_fast<double, 3, 6, 6, 6, true, false>,
      k_decode_fast<double, 3, 6, 6, 6, false, true>}},
    {{k_decode_fast<float, 2, 1, 16, 16, false, false>, k_decode_fast<float, 2, 1, 16, 16, true, false>,
      k_decode_fast<float, 2, 1, 16, 16, false, true>},
     {k_decode_fast<double, 2, 1, 16, 16, false, false>, k_decode_fast<double, 2, 1, 16, 16, true, false>,
      k_decode_fast<double, 2, 1, 16, 16, false, true>}}};

// Lanes per work-group (one block per lane) of the specialised kernels, by
// stage, shape class and data type: the first entry whose max_blocks holds
// the launch's block count, 256 beyond the last (set by the autotuner).
constexpr int kTuneStages = 4;  // prediction/quantization, code check, encoding, decoding
enum { TS_PREDICT, TS_CHECK, TS_ENCODE, TS_DECODE };
struct TuneRow {
  uint32_t n = 0;
  uint64_t max_blocks[SDCSZ_TUNE_MAX] = {};
  uint32_t lanes[SDCSZ_TUNE_MAX] = {};
};
TuneRow g_tune[kTuneStages][kClasses][2];

uint32_t tuned_lanes(int stage, int cls, uint32_t dtype, uint64_t blocks) {
  const TuneRow &r = g_tune[stage][cls][dtype];
  for (uint32_t i = 0; i < r.n; i++)
    if (blocks <= r.max_blocks[i]) return r.lanes[i];
  return 256;
}

// One launch of a specialised kernel: the first work-groups take the
// sub-grid of full blocks, the others the shell of partial blocks along the
// upper faces.  Returns the number of work-groups of `lanes` lanes.
uint32_t fast_launch(const Geo &g, Launch *L, uint32_t lanes) {
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
  L->full_wgs = (uint32_t)((L->full_count + lanes - 1) / lanes);
  return L->full_wgs + (uint32_t)((L->shell_count + lanes - 1) / lanes);
}

uint32_t scan_chunks(uint64_t nb) { return (uint32_t)((nb + scan_chunk(nb) - 1) / scan_chunk(nb)); }

// ---------------------------------------------------------------------------
// pinned host staging of the calling thread (grown on demand, kept until the
// process ends): job tables go to the device and histograms, headers and
// results come back through it
// ---------------------------------------------------------------------------
struct Staging {
  uint8_t *p = nullptr;
  size_t cap = 0;
  bool fixed = false;  // a caller-provided buffer: never grown nor freed
  // only called between calls or after a synchronisation (no copy in flight);
  // starts at 8 MiB (a field's histogram pairs and codebook list need up to
  // about 1 MiB) and at least doubles, so regrowing (a device-wide wait in
  // hipHostFree plus a new pinned allocation) stays rare
  uint8_t *get(size_t n) {
    if (fixed) return n <= cap ? p : nullptr;
    if (n > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      const size_t want = std::max<size_t>({n, 2 * cap, size_t(8) << 20});
      cap = 0;
      if (hipHostMalloc((void **)&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
      cap = want;
    }
    return p;
  }
  ~Staging() {
    if (p && !fixed) (void)hipHostFree(p);
  }
};
thread_local Staging t_stage;

// A second stream of the calling thread (default priority, made on first use
// on a device and kept until the thread exits): a call's fault-plan work
// (and, on another one, the compressor's partial shells) runs there beside
// the main launch, between a fork and a join event.
struct SideStream {
  int dev = -1;
  hipStream_t s = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  void drop() {
    if (s) (void)hipStreamDestroy(s);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    s = nullptr;
    fork_ev = join_ev = nullptr;
    dev = -1;
  }
  // the side stream, after the work queued so far on `main`; null on error
  hipStream_t fork(hipStream_t main) {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return nullptr;
    if (d != dev) {
      drop();
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&join_ev, hipEventDisableTiming) != hipSuccess) {
        drop();
        return nullptr;
      }
      dev = d;
    }
    if (hipEventRecord(fork_ev, main) != hipSuccess || hipStreamWaitEvent(s, fork_ev, 0) != hipSuccess) return nullptr;
    return s;
  }
  // `main` waits for the side stream's work
  hipError_t join(hipStream_t main) {
    hipError_t e = hipEventRecord(join_ev, s);
    return e != hipSuccess ? e : hipStreamWaitEvent(main, join_ev, 0);
  }
  ~SideStream() { drop(); }
};
thread_local SideStream t_side;
thread_local SideStream t_shell_side;  // compression: the partial shells of the specialised launches
// calls that must not create resources run their plan and shell work on the main stream
thread_local bool t_no_side = false;
// the staging of decompression calls: the thread's own, unless a call that
// must not allocate has put a fixed buffer in its place
thread_local Staging *t_stage_over = nullptr;
Staging &dec_stage() { return t_stage_over ? *t_stage_over : t_stage; }

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

void fill_report(sdcsz_report *r, const uint64_t *cnt, uint64_t nb) {
  std::memset(r, 0, sizeof(*r));
  r->n_blocks = nb;
  for (int t = 0; t < SDCSZ_N_TARGETS; t++) {
    r->injected[t] = cnt[C_INJ + t];
    r->detected[t] = cnt[C_DET + t];
    r->corrected[t] = cnt[C_COR + t];
    r->uncorrectable[t] = cnt[C_UNC + t];
  }
  r->generic_plan_blocks = cnt[C_LIST];
}

// The blocks of a sorted plan on a field of the lane-per-block kernels,
// split between the wave-per-block routine (out) and the lane-per-block
// kernels' fault-applying instantiation (fast).  The wave routine takes all
// of them when the launch cannot apply plans (faults_ok false: the wide
// instantiation), else those whose entries the fault-applying instantiation
// does not model: errors of the prediction
// preparation, more than one flip of a kind, or a flip of the duplicated
// reconstruction together with an input or prediction flip (compression:
// the specialised pass meets the reconstruction flip with the earlier error
// still in its values, where the paper-order routine has corrected it, and
// whether a reconstruction is computed at all depends on those values), more
// than one RECON flip (decompression).
void split_plan(const std::vector<sdcsz_fault> &plan, bool faults_ok, bool decomp, std::vector<uint64_t> &out,
                std::vector<uint64_t> &fast) {
  out.clear();
  fast.clear();
  for (size_t i = 0; i < plan.size();) {
    size_t j = i;
    uint32_t cnt[SDCSZ_N_TARGETS] = {};
    for (; j < plan.size() && plan[j].block == plan[i].block; j++) cnt[plan[j].target]++;
    bool gen = !faults_ok;
    if (decomp) gen = gen || cnt[SDCSZ_T_RECON] > 1;
    else
      gen = gen || cnt[SDCSZ_T_PREP_INPUT] || cnt[SDCSZ_T_PREP_COEF] || cnt[SDCSZ_T_PREP_SAMPLE] ||
            cnt[SDCSZ_T_INPUT] > 1 || cnt[SDCSZ_T_COEF] > 1 || cnt[SDCSZ_T_DUP_PRED] > 1 ||
            cnt[SDCSZ_T_DUP_RECON] > 1 || (cnt[SDCSZ_T_DUP_RECON] && (cnt[SDCSZ_T_INPUT] || cnt[SDCSZ_T_DUP_PRED]));
    (gen ? out : fast).push_back(plan[i].block);
    i = j;
  }
}

// One pageable copy of a plan's entries and block lists to its device area;
// fills the job's PlanDev (its bitmap is set on the device by k_plan_bits).
hipError_t upload_plan(const std::vector<sdcsz_fault> &plan, const std::vector<uint64_t> &pb,
                       const std::vector<uint64_t> &fl, std::vector<uint8_t> &buf, uint8_t *dev, PlanDev &P,
                       hipStream_t st) {
  const size_t eb = plan.size() * sizeof(sdcsz_fault);
  buf.resize(eb + 8 * (pb.size() + fl.size()));
  std::memcpy(buf.data(), plan.data(), eb);
  if (!pb.empty()) std::memcpy(buf.data() + eb, pb.data(), 8 * pb.size());
  if (!fl.empty()) std::memcpy(buf.data() + eb + 8 * pb.size(), fl.data(), 8 * fl.size());
  P.list = (const uint64_t *)(dev + eb);
  P.nlist = (uint32_t)pb.size();
  P.flist = (const uint64_t *)(dev + eb) + pb.size();
  P.nflist = (uint32_t)fl.size();
  return hipMemcpyAsync(dev, buf.data(), buf.size(), hipMemcpyHostToDevice, st);
}


// ---------------------------------------------------------------------------
// launch tables: the jobs of one launch and the work-groups each owns
// ---------------------------------------------------------------------------
struct Tab {
  std::vector<uint32_t> wg{0}, id;
  void add(uint32_t job, uint64_t wgs) {
    if (!wgs) return;
    id.push_back(job);
    wg.push_back(wg.back() + (uint32_t)wgs);
  }
  uint32_t total() const { return wg.back(); }
  uint32_t n() const { return (uint32_t)id.size(); }
};

// The jobs and the launch tables of one stage, laid out in pinned memory and
// copied to the batch area of the workspace with one transfer.
struct Upload {
  std::vector<Tab *> tabs;
  std::vector<JobTab> dev;
  size_t bytes(size_t njobs) const {
    size_t b = a256(sizeof(Job) * njobs);
    for (auto *t : tabs) b += 4 * (t->wg.size() + t->id.size());
    return a256(b);
  }
  // writes jobs + tables at host[0..) for device address dbase; fills dev[]
  void place(const std::vector<Job> &jobs, uint8_t *host, uint8_t *dbase) {
    std::memcpy(host, jobs.data(), sizeof(Job) * jobs.size());
    size_t at = a256(sizeof(Job) * jobs.size());
    dev.clear();
    for (auto *t : tabs) {
      JobTab jt;
      jt.jobs = (const Job *)dbase;
      jt.n = t->n();
      std::memcpy(host + at, t->wg.data(), 4 * t->wg.size());
      jt.wg = (const uint32_t *)(dbase + at);
      at += 4 * t->wg.size();
      std::memcpy(host + at, t->id.data(), 4 * t->id.size());
      jt.id = (const uint32_t *)(dbase + at);
      at += 4 * t->id.size();
      dev.push_back(jt);
    }
  }
};

// A phase's launches (one per kernel class), the first recording the
// phase's start event and the last its stop event.
struct PhaseLaunch {
  int ph;
  std::vector<std::function<void(bool, bool)>> fs;
  void run() {
    for (size_t i = 0; i < fs.size(); i++) fs[i](i == 0, i + 1 == fs.size());
  }
};

// ---------------------------------------------------------------------------
// Huffman codebooks of a batch, built on host threads
// ---------------------------------------------------------------------------
struct CodebookJob {
  const uint64_t *pairs;  // (symbol << 32 | count), ascending symbols
  uint32_t n;
  uint32_t *out;          // n pairs (symbol << 8 | length, codeword)
};

void build_codebook(const CodebookJob &c, HuffmanBuilder &b, std::vector<uint64_t> &cnt, std::vector<uint8_t> &len,
                    std::vector<uint32_t> &code) {
  cnt.resize(c.n);
  for (uint32_t i = 0; i < c.n; i++) cnt[i] = c.pairs[i] & 0xFFFFFFFFull;
  b.lengths(cnt, kMaxLen, len);
  canonical_codes(len, kMaxLen, code);
  for (uint32_t i = 0; i < c.n; i++) {
    c.out[2 * i] = ((uint32_t)(c.pairs[i] >> 32) << 8) | len[i];
    c.out[2 * i + 1] = code[i];
  }
}

// Threads take the fields largest first from a shared counter, so that the
// few fields with tens of thousands of symbols start at once and the small
// ones fill in around them.
void build_codebooks(const std::vector<CodebookJob> &cj) {
  uint64_t work = 0;
  for (auto &c : cj) work += c.n;
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const unsigned nt = (unsigned)std::min<uint64_t>(hw, std::max<uint64_t>(1, std::min<uint64_t>(cj.size(), work / 4096)));
  std::vector<uint32_t> order(cj.size());
  for (uint32_t i = 0; i < order.size(); i++) order[i] = i;
  if (nt > 1) std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cj[a].n > cj[b].n; });
  std::atomic<size_t> next{0};
  auto run = [&](unsigned) {
    HuffmanBuilder b;
    std::vector<uint64_t> cnt;
    std::vector<uint8_t> len;
    std::vector<uint32_t> code;
    for (size_t k; (k = next.fetch_add(1)) < order.size();) build_codebook(cj[order[k]], b, cnt, len, code);
  };
  if (nt <= 1) {
    run(0);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; t++) th.emplace_back(run, t);
  run(0);
  for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------
// compression of a batch of fields
// ---------------------------------------------------------------------------
struct CompItem {  // one field of a compression call
  const void *d_in;
  const sdcsz_params *p;
  uint8_t *d_out;
  uint64_t out_cap;
  uint64_t out_size;
  int rc;
  sdcsz_report rep;
  uint8_t header[kHeader];  // the stream's header, when written
};

// Histogram entries returned with the first synchronisation (the rest, if
// any, take a second one): twice the last call's total on this thread, or
// half the previous guess if that is more (at least kPairMin), so that a
// steady workload copies little more than it needs and a mixed one rarely
// takes the second round trip.
constexpr uint64_t kPairPrefix = 32768;  // guess of a thread's first call
constexpr uint64_t kPairMin = 4096;
thread_local uint64_t t_pair_guess = kPairPrefix;
// u64 words per field read back at the end of a compression: counters,
// results, redo count, header bytes
constexpr uint32_t kResWords = C_N + R_N + 1 + kHeader / 8;

struct CompPlan {  // host state of one field
  Geo g;
  CompLayout L;
  uint8_t *ws;
  bool fast;
  int cls;  // shape class of the specialised kernels, -1 for generic
  std::vector<sdcsz_fault> plan;
  std::vector<uint64_t> pb;  // blocks the wave-per-block routine takes (k_compress_wave_list)
  std::vector<uint64_t> fl;  // blocks the fault-applying instantiation takes
  std::vector<uint8_t> up;   // plan area as uploaded (entries, pb, fl)
  bool any_code;
  bool fused;         // code check and encoding in one pass (k_checkenc_fast)
  uint64_t pair_off;  // first entry of the field's histogram / codebook list
};


// work-groups per field of the re-execution kernels: the queue is almost
// always empty, and on a large batch thousands of work-groups that only
// find it empty cost tens of microseconds
constexpr uint32_t kRedoWgs = 8;

struct BatchArea {  // device batch area and its size
  uint64_t jobs, cb, counts, pairs, chunks, res, total;
};

constexpr uint32_t kHistChunks = 64;  // histogram chunks per field (k_hist_*)

// jobs + up to 32 launch tables of (2 n + 1) entries
uint64_t jobs_region(uint64_t njobs) { return a256(sizeof(Job) * njobs) + 32 * a256(4 * (2 * njobs + 1)); }

BatchArea comp_batch_area(uint64_t njobs, uint64_t cap_pairs) {
  BatchArea B;
  uint64_t at = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = at;
    at = a256(at + bytes);
    return o;
  };
  B.jobs = take(jobs_region(njobs));
  B.cb = B.jobs + jobs_region(njobs);  // right after the tables: one upload carries both
  at = a256(B.cb + 8 * cap_pairs);
  B.counts = take(4 * njobs + 8);      // the pairs follow right after, for one copy back
  B.pairs = B.counts + ((4 * njobs + 7) & ~7ull);
  at = a256(B.pairs + 8 * cap_pairs);
  B.chunks = take(4ull * kHistChunks * njobs);
  B.res = take(8ull * kResWords * njobs);
  B.total = at;
  return B;
}

uint64_t pair_cap(const Geo &g) { return std::min<uint64_t>(65536, g.n_values + 1); }

// workspace of a batch: the batch area, then each valid field's area
uint64_t comp_batch_ws(const CompItem *it, uint32_t n) {
  uint64_t per = 0, cap = 0, nj = 0;
  for (uint32_t i = 0; i < n; i++) {
    Geo g;
    if (check_params(it[i].p, &g)) continue;
    per += comp_layout(g, it[i].p->dtype, it[i].p->n_faults).total;
    cap += pair_cap(g);
    nj++;
  }
  return comp_batch_area(nj, cap).total + per;
}

template <typename T> void fill_rt(Job &J) {
  if (sizeof(T) == 4) J.rtf = reg_table<float>(J.g);
  else J.rtd = reg_table<double>(J.g);
}

int compress_batch(CompItem *it, uint32_t n, uint8_t *ws, uint64_t ws_size, hipStream_t st) {
  HostSpan call(PH_HOST_CALL);
  // ---- validation and layouts
  std::vector<CompPlan> fp;
  std::vector<uint32_t> item_of;  // job -> item
  uint64_t cap = 0, per = 0;
  for (uint32_t i = 0; i < n; i++) {
    CompItem &c = it[i];
    c.out_size = 0;
    std::memset(&c.rep, 0, sizeof(c.rep));
    CompPlan f;
    c.rc = check_params(c.p, &f.g);
    if (!c.rc && f.g.n_values && !c.d_in) c.rc = SDCSZ_EINVAL;
    if (!c.rc) c.rc = check_plan(f.g, c.p->dtype, c.p->faults, c.p->n_faults, false, f.plan);
    if (c.rc) continue;
    f.L = comp_layout(f.g, c.p->dtype, c.p->n_faults);
    f.cls = fast_class(f.g, vbytes(c.p->dtype));
    f.fast = f.cls >= 0;
    // the one-pass check and encoding writes the stream before it knows the
    // stream's size: only into an output that holds the largest one
    f.fused = f.cls == 0 && f.g.n_blocks > 0 && c.d_out && c.out_cap >= max_stream_size(f.g, c.p->dtype);
    f.any_code = false;
    for (auto &e : f.plan) f.any_code |= e.target == SDCSZ_T_CODE;
    f.pair_off = cap;
    cap += pair_cap(f.g);
    per += f.L.total;
    fp.push_back(std::move(f));
    item_of.push_back(i);
  }
  const uint32_t nj = (uint32_t)fp.size();
  if (nj == 0) return SDCSZ_OK;
  const BatchArea B = comp_batch_area(nj, cap);
  if (!ws || ws_size < B.total + per) {
    for (uint32_t j = 0; j < nj; j++) it[item_of[j]].rc = SDCSZ_ENOSPC;
    return SDCSZ_ENOSPC;
  }
  // a launch with a field of 2 GiB or more takes the wide kernel, which
  // applies no fault plan: its fields' plan blocks take the generic routine
  bool wide_fast[kClasses][2][2] = {};
  for (uint32_t j = 0; j < nj; j++) {
    const sdcsz_params *p = it[item_of[j]].p;
    if (fp[j].fast) wide_fast[fp[j].cls][p->dtype][p->abft ? 1 : 0] |= wide_field(fp[j].g, vbytes(p->dtype));
  }
  for (uint32_t j = 0; j < nj; j++) {
    CompPlan &f = fp[j];
    const sdcsz_params *p = it[item_of[j]].p;
    if (!f.fast || f.plan.empty()) continue;
    const bool wide = wide_fast[f.cls][p->dtype][p->abft ? 1 : 0];
    split_plan(f.plan, !wide, false, f.pb, f.fl);
  }
  // ---- jobs
  std::vector<Job> jobs(nj);
  uint64_t at = B.total;
  for (uint32_t j = 0; j < nj; j++) {
    CompPlan &f = fp[j];
    const CompItem &c = it[item_of[j]];
    f.ws = ws + at;
    at += f.L.total;
    Job &J = jobs[j];
    std::memset(&J, 0, sizeof(J));
    uint8_t *w = f.ws;
    J.g = f.g;
    CompWork &cw = J.cw;
    cw.codes = (uint16_t *)(w + f.L.codes);
    cw.vals = w + f.L.vals;
    cw.recon = w + f.L.recon;
    cw.meta = (uint32_t *)(w + f.L.meta);
    cw.words = (uint32_t *)(w + f.L.words);
    cw.coef = w + f.L.coef;
    cw.sum_dc = (uint64_t *)(w + f.L.sum_dc);
    cw.sum_q = (uint64_t *)(w + f.L.sum_q);
    cw.isum_q = (uint64_t *)(w + f.L.isum_q);
    cw.hist = (uint32_t *)(w + f.L.hist);
    cw.enc = (uint32_t *)(w + f.L.enc);
    cw.cnt = (unsigned long long *)(w + f.L.cnt);
    cw.off_pay = (uint64_t *)(w + f.L.off_pay);
    cw.off_out = (uint32_t *)(w + f.L.off_out);
    cw.off_coef = (uint32_t *)(w + f.L.off_coef);
    cw.scan_part = (uint64_t *)(w + f.L.scan);
    cw.range_part = w + f.L.range;
    cw.eb = (EbDev *)(w + f.L.eb);
    cw.redo_n = (uint32_t *)(w + f.L.redo_n);
    cw.redo = (uint64_t *)(w + f.L.redo);
    cw.hdr = (Header *)(w + f.L.hdr);
    cw.hdr_bytes = w + f.L.redo_n + 8;
    cw.res = (uint64_t *)(w + f.L.res);
    cw.cb = (uint32_t *)(ws + B.cb) + 2 * f.pair_off;
    cw.tot = (uint64_t *)(w + f.L.tot);
    cw.tiles = (uint64_t *)(w + f.L.tiles);
    cw.ticket = (uint32_t *)(cw.tiles + tiles_of(f.g.n_blocks));
    J.plan.n = (uint32_t)f.plan.size();
    J.plan.f = (const sdcsz_fault *)(w + f.L.plan);
    J.plan.bits = (const uint32_t *)(w + f.L.bits);
    J.plan.list = J.plan.flist = nullptr;
    J.plan.nlist = J.plan.nflist = 0;
    Header &h = J.h;
    h.dtype = c.p->dtype;
    h.ndim = c.p->ndim;
    for (int a = 0; a < 3; a++) {
      h.d[a] = f.g.d[a];
      h.b[a] = f.g.b[a];
    }
    h.eb_mode = c.p->eb_mode;
    h.eb = c.p->eb;
    h.abft = c.p->abft;
    h.n_blocks = f.g.n_blocks;
    h.predictor = c.p->predictor;
    // a one-pass field scans its outliers and regression blocks in stage A
    // (no payload words yet); the others scan all three after the check
    J.ss = ScanSrc{f.fused ? nullptr : cw.words, cw.meta, 1};
    J.sc_part = cw.scan_part;
    J.sc_off_pay = cw.off_pay;
    J.sc_off_out = cw.off_out;
    J.sc_off_coef = cw.off_coef;
    J.sc_tot = cw.tot;
    J.src = (const uint8_t *)c.d_in;
    J.dst = c.d_out;
    J.dst_cap = c.d_out ? c.out_cap : 0;
    J.zero = (uint32_t *)(w + f.L.cnt);
    J.zero_words = ((f.plan.empty() ? f.L.zero_end : f.L.bits_end) - f.L.cnt) / 4;
    J.stat = (const uint64_t *)(w + f.L.cnt);
    J.stat_words = kResWords;
    J.eb = c.p->eb;
    J.dtype = c.p->dtype;
    J.abft = c.p->abft;
    J.predictor = c.p->predictor;
    J.eb_mode = c.p->eb_mode;
    J.nparts = (c.p->eb_mode == SDCSZ_REL && f.g.n_values)
                   ? (uint32_t)std::min<uint64_t>(kRangeBlocks, grid_for(f.g.n_values, kRangeThreads * 8))
                   : 1u;
    // LDS histogram window of the compression kernel: the codes of loose
    // value-range bounds stay within +-1024 of the zero residual; tighter
    // (and absolute) bounds spread further, and codes outside the window cost
    // a global atomic each
    J.hist_win = c.p->eb_mode != SDCSZ_REL ? 8192u : c.p->eb >= 5e-4 ? 2048u : c.p->eb >= 5e-5 ? 8192u : kHistWin;
    if (J.dtype == SDCSZ_F32) fill_rt<float>(J);
    else fill_rt<double>(J);
    // fault plans: entries and block lists in one copy (the pageable source
    // lives in fp until the first synchronisation); the block bitmap is set
    // on the device
    if (!f.plan.empty()) {
      HIPCHK(upload_plan(f.plan, f.pb, f.fl, f.up, w + f.L.plan, J.plan, st));
    }
  }
  // ---- stage A tables: zero, range + constants, prediction/quantization,
  // re-runs, histogram compaction
  // t_gen: one thread per block; t_wave, t_wlist, t_redo: a wave per block;
  // t_flist: the fault-applying instantiation over the plans' lists
  Tab t_zero, t_plan, t_range[2], t_fast[kClasses][2][2], t_flist[kClasses][2][2], t_gen[2], t_wave[2], t_wlist[2],
      t_redo[2], t_hist, t_hchunk, t_sa;  // t_sa: the stage-A scans of one-pass fields
  Tab t_shell[kClasses][2][2];  // the partial shells of the t_fast launches, beside them
  uint32_t lds_wlist[2] = {}, lds_redo[2] = {};  // dynamic LDS of the wave launches
  uint32_t slice_wave[2] = {}, hw_wave[2] = {};  // k_compress_wave: widest block slice and histogram window
  uint64_t nb_fast[kClasses][2][2] = {}, nb_cls[kClasses] = {}, nb_enc[kClasses][2] = {};
  uint32_t hw_fast[kClasses][2][2] = {};  // widest histogram window of each launch
  for (uint32_t j = 0; j < nj; j++)
    if (fp[j].fast) {
      uint32_t &hw = hw_fast[fp[j].cls][jobs[j].dtype][jobs[j].abft ? 1 : 0];
      hw = std::max(hw, jobs[j].hist_win);
      nb_fast[fp[j].cls][jobs[j].dtype][jobs[j].abft ? 1 : 0] += fp[j].g.n_blocks;
      nb_cls[fp[j].cls] += fp[j].g.n_blocks;
      nb_enc[fp[j].cls][jobs[j].dtype] += fp[j].g.n_blocks;
    }
  uint32_t ln_fast[kClasses][2][2], ln_chk[kClasses], ln_enc[kClasses][2];
  for (int c = 0; c < kClasses; c++) {
    ln_chk[c] = tuned_lanes(TS_CHECK, c, 0, nb_cls[c]);
    for (int d = 0; d < 2; d++) {
      ln_enc[c][d] = tuned_lanes(TS_ENCODE, c, d, nb_enc[c][d]);
      for (int a = 0; a < 2; a++) ln_fast[c][d][a] = tuned_lanes(TS_PREDICT, c, d, nb_fast[c][d][a]);
    }
  }
  for (uint32_t j = 0; j < nj; j++) {
    Job &J = jobs[j];
    const CompPlan &f = fp[j];
    t_zero.add(j, std::min<uint64_t>(64, grid_for(J.zero_words, 256)));
    if (!f.plan.empty()) t_plan.add(j, grid_for(f.plan.size(), 256));
    if (J.eb_mode == SDCSZ_REL && f.g.n_values) t_range[J.dtype].add(j, J.nparts);
    if (f.fast) {
      const int a = J.abft ? 1 : 0;
      const uint32_t nwg = fast_launch(f.g, &J.L, ln_fast[f.cls][J.dtype][a]);
      t_fast[f.cls][J.dtype][a].add(j, J.L.full_wgs);
      t_shell[f.cls][J.dtype][a].add(j, nwg - J.L.full_wgs);
      if (!f.fl.empty()) t_flist[f.cls][J.dtype][a].add(j, grid_for(f.fl.size(), 64));
      const uint32_t lb = wave_lds_bytes(f.g, vbytes(J.dtype));
      if (J.abft) {
        t_redo[J.dtype].add(j, kRedoWgs);
        lds_redo[J.dtype] = std::max(lds_redo[J.dtype], lb);
      }
      if (!f.pb.empty()) {
        t_wlist[J.dtype].add(j, f.pb.size());
        lds_wlist[J.dtype] = std::max(lds_wlist[J.dtype], lb);
      }
    } else if (f.g.n_blocks) {
      const uint32_t lb = wave_slice_bytes(f.g, vbytes(J.dtype));
      if (lb <= kWaveLdsMax) {
        t_wave[J.dtype].add(j, std::min<uint64_t>(kWaveWgMax, (f.g.n_blocks + kWaveWgWaves - 1) / kWaveWgWaves));
        slice_wave[J.dtype] = std::max(slice_wave[J.dtype], lb);
        hw_wave[J.dtype] = std::max(hw_wave[J.dtype], J.hist_win);
      } else {
        t_gen[J.dtype].add(j, grid_for(f.g.n_blocks, 64));
      }
    }
    t_hist.add(j, 1);
    t_hchunk.add(j, kHistChunks);
    if (f.fused) t_sa.add(j, scan_chunks(f.g.n_blocks));
  }
  Upload up;
  up.tabs = {&t_zero,     &t_range[0], &t_range[1], &t_gen[0],  &t_gen[1],  &t_hist,    &t_hchunk,
             &t_wave[0],  &t_wave[1],  &t_wlist[0], &t_wlist[1], &t_redo[0], &t_redo[1], &t_plan};
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++)
      for (int a = 0; a < 2; a++) up.tabs.push_back(&t_fast[c][d][a]);
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++)
      for (int a = 0; a < 2; a++) up.tabs.push_back(&t_flist[c][d][a]);
  up.tabs.push_back(&t_sa);
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++)
      for (int a = 0; a < 2; a++) up.tabs.push_back(&t_shell[c][d][a]);
  // the histogram kernels also write the counts and the first `pre` pairs
  // straight into this pinned staging, laid out as the device's counts and
  // pairs (so no copy is queued after them)
  const uint64_t head = B.pairs - B.counts;
  const uint64_t pre = std::min<uint64_t>(t_pair_guess, cap);
  uint8_t *hs = t_stage.get(std::max<size_t>(up.bytes(nj), head + 8 * pre + 64));
  if (!hs) return SDCSZ_EHIP;
  up.place(jobs, hs, ws + B.jobs);
  HIPCHK(hipMemcpyAsync(ws + B.jobs, hs, up.bytes(nj), hipMemcpyHostToDevice, st));
  const JobTab &d_zero = up.dev[0];
  const JobTab *d_range = &up.dev[1];
  const JobTab *d_gen = &up.dev[3];
  const JobTab &d_hist = up.dev[5];
  const JobTab &d_hchunk = up.dev[6];
  const JobTab *d_wave = &up.dev[7], *d_wlist = &up.dev[9], *d_redo = &up.dev[11];  // [dtype]
  const JobTab &d_plan = up.dev[13];
  const JobTab *d_fast = &up.dev[14];                       // [class][dtype][abft] in that order
  const JobTab *d_flist = &up.dev[14 + kClasses * 2 * 2];  // the same
  const JobTab &d_sa = up.dev[14 + 2 * kClasses * 2 * 2];
  const JobTab *d_shell = &up.dev[15 + 2 * kClasses * 2 * 2];  // [class][dtype][abft]
  auto grid = [](const Tab &t) { return dim3(t.total()); };
  launch(PH_NONE, false, false, k_zero_jobs, grid(t_zero), dim3(256), st, d_zero);
  if (t_plan.total()) launch(PH_NONE, false, false, k_plan_bits, grid(t_plan), dim3(256), st, d_plan);
  {
    PhaseLaunch pl{PH_RANGE, {}};
    if (t_range[0].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_RANGE, a, b, k_range<float>, grid(t_range[0]), dim3(kRangeThreads), st, d_range[0]); });
    if (t_range[1].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_RANGE, a, b, k_range<double>, grid(t_range[1]), dim3(kRangeThreads), st, d_range[1]); });
    pl.run();
  }
  launch(PH_NONE, false, false, k_consts, grid(t_hist), dim3(kRangeThreads), st, d_hist);
  // plan blocks, which the production kernels leave, beside them on a second
  // stream: the fault-applying instantiation over its lists, a wave per
  // block for the others; the partial shell of the specialised launches on
  // a third stream
  bool side_work = t_wlist[0].total() || t_wlist[1].total(), shell_work = false;
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++)
      for (int a = 0; a < 2; a++) {
        side_work |= t_flist[c][d][a].total() != 0;
        shell_work |= t_shell[c][d][a].total() != 0;
      }
  if (shell_work) {
    hipStream_t s2 = st;
    if (!t_no_side) {
      s2 = t_shell_side.fork(st);
      if (!s2) return SDCSZ_EHIP;
    }
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++)
        for (int a = 1; a >= 0; a--)
          if (t_shell[c][d][a].total())
            launch_shm(PH_NONE, false, false, kCompFast[c][d][a][wide_fast[c][d][a] ? 4 : 3], grid(t_shell[c][d][a]),
                       dim3(ln_fast[c][d][a]), 4 * hw_fast[c][d][a], s2, d_shell[(c * 2 + d) * 2 + a]);
  }
  hipStream_t side = st;
  if (side_work) {
    if (!t_no_side) {
      side = t_side.fork(st);
      if (!side) return SDCSZ_EHIP;
    }
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++)
        for (int a = 0; a < 2; a++)
          if (t_flist[c][d][a].total())
            launch_shm(PH_NONE, false, false, kCompFast[c][d][a][2], grid(t_flist[c][d][a]), dim3(64),
                       4 * hw_fast[c][d][a], side, d_flist[(c * 2 + d) * 2 + a]);
    if (t_wlist[0].total())
      launch_shm(PH_NONE, false, false, k_compress_wave_list<float>, grid(t_wlist[0]), dim3(64), lds_wlist[0], side,
                 d_wlist[0]);
    if (t_wlist[1].total())
      launch_shm(PH_NONE, false, false, k_compress_wave_list<double>, grid(t_wlist[1]), dim3(64), lds_wlist[1], side,
                 d_wlist[1]);
  }
  {
    PhaseLaunch pl{PH_PREDICT, {}};
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++)
        for (int a = 1; a >= 0; a--) {
          const Tab &t = t_fast[c][d][a];
          if (!t.total()) continue;
          const JobTab jt = d_fast[(c * 2 + d) * 2 + a];
          const JobKernel k = kCompFast[c][d][a][wide_fast[c][d][a] ? 1 : 0];
          const uint32_t ln = ln_fast[c][d][a], shm = 4 * hw_fast[c][d][a];
          pl.fs.push_back([&t, jt, k, ln, shm, st, &grid](bool x, bool y) {
            launch_shm(PH_PREDICT, x, y, k, grid(t), dim3(ln), shm, st, jt);
          });
        }
    for (int d = 0; d < 2; d++) {
      if (!t_wave[d].total()) continue;
      // as many waves per work-group (up to 4) as the LDS holds
      uint32_t nwv = kWaveWgWaves;
      while (nwv > 1 && nwv * slice_wave[d] + 4 * hw_wave[d] > kWaveWgLds) nwv--;
      const uint32_t shm = nwv * slice_wave[d] + 4 * hw_wave[d], slice = slice_wave[d];
      const JobTab jt = d_wave[d];
      const Tab &t = t_wave[d];
      const auto k = d == 0 ? k_compress_wave<float> : k_compress_wave<double>;
      pl.fs.push_back([&t, jt, k, nwv, shm, slice, st, &grid](bool a, bool b) {
        launch_shm(PH_PREDICT, a, b, k, grid(t), dim3(64 * nwv), shm, st, jt, slice);
      });
    }
    if (t_gen[0].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_PREDICT, a, b, k_compress_generic<float>, grid(t_gen[0]), dim3(64), st, d_gen[0]); });
    if (t_gen[1].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_PREDICT, a, b, k_compress_generic<double>, grid(t_gen[1]), dim3(64), st, d_gen[1]); });
    pl.run();
  }
  if (side_work && !t_no_side) HIPCHK(t_side.join(st));
  if (shell_work && !t_no_side) HIPCHK(t_shell_side.join(st));
  if (t_redo[0].total())
    launch_shm(PH_NONE, false, false, k_redo_wave<float>, grid(t_redo[0]), dim3(64), lds_redo[0], st, d_redo[0]);
  if (t_redo[1].total())
    launch_shm(PH_NONE, false, false, k_redo_wave<double>, grid(t_redo[1]), dim3(64), lds_redo[1], st, d_redo[1]);
  for (uint32_t j = 0; j < nj; j++)
    if (fp[j].any_code)
      launch(PH_CODEFAULT, true, true, k_code_faults, dim3(1), dim3(64), st, jobs[j].plan, jobs[j].g,
             jobs[j].cw.codes, jobs[j].cw.cnt);
  // one-pass fields: offsets and totals of the outliers and regression
  // blocks (final once the re-runs are done)
  if (t_sa.total()) {
    launch(PH_NONE, false, false, k_scan1, grid(t_sa), dim3(kScanThreads), st, d_sa);
    launch(PH_NONE, false, false, k_scan3, grid(t_sa), dim3(kScanThreads), st, d_sa);
  }
  uint32_t *d_counts = (uint32_t *)(ws + B.counts);
  uint64_t *d_pairs = (uint64_t *)(ws + B.pairs);
  uint32_t *d_chunks = (uint32_t *)(ws + B.chunks);
  launch(PH_NONE, false, false, k_hist_count, grid(t_hchunk), dim3(256), st, d_hchunk, d_chunks);
  launch(PH_NONE, false, false, k_hist_scan, dim3(1), dim3(256), st, nj, d_chunks, d_counts, (uint32_t *)hs);
  launch(PH_NONE, false, false, k_hist_pack, grid(t_hchunk), dim3(256), st, d_hchunk, (const uint32_t *)d_chunks,
         d_pairs, (uint64_t *)(hs + head), pre);
  HIPCHK(hipGetLastError());

  // ---- histograms back (the counts and the first t_pair_guess entries,
  // written into the staging by the kernels)
  HIPCHK(sync_wait(st));
  std::vector<uint32_t> cnt_sym((const uint32_t *)hs, (const uint32_t *)hs + nj);
  uint64_t total_pairs = 0;
  for (uint32_t j = 0; j < nj; j++) total_pairs += cnt_sym[j];
  t_pair_guess = std::max<uint64_t>({kPairMin, 2 * total_pairs, t_pair_guess / 2});
  // pinned room, in stage B: [jobs and tables | codebook lists] (one upload,
  // mirroring the device batch area), then the histogram pairs, then results
  const uint64_t JR = jobs_region(nj);
  const uint64_t at_pairs = a256(JR + 8 * total_pairs);
  const uint64_t at_res = a256(at_pairs + 8 * total_pairs);
  const size_t need = at_res + 8ull * kResWords * nj + 256;
  std::vector<uint64_t> first_pairs;
  if (total_pairs <= pre) {
    first_pairs.assign((const uint64_t *)(hs + head), (const uint64_t *)(hs + head) + total_pairs);
    hs = t_stage.get(need);
    if (!hs) return SDCSZ_EHIP;
    std::memcpy(hs + at_pairs, first_pairs.data(), 8 * total_pairs);
  } else {
    hs = t_stage.get(need);
    if (!hs) return SDCSZ_EHIP;
    HIPCHK(hipMemcpyAsync(hs + at_pairs, ws + B.pairs, 8 * total_pairs, hipMemcpyDeviceToHost, st));
    HIPCHK(sync_wait(st));
  }
  // ---- codebooks (host), then stage B: codewords, code check, scans,
  // header, encoding, results
  const uint64_t *pairs = (const uint64_t *)(hs + at_pairs);
  uint32_t *cbh = (uint32_t *)(hs + JR);
  std::vector<CodebookJob> cj(nj);
  uint64_t off = 0;
  for (uint32_t j = 0; j < nj; j++) {
    cj[j] = CodebookJob{pairs + off, cnt_sym[j], cbh + 2 * off};
    jobs[j].n_sym = cnt_sym[j];
    jobs[j].h.n_sym = cnt_sym[j];
    jobs[j].cw.cb = (uint32_t *)(ws + B.cb) + 2 * off;
    off += cnt_sym[j];
  }
  {
    HostSpan h(PH_HOST_CODEBOOK);
    build_codebooks(cj);
  }
  Tab t_put, t_chk_fast[kClasses], t_chk_gen, t_s1, t_s2, t_hdr, t_enc_fast[kClasses][2], t_enc_gen[2], t_res;
  Tab t_fuse[2];  // one-pass check and encoding, a tile of blocks per work-group
  bool any_empty = false;
  for (uint32_t j = 0; j < nj; j++) {
    const Job &J = jobs[j];
    const CompPlan &f = fp[j];
    if (J.n_sym) t_put.add(j, grid_for(J.n_sym, 256));
    t_hdr.add(j, grid_for(J.n_sym, 256));
    t_res.add(j, 1);
    if (f.fused) {
      t_fuse[J.dtype].add(j, tiles_of(f.g.n_blocks));
      continue;
    }
    if (f.fast) {
      t_chk_fast[f.cls].add(j, grid_for(f.g.n_blocks, ln_chk[f.cls]));
      t_enc_fast[f.cls][J.dtype].add(j, grid_for(f.g.n_blocks, ln_enc[f.cls][J.dtype]));
    } else if (f.g.n_blocks) {
      t_chk_gen.add(j, grid_for(f.g.n_blocks, 256));
      t_enc_gen[J.dtype].add(j, grid_for(f.g.n_blocks, 256));
    }
    t_s1.add(j, scan_chunks(f.g.n_blocks));
    t_s2.add(j, 1);
    any_empty |= f.g.n_blocks == 0;
  }
  Upload ub;
  ub.tabs = {&t_put, &t_chk_gen, &t_s1, &t_s2, &t_hdr, &t_enc_gen[0], &t_enc_gen[1], &t_res};
  for (int c = 0; c < kClasses; c++) {
    ub.tabs.push_back(&t_chk_fast[c]);
    for (int d = 0; d < 2; d++) ub.tabs.push_back(&t_enc_fast[c][d]);
  }
  ub.tabs.push_back(&t_fuse[0]);
  ub.tabs.push_back(&t_fuse[1]);
  ub.place(jobs, hs, ws + B.jobs);
  HIPCHK(hipMemcpyAsync(ws + B.jobs, hs, JR + 8 * total_pairs, hipMemcpyHostToDevice, st));
  const std::vector<JobTab> &D = ub.dev;
  if (t_put.total()) launch(PH_NONE, false, false, k_put_codes, grid(t_put), dim3(256), st, D[0]);
  {
    PhaseLaunch pl{PH_CHECK, {}};
    for (int c = 0; c < kClasses; c++) {
      const Tab &t = t_chk_fast[c];
      if (!t.total()) continue;
      const JobTab jt = D[8 + 3 * c];
      const JobKernel k = kCheckFast[c];
      const uint32_t ln = ln_chk[c];
      pl.fs.push_back([&t, jt, k, ln, st, &grid](bool x, bool y) { launch(PH_CHECK, x, y, k, grid(t), dim3(ln), st, jt); });
    }
    if (t_chk_gen.total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_CHECK, a, b, k_codes_check, grid(t_chk_gen), dim3(256), st, D[1]); });
    if (t_fuse[0].total())
      pl.fs.push_back([&](bool a, bool b) {
        launch(PH_CHECK, a, b, k_checkenc_fast<float, 6, 6, 6>, grid(t_fuse[0]), dim3(kEncTile), st,
               D[8 + 3 * kClasses]);
      });
    if (t_fuse[1].total())
      pl.fs.push_back([&](bool a, bool b) {
        launch(PH_CHECK, a, b, k_checkenc_fast<double, 6, 6, 6>, grid(t_fuse[1]), dim3(kEncTile), st,
               D[8 + 3 * kClasses + 1]);
      });
    pl.run();
  }
  if (any_empty) launch(PH_SCAN_C, true, !t_s1.total(), k_scan2, grid(t_s2), dim3(kScanThreads), st, D[3]);
  if (t_s1.total()) {
    launch(PH_SCAN_C, !any_empty, false, k_scan1, grid(t_s1), dim3(kScanThreads), st, D[2]);
    launch(PH_SCAN_C, false, true, k_scan3, grid(t_s1), dim3(kScanThreads), st, D[2]);
  }
  launch(PH_NONE, false, false, k_header, grid(t_hdr), dim3(256), st, D[4]);
  {
    PhaseLaunch pl{PH_ENCODE, {}};
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++) {
        const Tab &t = t_enc_fast[c][d];
        if (!t.total()) continue;
        const JobTab jt = D[8 + 3 * c + 1 + d];
        const JobKernel k = kEncFast[c][d];
        const uint32_t ln = ln_enc[c][d];
        pl.fs.push_back([&t, jt, k, ln, st, &grid](bool x, bool y) { launch(PH_ENCODE, x, y, k, grid(t), dim3(ln), st, jt); });
      }
    if (t_enc_gen[0].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_ENCODE, a, b, k_encode<float>, grid(t_enc_gen[0]), dim3(256), st, D[5]); });
    if (t_enc_gen[1].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_ENCODE, a, b, k_encode<double>, grid(t_enc_gen[1]), dim3(256), st, D[6]); });
    pl.run();
  }
  const uint64_t *d_res = (const uint64_t *)(ws + B.res);
  if (nj == 1) d_res = jobs[0].stat;  // one field: no gather needed
  else launch(PH_NONE, false, false, k_results, grid(t_res), dim3(64), st, D[7], (uint64_t *)d_res,
              (uint32_t)kResWords);
  HIPCHK(hipGetLastError());
  uint64_t *hres = (uint64_t *)(hs + at_res);
  HIPCHK(hipMemcpyAsync(hres, d_res, 8ull * kResWords * nj, hipMemcpyDeviceToHost, st));
  HIPCHK(sync_wait(st));
  g_timer.resolve();

  // ---- per-field outcome
  int first = SDCSZ_OK;
  for (uint32_t j = 0; j < nj; j++) {
    CompItem &c = it[item_of[j]];
    const uint64_t *cnt = hres + (uint64_t)j * kResWords, *res = cnt + C_N;
    fill_report(&c.rep, cnt, fp[j].g.n_blocks);
    std::memcpy(&c.rep.eb_abs, &res[R_EB], 8);
    // more blocks queued for re-execution than the queue holds: the others
    // keep the results of their disagreeing pass
    const bool overflow = (uint32_t)res[R_N] > kMaxRedo;
    const bool unc = cnt[C_UNC + SDCSZ_T_INPUT] || cnt[C_UNC + SDCSZ_T_COEF] || cnt[C_UNC + SDCSZ_T_CODE] ||
                     cnt[C_UNC + SDCSZ_T_PREP_INPUT] || cnt[C_MISSING] || overflow;
    if (cnt[C_SPIN]) {  // a one-pass tile gave up waiting for its predecessor
      c.out_size = 0;
      c.rc = SDCSZ_EHIP;
    } else if (unc) {
      c.out_size = 0;
      c.rc = SDCSZ_ESDC;
    } else {
      c.rep.n_outliers = res[R_OUTLIERS];
      c.rep.n_regression = res[R_REGRESSION];
      c.rep.payload_words = res[R_WORDS];
      c.rep.stream_size = res[R_SIZE];
      c.out_size = res[R_SIZE];
      c.rc = res[R_WRITTEN] ? SDCSZ_OK : SDCSZ_ENOSPC;
      if (c.rc == SDCSZ_OK) std::memcpy(c.header, res + R_N + 1, kHeader);
    }
  }
  for (uint32_t i = 0; i < n; i++)
    if (it[i].rc && !first) first = it[i].rc;
  return first;
}

// ---------------------------------------------------------------------------
// decompression, verification and region decompression of a batch
// ---------------------------------------------------------------------------
struct DecItem {  // one stream of a decompression call
  const uint8_t *d_stream;
  uint64_t stream_size;
  uint8_t *d_out;
  uint64_t out_cap;
  uint32_t mode;  // 0 decompress, 1 verify, 2 region
  Region reg;
  uint64_t need;  // bytes the output must hold
  const sdcsz_fault *faults;
  uint32_t n_faults;
  const uint8_t *h_header;  // the caller's copy of the header, or null
  bool small_recon;  // the no-allocation call: no recon scratch for the specialised decoder
  uint32_t prep;     // region state in the workspace: 0 none, 1 build it (no decoding), 2 reuse it
  int rc;
  sdcsz_report rep;
  Header h;
  Geo g;
};

struct DecPlan {
  DecLayout L;
  uint8_t *ws;
  bool fast;
  bool small;  // no recon scratch (see dec_layout)
  int cls;
  std::vector<sdcsz_fault> plan;
  std::vector<uint64_t> pb;  // blocks the wave-per-block routine takes (k_decode_wave_list)
  std::vector<uint64_t> fl;  // blocks the fault-applying instantiation takes
  std::vector<uint8_t> up;   // plan area as uploaded (entries, pb, fl)
};

uint64_t dec_batch_area(uint64_t njobs) {
  return a256(sizeof(Job) * njobs) + 32 * a256(4 * (2 * njobs + 1)) + a256(8ull * (C_N + 1) * njobs) +
         a256(kHeader * njobs);
}

// read and check the headers of a batch of streams (one synchronisation)
int read_headers(DecItem *it, uint32_t n, uint8_t *ws, uint64_t ws_size, hipStream_t st) {
  std::vector<uint32_t> idx;
  for (uint32_t i = 0; i < n; i++) {
    it[i].rc = SDCSZ_OK;
    std::memset(&it[i].rep, 0, sizeof(it[i].rep));
    if (!it[i].d_stream) it[i].rc = SDCSZ_EINVAL;
    else if (it[i].stream_size < kHeader) it[i].rc = SDCSZ_EFORMAT;
    else if (it[i].h_header) it[i].rc = unpack_header(it[i].h_header, it[i].stream_size, it[i].h, it[i].g);
    else idx.push_back(i);
  }
  if (idx.empty()) return SDCSZ_OK;
  uint8_t *hs = dec_stage().get(kHeader * idx.size() + (sizeof(Job) + 64) * idx.size() + 4096);
  if (!hs) return SDCSZ_EHIP;
  if (idx.size() == 1) {
    HIPCHK(hipMemcpyAsync(hs, it[idx[0]].d_stream, kHeader, hipMemcpyDeviceToHost, st));
  } else {
    // gather the headers on the device, then one copy back
    const uint64_t need = dec_batch_area(idx.size());
    if (!ws || ws_size < need) return SDCSZ_ENOSPC;
    std::vector<Job> jobs(idx.size());
    Tab t;
    for (size_t j = 0; j < idx.size(); j++) {
      std::memset(&jobs[j], 0, sizeof(Job));
      jobs[j].src = it[idx[j]].d_stream;
      t.add((uint32_t)j, 1);
    }
    Upload up;
    up.tabs = {&t};
    uint8_t *hj = hs + a256(kHeader * idx.size());
    up.place(jobs, hj, ws);
    HIPCHK(hipMemcpyAsync(ws, hj, up.bytes(idx.size()), hipMemcpyHostToDevice, st));
    uint8_t *dh = ws + a256(up.bytes(idx.size()));
    launch(PH_NONE, false, false, k_headers, dim3(t.total()), dim3(64), st, up.dev[0], dh);
    HIPCHK(hipMemcpyAsync(hs, dh, kHeader * idx.size(), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(sync_wait(st));
  for (size_t j = 0; j < idx.size(); j++) {
    DecItem &d = it[idx[j]];
    d.rc = unpack_header(hs + kHeader * j, d.stream_size, d.h, d.g);
  }
  return SDCSZ_OK;
}

uint64_t dec_batch_ws(const Geo *g, const uint32_t *dtype, const uint32_t *nf, uint32_t n) {
  uint64_t per = 0;
  for (uint32_t i = 0; i < n; i++) per += dec_layout(g[i], dtype[i], nf[i]).total;
  return dec_batch_area(n) + per;
}

// items whose headers were read (rc == OK): decode with one more synchronisation
int decode_batch(DecItem *it, uint32_t n, uint8_t *ws, uint64_t ws_size, hipStream_t st) {
  HostSpan call(PH_HOST_CALL);
  std::vector<DecPlan> fp;
  std::vector<uint32_t> item_of;
  uint64_t per = 0;
  for (uint32_t i = 0; i < n; i++) {
    DecItem &d = it[i];
    if (d.rc) continue;
    if (d.mode == 1 && !d.h.abft) d.rc = SDCSZ_EINVAL;
    else if (d.mode == 2) {
      uint64_t cnt = 1;
      for (int a = 0; a < 3; a++) {
        if (d.reg.lo[a] >= d.reg.hi[a] || d.reg.hi[a] > d.g.d[a]) d.rc = SDCSZ_EINVAL;
        cnt *= d.reg.hi[a] - d.reg.lo[a];
      }
      d.need = cnt * vbytes(d.h.dtype);
    } else {
      d.need = d.g.n_values * vbytes(d.h.dtype);
    }
    if (d.rc) continue;
    if (d.prep != 1 && (d.out_cap < d.need || (d.need && !d.d_out))) {
      d.rc = SDCSZ_ENOSPC;
      continue;
    }
    DecPlan f;
    d.rc = check_plan(d.g, d.h.dtype, d.faults, d.n_faults, true, f.plan);
    if (d.rc) continue;
    // full and region decompression take the specialised decoder where the
    // block shape has one; verification the generic kernel
    f.cls = d.mode != 1 ? fast_class(d.g, vbytes(d.h.dtype)) : -1;
    f.fast = f.cls >= 0;
    fp.push_back(std::move(f));
    item_of.push_back(i);
  }
  const uint32_t nj = (uint32_t)fp.size();
  if (nj == 0) return SDCSZ_OK;
  // a launch with a field of 2 GiB or more takes the wide kernel, which
  // applies no fault plan: its fields' plan blocks take the generic routine
  bool wide_dec[kClasses][2] = {};
  for (uint32_t j = 0; j < nj; j++) {
    const DecItem &d = it[item_of[j]];
    if (fp[j].fast) wide_dec[fp[j].cls][d.h.dtype] |= wide_field(d.g, vbytes(d.h.dtype));
  }
  for (uint32_t j = 0; j < nj; j++) {
    DecPlan &f = fp[j];
    const DecItem &d = it[item_of[j]];
    if (f.fast && !f.plan.empty()) split_plan(f.plan, !wide_dec[f.cls][d.h.dtype], true, f.pb, f.fl);
    f.small = d.small_recon && f.fast && f.pb.empty();
    f.L = dec_layout(d.g, d.h.dtype, d.n_faults, f.small);
    per += f.L.total;
  }
  const uint64_t area = dec_batch_area(nj);
  if (!ws || ws_size < area + per) {
    for (uint32_t j = 0; j < nj; j++) it[item_of[j]].rc = SDCSZ_ENOSPC;
    return SDCSZ_ENOSPC;
  }
  std::vector<Job> jobs(nj);
  uint64_t at = area;
  for (uint32_t j = 0; j < nj; j++) {
    DecPlan &f = fp[j];
    const DecItem &d = it[item_of[j]];
    f.ws = ws + at;
    at += f.L.total;
    uint8_t *w = f.ws;
    Job &J = jobs[j];
    std::memset(&J, 0, sizeof(J));
    J.g = d.g;
    J.h = d.h;
    DecWork &dw = J.dw;
    dw.cnt = (unsigned long long *)(w + f.L.cnt);
    dw.symbols = (uint16_t *)(w + f.L.symbols);
    dw.tab = (DecTab *)(w + f.L.tab);
    dw.recon = w + f.L.recon;
    dw.off_pay = (uint64_t *)(w + f.L.off_pay);
    dw.off_out = (uint32_t *)(w + f.L.off_out);
    dw.off_coef = (uint32_t *)(w + f.L.off_coef);
    dw.scan_part = (uint64_t *)(w + f.L.scan);
    dw.lut = (uint32_t *)(w + f.L.lut);
    dw.lut2 = (uint32_t *)(w + f.L.lut2);
    dw.sub = (uint32_t *)(w + f.L.sub);
    dw.redo_n = (uint32_t *)(w + f.L.redo_n);
    dw.redo = (uint64_t *)(w + f.L.redo);
    dw.err = (uint32_t *)(w + f.L.err);
    dw.tot = (uint64_t *)(w + f.L.tot);
    J.plan.n = (uint32_t)f.plan.size();
    J.plan.f = (const sdcsz_fault *)(w + f.L.plan);
    J.plan.bits = (const uint32_t *)(w + f.L.bits);
    J.plan.list = J.plan.flist = nullptr;
    J.plan.nlist = J.plan.nflist = 0;
    J.reg = d.reg;
    J.mode = d.mode;
    const uint32_t *table = (const uint32_t *)(d.d_stream + d.h.off_table);
    J.ss = ScanSrc{table, table + 1, 2};
    J.sc_part = dw.scan_part;
    J.sc_off_pay = dw.off_pay;
    J.sc_off_out = dw.off_out;
    J.sc_off_coef = dw.off_coef;
    J.sc_tot = dw.tot;
    J.src = d.d_stream;
    J.dst = d.d_out;
    J.dst_cap = d.out_cap;
    J.zero = (uint32_t *)(w + f.L.cnt);
    J.zero_words = ((f.plan.empty() ? f.L.zero_end : f.L.bits_end) - f.L.cnt) / 4;
    J.stat = (const uint64_t *)(w + f.L.cnt);
    J.stat_words = C_N + 1;
    J.dtype = d.h.dtype;
    J.abft = d.h.abft;
    J.hdr_keep = (uint32_t *)(w + f.L.hdr);
    if (!f.plan.empty()) HIPCHK(upload_plan(f.plan, f.pb, f.fl, f.up, w + f.L.plan, J.plan, st));
  }
  // t_list, t_redo: a wave per block; t_flist: the fault-applying
  // instantiation over the plans' lists
  Tab t_zero, t_plan, t_one, t_s1, t_fast[kClasses][2], t_flist[kClasses][2], t_gen[2], t_list[2], t_redo[2];
  Tab t_wreg[2];  // regions of few blocks: a wave per block
  uint32_t lds_list[2] = {}, lds_redo[2] = {}, lds_wreg[2] = {};
  uint64_t nb_dec[kClasses][2] = {};
  for (uint32_t j = 0; j < nj; j++)
    if (fp[j].fast) nb_dec[fp[j].cls][jobs[j].dtype] += jobs[j].g.n_blocks;
  uint32_t ln_dec[kClasses][2];
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++) ln_dec[c][d] = tuned_lanes(TS_DECODE, c, d, nb_dec[c][d]);
  for (uint32_t j = 0; j < nj; j++) {
    Job &J = jobs[j];
    t_zero.add(j, 1);
    if (!fp[j].plan.empty()) t_plan.add(j, grid_for(fp[j].plan.size(), 256));
    if (!fp[j].fl.empty()) t_flist[fp[j].cls][J.dtype].add(j, grid_for(fp[j].fl.size(), 64));
    t_one.add(j, 1);
    t_s1.add(j, scan_chunks(J.g.n_blocks));
    uint64_t nbox = 0;
    if (J.mode == 2) {
      // the box of blocks the region touches
      nbox = 1;
      for (int a = 0; a < 3; a++) {
        J.rblk.lo[a] = J.reg.lo[a] / J.g.b[a];
        J.rblk.hi[a] = (J.reg.hi[a] - 1) / J.g.b[a] + 1;
        nbox *= J.rblk.hi[a] - J.rblk.lo[a];
      }
      std::memset(&J.L, 0, sizeof(J.L));
      J.L.shell_count = nbox;
    }
    const uint32_t wlds = wave_lds_bytes(J.g, vbytes(J.dtype));
    if (J.mode == 2 && nbox <= kWaveRegionBlocks && wlds <= kWaveLdsMax) {
      // few blocks: a wave each (one block's serial decoding time in all)
      t_wreg[J.dtype].add(j, nbox);
      lds_wreg[J.dtype] = std::max(lds_wreg[J.dtype], wlds);
    } else if (fp[j].fast && J.mode == 2) {
      // one lane per block of the box (masked path)
      const uint32_t ln = ln_dec[fp[j].cls][J.dtype];
      t_fast[fp[j].cls][J.dtype].add(j, grid_for(nbox, ln));
    } else if (fp[j].fast) {
      t_fast[fp[j].cls][J.dtype].add(j, fast_launch(J.g, &J.L, ln_dec[fp[j].cls][J.dtype]));
    } else if (J.g.n_blocks) {
      t_gen[J.dtype].add(j, grid_for(J.g.n_blocks, 64));
    }
  }
  for (uint32_t j = 0; j < nj; j++) {
    const Job &J = jobs[j];
    if (!fp[j].fast) continue;
    const uint32_t lb = wave_lds_bytes(J.g, vbytes(J.dtype));
    t_redo[J.dtype].add(j, kRedoWgs);
    lds_redo[J.dtype] = std::max(lds_redo[J.dtype], lb);
    if (!fp[j].pb.empty()) {
      t_list[J.dtype].add(j, fp[j].pb.size());
      lds_list[J.dtype] = std::max(lds_list[J.dtype], lb);
    }
  }
  Upload up;
  up.tabs = {&t_zero, &t_one, &t_s1, &t_gen[0], &t_gen[1], &t_list[0], &t_list[1], &t_redo[0], &t_redo[1], &t_plan};
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++) up.tabs.push_back(&t_fast[c][d]);
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++) up.tabs.push_back(&t_flist[c][d]);
  up.tabs.push_back(&t_wreg[0]);
  up.tabs.push_back(&t_wreg[1]);
  const size_t res_bytes = 8ull * (C_N + 1) * nj;
  // caller-given headers go to the end of the batch area (uploaded with the
  // jobs) for k_dectab to check against the streams
  const uint64_t hdr_at = dec_batch_area(nj) - a256(kHeader * nj);
  bool any_hdr = false;
  for (uint32_t j = 0; j < nj; j++) {
    const DecItem &d = it[item_of[j]];
    jobs[j].hdr_expect = d.h_header ? (const uint32_t *)(ws + hdr_at + kHeader * j) : nullptr;
    any_hdr |= d.h_header != nullptr;
  }
  const uint64_t up_bytes = any_hdr ? hdr_at + kHeader * nj : up.bytes(nj);
  uint8_t *hs = dec_stage().get(std::max<uint64_t>(up_bytes, up.bytes(nj) + res_bytes) + 4096);
  if (!hs) return SDCSZ_EHIP;
  up.place(jobs, hs, ws);
  for (uint32_t j = 0; j < nj; j++)
    if (it[item_of[j]].h_header) std::memcpy(hs + hdr_at + kHeader * j, it[item_of[j]].h_header, kHeader);
  HIPCHK(hipMemcpyAsync(ws, hs, up_bytes, hipMemcpyHostToDevice, st));
  const std::vector<JobTab> &D = up.dev;
  auto grid = [](const Tab &t) { return dim3(t.total()); };
  launch(PH_NONE, false, false, k_zero_jobs, grid(t_zero), dim3(256), st, D[0]);
  if (t_plan.total()) launch(PH_NONE, false, false, k_plan_bits, grid(t_plan), dim3(256), st, D[9]);
  // region state (single-stream calls only): built once, then reused
  const uint32_t prep = nj == 1 ? it[item_of[0]].prep : 0u;
  if (prep == 2) {
    launch(PH_NONE, false, false, k_hdr_keep, grid(t_one), dim3(64), st, D[1], 2u);
  } else {
    launch(PH_NONE, false, false, k_dectab, grid(t_one), dim3(kDecTabThreads), st, D[1]);
    bool any_empty = false;
    for (uint32_t j = 0; j < nj; j++) any_empty |= jobs[j].g.n_blocks == 0;
    if (any_empty) launch(PH_SCAN_D, true, !t_s1.total(), k_scan2, grid(t_one), dim3(kScanThreads), st, D[1]);
    if (t_s1.total()) {
      launch(PH_SCAN_D, !any_empty, false, k_scan1, grid(t_s1), dim3(kScanThreads), st, D[2]);
      launch(PH_SCAN_D, false, true, k_scan3, grid(t_s1), dim3(kScanThreads), st, D[2]);
    }
    launch(PH_NONE, false, false, k_dec_check, grid(t_one), dim3(64), st, D[1]);
    if (prep == 1) launch(PH_NONE, false, false, k_hdr_keep, grid(t_one), dim3(64), st, D[1], 1u);
  }
  if (prep == 1) {
    // tables and offsets only: no decoding
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++) t_fast[c][d] = Tab(), t_flist[c][d] = Tab();
    for (int d = 0; d < 2; d++) t_gen[d] = Tab(), t_list[d] = Tab(), t_redo[d] = Tab(), t_wreg[d] = Tab();
  }
  // plan blocks (full decompression), which the production decoder leaves,
  // beside it on a second stream: the fault-applying instantiation over its
  // lists, a wave per block for the others
  bool any_plan_work = t_list[0].total() || t_list[1].total();
  for (int c = 0; c < kClasses; c++)
    for (int d = 0; d < 2; d++) any_plan_work |= t_flist[c][d].total() != 0;
  hipStream_t side = st;
  if (any_plan_work) {
    if (!t_no_side) {
      side = t_side.fork(st);
      if (!side) return SDCSZ_EHIP;
    }
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++)
        if (t_flist[c][d].total())
          launch(PH_NONE, false, false, kDecFast[c][d][2], grid(t_flist[c][d]), dim3(64), side,
                 D[10 + 2 * kClasses + 2 * c + d]);
    if (t_list[0].total())
      launch_shm(PH_NONE, false, false, k_decode_wave_list<float>, grid(t_list[0]), dim3(64), lds_list[0], side, D[5]);
    if (t_list[1].total())
      launch_shm(PH_NONE, false, false, k_decode_wave_list<double>, grid(t_list[1]), dim3(64), lds_list[1], side, D[6]);
    // the blocks the fault-applying decoder queued, re-executed on the side
    // stream as soon as it is done (its own queue: the production decoder
    // may still be adding to the other)
    for (int d = 0; d < 2; d++) {
      bool fl = false;
      for (int c = 0; c < kClasses; c++) fl |= t_flist[c][d].total() != 0;
      if (fl && t_redo[d].total())
        launch_shm(PH_NONE, false, false, d ? k_decode_wave_redo<double> : k_decode_wave_redo<float>, grid(t_redo[d]),
                   dim3(64), lds_redo[d], side, D[7 + d], 1u);
    }
  }
  {
    PhaseLaunch pl{PH_DECODE, {}};
    for (int c = 0; c < kClasses; c++)
      for (int d = 0; d < 2; d++) {
        const Tab &t = t_fast[c][d];
        if (!t.total()) continue;
        const JobTab jt = D[10 + 2 * c + d];
        const JobKernel k = kDecFast[c][d][wide_dec[c][d] ? 1 : 0];
        const uint32_t ln = ln_dec[c][d];
        pl.fs.push_back([&t, jt, k, ln, st, &grid](bool x, bool y) { launch(PH_DECODE, x, y, k, grid(t), dim3(ln), st, jt); });
      }
    if (t_gen[0].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_DECODE, a, b, k_decode_generic<float>, grid(t_gen[0]), dim3(64), st, D[3]); });
    if (t_gen[1].total())
      pl.fs.push_back([&](bool a, bool b) { launch(PH_DECODE, a, b, k_decode_generic<double>, grid(t_gen[1]), dim3(64), st, D[4]); });
    if (t_wreg[0].total())
      pl.fs.push_back([&](bool a, bool b) {
        launch_shm(PH_DECODE, a, b, k_decode_wave_region<float>, grid(t_wreg[0]), dim3(64), lds_wreg[0], st,
                   D[10 + 4 * kClasses]);
      });
    if (t_wreg[1].total())
      pl.fs.push_back([&](bool a, bool b) {
        launch_shm(PH_DECODE, a, b, k_decode_wave_region<double>, grid(t_wreg[1]), dim3(64), lds_wreg[1], st,
                   D[10 + 4 * kClasses + 1]);
      });
    pl.run();
  }
  if (any_plan_work && !t_no_side) HIPCHK(t_side.join(st));
  if (t_redo[0].total())
    launch_shm(PH_NONE, false, false, k_decode_wave_redo<float>, grid(t_redo[0]), dim3(64), lds_redo[0], st, D[7], 0u);
  if (t_redo[1].total())
    launch_shm(PH_NONE, false, false, k_decode_wave_redo<double>, grid(t_redo[1]), dim3(64), lds_redo[1], st, D[8],
               0u);
  const uint64_t *d_res = (const uint64_t *)(ws + a256(up.bytes(nj)));
  if (nj == 1) d_res = jobs[0].stat;  // one stream: no gather needed
  else launch(PH_NONE, false, false, k_results, grid(t_one), dim3(64), st, D[1], (uint64_t *)d_res,
              (uint32_t)(C_N + 1));
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hs + up.bytes(nj), d_res, res_bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(sync_wait(st));
  g_timer.resolve();
  std::vector<uint64_t> resv((const uint64_t *)(hs + up.bytes(nj)), (const uint64_t *)(hs + up.bytes(nj)) + (C_N + 1) * nj);
  // more blocks to re-execute than the queue holds: decode those fields again
  // in full with the generic kernel
  // (a call without recon scratch cannot: the blocks beyond the queue stay
  // uncorrected and the item ends in ESDC)
  std::vector<uint32_t> again;
  std::vector<uint64_t> overflow(nj, 0);
  for (uint32_t j = 0; j < nj; j++) {
    const uint64_t *cj = resv.data() + (uint64_t)j * (C_N + 1);
    const uint32_t *tail = (const uint32_t *)(cj + C_N);
    const uint64_t more = (tail[0] > kMaxRedo ? tail[0] - kMaxRedo : 0) +
                          (cj[C_REDO2] > kMaxRedo ? cj[C_REDO2] - kMaxRedo : 0);
    if (!tail[1] && fp[j].fast && more) {
      if (fp[j].small) overflow[j] = more;
      else again.push_back(j);
    }
  }
  if (!again.empty()) {
    Tab t_ag[2], t_res2;
    for (uint32_t j : again) {  // full (mode 0) or region (mode 2) decompression, as in the first pass
      t_ag[jobs[j].dtype].add(j, grid_for(jobs[j].g.n_blocks, 64));
      t_res2.add(j, 1);
      launch(PH_NONE, false, false, k_zero_u64, dim3(1), dim3(64), st, jobs[j].dw.cnt, (uint64_t)C_N);
    }
    Upload u2;
    u2.tabs = {&t_ag[0], &t_ag[1], &t_res2};
    uint8_t *h2 = dec_stage().get(u2.bytes(nj) + res_bytes + 4096);
    if (!h2) return SDCSZ_EHIP;
    u2.place(jobs, h2, ws);
    HIPCHK(hipMemcpyAsync(ws, h2, u2.bytes(nj), hipMemcpyHostToDevice, st));
    if (t_ag[0].total())
      launch(PH_NONE, false, false, k_decode_generic<float>, grid(t_ag[0]), dim3(64), st, u2.dev[0]);
    if (t_ag[1].total())
      launch(PH_NONE, false, false, k_decode_generic<double>, grid(t_ag[1]), dim3(64), st, u2.dev[1]);
    uint64_t *d_res2 = (uint64_t *)(ws + a256(u2.bytes(nj)));
    launch(PH_NONE, false, false, k_results, grid(t_res2), dim3(64), st, u2.dev[2], d_res2, (uint32_t)(C_N + 1));
    HIPCHK(hipMemcpyAsync(h2 + u2.bytes(nj), d_res2, 8ull * (C_N + 1) * again.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(sync_wait(st));
    const uint64_t *r2 = (const uint64_t *)(h2 + u2.bytes(nj));
    for (size_t q = 0; q < again.size(); q++)
      std::memcpy(resv.data() + (uint64_t)again[q] * (C_N + 1), r2 + q * (C_N + 1), 8 * (C_N + 1));
  }
  const uint64_t *hres = resv.data();
  int first = SDCSZ_OK;
  for (uint32_t j = 0; j < nj; j++) {
    DecItem &d = it[item_of[j]];
    const uint64_t *cnt = hres + (uint64_t)j * (C_N + 1);
    const uint32_t *tail = (const uint32_t *)(cnt + C_N);
    fill_report(&d.rep, cnt, d.g.n_blocks);
    d.rep.eb_abs = d.h.eb_abs;
    d.rep.n_outliers = d.h.n_outliers;
    d.rep.n_regression = d.h.n_regression;
    d.rep.payload_words = d.h.payload_words;
    d.rep.stream_size = d.h.total;
    d.rep.uncorrectable[SDCSZ_T_RECON] += overflow[j];
    if (tail[1]) d.rc = SDCSZ_EFORMAT;
    else d.rc = (cnt[C_UNC + SDCSZ_T_RECON] || overflow[j]) ? SDCSZ_ESDC : SDCSZ_OK;
  }
  for (uint32_t i = 0; i < n; i++)
    if (it[i].rc && !first) first = it[i].rc;
  return first;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// Region decompression (prep 0), building the region state of a stream in
// the workspace (prep 1: the region is the whole field and nothing is
// decoded), or a region decoded with that state (prep 2; a region that is
// the whole field takes the full-field launch, whose output is the same).
static int region_call(const void *d_stream, uint64_t stream_size, const uint8_t *h_header, const uint64_t *h_lo,
                const uint64_t *h_hi, void *d_out, uint64_t out_cap, sdcsz_report *h_rep, void *d_ws,
                uint64_t ws_size, hipStream_t st, uint32_t prep) {
  DecItem d{};
  d.d_stream = (const uint8_t *)d_stream;
  d.stream_size = stream_size;
  d.d_out = (uint8_t *)d_out;
  d.out_cap = out_cap;
  d.mode = 2;
  d.h_header = h_header;
  d.prep = prep;
  int rc = read_headers(&d, 1, nullptr, 0, st);
  if (rc) return rc;
  if (d.rc) return d.rc;
  if (prep != 1 && (!h_lo || !h_hi)) return SDCSZ_EINVAL;
  const uint32_t off = 3 - d.h.ndim;
  bool whole = true;
  for (int a = 0; a < 3; a++) {
    d.reg.lo[a] = 0;
    d.reg.hi[a] = a < (int)off || prep == 1 ? d.g.d[a] : 1;
  }
  if (prep != 1)
    for (uint32_t a = 0; a < d.h.ndim; a++) {
      d.reg.lo[off + a] = h_lo[a];
      d.reg.hi[off + a] = h_hi[a];
      whole = whole && h_lo[a] == 0 && h_hi[a] == d.g.d[off + a];
    }
  if (prep == 2 && whole) d.mode = 0;
  rc = decode_batch(&d, 1, (uint8_t *)d_ws, ws_size, st);
  if (rc == SDCSZ_EHIP) return rc;
  if (h_rep && (d.rc == SDCSZ_OK || d.rc == SDCSZ_ESDC)) *h_rep = d.rep;
  return d.rc;
}

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

int sdcsz_tune_set(int stage, int shape_class, int dtype, uint32_t n, const uint64_t *max_blocks,
                   const uint32_t *lanes) {
  if (stage < 0 || stage >= kTuneStages || shape_class < 0 || shape_class >= kClasses || dtype < 0 || dtype > 1 ||
      n > SDCSZ_TUNE_MAX || (n && (!max_blocks || !lanes)))
    return SDCSZ_EINVAL;
  for (uint32_t i = 0; i < n; i++) {
    if (lanes[i] != 64 && lanes[i] != 128 && lanes[i] != 256) return SDCSZ_EINVAL;
    if (i && max_blocks[i] <= max_blocks[i - 1]) return SDCSZ_EINVAL;
  }
  TuneRow r;
  r.n = n;
  for (uint32_t i = 0; i < n; i++) {
    r.max_blocks[i] = max_blocks[i];
    r.lanes[i] = lanes[i];
  }
  g_tune[stage][shape_class][dtype] = r;
  return SDCSZ_OK;
}

int sdcsz_tune_get(int stage, int shape_class, int dtype, uint32_t *n, uint64_t *max_blocks, uint32_t *lanes) {
  if (stage < 0 || stage >= kTuneStages || shape_class < 0 || shape_class >= kClasses || dtype < 0 || dtype > 1 ||
      !n || !max_blocks || !lanes)
    return SDCSZ_EINVAL;
  const TuneRow &r = g_tune[stage][shape_class][dtype];
  *n = r.n;
  for (uint32_t i = 0; i < r.n; i++) {
    max_blocks[i] = r.max_blocks[i];
    lanes[i] = r.lanes[i];
  }
  return SDCSZ_OK;
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
  return max_stream_size(g, p->dtype);
}

uint64_t sdcsz_compress_workspace_size(const sdcsz_params *p) {
  Geo g;
  if (check_params(p, &g)) return 0;
  CompItem c{};
  c.p = p;
  return comp_batch_ws(&c, 1);
}

int sdcsz_compress(const void *d_in, const sdcsz_params *p, void *d_out, uint64_t out_cap, uint64_t *h_out_size,
                   sdcsz_report *h_rep, void *d_ws, uint64_t ws_size, void *stream) {
  Geo g;
  int rc = check_params(p, &g);
  if (rc) return rc;
  if (!h_out_size || (g.n_values && !d_in)) return SDCSZ_EINVAL;
  CompItem c{};
  c.d_in = d_in;
  c.p = p;
  c.d_out = (uint8_t *)d_out;
  c.out_cap = out_cap;
  rc = compress_batch(&c, 1, (uint8_t *)d_ws, ws_size, (hipStream_t)stream);
  if (rc == SDCSZ_EHIP) return rc;
  *h_out_size = c.out_size;
  if (h_rep && (c.rc == SDCSZ_OK || c.rc == SDCSZ_ENOSPC || c.rc == SDCSZ_ESDC)) *h_rep = c.rep;
  return c.rc;
}

uint64_t sdcsz_compress_batch_workspace_size(const sdcsz_comp_item *h_items, uint32_t n) {
  if (!h_items) return 0;
  std::vector<CompItem> c(n);
  for (uint32_t i = 0; i < n; i++) c[i].p = &h_items[i].params;
  return comp_batch_ws(c.data(), n);
}

int sdcsz_compress_batch(sdcsz_comp_item *h_items, uint32_t n, void *d_ws, uint64_t ws_size, void *stream) {
  if (!h_items && n) return SDCSZ_EINVAL;
  std::vector<CompItem> c(n);
  for (uint32_t i = 0; i < n; i++) {
    c[i].d_in = h_items[i].d_in;
    c[i].p = &h_items[i].params;
    c[i].d_out = (uint8_t *)h_items[i].d_out;
    c[i].out_cap = h_items[i].out_cap;
  }
  const int rc = compress_batch(c.data(), n, (uint8_t *)d_ws, ws_size, (hipStream_t)stream);
  for (uint32_t i = 0; i < n; i++) {
    h_items[i].out_size = c[i].out_size;
    h_items[i].rc = rc == SDCSZ_EHIP ? SDCSZ_EHIP : c[i].rc;
    h_items[i].rep = c[i].rep;
    if (h_items[i].rc == SDCSZ_OK) std::memcpy(h_items[i].header, c[i].header, kHeader);
    else std::memset(h_items[i].header, 0, kHeader);
  }
  return rc;
}

int sdcsz_stream_info(const void *d_stream, uint64_t stream_size, sdcsz_params *h_p, uint64_t *h_n_blocks,
                      double *h_eb_abs, void *stream) {
  DecItem d{};
  d.d_stream = (const uint8_t *)d_stream;
  d.stream_size = stream_size;
  int rc = read_headers(&d, 1, nullptr, 0, (hipStream_t)stream);
  if (rc) return rc;
  if (d.rc) return d.rc;
  if (h_p) {
    std::memset(h_p, 0, sizeof(*h_p));
    h_p->dtype = d.h.dtype;
    h_p->ndim = d.h.ndim;
    for (uint32_t a = 0; a < d.h.ndim; a++) {
      h_p->dims[a] = d.h.d[3 - d.h.ndim + a];
      h_p->block[a] = d.h.b[3 - d.h.ndim + a];
    }
    h_p->eb_mode = d.h.eb_mode;
    h_p->predictor = d.h.predictor;
    h_p->eb = d.h.eb;
    h_p->abft = d.h.abft;
  }
  if (h_n_blocks) *h_n_blocks = d.h.n_blocks;
  if (h_eb_abs) *h_eb_abs = d.h.eb_abs;
  return SDCSZ_OK;
}

uint64_t sdcsz_decompress_workspace_size(const sdcsz_params *p) {
  Geo g;
  if (!p || p->dtype > 1 || !geometry(p->ndim, p->dims, p->block, &g)) return 0;
  const uint32_t dt = p->dtype, nf = p->n_faults;
  return dec_batch_ws(&g, &dt, &nf, 1);
}

uint64_t sdcsz_decompress_batch_workspace_size(const sdcsz_params *h_params, uint32_t n) {
  if (!h_params && n) return 0;
  std::vector<Geo> g(n);
  std::vector<uint32_t> dt(n), nf(n);
  for (uint32_t i = 0; i < n; i++) {
    const sdcsz_params *p = &h_params[i];
    if (p->dtype > 1 || !geometry(p->ndim, p->dims, p->block, &g[i])) return 0;
    dt[i] = p->dtype;
    nf[i] = p->n_faults;
  }
  return dec_batch_ws(g.data(), dt.data(), nf.data(), n);
}

namespace {
// sdcsz_decompress_noalloc: the device address of `scratch` per device, and a
// static pageable host buffer for the call's job tables, header and results
// (a single stream needs a few KiB).  One call at a time in the process.
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void *g_scratch_ptr[kNoAllocDevices] = {};
alignas(256) uint8_t g_noalloc_host[1u << 20];

int decode_one_call(DecItem &d, uint8_t *ws, uint64_t ws_size, hipStream_t st, sdcsz_report *h_rep) {
  int rc = read_headers(&d, 1, nullptr, 0, st);
  if (rc) return rc;
  if (d.rc) return d.rc;
  rc = decode_batch(&d, 1, ws, ws_size, st);
  if (rc == SDCSZ_EHIP) return rc;
  if (h_rep && (d.rc == SDCSZ_OK || d.rc == SDCSZ_ESDC)) *h_rep = d.rep;
  return d.rc;
}
}  // namespace

int sdcsz_decompress(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap,
                     const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                     void *stream) {
  DecItem d{};
  d.d_stream = (const uint8_t *)d_stream;
  d.stream_size = stream_size;
  d.d_out = (uint8_t *)d_out;
  d.out_cap = out_cap;
  d.faults = h_faults;
  d.n_faults = n_faults;
  return decode_one_call(d, (uint8_t *)d_ws, ws_size, (hipStream_t)stream, h_rep);
}

int sdcsz_decompress_noalloc(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap,
                             const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *stream) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) return SDCSZ_EHIP;
  if (!g_scratch_ptr[dev]) {
    // the array's device address on this device (the host-side name is only
    // a stand-in); looked up once per device, with that device current
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SDCSZ_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  Staging fixed;
  fixed.p = g_noalloc_host;
  fixed.cap = sizeof(g_noalloc_host);
  fixed.fixed = true;
  t_stage_over = &fixed;
  t_no_side = true;  // no second stream to create
  DecItem d{};
  d.d_stream = (const uint8_t *)d_stream;
  d.stream_size = stream_size;
  d.d_out = (uint8_t *)d_out;
  d.out_cap = out_cap;
  d.faults = h_faults;
  d.n_faults = n_faults;
  d.small_recon = true;
  const int rc = decode_one_call(d, (uint8_t *)g_scratch_ptr[dev], SDCSZ_NOALLOC_SCRATCH_BYTES,
                                 (hipStream_t)stream, h_rep);
  t_stage_over = nullptr;
  t_no_side = false;
  return rc;
}

int sdcsz_verify(const void *d_stream, uint64_t stream_size, void *d_data, uint64_t data_size,
                 const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                 void *stream) {
  DecItem d{};
  d.d_stream = (const uint8_t *)d_stream;
  d.stream_size = stream_size;
  d.d_out = (uint8_t *)d_data;
  d.out_cap = data_size;
  d.mode = 1;
  d.faults = h_faults;
  d.n_faults = n_faults;
  return decode_one_call(d, (uint8_t *)d_ws, ws_size, (hipStream_t)stream, h_rep);
}

int sdcsz_decompress_region(const void *d_stream, uint64_t stream_size, const uint64_t *h_lo, const uint64_t *h_hi,
                            void *d_out, uint64_t out_cap, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                            void *stream) {
  return region_call(d_stream, stream_size, nullptr, h_lo, h_hi, d_out, out_cap, h_rep, d_ws, ws_size,
                     (hipStream_t)stream, 0);
}

int sdcsz_region_prepare(const void *d_stream, uint64_t stream_size, const void *h_header, void *d_ws,
                         uint64_t ws_size, void *stream) {
  return region_call(d_stream, stream_size, (const uint8_t *)h_header, nullptr, nullptr, nullptr, 0, nullptr, d_ws,
                     ws_size, (hipStream_t)stream, 1);
}

int sdcsz_decompress_region_prepared(const void *d_stream, uint64_t stream_size, const void *h_header,
                                     const uint64_t *h_lo, const uint64_t *h_hi, void *d_out, uint64_t out_cap,
                                     sdcsz_report *h_rep, void *d_ws, uint64_t ws_size, void *stream) {
  return region_call(d_stream, stream_size, (const uint8_t *)h_header, h_lo, h_hi, d_out, out_cap, h_rep, d_ws,
                     ws_size, (hipStream_t)stream, 2);
}

int sdcsz_decompress_batch(sdcsz_dec_item *h_items, uint32_t n, void *d_ws, uint64_t ws_size, void *stream) {
  if (!h_items && n) return SDCSZ_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  std::vector<DecItem> d(n);
  for (uint32_t i = 0; i < n; i++) {
    std::memset(&d[i], 0, sizeof(DecItem));
    d[i].d_stream = (const uint8_t *)h_items[i].d_stream;
    d[i].stream_size = h_items[i].stream_size;
    d[i].d_out = (uint8_t *)h_items[i].d_out;
    d[i].out_cap = h_items[i].out_cap;
    d[i].faults = h_items[i].faults;
    d[i].n_faults = h_items[i].n_faults;
    d[i].h_header = (const uint8_t *)h_items[i].h_header;
  }
  int rc = read_headers(d.data(), n, (uint8_t *)d_ws, ws_size, st);
  if (rc == SDCSZ_OK) rc = decode_batch(d.data(), n, (uint8_t *)d_ws, ws_size, st);
  for (uint32_t i = 0; i < n; i++) {
    h_items[i].rc = rc == SDCSZ_EHIP ? SDCSZ_EHIP : d[i].rc;
    h_items[i].rep = d[i].rep;
  }
  if (rc) return rc;
  for (uint32_t i = 0; i < n; i++)
    if (d[i].rc) return d[i].rc;
  return SDCSZ_OK;
}

}  // extern "C"
