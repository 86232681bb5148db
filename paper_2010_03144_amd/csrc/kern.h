// kern.h -- kernel declarations (definitions in kern_*.hip) and the job
// tables through which every launch covers one or many fields.
#pragma once

#include "common.h"

namespace sdcsz {

struct Region {
  uint64_t lo[3], hi[3];
};

// streams of counts scanned per block: payload words, outliers, regression
struct ScanSrc {
  const uint32_t *words;
  const uint32_t *meta;
  uint32_t stride;
};

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kDecTabThreads = 1024, kDecTabWaves = kDecTabThreads / 64;  // decoder-table kernel
// Blocks per thread of the scans: 2 (many small work-groups hide latency
// best), more for fields of over 2^20 blocks so that a job has at most
// kScanMaxChunks chunks (each offsets work-group adds up the totals of the
// chunks before its own).
constexpr uint32_t kScanMaxChunks = 2048;
__host__ __device__ inline uint32_t scan_items(uint64_t nb) {
  const uint64_t per = (nb + (uint64_t)kScanThreads * kScanMaxChunks - 1) / ((uint64_t)kScanThreads * kScanMaxChunks);
  return per > 2 ? (uint32_t)per : 2u;
}
__host__ __device__ inline uint64_t scan_chunk(uint64_t nb) { return (uint64_t)kScanThreads * scan_items(nb); }
constexpr uint32_t kRangeThreads = 256;
constexpr uint32_t kHistWin = 16384;  // largest LDS histogram window of the compression kernel (64 KiB)
constexpr uint32_t kRangeBlocks = 2048;

// Work of one specialised launch: work-groups [0, full_wgs) take the
// sub-grid of full blocks, the others the shell of partial blocks at the
// upper edges (the slab of blocks partial along the fastest axis, then the
// middle, then the slowest, each excluding the earlier slabs).  The
// compressor launches the two apart, each numbering its work-groups from 0.
struct Launch {
  uint32_t nf[3];      // full blocks per axis
  uint32_t full_wgs;   // work-groups of full blocks
  uint64_t s2, s1;     // sizes of the first two shell slabs
  uint64_t full_count, shell_count;
};

// One field of a launch: its geometry, device work areas and parameters.
struct Job {
  Geo g;
  CompWork cw;          // compression work areas
  DecWork dw;           // decompression work areas
  PlanDev plan;
  Launch L;
  Header h;             // compression: fixed header fields; decompression: the stream's header
  Region reg;           // decompression mode 2: the region (values)
  Region rblk;          // decompression mode 2 on the specialised decoder: the blocks it touches
  ScanSrc ss;           // what the block scans read, and where they write
  uint64_t *sc_part, *sc_off_pay, *sc_tot;
  uint32_t *sc_off_out, *sc_off_coef;
  const uint8_t *src;   // compression: the field's values; decompression: its stream
  uint8_t *dst;         // compression: the stream buffer; decompression: the output values
  uint64_t dst_cap;
  uint32_t *zero;       // cleared at the start of the call
  uint64_t zero_words;
  const uint64_t *stat; // counters and results read back at the end of the call
  uint32_t stat_words;
  double eb;
  uint32_t dtype, abft, predictor, eb_mode, mode, nparts, n_sym;
  uint32_t hist_win;  // codes counted in LDS by the compression kernel (<= kHistWin)
  const uint32_t *hdr_expect;  // decompression: the header the caller gave (device copy), or null
  uint32_t *hdr_keep;          // region decoding state: the header its tables were built from
  RegTab<float> rtf;
  RegTab<double> rtd;
};

template <typename T> __device__ __host__ inline const RegTab<T> &rt_of(const Job &J);
template <> __device__ __host__ inline const RegTab<float> &rt_of<float>(const Job &J) { return J.rtf; }
template <> __device__ __host__ inline const RegTab<double> &rt_of<double>(const Job &J) { return J.rtd; }

// The work-groups of one launch: the slot-th job of the launch is
// jobs[id[slot]] and owns work-groups [wg[slot], wg[slot + 1]).
struct JobTab {
  const Job *jobs;
  const uint32_t *wg;  // n + 1 entries
  const uint32_t *id;  // n entries
  uint32_t n;
};

// slot of the job that owns work-group b (wg[] ascending, wg[0] = 0)
__device__ inline uint32_t job_slot(const JobTab &t, uint32_t b) {
  uint32_t lo = 0, hi = t.n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (t.wg[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The calling work-group's job, its index in the job's share of the launch
// and the size of that share.
struct JobWg {
  const Job *J;
  uint32_t b, nb, slot;
};
__device__ inline JobWg job_of(const JobTab &t) {
  const uint32_t s = job_slot(t, blockIdx.x);
  return JobWg{t.jobs + t.id[s], blockIdx.x - t.wg[s], t.wg[s + 1] - t.wg[s], s};
}

__global__ void k_zero_u64(unsigned long long *p, uint64_t n);
__global__ void k_zero_u32(uint32_t *p, uint64_t n);
__global__ void k_zero_jobs(JobTab t);
__global__ void k_plan_bits(JobTab t);
template <typename T> __global__ void k_range(JobTab t);
__global__ void k_consts(JobTab t);
__global__ void k_code_faults(PlanDev plan, Geo g, uint16_t *codes, unsigned long long *cnt);
__global__ void k_codes_check(JobTab t);
__global__ void k_scan1(JobTab t);
__global__ void k_scan2(JobTab t);
__global__ void k_scan3(JobTab t);
template <typename T> __global__ void k_encode(JobTab t);
__global__ void k_hist_count(JobTab t, uint32_t *chunk_cnt);
__global__ void k_hist_scan(uint32_t n, uint32_t *chunk_cnt, uint32_t *counts, uint32_t *hcounts);
__global__ void k_hist_pack(JobTab t, const uint32_t *chunk_off, uint64_t *dst, uint64_t *hdst, uint64_t hn);
__global__ void k_put_codes(JobTab t);
__global__ void k_header(JobTab t);
__global__ void k_results(JobTab t, uint64_t *dst, uint32_t per);
__global__ void k_headers(JobTab t, uint8_t *dst);
__global__ void k_dectab(JobTab t);
__global__ void k_dec_check(JobTab t);
__global__ void k_hdr_keep(JobTab t, uint32_t mode);

template <typename T, int ND, int B0, int B1, int B2, bool ABFT, bool WIDE, bool FAULTS, int PART>
__global__ void k_compress_fast(JobTab t);
template <typename T, int ND, int B0, int B1, int B2, bool WIDE, bool FAULTS> __global__ void k_decode_fast(JobTab t);

template <int ND, int B0, int B1, int B2> __global__ void k_check_fast(JobTab t);
template <typename T, int ND, int B0, int B1, int B2> __global__ void k_encode_fast(JobTab t);
template <typename T, int B0, int B1, int B2> __global__ void k_checkenc_fast(JobTab t);
constexpr uint32_t kEncTile = 256;  // blocks per tile of k_checkenc_fast (its work-group)

// Wave-per-block kernels (kern_wave.hip): one block per work-group of 64
// lanes, staged in dynamic LDS of wave_lds_bytes().
constexpr uint32_t kWaveDupBytes = 12;            // LDS per plan entry of the duplicated computations
constexpr uint32_t kWaveLdsMax = 64 * 1024;       // blocks needing more take the one-thread kernels
__host__ __device__ inline uint32_t wave_rsz(const Geo &g) {
  const uint32_t parts = g.b[0] * g.b[1] + g.b[0] * g.b[2] + 3 * g.b[0];
  return g.bpts > parts ? g.bpts : parts;
}
__host__ __device__ inline uint32_t wave_lds_bytes(const Geo &g, uint32_t vbytes) {
  const uint32_t rsz = wave_rsz(g);
  return 2 * rsz * vbytes + 4 * ((rsz + 31) / 32) + kMaxPatches * kWaveDupBytes;
}
// one wave's slice of a multi-wave work-group (16-byte aligned)
__host__ __device__ inline uint32_t wave_slice_bytes(const Geo &g, uint32_t vbytes) {
  return (wave_lds_bytes(g, vbytes) + 15) & ~15u;
}
constexpr uint32_t kWaveWgWaves = 4;          // most waves per work-group of k_compress_wave
constexpr uint32_t kWaveWgMax = 2048;          // work-groups per field of k_compress_wave
constexpr uint32_t kWaveWgLds = 150 * 1024;    // dynamic LDS of one of its work-groups at most
template <typename T> __global__ void k_compress_wave(JobTab t, uint32_t slice);
template <typename T> __global__ void k_compress_wave_list(JobTab t);
template <typename T> __global__ void k_redo_wave(JobTab t);
template <typename T> __global__ void k_decode_wave_list(JobTab t);
template <typename T> __global__ void k_decode_wave_redo(JobTab t, uint32_t queue);
template <typename T> __global__ void k_decode_wave_region(JobTab t);
constexpr uint64_t kWaveRegionBlocks = 4096;  // regions of at most this many blocks take k_decode_wave_region

template <typename T> __global__ void k_compress_generic(JobTab t);
template <typename T> __global__ void k_decode_generic(JobTab t);

// Lossless stage (kern_pack.hip): the block table and sum_dc packed per chunk
// of kPackChunk blocks by frame of reference; every other section verbatim.
constexpr uint32_t kPackChunk = 256;
constexpr uint32_t kPackColWords = kPackChunk * 64 / 32;  // packed words of a chunk column at most
struct PackChunk {
  uint64_t base[3];   // column minima: payload words, outliers << 1 | regression, sum_dc
  uint32_t width[3];  // bits per packed difference (0..64)
  uint32_t words_t, words_s;  // words of the chunk in the table and sum_dc sections
  uint32_t off_t, off_s;      // their word offsets in the sections' data (after the scan)
};
struct PackArgs {
  const uint8_t *src;      // plain stream
  uint8_t *dst;            // packed stream
  PackChunk *info;         // nch entries
  uint64_t *res;           // [0] table section words, [1] sum_dc section words
  uint64_t nb, nch;
  uint64_t src_table, src_sumdc;  // plain-stream byte offsets
  uint64_t dst_table, dst_sumdc;  // packed-stream byte offsets (dst_sumdc set once scanned)
  uint32_t abft, n_pads;
  uint64_t pads[6];        // 4-byte words of alignment padding to clear
  uint32_t hdr[kHeader / 4];
};
struct UnpackArgs {
  const uint8_t *src;      // packed stream
  uint8_t *dst;            // plain stream
  uint32_t *err;           // set when the packed sections are not valid
  uint64_t nb, nch;
  uint64_t src_table, src_sumdc, src_total;  // packed-stream byte offsets
  uint64_t dst_table, dst_sumdc;             // plain-stream byte offsets
  uint32_t abft, n_pads;
  uint32_t write;          // 0: check the sections only (the output is too small)
  uint64_t pads[6];
  uint32_t hdr[kHeader / 4];
};
__global__ void k_pack_sizes(PackArgs a);
__global__ void k_pack_scan(PackArgs a);
__global__ void k_pack_write(PackArgs a);
__global__ void k_unpack_check(UnpackArgs a);
__global__ void k_unpack_chunks(UnpackArgs a);

}  // namespace sdcsz
