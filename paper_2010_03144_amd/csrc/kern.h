// kern.h -- kernel declarations (definitions in kern_*.hip).
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
constexpr uint32_t kScanItems = 8;
constexpr uint32_t kScanChunk = kScanThreads * kScanItems;
constexpr uint32_t kRangeThreads = 256;
constexpr uint32_t kHistWin = 2048;  // codes counted in LDS around the radius

// Work of one specialised launch: work-groups [0, full_wgs) take the
// sub-grid of full blocks, the others the shell of partial blocks at the
// upper edges (the slab of blocks partial along the fastest axis, then the
// middle, then the slowest, each excluding the earlier slabs).
struct Launch {
  uint32_t nf[3];      // full blocks per axis
  uint32_t full_wgs;   // work-groups of full blocks
  uint64_t s2, s1;     // sizes of the first two shell slabs
  uint64_t full_count, shell_count;
};
constexpr uint32_t kRangeBlocks = 2048;

__global__ void k_zero_u64(unsigned long long *p, uint64_t n);
__global__ void k_zero_u32(uint32_t *p, uint64_t n);
template <typename T> __global__ void k_range(const T *in, uint64_t n, double *part);
__global__ void k_consts(const double *part, uint32_t nparts, uint32_t mode, double eb, EbDev *out);
__global__ void k_code_faults(PlanDev plan, Geo g, uint16_t *codes, unsigned long long *cnt);
__global__ void k_codes_check(Geo g, CompWork w, uint32_t abft);
__global__ void k_scan1(ScanSrc src, uint64_t n, uint64_t *part);
__global__ void k_scan2(uint64_t *part, uint32_t nparts);
__global__ void k_scan3(ScanSrc src, uint64_t n, const uint64_t *part, uint64_t *off_pay,
                        uint32_t *off_out, uint32_t *off_coef, uint64_t *tot);
__global__ void k_put_codes(const uint32_t *cb, uint32_t n_sym, uint32_t *enc);
__global__ void k_header(Header h, CompWork w, uint8_t *out, uint64_t out_cap);
__global__ void k_dectab(const uint32_t *cbk, uint32_t n_sym, DecWork w);
__global__ void k_dec_check(const uint64_t *tot, uint64_t payload_words, uint64_t n_outliers,
                            uint64_t n_regression, uint32_t *err);
template <typename T>
__global__ void k_encode(Geo g, CompWork w, uint8_t *out);

template <typename T, int ND, int B0, int B1, int B2, bool ABFT>
__global__ void k_compress_fast(const T *in, Geo g, RegTab<T> rt, PlanDev plan, CompWork w, uint32_t predictor,
                                Launch L);
template <typename T>
__global__ void k_compress_list(const T *in, Geo g, RegTab<T> rt, PlanDev plan, CompWork w, uint32_t abft,
                                uint32_t predictor, const uint64_t *list, uint32_t n);
template <typename T>
__global__ void k_redo(const T *in, Geo g, RegTab<T> rt, PlanDev plan, CompWork w, uint32_t abft,
                       uint32_t predictor);

template <typename T, int ND, int B0, int B1, int B2>
__global__ void k_decode_fast(const uint8_t *s, Header h, Geo g, DecWork w, PlanDev plan, T *out, Launch L);
template <typename T>
__global__ void k_decode_list(const uint8_t *s, Header h, Geo g, DecWork w, PlanDev plan, T *out,
                              const uint64_t *list, uint32_t n);
template <typename T>
__global__ void k_decode_redo(const uint8_t *s, Header h, Geo g, DecWork w, T *out);

template <int B0, int B1, int B2> __global__ void k_check_fast(Geo g, CompWork w, uint32_t abft);
template <typename T, int B0, int B1, int B2>
__global__ void k_encode_fast(Geo g, CompWork w, uint8_t *out);

template <typename T>
__global__ void k_compress_generic(const T *in, Geo g, RegTab<T> rt, PlanDev plan, CompWork w,
                                   uint32_t abft, uint32_t predictor);
template <typename T>
__global__ void k_decode_generic(const uint8_t *s, Header h, Geo g, DecWork w, PlanDev plan,
                                 T *out, uint32_t mode, Region reg);

}  // namespace sdcsz
