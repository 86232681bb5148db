/*
 * sdcsz_ref.h -- CPU oracle of the SDC-resilient independent-block compressor.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle/sdcsz_ref.cpp are a plain,
 * slow, single-threaded restatement of the method of "SDC Resilient
 * Error-bounded Lossy Compressor" (arXiv 2010.03144): Algorithm 1 (fault
 * tolerant compression), Algorithm 2 (fault tolerant decompression), the
 * checksum pair of Sec. 3.2 and the integer reinterpretation of Sec. 5.4.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or table with the HIP library; the
 * structures below only mirror the public ABI's layout so that a test can
 * hand both sides the same bytes.
 *
 * Every function is pure host code on host pointers.
 */
#ifndef SDCSZ_REF_H
#define SDCSZ_REF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_F32 = 0, REF_F64 = 1 };
enum { REF_ABS = 0, REF_REL = 1 };
enum { REF_PRED_AUTO = 0, REF_PRED_LORENZO = 1, REF_PRED_REGRESSION = 2 };
enum {
  REF_T_INPUT = 0,     /* input word after its checksums were taken      */
  REF_T_COEF = 1,      /* regression-coefficient word                    */
  REF_T_CODE = 2,      /* quantization code at rest before encoding      */
  REF_T_RECON = 3,     /* decompressed word before its checksum          */
  REF_T_DUP_PRED = 4,  /* first copy of the duplicated prediction        */
  REF_T_DUP_RECON = 5, /* first copy of the duplicated reconstruction    */
  REF_T_PREP_INPUT = 6,  /* input word after its checksums, before the
                            regression and the sampling read it           */
  REF_T_PREP_COEF = 7,   /* computed coefficient before its checksums     */
  REF_T_PREP_SAMPLE = 8, /* sampled estimate (word 0 Lorenzo, 1 regression,
                            bit < 64) before the predictor comparison     */
  REF_N_TARGETS = 9
};
enum { REF_OK = 0, REF_EINVAL = -1, REF_ENOSPC = -2, REF_EFORMAT = -3, REF_ESDC = -4 };

typedef struct {
  uint32_t target; /* REF_T_*                                                  */
  uint32_t bit;    /* bit to flip (CODE: taken modulo 16)                      */
  uint64_t block;  /* linear block id                                          */
  uint64_t word;   /* INPUT/RECON: 32-bit word index in the block; COEF: word of
                      the 4 coefficients; CODE/DUP_*: point index in the block */
} ref_fault;

typedef struct {
  uint32_t dtype;     /* REF_F32 / REF_F64                                   */
  uint32_t ndim;      /* 1..3                                                */
  uint64_t dims[3];   /* first ndim entries used, C order, dims[0] slowest   */
  uint32_t block[3];  /* block edge per used axis                            */
  uint32_t eb_mode;   /* REF_ABS / REF_REL                                   */
  uint32_t predictor; /* REF_PRED_*                                          */
  double eb;          /* error bound (absolute, or relative to value range)  */
  uint32_t abft;      /* 1: checksums + duplicated instructions; 0: plain     */
  uint32_t n_faults;
  const ref_fault *faults; /* host array, may be NULL when n_faults == 0     */
} ref_params;

typedef struct {
  uint64_t n_blocks;
  uint64_t injected[REF_N_TARGETS];
  uint64_t detected[REF_N_TARGETS];
  uint64_t corrected[REF_N_TARGETS];
  uint64_t uncorrectable[REF_N_TARGETS];
  uint64_t n_outliers;
  uint64_t n_regression;
  uint64_t payload_words;
  uint64_t stream_size;
  double eb_abs;
} ref_report;

/* Optional per-point / per-block views of compression internals, for tests.
 * Any pointer may be NULL.  codes: n_values entries in block order, C order
 * inside each block (after the bound check, before CODE faults).
 * is_regression: n_blocks bytes.  coef: 4*n_blocks values of the field type.
 * hist: 65536 counts.  lengths: 65536 code lengths. */
typedef struct {
  uint16_t *codes;
  uint8_t *is_regression;
  void *coef;
  uint64_t *hist;
  uint8_t *lengths;
} ref_debug;

uint64_t sdcsz_ref_max_stream_size(const ref_params *p);
int sdcsz_ref_compress(const void *in, const ref_params *p, void *out, uint64_t out_cap,
                       uint64_t *out_size, ref_report *rep, ref_debug *dbg);
int sdcsz_ref_decompress(const void *stream, uint64_t stream_size, void *out, uint64_t out_cap,
                         const ref_fault *faults, uint32_t n_faults, ref_report *rep);
int sdcsz_ref_decompress_region(const void *stream, uint64_t stream_size, const uint64_t lo[3],
                                const uint64_t hi[3], void *out, uint64_t out_cap,
                                ref_report *rep);
int sdcsz_ref_verify(const void *stream, uint64_t stream_size, void *data, uint64_t data_size,
                     const ref_fault *faults, uint32_t n_faults, ref_report *rep);

/* Lossless stage after Huffman coding: the block table and sum_dc of a plain
 * stream ("v1") packed per chunk of 256 blocks by frame of reference into a
 * packed stream ("v2"), and back.  *out_size receives the size (also the
 * required size on REF_ENOSPC).  REF_EFORMAT: not a stream of the input
 * version, or inconsistent sections. */
int sdcsz_ref_pack(const void *stream, uint64_t size, void *out, uint64_t cap, uint64_t *out_size);
int sdcsz_ref_unpack(const void *packed, uint64_t size, void *out, uint64_t cap, uint64_t *out_size);
/* One frame-of-reference column of n values: base low, base high, width,
 * packed words; returns the word count (out may be NULL to size it). */
uint64_t sdcsz_ref_pack_column(const uint64_t *v, uint64_t n, uint32_t *out);
/* Building blocks exposed so that tests can pin them one by one. */
void sdcsz_ref_checksums(const uint32_t *w, uint64_t n, uint64_t *sum, uint64_t *isum);
/* 0 = clean, 1 = corrected, -1 = uncorrectable; width = 32 or 16 bits. */
int sdcsz_ref_correct(uint32_t *w, uint64_t n, uint64_t sum, uint64_t isum, uint32_t width);
/* coef[4] = beta0, beta1, beta2, mu of the centred least-squares plane. */
void sdcsz_ref_regression(const void *vals, uint32_t dtype, const uint32_t ext[3], void *coef);
/* Code lengths of the length-limited Huffman code (limit 24). */
void sdcsz_ref_huffman_lengths(const uint64_t *hist, uint8_t *lengths);
int sdcsz_ref_read_header(const void *stream, uint64_t stream_size, ref_params *p,
                          double *eb_abs, uint64_t *n_blocks);

#ifdef __cplusplus
}
#endif
#endif
