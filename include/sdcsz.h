/*
 * sdcsz.h -- C ABI of the MI355X (gfx950) SDC-resilient error-bounded lossy
 * compressor: independent-block compression and decompression of FP32/FP64
 * fields with ABFT protection, after "SDC Resilient Error-bounded Lossy
 * Compressor" (arXiv 2010.03144).
 *
 * Conventions shared by every entry point
 *  - Pointers named d_* are device pointers (HIP device memory of the current
 *    device); h_* and plain structs are host memory.  `stream` is a
 *    hipStream_t passed as void* (NULL = the legacy default stream).
 *  - The caller owns every buffer.  The library allocates no device memory
 *    and frees nothing: each call takes a caller-provided device workspace of
 *    at least the size the matching *_workspace_size() reports.
 *  - All device work starts after the work queued on `stream` before the
 *    call, and `stream` waits for all of it: part of it (fault-plan blocks,
 *    the compressor's partial blocks) runs on streams the library keeps per
 *    calling thread, forked from `stream` and joined back into it.  Calls
 *    that return host results (sizes, reports) synchronise that stream
 *    before returning.
 *  - Errors are negative return codes (SDCSZ_E*); nothing throws or aborts
 *    across the ABI.  sdcsz_strerror() names them.
 */
#ifndef SDCSZ_H
#define SDCSZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDCSZ_OK 0
#define SDCSZ_EINVAL (-1)  /* bad dims/block/eb/fault plan/size argument          */
#define SDCSZ_ENOSPC (-2)  /* output or workspace too small (required size set)    */
#define SDCSZ_EFORMAT (-3) /* not a stream of this format, or inconsistent sections */
#define SDCSZ_ESDC (-4)    /* uncorrectable silent data corruption (Algorithm 2,
                              "SDC in compression"), or a code with no codeword   */
#define SDCSZ_EHIP (-5)    /* HIP runtime error                                     */

enum { SDCSZ_F32 = 0, SDCSZ_F64 = 1 };
/* error-bound mode: absolute, or relative to the value range of the finite
 * values (Sec. 6.1, "value-range based error bound") */
enum { SDCSZ_ABS = 0, SDCSZ_REL = 1 };
/* predictor choice per block: sampled selection (Algorithm 1, second loop), or
 * forced */
enum { SDCSZ_PRED_AUTO = 0, SDCSZ_PRED_LORENZO = 1, SDCSZ_PRED_REGRESSION = 2 };

/* Fault-injection targets (evaluation mode A, Sec. 6.1; decompression errors,
 * Sec. 5.3; errors in the prediction preparation, Sec. 4.1 and 4.2).  A plan
 * is plain data applied at fixed program points. */
enum {
  SDCSZ_T_INPUT = 0,     /* input word, after the block's input checksums and
                            after predictor selection                          */
  SDCSZ_T_COEF = 1,      /* regression-coefficient word, after its checksums  */
  SDCSZ_T_CODE = 2,      /* quantization code at rest, before encoding        */
  SDCSZ_T_RECON = 3,     /* decompressed word, before its checksum            */
  SDCSZ_T_DUP_PRED = 4,  /* first copy of the duplicated prediction           */
  SDCSZ_T_DUP_RECON = 5, /* first copy of the duplicated reconstruction       */
  SDCSZ_T_PREP_INPUT = 6,  /* input word, after the input checksums but before
                              regression and sampling read it (the memory
                              error persists until the input is checked)     */
  SDCSZ_T_PREP_COEF = 7,   /* computed regression coefficient, before its
                              checksums are taken (a computation error)      */
  SDCSZ_T_PREP_SAMPLE = 8, /* sampled error estimate before the predictor
                              comparison (a computation error): word 0 the
                              Lorenzo estimate, word 1 the regression one    */
  SDCSZ_N_TARGETS = 9
};

typedef struct {
  uint32_t target; /* SDCSZ_T_*                                                 */
  uint32_t bit;    /* bit to flip: < 32 for word targets (CODE: taken mod 16),
                      < 32 * words-per-value for DUP_* targets, < 64 for
                      PREP_SAMPLE (the estimates are 64-bit integers)          */
  uint64_t block;  /* linear block id (C order over the block grid)             */
  uint64_t word;   /* INPUT/PREP_INPUT/RECON: 32-bit word in the block (FP64: 2
                      per value, low half first); COEF/PREP_COEF: word of the
                      4 coefficients; CODE/DUP_*: point index (C order inside
                      the block); PREP_SAMPLE: 0 or 1                          */
} sdcsz_fault;

typedef struct {
  uint32_t dtype;     /* SDCSZ_F32 / SDCSZ_F64                                  */
  uint32_t ndim;      /* 1..3                                                   */
  uint64_t dims[3];   /* first ndim entries, C order (dims[0] slowest)          */
  uint32_t block[3];  /* block edge per used axis (Sec. 5.1; 6x6x6 in SZ)       */
  uint32_t eb_mode;   /* SDCSZ_ABS / SDCSZ_REL                                  */
  uint32_t predictor; /* SDCSZ_PRED_*                                           */
  double eb;          /* error bound: finite and > 0                            */
  uint32_t abft;      /* 1: checksums + instruction duplication (ftrsz); 0: not */
  uint32_t n_faults;  /* entries in `faults` (compression uses every target but
                         RECON, which it ignores)                               */
  const sdcsz_fault *faults; /* host array, NULL when n_faults == 0             */
} sdcsz_params;

typedef struct {
  uint64_t n_blocks;
  uint64_t injected[SDCSZ_N_TARGETS];
  uint64_t detected[SDCSZ_N_TARGETS];
  uint64_t corrected[SDCSZ_N_TARGETS];
  uint64_t uncorrectable[SDCSZ_N_TARGETS];
  uint64_t n_outliers;    /* values stored verbatim                          */
  uint64_t n_regression;  /* blocks predicted by regression                  */
  uint64_t payload_words; /* 32-bit words of Huffman payload                 */
  uint64_t stream_size;   /* bytes of the compressed stream                  */
  double eb_abs;          /* absolute bound actually enforced                */
  uint64_t generic_plan_blocks; /* fault-plan blocks of a field with specialised
                             kernels that the generic per-block routine ran
                             instead (errors of the prediction preparation,
                             several flips of a kind in one block, fields of
                             2 GiB or more); the others run in the specialised
                             kernels' fault-applying instantiation            */
} sdcsz_report;

/* Upper bound of the stream size for these parameters (0 if invalid). */
uint64_t sdcsz_max_compressed_size(const sdcsz_params *p);

/* Device workspace that sdcsz_compress needs for these parameters (0 if
 * invalid).  Dominated by the per-point code and outlier staging areas. */
uint64_t sdcsz_compress_workspace_size(const sdcsz_params *p);

/*
 * Compress a field: Algorithm 1 (fault tolerant compression) without its final
 * lossless stage.  Per independent block (Sec. 5.1): regression coefficients
 * and input/coefficient checksums (Sec. 3.2, integer words per Sec. 5.4);
 * sampled predictor selection; detection and correction of the input and the
 * coefficients; duplicated prediction and reconstruction; linear-scaling
 * quantization with outliers kept verbatim and the double check of the bound;
 * code checksums and the decompressed-data checksum sum_dc.  Then one
 * Huffman code over all codes, detection/correction of the codes and
 * per-block encoding.
 *   d_in      device, dims[0]*dims[1]*dims[2] values of dtype, C order; read only
 *   d_out     device, out_cap bytes, 8-byte aligned; receives the stream.
 *             Nothing is written to it on SDCSZ_ENOSPC.  On SDCSZ_ESDC its
 *             contents are undefined when out_cap >= sdcsz_max_compressed_size
 *             (6x6x6 fields then check and encode their codes in one pass,
 *             which writes the stream before the call knows that a block
 *             stays uncorrectable), else nothing is written.
 *   h_out_size host; receives the stream size (also on SDCSZ_ENOSPC: the
 *             required size)
 *   h_rep     host, may be NULL; fault counters and stream statistics
 *   d_ws      device workspace of ws_size >= sdcsz_compress_workspace_size(p)
 * Returns SDCSZ_OK, SDCSZ_EINVAL, SDCSZ_ENOSPC, SDCSZ_ESDC (an uncorrectable
 * corruption, a code without codeword when ABFT is off, or more than 4096
 * blocks whose checks disagree in one call: the re-execution queue holds
 * 4096), SDCSZ_EHIP.
 * Synchronises `stream` twice: for the code histogram (the Huffman code is
 * built on the host; a third time when more than 32768 symbols are used) and
 * at the end.  The calling thread keeps a pinned host staging buffer (8 MiB,
 * doubled when a large batch needs more) from its first call until it exits.
 */
int sdcsz_compress(const void *d_in, const sdcsz_params *p, void *d_out, uint64_t out_cap,
                   uint64_t *h_out_size, sdcsz_report *h_rep, void *d_ws, uint64_t ws_size,
                   void *stream);

/*
 * Read the parameters recorded in a stream's header (the stream may stay in
 * device memory).  Fills *h_p (faults = NULL), *h_n_blocks and *h_eb_abs
 * (either may be NULL).  Returns SDCSZ_OK or SDCSZ_EFORMAT.  Synchronises.
 */
int sdcsz_stream_info(const void *d_stream, uint64_t stream_size, sdcsz_params *h_p,
                      uint64_t *h_n_blocks, double *h_eb_abs, void *stream);

/* Device workspace that sdcsz_decompress / sdcsz_verify / region decoding
 * need for a stream with these parameters (0 if invalid). */
uint64_t sdcsz_decompress_workspace_size(const sdcsz_params *p);

/*
 * Decompress a stream: Algorithm 2.  Every block is decoded and
 * reconstructed with the arithmetic of compression; with ABFT its checksum is
 * compared with sum_dc and a mismatch re-executes the block from the
 * compressed bytes (random-access decompression); a second mismatch marks the
 * block uncorrectable, the other blocks still finish, and SDCSZ_ESDC is
 * returned.  RECON entries of the fault plan strike the decompressed words
 * before the checksum.
 *   d_stream  device, stream_size bytes
 *   d_out     device, out_cap >= n_values * sizeof(dtype) bytes, C order
 *   h_faults  host, n_faults entries (only SDCSZ_T_RECON is used), may be NULL
 * Returns SDCSZ_OK, SDCSZ_EINVAL, SDCSZ_ENOSPC, SDCSZ_EFORMAT, SDCSZ_ESDC,
 * SDCSZ_EHIP.  Synchronises `stream`.
 */
int sdcsz_decompress(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap,
                     const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep,
                     void *d_ws, uint64_t ws_size, void *stream);

/*
 * Decompression that allocates nothing, for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): sdcsz_decompress with the same kernels and results,
 * but its workspace is a fixed device array of SDCSZ_NOALLOC_SCRATCH_BYTES
 * inside the library (one per GPU, held from the library's load until the
 * process ends) and its host staging a static buffer; it calls no hipMalloc,
 * hipFree, hipHostMalloc or other device or pinned-memory allocator.
 *   d_stream, d_out, h_faults, h_rep: as for sdcsz_decompress (the caller
 *             passes the stream and the output buffer)
 * Streams of block shapes with a specialised decoder (6x6x6 in 3D, 16x16 in
 * 2D) and no fault plan need about 16 bytes per block plus 0.5 MiB of the
 * array, so fields up to about 4 million blocks fit; other shapes and
 * fault plans stage every block's values there and fit only when small.
 * A stream whose workspace exceeds the array returns SDCSZ_ENOSPC and
 * writes nothing.  More than 4096 blocks that fail their checksum cannot
 * all be re-executed here: the others stay uncorrected, are counted
 * uncorrectable and the call returns SDCSZ_ESDC.
 * Calls are serialised inside the process (the array and the host staging
 * are shared); each call clears the counters it needs with a kernel, and the
 * array keeps the last call's contents.  Synchronises `stream`.
 */
#define SDCSZ_NOALLOC_SCRATCH_BYTES (64ull * 1024 * 1024)
int sdcsz_decompress_noalloc(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap,
                             const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *stream);

/*
 * Stand-alone check of a decompressed buffer held by the caller (the checksum
 * half of Algorithm 2): each block's checksum is compared with sum_dc; a
 * mismatching block is decoded again from the stream and written over the
 * caller's copy.  The stream must carry ABFT checksums (else SDCSZ_EINVAL).
 *   d_data    device, data_size bytes, repaired in place
 * RECON entries of the plan strike d_data's words before the check.
 */
int sdcsz_verify(const void *d_stream, uint64_t stream_size, void *d_data, uint64_t data_size,
                 const sdcsz_fault *h_faults, uint32_t n_faults, sdcsz_report *h_rep, void *d_ws,
                 uint64_t ws_size, void *stream);

/*
 * Random-access decompression of the box [lo, hi) (Sec. 5.1): only the blocks
 * that intersect the box are decoded (checked and re-executed as in
 * sdcsz_decompress); the box is written to d_out in C order.
 *   h_lo, h_hi host arrays of ndim entries, lo < hi <= dims
 *   d_out      device, out_cap >= prod(hi - lo) * sizeof(dtype)
 */
int sdcsz_decompress_region(const void *d_stream, uint64_t stream_size, const uint64_t *h_lo,
                            const uint64_t *h_hi, void *d_out, uint64_t out_cap,
                            sdcsz_report *h_rep, void *d_ws, uint64_t ws_size, void *stream);

/*
 * Repeated random access to one stream (Sec. 5.1): sdcsz_region_prepare
 * builds the stream's decoding tables and its per-block offsets (a scan of
 * the whole block table) in d_ws, together with a copy of the header;
 * sdcsz_decompress_region_prepared then decodes a box [lo, hi) with them,
 * touching only the blocks that intersect it (a box that is the whole field
 * takes the full-field decoder).  Each prepared call first checks on the
 * device that the stream still carries the header the state was built
 * from, and returns SDCSZ_EFORMAT if not; the stream's other bytes must not
 * change in between (ABFT streams would report the blocks that then fail
 * their checksum).
 *   h_header  host, the stream's 192 header bytes (as compression returned
 *             them), or NULL to read them from the device (one more
 *             synchronisation); checked against the stream on the device
 *   d_ws      device workspace of ws_size >= sdcsz_decompress_workspace_size()
 *             for the stream's parameters; the same buffer, unchanged by other
 *             calls, for the prepare call and the calls that use it
 *   h_lo, h_hi, d_out, out_cap, h_rep: as for sdcsz_decompress_region
 * Return codes as for sdcsz_decompress_region.  Each call synchronises
 * `stream` once at its end.
 */
int sdcsz_region_prepare(const void *d_stream, uint64_t stream_size, const void *h_header, void *d_ws,
                         uint64_t ws_size, void *stream);
int sdcsz_decompress_region_prepared(const void *d_stream, uint64_t stream_size, const void *h_header,
                                     const uint64_t *h_lo, const uint64_t *h_hi, void *d_out, uint64_t out_cap,
                                     sdcsz_report *h_rep, void *d_ws, uint64_t ws_size, void *stream);

/*
 * Lossless stage (the last pass of Algorithm 1 and the first of Algorithm 2):
 * the per-block metadata that Huffman coding leaves redundant -- the block
 * table (payload words; outliers << 1 | regression flag) and, with ABFT,
 * sum_dc -- is packed per chunk of 256 blocks by frame of reference (each
 * chunk column: its minimum, a bit width, the differences in that width), so
 * a block's entries are still read from its own chunk (random access).
 * Codebook, coefficients, outliers and payload move unchanged.  A packed
 * stream has the magic "SDCSZ\0v2"; the other entry points take plain
 * streams, so a packed one is unpacked first.  Any change to the packed
 * metadata that still unpacks is caught by the block checksums of
 * decompression (ABFT streams), like a change to the plain stream.
 */
/* Device workspace of sdcsz_pack for a stream of n_blocks blocks (the
 * header's block count). */
uint64_t sdcsz_pack_workspace_size(uint64_t n_blocks);
#define SDCSZ_UNPACK_WORKSPACE_BYTES 256

/*
 * Pack a plain stream.
 *   d_stream  device, stream_size bytes, 8-byte aligned; read only
 *   d_out     device, out_cap bytes, 8-byte aligned, not overlapping d_stream;
 *             receives the packed stream (nothing is written on an error);
 *             NULL with out_cap 0 asks for the size (SDCSZ_ENOSPC)
 *   h_out_size host; the packed size (also on SDCSZ_ENOSPC: the size needed)
 *   d_ws      device workspace, ws_size >= sdcsz_pack_workspace_size()
 * Returns SDCSZ_OK, SDCSZ_EINVAL (null or misaligned pointer), SDCSZ_EFORMAT
 * (not a plain stream), SDCSZ_ENOSPC, SDCSZ_EHIP.  Synchronises `stream`
 * twice (header, section sizes); the writes of the packed stream are queued
 * on `stream` when the call returns.
 */
int sdcsz_pack(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap, uint64_t *h_out_size,
               void *d_ws, uint64_t ws_size, void *stream);

/*
 * Unpack a packed stream into the plain stream it was made from (byte for
 * byte).
 *   d_packed  device, packed_size bytes, 8-byte aligned; read only
 *   d_out     device, out_cap bytes, 8-byte aligned, not overlapping d_packed;
 *             NULL with out_cap 0 asks for the size (SDCSZ_ENOSPC)
 *   h_out_size host; the plain size (also on SDCSZ_ENOSPC)
 *   d_ws      device workspace of ws_size >= SDCSZ_UNPACK_WORKSPACE_BYTES
 * Returns SDCSZ_OK, SDCSZ_EINVAL, SDCSZ_EFORMAT (not a packed stream, or its
 * packed sections are inconsistent: then d_out's contents are undefined),
 * SDCSZ_ENOSPC (nothing written), SDCSZ_EHIP.  Synchronises `stream` twice.
 */
int sdcsz_unpack(const void *d_packed, uint64_t packed_size, void *d_out, uint64_t out_cap, uint64_t *h_out_size,
                 void *d_ws, uint64_t ws_size, void *stream);

/*
 * Batches: many fields in one call (the independent-block design of Sec. 5.1
 * makes fields, like blocks, independent units of work).  Each phase runs as
 * one launch per kernel class over all fields of the batch (a table on the
 * device names the field of every work-group), and the host synchronises
 * for the whole batch: compression once for the code histograms (twice when
 * they hold more than 32768 used symbols in all), once at the end;
 * decompression once for the headers (skipped when every item brings its
 * header) and once at the end.  Every field is
 * processed exactly as a single call would process it: its stream, output
 * and report are identical.  Huffman codes of a batch are built on up to 16
 * host threads.
 */
#define SDCSZ_HEADER_BYTES 192 /* fixed size of a stream's header */

typedef struct {
  const void *d_in;      /* device: the field, C order (as for sdcsz_compress)      */
  sdcsz_params params;   /* the field's parameters (faults: host array or NULL)    */
  void *d_out;           /* device: the field's stream buffer, out_cap bytes       */
  uint64_t out_cap;
  uint64_t out_size;     /* out: stream size (required size on SDCSZ_ENOSPC)      */
  int rc;                /* out: this field's return code                          */
  sdcsz_report rep;      /* out                                                    */
  uint8_t header[SDCSZ_HEADER_BYTES]; /* out: the stream's header, when written;
                            pass it to sdcsz_decompress_batch to spare the
                            header read-back there                              */
} sdcsz_comp_item;

/* Device workspace for sdcsz_compress_batch on these items (fields with
 * invalid parameters count for nothing). */
uint64_t sdcsz_compress_batch_workspace_size(const sdcsz_comp_item *h_items, uint32_t n);

/*
 * Compress n fields.  h_items: host array; each item's rc, out_size and rep
 * are written.  Returns SDCSZ_OK when every field succeeded, else the first
 * failing item's code (SDCSZ_ENOSPC for every item when the workspace is too
 * small, SDCSZ_EHIP on a runtime error).  Synchronises `stream`.
 */
int sdcsz_compress_batch(sdcsz_comp_item *h_items, uint32_t n, void *d_ws, uint64_t ws_size,
                         void *stream);

typedef struct {
  const void *d_stream;  /* device: a stream, stream_size bytes                    */
  uint64_t stream_size;
  void *d_out;           /* device: n_values * sizeof(dtype) bytes, C order        */
  uint64_t out_cap;
  const sdcsz_fault *faults;  /* host, n_faults entries (SDCSZ_T_RECON), or NULL   */
  uint32_t n_faults;
  const void *h_header;  /* host copy of the stream's SDCSZ_HEADER_BYTES header (as
                            returned by the compression), or NULL: then the
                            header is read back from the device first (one
                            more synchronisation).  A given header is checked
                            against the stream's own on the device; a mismatch
                            ends the item in SDCSZ_EFORMAT (the output is then
                            unspecified)                                         */
  int rc;                /* out                                                    */
  sdcsz_report rep;      /* out                                                    */
} sdcsz_dec_item;

/* Device workspace for sdcsz_decompress_batch: the parameters of each stream
 * (from sdcsz_stream_info or the compression call; n_faults = the item's
 * plan length), in item order. */
uint64_t sdcsz_decompress_batch_workspace_size(const sdcsz_params *h_params, uint32_t n);

/*
 * Decompress n streams (Algorithm 2 for each, with each item's RECON fault
 * plan applied as in sdcsz_decompress).  Returns
 * SDCSZ_OK when every stream decoded, else the first failing item's code.
 * Synchronises `stream` once, or twice when an item gives no header.
 */
int sdcsz_decompress_batch(sdcsz_dec_item *h_items, uint32_t n, void *d_ws, uint64_t ws_size,
                           void *stream);

/*
 * Launch shapes of the block-shape-specialised kernels (set by an
 * autotuner; they never change a result).  stage: 0 prediction and
 * quantization, 1 code check, 2 encoding, 3 decoding.  shape_class: 0 the
 * 6x6x6 3D kernels, 1 the 16x16 2D kernels.  dtype: SDCSZ_F32 or SDCSZ_F64.
 * A launch over `blocks` blocks (summed over the fields of a batch that share
 * the kernel) runs lanes[i] lanes per work-group, one block per lane, for the
 * first i with blocks <= max_blocks[i], and 256 lanes beyond the last entry.
 * n <= SDCSZ_TUNE_MAX entries with strictly ascending max_blocks and lanes
 * 64, 128 or 256 (host arrays, copied); n = 0 restores the default.
 * Process-wide state: set it while no call is running.  Returns SDCSZ_OK or
 * SDCSZ_EINVAL.
 */
#define SDCSZ_TUNE_MAX 8
int sdcsz_tune_set(int stage, int shape_class, int dtype, uint32_t n, const uint64_t *max_blocks,
                   const uint32_t *lanes);
/* The current entries (max_blocks and lanes hold SDCSZ_TUNE_MAX entries). */
int sdcsz_tune_get(int stage, int shape_class, int dtype, uint32_t *n, uint64_t *max_blocks, uint32_t *lanes);

/* Human-readable name of a return code. */
const char *sdcsz_strerror(int code);

/*
 * Phase timing (instrumentation).  When enabled, every call records HIP
 * events on its stream around each kernel phase and accumulates the elapsed
 * device time per phase, and accumulates host wall time in the host phases.
 * Process-wide state; not thread safe.
 * Device phases: 0 range, 1 predict+quantize (per block), 2 code faults,
 * 3 code check+size, 4 compression scan, 5 encode+assemble,
 * 6 decompression scan, 7 decode+check (per block).
 * Host phases: 8 codebook construction, 9 waiting in stream
 * synchronisations, 10 whole compression/decompression calls.
 */
#define SDCSZ_N_PHASES 11
typedef struct {
  double ms[SDCSZ_N_PHASES];       /* accumulated milliseconds */
  uint64_t launches[SDCSZ_N_PHASES];  /* kernel phases timed / host spans */
} sdcsz_timing;
/* on != 0 enables and clears the accumulators; 0 disables. */
void sdcsz_timing_enable(int on);
void sdcsz_timing_read(sdcsz_timing *h_out);
const char *sdcsz_phase_name(int phase);

#ifdef __cplusplus
}
#endif
#endif
