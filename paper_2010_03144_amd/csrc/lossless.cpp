// lossless.cpp -- host side of the lossless stage: sdcsz_pack and
// sdcsz_unpack (layout of a packed stream and the kernels: kern_pack.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "common.h"
#include "kern.h"

using namespace sdcsz;

namespace {

#define HIPCHK(x)                             \
  do {                                        \
    if ((x) != hipSuccess) return SDCSZ_EHIP; \
  } while (0)

const uint8_t kMagicPlain[8] = {'S', 'D', 'C', 'S', 'Z', 0, 'v', '1'};
const uint8_t kMagicPacked[8] = {'S', 'D', 'C', 'S', 'Z', 0, 'v', '2'};
constexpr uint64_t kUnpackWs = 256;
// blocks of a stream the stage takes at most (its section offsets are 32-bit)
constexpr uint64_t kMaxPackBlocks = 1ull << 30;

template <typename V> V rd(const uint8_t *b, uint64_t off) {
  V v;
  std::memcpy(&v, b + off, sizeof(V));
  return v;
}
template <typename V> void wr(uint8_t *b, uint64_t off, V v) { std::memcpy(b + off, &v, sizeof(V)); }

// every header field, whatever the layout version
void read_fields(const uint8_t *o, Header &h) {
  h.dtype = rd<uint32_t>(o, 8);
  h.ndim = rd<uint32_t>(o, 12);
  for (int a = 0; a < 3; a++) h.d[a] = rd<uint64_t>(o, 16 + 8 * a);
  for (int a = 0; a < 3; a++) h.b[a] = rd<uint32_t>(o, 40 + 4 * a);
  h.eb_mode = rd<uint32_t>(o, 52);
  h.eb = rd<double>(o, 56);
  h.eb_abs = rd<double>(o, 64);
  h.abft = rd<uint32_t>(o, 72);
  h.n_sym = rd<uint32_t>(o, 76);
  h.n_blocks = rd<uint64_t>(o, 80);
  h.n_outliers = rd<uint64_t>(o, 88);
  h.n_regression = rd<uint64_t>(o, 96);
  h.payload_words = rd<uint64_t>(o, 104);
  h.off_codebook = rd<uint64_t>(o, 112);
  h.off_table = rd<uint64_t>(o, 120);
  h.off_coef = rd<uint64_t>(o, 128);
  h.off_sumdc = rd<uint64_t>(o, 136);
  h.off_outliers = rd<uint64_t>(o, 144);
  h.off_payload = rd<uint64_t>(o, 152);
  h.total = rd<uint64_t>(o, 160);
  h.predictor = rd<uint32_t>(o, 168);
}

void write_fields(uint32_t *words, const Header &h, const uint8_t *magic) {
  uint8_t o[kHeader];
  std::memset(o, 0, kHeader);
  std::memcpy(o, magic, 8);
  wr<uint32_t>(o, 8, h.dtype);
  wr<uint32_t>(o, 12, h.ndim);
  for (int a = 0; a < 3; a++) wr<uint64_t>(o, 16 + 8 * a, h.d[a]);
  for (int a = 0; a < 3; a++) wr<uint32_t>(o, 40 + 4 * a, h.b[a]);
  wr<uint32_t>(o, 52, h.eb_mode);
  wr<double>(o, 56, h.eb);
  wr<double>(o, 64, h.eb_abs);
  wr<uint32_t>(o, 72, h.abft);
  wr<uint32_t>(o, 76, h.n_sym);
  wr<uint64_t>(o, 80, h.n_blocks);
  wr<uint64_t>(o, 88, h.n_outliers);
  wr<uint64_t>(o, 96, h.n_regression);
  wr<uint64_t>(o, 104, h.payload_words);
  wr<uint64_t>(o, 112, h.off_codebook);
  wr<uint64_t>(o, 120, h.off_table);
  wr<uint64_t>(o, 128, h.off_coef);
  wr<uint64_t>(o, 136, h.off_sumdc);
  wr<uint64_t>(o, 144, h.off_outliers);
  wr<uint64_t>(o, 152, h.off_payload);
  wr<uint64_t>(o, 160, h.total);
  wr<uint32_t>(o, 168, h.predictor);
  std::memcpy(words, o, kHeader);
}

uint64_t value_bytes(const Header &h) { return h.dtype == SDCSZ_F32 ? 4 : 8; }

// Section counts small enough that no offset computed from them wraps: each
// section of a well-formed stream lies inside the stream.
bool counts_fit(const Header &h, uint64_t size) {
  const uint64_t vb = value_bytes(h);
  return h.n_regression <= size / (4 * vb) && h.n_outliers <= size / vb && h.payload_words <= size / 4 &&
         h.n_blocks <= kMaxPackBlocks;
}

// Offsets of a packed stream's verbatim sections and of its table section.
void packed_front(Header &h) {
  const uint64_t vb = value_bytes(h);
  h.off_codebook = kHeader;
  h.off_coef = align8(h.off_codebook + 4ull * h.n_sym);
  h.off_outliers = align8(h.off_coef + 4ull * vb * h.n_regression);
  h.off_payload = align8(h.off_outliers + vb * h.n_outliers);
  h.off_table = align8(h.off_payload + 4ull * h.payload_words);
}

// the 4-byte pad behind a section ending at `end` (4-byte aligned), if any
void add_pad(uint64_t *pads, uint32_t &n, uint64_t end) {
  if (end % 8) pads[n++] = end;
}

hipError_t read_back(const void *d, void *h, uint64_t n, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(h, d, n, hipMemcpyDeviceToHost, st);
  return e != hipSuccess ? e : hipStreamSynchronize(st);
}

hipError_t copy_d2d(uint8_t *dst, const uint8_t *src, uint64_t n, hipStream_t st) {
  return n ? hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, st) : hipSuccess;
}

// codebook, coefficients, outliers and payload from layout `from` to layout `to`
hipError_t copy_verbatim(uint8_t *dst, const Header &to, const uint8_t *src, const Header &from, hipStream_t st) {
  const uint64_t vb = value_bytes(from);
  hipError_t e = copy_d2d(dst + to.off_codebook, src + from.off_codebook, 4ull * from.n_sym, st);
  if (e == hipSuccess) e = copy_d2d(dst + to.off_coef, src + from.off_coef, 4 * vb * from.n_regression, st);
  if (e == hipSuccess) e = copy_d2d(dst + to.off_outliers, src + from.off_outliers, vb * from.n_outliers, st);
  if (e == hipSuccess) e = copy_d2d(dst + to.off_payload, src + from.off_payload, 4ull * from.payload_words, st);
  return e;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

extern "C" {

uint64_t sdcsz_pack_workspace_size(uint64_t n_blocks) {
  const uint64_t nch = std::max<uint64_t>((n_blocks + kPackChunk - 1) / kPackChunk, 1);
  return ((sizeof(PackChunk) * nch + 255) & ~255ull) + 256;
}

int sdcsz_pack(const void *d_stream, uint64_t stream_size, void *d_out, uint64_t out_cap, uint64_t *h_out_size,
               void *d_ws, uint64_t ws_size, void *stream) {
  if (!d_stream || (!d_out && out_cap) || !h_out_size || !d_ws || !aligned8(d_stream) || !aligned8(d_out) ||
      !aligned8(d_ws))
    return SDCSZ_EINVAL;
  if (stream_size < kHeader) return SDCSZ_EFORMAT;
  hipStream_t st = (hipStream_t)stream;
  const uint8_t *src = (const uint8_t *)d_stream;
  uint8_t *dst = (uint8_t *)d_out;
  uint8_t hb[kHeader];
  HIPCHK(read_back(src, hb, kHeader, st));
  if (std::memcmp(hb, kMagicPlain, 8) != 0) return SDCSZ_EFORMAT;
  Header h;
  read_fields(hb, h);
  if (h.dtype > 1 || h.abft > 1 || h.n_sym > 65536 || !counts_fit(h, stream_size)) return SDCSZ_EFORMAT;
  Header chk = h;
  section_offsets(chk);
  if (chk.off_table != h.off_table || chk.off_coef != h.off_coef || chk.off_sumdc != h.off_sumdc ||
      chk.off_outliers != h.off_outliers || chk.off_payload != h.off_payload || chk.total != h.total ||
      h.total > stream_size)
    return SDCSZ_EFORMAT;
  h.off_codebook = kHeader;
  const uint64_t nb = h.n_blocks, nch = (nb + kPackChunk - 1) / kPackChunk;
  if (ws_size < sdcsz_pack_workspace_size(nb)) return SDCSZ_ENOSPC;

  PackArgs a;
  std::memset(&a, 0, sizeof(a));
  a.src = src;
  a.dst = dst;
  a.info = (PackChunk *)d_ws;
  a.res = (uint64_t *)((uint8_t *)d_ws + sdcsz_pack_workspace_size(nb) - 256);
  a.nb = nb;
  a.nch = nch;
  a.src_table = h.off_table;
  a.src_sumdc = h.off_sumdc;
  a.abft = h.abft;
  if (nch) hipLaunchKernelGGL(k_pack_sizes, dim3((uint32_t)nch), dim3(kPackChunk), 0, st, a);
  hipLaunchKernelGGL(k_pack_scan, dim3(1), dim3(1024), 0, st, a);
  HIPCHK(hipGetLastError());
  uint64_t words[2];
  HIPCHK(read_back(a.res, words, sizeof(words), st));

  Header p = h;
  packed_front(p);
  const uint64_t vb = value_bytes(h);
  const uint64_t tend = p.off_table + 4 * (nch + 1 + words[0]);
  p.off_sumdc = align8(tend);
  const uint64_t send = p.off_sumdc + 4 * (nch + 1 + words[1]);
  p.total = h.abft ? align8(send) : p.off_sumdc;
  *h_out_size = p.total;
  if (p.total > out_cap) return SDCSZ_ENOSPC;
  a.dst_table = p.off_table;
  a.dst_sumdc = p.off_sumdc;
  add_pad(a.pads, a.n_pads, p.off_codebook + 4ull * h.n_sym);
  add_pad(a.pads, a.n_pads, p.off_coef + 4 * vb * h.n_regression);
  add_pad(a.pads, a.n_pads, p.off_outliers + vb * h.n_outliers);
  add_pad(a.pads, a.n_pads, p.off_payload + 4ull * h.payload_words);
  add_pad(a.pads, a.n_pads, tend);
  if (h.abft) add_pad(a.pads, a.n_pads, send);
  write_fields(a.hdr, p, kMagicPacked);
  HIPCHK(copy_verbatim(dst, p, src, h, st));
  hipLaunchKernelGGL(k_pack_write, dim3((uint32_t)std::max<uint64_t>(nch, 1)), dim3(kPackChunk), 0, st, a);
  HIPCHK(hipGetLastError());
  return SDCSZ_OK;
}

int sdcsz_unpack(const void *d_packed, uint64_t packed_size, void *d_out, uint64_t out_cap, uint64_t *h_out_size,
                 void *d_ws, uint64_t ws_size, void *stream) {
  if (!d_packed || (!d_out && out_cap) || !h_out_size || !d_ws || !aligned8(d_packed) || !aligned8(d_out) ||
      !aligned8(d_ws))
    return SDCSZ_EINVAL;
  if (ws_size < kUnpackWs) return SDCSZ_ENOSPC;
  if (packed_size < kHeader) return SDCSZ_EFORMAT;
  hipStream_t st = (hipStream_t)stream;
  const uint8_t *src = (const uint8_t *)d_packed;
  uint8_t hb[kHeader];
  HIPCHK(read_back(src, hb, kHeader, st));
  if (std::memcmp(hb, kMagicPacked, 8) != 0) return SDCSZ_EFORMAT;
  Header q;
  read_fields(hb, q);
  if (q.dtype > 1 || q.abft > 1 || q.n_sym > 65536 || q.total > packed_size || !counts_fit(q, packed_size))
    return SDCSZ_EFORMAT;
  Header chk = q;
  packed_front(chk);
  if (chk.off_codebook != q.off_codebook || chk.off_coef != q.off_coef || chk.off_outliers != q.off_outliers ||
      chk.off_payload != q.off_payload || chk.off_table != q.off_table || q.off_sumdc < q.off_table ||
      q.total < q.off_sumdc || q.off_sumdc % 8 != 0 || (!q.abft && q.total != q.off_sumdc))
    return SDCSZ_EFORMAT;
  const uint64_t nb = q.n_blocks, nch = (nb + kPackChunk - 1) / kPackChunk;
  if (4 * (nch + 1) > q.off_sumdc - q.off_table) return SDCSZ_EFORMAT;

  Header h = q;
  section_offsets(h);
  *h_out_size = h.total;
  const bool fits = h.total <= out_cap;
  UnpackArgs a;
  std::memset(&a, 0, sizeof(a));
  a.src = src;
  a.dst = (uint8_t *)d_out;
  a.err = (uint32_t *)d_ws;
  a.nb = nb;
  a.nch = nch;
  a.src_table = q.off_table;
  a.src_sumdc = q.off_sumdc;
  a.src_total = q.total;
  a.dst_table = h.off_table;
  a.dst_sumdc = h.off_sumdc;
  a.abft = q.abft;
  a.write = fits ? 1 : 0;
  const uint64_t vb = value_bytes(h);
  add_pad(a.pads, a.n_pads, h.off_codebook + 4ull * h.n_sym);
  add_pad(a.pads, a.n_pads, h.off_coef + 4 * vb * h.n_regression);
  add_pad(a.pads, a.n_pads, h.off_outliers + vb * h.n_outliers);
  add_pad(a.pads, a.n_pads, h.off_payload + 4ull * h.payload_words);
  write_fields(a.hdr, h, kMagicPlain);
  hipLaunchKernelGGL(k_unpack_check, dim3(1), dim3(64), 0, st, a);
  if (nch) hipLaunchKernelGGL(k_unpack_chunks, dim3((uint32_t)nch), dim3(kPackChunk), 0, st, a);
  HIPCHK(hipGetLastError());
  if (fits) HIPCHK(copy_verbatim((uint8_t *)d_out, h, src, q, st));
  uint32_t err = 0;
  HIPCHK(read_back(a.err, &err, sizeof(err), st));
  if (err) return SDCSZ_EFORMAT;
  return fits ? SDCSZ_OK : SDCSZ_ENOSPC;
}

}  // extern "C"
