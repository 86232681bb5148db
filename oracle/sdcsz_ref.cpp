/*
 * sdcsz_ref.cpp -- CPU oracle (test infrastructure only; see sdcsz_ref.h).
 *
 * Plain, slow, single-threaded.  Built by build_oracle.py with -O2
 * -ffp-contract=off and no fast math, so every floating-point operation below
 * is one IEEE operation in the field's own type T, rounded to nearest, in the
 * order written.
 *
 * Parity is against this file.  Where the paper leaves a detail open the
 * reading taken is stated next to the code and listed in the design notes.
 *
 * Parity unpinned: the predictor selection (Algorithm 1, second loop).  The
 * paper fixes neither the sample set, nor the error measure, nor the rule on
 * equal estimates, so three parts of it are readings that no closed form or
 * paper value can check: the sample set of a partial block (the configured
 * block's diagonals clipped to the partial extents), the tie rule (regression
 * when E_reg <= E_lor) and the allowance of one bound per sample added to
 * E_lor.  The selection only moves the compression ratio; the error bound
 * holds under either predictor.
 */
#include "sdcsz_ref.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

const uint32_t kRadius = 32768;      /* code of a zero residual           */
const uint32_t kMaxCodeLen = 24;     /* Huffman length limit              */
const uint64_t kHeaderBytes = 192;   /* fixed stream header               */
const uint64_t kMaxBlockPoints = 8192;

/* ------------------------------------------------------------------------ */
/* Geometry: blocks in C order, partial blocks at the upper edges.           */
/* (Sec. 5.1: the field is cut into blocks that are compressed independently) */
/* ------------------------------------------------------------------------ */
struct Geometry {
  uint32_t ndim;
  uint64_t d[3];  /* normalised to 3 axes, leading axes of extent 1 */
  uint64_t b[3];
  uint64_t nb[3];
  uint64_t n_blocks;
  uint64_t n_values;
};

bool make_geometry(uint32_t ndim, const uint64_t *dims, const uint32_t *block, Geometry *g) {
  if (ndim < 1 || ndim > 3) return false;
  uint32_t off = 3 - ndim;
  for (int a = 0; a < 3; a++) { g->d[a] = 1; g->b[a] = 1; }
  for (uint32_t a = 0; a < ndim; a++) {
    g->d[off + a] = dims[a];
    g->b[off + a] = block[a];
    if (block[a] < 1 || block[a] > 4096) return false;
  }
  if (g->b[0] * g->b[1] * g->b[2] > kMaxBlockPoints) return false;
  g->ndim = ndim;
  g->n_values = g->d[0] * g->d[1] * g->d[2];
  if (g->n_values >= (1ull << 32)) return false;
  for (int a = 0; a < 3; a++) g->nb[a] = (g->d[a] + g->b[a] - 1) / g->b[a];
  g->n_blocks = g->nb[0] * g->nb[1] * g->nb[2];
  return true;
}

struct BlockBox {
  uint64_t o[3]; /* origin in the field */
  uint64_t n[3]; /* extents (partial at the upper edges) */
  uint64_t pts;
};

BlockBox block_box(const Geometry &g, uint64_t blk) {
  BlockBox bb;
  uint64_t c[3];
  c[2] = blk % g.nb[2];
  c[1] = (blk / g.nb[2]) % g.nb[1];
  c[0] = blk / (g.nb[2] * g.nb[1]);
  for (int a = 0; a < 3; a++) {
    bb.o[a] = c[a] * g.b[a];
    bb.n[a] = std::min(g.b[a], g.d[a] - bb.o[a]);
  }
  bb.pts = bb.n[0] * bb.n[1] * bb.n[2];
  return bb;
}

uint64_t field_index(const Geometry &g, const BlockBox &bb, uint64_t i, uint64_t j, uint64_t k) {
  return ((bb.o[0] + i) * g.d[1] + (bb.o[1] + j)) * g.d[2] + (bb.o[2] + k);
}

/* ------------------------------------------------------------------------ */
/* Words of a value (Sec. 5.4): an FP32 value is one 32-bit word; an FP64     */
/* value is two, low half first.                                              */
/* ------------------------------------------------------------------------ */
template <typename T> struct W;
template <> struct W<float> {
  static const uint32_t per = 1;
  static void put(float v, uint32_t *w) { std::memcpy(w, &v, 4); }
  static float get(const uint32_t *w) { float v; std::memcpy(&v, w, 4); return v; }
};
template <> struct W<double> {
  static const uint32_t per = 2;
  static void put(double v, uint32_t *w) {
    uint64_t u; std::memcpy(&u, &v, 8);
    w[0] = (uint32_t)u; w[1] = (uint32_t)(u >> 32);
  }
  static double get(const uint32_t *w) {
    uint64_t u = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    double v; std::memcpy(&v, &u, 8); return v;
  }
};

template <typename T> T flip_bit(T v, uint32_t bit) {
  uint32_t w[2] = {0, 0};
  W<T>::put(v, w);
  bit %= 32 * W<T>::per;
  w[bit / 32] ^= 1u << (bit % 32);
  return W<T>::get(w);
}

template <typename T> bool same_bits(T a, T b) { return std::memcmp(&a, &b, sizeof(T)) == 0; }

}  // namespace

/* ------------------------------------------------------------------------ */
/* Checksum pair of Sec. 3.2 over integer words (Sec. 5.4):                   */
/*   sum = sum_j w_j,  isum = sum_j j * w_j,  unsigned 64-bit, j from 0.      */
/* ------------------------------------------------------------------------ */
extern "C" void sdcsz_ref_checksums(const uint32_t *w, uint64_t n, uint64_t *sum, uint64_t *isum) {
  uint64_t s = 0, is = 0;
  for (uint64_t j = 0; j < n; j++) {
    s += (uint64_t)w[j];
    is += j * (uint64_t)w[j];
  }
  *sum = s;
  *isum = is;
}

/* Detection, location and repair of one corrupted word (Sec. 3.2): the word
 * index is the ratio of the isum difference to the sum difference. */
extern "C" int sdcsz_ref_correct(uint32_t *w, uint64_t n, uint64_t sum, uint64_t isum,
                                 uint32_t width) {
  uint64_t s2, i2;
  sdcsz_ref_checksums(w, n, &s2, &i2);
  if (s2 == sum && i2 == isum) return 0;
  int64_t ds = (int64_t)(s2 - sum);
  int64_t di = (int64_t)(i2 - isum);
  if (ds == 0) return -1;
  if (di % ds != 0) return -1;
  int64_t j = di / ds;
  if (j < 0 || (uint64_t)j >= n) return -1;
  int64_t repaired = (int64_t)w[j] - ds;
  int64_t top = width == 16 ? 0xFFFF : 0xFFFFFFFFll;
  if (repaired < 0 || repaired > top) return -1;
  uint32_t old = w[j];
  w[j] = (uint32_t)repaired;
  sdcsz_ref_checksums(w, n, &s2, &i2);
  if (s2 == sum && i2 == isum) return 1;
  w[j] = old;
  return -1;
}

namespace {

/* ------------------------------------------------------------------------ */
/* Linear regression of a block (Algorithm 1, first loop; Sec. 3.1 names the  */
/* regression predictor).  Reading: centred least-squares plane over the      */
/* block's own points, beta_a = 12/(n (n_a^2-1)) * sum_p x_p (idx_a - c_a),   */
/* mu = mean, c_a = (n_a-1)/2.  Summation order (part of the definition):     */
/* per plane i: row sums R_ij, column sums D_ik; the plane quantities         */
/* P_i = sum_j R_ij, A_i = sum_j w1(j) R_ij, B_i = sum_k w2(k) D_ik; then the */
/* block sums over i.  Every accumulator starts at +0 and adds left to right. */
/* ------------------------------------------------------------------------ */
template <typename T> void regression(const T *x, const uint64_t n[3], T coef[4]) {
  const uint64_t pts = n[0] * n[1] * n[2];
  T c[3], wt[3][4096];
  for (int a = 0; a < 3; a++) {
    c[a] = (T)(0.5 * (double)(n[a] - 1));
    for (uint64_t t = 0; t < n[a]; t++) wt[a][t] = (T)t - c[a];
  }
  T S0 = 0, Sa0 = 0, Sa1 = 0, Sa2 = 0;
  std::vector<T> D(n[2]);
  for (uint64_t i = 0; i < n[0]; i++) {
    T P = 0, A = 0, B = 0;
    for (uint64_t k = 0; k < n[2]; k++) D[k] = 0;
    for (uint64_t j = 0; j < n[1]; j++) {
      T R = 0;
      for (uint64_t k = 0; k < n[2]; k++) {
        T v = x[(i * n[1] + j) * n[2] + k];
        R = R + v;
        D[k] = D[k] + v;
      }
      P = P + R;
      A = A + wt[1][j] * R;
    }
    for (uint64_t k = 0; k < n[2]; k++) B = B + wt[2][k] * D[k];
    S0 = S0 + P;
    Sa0 = Sa0 + wt[0][i] * P;
    Sa1 = Sa1 + A;
    Sa2 = Sa2 + B;
  }
  T S[3] = {Sa0, Sa1, Sa2};
  for (int a = 0; a < 3; a++) {
    if (n[a] > 1) {
      T K = (T)(12.0 / ((double)pts * ((double)n[a] * (double)n[a] - 1.0)));
      coef[a] = S[a] * K;
    } else {
      coef[a] = 0;
    }
  }
  coef[3] = S0 * (T)(1.0 / (double)pts);
}

template <typename T>
T regression_predict(const T coef[4], const T c[3], uint64_t i, uint64_t j, uint64_t k) {
  T w0 = (T)i - c[0], w1 = (T)j - c[1], w2 = (T)k - c[2];
  return ((coef[0] * w0 + coef[1] * w1) + coef[2] * w2) + coef[3];
}

/* Lorenzo predictor inside the block, neighbours outside the block read as
 * zero (the blocks are independent, Sec. 5.1).  Fixed operation order per
 * block dimensionality. */
template <typename T>
T lorenzo(const T *r, const uint64_t n[3], uint32_t ndim, uint64_t i, uint64_t j, uint64_t k) {
  auto at = [&](int64_t a, int64_t b, int64_t c) -> T {
    if (a < 0 || b < 0 || c < 0) return (T)0;
    return r[((uint64_t)a * n[1] + (uint64_t)b) * n[2] + (uint64_t)c];
  };
  int64_t I = (int64_t)i, J = (int64_t)j, K = (int64_t)k;
  if (ndim == 1) return at(I, J, K - 1);
  if (ndim == 2) return (at(I, J - 1, K) + at(I, J, K - 1)) - at(I, J - 1, K - 1);
  /* inclusion-exclusion over the 7 earlier neighbours, grouped as the
   * current neighbour c plus the difference of the two 2D face stencils
   * u(k) = (a + b) - d and u(k-1) = (e + f) - g */
  T a = at(I - 1, J, K), b = at(I, J - 1, K), c = at(I, J, K - 1);
  T d = at(I - 1, J - 1, K), e = at(I - 1, J, K - 1), f = at(I, J - 1, K - 1);
  T g = at(I - 1, J - 1, K - 1);
  T u = (a + b) - d;
  T u_prev = (e + f) - g;
  return c + (u - u_prev);
}

/* Sampling cost in units of the error bound, saturated (Algorithm 1, second
 * loop).  Integer so that the per-block totals do not depend on order. */
template <typename T> uint32_t sample_cost(T diff, T inv_e) {
  T t = std::fabs(diff) * inv_e;
  if (t < (T)65536) return (uint32_t)t;
  return 65536;
}

/* Sample points: the space diagonals of the block as configured (4 in 3D,
 * 2 in 2D; every point in 1D), keeping the points that fall inside the
 * block's actual extents (partial blocks at the field's upper edges);
 * duplicates removed. */
void sample_points(const uint64_t bs[3], const uint64_t n[3], uint32_t ndim, std::vector<uint64_t> &out) {
  out.clear();
  auto push = [&](uint64_t i, uint64_t j, uint64_t k) {
    if (i >= n[0] || j >= n[1] || k >= n[2]) return;
    uint64_t p = (i * n[1] + j) * n[2] + k;
    for (uint64_t q : out)
      if (q == p) return;
    out.push_back(p);
  };
  if (ndim == 1) {
    for (uint64_t k = 0; k < n[2]; k++) push(0, 0, k);
    return;
  }
  if (ndim == 2) {
    uint64_t m = std::min(bs[1], bs[2]);
    for (uint64_t t = 0; t < m; t++) {
      push(0, t, t);
      push(0, t, bs[2] - 1 - t);
    }
    return;
  }
  uint64_t m = std::min(bs[0], std::min(bs[1], bs[2]));
  for (uint64_t t = 0; t < m; t++) {
    push(t, t, t);
    push(t, t, bs[2] - 1 - t);
    push(t, bs[1] - 1 - t, t);
    push(bs[0] - 1 - t, t, t);
  }
}

/* ------------------------------------------------------------------------ */
/* Huffman code (Algorithm 1, "construct Huffman tree").  Reading: leaves are */
/* the symbols with a non-zero count sorted by (count, symbol); two-queue     */
/* merge, ties to the leaf queue; one symbol gets length 1; when the longest  */
/* code exceeds 24 bits every count is halved (minimum 1) and the tree built  */
/* again.                                                                     */
/* ------------------------------------------------------------------------ */
void huffman_build(const std::vector<uint64_t> &cnt, uint8_t *len) {
  std::memset(len, 0, 65536);
  std::vector<std::pair<uint64_t, uint32_t>> leaves;
  for (uint32_t s = 0; s < 65536; s++)
    if (cnt[s] > 0) leaves.push_back({cnt[s], s});
  size_t S = leaves.size();
  if (S == 0) return;
  if (S == 1) { len[leaves[0].second] = 1; return; }
  std::sort(leaves.begin(), leaves.end());
  std::vector<uint64_t> weight(2 * S - 1);
  std::vector<size_t> parent(2 * S - 1, 0);
  for (size_t t = 0; t < S; t++) weight[t] = leaves[t].first;
  size_t next_leaf = 0, next_inner = S, made = S;
  auto take = [&]() -> size_t {
    if (next_leaf < S && (next_inner == made || weight[next_leaf] <= weight[next_inner]))
      return next_leaf++;
    return next_inner++;
  };
  for (size_t step = 0; step + 1 < S; step++) {
    size_t a = take();
    size_t b = take();
    weight[made] = weight[a] + weight[b];
    parent[a] = made;
    parent[b] = made;
    made++;
  }
  std::vector<uint32_t> depth(2 * S - 1, 0);
  for (size_t v = 2 * S - 2; v-- > 0;) depth[v] = depth[parent[v]] + 1;
  for (size_t t = 0; t < S; t++) len[leaves[t].second] = (uint8_t)std::min<uint32_t>(depth[t], 255);
}

void huffman_lengths(const uint64_t *hist, uint8_t *len) {
  std::vector<uint64_t> cnt(hist, hist + 65536);
  for (;;) {
    huffman_build(cnt, len);
    uint32_t mx = 0;
    for (uint32_t s = 0; s < 65536; s++) mx = std::max<uint32_t>(mx, len[s]);
    if (mx <= kMaxCodeLen) return;
    for (uint32_t s = 0; s < 65536; s++)
      if (cnt[s] > 0) cnt[s] = std::max<uint64_t>(1, cnt[s] >> 1);
  }
}

/* Canonical codes: symbols ordered by (length, symbol); the first gets 0,
 * each next one (previous + 1) shifted left by the length increase. */
void canonical_codes(const uint8_t *len, uint32_t *code) {
  std::vector<std::pair<uint32_t, uint32_t>> order;
  for (uint32_t s = 0; s < 65536; s++) {
    code[s] = 0;
    if (len[s]) order.push_back({len[s], s});
  }
  std::sort(order.begin(), order.end());
  uint32_t c = 0, prev = 0;
  for (size_t t = 0; t < order.size(); t++) {
    uint32_t l = order[t].first;
    if (t > 0) c = (c + 1) << (l - prev);
    code[order[t].second] = c;
    prev = l;
  }
}

/* ------------------------------------------------------------------------ */
/* Stream layout (all little endian, sections 8-byte aligned):                */
/*   header (192 B), codebook (u32 per used symbol: symbol<<8 | length,       */
/*   ascending symbols), block table (u32 payload words, u32 outliers<<1 |    */
/*   regression), coefficients (4 values per regression block), sum_dc (u64   */
/*   per block, ABFT only), outliers (values), payload (u32 words, MSB first).*/
/* ------------------------------------------------------------------------ */
struct Header {
  uint32_t dtype, ndim;
  uint64_t d[3];
  uint32_t b[3];
  uint32_t eb_mode;
  double eb, eb_abs;
  uint32_t abft, n_sym;
  uint64_t n_blocks, n_outliers, n_regression, payload_words;
  uint64_t off_codebook, off_table, off_coef, off_sumdc, off_outliers, off_payload, total;
  uint32_t predictor;
};

uint64_t align8(uint64_t v) { return (v + 7) & ~7ull; }

void put32(uint8_t *p, uint32_t v) { std::memcpy(p, &v, 4); }
void put64(uint8_t *p, uint64_t v) { std::memcpy(p, &v, 8); }
void putd(uint8_t *p, double v) { std::memcpy(p, &v, 8); }
uint32_t get32(const uint8_t *p) { uint32_t v; std::memcpy(&v, p, 4); return v; }
uint64_t get64(const uint8_t *p) { uint64_t v; std::memcpy(&v, p, 8); return v; }
double getd(const uint8_t *p) { double v; std::memcpy(&v, p, 8); return v; }

const uint8_t kMagic[8] = {'S', 'D', 'C', 'S', 'Z', 0, 'v', '1'};

void layout(Header &h, uint64_t value_bytes) {
  h.off_codebook = kHeaderBytes;
  h.off_table = align8(h.off_codebook + 4ull * h.n_sym);
  h.off_coef = h.off_table + 8ull * h.n_blocks;
  h.off_sumdc = align8(h.off_coef + 4ull * value_bytes * h.n_regression);
  h.off_outliers = h.off_sumdc + (h.abft ? 8ull * h.n_blocks : 0);
  h.off_payload = align8(h.off_outliers + value_bytes * h.n_outliers);
  h.total = align8(h.off_payload + 4ull * h.payload_words);
}

void write_header(uint8_t *o, const Header &h) {
  std::memset(o, 0, kHeaderBytes);
  std::memcpy(o, kMagic, 8);
  put32(o + 8, h.dtype);
  put32(o + 12, h.ndim);
  for (int a = 0; a < 3; a++) put64(o + 16 + 8 * a, h.d[a]);
  for (int a = 0; a < 3; a++) put32(o + 40 + 4 * a, h.b[a]);
  put32(o + 52, h.eb_mode);
  putd(o + 56, h.eb);
  putd(o + 64, h.eb_abs);
  put32(o + 72, h.abft);
  put32(o + 76, h.n_sym);
  put64(o + 80, h.n_blocks);
  put64(o + 88, h.n_outliers);
  put64(o + 96, h.n_regression);
  put64(o + 104, h.payload_words);
  put64(o + 112, h.off_codebook);
  put64(o + 120, h.off_table);
  put64(o + 128, h.off_coef);
  put64(o + 136, h.off_sumdc);
  put64(o + 144, h.off_outliers);
  put64(o + 152, h.off_payload);
  put64(o + 160, h.total);
  put32(o + 168, h.predictor);
}

/* The header's fields, whatever the stream version (magic not checked). */
void read_fields(const uint8_t *s, Header &h) {
  h.dtype = get32(s + 8);
  h.ndim = get32(s + 12);
  for (int a = 0; a < 3; a++) h.d[a] = get64(s + 16 + 8 * a);
  for (int a = 0; a < 3; a++) h.b[a] = get32(s + 40 + 4 * a);
  h.eb_mode = get32(s + 52);
  h.eb = getd(s + 56);
  h.eb_abs = getd(s + 64);
  h.abft = get32(s + 72);
  h.n_sym = get32(s + 76);
  h.n_blocks = get64(s + 80);
  h.n_outliers = get64(s + 88);
  h.n_regression = get64(s + 96);
  h.payload_words = get64(s + 104);
  h.off_codebook = get64(s + 112);
  h.off_table = get64(s + 120);
  h.off_coef = get64(s + 128);
  h.off_sumdc = get64(s + 136);
  h.off_outliers = get64(s + 144);
  h.off_payload = get64(s + 152);
  h.total = get64(s + 160);
  h.predictor = get32(s + 168);
}

bool read_header(const uint8_t *s, uint64_t size, Header &h) {
  if (size < kHeaderBytes || std::memcmp(s, kMagic, 8) != 0) return false;
  read_fields(s, h);
  if (h.dtype > 1 || h.abft > 1 || h.n_sym > 65536) return false;
  Header chk = h;
  layout(chk, h.dtype == 0 ? 4 : 8);
  if (chk.off_table != h.off_table || chk.off_coef != h.off_coef || chk.off_sumdc != h.off_sumdc ||
      chk.off_outliers != h.off_outliers || chk.off_payload != h.off_payload || chk.total != h.total)
    return false;
  if (h.total > size) return false;
  return true;
}

/* Bit writer / reader, most significant bit of each 32-bit word first. */
struct BitWriter {
  std::vector<uint32_t> words;
  uint64_t nbits = 0;
  void put(uint32_t code, uint32_t len) {
    for (uint32_t t = len; t-- > 0;) {
      uint32_t bit = (code >> t) & 1u;
      if (nbits % 32 == 0) words.push_back(0);
      if (bit) words.back() |= 1u << (31 - nbits % 32);
      nbits++;
    }
  }
};

struct Decoder {
  /* canonical decoding tables by length */
  uint32_t first[kMaxCodeLen + 2];
  uint32_t count[kMaxCodeLen + 2];
  uint32_t start[kMaxCodeLen + 2];
  std::vector<uint32_t> symbols;  /* ordered by (length, symbol) */
  bool build(const uint8_t *len) {
    std::vector<std::pair<uint32_t, uint32_t>> order;
    for (uint32_t s = 0; s < 65536; s++)
      if (len[s]) {
        if (len[s] > kMaxCodeLen) return false;
        order.push_back({len[s], s});
      }
    std::sort(order.begin(), order.end());
    symbols.clear();
    for (auto &o : order) symbols.push_back(o.second);
    std::vector<uint32_t> code(65536);
    canonical_codes(len, code.data());
    for (uint32_t l = 0; l <= kMaxCodeLen + 1; l++) { first[l] = 0; count[l] = 0; start[l] = 0; }
    for (size_t t = 0; t < order.size(); t++) {
      uint32_t l = order[t].first;
      if (count[l] == 0) { first[l] = code[order[t].second]; start[l] = (uint32_t)t; }
      count[l]++;
    }
    return true;
  }
  /* returns symbol or -1 on an invalid code / overrun */
  int64_t decode(const uint32_t *words, uint64_t nwords, uint64_t &bitpos) const {
    uint32_t c = 0;
    for (uint32_t l = 1; l <= kMaxCodeLen; l++) {
      if (bitpos >= nwords * 32) return -1;
      uint32_t bit = (words[bitpos / 32] >> (31 - bitpos % 32)) & 1u;
      bitpos++;
      c = (c << 1) | bit;
      if (count[l] && c >= first[l] && c - first[l] < count[l]) return symbols[start[l] + c - first[l]];
    }
    return -1;
  }
};

/* ------------------------------------------------------------------------ */
/* Per-block reconstruction shared by compression (Algorithm 1 per-point      */
/* loop) and decompression (Algorithm 2): identical arithmetic on both sides  */
/* is what keeps predictions consistent (Sec. 4.1, "type-3" behaviour).       */
/* ------------------------------------------------------------------------ */
template <typename T> struct Consts {
  double eb_abs;
  T q;      /* 2 * eb_abs in T            */
  T inv;    /* 1 / (2 * eb_abs) in T      */
  T inv_e;  /* 1 / eb_abs in T (sampling) */
};

template <typename T> Consts<T> make_consts(double eb_abs) {
  Consts<T> k;
  k.eb_abs = eb_abs;
  k.q = (T)(2.0 * eb_abs);
  k.inv = (T)(1.0 / (2.0 * eb_abs));
  k.inv_e = (T)(1.0 / eb_abs);
  return k;
}

struct FaultIndex {
  std::vector<ref_fault> list;
  bool any(uint32_t target, uint64_t blk) const {
    for (auto &f : list)
      if (f.target == target && f.block == blk) return true;
    return false;
  }
};

template <typename T> struct BlockOut {
  std::vector<uint16_t> codes;
  std::vector<T> outliers;
  T coef[4];
  bool is_reg;
  uint64_t sum_in, isum_in, sum_c, isum_c;
  uint64_t sum_dc, sum_q, isum_q;
};

/* ------------------------------------------------------------------------ */
/* Compression, Algorithm 1.                                                  */
/* ------------------------------------------------------------------------ */
template <typename T>
int compress_impl(const T *in, const ref_params *p, const Geometry &g, uint8_t *out, uint64_t cap,
                  uint64_t *out_size, ref_report *rep, ref_debug *dbg) {
  const uint32_t nd = p->ndim;
  const bool abft = p->abft != 0;

  /* Error bound: absolute, or relative to the value range of the finite
   * values (the evaluation's "value-range based error bound"). */
  double eb_abs = p->eb;
  if (p->eb_mode == REF_REL) {
    bool seen = false;
    double lo = 0, hi = 0;
    for (uint64_t t = 0; t < g.n_values; t++) {
      double v = (double)in[t];
      if (!std::isfinite(v)) continue;
      if (!seen) { lo = hi = v; seen = true; }
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
    eb_abs = seen ? p->eb * (hi - lo) : 0.0;
  }
  const Consts<T> K = make_consts<T>(eb_abs);
  rep->eb_abs = eb_abs;
  rep->n_blocks = g.n_blocks;

  FaultIndex faults;
  for (uint32_t t = 0; t < p->n_faults; t++) faults.list.push_back(p->faults[t]);

  /* working copy of the input: the memory that mode-A errors strike */
  std::vector<T> X(in, in + g.n_values);
  std::vector<BlockOut<T>> B(g.n_blocks);
  std::vector<T> xb, rb;

  /* Loop 1: input checksums and regression coefficients of every block.
   * Errors in the prediction preparation (Sec. 4.1, 4.2): a PREP_INPUT flip
   * strikes the input memory after its checksums were taken, so the
   * regression and the sampling read the corrupted word (and the third loop
   * finds it); a PREP_COEF flip is a computation error in the coefficients,
   * made before their checksums are taken. */
  for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
    BlockBox bb = block_box(g, blk);
    xb.resize(bb.pts);
    for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
      for (uint64_t j = 0; j < bb.n[1]; j++)
        for (uint64_t k = 0; k < bb.n[2]; k++) xb[q++] = X[field_index(g, bb, i, j, k)];
    if (abft) {
      std::vector<uint32_t> w(bb.pts * W<T>::per);
      for (uint64_t q = 0; q < bb.pts; q++) W<T>::put(xb[q], &w[q * W<T>::per]);
      sdcsz_ref_checksums(w.data(), w.size(), &B[blk].sum_in, &B[blk].isum_in);
    }
    for (auto &f : faults.list) {
      if (f.block != blk || f.target != REF_T_PREP_INPUT) continue;
      uint64_t q = f.word / W<T>::per;
      uint64_t k = q % bb.n[2], j = (q / bb.n[2]) % bb.n[1], i = q / (bb.n[2] * bb.n[1]);
      uint64_t at = field_index(g, bb, i, j, k);
      uint32_t w[2] = {0, 0};
      W<T>::put(X[at], w);
      w[f.word % W<T>::per] ^= 1u << (f.bit % 32);
      X[at] = W<T>::get(w);
      xb[q] = X[at];
      rep->injected[REF_T_PREP_INPUT]++;
    }
    regression<T>(xb.data(), bb.n, B[blk].coef);
    for (auto &f : faults.list) {
      if (f.block != blk || f.target != REF_T_PREP_COEF) continue;
      uint32_t cw[8];
      for (int a = 0; a < 4; a++) W<T>::put(B[blk].coef[a], &cw[a * W<T>::per]);
      cw[f.word] ^= 1u << (f.bit % 32);
      for (int a = 0; a < 4; a++) B[blk].coef[a] = W<T>::get(&cw[a * W<T>::per]);
      rep->injected[REF_T_PREP_COEF]++;
    }
    if (abft) {
      uint32_t cw[8];
      for (int a = 0; a < 4; a++) W<T>::put(B[blk].coef[a], &cw[a * W<T>::per]);
      sdcsz_ref_checksums(cw, 4 * W<T>::per, &B[blk].sum_c, &B[blk].isum_c);
    }
  }

  /* Loop 2: sample and estimate E_reg and E_lor, keep the smaller.
   * Selection: parity unpinned (sample set of partial blocks, the tie rule
   * and the per-sample allowance are readings; see the file header). */
  std::vector<uint64_t> samples;
  for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
    BlockBox bb = block_box(g, blk);
    if (p->predictor == REF_PRED_LORENZO) { B[blk].is_reg = false; continue; }
    if (p->predictor == REF_PRED_REGRESSION) { B[blk].is_reg = true; continue; }
    xb.resize(bb.pts);
    for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
      for (uint64_t j = 0; j < bb.n[1]; j++)
        for (uint64_t k = 0; k < bb.n[2]; k++) xb[q++] = X[field_index(g, bb, i, j, k)];
    T c[3];
    for (int a = 0; a < 3; a++) c[a] = (T)(0.5 * (double)(bb.n[a] - 1));
    sample_points(g.b, bb.n, nd, samples);
    uint64_t e_lor = samples.size(), e_reg = 0;  /* one bound of slack per
        sample for the reconstructed (not original) neighbours Lorenzo uses */
    for (uint64_t sp : samples) {
      uint64_t k = sp % bb.n[2], j = (sp / bb.n[2]) % bb.n[1], i = sp / (bb.n[2] * bb.n[1]);
      T x = xb[sp];
      T pl = lorenzo<T>(xb.data(), bb.n, nd, i, j, k);
      T pr = regression_predict<T>(B[blk].coef, c, i, j, k);
      e_lor += sample_cost<T>(x - pl, K.inv_e);
      e_reg += sample_cost<T>(x - pr, K.inv_e);
    }
    for (auto &f : faults.list) {  /* computation errors in the estimates */
      if (f.block != blk || f.target != REF_T_PREP_SAMPLE) continue;
      (f.word == 0 ? e_lor : e_reg) ^= 1ull << (f.bit % 64);
      rep->injected[REF_T_PREP_SAMPLE]++;
    }
    B[blk].is_reg = e_reg <= e_lor;
  }

  /* Mode-A memory errors: strike the input words and the coefficient words
   * after their checksums were taken. */
  for (auto &f : faults.list) {
    if (f.target == REF_T_INPUT) {
      BlockBox bb = block_box(g, f.block);
      uint64_t q = f.word / W<T>::per;
      uint64_t k = q % bb.n[2], j = (q / bb.n[2]) % bb.n[1], i = q / (bb.n[2] * bb.n[1]);
      uint64_t at = field_index(g, bb, i, j, k);
      uint32_t w[2] = {0, 0};
      W<T>::put(X[at], w);
      w[f.word % W<T>::per] ^= 1u << (f.bit % 32);
      X[at] = W<T>::get(w);
      rep->injected[REF_T_INPUT]++;
    } else if (f.target == REF_T_COEF) {
      uint32_t cw[8];
      for (int a = 0; a < 4; a++) W<T>::put(B[f.block].coef[a], &cw[a * W<T>::per]);
      cw[f.word] ^= 1u << (f.bit % 32);
      for (int a = 0; a < 4; a++) B[f.block].coef[a] = W<T>::get(&cw[a * W<T>::per]);
      rep->injected[REF_T_COEF]++;
    }
  }

  /* Loop 3: detect/correct the input, then predict, quantize, reconstruct. */
  uint64_t n_unc = 0;
  for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
    BlockBox bb = block_box(g, blk);
    BlockOut<T> &o = B[blk];
    xb.resize(bb.pts);
    for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
      for (uint64_t j = 0; j < bb.n[1]; j++)
        for (uint64_t k = 0; k < bb.n[2]; k++) xb[q++] = X[field_index(g, bb, i, j, k)];
    if (abft) {
      std::vector<uint32_t> w(bb.pts * W<T>::per);
      for (uint64_t q = 0; q < bb.pts; q++) W<T>::put(xb[q], &w[q * W<T>::per]);
      int st = sdcsz_ref_correct(w.data(), w.size(), o.sum_in, o.isum_in, 32);
      /* a detection in a block struck before its preparation counts there */
      const int ti = faults.any(REF_T_PREP_INPUT, blk) ? REF_T_PREP_INPUT : REF_T_INPUT;
      if (st != 0) rep->detected[ti]++;
      if (st == 1) rep->corrected[ti]++;
      if (st < 0) { rep->uncorrectable[ti]++; n_unc++; }
      for (uint64_t q = 0; q < bb.pts; q++) xb[q] = W<T>::get(&w[q * W<T>::per]);
      uint32_t cw[8];
      for (int a = 0; a < 4; a++) W<T>::put(o.coef[a], &cw[a * W<T>::per]);
      st = sdcsz_ref_correct(cw, 4 * W<T>::per, o.sum_c, o.isum_c, 32);
      if (st != 0) rep->detected[REF_T_COEF]++;
      if (st == 1) rep->corrected[REF_T_COEF]++;
      if (st < 0) { rep->uncorrectable[REF_T_COEF]++; n_unc++; }
      for (int a = 0; a < 4; a++) o.coef[a] = W<T>::get(&cw[a * W<T>::per]);
    }
    T c[3];
    for (int a = 0; a < 3; a++) c[a] = (T)(0.5 * (double)(bb.n[a] - 1));
    o.codes.assign(bb.pts, 0);
    o.outliers.clear();
    rb.assign(bb.pts, (T)0);
    const bool dp = faults.any(REF_T_DUP_PRED, blk), dr = faults.any(REF_T_DUP_RECON, blk);
    auto predict = [&](uint64_t i, uint64_t j, uint64_t k) -> T {
      return o.is_reg ? regression_predict<T>(o.coef, c, i, j, k)
                      : lorenzo<T>(rb.data(), bb.n, nd, i, j, k);
    };
    for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
      for (uint64_t j = 0; j < bb.n[1]; j++)
        for (uint64_t k = 0; k < bb.n[2]; k++, q++) {
          const T x = xb[q];
          /* pred' <- f_dup(): computed twice and compared bit for bit; a
           * mismatch is settled by a third evaluation (majority). */
          T pred = predict(i, j, k);
          if (dp)
            for (auto &f : faults.list)
              if (f.target == REF_T_DUP_PRED && f.block == blk && f.word == q) {
                pred = flip_bit<T>(pred, f.bit);
                rep->injected[REF_T_DUP_PRED]++;
              }
          if (abft) {
            T pred2 = predict(i, j, k);
            if (!same_bits(pred, pred2)) {
              rep->detected[REF_T_DUP_PRED]++;
              T pred3 = predict(i, j, k);
              if (same_bits(pred3, pred2)) rep->corrected[REF_T_DUP_PRED]++;
              else rep->uncorrectable[REF_T_DUP_PRED]++;
              pred = same_bits(pred3, pred) ? pred : pred2;
            }
          }
          /* diff and linear-scaling quantization (radius 32768, code 0 means
           * "unpredictable"); half-up rounding of |diff| / (2 eb). */
          const T diff = x - pred;
          const T t = std::fabs(diff) * K.inv + (T)0.5;
          uint16_t code = 0;
          T recon = x;
          if (t < (T)32768) {
            int m = (int)t;
            int sm = diff < 0 ? -m : m;
            /* dcmp <- dec_dup(q_bin, pred') */
            T r = pred + (T)sm * K.q;
            if (dr)
              for (auto &f : faults.list)
                if (f.target == REF_T_DUP_RECON && f.block == blk && f.word == q) {
                  r = flip_bit<T>(r, f.bit);
                  rep->injected[REF_T_DUP_RECON]++;
                }
            if (abft) {
              T r2 = pred + (T)sm * K.q;
              if (!same_bits(r, r2)) {
                rep->detected[REF_T_DUP_RECON]++;
                T r3 = pred + (T)sm * K.q;
                if (same_bits(r3, r2)) rep->corrected[REF_T_DUP_RECON]++;
                else rep->uncorrectable[REF_T_DUP_RECON]++;
                r = same_bits(r3, r) ? r : r2;
              }
            }
            /* double check of the bound, in double precision */
            if (std::fabs((double)x - (double)r) <= K.eb_abs) {
              code = (uint16_t)(sm + (int)kRadius);
              recon = r;
            }
          }
          o.codes[q] = code;
          rb[q] = recon;
          if (code == 0) o.outliers.push_back(x);
        }
    /* checksums of the finished block: decompressed words (sum_dc) and the
     * final codes (sum_q, isum_q), taken after the double check */
    {
      std::vector<uint32_t> w(bb.pts * W<T>::per);
      for (uint64_t q = 0; q < bb.pts; q++) W<T>::put(rb[q], &w[q * W<T>::per]);
      uint64_t dummy;
      sdcsz_ref_checksums(w.data(), w.size(), &o.sum_dc, &dummy);
      std::vector<uint32_t> cw(o.codes.begin(), o.codes.end());
      sdcsz_ref_checksums(cw.data(), cw.size(), &o.sum_q, &o.isum_q);
    }
  }

  /* histogram of every code, taken before any code fault */
  std::vector<uint64_t> hist(65536, 0);
  for (uint64_t blk = 0; blk < g.n_blocks; blk++)
    for (uint16_t cd : B[blk].codes) hist[cd]++;

  if (dbg) {
    uint64_t at = 0;
    for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
      if (dbg->codes) std::memcpy(dbg->codes + at, B[blk].codes.data(), 2 * B[blk].codes.size());
      at += B[blk].codes.size();
      if (dbg->is_regression) dbg->is_regression[blk] = B[blk].is_reg ? 1 : 0;
      if (dbg->coef) std::memcpy((T *)dbg->coef + 4 * blk, B[blk].coef, 4 * sizeof(T));
    }
    if (dbg->hist) std::memcpy(dbg->hist, hist.data(), 8 * 65536);
  }

  /* code memory errors: codes at rest between prediction and encoding */
  for (auto &f : faults.list)
    if (f.target == REF_T_CODE) {
      B[f.block].codes[f.word] ^= (uint16_t)(1u << (f.bit % 16));
      rep->injected[REF_T_CODE]++;
    }

  std::vector<uint8_t> lens(65536);
  huffman_lengths(hist.data(), lens.data());
  std::vector<uint32_t> codes_tab(65536);
  canonical_codes(lens.data(), codes_tab.data());
  if (dbg && dbg->lengths) std::memcpy(dbg->lengths, lens.data(), 65536);

  /* Loop 4: detect/correct the codes, then encode every block on its own. */
  std::vector<std::vector<uint32_t>> payload(g.n_blocks);
  bool missing_symbol = false;
  for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
    BlockOut<T> &o = B[blk];
    if (abft) {
      std::vector<uint32_t> cw(o.codes.begin(), o.codes.end());
      int st = sdcsz_ref_correct(cw.data(), cw.size(), o.sum_q, o.isum_q, 16);
      if (st != 0) rep->detected[REF_T_CODE]++;
      if (st == 1) rep->corrected[REF_T_CODE]++;
      if (st < 0) { rep->uncorrectable[REF_T_CODE]++; n_unc++; }
      for (size_t q = 0; q < cw.size(); q++) o.codes[q] = (uint16_t)cw[q];
    }
    BitWriter bw;
    for (uint16_t cd : o.codes) {
      if (lens[cd] == 0) { missing_symbol = true; continue; }
      bw.put(codes_tab[cd], lens[cd]);
    }
    payload[blk] = bw.words;
  }
  if (n_unc || missing_symbol) {
    *out_size = 0;
    return REF_ESDC;
  }

  Header h{};
  h.dtype = p->dtype;
  h.ndim = nd;
  for (int a = 0; a < 3; a++) { h.d[a] = g.d[a]; h.b[a] = (uint32_t)g.b[a]; }
  h.eb_mode = p->eb_mode;
  h.eb = p->eb;
  h.eb_abs = eb_abs;
  h.abft = abft ? 1 : 0;
  h.predictor = p->predictor;
  h.n_blocks = g.n_blocks;
  for (uint32_t s = 0; s < 65536; s++) h.n_sym += lens[s] ? 1 : 0;
  for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
    h.n_outliers += B[blk].outliers.size();
    h.n_regression += B[blk].is_reg ? 1 : 0;
    h.payload_words += payload[blk].size();
  }
  layout(h, sizeof(T));
  rep->n_outliers = h.n_outliers;
  rep->n_regression = h.n_regression;
  rep->payload_words = h.payload_words;
  rep->stream_size = h.total;
  *out_size = h.total;
  if (h.total > cap) return REF_ENOSPC;

  std::memset(out, 0, h.total);
  write_header(out, h);
  uint8_t *cb = out + h.off_codebook;
  for (uint32_t s = 0; s < 65536; s++)
    if (lens[s]) { put32(cb, (s << 8) | lens[s]); cb += 4; }
  uint8_t *coef = out + h.off_coef, *outl = out + h.off_outliers;
  uint8_t *pay = out + h.off_payload;
  for (uint64_t blk = 0; blk < g.n_blocks; blk++) {
    const BlockOut<T> &o = B[blk];
    put32(out + h.off_table + 8 * blk, (uint32_t)payload[blk].size());
    put32(out + h.off_table + 8 * blk + 4, (uint32_t)((o.outliers.size() << 1) | (o.is_reg ? 1 : 0)));
    if (o.is_reg) { std::memcpy(coef, o.coef, 4 * sizeof(T)); coef += 4 * sizeof(T); }
    if (abft) put64(out + h.off_sumdc + 8 * blk, o.sum_dc);
    if (!o.outliers.empty()) {
      std::memcpy(outl, o.outliers.data(), sizeof(T) * o.outliers.size());
      outl += sizeof(T) * o.outliers.size();
    }
    if (!payload[blk].empty()) {
      std::memcpy(pay, payload[blk].data(), 4 * payload[blk].size());
      pay += 4 * payload[blk].size();
    }
  }
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Lossless stage after Huffman coding (the place of Algorithm 1's final      */
/* lossless pass and Algorithm 2's first one).  The Huffman payload is close  */
/* to its entropy; the per-block metadata is not: neighbouring blocks have    */
/* similar payload sizes, outlier counts and checksums.  The packed stream    */
/* ("SDCSZ\0v2") keeps the header, codebook, coefficients, outliers and       */
/* payload of the plain one ("v1") verbatim and moves the block table and     */
/* sum_dc to the end, each cut into chunks of 256 blocks, every column of a   */
/* chunk coded by frame of reference: its minimum, then each value minus the  */
/* minimum in as many bits as the largest difference needs, packed LSB first. */
/*   section: u32 off[n_chunks + 1] (word offsets of the chunks after the     */
/*            array, off[0] = 0), then the chunks' words                      */
/*   column:  u32 base low, u32 base high, u32 width (0..64), then            */
/*            ceil(n * width / 32) words: bit t of the column's bit string is */
/*            bit t % 32 of word t / 32; value i holds bits [i*w, (i+1)*w)    */
/*   table chunk: column of payload words, column of outliers<<1|regression; */
/*   sum_dc chunk (ABFT streams only): column of sum_dc                       */
/* Header offsets of a packed stream: codebook, coefficients, outliers,      */
/* payload, table, sum_dc, in that order, each 8-byte aligned.                */
/* ------------------------------------------------------------------------ */
const uint8_t kMagicPacked[8] = {'S', 'D', 'C', 'S', 'Z', 0, 'v', '2'};
const uint64_t kPackChunk = 256;

uint32_t bit_width(uint64_t v) {
  uint32_t w = 0;
  while (v) { w++; v >>= 1; }
  return w;
}

/* Frame-of-reference column: appends its words to out. */
void pack_column(const std::vector<uint64_t> &v, std::vector<uint32_t> &out) {
  uint64_t lo = v.empty() ? 0 : v[0], hi = lo;
  for (uint64_t x : v) { lo = std::min(lo, x); hi = std::max(hi, x); }
  const uint32_t w = bit_width(hi - lo);
  out.push_back((uint32_t)lo);
  out.push_back((uint32_t)(lo >> 32));
  out.push_back(w);
  const uint64_t nbits = (uint64_t)v.size() * w, first = out.size();
  out.resize(first + (nbits + 31) / 32, 0u);
  for (uint64_t i = 0; i < v.size(); i++) {
    const uint64_t d = v[i] - lo;
    for (uint32_t t = 0; t < w; t++)
      if ((d >> t) & 1) {
        const uint64_t bit = i * w + t;
        out[first + bit / 32] |= 1u << (bit % 32);
      }
  }
}

/* Reads n values of a column at words[at..end); false when it does not fit
 * or its width exceeds maxw.  at advances past the column. */
bool unpack_column(const uint32_t *words, uint64_t &at, uint64_t end, uint64_t n, uint32_t maxw,
                   std::vector<uint64_t> &v) {
  if (at + 3 > end) return false;
  const uint64_t lo = (uint64_t)words[at] | ((uint64_t)words[at + 1] << 32);
  const uint32_t w = words[at + 2];
  if (w > maxw) return false;
  at += 3;
  const uint64_t nwords = (n * w + 31) / 32;
  if (at + nwords > end) return false;
  v.assign(n, 0);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t d = 0;
    for (uint32_t t = 0; t < w; t++) {
      const uint64_t bit = i * w + t;
      d |= (uint64_t)((words[at + bit / 32] >> (bit % 32)) & 1u) << t;
    }
    v[i] = lo + d;
  }
  at += nwords;
  return true;
}

/* One packed section: chunk word offsets then the chunks' columns. */
std::vector<uint32_t> pack_section(const std::vector<std::vector<uint64_t>> &cols, uint64_t nb) {
  const uint64_t nch = (nb + kPackChunk - 1) / kPackChunk;
  std::vector<uint32_t> data, off(nch + 1, 0);
  for (uint64_t c = 0; c < nch; c++) {
    const uint64_t b0 = c * kPackChunk, b1 = std::min(nb, b0 + kPackChunk);
    for (const auto &col : cols) {
      std::vector<uint64_t> v(col.begin() + b0, col.begin() + b1);
      pack_column(v, data);
    }
    off[c + 1] = (uint32_t)data.size();
  }
  off.insert(off.end(), data.begin(), data.end());
  return off;
}

bool unpack_section(const uint8_t *s, uint64_t off, uint64_t bytes, uint64_t nb, const uint32_t *maxw, int ncols,
                    std::vector<std::vector<uint64_t>> &cols) {
  const uint64_t nch = (nb + kPackChunk - 1) / kPackChunk;
  if (bytes % 4 != 0 || bytes / 4 < nch + 1) return false;
  std::vector<uint32_t> w(bytes / 4);
  std::memcpy(w.data(), s + off, bytes);
  const uint64_t data = nch + 1, nwords = w.size() - data;
  if (w[0] != 0) return false;
  cols.assign(ncols, std::vector<uint64_t>());
  std::vector<uint64_t> v;
  for (uint64_t c = 0; c < nch; c++) {
    if (w[c + 1] < w[c] || w[c + 1] > nwords) return false;
    uint64_t at = data + w[c];
    const uint64_t end = data + w[c + 1];
    const uint64_t n = std::min(nb, (c + 1) * kPackChunk) - c * kPackChunk;
    for (int k = 0; k < ncols; k++) {
      if (!unpack_column(w.data(), at, end, n, maxw[k], v)) return false;
      cols[k].insert(cols[k].end(), v.begin(), v.end());
    }
    if (at != end) return false;
  }
  return true;
}

/* The v2 offsets of the verbatim sections (everything but table and sum_dc). */
void layout_packed_front(Header &h, uint64_t vb) {
  h.off_codebook = kHeaderBytes;
  h.off_coef = align8(h.off_codebook + 4ull * h.n_sym);
  h.off_outliers = align8(h.off_coef + 4ull * vb * h.n_regression);
  h.off_payload = align8(h.off_outliers + vb * h.n_outliers);
  h.off_table = align8(h.off_payload + 4ull * h.payload_words);
}

/* ------------------------------------------------------------------------ */
/* Decompression, Algorithm 2.                                                */
/* ------------------------------------------------------------------------ */
struct Parsed {
  Header h;
  Geometry g;
  std::vector<uint8_t> lens;
  Decoder dec;
  std::vector<uint64_t> pay_off, out_off, coef_off;
};

int parse(const uint8_t *s, uint64_t size, Parsed &P) {
  if (!read_header(s, size, P.h)) return REF_EFORMAT;
  Header &h = P.h;
  if (h.ndim < 1 || h.ndim > 3) return REF_EFORMAT;
  uint64_t dims[3];
  uint32_t blk[3];
  for (uint32_t a = 0; a < h.ndim; a++) { dims[a] = h.d[3 - h.ndim + a]; blk[a] = h.b[3 - h.ndim + a]; }
  for (uint32_t a = 0; a < 3 - h.ndim; a++)
    if (h.d[a] != 1 || h.b[a] != 1) return REF_EFORMAT;
  if (!make_geometry(h.ndim, dims, blk, &P.g)) return REF_EFORMAT;
  if (P.g.n_blocks != h.n_blocks) return REF_EFORMAT;
  P.lens.assign(65536, 0);
  for (uint32_t t = 0; t < h.n_sym; t++) {
    uint32_t e = get32(s + h.off_codebook + 4 * t);
    uint32_t sym = e >> 8, l = e & 0xFF;
    if (sym > 65535 || l == 0 || l > kMaxCodeLen || P.lens[sym]) return REF_EFORMAT;
    P.lens[sym] = (uint8_t)l;
  }
  if (!P.dec.build(P.lens.data())) return REF_EFORMAT;
  P.pay_off.resize(h.n_blocks + 1);
  P.out_off.resize(h.n_blocks + 1);
  P.coef_off.resize(h.n_blocks + 1);
  P.pay_off[0] = P.out_off[0] = P.coef_off[0] = 0;
  for (uint64_t b = 0; b < h.n_blocks; b++) {
    uint32_t words = get32(s + h.off_table + 8 * b);
    uint32_t meta = get32(s + h.off_table + 8 * b + 4);
    P.pay_off[b + 1] = P.pay_off[b] + words;
    P.out_off[b + 1] = P.out_off[b] + (meta >> 1);
    P.coef_off[b + 1] = P.coef_off[b] + (meta & 1);
  }
  if (P.pay_off[h.n_blocks] != h.payload_words || P.out_off[h.n_blocks] != h.n_outliers ||
      P.coef_off[h.n_blocks] != h.n_regression)
    return REF_EFORMAT;
  return REF_OK;
}

/* Decode one block into r (C order over its extents).  false on a corrupt
 * payload (invalid code, overrun, outlier list mismatch). */
template <typename T>
bool decode_block(const uint8_t *s, const Parsed &P, const Consts<T> &K, uint64_t blk, std::vector<T> &r) {
  const Header &h = P.h;
  BlockBox bb = block_box(P.g, blk);
  uint32_t meta = get32(s + h.off_table + 8 * blk + 4);
  const bool is_reg = meta & 1;
  const uint64_t nout = meta >> 1;
  const uint32_t *words = (const uint32_t *)(s + h.off_payload) + P.pay_off[blk];
  const uint64_t nwords = P.pay_off[blk + 1] - P.pay_off[blk];
  const T *outl = (const T *)(s + h.off_outliers) + P.out_off[blk];
  T coef[4] = {0, 0, 0, 0};
  if (is_reg) std::memcpy(coef, s + h.off_coef + 4 * sizeof(T) * P.coef_off[blk], 4 * sizeof(T));
  T c[3];
  for (int a = 0; a < 3; a++) c[a] = (T)(0.5 * (double)(bb.n[a] - 1));
  r.assign(bb.pts, (T)0);
  uint64_t bitpos = 0, used = 0;
  for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
    for (uint64_t j = 0; j < bb.n[1]; j++)
      for (uint64_t k = 0; k < bb.n[2]; k++, q++) {
        int64_t sym = P.dec.decode(words, nwords, bitpos);
        if (sym < 0) return false;
        if (sym == 0) {
          if (used >= nout) return false;
          r[q] = outl[used++];
          continue;
        }
        T pred = is_reg ? regression_predict<T>(coef, c, i, j, k) : lorenzo<T>(r.data(), bb.n, h.ndim, i, j, k);
        int sm = (int)sym - (int)kRadius;
        r[q] = pred + (T)sm * K.q;
      }
  return used == nout;
}

template <typename T>
uint64_t block_sum(const std::vector<T> &r) {
  uint64_t s = 0;
  uint32_t w[2];
  for (const T &v : r) {
    W<T>::put(v, w);
    for (uint32_t t = 0; t < W<T>::per; t++) s += w[t];
  }
  return s;
}

template <typename T>
void store_block(const Geometry &g, uint64_t blk, const std::vector<T> &r, T *out) {
  BlockBox bb = block_box(g, blk);
  for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
    for (uint64_t j = 0; j < bb.n[1]; j++)
      for (uint64_t k = 0; k < bb.n[2]; k++) out[field_index(g, bb, i, j, k)] = r[q++];
}

template <typename T>
void load_block(const Geometry &g, uint64_t blk, const T *in, std::vector<T> &r) {
  BlockBox bb = block_box(g, blk);
  r.resize(bb.pts);
  for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
    for (uint64_t j = 0; j < bb.n[1]; j++)
      for (uint64_t k = 0; k < bb.n[2]; k++) r[q++] = in[field_index(g, bb, i, j, k)];
}

template <typename T>
void apply_recon_faults(const std::vector<ref_fault> &faults, uint64_t blk, std::vector<T> &r, ref_report *rep) {
  for (auto &f : faults)
    if (f.target == REF_T_RECON && f.block == blk) {
      uint64_t q = f.word / W<T>::per;
      uint32_t w[2] = {0, 0};
      W<T>::put(r[q], w);
      w[f.word % W<T>::per] ^= 1u << (f.bit % 32);
      r[q] = W<T>::get(w);
      rep->injected[REF_T_RECON]++;
    }
}

template <typename T>
int decompress_impl(const uint8_t *s, const Parsed &P, T *out, const ref_fault *faults, uint32_t n_faults,
                    ref_report *rep) {
  const Header &h = P.h;
  const Consts<T> K = make_consts<T>(h.eb_abs);
  std::vector<ref_fault> fl(faults, faults + n_faults);
  std::vector<T> r;
  std::vector<uint8_t> failed(h.n_blocks, 0);
  bool bad = false;
  /* lines 1-9: block-wise decoding and reconstruction */
  for (uint64_t blk = 0; blk < h.n_blocks; blk++) {
    if (!decode_block<T>(s, P, K, blk, r)) {
      failed[blk] = 1;
      r.assign(block_box(P.g, blk).pts, (T)0);
    }
    store_block<T>(P.g, blk, r, out);
  }
  /* lines 10-21: checksum of every decompressed block against sum_dc; a
   * mismatch re-executes the block from the compressed bytes (random-access
   * decompression); a second mismatch is an error in the compressed data.
   * RECON faults strike the decompressed words just before the checksum
   * (and strike unprotected streams all the same). */
  const uint8_t *sumdc = s + h.off_sumdc;
  for (uint64_t blk = 0; blk < h.n_blocks; blk++) {
    if (failed[blk]) { rep->uncorrectable[REF_T_RECON]++; bad = true; continue; }
    load_block<T>(P.g, blk, out, r);
    apply_recon_faults<T>(fl, blk, r, rep);
    store_block<T>(P.g, blk, r, out);
    if (!h.abft) continue;
    if (block_sum<T>(r) == get64(sumdc + 8 * blk)) continue;
    rep->detected[REF_T_RECON]++;
    if (decode_block<T>(s, P, K, blk, r) && block_sum<T>(r) == get64(sumdc + 8 * blk)) {
      store_block<T>(P.g, blk, r, out);
      rep->corrected[REF_T_RECON]++;
    } else {
      rep->uncorrectable[REF_T_RECON]++;
      bad = true;
    }
  }
  return bad ? REF_ESDC : REF_OK;
}

template <typename T>
int verify_impl(const uint8_t *s, const Parsed &P, T *data, const ref_fault *faults, uint32_t n_faults,
                ref_report *rep) {
  const Header &h = P.h;
  const Consts<T> K = make_consts<T>(h.eb_abs);
  std::vector<ref_fault> fl(faults, faults + n_faults);
  std::vector<T> r;
  bool bad = false;
  const uint8_t *sumdc = s + h.off_sumdc;
  for (uint64_t blk = 0; blk < h.n_blocks; blk++) {
    load_block<T>(P.g, blk, data, r);
    apply_recon_faults<T>(fl, blk, r, rep);
    store_block<T>(P.g, blk, r, data);
    if (block_sum<T>(r) == get64(sumdc + 8 * blk)) continue;
    rep->detected[REF_T_RECON]++;
    if (decode_block<T>(s, P, K, blk, r) && block_sum<T>(r) == get64(sumdc + 8 * blk)) {
      store_block<T>(P.g, blk, r, data);
      rep->corrected[REF_T_RECON]++;
    } else {
      rep->uncorrectable[REF_T_RECON]++;
      bad = true;
    }
  }
  return bad ? REF_ESDC : REF_OK;
}

template <typename T>
int region_impl(const uint8_t *s, const Parsed &P, const uint64_t lo[3], const uint64_t hi[3], T *out,
                ref_report *rep) {
  const Header &h = P.h;
  const Geometry &g = P.g;
  const Consts<T> K = make_consts<T>(h.eb_abs);
  uint64_t ext[3];
  for (int a = 0; a < 3; a++) ext[a] = hi[a] - lo[a];
  std::vector<T> r;
  bool bad = false;
  for (uint64_t blk = 0; blk < h.n_blocks; blk++) {
    BlockBox bb = block_box(g, blk);
    bool hit = true;
    for (int a = 0; a < 3; a++)
      if (bb.o[a] + bb.n[a] <= lo[a] || bb.o[a] >= hi[a]) hit = false;
    if (!hit) continue;
    bool ok = decode_block<T>(s, P, K, blk, r);
    if (ok && h.abft && block_sum<T>(r) != get64(s + h.off_sumdc + 8 * blk)) {
      rep->detected[REF_T_RECON]++;
      ok = decode_block<T>(s, P, K, blk, r) && block_sum<T>(r) == get64(s + h.off_sumdc + 8 * blk);
      if (ok) rep->corrected[REF_T_RECON]++;
    }
    if (!ok) { bad = true; rep->uncorrectable[REF_T_RECON]++; continue; }
    for (uint64_t i = 0, q = 0; i < bb.n[0]; i++)
      for (uint64_t j = 0; j < bb.n[1]; j++)
        for (uint64_t k = 0; k < bb.n[2]; k++, q++) {
          uint64_t z = bb.o[0] + i, y = bb.o[1] + j, x = bb.o[2] + k;
          if (z < lo[0] || z >= hi[0] || y < lo[1] || y >= hi[1] || x < lo[2] || x >= hi[2]) continue;
          out[((z - lo[0]) * ext[1] + (y - lo[1])) * ext[2] + (x - lo[2])] = r[q];
        }
  }
  return bad ? REF_ESDC : REF_OK;
}

bool valid_params(const ref_params *p, Geometry *g) {
  if (!p || p->dtype > 1 || p->eb_mode > 1 || p->predictor > 2 || p->abft > 1) return false;
  if (!(p->eb > 0) || !std::isfinite(p->eb)) return false;
  if (!make_geometry(p->ndim, p->dims, p->block, g)) return false;
  if (p->n_faults && !p->faults) return false;
  for (uint32_t t = 0; t < p->n_faults; t++) {
    const ref_fault &f = p->faults[t];
    if (f.target >= REF_N_TARGETS || f.block >= g->n_blocks) return false;
    BlockBox bb = block_box(*g, f.block);
    uint32_t per = p->dtype == 0 ? 1 : 2;
    switch (f.target) {
      case REF_T_INPUT:
      case REF_T_PREP_INPUT:
      case REF_T_RECON:
        if (f.word >= bb.pts * per || f.bit >= 32) return false;
        break;
      case REF_T_COEF:
      case REF_T_PREP_COEF:
        if (f.word >= 4ull * per || f.bit >= 32) return false;
        break;
      case REF_T_PREP_SAMPLE:
        if (f.word >= 2 || f.bit >= 64) return false;
        break;
      case REF_T_CODE:
        if (f.word >= bb.pts || f.bit >= 32) return false;
        break;
      default:
        if (f.word >= bb.pts || f.bit >= 32 * per) return false;
        break;
    }
  }
  return true;
}

}  // namespace

extern "C" void sdcsz_ref_regression(const void *vals, uint32_t dtype, const uint32_t ext[3], void *coef) {
  uint64_t n[3] = {ext[0], ext[1], ext[2]};
  if (dtype == REF_F32) regression<float>((const float *)vals, n, (float *)coef);
  else regression<double>((const double *)vals, n, (double *)coef);
}

extern "C" void sdcsz_ref_huffman_lengths(const uint64_t *hist, uint8_t *lengths) {
  huffman_lengths(hist, lengths);
}

extern "C" uint64_t sdcsz_ref_max_stream_size(const ref_params *p) {
  Geometry g;
  if (!p || !make_geometry(p->ndim, p->dims, p->block, &g)) return 0;
  uint64_t vb = p->dtype == REF_F32 ? 4 : 8;
  Header h{};
  h.abft = 1;
  h.n_sym = 65536;
  h.n_blocks = g.n_blocks;
  h.n_regression = g.n_blocks;
  h.n_outliers = g.n_values;
  h.payload_words = (g.n_values * kMaxCodeLen + 31) / 32 + g.n_blocks;
  layout(h, vb);
  return h.total;
}

extern "C" int sdcsz_ref_compress(const void *in, const ref_params *p, void *out, uint64_t out_cap,
                                  uint64_t *out_size, ref_report *rep, ref_debug *dbg) {
  ref_report local;
  if (!rep) rep = &local;
  std::memset(rep, 0, sizeof(*rep));
  uint64_t dummy;
  if (!out_size) out_size = &dummy;
  *out_size = 0;
  Geometry g;
  if (!valid_params(p, &g)) return REF_EINVAL;
  if (g.n_values && !in) return REF_EINVAL;
  if (p->dtype == REF_F32)
    return compress_impl<float>((const float *)in, p, g, (uint8_t *)out, out_cap, out_size, rep, dbg);
  return compress_impl<double>((const double *)in, p, g, (uint8_t *)out, out_cap, out_size, rep, dbg);
}

extern "C" int sdcsz_ref_read_header(const void *stream, uint64_t stream_size, ref_params *p, double *eb_abs,
                                     uint64_t *n_blocks) {
  Parsed P;
  int st = parse((const uint8_t *)stream, stream_size, P);
  if (st) return st;
  std::memset(p, 0, sizeof(*p));
  p->dtype = P.h.dtype;
  p->ndim = P.h.ndim;
  for (uint32_t a = 0; a < P.h.ndim; a++) {
    p->dims[a] = P.h.d[3 - P.h.ndim + a];
    p->block[a] = P.h.b[3 - P.h.ndim + a];
  }
  p->eb_mode = P.h.eb_mode;
  p->eb = P.h.eb;
  p->abft = P.h.abft;
  p->predictor = P.h.predictor;
  if (eb_abs) *eb_abs = P.h.eb_abs;
  if (n_blocks) *n_blocks = P.h.n_blocks;
  return REF_OK;
}

static bool valid_recon_faults(const Parsed &P, const ref_fault *faults, uint32_t n) {
  if (n && !faults) return false;
  uint32_t per = P.h.dtype == 0 ? 1 : 2;
  for (uint32_t t = 0; t < n; t++) {
    if (faults[t].target != REF_T_RECON) continue;
    if (faults[t].block >= P.h.n_blocks || faults[t].bit >= 32) return false;
    BlockBox bb = block_box(P.g, faults[t].block);
    if (faults[t].word >= bb.pts * per) return false;
  }
  return true;
}

extern "C" int sdcsz_ref_decompress(const void *stream, uint64_t stream_size, void *out, uint64_t out_cap,
                                    const ref_fault *faults, uint32_t n_faults, ref_report *rep) {
  ref_report local;
  if (!rep) rep = &local;
  std::memset(rep, 0, sizeof(*rep));
  Parsed P;
  int st = parse((const uint8_t *)stream, stream_size, P);
  if (st) return st;
  if (!valid_recon_faults(P, faults, n_faults)) return REF_EINVAL;
  uint64_t vb = P.h.dtype == 0 ? 4 : 8;
  if (out_cap < P.g.n_values * vb) return REF_ENOSPC;
  rep->n_blocks = P.h.n_blocks;
  rep->eb_abs = P.h.eb_abs;
  rep->n_outliers = P.h.n_outliers;
  rep->n_regression = P.h.n_regression;
  rep->payload_words = P.h.payload_words;
  rep->stream_size = P.h.total;
  if (P.h.dtype == 0) return decompress_impl<float>((const uint8_t *)stream, P, (float *)out, faults, n_faults, rep);
  return decompress_impl<double>((const uint8_t *)stream, P, (double *)out, faults, n_faults, rep);
}

extern "C" int sdcsz_ref_decompress_region(const void *stream, uint64_t stream_size, const uint64_t lo[3],
                                           const uint64_t hi[3], void *out, uint64_t out_cap, ref_report *rep) {
  ref_report local;
  if (!rep) rep = &local;
  std::memset(rep, 0, sizeof(*rep));
  Parsed P;
  int st = parse((const uint8_t *)stream, stream_size, P);
  if (st) return st;
  uint64_t L[3] = {0, 0, 0}, H[3] = {1, 1, 1};
  uint32_t off = 3 - P.h.ndim;
  for (uint32_t a = 0; a < P.h.ndim; a++) { L[off + a] = lo[a]; H[off + a] = hi[a]; }
  uint64_t cnt = 1;
  for (int a = 0; a < 3; a++) {
    if (L[a] >= H[a] || H[a] > P.g.d[a]) return REF_EINVAL;
    cnt *= H[a] - L[a];
  }
  uint64_t vb = P.h.dtype == 0 ? 4 : 8;
  if (out_cap < cnt * vb) return REF_ENOSPC;
  rep->n_blocks = P.h.n_blocks;
  rep->eb_abs = P.h.eb_abs;
  if (P.h.dtype == 0) return region_impl<float>((const uint8_t *)stream, P, L, H, (float *)out, rep);
  return region_impl<double>((const uint8_t *)stream, P, L, H, (double *)out, rep);
}

extern "C" int sdcsz_ref_verify(const void *stream, uint64_t stream_size, void *data, uint64_t data_size,
                                const ref_fault *faults, uint32_t n_faults, ref_report *rep) {
  ref_report local;
  if (!rep) rep = &local;
  std::memset(rep, 0, sizeof(*rep));
  Parsed P;
  int st = parse((const uint8_t *)stream, stream_size, P);
  if (st) return st;
  if (!P.h.abft) return REF_EINVAL;
  if (!valid_recon_faults(P, faults, n_faults)) return REF_EINVAL;
  uint64_t vb = P.h.dtype == 0 ? 4 : 8;
  if (data_size < P.g.n_values * vb) return REF_ENOSPC;
  rep->n_blocks = P.h.n_blocks;
  rep->eb_abs = P.h.eb_abs;
  if (P.h.dtype == 0) return verify_impl<float>((const uint8_t *)stream, P, (float *)data, faults, n_faults, rep);
  return verify_impl<double>((const uint8_t *)stream, P, (double *)data, faults, n_faults, rep);
}

/* ------------------------------------------------------------------------ */
/* Lossless stage: entry points.                                              */
/* ------------------------------------------------------------------------ */
extern "C" uint64_t sdcsz_ref_pack_column(const uint64_t *v, uint64_t n, uint32_t *out) {
  std::vector<uint32_t> w;
  pack_column(std::vector<uint64_t>(v, v + n), w);
  if (out) std::memcpy(out, w.data(), 4 * w.size());
  return w.size();
}

extern "C" int sdcsz_ref_pack(const void *stream, uint64_t size, void *out, uint64_t cap, uint64_t *out_size) {
  const uint8_t *s = (const uint8_t *)stream;
  Header h;
  if (!read_header(s, size, h) || h.total > size) return REF_EFORMAT;
  const uint64_t vb = h.dtype == REF_F32 ? 4 : 8, nb = h.n_blocks;
  Header v1 = h;
  std::vector<std::vector<uint64_t>> tcols(2, std::vector<uint64_t>(nb)), scols(1, std::vector<uint64_t>(nb));
  for (uint64_t b = 0; b < nb; b++) {
    tcols[0][b] = get32(s + v1.off_table + 8 * b);
    tcols[1][b] = get32(s + v1.off_table + 8 * b + 4);
    if (h.abft) scols[0][b] = get64(s + v1.off_sumdc + 8 * b);
  }
  const std::vector<uint32_t> tsec = pack_section(tcols, nb);
  const std::vector<uint32_t> ssec = h.abft ? pack_section(scols, nb) : std::vector<uint32_t>();
  Header h2 = h;
  layout_packed_front(h2, vb);
  h2.off_sumdc = align8(h2.off_table + 4ull * tsec.size());
  h2.total = align8(h2.off_sumdc + 4ull * ssec.size());
  *out_size = h2.total;
  if (h2.total > cap) return REF_ENOSPC;
  uint8_t *o = (uint8_t *)out;
  std::memset(o, 0, h2.total);
  write_header(o, h2);
  std::memcpy(o, kMagicPacked, 8);
  std::memcpy(o + h2.off_codebook, s + v1.off_codebook, 4ull * h.n_sym);
  std::memcpy(o + h2.off_coef, s + v1.off_coef, 4ull * vb * h.n_regression);
  std::memcpy(o + h2.off_outliers, s + v1.off_outliers, vb * h.n_outliers);
  std::memcpy(o + h2.off_payload, s + v1.off_payload, 4ull * h.payload_words);
  std::memcpy(o + h2.off_table, tsec.data(), 4 * tsec.size());
  if (!ssec.empty()) std::memcpy(o + h2.off_sumdc, ssec.data(), 4 * ssec.size());
  return REF_OK;
}

extern "C" int sdcsz_ref_unpack(const void *packed, uint64_t size, void *out, uint64_t cap, uint64_t *out_size) {
  const uint8_t *s = (const uint8_t *)packed;
  if (size < kHeaderBytes || std::memcmp(s, kMagicPacked, 8) != 0) return REF_EFORMAT;
  Header h2;
  read_fields(s, h2);
  if (h2.dtype > 1 || h2.abft > 1 || h2.n_sym > 65536 || h2.total > size) return REF_EFORMAT;
  const uint64_t vb = h2.dtype == REF_F32 ? 4 : 8, nb = h2.n_blocks;
  Header chk = h2;
  layout_packed_front(chk, vb);
  if (chk.off_codebook != h2.off_codebook || chk.off_coef != h2.off_coef || chk.off_outliers != h2.off_outliers ||
      chk.off_payload != h2.off_payload || chk.off_table != h2.off_table || h2.off_sumdc < h2.off_table ||
      h2.total < h2.off_sumdc || h2.off_sumdc % 8 != 0)
    return REF_EFORMAT;
  const uint32_t tmax[2] = {32, 32}, smax[1] = {64};
  std::vector<std::vector<uint64_t>> tcols, scols;
  const uint64_t tbytes = h2.off_sumdc - h2.off_table;
  /* the table section ends at the last chunk's word, then pads to 8 bytes */
  const uint64_t nch = (nb + kPackChunk - 1) / kPackChunk;
  if (tbytes < 4 * (nch + 1)) return REF_EFORMAT;
  const uint32_t tlast = get32(s + h2.off_table + 4 * nch);
  const uint64_t tused = 4 * (nch + 1 + (uint64_t)tlast);
  if (tused > tbytes || align8(h2.off_table + tused) != h2.off_sumdc) return REF_EFORMAT;
  if (!unpack_section(s, h2.off_table, tused, nb, tmax, 2, tcols)) return REF_EFORMAT;
  if (h2.abft) {
    const uint64_t sbytes = h2.total - h2.off_sumdc;
    if (sbytes < 4 * (nch + 1)) return REF_EFORMAT;
    const uint32_t slast = get32(s + h2.off_sumdc + 4 * nch);
    const uint64_t sused = 4 * (nch + 1 + (uint64_t)slast);
    if (sused > sbytes || align8(h2.off_sumdc + sused) != h2.total) return REF_EFORMAT;
    if (!unpack_section(s, h2.off_sumdc, sused, nb, smax, 1, scols)) return REF_EFORMAT;
  } else if (h2.total != h2.off_sumdc) {
    return REF_EFORMAT;
  }
  for (uint64_t b = 0; b < nb; b++)
    if (tcols[0][b] > 0xFFFFFFFFull || tcols[1][b] > 0xFFFFFFFFull) return REF_EFORMAT;
  Header h = h2;
  layout(h, vb);
  *out_size = h.total;
  if (h.total > cap) return REF_ENOSPC;
  uint8_t *o = (uint8_t *)out;
  std::memset(o, 0, h.total);
  write_header(o, h);
  std::memcpy(o + h.off_codebook, s + h2.off_codebook, 4ull * h.n_sym);
  for (uint64_t b = 0; b < nb; b++) {
    put32(o + h.off_table + 8 * b, (uint32_t)tcols[0][b]);
    put32(o + h.off_table + 8 * b + 4, (uint32_t)tcols[1][b]);
    if (h.abft) put64(o + h.off_sumdc + 8 * b, scols[0][b]);
  }
  std::memcpy(o + h.off_coef, s + h2.off_coef, 4ull * vb * h.n_regression);
  std::memcpy(o + h.off_outliers, s + h2.off_outliers, vb * h.n_outliers);
  std::memcpy(o + h.off_payload, s + h2.off_payload, 4ull * h.payload_words);
  return REF_OK;
}
