/*
 * hoszp_ref.c -- CPU oracle for HoSZp (arXiv 2408.11971).
 *
 * TEST INFRASTRUCTURE ONLY: linked by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  The GPU library never includes, links
 * or calls anything in this directory.
 *
 * Plain single-threaded C11 (plus gcc's __int128).  Every step is written in
 * the order the paper gives it, one element and one bit at a time, so it can
 * be checked against the paper by eye:
 *
 *   Sec. IV-A step 1  (Eq. 3)  quantization       q = floor((a + eps) / (2 eps))
 *   Sec. IV-A step 2  (Eq. 4)  1-D Lorenzo        P^i = q^i - q^(i-1), outlier O = q^0
 *   Sec. IV-A (signs)          sign array         1 = negative, 0 = positive or zero
 *   Sec. IV-A step 3           fixed-length BF    every |P| of a block at the
 *                                                 block's maximum bit length
 *   Sec. IV-A, Fig. 3          stream order       widths, outliers, signs, bits
 *   Sec. V-A-1  negation       flip signs (and the outliers, see below)
 *   Sec. V-A-4  scalar mul     bins -> floor(s q + 1/2) -> LZ -> BF
 *   Sec. V-B-1  mean           2 eps * (sum q) / N
 *   Sec. V-B-2  variance       population variance of the bins times (2 eps)^2
 *   Sec. V-C-1  element add    O_A + O_B and signed P_A + P_B, then BF
 *   Sec. V-A    scalar add/sub O +- q_s, q_s the scalar's bin by Eq. 3
 *   Sec. V-B    std            sqrt of the variance
 *   Sec. V-B    block means    2 eps * (sum of a block's q) / its length
 *   Sec. V-C    element sub    bins q_A - q_B, then LZ -> BF
 *   Sec. V-C    Hadamard       bins floor(2 eps q_A q_B + 1/2), then LZ -> BF
 *   Sec. V-D    covariance     (2 eps_A)(2 eps_B) (n sum q_A q_B - S_A S_B) / n^2
 *
 * Readings of points the paper leaves open (each is listed with its reason in
 * the design notes of the repository):
 *   - Eq. 3 is evaluated in binary64 as floor(((double)a + eps) * inv) with
 *     inv = 1 / (2 eps); the two operations are rounded separately (no FMA).
 *   - Blocks are flat runs of `block` consecutive elements of the row-major
 *     field; the last block may be shorter (its missing slots are zeros).
 *   - Slot 0 of every block carries delta 0; the outlier holds its bin (the
 *     worked example of Sec. IV-A, not the literal i = 0 case of Eq. 4).
 *   - Widths are bit lengths of the largest magnitude (0 = constant block);
 *     fields are packed element-major, most significant bit first, into a
 *     big-endian bit string; the same bit order holds the sign bits.  This is
 *     the only order that reproduces the example's packed byte 0x08.
 *   - Every block owns block/8 sign bytes, constant blocks included.
 *   - Negation also negates the outliers (without that the decoded field is
 *     not the negated field) and flips the sign bits of the valid slots of
 *     non-constant blocks.
 *   - Scalar multiplication uses the unquantized scalar and rounds half up,
 *     which equals re-quantizing s * (2 eps q) with Eq. 3.
 *   - Scalar addition and subtraction use the scalar's bin by Eq. 3 (the
 *     bin printed in the paper's example, 33 for 0.67 at eps 0.01, is one
 *     below what Eq. 3 gives, 34).  The Hadamard product re-quantizes the
 *     product of the decoded values at the operands' eps with half-up
 *     rounding, as scalar multiplication does.  Covariance and the block
 *     means divide exact integer sums, as the mean and variance do.
 *
 * Stream layout (all integers little-endian):
 *   header, 64 bytes:  "HOSZ" | u16 version=1 | u16 flags=0 | u32 block |
 *                      u32 0 | u64 n | f64 eb | u64 nb | u64 payload_bytes |
 *                      u64 total_bytes | u64 0
 *   then, each section starting at the next multiple of 16 bytes:
 *   W  nb bytes        block widths
 *   O  4*nb bytes      outliers as int32
 *   S  nb*block/8      sign bits, slot k of a block at bit 7-(k%8) of byte k/8
 *   P  payload_bytes   each block's block*width bits, blocks back to back
 */
#include "hoszp_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define HEADER_BYTES 64u
#define BIN_MAX 2147483647LL /* bins live in [-BIN_MAX, BIN_MAX] */
#define N_LIMIT 4294967295ULL /* n must stay below 2^32 */

typedef __int128 i128;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* little-endian scalar access, one byte at a time                      */
/* ------------------------------------------------------------------ */

static void put_u16(uint8_t* p, uint16_t v) {
  for (int i = 0; i < 2; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
static uint16_t get_u16(const uint8_t* p) {
  uint16_t v = 0;
  for (int i = 1; i >= 0; --i) v = (uint16_t)((v << 8) | p[i]);
  return v;
}
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  for (int i = 3; i >= 0; --i) v = (v << 8) | p[i];
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; --i) v = (v << 8) | p[i];
  return v;
}
static void put_f64(uint8_t* p, double d) {
  uint64_t v;
  memcpy(&v, &d, 8);
  put_u64(p, v);
}
static double get_f64(const uint8_t* p) {
  uint64_t v = get_u64(p);
  double d;
  memcpy(&d, &v, 8);
  return d;
}

/* ------------------------------------------------------------------ */
/* bit string: bit position p lives in byte p/8 at bit 7 - p%8          */
/* ------------------------------------------------------------------ */

static void put_bit(uint8_t* buf, uint64_t p, unsigned bit) {
  if (bit) buf[p >> 3] |= (uint8_t)(0x80u >> (p & 7u));
}
static unsigned get_bit(const uint8_t* buf, uint64_t p) {
  return (buf[p >> 3] >> (7u - (unsigned)(p & 7u))) & 1u;
}
/* write `width` bits of v, most significant first, starting at bit p */
static void put_field(uint8_t* buf, uint64_t p, uint32_t v, unsigned width) {
  for (unsigned j = 0; j < width; ++j) put_bit(buf, p + j, (v >> (width - 1u - j)) & 1u);
}
static uint32_t get_field(const uint8_t* buf, uint64_t p, unsigned width) {
  uint32_t v = 0;
  for (unsigned j = 0; j < width; ++j) v = (v << 1) | get_bit(buf, p + j);
  return v;
}

/* ------------------------------------------------------------------ */
/* layout                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
  uint64_t n, nb;
  uint32_t block;
  double eb;
  uint64_t off_w, off_o, off_s, off_p;
  uint64_t payload_bytes, total_bytes;
} layout;

static uint64_t round16(uint64_t x) { return (x + 15u) / 16u * 16u; }

#define MAX_BLOCK 256 /* largest block size accepted */
static int block_ok(uint32_t block) {
  return block == 32 || block == 64 || block == 128 || block == 256;
}

static void place_sections(layout* g) {
  g->nb = (g->n + g->block - 1) / g->block;
  g->off_w = HEADER_BYTES;
  g->off_o = round16(g->off_w + g->nb);
  g->off_s = round16(g->off_o + 4u * g->nb);
  g->off_p = round16(g->off_s + g->nb * (g->block / 8u));
}

size_t hoszp_ref_bound(uint64_t n, uint32_t block) {
  if (n == 0 || n > N_LIMIT || !block_ok(block)) return 0;
  layout g;
  memset(&g, 0, sizeof g);
  g.n = n;
  g.block = block;
  place_sections(&g);
  /* every block at width 32: block * 32 bits = 4 * block bytes */
  return (size_t)(g.off_p + g.nb * 4u * block);
}

static void write_header(uint8_t* out, const layout* g) {
  memset(out, 0, HEADER_BYTES);
  out[0] = 'H';
  out[1] = 'O';
  out[2] = 'S';
  out[3] = 'Z';
  put_u16(out + 4, 1);
  put_u16(out + 6, 0);
  put_u32(out + 8, g->block);
  put_u32(out + 12, 0);
  put_u64(out + 16, g->n);
  put_f64(out + 24, g->eb);
  put_u64(out + 32, g->nb);
  put_u64(out + 40, g->payload_bytes);
  put_u64(out + 48, g->total_bytes);
  put_u64(out + 56, 0);
}

/* Parse and validate a stream; every decoder goes through here. */
static int read_layout(const uint8_t* c, size_t c_bytes, layout* g) {
  if (c == NULL || c_bytes < HEADER_BYTES) return REF_ERR_FORMAT;
  if (c[0] != 'H' || c[1] != 'O' || c[2] != 'S' || c[3] != 'Z') return REF_ERR_FORMAT;
  if (get_u16(c + 4) != 1 || get_u16(c + 6) != 0) return REF_ERR_FORMAT;
  memset(g, 0, sizeof *g);
  g->block = get_u32(c + 8);
  g->n = get_u64(c + 16);
  g->eb = get_f64(c + 24);
  if (!block_ok(g->block) || g->n == 0 || g->n > N_LIMIT) return REF_ERR_FORMAT;
  if (!isfinite(g->eb) || !(g->eb > 0.0)) return REF_ERR_FORMAT;
  place_sections(g);
  if (get_u64(c + 32) != g->nb) return REF_ERR_FORMAT;
  g->payload_bytes = get_u64(c + 40);
  g->total_bytes = get_u64(c + 48);
  if (g->total_bytes > c_bytes) return REF_ERR_FORMAT;
  if (g->off_p > g->total_bytes || g->total_bytes - g->off_p != g->payload_bytes)
    return REF_ERR_FORMAT;
  /* widths: each at most 32, and together they must fill the payload */
  uint64_t bits = 0;
  for (uint64_t b = 0; b < g->nb; ++b) {
    uint8_t w = c[g->off_w + b];
    if (w > 32) return REF_ERR_FORMAT;
    bits += (uint64_t)w * g->block;
  }
  if (bits / 8u != g->payload_bytes) return REF_ERR_FORMAT;
  return REF_OK;
}

int hoszp_ref_info(const uint8_t* c, size_t c_bytes, uint64_t* n, uint32_t* block,
                   double* eb, uint64_t* payload_bytes, uint64_t* total_bytes) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (n) *n = g.n;
  if (block) *block = g.block;
  if (eb) *eb = g.eb;
  if (payload_bytes) *payload_bytes = g.payload_bytes;
  if (total_bytes) *total_bytes = g.total_bytes;
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. IV-A step 1: quantization (Eq. 3)                              */
/* ------------------------------------------------------------------ */

int hoszp_ref_quantize(const float* x, uint64_t n, double eb, int32_t* q) {
  if (x == NULL || q == NULL || n == 0 || !isfinite(eb) || !(eb > 0.0)) return REF_ERR_ARG;
  for (uint64_t i = 0; i < n; ++i)
    if (!isfinite(x[i])) return REF_ERR_NONFINITE;
  const double two_eb = 2.0 * eb;
  const double inv = 1.0 / two_eb;
  for (uint64_t i = 0; i < n; ++i) {
    /* two separately rounded operations (built with -ffp-contract=off) */
    double shifted = (double)x[i] + eb;
    double scaled = shifted * inv;
    double f = floor(scaled);
    if (f < -(double)BIN_MAX || f > (double)BIN_MAX) return REF_ERR_RANGE;
    q[i] = (int32_t)f;
  }
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. IV-A steps 2-3 for one block: signs, width, fixed-length bits   */
/* ------------------------------------------------------------------ */

/* d[k] are the signed Lorenzo deltas of the block (d[0] = 0, slots beyond
 * the block's length are 0); `outlier` is its first bin.  `bitpos` is the
 * block's first payload bit; returns the block width. */
static unsigned encode_block(uint8_t* out, const layout* g, uint64_t b, int32_t outlier,
                             const int64_t* d, uint64_t bitpos) {
  const uint32_t L = g->block;
  uint32_t mag[MAX_BLOCK];
  unsigned neg[MAX_BLOCK];
  uint32_t biggest = 0;
  for (uint32_t k = 0; k < L; ++k) {
    neg[k] = d[k] < 0 ? 1u : 0u;
    mag[k] = (uint32_t)(d[k] < 0 ? -d[k] : d[k]);
    if (mag[k] > biggest) biggest = mag[k];
  }
  unsigned width = 0;
  while (width < 32 && (biggest >> width) != 0) ++width;

  out[g->off_w + b] = (uint8_t)width;
  put_u32(out + g->off_o + 4u * b, (uint32_t)outlier);
  uint8_t* signs = out + g->off_s + b * (L / 8u);
  for (uint32_t k = 0; k < L; ++k) put_bit(signs, k, neg[k]);
  for (uint32_t k = 0; k < L; ++k) put_field(out + g->off_p, bitpos + (uint64_t)k * width, mag[k], width);
  return width;
}

/* Lorenzo deltas of a block of bins (Eq. 4 with the outlier split off). */
static void block_deltas(const int32_t* q, uint64_t first, uint32_t len, uint32_t L, int64_t* d) {
  for (uint32_t k = 0; k < L; ++k) d[k] = 0;
  for (uint32_t k = 1; k < len; ++k) d[k] = (int64_t)q[first + k] - (int64_t)q[first + k - 1];
}

static uint32_t block_len(const layout* g, uint64_t b) {
  uint64_t first = b * g->block;
  uint64_t left = g->n - first;
  return left < g->block ? (uint32_t)left : g->block;
}

static void finish_stream(uint8_t* out, layout* g, uint64_t bits) {
  g->payload_bytes = bits / 8u;
  g->total_bytes = g->off_p + g->payload_bytes;
  write_header(out, g);
}

int hoszp_ref_encode_bins(const int32_t* q, uint64_t n, double eb, uint32_t block,
                          uint8_t* out, size_t out_cap, size_t* out_bytes) {
  if (q == NULL || out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  if (n == 0 || n > N_LIMIT || !block_ok(block) || !isfinite(eb) || !(eb > 0.0))
    return REF_ERR_ARG;
  size_t bound = hoszp_ref_bound(n, block);
  if (out_cap < bound) return REF_ERR_CAPACITY;
  for (uint64_t i = 0; i < n; ++i)
    if (q[i] < -BIN_MAX) return REF_ERR_RANGE;
  layout g;
  memset(&g, 0, sizeof g);
  g.n = n;
  g.block = block;
  g.eb = eb;
  place_sections(&g);
  memset(out, 0, bound);
  int64_t d[MAX_BLOCK];
  uint64_t bits = 0;
  for (uint64_t b = 0; b < g.nb; ++b) {
    uint64_t first = b * block;
    uint32_t len = block_len(&g, b);
    block_deltas(q, first, len, block, d);
    unsigned width = encode_block(out, &g, b, q[first], d, bits);
    bits += (uint64_t)block * width;
  }
  finish_stream(out, &g, bits);
  *out_bytes = (size_t)g.total_bytes;
  return REF_OK;
}

int hoszp_ref_compress(const float* x, uint64_t n, double eb, uint32_t block,
                       uint8_t* out, size_t out_cap, size_t* out_bytes) {
  if (x == NULL || out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  if (n == 0 || n > N_LIMIT || !block_ok(block) || !isfinite(eb) || !(eb > 0.0))
    return REF_ERR_ARG;
  if (out_cap < hoszp_ref_bound(n, block)) return REF_ERR_CAPACITY;
  int32_t* q = (int32_t*)malloc(n * sizeof(int32_t));
  if (q == NULL) return REF_ERR_ARG;
  int rc = hoszp_ref_quantize(x, n, eb, q);
  if (rc == REF_OK) rc = hoszp_ref_encode_bins(q, n, eb, block, out, out_cap, out_bytes);
  free(q);
  return rc;
}

/* ------------------------------------------------------------------ */
/* decoding: inverse BF then inverse LZ                                 */
/* ------------------------------------------------------------------ */

/* Signed deltas of block b.  Slot 0 and slots past the block's length are
 * reported as 0 whatever bits they hold: slot 0's bin is the outlier. */
static void decode_block(const uint8_t* c, const layout* g, uint64_t b, uint64_t bitpos,
                         int32_t* outlier, int64_t* d, unsigned* width_out) {
  const uint32_t L = g->block;
  unsigned width = c[g->off_w + b];
  uint32_t len = block_len(g, b);
  *outlier = (int32_t)get_u32(c + g->off_o + 4u * b);
  const uint8_t* signs = c + g->off_s + b * (L / 8u);
  for (uint32_t k = 0; k < L; ++k) {
    int64_t m = (int64_t)get_field(c + g->off_p, bitpos + (uint64_t)k * width, width);
    d[k] = get_bit(signs, k) ? -m : m;
    if (k == 0 || k >= len) d[k] = 0;
  }
  *width_out = width;
}

/* Walk every block in order, handing its outlier and deltas to `visit`. */
typedef int (*block_visitor)(void* user, uint64_t b, uint32_t len, int32_t outlier,
                             const int64_t* d);

static int for_each_block(const uint8_t* c, const layout* g, block_visitor visit, void* user) {
  int64_t d[MAX_BLOCK];
  uint64_t bits = 0;
  for (uint64_t b = 0; b < g->nb; ++b) {
    int32_t outlier;
    unsigned width;
    decode_block(c, g, b, bits, &outlier, d, &width);
    int rc = visit(user, b, block_len(g, b), outlier, d);
    if (rc) return rc;
    bits += (uint64_t)g->block * width;
  }
  return REF_OK;
}

typedef struct {
  int32_t* q;
  uint32_t block;
} bins_sink;

/* inverse Lorenzo: q^0 = O, q^k = q^(k-1) + P^k */
static int store_bins(void* user, uint64_t b, uint32_t len, int32_t outlier, const int64_t* d) {
  bins_sink* s = (bins_sink*)user;
  int32_t* q = s->q + b * s->block;
  int64_t v = outlier;
  for (uint32_t k = 0; k < len; ++k) {
    if (k > 0) v += d[k];
    if (v < -BIN_MAX || v > BIN_MAX) return REF_ERR_FORMAT; /* bins stay in range */
    q[k] = (int32_t)v;
  }
  return REF_OK;
}

int hoszp_ref_decode_bins(const uint8_t* c, size_t c_bytes, int32_t* q, uint64_t n_cap) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (q == NULL || n_cap < g.n) return REF_ERR_CAPACITY;
  bins_sink s = {q, g.block};
  return for_each_block(c, &g, store_bins, &s);
}

int hoszp_ref_decompress(const uint8_t* c, size_t c_bytes, float* x, uint64_t n_cap) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (x == NULL || n_cap < g.n) return REF_ERR_CAPACITY;
  int32_t* q = (int32_t*)malloc(g.n * sizeof(int32_t));
  if (q == NULL) return REF_ERR_ARG;
  bins_sink s = {q, g.block};
  rc = for_each_block(c, &g, store_bins, &s);
  if (rc == REF_OK) {
    const double two_eb = 2.0 * g.eb;
    for (uint64_t i = 0; i < g.n; ++i) x[i] = (float)((double)q[i] * two_eb);
  }
  free(q);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Sec. V-A-1: negation                                                 */
/* ------------------------------------------------------------------ */

int hoszp_ref_negate(const uint8_t* c, size_t c_bytes, uint8_t* out, size_t out_cap,
                     size_t* out_bytes) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  if (out_cap < g.total_bytes) return REF_ERR_CAPACITY;
  if (out != c) memmove(out, c, (size_t)g.total_bytes);
  for (uint64_t b = 0; b < g.nb; ++b) {
    /* O -> -O in 32-bit two's complement (valid outliers never wrap) */
    uint32_t o = get_u32(out + g.off_o + 4u * b);
    put_u32(out + g.off_o + 4u * b, 0u - o);
    if (out[g.off_w + b] == 0) continue;             /* constant block: no signs */
    uint8_t* signs = out + g.off_s + b * (g.block / 8u);
    uint32_t len = block_len(&g, b);
    for (uint32_t k = 0; k < len; ++k) signs[k >> 3] ^= (uint8_t)(0x80u >> (k & 7u));
  }
  *out_bytes = (size_t)g.total_bytes;
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. V-C-1: element-wise addition                                    */
/* ------------------------------------------------------------------ */

static int same_shape(const layout* a, const layout* b) {
  uint64_t ea, eb;
  memcpy(&ea, &a->eb, 8);
  memcpy(&eb, &b->eb, 8);
  return a->n == b->n && a->block == b->block && ea == eb;
}

int hoszp_ref_add(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                  uint8_t* out, size_t out_cap, size_t* out_bytes) {
  layout ga, gb;
  int rc = read_layout(a, a_bytes, &ga);
  if (rc) return rc;
  rc = read_layout(b, b_bytes, &gb);
  if (rc) return rc;
  if (out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  if (!same_shape(&ga, &gb)) return REF_ERR_MISMATCH;
  size_t bound = hoszp_ref_bound(ga.n, ga.block);
  if (out_cap < bound) return REF_ERR_CAPACITY;

  layout g = ga;
  uint8_t* z = (uint8_t*)calloc(bound, 1); /* output may alias an input */
  if (z == NULL) return REF_ERR_ARG;
  int64_t da[MAX_BLOCK], db[MAX_BLOCK], dz[MAX_BLOCK];
  uint64_t bits_a = 0, bits_b = 0, bits_z = 0;
  for (uint64_t k = 0; k < g.nb && rc == REF_OK; ++k) {
    int32_t oa, ob;
    unsigned wa, wb;
    decode_block(a, &ga, k, bits_a, &oa, da, &wa);
    decode_block(b, &gb, k, bits_b, &ob, db, &wb);
    bits_a += (uint64_t)g.block * wa;
    bits_b += (uint64_t)g.block * wb;
    /* O_{A+B} = O_A + O_B, P_{A+B} = P_A + P_B (signed) */
    int64_t oz = (int64_t)oa + (int64_t)ob;
    for (uint32_t i = 0; i < g.block; ++i) dz[i] = da[i] + db[i];
    /* the summed field must still have every bin in range */
    uint32_t len = block_len(&g, k);
    int64_t v = oz;
    if (v < -BIN_MAX || v > BIN_MAX) rc = REF_ERR_RANGE;
    for (uint32_t i = 1; i < len && rc == REF_OK; ++i) {
      v += dz[i];
      if (v < -BIN_MAX || v > BIN_MAX) rc = REF_ERR_RANGE;
    }
    if (rc) break;
    unsigned wz = encode_block(z, &g, k, (int32_t)oz, dz, bits_z);
    bits_z += (uint64_t)g.block * wz;
  }
  if (rc == REF_OK) {
    finish_stream(z, &g, bits_z);
    memcpy(out, z, bound);
    *out_bytes = (size_t)g.total_bytes;
  }
  free(z);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Sec. V-A-4: scalar multiplication                                    */
/* ------------------------------------------------------------------ */

/* floor(s * q + 1/2) computed exactly: s = m * 2^e with an integer m. */
static int exact_scaled_bin(double s, int32_t q, int64_t* result) {
  int e2;
  double frac = frexp(s, &e2);                 /* s = frac * 2^e2, |frac| in [0.5, 1) */
  int64_t m = (int64_t)ldexp(frac, 53);        /* exact: 53-bit integer */
  int e = e2 - 53;                             /* s = m * 2^e */
  i128 p = (i128)m * (i128)q;                  /* |p| < 2^84 */
  i128 r;
  if (m == 0 || q == 0) {
    r = 0;
  } else if (e >= 0) {
    if (e > 40) return REF_ERR_RANGE;          /* |p| >= 1, so |p 2^e| > 2^40 */
    r = p * ((i128)1 << e);
  } else if (-e > 100) {
    r = 0;                                     /* |s q| < 2^-16: rounds to 0 */
  } else {
    int sh = -e;
    i128 half = (i128)1 << (sh - 1);
    i128 t = p + half;
    /* floor division by 2^sh */
    i128 quo = t / ((i128)1 << sh);
    if (t < 0 && quo * ((i128)1 << sh) != t) quo -= 1;
    r = quo;
  }
  if (r < -(i128)BIN_MAX || r > (i128)BIN_MAX) return REF_ERR_RANGE;
  *result = (int64_t)r;
  return REF_OK;
}

int hoszp_ref_mul(const uint8_t* c, size_t c_bytes, double s, uint8_t* out,
                  size_t out_cap, size_t* out_bytes) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (out == NULL || out_bytes == NULL || !isfinite(s)) return REF_ERR_ARG;
  if (out_cap < hoszp_ref_bound(g.n, g.block)) return REF_ERR_CAPACITY;
  int32_t* q = (int32_t*)malloc(g.n * sizeof(int32_t));
  if (q == NULL) return REF_ERR_ARG;
  bins_sink sink = {q, g.block};
  rc = for_each_block(c, &g, store_bins, &sink); /* inverse BF + inverse LZ */
  for (uint64_t i = 0; i < g.n && rc == REF_OK; ++i) {
    int64_t r;
    rc = exact_scaled_bin(s, q[i], &r);
    if (rc == REF_OK) q[i] = (int32_t)r;
  }
  if (rc == REF_OK) {
    uint8_t* z = (uint8_t*)malloc(hoszp_ref_bound(g.n, g.block)); /* out may alias c */
    if (z == NULL) {
      rc = REF_ERR_ARG;
    } else {
      size_t nbytes = 0;
      rc = hoszp_ref_encode_bins(q, g.n, g.eb, g.block, z, hoszp_ref_bound(g.n, g.block), &nbytes);
      if (rc == REF_OK) {
        memcpy(out, z, hoszp_ref_bound(g.n, g.block));
        *out_bytes = nbytes;
      }
      free(z);
    }
  }
  free(q);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Sec. V-B: mean and variance from exact integer sums                 */
/* ------------------------------------------------------------------ */

typedef struct {
  i128 s;
  u128 q;
} sums_acc;

static int add_sums(void* user, uint64_t b, uint32_t len, int32_t outlier, const int64_t* d) {
  (void)b;
  sums_acc* acc = (sums_acc*)user;
  int64_t v = outlier;
  for (uint32_t k = 0; k < len; ++k) {
    if (k > 0) v += d[k];
    if (v < -BIN_MAX || v > BIN_MAX) return REF_ERR_FORMAT;
    acc->s += v;
    acc->q += (u128)((i128)v * (i128)v);
  }
  return REF_OK;
}

static int exact_sums(const uint8_t* c, size_t c_bytes, layout* g, sums_acc* acc) {
  int rc = read_layout(c, c_bytes, g);
  if (rc) return rc;
  acc->s = 0;
  acc->q = 0;
  return for_each_block(c, g, add_sums, acc);
}

int hoszp_ref_sums(const uint8_t* c, size_t c_bytes, int64_t* s, uint64_t* q_lo,
                   uint64_t* q_hi) {
  layout g;
  sums_acc acc;
  int rc = exact_sums(c, c_bytes, &g, &acc);
  if (rc) return rc;
  if (s) *s = (int64_t)acc.s;
  if (q_lo) *q_lo = (uint64_t)acc.q;
  if (q_hi) *q_hi = (uint64_t)(acc.q >> 64);
  return REF_OK;
}

int hoszp_ref_mean(const uint8_t* c, size_t c_bytes, double* mean) {
  layout g;
  sums_acc acc;
  int rc = exact_sums(c, c_bytes, &g, &acc);
  if (rc) return rc;
  if (mean == NULL) return REF_ERR_ARG;
  const double two_eb = 2.0 * g.eb;
  *mean = ((double)(int64_t)acc.s / (double)g.n) * two_eb;
  return REF_OK;
}

int hoszp_ref_variance(const uint8_t* c, size_t c_bytes, double* var) {
  layout g;
  sums_acc acc;
  int rc = exact_sums(c, c_bytes, &g, &acc);
  if (rc) return rc;
  if (var == NULL) return REF_ERR_ARG;
  /* sum_i (q_i - S/N)^2 = (N Q - S^2) / N, exactly; then divide by N */
  i128 m = (i128)g.n * (i128)acc.q - acc.s * acc.s; /* Q < 2^94, N < 2^32 */
  const double two_eb = 2.0 * g.eb;
  *var = (((double)m / (double)g.n) / (double)g.n) * (two_eb * two_eb);
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. V-A: scalar addition and subtraction (workflow 1)               */
/* ------------------------------------------------------------------ */

/* Quantization bin of a scalar by Eq. 3, evaluated like every element. */
static int scalar_bin(double s, double eb, int64_t* qs) {
  if (!isfinite(s)) return REF_ERR_ARG;
  const double two_eb = 2.0 * eb;
  const double inv = 1.0 / two_eb;
  double sum = s + eb; /* two separately rounded operations, as Eq. 3 */
  double t = sum * inv;
  double bin = floor(t);
  if (!(bin >= -(double)BIN_MAX && bin <= (double)BIN_MAX)) return REF_ERR_RANGE;
  *qs = (int64_t)bin;
  return REF_OK;
}

typedef struct {
  int64_t delta;
} shift_check;

/* every shifted bin q + delta must stay in the bin range */
static int check_shifted(void* user, uint64_t b, uint32_t len, int32_t outlier, const int64_t* d) {
  (void)b;
  const shift_check* sc = (const shift_check*)user;
  int64_t v = outlier;
  for (uint32_t k = 0; k < len; ++k) {
    if (k > 0) v += d[k];
    if (v < -BIN_MAX || v > BIN_MAX) return REF_ERR_FORMAT;
    if (v + sc->delta < -BIN_MAX || v + sc->delta > BIN_MAX) return REF_ERR_RANGE;
  }
  return REF_OK;
}

/* Add `delta` to every bin by adding it to every outlier; widths, signs and
 * magnitudes are copied unchanged (the deltas do not change). */
static int shift_outliers(const uint8_t* c, size_t c_bytes, double s, int sign, uint8_t* out,
                          size_t out_cap, size_t* out_bytes) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  int64_t qs = 0;
  rc = scalar_bin(s, g.eb, &qs);
  if (rc) return rc;
  if (out_cap < g.total_bytes) return REF_ERR_CAPACITY;
  shift_check sc = {sign * qs};
  rc = for_each_block(c, &g, check_shifted, &sc);
  if (rc) return rc;
  if (out != c) memmove(out, c, (size_t)g.total_bytes);
  for (uint64_t b = 0; b < g.nb; ++b) {
    int64_t o = (int64_t)(int32_t)get_u32(out + g.off_o + 4u * b);
    put_u32(out + g.off_o + 4u * b, (uint32_t)(int32_t)(o + sc.delta));
  }
  *out_bytes = (size_t)g.total_bytes;
  return REF_OK;
}

int hoszp_ref_scalar_add(const uint8_t* c, size_t c_bytes, double s, uint8_t* out,
                         size_t out_cap, size_t* out_bytes) {
  return shift_outliers(c, c_bytes, s, 1, out, out_cap, out_bytes);
}

int hoszp_ref_scalar_sub(const uint8_t* c, size_t c_bytes, double s, uint8_t* out,
                         size_t out_cap, size_t* out_bytes) {
  return shift_outliers(c, c_bytes, s, -1, out, out_cap, out_bytes);
}

/* ------------------------------------------------------------------ */
/* Sec. V-B: standard deviation                                         */
/* ------------------------------------------------------------------ */

int hoszp_ref_std(const uint8_t* c, size_t c_bytes, double* std) {
  double var = 0.0;
  int rc = hoszp_ref_variance(c, c_bytes, &var);
  if (rc) return rc;
  if (std == NULL) return REF_ERR_ARG;
  *std = sqrt(var);
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* Bivariate operations (Sec. V-C, V-D): both operands decoded to bins   */
/* ------------------------------------------------------------------ */

/* Bins of both operands; `need_eb` additionally requires equal error bounds. */
static int decode_pair(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                       int need_eb, layout* ga, layout* gb, int32_t** qa, int32_t** qb) {
  int rc = read_layout(a, a_bytes, ga);
  if (rc) return rc;
  rc = read_layout(b, b_bytes, gb);
  if (rc) return rc;
  if (need_eb ? !same_shape(ga, gb) : (ga->n != gb->n || ga->block != gb->block))
    return REF_ERR_MISMATCH;
  *qa = (int32_t*)malloc(ga->n * sizeof(int32_t));
  *qb = (int32_t*)malloc(gb->n * sizeof(int32_t));
  if (*qa == NULL || *qb == NULL) {
    free(*qa);
    free(*qb);
    *qa = *qb = NULL;
    return REF_ERR_ARG;
  }
  rc = hoszp_ref_decode_bins(a, a_bytes, *qa, ga->n);
  if (rc == REF_OK) rc = hoszp_ref_decode_bins(b, b_bytes, *qb, gb->n);
  if (rc) {
    free(*qa);
    free(*qb);
    *qa = *qb = NULL;
  }
  return rc;
}

/* Sec. V-C: element-wise subtraction, bins q_A - q_B re-encoded. */
int hoszp_ref_sub(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                  uint8_t* out, size_t out_cap, size_t* out_bytes) {
  if (out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  layout ga, gb;
  int32_t *qa, *qb;
  int rc = decode_pair(a, a_bytes, b, b_bytes, 1, &ga, &gb, &qa, &qb);
  if (rc) return rc;
  if (out_cap < hoszp_ref_bound(ga.n, ga.block)) rc = REF_ERR_CAPACITY;
  for (uint64_t i = 0; i < ga.n && rc == REF_OK; ++i) {
    int64_t v = (int64_t)qa[i] - (int64_t)qb[i];
    if (v < -BIN_MAX || v > BIN_MAX) rc = REF_ERR_RANGE;
    else qa[i] = (int32_t)v;
  }
  if (rc == REF_OK) rc = hoszp_ref_encode_bins(qa, ga.n, ga.eb, ga.block, out, out_cap, out_bytes);
  free(qa);
  free(qb);
  return rc;
}

/* floor(2 eps * p + 1/2) in exact arithmetic for an integer p (|p| < 2^62):
 * 2 eps = m * 2^e with an integer m (|m| < 2^53). */
static int exact_scaled_product(double two_eb, i128 p, int64_t* result) {
  int e2;
  double frac = frexp(two_eb, &e2);
  int64_t m = (int64_t)ldexp(frac, 53);
  int e = e2 - 53;
  i128 t = (i128)m * p; /* |t| < 2^115 */
  i128 r;
  if (t == 0) {
    r = 0;
  } else if (e >= 0) {
    if (e > 40) return REF_ERR_RANGE;
    r = t * ((i128)1 << e);
  } else if (-e > 120) {
    r = 0; /* |t 2^e| < 2^-5: rounds to 0 */
  } else {
    int sh = -e;
    i128 rnd = (i128)1 << (sh - 1); /* + 1/2 */
    i128 num = t + rnd;
    i128 quo = num / ((i128)1 << sh);
    if (num < 0 && quo * ((i128)1 << sh) != num) quo -= 1; /* floor */
    r = quo;
  }
  if (r < -(i128)BIN_MAX || r > (i128)BIN_MAX) return REF_ERR_RANGE;
  *result = (int64_t)r;
  return REF_OK;
}

/* Sec. V-C: Hadamard product.  The decoded values multiply to
 * (2 eps)^2 q_A q_B; re-quantized at eps with half-up rounding (as scalar
 * multiplication) that is floor(2 eps q_A q_B + 1/2). */
int hoszp_ref_hadamard(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                       uint8_t* out, size_t out_cap, size_t* out_bytes) {
  if (out == NULL || out_bytes == NULL) return REF_ERR_ARG;
  layout ga, gb;
  int32_t *qa, *qb;
  int rc = decode_pair(a, a_bytes, b, b_bytes, 1, &ga, &gb, &qa, &qb);
  if (rc) return rc;
  if (out_cap < hoszp_ref_bound(ga.n, ga.block)) rc = REF_ERR_CAPACITY;
  const double two_eb = 2.0 * ga.eb;
  for (uint64_t i = 0; i < ga.n && rc == REF_OK; ++i) {
    int64_t r;
    rc = exact_scaled_product(two_eb, (i128)qa[i] * (i128)qb[i], &r);
    if (rc == REF_OK) qa[i] = (int32_t)r;
  }
  if (rc == REF_OK) rc = hoszp_ref_encode_bins(qa, ga.n, ga.eb, ga.block, out, out_cap, out_bytes);
  free(qa);
  free(qb);
  return rc;
}

/* Sec. V-D: population covariance of the two decoded fields,
 * ((double)(n P - S_A S_B) / n / n) * (2 eps_A) (2 eps_B) with P = sum q_A q_B
 * and S = sum q, all exact.  The operands need equal n and block size; their
 * error bounds may differ. */
int hoszp_ref_covariance(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                         double* cov) {
  if (cov == NULL) return REF_ERR_ARG;
  layout ga, gb;
  int32_t *qa, *qb;
  int rc = decode_pair(a, a_bytes, b, b_bytes, 0, &ga, &gb, &qa, &qb);
  if (rc) return rc;
  i128 sa = 0, sb = 0, p = 0;
  for (uint64_t i = 0; i < ga.n; ++i) {
    sa += qa[i];
    sb += qb[i];
    p += (i128)qa[i] * (i128)qb[i];
  }
  /* |n P - S_A S_B| <= n sqrt(Q_A Q_B) < 2^126 (Cauchy-Schwarz) */
  i128 m = (i128)ga.n * p - sa * sb;
  *cov = (((double)m / (double)ga.n) / (double)ga.n) * ((2.0 * ga.eb) * (2.0 * gb.eb));
  free(qa);
  free(qb);
  return REF_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. V-B: block-wise means and constant blocks (Table VI)            */
/* ------------------------------------------------------------------ */

typedef struct {
  double* means;
  double two_eb;
  uint64_t constant;
  const uint8_t* widths;
} block_mean_sink;

static int store_block_mean(void* user, uint64_t b, uint32_t len, int32_t outlier,
                            const int64_t* d) {
  block_mean_sink* s = (block_mean_sink*)user;
  int64_t v = outlier, sum = 0;
  for (uint32_t k = 0; k < len; ++k) {
    if (k > 0) v += d[k];
    if (v < -BIN_MAX || v > BIN_MAX) return REF_ERR_FORMAT;
    sum += v;
  }
  s->means[b] = ((double)sum / (double)len) * s->two_eb;
  if (s->widths[b] == 0) s->constant += 1; /* width 0: every bin equals the outlier */
  return REF_OK;
}

/* means[b] = ((double)S_b / len_b) * 2 eps for every block b (S_b = exact sum
 * of the block's bins); *constant_blocks = blocks of width 0. */
int hoszp_ref_block_means(const uint8_t* c, size_t c_bytes, double* means, uint64_t nb_cap,
                          uint64_t* constant_blocks) {
  layout g;
  int rc = read_layout(c, c_bytes, &g);
  if (rc) return rc;
  if (means == NULL || constant_blocks == NULL) return REF_ERR_ARG;
  if (nb_cap < g.nb) return REF_ERR_CAPACITY;
  block_mean_sink s = {means, 2.0 * g.eb, 0, c + g.off_w};
  rc = for_each_block(c, &g, store_block_mean, &s);
  if (rc == REF_OK) *constant_blocks = s.constant;
  return rc;
}
