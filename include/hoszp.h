/*
 * hoszp.h -- C ABI of the MI355X (gfx950) HoSZp library.
 *
 * HoSZp (Agarwal et al., arXiv 2408.11971) is an error-bounded lossy
 * compressor whose compressed form supports arithmetic without full
 * decompression.  This library implements its data-parallel path on one GPU:
 *   compression        Sec. IV-A: quantization (Eq. 3), 1-D Lorenzo with the
 *                      block's first bin split off as the outlier (Eq. 4),
 *                      sign split, blockwise fixed-length bit packing, and the
 *                      section order of Fig. 3;
 *   decompression      the inverse of all steps (Fig. 2 caption);
 *   homomorphic ops    Sec. V / Table II: negation (workflow 1), element-wise
 *                      addition (workflow 2), scalar multiplication, mean and
 *                      variance (workflow 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - `d_*` arguments are device pointers owned by the caller (for instance a
 *   torch tensor's data pointer); the library never frees them and never keeps
 *   them after the call returns.  Host pointers are named `h_*` or are plain
 *   output scalars.
 * - `stream` is a hipStream_t passed as `void*` (NULL = the null stream).
 *   Every kernel of a call runs on that stream, in order.
 * - Return value: a HOSZP_* status code, 0 on success.  Synchronous calls
 *   (those with host outputs such as `out_bytes`, `mean`) block on `stream`
 *   and report errors the kernels detected; on any error the contents of the
 *   output buffers are unspecified.
 * - `*_async` variants only enqueue work.  They write their outcome into a
 *   caller-owned device record `hoszp_result` (status bit mask, output size,
 *   scalar result) and never synchronize, so they can be chained and captured
 *   in a hipGraph.  Arguments checkable on the host are still checked before
 *   anything is enqueued (the call then returns the error and enqueues
 *   nothing).
 * - A context owns the device scratch the kernels use (look-back status words,
 *   tile tickets, reduction accumulators).  Calls that share a context must not
 *   run concurrently (use one stream per context, or one context per stream).
 * - Streams are self-describing: the 64-byte header carries n, the block size
 *   and the error bound, so decoders take no shape arguments.
 * - Limits: 1 <= n <= 2^32 - 1 elements; block size 32, 64, 128 or 256; the error
 *   bound `eb` is absolute, finite and > 0; quantization bins must lie in
 *   [-(2^31 - 1), 2^31 - 1].  Float input pointers must be 16-byte aligned;
 *   stream pointers 16-byte aligned.
 *
 * Stream layout (little-endian)
 * -----------------------------
 *   header (64 B): "HOSZ", u16 version 1, u16 flags 0, u32 block, u32 0,
 *                  u64 n, f64 eb, u64 nb (= ceil(n / block)),
 *                  u64 payload_bytes, u64 total_bytes, u64 0
 *   W  nb bytes           width of every block (0 = constant block)
 *   O  4 nb bytes         outlier (first bin) of every block, int32
 *   S  nb block/8 bytes   sign bits, slot k of a block at bit 7-(k%8) of its
 *                         byte k/8; 1 = negative delta
 *   P  payload_bytes      every block's `block` magnitudes at the block's
 *                         width, most significant bit first, blocks in order
 *   Each section starts at the next 16-byte boundary; padding bytes are 0.
 */
#ifndef HOSZP_H
#define HOSZP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define HOSZP_OK 0
#define HOSZP_ERR_ARG 1       /* invalid argument (null pointer, eb <= 0, block, n, alignment) */
#define HOSZP_ERR_NONFINITE 2 /* NaN or Inf in the input field */
#define HOSZP_ERR_RANGE 3     /* a result bin leaves [-(2^31-1), 2^31-1] */
#define HOSZP_ERR_FORMAT 4    /* malformed, truncated or inconsistent stream */
#define HOSZP_ERR_MISMATCH 5  /* add: operands differ in n, block size or eb */
#define HOSZP_ERR_CAPACITY 6  /* output buffer too small */
#define HOSZP_ERR_DEVICE 7    /* a HIP runtime call failed */
#define HOSZP_ERR_NOMEM 8     /* device or pinned allocation failed */
#define HOSZP_ERR_LIMIT 9     /* input larger than an allocation-free entry point allows */
#define HOSZP_ERR_TIMEOUT 10  /* an encoder gave up waiting on its look-back (see hoszp_set_wait_limit) */

/* Outcome of an asynchronous call, written by the GPU into caller-owned
 * device memory (64 bytes, 8-byte aligned).
 *   status     bit (1 << code) set for every error the kernels detected;
 *              0 = success.  hoszp_status_code() picks the reported code.
 *   out_bytes  size of the produced stream (compress, negate, add, mul, ...).
 *   value      mean, variance or covariance (reductions; block means: the
 *              field's mean).
 *   count      block means: the number of constant (width 0) blocks. */
typedef struct hoszp_result {
  uint32_t status;
  uint32_t reserved0;
  uint64_t out_bytes;
  double value;
  uint64_t count;
  uint64_t reserved[4];
} hoszp_result;

/* Host-side view of a stream header. */
typedef struct hoszp_info {
  uint64_t n;
  uint32_t block;
  uint32_t version;
  double eb;
  uint64_t nb;
  uint64_t payload_bytes;
  uint64_t total_bytes;
} hoszp_info;

typedef struct hoszp_ctx hoszp_ctx;

/* Create a context on HIP device `device` (allocates its scratch, about
 * 22 MB of device memory plus one pinned host record).  Returns HOSZP_OK and
 * sets *out, or HOSZP_ERR_DEVICE / HOSZP_ERR_NOMEM. */
int hoszp_ctx_create(int device, hoszp_ctx** out);

/* Release a context (waits for nothing: the caller must have synchronized
 * every stream that used it). NULL is accepted. */
int hoszp_ctx_destroy(hoszp_ctx* ctx);

/* Bound the look-back waits of the encoders (compress, add, sub, mul,
 * Hadamard product, and batches created afterwards) launched on `ctx` from
 * now on.  An encoder tile finds its payload offset by waiting for the tiles
 * before it (a decoupled look-back, the device-wide form of the prefix sum of
 * block sizes that the byte layout of Sec. IV-A needs); a tile that polls its
 * predecessors `polls` times without finishing gives up, the launch still
 * drains, and its result reports HOSZP_ERR_TIMEOUT with the output invalid.
 * Predecessors are always running workgroups, so a correct call never comes
 * near the default (2^24 polls, seconds); the limit turns a wait that cannot
 * end (for instance overlapping calls that share scratch, which the
 * allocation-free entry point forbids) into an error instead of a hang.
 * 0 makes every tile but the first give up at once, which forces the error
 * path from the host.  Not thread-safe against calls enqueueing on `ctx`.
 * Returns HOSZP_OK, or HOSZP_ERR_ARG for a NULL context. */
int hoszp_set_wait_limit(hoszp_ctx* ctx, uint32_t polls);

/* Worst-case stream size for n elements (every block at width 32); 0 when n or
 * block is invalid.  Output buffers of compress/add/mul must be at least this
 * large. */
size_t hoszp_compress_bound(uint64_t n, uint32_t block);

/* Parse a stream header held in host memory (`header_bytes` >= 64).  Checks the
 * magic, version, block size, n, nb, eb and section sizes; the widths are not
 * visible here and are checked by the kernels. */
int hoszp_parse_header(const void* h_header, size_t header_bytes, hoszp_info* out);

/* Map a status bit mask (hoszp_result.status) to one code, by precedence
 * TIMEOUT, ARG, FORMAT, MISMATCH, CAPACITY, NONFINITE, RANGE. */
int hoszp_status_code(uint32_t status_mask);

/* Human-readable name of a status code. */
const char* hoszp_strerror(int code);

/* ---- compression (Sec. IV-A) ------------------------------------------- */

/* Compress n float32 values at absolute error bound eb with `block` elements
 * per block into d_out (capacity out_cap >= hoszp_compress_bound(n, block)).
 * *out_bytes receives the stream size.  Every decompressed value lies within
 * eb of its input (plus float32 rounding of the reconstruction). */
int hoszp_compress(hoszp_ctx* ctx, const float* d_x, uint64_t n, double eb, uint32_t block,
                   void* d_out, size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_compress_async(hoszp_ctx* ctx, const float* d_x, uint64_t n, double eb,
                         uint32_t block, void* d_out, size_t out_cap, hoszp_result* d_res,
                         void* stream);

/* The float inputs compress accepts at error bound eb: the interval
 * [*h_lo, *h_hi] of float32 values whose quantization bin (Eq. 3, evaluated
 * as the kernels do: floor(((double)x + eb) * (1 / (2 eb))) in binary64)
 * lies in [-(2^31-1), 2^31-1].  The bin is non-decreasing in x, so compress
 * reports RANGE exactly when some finite input is outside the interval (and
 * NONFINITE for NaN or infinity).  Both bounds are finite (0 is always
 * inside).  Returns ARG for eb <= 0, a non-finite eb or a NULL pointer, else
 * OK.  Host only; needs no device. */
int hoszp_bin_range(double eb, float* h_lo, float* h_hi);

/* Full decompression: d_x[i] = (float)((double)bin_i * 2 eb) for the stream's
 * n elements; n_cap is the capacity of d_x in elements (>= n). */
int hoszp_decompress(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, float* d_x,
                     uint64_t n_cap, void* stream);
int hoszp_decompress_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, float* d_x,
                           uint64_t n_cap, hoszp_result* d_res, void* stream);

/* ---- homomorphic operations (Sec. V) ----------------------------------- */

/* Negation (Sec. V-A-1, workflow 1): every outlier negated and, in every
 * non-constant block, the sign bits of its valid slots inverted; widths and
 * payload are copied.  out_cap >= the input's total size.  d_out may equal
 * d_c (in place); any other overlap of the two ranges gives ARG.  The decoded
 * result is exactly the negated field. */
int hoszp_negate(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, void* d_out, size_t out_cap,
                 size_t* out_bytes, void* stream);
int hoszp_negate_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, void* d_out,
                       size_t out_cap, hoszp_result* d_res, void* stream);

/* Element-wise addition (Sec. V-C-1, workflow 2): outliers added, signed
 * deltas added, then widths, signs and bits re-derived.  Both operands must
 * have the same n, block size and bitwise-equal eb (else MISMATCH); a sum bin
 * outside the bin range gives RANGE.  The output is the canonical stream of
 * the summed bins.  d_out must not overlap the inputs: a byte range
 * [d_out, d_out + out_cap) that meets either input gives ARG. */
int hoszp_add(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b, size_t b_bytes,
              void* d_out, size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_add_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                    size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                    void* stream);

/* Element-wise subtraction A - B (Sec. V-C, workflow 2): as hoszp_add with
 * B's outliers and signed deltas negated; the output is the canonical stream
 * of the bins q_A - q_B.  Same operand, capacity, range and overlap rules as
 * hoszp_add. */
int hoszp_sub(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b, size_t b_bytes,
              void* d_out, size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_sub_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                    size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                    void* stream);

/* Scalar addition / subtraction (Sec. V-A, workflow 1: fully compressed
 * space).  The scalar's bin q_s = floor((s + eb) * (1 / (2 eb))) (Eq. 3,
 * evaluated in binary64 like every element) is added to (subtracted from)
 * every outlier; widths, signs and magnitudes are copied unchanged, so every
 * decoded bin moves by +-q_s.  s must be finite (ARG); q_s or a shifted bin
 * outside the bin range gives RANGE.  out_cap >= the input's total size.
 * d_out may equal d_c (in place: only the outliers are rewritten); any other
 * overlap gives ARG.  A width pre-pass runs first: blocks whose outlier and
 * width cannot rule out an out-of-range bin are decoded to check exactly. */
int hoszp_scalar_add(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                     size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_scalar_add_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s,
                           void* d_out, size_t out_cap, hoszp_result* d_res, void* stream);
int hoszp_scalar_sub(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                     size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_scalar_sub_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s,
                           void* d_out, size_t out_cap, hoszp_result* d_res, void* stream);

/* Scalar multiplication (Sec. V-A-4, workflow 3): bins decoded, replaced by
 * floor(s * bin + 1/2) computed exactly, then re-encoded.  s must be finite;
 * a result outside the bin range gives RANGE.  d_out must not overlap d_c
 * ([d_out, d_out + out_cap) meeting [d_c, d_c + c_bytes) gives ARG). */
int hoszp_mul(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
              size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_mul_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                    size_t out_cap, hoszp_result* d_res, void* stream);

/* The scalar-multiplication rounding rule alone, on the host (Sec. V-A-4):
 * h_out[i] = floor(s * h_q[i] + 1/2) in exact arithmetic, computed by the
 * same function the kernels use.  h_q and h_out are n int32 values in host
 * memory (caller-owned, may be the same array).  Returns ARG for a
 * non-finite s or a NULL array with n > 0, RANGE when some result leaves
 * [-(2^31-1), 2^31-1] (that h_out[i] is then 0; the others are still
 * written), else OK.  Needs no device. */
int hoszp_mul_bins(double s, const int32_t* h_q, int32_t* h_out, uint64_t n);

/* Mean (Sec. V-B-1): ((double)S / n) * 2 eb with S the exact int64 sum of
 * the bins. */
int hoszp_mean(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* mean, void* stream);
int hoszp_mean_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, hoszp_result* d_res,
                     void* stream);

/* Population variance (Sec. V-B-2): ((double)(n Q - S^2) / n / n) * (2 eb)^2
 * with S and Q = sum of squared bins held exactly (128-bit). */
int hoszp_variance(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* var, void* stream);
int hoszp_variance_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, hoszp_result* d_res,
                         void* stream);

/* Hadamard product (Sec. V-C, workflow 3): both operands' bins decoded,
 * multiplied element by element and re-quantized at the same eb with half-up
 * rounding, exactly: q = floor(2 eb q_A q_B + 1/2) (the decoded product
 * (2 eb)^2 q_A q_B over the bin width 2 eb, rounded as scalar
 * multiplication rounds), then re-encoded canonically.  Operands as
 * hoszp_add (equal n, block size and eb bits, else MISMATCH); a product bin
 * outside the bin range gives RANGE; d_out must not overlap the inputs. */
int hoszp_hadamard(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                   size_t b_bytes, void* d_out, size_t out_cap, size_t* out_bytes, void* stream);
int hoszp_hadamard_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                         size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                         void* stream);

/* Population covariance of two decoded fields (Sec. V-D):
 * ((double)(n P - S_A S_B) / n / n) * (2 eb_A)(2 eb_B) with S = sum of bins
 * and P = sum q_A q_B held exactly (128-bit).  The operands need equal n and
 * block size (MISMATCH otherwise); their error bounds may differ.  The async
 * variant puts the value in d_res->value. */
int hoszp_covariance(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                     size_t b_bytes, double* cov, void* stream);
int hoszp_covariance_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                           size_t b_bytes, hoszp_result* d_res, void* stream);

/* Block-wise means (Sec. V-B: the mean kernel applied per block) and the
 * constant-block count (the statistic of Table VI): d_means[b] =
 * ((double)S_b / len_b) * 2 eb for every block b, S_b the exact sum of the
 * block's bins and len_b its length (the last block may be short);
 * *constant_blocks = blocks of width 0 (all bins equal).  d_means is a
 * caller-owned device array of means_cap >= nb doubles (8-byte aligned;
 * CAPACITY otherwise).  The async variant puts the count in d_res->count and
 * the field's mean in d_res->value. */
int hoszp_block_means(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* d_means,
                      uint64_t means_cap, uint64_t* constant_blocks, void* stream);
int hoszp_block_means_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* d_means,
                            uint64_t means_cap, hoszp_result* d_res, void* stream);

/* Standard deviation (Sec. V-B): the square root, taken on the host, of
 * hoszp_variance's result.  Synchronous only. */
int hoszp_std(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* std, void* stream);

/* ---- decompress-then-compute path (the comparison workflow) ------------ */

/* Float32 operations on decompressed fields, used to time the traditional
 * workflow (Sec. VI-B, Fig. 4a): y = -x, y = a + b, y = (float)(s * x),
 * y = a - b, y = (float)(x + s), y = a * b over n elements, and the float64
 * mean / population variance of x.  Results of the
 * reductions land in d_res->value. */
int hoszp_f32_negate_async(hoszp_ctx* ctx, const float* d_x, float* d_y, uint64_t n, void* stream);
int hoszp_f32_add_async(hoszp_ctx* ctx, const float* d_a, const float* d_b, float* d_y,
                        uint64_t n, void* stream);
int hoszp_f32_mul_async(hoszp_ctx* ctx, const float* d_x, double s, float* d_y, uint64_t n,
                        void* stream);
int hoszp_f32_sub_async(hoszp_ctx* ctx, const float* d_a, const float* d_b, float* d_y,
                        uint64_t n, void* stream);
int hoszp_f32_scalar_add_async(hoszp_ctx* ctx, const float* d_x, double s, float* d_y,
                               uint64_t n, void* stream);
int hoszp_f32_hadamard_async(hoszp_ctx* ctx, const float* d_a, const float* d_b, float* d_y,
                             uint64_t n, void* stream);
int hoszp_f32_mean_async(hoszp_ctx* ctx, const float* d_x, uint64_t n, hoszp_result* d_res,
                         void* stream);
int hoszp_f32_variance_async(hoszp_ctx* ctx, const float* d_x, uint64_t n, hoszp_result* d_res,
                             void* stream);

/* ---- batched compression with per-field statistics ---------------------
 *
 * Many fields of uneven sizes compressed in ONE persistent kernel launch,
 * captured once in a hipGraph and replayed by hoszp_batch_launch.  The tiles
 * of all fields form one work list; each field gets its own payload prefix
 * scan, its own stream (byte-identical to hoszp_compress of that field with
 * the same block size) and, from the same pass over its bins, the values
 * hoszp_mean and hoszp_variance would return for that stream (Sec. IV-A for
 * the stream, Sec. V-B for the reductions).
 *
 * An autotuner runs inside hoszp_batch_create:
 *   - block size, for every field whose `block` is 0: each of 32, 64, 128 is
 *     tried on the field's first min(n, 2^20) elements and the smallest
 *     stream wins (ties go to the larger block);
 *   - launch shape, with HOSZP_BATCH_TUNE_GRID: the whole batch is run with
 *     tiles of 1024 and of 512 segments (workgroup sizes), each at a few
 *     persistent grid sizes, and the fastest pair is kept.  The choice is
 *     remembered per batch shape (device compute units, field count, every
 *     field's n and block size) in a JSON Lines cache file, one object
 *     {"key", "threads", "grid", "ms"} per line, at $HOSZP_TUNE_CACHE (empty:
 *     no cache), else $XDG_CACHE_HOME/hoszp/batch_tune.jsonl, else
 *     ~/.cache/hoszp/batch_tune.jsonl; a plan of a known shape skips the
 *     timing runs.  Cache read or write failures are ignored.
 * The tuning runs the real kernels on the caller's data, so they write the
 * output buffers; the captured launch rewrites them. */

typedef struct hoszp_field {
  const float* d_x;  /* n float32 values, 16-byte aligned, caller-owned */
  uint64_t n;        /* 1 <= n <= 2^32 - 1 */
  double eb;         /* absolute error bound, finite and > 0 */
  uint32_t block;    /* 32, 64, 128, or 0 = chosen by the autotuner (a batch takes no 256) */
  uint32_t reserved; /* must be 0 */
  void* d_out;       /* output stream, 16-byte aligned, caller-owned */
  uint64_t out_cap;  /* >= hoszp_compress_bound(n, block); with block 0 the
                        largest bound over the three block sizes */
} hoszp_field;

/* Per-field outcome (64 bytes), written by the GPU. */
typedef struct hoszp_field_result {
  uint32_t status;    /* status bit mask as in hoszp_result (NONFINITE, RANGE) */
  uint32_t block;     /* block size the field was compressed with */
  uint64_t out_bytes; /* stream size */
  double mean;        /* = hoszp_mean of the stream (0 when status != 0) */
  double variance;    /* = hoszp_variance of the stream (0 when status != 0) */
  uint64_t reserved[4];
} hoszp_field_result;

typedef struct hoszp_batch_info {
  uint64_t fields;
  uint64_t total_tiles; /* work-list length (tiles of 32768 slots) */
  uint64_t raw_bytes;   /* sum of 4 n over the fields */
  uint64_t device_bytes;/* device memory the plan holds */
  uint32_t grid;        /* persistent workgroups per launch */
  uint32_t threads;     /* workgroup size = 32-element segments per work-list tile */
} hoszp_batch_info;

#define HOSZP_BATCH_TUNE_GRID 1u

typedef struct hoszp_batch hoszp_batch;

/* Plan a batch: check every field (ARG / CAPACITY, with *bad_field set to the
 * first offending index when bad_field is not NULL), run the autotuner on
 * `stream`, allocate the plan's device state (about 12 bytes per 32768 input
 * elements plus 192 bytes per field), and capture the launch.  The field
 * table is copied; the buffers it points to must stay valid while the plan
 * is used.  Synchronizes `stream`. */
int hoszp_batch_create(hoszp_ctx* ctx, const hoszp_field* fields, uint64_t count,
                       uint32_t flags, void* stream, hoszp_batch** out, uint64_t* bad_field);

/* Enqueue one replay of the captured launch on `stream` (never synchronizes).
 * Launches of one plan must not overlap in time (the plan owns one set of
 * counters); different plans and contexts may run concurrently. */
int hoszp_batch_launch(hoszp_batch* b, void* stream);

/* Wait for `stream` and copy the `count` per-field records of the last
 * completed launch to h_out.  Returns the code of the first failed field
 * (HOSZP_OK if none). */
int hoszp_batch_results(hoszp_batch* b, hoszp_field_result* h_out, void* stream);

/* Device address of the per-field records (count x 64 bytes), for callers
 * that consume them on the GPU. */
const hoszp_field_result* hoszp_batch_device_results(const hoszp_batch* b);

int hoszp_batch_info_get(const hoszp_batch* b, hoszp_batch_info* out);

/* Release a plan (the caller must have synchronized its launches). */
int hoszp_batch_destroy(hoszp_batch* b);

/* ---- serving: continuous batching of queries over a device store ------
 *
 * A server owns `slots` execution slots (each a context, a stream and a
 * result record) and a device memory pool of `pool_bytes`.  Queries on
 * caller-owned compressed streams are queued by hoszp_server_submit; each
 * hoszp_server_poll admits queued queries, oldest first, into free slots as
 * soon as the pool can hold their outputs and intermediates (a query that
 * does not fit may be passed by younger ones that do, unless it has waited
 * longer than the starvation limit), launches them on the slot's stream, so
 * admitted queries overlap on the device, and returns finished ones.  The
 * operations are those of Sec. V (Table II), on either path:
 *   HOSZP_PATH_HOMOMORPHIC   the homomorphic entry points above;
 *   HOSZP_PATH_TRADITIONAL   decompress, float32 op, re-compress (Fig. 4a),
 *                            the comparison workflow.
 * A query's result does not depend on what runs beside it: every slot has
 * its own scratch, and each kernel's result is a deterministic function of
 * its inputs. */

#define HOSZP_OP_MEAN 0u
#define HOSZP_OP_VARIANCE 1u
#define HOSZP_OP_NEGATE 2u
#define HOSZP_OP_ADD 3u
#define HOSZP_OP_MUL 4u
#define HOSZP_PATH_HOMOMORPHIC 0u
#define HOSZP_PATH_TRADITIONAL 1u

typedef struct hoszp_request {
  uint32_t op;          /* HOSZP_OP_* */
  uint32_t path;        /* HOSZP_PATH_* */
  const void* d_a;      /* compressed operand (caller-owned, stays valid until done) */
  uint64_t a_bytes;
  const void* d_b;      /* second operand of ADD (same n, block and eb), else NULL */
  uint64_t b_bytes;
  uint64_t n;           /* elements of the operands (from their headers) */
  uint32_t block;       /* block size of the operands */
  uint32_t reserved;    /* must be 0 */
  double eb;            /* error bound of the operands (re-compression of the
                           traditional path) */
  double scalar;        /* MUL */
  uint64_t tag;         /* caller's id, returned in the completion */
} hoszp_request;

typedef struct hoszp_completion {
  uint64_t tag;
  int32_t code;         /* HOSZP_OK or the query's error code */
  uint32_t op;
  double value;         /* MEAN / VARIANCE */
  void* d_out;          /* NEGATE / ADD / MUL: output stream in the server's
                           pool, valid until hoszp_server_release (NULL when
                           the server was told not to keep outputs) */
  uint64_t out_bytes;
  double submit_s;      /* host clock (seconds, server epoch): queued, */
  double admit_s;       /* launched, */
  double done_s;        /* and seen finished by a poll */
} hoszp_completion;

typedef struct hoszp_server_config {
  uint32_t slots;        /* concurrent queries on the device (1..64) */
  uint32_t keep_outputs; /* 1: completions own their output until released;
                            0: outputs are returned to the pool at completion */
  uint64_t pool_bytes;   /* device memory for outputs and intermediates */
  double starve_s;       /* a query older than this is never passed (0 = 0.05 s) */
} hoszp_server_config;

typedef struct hoszp_server_stats {
  uint64_t submitted, admitted, completed, failed;
  uint64_t pool_bytes, pool_peak;  /* pool size and its high-water mark */
  uint64_t queue_peak;             /* longest queue seen */
} hoszp_server_stats;

typedef struct hoszp_server hoszp_server;

/* Create a server on `device` (allocates the pool, one context, stream and
 * pinned result record per slot).  ARG for a bad config, NOMEM / DEVICE. */
int hoszp_server_create(int device, const hoszp_server_config* cfg, hoszp_server** out);

/* Queue a query (never blocks, launches nothing).  ARG for a malformed
 * query, CAPACITY if its memory need exceeds the whole pool. */
int hoszp_server_submit(hoszp_server* s, const hoszp_request* req);

/* Admit what fits, launch it, and return up to max_out finished queries
 * (*n_out of them).  Never blocks. */
int hoszp_server_poll(hoszp_server* s, hoszp_completion* out, uint32_t max_out, uint32_t* n_out);

/* Number of queries queued or running. */
uint64_t hoszp_server_pending(const hoszp_server* s);

/* Return a completed query's output stream to the pool. */
int hoszp_server_release(hoszp_server* s, void* d_out);

/* Open-loop replay: submit reqs[i] at arrival_s[i] seconds after the call
 * starts (non-decreasing), poll until every query has finished, and write
 * completion i for reqs[i] (out[i]).  The host thread spins between events.
 * Latency of query i = out[i].done_s - (start + arrival_s[i]); the call's
 * start is returned in *start_s on the same clock. */
int hoszp_server_replay(hoszp_server* s, const hoszp_request* reqs, const double* arrival_s,
                        uint64_t count, hoszp_completion* out, double* start_s);

int hoszp_server_stats_get(const hoszp_server* s, hoszp_server_stats* out);

/* Wait for every running query, then free everything (outputs still held by
 * completions are freed with the pool). */
int hoszp_server_destroy(hoszp_server* s);

/* ---- allocation-free compression ---------------------------------------
 *
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * compression as hoszp_compress_async (identical stream, same result record)
 * with no context.  Its scratch (tile ticket, counters, one look-back status
 * word per 32768-element tile) is a fixed 66 KB array in device global
 * memory that every device holds from its first call until the process ends;
 * the first call on a device looks up that array's address (nothing is
 * allocated, launched or synchronized then).  Each call clears the part of
 * the array it uses with a small kernel on `stream`, then enqueues the
 * compression; it never allocates, frees or synchronizes, so it can be
 * captured.  The device is the calling thread's current HIP device.
 *
 * Limits: 1 <= n <= HOSZP_NOALLOC_MAX_N (2^28 elements = 1 GiB of float32);
 * a larger n returns HOSZP_ERR_LIMIT and enqueues nothing.  Other arguments
 * and errors as hoszp_compress_async.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (two streams, two
 * threads) race and give undefined results; calls in one stream are ordered
 * and safe.  Concurrent use of hoszp_compress_async with a context is
 * unaffected. */
#define HOSZP_NOALLOC_MAX_N (1ull << 28)
int hoszp_compress_noalloc(const float* d_x, uint64_t n, double eb, uint32_t block, void* d_out,
                           size_t out_cap, hoszp_result* d_res, void* stream);

/* Block until `stream` is idle and return the code of a result record that
 * an async call filled (also copying it to *h_out when h_out is not NULL). */
int hoszp_result_wait(hoszp_ctx* ctx, const hoszp_result* d_res, hoszp_result* h_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
