/*
 * hoszp_ref.h -- CPU oracle for the HoSZp compressed format and its
 * homomorphic operations (Agarwal et al., "HoSZp: An Efficient Homomorphic
 * Error-bounded Lossy Compressor for Scientific Data", arXiv 2408.11971).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * All pointers are host pointers.  Every function returns one of the
 * REF_* status codes below (0 = success); on failure output buffers hold
 * unspecified bytes.
 */
#ifndef HOSZP_REF_H
#define HOSZP_REF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (numeric values are part of the documented interface). */
#define REF_OK 0
#define REF_ERR_ARG 1       /* bad argument (eb <= 0, block size, n == 0 ...) */
#define REF_ERR_NONFINITE 2 /* NaN or Inf in the input field */
#define REF_ERR_RANGE 3     /* a quantization bin leaves [-(2^31-1), 2^31-1] */
#define REF_ERR_FORMAT 4    /* malformed or truncated compressed stream */
#define REF_ERR_MISMATCH 5  /* binary op on streams with different n/block/eb */
#define REF_ERR_CAPACITY 6  /* output buffer smaller than required */

/* Worst-case stream size for n elements in blocks of `block` (every block at
 * width 32); 0 when the arguments are invalid. */
size_t hoszp_ref_bound(uint64_t n, uint32_t block);

/* Quantization of Sec. IV-A step 1 (Eq. 3): q[i] = floor((x[i] + eb) / (2 eb)),
 * evaluated in binary64 as floor(((double)x + eb) * (1 / (2 eb))). */
int hoszp_ref_quantize(const float* x, uint64_t n, double eb, int32_t* q);

/* Full pipeline QZ -> LZ -> sign split -> BF (Sec. IV-A, Fig. 3 layout). */
int hoszp_ref_compress(const float* x, uint64_t n, double eb, uint32_t block,
                       uint8_t* out, size_t out_cap, size_t* out_bytes);

/* Same encoder applied to bins that are already quantized. */
int hoszp_ref_encode_bins(const int32_t* q, uint64_t n, double eb, uint32_t block,
                          uint8_t* out, size_t out_cap, size_t* out_bytes);

/* Header fields of a stream (validated like every decoder does). */
int hoszp_ref_info(const uint8_t* c, size_t c_bytes, uint64_t* n, uint32_t* block,
                   double* eb, uint64_t* payload_bytes, uint64_t* total_bytes);

/* Inverse of BF and LZ: the quantization bins of every element. */
int hoszp_ref_decode_bins(const uint8_t* c, size_t c_bytes, int32_t* q, uint64_t n_cap);

/* Full decompression: x[i] = (float)((double)q[i] * (2 eb)). */
int hoszp_ref_decompress(const uint8_t* c, size_t c_bytes, float* x, uint64_t n_cap);

/* Homomorphic negation (Sec. V-A-1; workflow 1). */
int hoszp_ref_negate(const uint8_t* c, size_t c_bytes, uint8_t* out, size_t out_cap,
                     size_t* out_bytes);

/* Homomorphic element-wise addition (Sec. V-C-1; workflow 2). */
int hoszp_ref_add(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                  uint8_t* out, size_t out_cap, size_t* out_bytes);

/* Homomorphic scalar multiplication (Sec. V-A-4; workflow 3):
 * q' = floor(s * q + 1/2) in exact arithmetic. */
int hoszp_ref_mul(const uint8_t* c, size_t c_bytes, double s, uint8_t* out,
                  size_t out_cap, size_t* out_bytes);

/* Exact integer aggregates of the bins: S = sum q (int64) and
 * Q = sum q^2 as an unsigned 128-bit value split into (lo, hi). */
int hoszp_ref_sums(const uint8_t* c, size_t c_bytes, int64_t* s, uint64_t* q_lo,
                   uint64_t* q_hi);

/* Homomorphic mean (Sec. V-B-1): ((double)S / (double)n) * (2 eb). */
int hoszp_ref_mean(const uint8_t* c, size_t c_bytes, double* mean);

/* Homomorphic population variance (Sec. V-B-2):
 * ((double)(n Q - S^2) / n / n) * ((2 eb) * (2 eb)). */
int hoszp_ref_variance(const uint8_t* c, size_t c_bytes, double* var);

/* Homomorphic scalar addition / subtraction (Sec. V-A; workflow 1): the
 * scalar's bin q_s by Eq. 3 is added to (subtracted from) every outlier;
 * widths, signs and magnitudes are copied.  RANGE if q_s or any result bin
 * leaves the bin range; out may equal c. */
int hoszp_ref_scalar_add(const uint8_t* c, size_t c_bytes, double s, uint8_t* out,
                         size_t out_cap, size_t* out_bytes);
int hoszp_ref_scalar_sub(const uint8_t* c, size_t c_bytes, double s, uint8_t* out,
                         size_t out_cap, size_t* out_bytes);

/* Standard deviation (Sec. V-B): sqrt of the population variance. */
int hoszp_ref_std(const uint8_t* c, size_t c_bytes, double* std);

/* Element-wise subtraction (Sec. V-C): bins q_A - q_B, canonical stream. */
int hoszp_ref_sub(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                  uint8_t* out, size_t out_cap, size_t* out_bytes);

/* Hadamard product (Sec. V-C): bins floor(2 eps q_A q_B + 1/2), exact. */
int hoszp_ref_hadamard(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                       uint8_t* out, size_t out_cap, size_t* out_bytes);

/* Population covariance (Sec. V-D) from exact integer sums; the operands
 * need equal n and block size (their error bounds may differ). */
int hoszp_ref_covariance(const uint8_t* a, size_t a_bytes, const uint8_t* b, size_t b_bytes,
                         double* cov);

/* Block-wise means (Sec. V-B): means[b] = ((double)S_b / len_b) * (2 eps),
 * and the number of constant (width 0) blocks. */
int hoszp_ref_block_means(const uint8_t* c, size_t c_bytes, double* means, uint64_t nb_cap,
                          uint64_t* constant_blocks);

#ifdef __cplusplus
}
#endif
#endif
