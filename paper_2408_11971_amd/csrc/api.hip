// api.hip -- host side of the C ABI declared in include/hoszp.h.
//
// Every entry point validates what the host can see and enqueues the
// operation's kernels on the caller's stream; the operation's last kernel
// fills the result record and returns the context's counters to zero.
// Synchronous entry points then copy the 64-byte result record to pinned host
// memory and wait for the stream.

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <new>

#include "hoszp_internal.h"

struct hoszp_ctx {
  int device;
  hz::Scratch s;
  hz::Grids grids;
  void* d_mem;
  hoszp_result* d_res;  // record used by the synchronous entry points
  hoszp_result* h_res;  // pinned host mirror of d_res
};

struct hoszp_batch {
  int device;
  uint64_t count;
  hz::BatchDev dev;
  void* d_mem;
  uint64_t device_bytes;
  uint64_t raw_bytes;
  int grid;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

constexpr uint32_t kMaxTiles = uint32_t((hz::kMaxN + hz::kMinTileSegs * 32ull) / (hz::kMinTileSegs * 32ull) + 1);
constexpr uint32_t kMaxPart = 4096;

class DeviceScope {
 public:
  explicit DeviceScope(int dev) {
    ok_ = hipGetDevice(&prev_) == hipSuccess;
    if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess, switched_ = ok_;
  }
  ~DeviceScope() {
    if (switched_) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_ = 0;
  bool ok_ = false, switched_ = false;
};

inline bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Whether the byte ranges [a, a + na) and [b, b + nb) share a byte.  Add and
// mul write payload words of a tile before later tiles have read theirs, so
// an output that overlaps an input would corrupt the result.
inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return na && nb && pa < pb + nb && pb < pa + na;
}

int device_status(hipError_t e) { return e == hipSuccess ? HOSZP_OK : HOSZP_ERR_DEVICE; }

// Status of an operation's launches; a failed launch can leave the context
// counters mid-operation, so they are cleared before reporting the error.
int launched(hoszp_ctx* ctx, hoszp_result* d_res, hipStream_t st, hipError_t e) {
  if (e == hipSuccess) return HOSZP_OK;
  (void)hipGetLastError();
  (void)hz::launch_reset(ctx->s, d_res, st);
  return HOSZP_ERR_DEVICE;
}

int wait_result(hoszp_ctx* ctx, const hoszp_result* d_res, hoszp_result* h_out, hipStream_t st) {
  if (hipMemcpyAsync(ctx->h_res, d_res, sizeof(hoszp_result), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return HOSZP_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return HOSZP_ERR_DEVICE;
  if (h_out) *h_out = *ctx->h_res;
  return hoszp_status_code(ctx->h_res->status);
}

bool stream_args_ok(hoszp_ctx* ctx, const void* d_c, hoszp_result* d_res) {
  return ctx && d_c && d_res && aligned(d_c, 16) && aligned(d_res, 8);
}

// Classify the scalar s = m 2^e (|m| < 2^53): e < -100 (|s| < 2^-48) makes
// every result 0, and the kernels then multiply by an exact 0.
hz::MulScalar mul_split(double s) {
  hz::MulScalar k{s, 0, 0};
  int e2 = 0;
  const double frac = frexp(s, &e2);
  const int64_t m = int64_t(ldexp(frac, 53));
  const int e = e2 - 53;
  if (m == 0 || -e > 100) k.zero = 1;  // |s q| < 2^-16: every result rounds to 0
  return k;
}

}  // namespace

extern "C" {

int hoszp_status_code(uint32_t m) {
  // a launch that gave up on its look-back reports that first: the other
  // bits it latched may be consequences of the prefix it could not finish
  static const int order[] = {HOSZP_ERR_TIMEOUT, HOSZP_ERR_ARG, HOSZP_ERR_FORMAT,
                              HOSZP_ERR_MISMATCH, HOSZP_ERR_CAPACITY, HOSZP_ERR_NONFINITE,
                              HOSZP_ERR_RANGE};
  for (int code : order)
    if (m & (1u << code)) return code;
  return m ? HOSZP_ERR_DEVICE : HOSZP_OK;
}

const char* hoszp_strerror(int code) {
  switch (code) {
    case HOSZP_OK: return "ok";
    case HOSZP_ERR_ARG: return "invalid argument";
    case HOSZP_ERR_NONFINITE: return "non-finite input value";
    case HOSZP_ERR_RANGE: return "quantization bin out of range";
    case HOSZP_ERR_FORMAT: return "malformed compressed stream";
    case HOSZP_ERR_MISMATCH: return "operands differ in n, block size or error bound";
    case HOSZP_ERR_CAPACITY: return "output buffer too small";
    case HOSZP_ERR_DEVICE: return "HIP runtime error";
    case HOSZP_ERR_NOMEM: return "out of memory";
    case HOSZP_ERR_TIMEOUT: return "look-back wait exceeded the context's poll limit; output invalid";
    case HOSZP_ERR_LIMIT: return "input larger than the allocation-free entry point allows (n <= 2^28)";
    default: return "unknown status";
  }
}

size_t hoszp_compress_bound(uint64_t n, uint32_t block) {
  if (n == 0 || n > hz::kMaxN || !hz::block_ok(block)) return 0;
  return size_t(hz::bound_bytes(n, block));
}

int hoszp_parse_header(const void* h_header, size_t header_bytes, hoszp_info* out) {
  if (!h_header || !out) return HOSZP_ERR_ARG;
  if (header_bytes < hz::kHeaderBytes) return HOSZP_ERR_FORMAT;
  uint64_t h[8];
  memcpy(h, h_header, sizeof h);
  if (uint32_t(h[0]) != hz::kMagic || (h[0] >> 32) != 1u) return HOSZP_ERR_FORMAT;
  const uint32_t L = uint32_t(h[1]);
  double eb;
  memcpy(&eb, &h[3], 8);
  if (!hz::block_ok(L) || h[2] == 0 || h[2] > hz::kMaxN || !(eb > 0.0) || !isfinite(eb))
    return HOSZP_ERR_FORMAT;
  hz::Layout g;
  hz::place(g, h[2], L, eb);
  if (h[4] != g.nb || h[6] < g.off_p || h[6] - g.off_p != h[5] || (h[5] & 3u))
    return HOSZP_ERR_FORMAT;
  out->n = h[2];
  out->block = L;
  out->version = 1;
  out->eb = eb;
  out->nb = g.nb;
  out->payload_bytes = h[5];
  out->total_bytes = h[6];
  return HOSZP_OK;
}

int hoszp_ctx_create(int device, hoszp_ctx** out) {
  if (!out) return HOSZP_ERR_ARG;
  *out = nullptr;
  DeviceScope scope(device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return HOSZP_ERR_DEVICE;
  hoszp_ctx* ctx = new (std::nothrow) hoszp_ctx();
  if (!ctx) return HOSZP_ERR_NOMEM;
  ctx->device = device;
  if (hz::query_grids(ctx->grids, cus) != hipSuccess) {
    delete ctx;
    return HOSZP_ERR_DEVICE;
  }
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };  // every array 256-byte aligned
  const size_t max_wtiles = size_t(kMaxTiles) * (hz::kMinTileSegs / hz::kWaveSegs);
  const size_t nchunk = max_wtiles / hz::kChunkTiles + 2;
  const size_t ctrl_b = 256, acc_b = 256, part_b = up(size_t(kMaxPart) * sizeof(double));
  const size_t st_b = up(size_t(kMaxTiles) * sizeof(uint64_t));
  const size_t off_b = up(nchunk * sizeof(uint64_t)), tw_b = up(max_wtiles * sizeof(uint32_t));
  const size_t cw_b = up(nchunk * sizeof(uint32_t));
  const size_t idx_b = off_b + tw_b + cw_b;
  const size_t bytes = ctrl_b + acc_b + part_b + st_b + 2 * idx_b + up(sizeof(hoszp_result));
  if (hipMalloc(&ctx->d_mem, bytes) != hipSuccess) {
    delete ctx;
    return HOSZP_ERR_NOMEM;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->h_res), sizeof(hoszp_result),
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(ctx->d_mem);
    delete ctx;
    return HOSZP_ERR_NOMEM;
  }
  uint8_t* q = static_cast<uint8_t*>(ctx->d_mem);
  ctx->s.ctrl = reinterpret_cast<uint32_t*>(q);
  q += ctrl_b;
  ctx->s.acc = reinterpret_cast<uint64_t*>(q);
  q += acc_b;
  ctx->s.part = reinterpret_cast<double*>(q);
  q += part_b;
  ctx->s.st_out = reinterpret_cast<uint64_t*>(q);
  q += st_b;
  for (int k = 0; k < 2; ++k) {
    ctx->s.idx[k].chunk_off = reinterpret_cast<uint64_t*>(q);
    ctx->s.idx[k].tile_words = reinterpret_cast<uint32_t*>(q + off_b);
    ctx->s.idx[k].chunk_words = reinterpret_cast<uint32_t*>(q + off_b + tw_b);
    q += idx_b;
  }
  ctx->d_res = reinterpret_cast<hoszp_result*>(q);
  ctx->s.max_tiles = kMaxTiles;
  ctx->s.max_part = kMaxPart;
  ctx->s.wait_limit = hz::kDefaultWaitLimit;
  if (hipMemset(ctx->d_mem, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipHostFree(ctx->h_res);
    (void)hipFree(ctx->d_mem);
    delete ctx;
    return HOSZP_ERR_DEVICE;
  }
  *out = ctx;
  return HOSZP_OK;
}

int hoszp_ctx_destroy(hoszp_ctx* ctx) {
  if (!ctx) return HOSZP_OK;
  DeviceScope scope(ctx->device);
  int rc = HOSZP_OK;
  if (hipHostFree(ctx->h_res) != hipSuccess) rc = HOSZP_ERR_DEVICE;
  if (hipFree(ctx->d_mem) != hipSuccess) rc = HOSZP_ERR_DEVICE;
  delete ctx;
  return rc;
}

int hoszp_set_wait_limit(hoszp_ctx* ctx, uint32_t polls) {
  if (!ctx) return HOSZP_ERR_ARG;
  ctx->s.wait_limit = polls;
  return HOSZP_OK;
}

int hoszp_result_wait(hoszp_ctx* ctx, const hoszp_result* d_res, hoszp_result* h_out,
                      void* stream) {
  if (!ctx || !d_res) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  return wait_result(ctx, d_res, h_out, static_cast<hipStream_t>(stream));
}

// ---- compression --------------------------------------------------------

int hoszp_compress_async(hoszp_ctx* ctx, const float* d_x, uint64_t n, double eb,
                         uint32_t block, void* d_out, size_t out_cap, hoszp_result* d_res,
                         void* stream) {
  if (!ctx || !d_x || !d_out || !d_res || !aligned(d_x, 16) || !aligned(d_out, 16) ||
      !aligned(d_res, 8))
    return HOSZP_ERR_ARG;
  if (n == 0 || n > hz::kMaxN || !hz::block_ok(block) || !(eb > 0.0) || !isfinite(eb))
    return HOSZP_ERR_ARG;
  if (out_cap < hz::bound_bytes(n, block)) return HOSZP_ERR_CAPACITY;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hz::Layout g;
  hz::place(g, n, block, eb);
  const double inv2e = 1.0 / (2.0 * eb);
  return launched(ctx, d_res, st, hz::launch_compress(ctx->s, ctx->grids, d_x, g, inv2e,
                                           static_cast<uint8_t*>(d_out), d_res, st));
}

int hoszp_compress(hoszp_ctx* ctx, const float* d_x, uint64_t n, double eb, uint32_t block,
                   void* d_out, size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  int rc = hoszp_compress_async(ctx, d_x, n, eb, block, d_out, out_cap, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *out_bytes = size_t(r.out_bytes);
  return rc;
}

int hoszp_decompress_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, float* d_x,
                           uint64_t n_cap, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res) || !d_x || !aligned(d_x, 16)) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_decompress(ctx->s, ctx->grids,
                                             static_cast<const uint8_t*>(d_c), c_bytes, d_x,
                                             n_cap, d_res, st));
}

int hoszp_decompress(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, float* d_x,
                     uint64_t n_cap, void* stream) {
  if (!ctx) return HOSZP_ERR_ARG;
  int rc = hoszp_decompress_async(ctx, d_c, c_bytes, d_x, n_cap, ctx->d_res, stream);
  if (rc) return rc;
  return hoszp_result_wait(ctx, ctx->d_res, nullptr, stream);
}

// ---- homomorphic operations ---------------------------------------------

int hoszp_negate_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, void* d_out,
                       size_t out_cap, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res) || !d_out || !aligned(d_out, 16) ||
      (d_out != d_c && overlap(d_out, out_cap, d_c, c_bytes)))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_negate(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_c),
                                         c_bytes, static_cast<uint8_t*>(d_out), out_cap, d_res,
                                         st));
}

int hoszp_negate(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, void* d_out, size_t out_cap,
                 size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  int rc = hoszp_negate_async(ctx, d_c, c_bytes, d_out, out_cap, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *out_bytes = size_t(r.out_bytes);
  return rc;
}

static int add_like(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                    size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                    void* stream, bool sub) {
  if (!stream_args_ok(ctx, d_a, d_res) || !d_b || !aligned(d_b, 16) || !d_out ||
      !aligned(d_out, 16) || overlap(d_out, out_cap, d_a, a_bytes) ||
      overlap(d_out, out_cap, d_b, b_bytes))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_add(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_a),
                                      a_bytes, static_cast<const uint8_t*>(d_b), b_bytes,
                                      static_cast<uint8_t*>(d_out), out_cap, d_res, st,
                                      sub));
}

// Wait for a stream-producing operation enqueued on ctx->d_res.
static int wait_stream_op(hoszp_ctx* ctx, int rc, size_t* out_bytes, void* stream) {
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *out_bytes = size_t(r.out_bytes);
  return rc;
}

int hoszp_add_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                    size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                    void* stream) {
  return add_like(ctx, d_a, a_bytes, d_b, b_bytes, d_out, out_cap, d_res, stream, false);
}

int hoszp_add(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b, size_t b_bytes,
              void* d_out, size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  return wait_stream_op(ctx, hoszp_add_async(ctx, d_a, a_bytes, d_b, b_bytes, d_out, out_cap,
                                             ctx->d_res, stream), out_bytes, stream);
}

int hoszp_sub_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                    size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                    void* stream) {
  return add_like(ctx, d_a, a_bytes, d_b, b_bytes, d_out, out_cap, d_res, stream, true);
}

int hoszp_sub(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b, size_t b_bytes,
              void* d_out, size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  return wait_stream_op(ctx, hoszp_sub_async(ctx, d_a, a_bytes, d_b, b_bytes, d_out, out_cap,
                                             ctx->d_res, stream), out_bytes, stream);
}

static int shift_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, int sign,
                       void* d_out, size_t out_cap, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res) || !d_out || !aligned(d_out, 16) || !isfinite(s) ||
      (d_out != d_c && overlap(d_out, out_cap, d_c, c_bytes)))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_shift(ctx->s, ctx->grids,
                                        static_cast<const uint8_t*>(d_c), c_bytes, s, sign,
                                        static_cast<uint8_t*>(d_out), out_cap, d_res, st));
}

int hoszp_scalar_add_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s,
                           void* d_out, size_t out_cap, hoszp_result* d_res, void* stream) {
  return shift_async(ctx, d_c, c_bytes, s, 1, d_out, out_cap, d_res, stream);
}

int hoszp_scalar_sub_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s,
                           void* d_out, size_t out_cap, hoszp_result* d_res, void* stream) {
  return shift_async(ctx, d_c, c_bytes, s, -1, d_out, out_cap, d_res, stream);
}

int hoszp_scalar_add(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                     size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  return wait_stream_op(ctx, shift_async(ctx, d_c, c_bytes, s, 1, d_out, out_cap, ctx->d_res,
                                         stream), out_bytes, stream);
}

int hoszp_scalar_sub(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                     size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  return wait_stream_op(ctx, shift_async(ctx, d_c, c_bytes, s, -1, d_out, out_cap, ctx->d_res,
                                         stream), out_bytes, stream);
}

int hoszp_mul_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                    size_t out_cap, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res) || !d_out || !aligned(d_out, 16) || !isfinite(s) ||
      overlap(d_out, out_cap, d_c, c_bytes))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_mul(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_c),
                                      c_bytes, mul_split(s), static_cast<uint8_t*>(d_out),
                                      out_cap, d_res, st));
}

int hoszp_mul(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
              size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  int rc = hoszp_mul_async(ctx, d_c, c_bytes, s, d_out, out_cap, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *out_bytes = size_t(r.out_bytes);
  return rc;
}

int hoszp_bin_range(double eb, float* h_lo, float* h_hi) {
  if (!h_lo || !h_hi || !(eb > 0.0) || !isfinite(eb)) return HOSZP_ERR_ARG;
  hz::bin_range_floats(eb, 1.0 / (2.0 * eb), *h_lo, *h_hi);
  return HOSZP_OK;
}

int hoszp_mul_bins(double s, const int32_t* h_q, int32_t* h_out, uint64_t n) {
  if ((n && (!h_q || !h_out)) || !isfinite(s)) return HOSZP_ERR_ARG;
  const double sc = mul_split(s).zero ? 0.0 : s;
  int rc = HOSZP_OK;
  for (uint64_t i = 0; i < n; ++i) {
    const double f = hz::mul_round(sc, double(h_q[i]));
    const bool ok = fabs(f) <= double(hz::kBinMax);
    h_out[i] = ok ? int32_t(f) : 0;
    if (!ok) rc = HOSZP_ERR_RANGE;
  }
  return rc;
}

static int reduce_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, bool variance,
                        hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res)) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_reduce(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_c),
                                         c_bytes, variance, d_res, st));
}

int hoszp_mean_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, hoszp_result* d_res,
                     void* stream) {
  return reduce_async(ctx, d_c, c_bytes, false, d_res, stream);
}

int hoszp_variance_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, hoszp_result* d_res,
                         void* stream) {
  return reduce_async(ctx, d_c, c_bytes, true, d_res, stream);
}

int hoszp_mean(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* mean, void* stream) {
  if (!ctx || !mean) return HOSZP_ERR_ARG;
  int rc = hoszp_mean_async(ctx, d_c, c_bytes, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *mean = r.value;
  return rc;
}

int hoszp_variance(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* var, void* stream) {
  if (!ctx || !var) return HOSZP_ERR_ARG;
  int rc = hoszp_variance_async(ctx, d_c, c_bytes, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *var = r.value;
  return rc;
}

int hoszp_hadamard_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                         size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                         void* stream) {
  if (!stream_args_ok(ctx, d_a, d_res) || !d_b || !aligned(d_b, 16) || !d_out ||
      !aligned(d_out, 16) || overlap(d_out, out_cap, d_a, a_bytes) ||
      overlap(d_out, out_cap, d_b, b_bytes))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_bivar(ctx->s, ctx->grids, false,
                                        static_cast<const uint8_t*>(d_a), a_bytes,
                                        static_cast<const uint8_t*>(d_b), b_bytes,
                                        static_cast<uint8_t*>(d_out), out_cap, d_res, st));
}

int hoszp_hadamard(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                   size_t b_bytes, void* d_out, size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  return wait_stream_op(ctx, hoszp_hadamard_async(ctx, d_a, a_bytes, d_b, b_bytes, d_out, out_cap,
                                                  ctx->d_res, stream), out_bytes, stream);
}

int hoszp_covariance_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                           size_t b_bytes, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_a, d_res) || !d_b || !aligned(d_b, 16)) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_bivar(ctx->s, ctx->grids, true,
                                        static_cast<const uint8_t*>(d_a), a_bytes,
                                        static_cast<const uint8_t*>(d_b), b_bytes, nullptr, 0,
                                        d_res, st));
}

int hoszp_covariance(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                     size_t b_bytes, double* cov, void* stream) {
  if (!ctx || !cov) return HOSZP_ERR_ARG;
  int rc = hoszp_covariance_async(ctx, d_a, a_bytes, d_b, b_bytes, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *cov = r.value;
  return rc;
}

int hoszp_block_means_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* d_means,
                            uint64_t means_cap, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res) || !d_means || !aligned(d_means, 8)) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_block_means(ctx->s, ctx->grids,
                                              static_cast<const uint8_t*>(d_c), c_bytes,
                                              d_means, means_cap, d_res, st));
}

int hoszp_block_means(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* d_means,
                      uint64_t means_cap, uint64_t* constant_blocks, void* stream) {
  if (!ctx || !constant_blocks) return HOSZP_ERR_ARG;
  int rc = hoszp_block_means_async(ctx, d_c, c_bytes, d_means, means_cap, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *constant_blocks = r.count;
  return rc;
}

int hoszp_std(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double* std, void* stream) {
  if (!ctx || !std) return HOSZP_ERR_ARG;
  double var = 0.0;
  const int rc = hoszp_variance(ctx, d_c, c_bytes, &var, stream);
  if (rc == HOSZP_OK) *std = sqrt(var);  // correctly rounded (IEEE sqrt on the host)
  return rc;
}

// ---- float32 workflow ops -----------------------------------------------

static int f32_map(hoszp_ctx* ctx, int op, const float* x, const float* y, double s, float* out,
                   uint64_t n, void* stream) {
  const bool two = op == 1 || op == 3 || op == 5;
  if (!ctx || !x || !out || (two && !y) || n == 0 || !aligned(x, 16) || !aligned(out, 16) ||
      (y && !aligned(y, 16)))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  return device_status(
      hz::launch_f32_unary(ctx->grids, op, x, y, s, out, n, static_cast<hipStream_t>(stream)));
}

int hoszp_f32_negate_async(hoszp_ctx* ctx, const float* d_x, float* d_y, uint64_t n,
                           void* stream) {
  return f32_map(ctx, 0, d_x, nullptr, 0.0, d_y, n, stream);
}

int hoszp_f32_add_async(hoszp_ctx* ctx, const float* d_a, const float* d_b, float* d_y,
                        uint64_t n, void* stream) {
  return f32_map(ctx, 1, d_a, d_b, 0.0, d_y, n, stream);
}

int hoszp_f32_mul_async(hoszp_ctx* ctx, const float* d_x, double s, float* d_y, uint64_t n,
                        void* stream) {
  return f32_map(ctx, 2, d_x, nullptr, s, d_y, n, stream);
}

int hoszp_f32_sub_async(hoszp_ctx* ctx, const float* d_a, const float* d_b, float* d_y,
                        uint64_t n, void* stream) {
  return f32_map(ctx, 3, d_a, d_b, 0.0, d_y, n, stream);
}

int hoszp_f32_scalar_add_async(hoszp_ctx* ctx, const float* d_x, double s, float* d_y,
                               uint64_t n, void* stream) {
  return f32_map(ctx, 4, d_x, nullptr, s, d_y, n, stream);
}

int hoszp_f32_hadamard_async(hoszp_ctx* ctx, const float* d_a, const float* d_b, float* d_y,
                             uint64_t n, void* stream) {
  return f32_map(ctx, 5, d_a, d_b, 0.0, d_y, n, stream);
}

static int f32_reduce(hoszp_ctx* ctx, const float* x, uint64_t n, bool variance,
                      hoszp_result* d_res, void* stream) {
  if (!ctx || !x || !d_res || n == 0 || !aligned(x, 16) || !aligned(d_res, 8)) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launched(ctx, d_res, st, hz::launch_f32_reduce(ctx->s, ctx->grids, x, n, variance, d_res, st));
}

int hoszp_f32_mean_async(hoszp_ctx* ctx, const float* d_x, uint64_t n, hoszp_result* d_res,
                         void* stream) {
  return f32_reduce(ctx, d_x, n, false, d_res, stream);
}

int hoszp_f32_variance_async(hoszp_ctx* ctx, const float* d_x, uint64_t n, hoszp_result* d_res,
                             void* stream) {
  return f32_reduce(ctx, d_x, n, true, d_res, stream);
}

// ---- batched compression ------------------------------------------------

namespace {

constexpr uint64_t kTuneSample = uint64_t(1) << 20;
const uint32_t kBlocks[3] = {32, 64, 128};

uint64_t field_cap_needed(const hoszp_field& f) {
  if (f.block) return hz::bound_bytes(f.n, f.block);
  uint64_t m = 0;
  for (uint32_t L : kBlocks) m = hz::bound_bytes(f.n, L) > m ? hz::bound_bytes(f.n, L) : m;
  return m;
}

int check_field(const hoszp_field& f) {
  if (!f.d_x || !f.d_out || !aligned(f.d_x, 16) || !aligned(f.d_out, 16) || f.reserved) return HOSZP_ERR_ARG;
  if (f.n == 0 || f.n > hz::kMaxN || !(f.eb > 0.0) || !isfinite(f.eb)) return HOSZP_ERR_ARG;
  // batches take blocks up to 128: a fourth tile body in the batch kernel
  // measurably slows the common block sizes
  if (f.block && (!hz::block_ok(f.block) || f.block > 128)) return HOSZP_ERR_ARG;
  if (f.out_cap < field_cap_needed(f)) return HOSZP_ERR_CAPACITY;
  return HOSZP_OK;
}

// Block size of every field whose block is 0: the smallest stream of the
// field's first min(n, kTuneSample) elements over the three block sizes.
int tune_blocks(hoszp_ctx* ctx, const hoszp_field* fields, uint64_t count, uint32_t* blocks,
                hipStream_t st) {
  uint64_t auto_n = 0;
  for (uint64_t i = 0; i < count; ++i) auto_n += fields[i].block == 0;
  for (uint64_t i = 0; i < count; ++i) blocks[i] = fields[i].block ? fields[i].block : 32;
  if (auto_n == 0) return HOSZP_OK;
  hoszp_result* d_r = nullptr;
  const size_t rb = size_t(auto_n) * 3 * sizeof(hoszp_result);
  if (hipMalloc(&d_r, rb) != hipSuccess) return HOSZP_ERR_NOMEM;
  int rc = HOSZP_OK;
  uint64_t k = 0;
  for (uint64_t i = 0; i < count && rc == HOSZP_OK; ++i) {
    const hoszp_field& f = fields[i];
    if (f.block) continue;
    const uint64_t m = f.n < kTuneSample ? f.n : kTuneSample;
    for (int j = 0; j < 3 && rc == HOSZP_OK; ++j)
      rc = hoszp_compress_async(ctx, f.d_x, m, f.eb, kBlocks[j], f.d_out, size_t(f.out_cap),
                                d_r + 3 * k + j, st);
    ++k;
  }
  hoszp_result* h_r = nullptr;
  if (rc == HOSZP_OK && !(h_r = new (std::nothrow) hoszp_result[auto_n * 3])) rc = HOSZP_ERR_NOMEM;
  if (rc == HOSZP_OK && (hipMemcpyAsync(h_r, d_r, rb, hipMemcpyDeviceToHost, st) != hipSuccess ||
                         hipStreamSynchronize(st) != hipSuccess))
    rc = HOSZP_ERR_DEVICE;
  if (rc == HOSZP_OK) {
    k = 0;
    for (uint64_t i = 0; i < count; ++i) {
      if (fields[i].block) continue;
      uint32_t best = 32;
      uint64_t best_bytes = ~uint64_t(0);
      for (int j = 0; j < 3; ++j) {
        const hoszp_result& r = h_r[3 * k + j];
        if (r.status == 0 && r.out_bytes <= best_bytes) best_bytes = r.out_bytes, best = kBlocks[j];
      }
      blocks[i] = best;  // a field that fails at every size keeps 32 and reports at launch
      ++k;
    }
  }
  delete[] h_r;
  (void)hipFree(d_r);
  return rc;
}

void batch_free(hoszp_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_mem) (void)hipFree(b->d_mem);
  delete b;
}

// Time one launch of the batch at `grid` workgroups (milliseconds).
int time_grid(hoszp_batch* b, int grid, hipStream_t st, float* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return HOSZP_ERR_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HOSZP_ERR_DEVICE;
  }
  int rc = HOSZP_OK;
  if (hz::launch_batch(b->dev, grid, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess ||
      hz::launch_batch(b->dev, grid, st) != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
      hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
    rc = HOSZP_ERR_DEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// Device state of a plan with tiles of `nt` segments (replacing any earlier
// one): the field table, the work list (the field of every tile), zeroed
// status words, counters and accumulators, look-back generation 1.
int build_plan(hoszp_batch* b, const hoszp_field* fields, const uint32_t* blocks, uint64_t count,
               uint32_t nt, hipStream_t st) {
  if (b->d_mem) {
    if (hipStreamSynchronize(st) != hipSuccess) return HOSZP_ERR_DEVICE;
    (void)hipFree(b->d_mem);
    b->d_mem = nullptr;
  }
  hz::BatchField* hf = new (std::nothrow) hz::BatchField[count];
  if (!hf) return HOSZP_ERR_NOMEM;
  uint64_t tiles = 0, raw = 0;
  for (uint64_t i = 0; i < count; ++i) {
    hz::Layout g;
    hz::place(g, fields[i].n, blocks[i], fields[i].eb);
    const double inv2e = 1.0 / (2.0 * fields[i].eb);
    hf[i] = hz::BatchField{fields[i].d_x, static_cast<uint8_t*>(fields[i].d_out), fields[i].n,
                           fields[i].eb, inv2e, tiles, blocks[i],
                           hz::abs_bound(fields[i].eb, inv2e),
                           hz::abs_bound(fields[i].eb, inv2e, hz::kSmallBin), 0};
    tiles += hz::batch_tiles(g, nt);
    raw += 4 * fields[i].n;
  }
  b->raw_bytes = raw;
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t f_b = up(count * sizeof(hz::BatchField)), tf_b = up(tiles * sizeof(uint32_t));
  const size_t st_b = up(tiles * sizeof(uint64_t)), ctrl_b = 256;
  const size_t acc_b = up(count * hz::kBatchAccWords * sizeof(uint64_t));
  const size_t res_b = up(count * sizeof(hoszp_field_result));
  b->device_bytes = f_b + tf_b + st_b + ctrl_b + acc_b + res_b;
  int rc = HOSZP_OK;
  if (hipMalloc(&b->d_mem, b->device_bytes) != hipSuccess) {
    b->d_mem = nullptr;
    rc = HOSZP_ERR_NOMEM;
  }
  uint32_t* tf = nullptr;
  if (rc == HOSZP_OK) {
    uint8_t* q = static_cast<uint8_t*>(b->d_mem);
    b->dev.fields = reinterpret_cast<hz::BatchField*>(q);
    b->dev.tile_field = reinterpret_cast<uint32_t*>(q + f_b);
    b->dev.st = reinterpret_cast<uint64_t*>(q + f_b + tf_b);
    b->dev.ctrl = reinterpret_cast<uint32_t*>(q + f_b + tf_b + st_b);
    b->dev.facc = reinterpret_cast<uint64_t*>(q + f_b + tf_b + st_b + ctrl_b);
    b->dev.res = reinterpret_cast<hoszp_field_result*>(q + f_b + tf_b + st_b + ctrl_b + acc_b);
    b->dev.total_tiles = tiles;
    b->dev.threads = nt;
    tf = new (std::nothrow) uint32_t[tiles];
    if (!tf) rc = HOSZP_ERR_NOMEM;
  }
  if (rc == HOSZP_OK) {
    uint64_t t = 0;
    for (uint64_t i = 0; i < count; ++i) {
      hz::Layout g;
      hz::place(g, hf[i].n, hf[i].block, hf[i].eb);
      for (uint64_t k = 0; k < hz::batch_tiles(g, nt); ++k) tf[t++] = uint32_t(i);
    }
    const uint32_t epoch1 = 1;
    if (hipMemsetAsync(b->d_mem, 0, b->device_bytes, st) != hipSuccess ||
        hipMemcpyAsync(b->dev.fields, hf, count * sizeof(hz::BatchField), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(const_cast<uint32_t*>(b->dev.tile_field), tf, tiles * sizeof(uint32_t),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->dev.ctrl + 2, &epoch1, sizeof epoch1, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = HOSZP_ERR_DEVICE;
  }
  delete[] tf;
  delete[] hf;
  return rc;
}

// ---- tuning cache -----------------------------------------------------------
//
// The launch shape a tuned plan chose (tile threads and grid), remembered per
// batch shape so that a later plan of the same shape skips the timing runs.
// A JSON Lines file, one object per tuned shape:
//   {"key": "<16 hex digits>", "threads": 1024, "grid": 512, "ms": 16.8}
// at $HOSZP_TUNE_CACHE (an empty value disables the cache), else
// $XDG_CACHE_HOME/hoszp/batch_tune.jsonl, else ~/.cache/hoszp/batch_tune.jsonl.
// Later lines win; unreadable or malformed lines are ignored, and failure to
// write is not an error.

struct TuneChoice {
  uint32_t threads;
  int grid;
  float ms;
};

// FNV-1a over the plan's shape: compute units, field count, every field's n
// and block size, and a format tag.
uint64_t batch_signature(const hoszp_field* fields, const uint32_t* blocks, uint64_t count,
                         int cus) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix(0x484f535a42415431ull);  // "HOSZBAT1"
  mix(uint64_t(cus));
  mix(count);
  for (uint64_t i = 0; i < count; ++i) {
    mix(fields[i].n);
    mix(blocks[i]);
  }
  return h;
}

bool tune_cache_path(char* path, size_t cap) {
  const char* env = getenv("HOSZP_TUNE_CACHE");
  if (env) {
    if (!*env || strlen(env) + 1 > cap) return false;
    strcpy(path, env);
    return true;
  }
  const char* xdg = getenv("XDG_CACHE_HOME");
  const char* home = getenv("HOME");
  char dir[3072];
  if (xdg && *xdg) {
    if (snprintf(dir, sizeof dir, "%s/hoszp", xdg) >= int(sizeof dir)) return false;
  } else if (home && *home) {
    if (snprintf(dir, sizeof dir, "%s/.cache/hoszp", home) >= int(sizeof dir)) return false;
  } else {
    return false;
  }
  return snprintf(path, cap, "%s/batch_tune.jsonl", dir) < int(cap);
}

bool tune_cache_lookup(uint64_t key, TuneChoice* out) {
  char path[4096];
  if (!tune_cache_path(path, sizeof path)) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    unsigned long long k = 0;
    unsigned threads = 0;
    int grid = 0;
    float ms = 0.f;
    if (sscanf(line, " {\"key\": \"%16llx\", \"threads\": %u, \"grid\": %d, \"ms\": %f",
               &k, &threads, &grid, &ms) == 4 &&
        k == key && grid > 0 &&
        (threads == uint32_t(hz::kBatchThreads) || threads == uint32_t(hz::kBatchThreadsSmall))) {
      *out = TuneChoice{threads, grid, ms};
      found = true;
    }
  }
  fclose(f);
  return found;
}

void tune_cache_store(uint64_t key, const TuneChoice& c) {
  char path[4096];
  if (!tune_cache_path(path, sizeof path)) return;
  // create the directory chain below the file (one or two missing levels)
  char dir[4096];
  strcpy(dir, path);
  for (char* p = dir + 1; *p; ++p) {
    if (*p != '/') continue;
    *p = 0;
    (void)mkdir(dir, 0755);
    *p = '/';
  }
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%016llx\", \"threads\": %u, \"grid\": %d, \"ms\": %.4f}\n",
          (unsigned long long)key, c.threads, c.grid, double(c.ms));
  fclose(f);
}

}  // namespace

int hoszp_batch_create(hoszp_ctx* ctx, const hoszp_field* fields, uint64_t count, uint32_t flags,
                       void* stream, hoszp_batch** out, uint64_t* bad_field) {
  if (!out) return HOSZP_ERR_ARG;
  *out = nullptr;
  if (!ctx || !fields || count == 0 || count > 0xffffffffull || (flags & ~HOSZP_BATCH_TUNE_GRID))
    return HOSZP_ERR_ARG;
  for (uint64_t i = 0; i < count; ++i) {
    const int rc = check_field(fields[i]);
    if (rc) {
      if (bad_field) *bad_field = i;
      return rc;
    }
  }
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
    return HOSZP_ERR_DEVICE;

  uint32_t* blocks = new (std::nothrow) uint32_t[count];
  if (!blocks) return HOSZP_ERR_NOMEM;
  int rc = tune_blocks(ctx, fields, count, blocks, st);
  hoszp_batch* b = rc == HOSZP_OK ? new (std::nothrow) hoszp_batch() : nullptr;
  if (rc == HOSZP_OK && !b) rc = HOSZP_ERR_NOMEM;
  if (rc == HOSZP_OK) {
    b->device = ctx->device;
    b->count = count;
    b->dev.wait_limit = ctx->s.wait_limit;
    rc = build_plan(b, fields, blocks, count, hz::kBatchThreads, st);
  }
  // tile size and launch width: the widest persistent grid of 1024-thread
  // tiles, or (tuning) the fastest of both tile sizes at a few grid sizes,
  // remembered per batch shape in the tuning cache
  if (rc == HOSZP_OK) {
    b->grid = hz::batch_max_grid(cus, b->dev.threads);
    if (flags & HOSZP_BATCH_TUNE_GRID) {
      const uint64_t key = batch_signature(fields, blocks, count, cus);
      TuneChoice best{0, 0, 0.f};
      if (!tune_cache_lookup(key, &best)) {
        const uint32_t sizes[2] = {hz::kBatchThreads, hz::kBatchThreadsSmall};
        for (int t = 0; t < 2 && rc == HOSZP_OK; ++t) {
          if (b->dev.threads != sizes[t]) rc = build_plan(b, fields, blocks, count, sizes[t], st);
          const int maxg = hz::batch_max_grid(cus, sizes[t]);
          const int cand[4] = {cus, 2 * cus, 3 * cus, maxg};
          for (int c = 0; c < 4 && rc == HOSZP_OK; ++c) {
            if (cand[c] > maxg || (c > 0 && cand[c] == cand[c - 1])) continue;
            float ms = 0.f;
            rc = time_grid(b, cand[c], st, &ms);
            if (rc == HOSZP_OK && (best.ms == 0.f || ms < best.ms))
              best = TuneChoice{sizes[t], cand[c], ms};
          }
        }
        if (rc == HOSZP_OK) tune_cache_store(key, best);
      }
      if (rc == HOSZP_OK && b->dev.threads != best.threads)
        rc = build_plan(b, fields, blocks, count, best.threads, st);
      if (rc == HOSZP_OK) b->grid = best.grid;
    }
  }
  delete[] blocks;
  if (rc == HOSZP_OK) {
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
      rc = HOSZP_ERR_DEVICE;
    } else {
      if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = HOSZP_ERR_DEVICE;
      } else {
        const hipError_t le = hz::launch_batch(b->dev, b->grid, cap);
        const hipError_t ce = hipStreamEndCapture(cap, &b->graph);
        if (le != hipSuccess || ce != hipSuccess ||
            hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
          rc = HOSZP_ERR_DEVICE;
      }
      (void)hipStreamDestroy(cap);
    }
  }
  if (rc != HOSZP_OK) {
    (void)hipGetLastError();
    if (b) batch_free(b);
    return rc;
  }
  *out = b;
  return HOSZP_OK;
}

int hoszp_batch_launch(hoszp_batch* b, void* stream) {
  if (!b) return HOSZP_ERR_ARG;
  DeviceScope scope(b->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  return device_status(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
}

int hoszp_batch_results(hoszp_batch* b, hoszp_field_result* h_out, void* stream) {
  if (!b || !h_out) return HOSZP_ERR_ARG;
  DeviceScope scope(b->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(h_out, b->dev.res, b->count * sizeof(hoszp_field_result),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HOSZP_ERR_DEVICE;
  for (uint64_t i = 0; i < b->count; ++i)
    if (h_out[i].status) return hoszp_status_code(h_out[i].status);
  return HOSZP_OK;
}

const hoszp_field_result* hoszp_batch_device_results(const hoszp_batch* b) {
  return b ? b->dev.res : nullptr;
}

int hoszp_batch_info_get(const hoszp_batch* b, hoszp_batch_info* out) {
  if (!b || !out) return HOSZP_ERR_ARG;
  out->fields = b->count;
  out->total_tiles = b->dev.total_tiles;
  out->raw_bytes = b->raw_bytes;
  out->device_bytes = b->device_bytes;
  out->grid = uint32_t(b->grid);
  out->threads = b->dev.threads;
  return HOSZP_OK;
}

int hoszp_batch_destroy(hoszp_batch* b) {
  if (!b) return HOSZP_OK;
  DeviceScope scope(b->device);
  batch_free(b);
  return HOSZP_OK;
}

}  // extern "C"
