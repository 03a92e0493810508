// api.hip -- host side of the C ABI declared in include/hoszp.h.
//
// Every entry point validates what the host can see and enqueues the
// operation's kernels on the caller's stream; the operation's last kernel
// fills the result record and returns the context's counters to zero.
// Synchronous entry points then copy the 64-byte result record to pinned host
// memory and wait for the stream.

#include <math.h>
#include <string.h>

#include <new>

#include "hoszp_internal.h"

struct hoszp_ctx {
  int device;
  hz::Scratch s;
  hz::Grids grids;
  void* d_mem;
  hoszp_result* d_res;  // record used by the synchronous entry points
  hoszp_result* h_res;  // pinned host mirror of d_res
  uint32_t epoch;       // look-back generation, 28 bits, never 0
};

namespace {

constexpr uint32_t kEpochMask = (1u << 28) - 1;
constexpr uint32_t kMaxTiles = uint32_t((hz::kMaxN + hz::kTileSegs * 32ull) / (hz::kTileSegs * 32ull) + 1);
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

// Next look-back generation.  Status words carry the generation, so they never
// need clearing -- except once every 2^28 - 1 calls when the counter wraps.
int next_epoch(hoszp_ctx* ctx, hipStream_t st, uint32_t* epoch) {
  uint32_t e = (ctx->epoch + 1) & kEpochMask;
  if (e == 0) {
    e = 1;
    const size_t bytes = size_t(ctx->s.max_tiles) * sizeof(uint64_t);
    if (hipMemsetAsync(ctx->s.st_out, 0, bytes, st) != hipSuccess) return HOSZP_ERR_DEVICE;
  }
  ctx->epoch = e;
  *epoch = e;
  return HOSZP_OK;
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

// s = m 2^-sh with |m| < 2^53 (see hz::MulScalar).
hz::MulScalar mul_split(double s) {
  hz::MulScalar k{0, 1, 0};
  int e2 = 0;
  const double frac = frexp(s, &e2);
  const int64_t m = int64_t(ldexp(frac, 53));
  const int e = e2 - 53;
  if (m == 0) return k;
  if (e >= 0) {
    k.big = 1;
    return k;
  }
  if (-e > 100) return k;  // |s q| < 2^-16: every result rounds to 0
  k.m = m;
  k.sh = -e;
  return k;
}

}  // namespace

extern "C" {

int hoszp_status_code(uint32_t m) {
  static const int order[] = {HOSZP_ERR_ARG, HOSZP_ERR_FORMAT, HOSZP_ERR_MISMATCH,
                              HOSZP_ERR_CAPACITY, HOSZP_ERR_NONFINITE, HOSZP_ERR_RANGE};
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
  const size_t nchunk = kMaxTiles / hz::kChunkTiles + 2;
  const size_t ctrl_b = 256, acc_b = 256, part_b = up(size_t(kMaxPart) * sizeof(double));
  const size_t st_b = up(size_t(kMaxTiles) * sizeof(uint64_t));
  const size_t off_b = up(nchunk * sizeof(uint64_t)), tw_b = up(size_t(kMaxTiles) * sizeof(uint32_t));
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
  ctx->epoch = 0;
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
  uint32_t epoch;
  int rc = next_epoch(ctx, st, &epoch);
  if (rc) return rc;
  return launched(ctx, d_res, st, hz::launch_compress(ctx->s, ctx->grids, d_x, g, inv2e,
                                           static_cast<uint8_t*>(d_out), epoch, d_res, st));
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
  uint32_t epoch;
  int rc = next_epoch(ctx, st, &epoch);
  if (rc) return rc;
  return launched(ctx, d_res, st, hz::launch_decompress(ctx->s, ctx->grids,
                                             static_cast<const uint8_t*>(d_c), c_bytes, d_x,
                                             n_cap, epoch, d_res, st));
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
  if (!stream_args_ok(ctx, d_c, d_res) || !d_out || !aligned(d_out, 16)) return HOSZP_ERR_ARG;
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

int hoszp_add_async(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b,
                    size_t b_bytes, void* d_out, size_t out_cap, hoszp_result* d_res,
                    void* stream) {
  if (!stream_args_ok(ctx, d_a, d_res) || !d_b || !aligned(d_b, 16) || !d_out ||
      !aligned(d_out, 16))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t epoch;
  int rc = next_epoch(ctx, st, &epoch);
  if (rc) return rc;
  return launched(ctx, d_res, st, hz::launch_add(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_a),
                                      a_bytes, static_cast<const uint8_t*>(d_b), b_bytes,
                                      static_cast<uint8_t*>(d_out), out_cap, epoch, d_res, st));
}

int hoszp_add(hoszp_ctx* ctx, const void* d_a, size_t a_bytes, const void* d_b, size_t b_bytes,
              void* d_out, size_t out_cap, size_t* out_bytes, void* stream) {
  if (!ctx || !out_bytes) return HOSZP_ERR_ARG;
  int rc = hoszp_add_async(ctx, d_a, a_bytes, d_b, b_bytes, d_out, out_cap, ctx->d_res, stream);
  if (rc) return rc;
  hoszp_result r;
  rc = hoszp_result_wait(ctx, ctx->d_res, &r, stream);
  if (rc == HOSZP_OK) *out_bytes = size_t(r.out_bytes);
  return rc;
}

int hoszp_mul_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, double s, void* d_out,
                    size_t out_cap, hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res) || !d_out || !aligned(d_out, 16) || !isfinite(s))
    return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t epoch;
  int rc = next_epoch(ctx, st, &epoch);
  if (rc) return rc;
  return launched(ctx, d_res, st, hz::launch_mul(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_c),
                                      c_bytes, mul_split(s), static_cast<uint8_t*>(d_out),
                                      out_cap, epoch, d_res, st));
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

static int reduce_async(hoszp_ctx* ctx, const void* d_c, size_t c_bytes, bool variance,
                        hoszp_result* d_res, void* stream) {
  if (!stream_args_ok(ctx, d_c, d_res)) return HOSZP_ERR_ARG;
  DeviceScope scope(ctx->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t epoch;
  int rc = next_epoch(ctx, st, &epoch);
  if (rc) return rc;
  return launched(ctx, d_res, st, hz::launch_reduce(ctx->s, ctx->grids, static_cast<const uint8_t*>(d_c),
                                         c_bytes, variance, epoch, d_res, st));
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

// ---- float32 workflow ops -----------------------------------------------

static int f32_map(hoszp_ctx* ctx, int op, const float* x, const float* y, double s, float* out,
                   uint64_t n, void* stream) {
  if (!ctx || !x || !out || (op == 1 && !y) || n == 0 || !aligned(x, 16) || !aligned(out, 16) ||
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

}  // extern "C"
