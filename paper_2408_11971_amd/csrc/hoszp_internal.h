// hoszp_internal.h -- definitions shared by the HIP kernels and the C-ABI
// host code of the library (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "hoszp.h"

namespace hz {

// ---- stream format --------------------------------------------------------
constexpr uint32_t kHeaderBytes = 64;
constexpr uint32_t kMagic = 0x5A534F48u;  // "HOSZ" read as a little-endian u32
constexpr int64_t kBinMax = 2147483647LL; // bins live in [-kBinMax, kBinMax]
constexpr uint64_t kMaxN = 4294967295ULL; // n < 2^32

// ---- work decomposition ---------------------------------------------------
// A block of L slots is cut into L/32 "segments" of 32 slots.  Because every
// block contributes L * width bits to the payload, segment s of a block owns
// exactly `width` 32-bit words of it, starting on a word boundary, and sign
// word s of the block.  Every kernel processes one segment per thread.
// Encoders (compress, add, mul, batch) take tiles of as many segments as
// their workgroup has threads; the other kernels use kThreads-thread
// workgroups.
constexpr int kThreads = 256;
// Smallest encoder tile: sizes the look-back status words (kMaxTiles).
constexpr int kMinTileSegs = kThreads;
// Segments (= threads) per tile of the single-field compress kernel.
constexpr int kCompressTileSegs = 1024;

// Decoders work per wave on "wave tiles" of kWaveSegs segments (2048 slots),
// with no workgroup barrier between tiles.  The width pre-pass stores every
// wave tile's payload word count and, for every chunk of kChunkTiles wave
// tiles, the exclusive prefix; a wave tile's offset is its chunk's prefix
// plus at most 63 counts (one wave-wide load).  An encoder tile of NT
// segments is NT / kWaveSegs consecutive wave tiles.
constexpr int kWaveSegs = 64;
constexpr int kWaveWords = kWaveSegs * 32;  // worst-case payload words of a wave tile
constexpr int kChunkTiles = 64;

// ---- status bits latched by the kernels (bit = 1 << code) -----------------
constexpr uint32_t ST_ARG = 1u << HOSZP_ERR_ARG;
constexpr uint32_t ST_NONFINITE = 1u << HOSZP_ERR_NONFINITE;
constexpr uint32_t ST_RANGE = 1u << HOSZP_ERR_RANGE;
constexpr uint32_t ST_FORMAT = 1u << HOSZP_ERR_FORMAT;
constexpr uint32_t ST_MISMATCH = 1u << HOSZP_ERR_MISMATCH;
constexpr uint32_t ST_CAPACITY = 1u << HOSZP_ERR_CAPACITY;
constexpr uint32_t ST_TIMEOUT = 1u << HOSZP_ERR_TIMEOUT;

// Section placement of a stream with n elements in blocks of L.
struct Layout {
  uint64_t n, nb, nseg, nwtiles;  // nwtiles: wave tiles
  uint32_t L, spb;  // block size, segments per block
  uint32_t spb_log2;
  double eb;
  uint64_t off_w, off_o, off_s, off_p;
  uint64_t payload_bytes, total_bytes;
};

__host__ __device__ inline uint64_t round16(uint64_t x) { return (x + 15u) & ~uint64_t(15); }
__host__ __device__ inline bool block_ok(uint32_t L) {
  return L == 32 || L == 64 || L == 128 || L == 256;
}

__host__ __device__ inline void place(Layout& g, uint64_t n, uint32_t L, double eb) {
  g.n = n;
  g.L = L;
  g.spb = L / 32;
  g.spb_log2 = L == 32 ? 0u : (L == 64 ? 1u : (L == 128 ? 2u : 3u));
  g.eb = eb;
  g.nb = (n + L - 1) / L;
  g.nseg = g.nb * g.spb;
  g.nwtiles = (g.nseg + kWaveSegs - 1) / kWaveSegs;
  g.off_w = kHeaderBytes;
  g.off_o = round16(g.off_w + g.nb);
  g.off_s = round16(g.off_o + 4 * g.nb);
  g.off_p = round16(g.off_s + 4 * g.nseg);
  g.payload_bytes = 0;
  g.total_bytes = g.off_p;
}

// Worst case: every block at width 32 (L words of payload per block).
__host__ __device__ inline uint64_t bound_bytes(uint64_t n, uint32_t L) {
  Layout g;
  place(g, n, L, 1.0);
  return g.off_p + 4 * uint64_t(L) * g.nb;
}



// Per-stream results of the width pre-pass.
struct TileIndex {
  uint32_t* tile_words;   // payload words of every wave tile
  uint32_t* chunk_words;  // payload words of every chunk
  uint64_t* chunk_off;    // exclusive prefix of chunk_words
};

// Device scratch owned by a context.
struct Scratch {
  uint32_t* ctrl;       // [0] tile ticket, [1] finished-workgroup counter,
                        // [2], [3] width pre-pass counters (stream A, B)
  uint64_t* acc;        // [0] S, [1] Q lo, [2] Q hi, [3] width sum
  double* part;         // per-workgroup partials of the float32 reductions
  uint64_t* st_out;     // look-back status words of an output stream
  TileIndex idx[2];     // width pre-pass of input stream A and B
  uint32_t max_tiles;   // capacity of the per-tile status words (and / 64 chunks)
  uint32_t max_part;    // capacity of `part`
  uint32_t wait_limit;  // polls an encoder tile may spend on its look-back
                        // before it gives up with ST_TIMEOUT
};
// Default look-back poll limit: a poll is one device-coherent load (about a
// microsecond) plus a short sleep, so a launch gives up after seconds, far
// beyond any wait on running predecessors (tens of microseconds).
constexpr uint32_t kDefaultWaitLimit = 1u << 24;

// The float inputs whose Eq. 3 bin, floor(((double)x + eb) * inv2e) in
// binary64 as the kernels evaluate it, lies in [-K, K] (by default the bin
// range [-(2^31-1), 2^31-1]): the bin is non-decreasing in x, so they form
// the interval [lo, hi], found by bisection over the ordered float bit
// patterns.  An empty side is NaN, which every comparison fails.
inline int32_t float_key(float x) {
  int32_t b;
  memcpy(&b, &x, 4);
  return b >= 0 ? b : (b ^ 0x7fffffff);
}
inline float key_float(int32_t k) {
  const int32_t b = k >= 0 ? k : (k ^ 0x7fffffff);
  float x;
  memcpy(&x, &b, 4);
  return x;
}
inline double host_bin(float x, double eb, double inv2e) {
  const double shifted = double(x) + eb;
  return floor(shifted * inv2e);
}
inline void bin_range_floats(double eb, double inv2e, float& lo, float& hi,
                             double K = 2147483647.0) {
  const int32_t kmin = float_key(-3.40282347e+38f), kmax = float_key(3.40282347e+38f);
  // hi: the largest key whose bin is <= K
  if (!(host_bin(key_float(kmin), eb, inv2e) <= K)) {
    hi = NAN;
  } else if (host_bin(key_float(kmax), eb, inv2e) <= K) {
    hi = key_float(kmax);
  } else {
    int64_t a = kmin, b = kmax;  // bin(a) <= K < bin(b)
    while (b - a > 1) {
      const int64_t m = a + (b - a) / 2;
      if (host_bin(key_float(int32_t(m)), eb, inv2e) <= K) a = m; else b = m;
    }
    hi = key_float(int32_t(a));
  }
  // lo: the smallest key whose bin is >= -K
  if (!(host_bin(key_float(kmax), eb, inv2e) >= -K)) {
    lo = NAN;
  } else if (host_bin(key_float(kmin), eb, inv2e) >= -K) {
    lo = key_float(kmin);
  } else {
    int64_t a = kmin, b = kmax;  // bin(a) < -K <= bin(b)
    while (b - a > 1) {
      const int64_t m = a + (b - a) / 2;
      if (host_bin(key_float(int32_t(m)), eb, inv2e) >= -K) b = m; else a = m;
    }
    lo = key_float(int32_t(b));
  }
}
// The largest T with [-T, T] inside [lo, hi] for the bound K (0 always is:
// its bin is floor(1/2) = 0), so |x| <= T guarantees |bin| <= K.
inline float abs_bound(double eb, double inv2e, double K = 2147483647.0) {
  float lo, hi;
  bin_range_floats(eb, inv2e, lo, hi, K);
  return (lo == lo && hi == hi) ? fmaxf(fminf(-lo, hi), 0.0f) : 0.0f;
}

// Bins below this bound in magnitude let a segment's bin sums be formed in
// binary64 without rounding (32 squares below 2^42 sum below 2^47).
constexpr double kSmallBin = 2097151.0;  // 2^21 - 1

// Scalar multiplier, classified on the host (see mul_split()).
struct MulScalar {
  double s;     // the scalar
  int32_t zero; // 1 when |s q| < 2^-16 for every int32 q: every result is 0
  int32_t pad;
};

// floor(s q + 1/2) in exact arithmetic (scalar multiplication of Sec. V-A,
// rounding half up), returned as a double that is exact whenever the result
// can be a bin; |result| > 2^31 - 1 (or infinite) means out of range.
// Requires s finite and s = 0 or |s| >= 2^-48 (smaller multipliers give 0 for
// every int32 q and are replaced by 0 on the host), so nothing underflows.
//   y = fl(s q) and e = fma(s, q, -y) give s q = y + e exactly, |e| <= ulp(y)/2.
//   h = rint(y) is an integer and r = y - h is exact with |r| <= 1/2: for
//   |y| >= 1/2 both are multiples of ulp(y) <= 1 and |r| <= 2^52 ulp(y); for
//   |y| < 1/2, h = 0 and r = y.
//   s q + 1/2 = h + (r + e + 1/2).  Unless r = +-1/2 exactly, r is at least
//   ulp(y) away from both (a multiple of ulp(y) when |y| >= 1/2; the largest
//   double below 1/2 is 1/2 - ulp(y) when |y| < 1/2), so r + e + 1/2 lies in
//   (0, 1) and the result is h.  At r = 1/2 it is h + 1 when e >= 0, else h;
//   at r = -1/2 it is h - 1 when e < 0, else h.
//   For |y| >= 2^52, r = 0 and |h| is far outside the bin range, as is the
//   exact result; overflow gives an infinite h.
// Shared by the kernels and the host function hoszp_mul_bins.
__host__ __device__ inline double mul_round(double s, double q) {
  const double y = s * q;
  const double e = fma(s, q, -y);
  const double h = rint(y);
  const double r = y - h;
  const double up = (r == 0.5 && e >= 0.0) ? 1.0 : 0.0;
  const double dn = (r == -0.5 && e < 0.0) ? 1.0 : 0.0;
  return (h + up) - dn;
}

// One field of a batched compress, as the kernel sees it.
struct BatchField {
  const float* x;
  uint8_t* out;
  uint64_t n;
  double eb, inv2e;
  uint64_t tile0;   // first work-list tile of the field
  uint32_t block;
  float abs_ok;     // abs_bound(eb, inv2e)
  float abs_small;  // abs_bound(eb, inv2e, kSmallBin)
  uint32_t pad;
};

// Device state of a batch plan (see k_batch).
struct BatchDev {
  BatchField* fields;
  uint32_t* tile_field;
  uint64_t total_tiles;
  uint64_t* st;
  uint32_t* ctrl;
  uint64_t* facc;
  hoszp_field_result* res;
  uint32_t threads;  // workgroup size = segments per tile (kBatchThreads or kBatchThreadsSmall)
  uint32_t wait_limit;  // look-back poll limit of the launch
};
constexpr int kBatchAccWords = 8;  // accumulator words per field
// Workgroup sizes of the batched compress (= segments per work-list tile);
// the autotuner picks one per plan.
constexpr int kBatchThreads = 1024;
constexpr int kBatchThreadsSmall = 512;
inline __host__ __device__ uint64_t batch_tiles(const Layout& g, uint32_t nt) {
  return (g.nseg + nt - 1) / nt;
}

// Occupancy-derived persistent grid sizes, filled at context creation.
struct Grids {
  int compress, decode, reduce, add, mul, negate, widths, f32, bivar;
  int cus;  // compute units of the device
};

// Segments per compress tile for a field of nseg segments: kSmallTileSegs
// when even those tiles are no more than the compute units (a field of at
// most ~2 M values on MI355X: the 1024-segment tiles would leave most CUs
// idle), else 1024 (one workgroup per CU).  Small tiles are not used for
// larger fields: with several small tiles per CU all starting at once, every
// look-back scans far back before any inclusive prefix exists (measured 2x
// slower on a 6.5 M-value field).  Launches and the status words they use
// (the allocation-free entry point clears them) both follow this.
constexpr int kSmallTileSegs = 256;
inline uint32_t compress_tile_segs(uint64_t nseg, int cus) {
  return (nseg + kSmallTileSegs - 1) / kSmallTileSegs <= uint64_t(cus > 0 ? cus : 1)
             ? uint32_t(kSmallTileSegs)
             : uint32_t(kCompressTileSegs);
}

// ---- launchers (kernels.hip) ----------------------------------------------
// Clears the context counters and a result record; only needed after a
// failed launch left an operation half-enqueued.
hipError_t launch_reset(const Scratch& s, hoszp_result* res, hipStream_t st);
hipError_t launch_compress(const Scratch& s, const Grids& gr, const float* x, const Layout& g,
                           double inv2e, uint8_t* out, hoszp_result* res, hipStream_t st);
hipError_t launch_decompress(const Scratch& s, const Grids& gr, const uint8_t* c,
                             uint64_t c_bytes, float* x, uint64_t n_cap, hoszp_result* res,
                             hipStream_t st);
hipError_t launch_reduce(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                         bool variance, hoszp_result* res, hipStream_t st);
hipError_t launch_negate(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                         uint8_t* out, uint64_t out_cap, hoszp_result* res, hipStream_t st);
hipError_t launch_block_means(const Scratch& s, const Grids& gr, const uint8_t* c,
                              uint64_t c_bytes, double* means, uint64_t means_cap,
                              hoszp_result* res, hipStream_t st);
// Scalar addition (sign +1) or subtraction (sign -1) on the outliers.
hipError_t launch_shift(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                        double scalar, int sign, uint8_t* out, uint64_t out_cap,
                        hoszp_result* res, hipStream_t st);
// Element-wise addition, or subtraction a - b when `sub`.
hipError_t launch_add(const Scratch& s, const Grids& gr, const uint8_t* a, uint64_t a_bytes,
                      const uint8_t* b, uint64_t b_bytes, uint8_t* out, uint64_t out_cap,
                      hoszp_result* res, hipStream_t st, bool sub = false);
hipError_t launch_mul(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                      MulScalar k, uint8_t* out, uint64_t out_cap, hoszp_result* res,
                      hipStream_t st);
// Hadamard product (out: the product stream) or covariance (value in res).
hipError_t launch_bivar(const Scratch& s, const Grids& gr, bool covariance, const uint8_t* a,
                        uint64_t a_bytes, const uint8_t* b, uint64_t b_bytes, uint8_t* out,
                        uint64_t out_cap, hoszp_result* res, hipStream_t st);
hipError_t launch_f32_unary(const Grids& gr, int op, const float* x, const float* y2, double s,
                            float* out, uint64_t n, hipStream_t st);
hipError_t launch_f32_reduce(const Scratch& s, const Grids& gr, const float* x, uint64_t n,
                             bool variance, hoszp_result* res, hipStream_t st);
hipError_t launch_zero64(uint64_t* p, uint64_t n, hipStream_t st);
hipError_t launch_batch(const BatchDev& b, int grid, hipStream_t st);
int batch_max_grid(int num_cus, uint32_t threads);
hipError_t query_grids(Grids& gr, int num_cus);

}  // namespace hz
