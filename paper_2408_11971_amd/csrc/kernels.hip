// kernels.hip -- gfx950 kernels of the HoSZp library (arXiv 2408.11971).
//
// Work decomposition (shared by every kernel): a block of L slots is split
// into L/32 segments of 32 slots and one thread owns one segment.  A segment
// of a block of width w owns exactly w payload words (32 slots x w bits), so
// payload offsets are prefix sums of per-segment widths:
//   - decoders (mean, variance, decompress) work per wave on tiles of 64
//     segments and get offsets from a width pre-pass (k_widths) that reads
//     only the width section and stores per-tile word counts, per-chunk
//     totals and (for streams of more than 64 chunks) per-chunk prefixes;
//   - encoders (compress, add, mul, batch) work per workgroup on tiles of
//     NT segments (1024 threads) and produce offsets with a single-pass
//     decoupled look-back over per-tile word counts, with tiles taken from an
//     atomic ticket so a tile only waits on tiles owned by running
//     workgroups.
// Payload words are staged in LDS as big-endian values (one byte swap per
// word), so a w-bit field at bit p of a segment is one funnel shift
// (v_alignbit) of two neighbouring LDS words.  Wave-level sums and minima are
// ds_swizzle butterflies, wave maxima and scans DPP row shifts and
// broadcasts, so no lane-index registers stay live in the kernels' loops.
//
// Every operation ends in one kernel whose last workgroup to finish writes
// the caller's result record and returns the context's counters to zero, so
// an operation needs no separate initialisation launch.

#include "hoszp_internal.h"

namespace hz {
namespace {

constexpr double kBinMaxD = 2147483647.0;
constexpr uint64_t kLbAgg = 1, kLbInc = 2;
constexpr uint64_t kLbValMask = (uint64_t(1) << 34) - 1;
constexpr uint32_t kNone = 0xffffffffu;
constexpr uint32_t kEpochLimit = 1u << 28;  // look-back epochs are 28-bit, never 0
// Workgroup size (= segments per look-back tile) of the single-field
// encoders: larger tiles halve the serial look-back steps.
constexpr int kCompressThreads = kCompressTileSegs;
constexpr int kMulThreads = 1024;
constexpr int kAddThreads = 1024;

enum { kMean = 0, kVariance = 1, kDecompress = 2, kBlockMean = 3 };
// context counters (Scratch::ctrl) and accumulators (Scratch::acc)
enum { C_TICKET = 0, C_DONE = 1, C_WIDTHS = 2 /* 2, 3 */, C_STATUS = 4, C_EPOCH = 5 };
enum { A_S = 0, A_QLO = 1, A_QHI = 2, A_WSUM = 3, A_OUT = 4, A_CONST = 5, A_SB = 6 };

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t bswap32(uint32_t v) { return __builtin_bswap32(v); }
__device__ __forceinline__ uint32_t bitlen32(uint32_t v) { return v ? 32u - __clz(int(v)) : 0u; }

// Values every lane holds identically, moved to scalar registers so that
// branches on them (loop exits next to barriers in particular) compile to
// uniform branches.
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return (uint64_t(uni32(uint32_t(v >> 32))) << 32) | uni32(uint32_t(v));
}

__device__ __forceinline__ void latch(const Scratch& s, uint32_t bits) {
  if (bits) atomicOr(&s.ctrl[C_STATUS], bits);
}

__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave reductions (call with every lane of the wave active; the result is
// wave-uniform).  Butterfly steps inside each 32-lane half use ds_swizzle's
// bit-mask mode (lane i reads lane i ^ M), whose pattern is an immediate, so
// no lane-index registers stay live; the two halves join through readlane.
template <int M>
__device__ __forceinline__ uint32_t swz_xor(uint32_t v) {
  return uint32_t(__builtin_amdgcn_ds_swizzle(int(v), 0x1f | (M << 10)));
}
__device__ __forceinline__ uint32_t lane_of(uint32_t v, int lane) {
  return uint32_t(__builtin_amdgcn_readlane(int(v), lane));
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  v = min(v, swz_xor<1>(v));
  v = min(v, swz_xor<2>(v));
  v = min(v, swz_xor<4>(v));
  v = min(v, swz_xor<8>(v));
  v = min(v, swz_xor<16>(v));
  return min(lane_of(v, 0), lane_of(v, 32));
}
__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
  v += swz_xor<1>(v);
  v += swz_xor<2>(v);
  v += swz_xor<4>(v);
  v += swz_xor<8>(v);
  v += swz_xor<16>(v);
  return lane_of(v, 0) + lane_of(v, 32);
}
template <int M>
__device__ __forceinline__ uint64_t swz_add64(uint64_t v) {
  const uint64_t o = (uint64_t(swz_xor<M>(uint32_t(v >> 32))) << 32) | swz_xor<M>(uint32_t(v));
  return v + o;
}
__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
  v = swz_add64<1>(v);
  v = swz_add64<2>(v);
  v = swz_add64<4>(v);
  v = swz_add64<8>(v);
  v = swz_add64<16>(v);
  const uint64_t a = (uint64_t(lane_of(uint32_t(v >> 32), 0)) << 32) | lane_of(uint32_t(v), 0);
  const uint64_t b = (uint64_t(lane_of(uint32_t(v >> 32), 32)) << 32) | lane_of(uint32_t(v), 32);
  return a + b;
}

// Inclusive scan over the wave (every lane active) with DPP row shifts
// inside each row of 16 lanes, then the row broadcasts of lane 15 and lane
// 31 across rows; a lane adds a moved value only where its source lane lies
// before it.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return uint32_t(__builtin_amdgcn_mov_dpp(int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = threadIdx.x & 63, rl = lane & 15;
  uint32_t t = dpp_mov<0x111>(x);  // row_shr:1
  x += rl >= 1 ? t : 0u;
  t = dpp_mov<0x112>(x);  // row_shr:2
  x += rl >= 2 ? t : 0u;
  t = dpp_mov<0x114>(x);  // row_shr:4
  x += rl >= 4 ? t : 0u;
  t = dpp_mov<0x118>(x);  // row_shr:8
  x += rl >= 8 ? t : 0u;
  t = dpp_mov<0x142>(x);  // row_bcast:15
  x += (lane & 31) >= 16 ? t : 0u;
  t = dpp_mov<0x143>(x);  // row_bcast:31
  x += lane >= 32 ? t : 0u;
  return x;
}

// Largest value over the wave (every lane active) by the same DPP pattern as
// the scan, all in VALU (no LDS round trips): lanes without a source lane
// read 0, which is no larger than any value here.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_or0(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
  x = max(x, dpp_or0<0x111>(x));  // row_shr:1
  x = max(x, dpp_or0<0x112>(x));  // row_shr:2
  x = max(x, dpp_or0<0x114>(x));  // row_shr:4
  x = max(x, dpp_or0<0x118>(x));  // row_shr:8
  x = max(x, dpp_or0<0x142>(x));  // row_bcast:15
  x = max(x, dpp_or0<0x143>(x));  // row_bcast:31
  return lane_of(x, 63);
}

// Count this workgroup as finished on `counter`.  True (uniform) in the last
// workgroup to finish.  Everything a last workgroup reads from the others
// travels through device-scope atomics (performed at the device coherence
// point, not in an XCD's L2), and each workgroup waits for its own memory
// operations to complete before counting itself, so no cache write-back or
// invalidation is needed.  Contains barriers: call from uniform control flow.
__device__ __forceinline__ bool finish_arrive(uint32_t* counter, uint32_t* s_flag) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's atomics and stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = old == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  return uni32(*s_flag) != 0;
}

// finish_arrive for a counter that reaches `total`, adding `count` arrivals.
__device__ __forceinline__ bool finish_arrive_n(uint32_t* counter, uint32_t count, uint32_t total,
                                                uint32_t* s_flag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old =
        __hip_atomic_fetch_add(counter, count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_flag = old + count == total ? 1u : 0u;
  }
  __syncthreads();
  return uni32(*s_flag) != 0;
}

// Last workgroup of an operation: fill the caller's record and return the
// context's counters and accumulators to zero for the next operation.
__device__ __forceinline__ void publish(const Scratch& s, hoszp_result* res, uint64_t out_bytes, double value) {
  if (threadIdx.x != 0) return;
  res->status = ld_dev32(&s.ctrl[C_STATUS]);
  res->out_bytes = out_bytes;
  res->value = value;
  s.ctrl[C_TICKET] = 0;
  s.ctrl[C_DONE] = 0;
  s.ctrl[C_STATUS] = 0;
  for (int k = 0; k < 8; ++k) s.acc[k] = 0;
}

// Validate a stream header and derive its section placement.
__device__ __forceinline__ uint32_t read_header(const uint8_t* c, uint64_t c_bytes, Layout& g) {
  if (c_bytes < kHeaderBytes) return ST_FORMAT;
  const uint64_t* h = reinterpret_cast<const uint64_t*>(c);
  const uint64_t h0 = uni64(h[0]), h1 = uni64(h[1]), h2 = uni64(h[2]), h3 = uni64(h[3]);
  const uint64_t h4 = uni64(h[4]), h5 = uni64(h[5]), h6 = uni64(h[6]);
  if (uint32_t(h0) != kMagic || (h0 >> 32) != 1u) return ST_FORMAT;  // magic, version 1, flags 0
  const uint32_t L = uint32_t(h1);
  const uint64_t n = h2;
  const double eb = __longlong_as_double((long long)h3);
  if (!block_ok(L) || n == 0 || n > kMaxN) return ST_FORMAT;
  if (!(eb > 0.0) || !isfinite(eb)) return ST_FORMAT;
  place(g, n, L, eb);
  if (h4 != g.nb) return ST_FORMAT;
  if (h6 > c_bytes || h6 < g.off_p || h6 - g.off_p != h5 || (h5 & 3u)) return ST_FORMAT;
  g.payload_bytes = h5;
  g.total_bytes = h6;
  return 0;
}

// Header and zero padding of an output stream whose payload is `payload` bytes.
__device__ __forceinline__ void write_header(uint8_t* out, const Layout& g, uint64_t payload) {
  uint64_t* h = reinterpret_cast<uint64_t*>(out);
  h[0] = uint64_t(kMagic) | (uint64_t(1) << 32);
  h[1] = g.L;
  h[2] = g.n;
  h[3] = uint64_t(__double_as_longlong(g.eb));
  h[4] = g.nb;
  h[5] = payload;
  h[6] = g.off_p + payload;
  h[7] = 0;
  for (uint64_t i = g.off_w + g.nb; i < g.off_o; ++i) out[i] = 0;
  for (uint64_t i = g.off_o + 4 * g.nb; i < g.off_s; ++i) out[i] = 0;
  for (uint64_t i = g.off_s + 4 * g.nseg; i < g.off_p; ++i) out[i] = 0;
}

// Exclusive scan of one value per thread over the workgroup, plus the total.
// Contains barriers: call from workgroup-uniform control flow.
template <int NT = kThreads>
__device__ __forceinline__ uint32_t wg_scan(uint32_t v, uint32_t& total, uint32_t* tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t x = wave_incl_scan(v);
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t t = tmp[w];
    before += (w < wave) ? t : 0u;
    all += t;
  }
  __syncthreads();
  total = uni32(all);
  return before + x - v;
}

__device__ __forceinline__ uint64_t wg_scan64(uint64_t v, uint64_t& total, uint64_t* tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint64_t t = tmp[w];
    before += (w < wave) ? t : 0u;
    all += t;
  }
  __syncthreads();
  total = all;
  return before + x - v;
}

// ------------------------------------------------------------ look-back scan

__device__ __forceinline__ uint64_t lb_word(uint32_t epoch, uint64_t flag, uint64_t v) {
  return (uint64_t(epoch) << 36) | (flag << 34) | (v & kLbValMask);
}

// Look-back generation of a single-stream encoder launch: one more than the
// previous launch's, kept in the context's counter word (28 bits, never 0).
// It lives on the device so that a launch captured in a graph gets a fresh
// generation at every replay: status words a previous replay published
// never look valid to the next one.
__device__ __forceinline__ uint32_t launch_epoch(const Scratch& s) {
  const uint32_t e = (uni32(ld_dev32(&s.ctrl[C_EPOCH])) + 1u) & (kEpochLimit - 1u);
  return e ? e : 1u;
}

// Last workgroup of an encoder launch (whole workgroup): record the launch's
// generation; before the counter wraps, clear every status word so no word
// of an earlier launch with the same generation survives.
__device__ __forceinline__ void retire_epoch(const Scratch& s, uint32_t epoch) {
  if (epoch == kEpochLimit - 1u)
    for (uint64_t k = threadIdx.x; k < s.max_tiles; k += blockDim.x) s.st_out[k] = 0;
  if (threadIdx.x == 0) s.ctrl[C_EPOCH] = epoch;
}

template <int NT = kThreads>
struct LbShared {
  uint32_t first_inc[NT / 64];
  uint32_t first_wait[NT / 64];
  uint64_t part[NT / 64];
  uint64_t near_sum;
  uint32_t near_found;  // 0: keep searching, 1: inclusive prefix found, 2: gave up
  uint32_t polls;
};

// Decoupled look-back: exclusive prefix over tiles of the per-tile `agg`.
// lb_publish stores the tile's aggregate as soon as it is known, so tiles
// waiting on it never block the tiles before them; the caller can then do
// work that needs no offset before calling lb_wait.  Phase 1: wave 0 polls
// the 64 nearest predecessors until every tile up to the nearest inclusive
// prefix has published.  Phase 2 (only when none of them holds an inclusive
// prefix): the whole workgroup reads older windows of kThreads status words,
// one per thread, so the search moves hundreds of tiles per device-coherent
// load.  (Also storing the inclusive prefix of every summed predecessor, to
// keep the frontier close, was measured slower on MI355X: the extra
// device-scope stores cost more than the shorter searches save.)
__device__ __forceinline__ void lb_publish(uint64_t* st, uint64_t tile, uint64_t agg,
                                           uint32_t epoch) {
  if (threadIdx.x == 0) st_dev(&st[tile], lb_word(epoch, tile == 0 ? kLbInc : kLbAgg, agg));
}

// The wait is bounded: after `limit` unsuccessful polls (phase 1 and 2
// together) the tile gives up, ORs ST_TIMEOUT into `bad`, takes what it has
// summed as its prefix and publishes as usual, so the launch still drains and
// every later wait ends.  A prefix taken this way is at most the true one, so
// the tile's stores stay inside the stream's worst-case bound; the launch's
// output is invalid and the error says so.  With limit 0 every tile but the
// first gives up without polling.  Contains barriers (except for tile 0, which
// returns at once).
template <int NT = kThreads>
__device__ __forceinline__ uint64_t lb_wait(uint64_t* st, uint64_t tile, uint64_t agg,
                                            uint32_t epoch, LbShared<NT>& sh, uint32_t limit,
                                            uint32_t& bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tile == 0) return 0;
  uint32_t polls = 0;
  if (wave == 0) {
    const int64_t idx = int64_t(tile) - 1 - lane;
    for (;;) {
      if (polls >= limit) {  // wave-uniform
        if (lane == 0) {
          sh.near_sum = 0;
          sh.near_found = 2u;
          sh.polls = polls;
        }
        break;
      }
      ++polls;
      bool ready = true, inc = true;
      uint64_t val = 0;
      if (idx >= 0) {
        const uint64_t w = ld_dev(&st[idx]);
        const uint64_t flag = (w >> 34) & 3u;
        ready = uint32_t(w >> 36) == epoch && flag != 0;
        inc = ready && flag == kLbInc;
        val = w & kLbValMask;
      }
      const uint64_t incm = __ballot(inc);
      const uint64_t waitm = __ballot(!ready);
      const uint64_t upto = incm ? (((incm & (~incm + 1)) << 1) - 1) : ~uint64_t(0);
      if (waitm & upto) {
        __builtin_amdgcn_s_sleep(2);
        continue;
      }
      const uint64_t part = wave_sum(((upto >> lane) & 1u) ? val : 0);
      if (lane == 0) {
        sh.near_sum = part;
        sh.near_found = incm ? 1u : 0u;
        sh.polls = polls;
      }
      break;
    }
  }
  __syncthreads();
  uint64_t excl = uni64(sh.near_sum);
  const uint32_t found = uni32(sh.near_found);
  polls = uni32(sh.polls);
  __syncthreads();
  if (found == 2u) bad |= ST_TIMEOUT;
  if (!found) {
    int64_t base = int64_t(tile) - 64;  // the window covers tiles base-1-tid
    for (;;) {
      if (polls >= limit) {  // workgroup-uniform
        bad |= ST_TIMEOUT;
        break;
      }
      ++polls;
      const int64_t idx = base - 1 - tid;
      uint32_t fi = kNone, fw = kNone;
      uint64_t val = 0;
      if (idx >= 0) {
        const uint64_t w = ld_dev(&st[idx]);
        const uint64_t flag = (w >> 34) & 3u;
        const bool ready = uint32_t(w >> 36) == epoch && flag != 0;
        if (!ready) fw = uint32_t(tid);
        if (ready && flag == kLbInc) fi = uint32_t(tid);
        val = w & kLbValMask;
      } else {
        fi = uint32_t(tid);  // before tile 0: an inclusive prefix of 0
      }
      fi = wave_min(fi);
      fw = wave_min(fw);
      if (lane == 0) {
        sh.first_inc[wave] = fi;
        sh.first_wait[wave] = fw;
      }
      __syncthreads();
      fi = kNone;
      fw = kNone;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) {
        fi = min(fi, sh.first_inc[k]);
        fw = min(fw, sh.first_wait[k]);
      }
      fi = uni32(fi);
      fw = uni32(fw);
      __syncthreads();
      if (fw < fi) {  // a tile before the nearest inclusive prefix is unpublished
        __builtin_amdgcn_s_sleep(4);
        continue;
      }
      const uint64_t part = wave_sum(uint32_t(tid) <= fi ? val : 0);
      if (lane == 0) sh.part[wave] = part;
      __syncthreads();
      uint64_t total = 0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) total += sh.part[k];
      __syncthreads();
      excl += uni64(total);
      if (fi != kNone) break;
      base -= NT;
    }
  }
  if (tid == 0) st_dev(&st[tile], lb_word(epoch, kLbInc, excl + agg));
  return excl;
}


// Streams of at most kDirectChunks chunks (up to 2^18 segments) skip the
// width pre-pass's last step (its completion count and the last workgroup's
// scan of the chunk totals): their consumers form a chunk's offset from the
// chunk totals themselves, one inclusive scan over a wave, and check that the
// totals fill the payload (which the pre-pass checks for larger streams).
constexpr uint64_t kDirectChunks = 64;
__device__ __forceinline__ uint64_t num_chunks(const Layout& g) {
  return (g.nwtiles + kChunkTiles - 1) / kChunkTiles;
}
// From every lane's chunk total (0 past the last chunk): the offset of chunk
// `chunk` (wave-uniform) and the check of the total.  Whole wave.
__device__ __forceinline__ uint64_t direct_chunk_off(uint32_t cw, uint64_t chunk,
                                                     uint64_t payload_words, uint32_t& bad) {
  // a chunk holds at most 64 x 2048 words, so 64 of them sum to at most 2^23
  const uint32_t x = wave_incl_scan(cw);
  if (lane_of(x, 63) != payload_words) bad |= ST_FORMAT;
  return chunk ? lane_of(x, int(chunk) - 1) : 0u;
}

// Payload word offset of wave tile `tile` of a stream (layout g) from its
// width pre-pass.  Run by one whole wave; every lane gets the result.
__device__ __forceinline__ uint64_t tile_offset(const TileIndex& ix, uint64_t tile, const Layout& g,
                                                uint32_t& bad) {
  const int lane = threadIdx.x & 63;
  const uint64_t chunk = tile / kChunkTiles;
  const uint32_t r = uint32_t(tile % kChunkTiles);
  const uint64_t nch = num_chunks(g);
  const bool direct = nch <= kDirectChunks;
  // both loads issued before either is waited on (lanes past r load the
  // chunk's first word and drop it)
  const uint32_t t = ix.tile_words[chunk * kChunkTiles + (uint32_t(lane) < r ? lane : 0)];
  uint64_t c = direct ? (uint32_t(lane) < nch ? ix.chunk_words[lane] : 0u) : ix.chunk_off[chunk];
  if (direct) c = direct_chunk_off(uint32_t(c), chunk, g.payload_bytes / 4, bad);
  // a wave tile holds at most 64 x 32 words, so 63 of them sum below 2^17
  return c + wave_sum32(uint32_t(lane) < r ? t : 0u);
}

// ------------------------------------------------------ segment primitives

// Number of valid slots (0..32) of segment `seg` from nfull = n / 32 and
// tail = n % 32: segment seg holds the slots 32 seg .. 32 seg + 31 of the
// field, as every block is a whole number of segments.
__device__ __forceinline__ uint32_t seg_valid(uint64_t seg, uint64_t nfull, uint32_t tail) {
  return seg < nfull ? 32u : (seg == nfull ? tail : 0u);
}

// Number of valid slots (0..32) of segment `sub` of block `blk`.
__device__ __forceinline__ uint32_t seg_count(const Layout& g, uint64_t blk, uint32_t sub,
                                              uint64_t& blen) {
  const uint64_t left = g.n - blk * g.L;
  blen = left < g.L ? left : g.L;
  const uint64_t lo = uint64_t(32) * sub;
  return blen > lo ? uint32_t(blen - lo < 32 ? blen - lo : 32) : 0u;
}

// w-bit field starting at bit p of a segment whose words start at sp (sp[-1]
// and the word after the segment must be readable LDS words); rshift = 32 - w.
__device__ __forceinline__ uint32_t window_at(const uint32_t* sp, uint32_t p) {
  const uint32_t i = (p + 31u) >> 5;  // the 32 bits from bit p on (MSB first)
  return __builtin_amdgcn_alignbit(sp[int(i) - 1], sp[i], 0u - p);
}
// p + 31 for field j's start bit p = j w (w <= 32, j < 32), as one
// instruction on the full-rate 24-bit multiplier: left to itself the compiler
// turns j w with a constant j into quarter-rate 32-bit multiplies.
__device__ __forceinline__ uint32_t field_q(uint32_t w, uint32_t j) {
  uint32_t q;
  asm("v_mad_u32_u24 %0, %1, %2, 31" : "=v"(q) : "v"(w), "s"(j));
  return q;
}
// window_at from q = p + 31 (~q equals -p modulo 32).
__device__ __forceinline__ uint32_t window_q(const uint32_t* sp, uint32_t q) {
  const uint32_t i = q >> 5;
  return __builtin_amdgcn_alignbit(sp[int(i) - 1], sp[i], ~q);
}
__device__ __forceinline__ uint32_t field_at(const uint32_t* sp, uint32_t p, uint32_t rshift) {
  return window_at(sp, p) >> rshift;
}

__device__ __forceinline__ uint32_t field(const uint32_t* sp, uint32_t j, uint32_t w) {
  return field_at(sp, __umul24(j, w), 32u - w);
}

// Magnitude and sign of delta d = q - prev for two in-range bins.
__device__ __forceinline__ uint32_t delta_mag(int32_t q, int32_t prev, bool& neg) {
  neg = q < prev;
  return neg ? uint32_t(prev) - uint32_t(q) : uint32_t(q) - uint32_t(prev);
}

// Pack 32 fields of width w (1..32), most significant bit first, into w
// consecutive LDS words starting at dst (as big-endian values).
__device__ __forceinline__ void pack32(uint32_t* dst, const uint32_t* mag, uint32_t w) {
  uint64_t acc = 0;
  uint32_t nbits = 0, o = 0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    acc = (acc << w) | mag[j];
    nbits += w;
    if (nbits >= 32) {
      nbits -= 32;
      dst[o++] = uint32_t(acc >> nbits);
    }
  }
}

// pack32 taking G fields per accumulator step: the G fields of a group are
// first joined in one 32-bit word (G w <= 32), so the 64-bit shift, the
// count and the conditional word store run 32 / G times instead of 32.
template <int G>
__device__ __forceinline__ void pack32_g(uint32_t* dst, const uint32_t* mag, uint32_t w) {
  uint64_t acc = 0;
  uint32_t nbits = 0, o = 0;
#pragma unroll
  for (int j = 0; j < 32; j += G) {
    constexpr int kLast = 32 % G;  // fields of a last, shorter group
    const int n = (j + G <= 32) ? G : kLast;
    uint32_t c = mag[j];
#pragma unroll
    for (int k = 1; k < G; ++k)
      if (k < n) c = (c << w) | mag[j + k];
    const uint32_t cw = uint32_t(n) * w;
    acc = (acc << cw) | c;
    nbits += cw;
    if (nbits >= 32) {
      nbits -= 32;
      dst[o++] = uint32_t(acc >> nbits);
    }
  }
}

// Group size for pack32_grouped: the most fields of the widest width in the
// wave that fit one 32-bit word (wave-uniform; call with every lane active).
__device__ __forceinline__ uint32_t pack_group(uint32_t w) {
  const uint32_t wmax = ~wave_min(~w);
  return uni32(wmax <= 8 ? 4u : wmax <= 10 ? 3u : wmax <= 16 ? 2u : 1u);
}

// pack32 with a wave-uniform group size from pack_group (w > 0).
__device__ __forceinline__ void pack32_grouped(uint32_t* dst, const uint32_t* mag, uint32_t w,
                                               uint32_t group) {
  switch (group) {
    case 4: pack32_g<4>(dst, mag, w); break;
    case 3: pack32_g<3>(dst, mag, w); break;
    case 2: pack32_g<2>(dst, mag, w); break;
    default: pack32_g<1>(dst, mag, w); break;
  }
}

// Bins of a block stay in range if |O| + (len-1)(2^w - 1) fits.
__device__ __forceinline__ bool bins_surely_in_range(int64_t outlier, uint64_t blen, uint32_t w) {
  const uint64_t a = uint64_t(outlier < 0 ? -outlier : outlier);
  const uint64_t step = (uint64_t(1) << w) - 1;
  return a + (blen - 1) * step <= uint64_t(kBinMax);
}
// The same test for any block of at most L slots (w <= 32), on 32-bit
// operands: one 32 x 32 -> 64-bit multiply-add.
__device__ __forceinline__ bool bins_in_range_upto(int32_t outlier, uint32_t L, uint32_t w) {
  const uint32_t a = outlier < 0 ? 0u - uint32_t(outlier) : uint32_t(outlier);
  const uint32_t step = w ? 0xffffffffu >> (32u - w) : 0u;
  return uint64_t(L - 1u) * step + a <= uint64_t(kBinMax);
}

// Stage na words from a, then nb words from b, into LDS as big-endian-decoded
// values: a's at sp[1..na], b's at sp[na + 2..na + nb + 1], each range with a
// zero guard word on both sides.  Every thread issues kStageUnroll loads before
// it waits on any, so one memory round trip moves kStageUnroll * NT words.
// (Only the words [0, na) of a and [0, nb) of b are read.)  COUNTED: skip, by
// workgroup-uniform branches, the loads a round needs for no thread (fewer
// loads for narrow tiles; which variant a kernel uses is a measured choice,
// as the branches change its register allocation).
constexpr int kStageUnroll = 16;
template <int NT = kThreads, bool COUNTED = true>
__device__ __forceinline__ void stage_words(uint32_t* sp, const uint32_t* a, uint32_t na,
                                            const uint32_t* b, uint32_t nb) {
  const uint32_t total = na + nb;
  // word k (k < total) is (k < na ? a : bk)[k]
  const uint32_t* bk = nb ? b - na : a;
  for (uint32_t k0 = threadIdx.x; k0 < total; k0 += kStageUnroll * NT) {
    uint32_t v[kStageUnroll];
    // loads this round needs at most (workgroup-uniform); past the end a
    // thread reloads the last word, so the loads carry no lane condition
    const uint32_t nu = (total - (k0 - threadIdx.x) + NT - 1) / NT;
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const uint32_t k = min(k0 + uint32_t(u) * NT, total - 1);
      if (!COUNTED || uint32_t(u) < nu) v[u] = (k < na ? a : bk)[k];
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const uint32_t k = k0 + uint32_t(u) * NT;
      if (k < total) sp[1 + k + (k >= na ? 1u : 0u)] = bswap32(v[u]);
    }
  }
  if (threadIdx.x == 0) {
    sp[0] = 0;
    sp[1 + na] = 0;
    if (nb) sp[2 + total] = 0;
  }
}

// Stage payload words [base, base + words) of a stream into LDS (sp[1..]) with
// a zero guard word on each side.  Returns false when the range leaves the
// payload section (nothing is read then).
template <int NT = kThreads>
__device__ __forceinline__ bool stage_payload(uint32_t* sp, const uint32_t* P, uint64_t base, uint32_t words,
                                              uint64_t payload_words) {
  const bool fits = base + words <= payload_words;
  stage_words<NT>(sp, P + base, fits ? words : 0u, nullptr, 0u);
  return fits;
}

// Signed delta j of a segment from its staged words, sign word and width.
__device__ __forceinline__ int64_t seg_delta(const uint32_t* sp, uint32_t sw, uint32_t w, int j) {
  const uint32_t m = field(sp, uint32_t(j), w);
  return ((sw >> (31 - j)) & 1u) ? -int64_t(m) : int64_t(m);
}

// Exclusive prefix of `v` over the `spb` consecutive threads of a block.
__device__ __forceinline__ int64_t block_excl(int64_t v, uint32_t spb) {
  const uint32_t pos = threadIdx.x & (spb - 1);
  int64_t x = v;
  for (uint32_t d = 1; d < spb; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    if (pos >= d) x += y;
  }
  return x - v;
}

__device__ __forceinline__ uint32_t block_max(uint32_t v, uint32_t spb) {
  for (uint32_t d = 1; d < spb; d <<= 1) v = max(v, uint32_t(__shfl_xor(v, int(d), 64)));
  return v;
}

// Correctly rounded conversion of the unsigned 128-bit value hi:lo.
__device__ __forceinline__ double u128_to_double(uint64_t hi, uint64_t lo) {
  if (hi == 0) return double(lo);
  const int lz = __clzll((long long)hi);
  const uint64_t top = lz ? (hi << lz) | (lo >> (64 - lz)) : hi;
  const uint64_t rest = lo << lz;
  const uint64_t jam = top | (rest != 0 ? 1u : 0u);  // sticky bit below the rounding bit
  return ldexp(double(jam), 64 - lz);
}

// Sum over the workgroup of an int64 and an unsigned 128-bit value (hi:lo);
// the result is valid in thread 0.  Contains barriers.
template <int NT = kThreads>
__device__ __forceinline__ void wg_sum_s_q(int64_t& s, uint64_t& qlo, uint64_t& qhi, int64_t* ts, uint64_t* tl,
                           uint64_t* th) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    s += __shfl_xor(s, d, 64);
    const uint64_t ol = __shfl_xor(qlo, d, 64);
    const uint64_t oh = __shfl_xor(qhi, d, 64);
    const uint64_t nl = qlo + ol;
    qhi = qhi + oh + (nl < qlo ? 1u : 0u);
    qlo = nl;
  }
  if (lane == 0) {
    ts[wave] = s;
    tl[wave] = qlo;
    th[wave] = qhi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s = 0;
    qlo = 0;
    qhi = 0;
    for (int w = 0; w < NT / 64; ++w) {
      s += ts[w];
      const uint64_t nl = qlo + tl[w];
      qhi = qhi + th[w] + (nl < qlo ? 1u : 0u);
      qlo = nl;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ kernels

// Clears the context counters and a result record (error recovery only).
__global__ void k_reset(uint32_t* ctrl, uint64_t* acc, hoszp_result* res) {
  const int t = threadIdx.x;
  if (t < 8) ctrl[t] = 0;
  if (t < 8) acc[t] = 0;
  if (t == 0 && res) {
    res->status = 0;
    res->out_bytes = 0;
    res->value = 0.0;
  }
}

// Zero n 64-bit words (used instead of a memset node so the enqueueing call
// stays capturable).
__global__ void k_zero64(uint64_t* p, uint64_t n) {
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * kThreads)
    p[i] = 0;
}

// One or two streams (the operands of a two-stream operation are indexed by
// one launch: the grid's first half takes stream 0, the second stream 1).
struct WidthParams {
  const uint8_t* c[2];
  uint64_t c_bytes[2];
  TileIndex ix[2];
  uint32_t* done[2];  // finished-workgroup counter of each stream's pre-pass
  Scratch s;
  uint32_t nstreams;
};

// Width bytes of the blocks of the 16 segments seg0 .. seg0+15, packed four
// to a word (zero past the last block).  seg0 is a multiple of 16, so the
// width bytes are aligned.
__device__ __forceinline__ uint4 widths_raw16(const uint8_t* c, const Layout& g, uint64_t seg0) {
  uint4 q = make_uint4(0u, 0u, 0u, 0u);
  if (seg0 >= g.nseg) return q;
  const uint8_t* W = c + g.off_w;
  const uint64_t b0 = seg0 >> g.spb_log2;               // first block
  const uint64_t nbk = 16u >> g.spb_log2;                // blocks covered when whole
  const uint64_t have = g.nb - b0 < nbk ? g.nb - b0 : nbk;
  if (have == nbk) {
    if (nbk == 16) {
      q = *reinterpret_cast<const uint4*>(W + b0);
    } else if (nbk == 8) {
      const uint2 v = *reinterpret_cast<const uint2*>(W + b0);
      q.x = v.x, q.y = v.y;
    } else if (nbk == 4) {
      q.x = *reinterpret_cast<const uint32_t*>(W + b0);
    } else {  // block 256: two blocks, b0 even
      q.x = *reinterpret_cast<const uint16_t*>(W + b0);
    }
  } else {
    uint32_t t[4] = {0, 0, 0, 0};
    for (uint32_t k = 0; k < uint32_t(have); ++k) t[k >> 2] |= uint32_t(W[b0 + k]) << (8 * (k & 3));
    q = make_uint4(t[0], t[1], t[2], t[3]);
  }
  return q;
}

// Payload words of those segments from their width bytes: each segment
// counts its block's width (widths above 32 are reported and counted as 0).
__device__ __forceinline__ uint32_t widths_sum16(uint4 q4, uint32_t spb, uint32_t& bad) {
  const uint32_t q[4] = {q4.x, q4.y, q4.z, q4.w};
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t packed = q[k];
    // a byte b > 32 has its top bit set or carries b + 95 into bit 7
    if ((packed | ((packed & 0x7f7f7f7fu) + 0x5f5f5f5fu)) & 0x80808080u) {
      bad |= ST_FORMAT;
      uint32_t ok = 0;
      for (int t = 0; t < 4; ++t) {
        const uint32_t v = (packed >> (8 * t)) & 0xffu;
        ok |= (v <= 32 ? v : 0u) << (8 * t);
      }
      packed = ok;
    }
    sum = __builtin_amdgcn_sad_u8(packed, 0u, sum);  // adds the 4 bytes
  }
  return sum * spb;
}

// Width pre-pass of a stream (reads only its width section): payload words of
// every wave tile and the exclusive prefix of every chunk of kChunkTiles wave
// tiles, so decoders locate any tile's payload without a serial scan.  Also
// checks every width <= 32 and that the widths fill the payload exactly.
// A workgroup takes up to kWidthChunks chunks per pass, gridDim.x apart (so
// every workgroup has one before any has two), with all their loads in flight
// at once; the last workgroup to finish turns the chunk counts into offsets,
// holding up to kOffRegs counts per thread in registers so each is read once.
constexpr int kWidthChunks = 4;
constexpr int kOffRegs = 8;
__global__ void __launch_bounds__(kThreads) k_widths(WidthParams p) {
  __shared__ uint32_t s_chunk[kWidthChunks][kThreads / 64];
  __shared__ uint64_t s_tmp[kThreads / 64];
  __shared__ uint32_t s_flag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t gsz = gridDim.x / p.nstreams;  // workgroups per stream
  const uint32_t which = blockIdx.x / gsz, bid = blockIdx.x - which * gsz;
  const uint8_t* c = p.c[which];
  const TileIndex ix = p.ix[which];
  Layout g;
  const uint32_t err = read_header(c, p.c_bytes[which], g);
  if (err) {  // decoders see the same header and stop; nothing to index
    if (tid == 0 && bid == 0) latch(p.s, err);
    return;
  }
  static_assert(kChunkTiles * kWaveSegs == kThreads * 16, "16 segments per thread per chunk");
  const uint64_t nchunks = (g.nwtiles + kChunkTiles - 1) / kChunkTiles;
  uint32_t bad = 0;
  const uint64_t gs = gsz;
  for (uint64_t c0 = bid; c0 < nchunks; c0 += gs * kWidthChunks) {
    // thread tid: segments 16 tid .. 16 tid + 15 of each chunk, a quarter of
    // wave tile tid / 4 (chunks past the last read nothing and count 0)
    uint4 q[kWidthChunks];
#pragma unroll
    for (int k = 0; k < kWidthChunks; ++k)
      q[k] = widths_raw16(c, g, (c0 + k * gs) * (kChunkTiles * kWaveSegs) + 16 * uint64_t(tid));
#pragma unroll
    for (int k = 0; k < kWidthChunks; ++k) {
      if (c0 + k * gs >= nchunks) break;  // (uniform) no dependent shuffles for absent chunks
      uint32_t v = widths_sum16(q[k], g.spb, bad);
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      const uint64_t wt = (c0 + k * gs) * kChunkTiles + uint64_t(tid >> 2);
      if ((tid & 3) == 0 && wt < g.nwtiles) ix.tile_words[wt] = v;
      const uint32_t wsum = wave_sum32((tid & 3) == 0 ? v : 0u);
      if (lane == 0) s_chunk[k][wave] = wsum;
    }
    __syncthreads();
    if (tid < kWidthChunks && c0 + tid * gs < nchunks) {
      uint32_t t = 0;
      for (int k = 0; k < kThreads / 64; ++k) t += s_chunk[tid][k];
      st_dev32(&ix.chunk_words[c0 + tid * gs], t);
    }
    __syncthreads();
  }
  latch(p.s, bad);
  if (nchunks <= kDirectChunks) return;  // consumers scan the chunk totals themselves
  if (!finish_arrive_n(p.done[which], 1u, gsz, &s_flag)) return;
  // last workgroup: chunk counts -> chunk offsets, and the total check
  const uint64_t per = (nchunks + kThreads - 1) / kThreads;
  const uint64_t lo = per * tid, hi = lo + per < nchunks ? lo + per : nchunks;
  uint64_t total;
  if (per <= uint64_t(kOffRegs)) {
    uint32_t cw[kOffRegs];
#pragma unroll
    for (int k = 0; k < kOffRegs; ++k) cw[k] = lo + k < hi ? ld_dev32(&ix.chunk_words[lo + k]) : 0u;
    uint64_t local = 0;
#pragma unroll
    for (int k = 0; k < kOffRegs; ++k) local += cw[k];
    uint64_t run = wg_scan64(local, total, s_tmp);
#pragma unroll
    for (int k = 0; k < kOffRegs; ++k) {
      if (lo + k < hi) ix.chunk_off[lo + k] = run;
      run += cw[k];
    }
  } else {
    uint64_t local = 0;
    for (uint64_t c = lo; c < hi; ++c) local += ld_dev32(&ix.chunk_words[c]);
    uint64_t run = wg_scan64(local, total, s_tmp);
    for (uint64_t c = lo; c < hi; ++c) {
      ix.chunk_off[c] = run;
      run += ld_dev32(&ix.chunk_words[c]);
    }
  }
  if (tid == 0) {
    if (total != g.payload_bytes / 4) latch(p.s, ST_FORMAT);
    *p.done[which] = 0;
  }
}

struct CompressParams {
  const float* x;
  uint8_t* out;
  Layout g;
  double eb, inv2e;
  float abs_ok;  // abs_bound(eb, inv2e)
  Scratch s;
  hoszp_result* res;
};

// Eq. 3 in binary64: floor(((double)x + eps) * (1 / (2 eps))).
__device__ __forceinline__ double bin_real(float v, double eb, double inv2e) {
  const double shifted = double(v) + eb;
  return floor(shifted * inv2e);
}

// Per-thread exact sums of bins: S = sum q (int64) and Q = sum q^2 (unsigned
// 128-bit as hi:lo).
struct BinSums {
  int64_t s = 0;
  uint64_t ql = 0, qh = 0;
  __device__ __forceinline__ void add(int32_t q) {
    s += q;
    const uint64_t sq = uint64_t(int64_t(q) * int64_t(q));
    ql += sq;
    qh += ql < sq ? 1u : 0u;
  }
  // a segment's sums: s32 = sum of its bins, sq = sum of their squares
  __device__ __forceinline__ void add_segment(int32_t s32, uint64_t sq) {
    s += s32;
    ql += sq;
    qh += ql < sq ? 1u : 0u;
  }
};

// Saturating binary64 -> integer conversions (one VALU op each, NaN -> 0):
// they are only reached with an out-of-range value when the segment's range
// flag is already down, and their results are then never used.
__device__ __forceinline__ uint32_t cvt_abs_u32(double d) {
  uint32_t r;
  asm("v_cvt_u32_f64 %0, |%1|" : "=v"(r) : "v"(d));
  return r;
}
__device__ __forceinline__ int32_t cvt_i32(double d) {
  int32_t r;
  asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(d));
  return r;
}

// Quantize the 32 values of a segment (Eq. 3), form the Lorenzo deltas
// (Eq. 4; slot 0 of a block's first segment is the outlier) and split them
// into sign bits (slot j at bit 31 - j) and magnitudes.  FULL: all 32 slots
// valid.  The deltas are formed in binary64: the bins f_j are integers below
// 2^31 in magnitude, so d = f_j - f_{j-1} is exact and |d| < 2^32 converts
// exactly.
// `prevf` is the bin before the segment (when it does not start its block).
// Range and finiteness are checked by the caller (abs_sum).  STATS: the sum
// of the valid bins and of their squares in binary64, exact when every bin is
// below kSmallBin in magnitude (the caller checks that, again with abs_sum).
template <bool FULL, bool STATS>
__device__ __forceinline__ void quantize_fast(const float* v, uint32_t cnt, bool first_seg,
                                              double prevf, double eb, double inv2e,
                                              uint32_t* mag, uint32_t& sgn, uint32_t& mx,
                                              int32_t& outlier, double& ssum, double& qsum) {
  double fp = prevf;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const double f = bin_real(v[j], eb, inv2e);
    const bool valid = FULL || uint32_t(j) < cnt;
    if (STATS && valid) {
      ssum += f;
      qsum = fma(f, f, qsum);
    }
    // d is +0 when f = fp, so its sign bit is the delta's sign
    const double d = f - fp;
    uint32_t m = cvt_abs_u32(d);
    uint32_t hi = uint32_t(__double2hiint(d));
    if (j == 0) {
      if (first_seg) {
        outlier = cvt_i32(f);
        m = 0;
        hi = 0;
      }
    }
    if (!valid) {
      m = 0;
      hi = 0;
    }
    mag[j] = m;
    // (sgn << 1) | sign bit of d: slot j ends at bit 31 - j
    sgn = __builtin_amdgcn_alignbit(sgn, hi, 31);
    mx = max(mx, m);
    fp = f;
    // one slot at a time: hoisting the independent binary64 chains of later
    // slots only lengthens live ranges (the other waves hide the latency)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Sum of |x| over the valid values of a segment, for the range tests before
// quantize_fast: a rounded sum of non-negative terms is at least each term,
// so sum <= abs_bound(eb, inv2e, K) guarantees every bin is within [-K, K];
// NaN, infinity and overflow fail every such test (the exact classification
// then decides).  Computed before the quantization loop, so the compiler
// cannot sink the tests past it (which would keep every slot's binary64 bin
// live).
template <bool FULL>
__device__ __forceinline__ float abs_sum(const float* v, uint32_t cnt) {
  float a = 0.0f;
#pragma unroll
  for (int j = 0; j < 32; ++j)
    if (FULL || uint32_t(j) < cnt) a += fabsf(v[j]);
  return a;
}

// Error bits of a segment whose quantize_fast failed (reads it again).
__device__ __noinline__ uint32_t segment_errors(const float* xs, uint32_t cnt, double eb,
                                                double inv2e) {
  uint32_t bad = 0;
  for (uint32_t j = 0; j < cnt; ++j) {
    const float xv = xs[j];
    if (!(fabs(bin_real(xv, eb, inv2e)) <= kBinMaxD)) bad |= isfinite(xv) ? ST_RANGE : ST_NONFINITE;
  }
  return bad;
}


// LDS of one compress workgroup.
template <int NT = kThreads>
struct CompressShared {
  uint32_t pay[NT * 32 + 2];
  uint32_t tmp[NT / 64];
  LbShared<NT> lb;
  int64_t rs[NT / 64];
  uint64_t rl[NT / 64], rh[NT / 64];
  uint64_t ticket;
  uint32_t flag;
};

// Compress tile `tile` of the field x (layout g) into `out`: Sec. IV-A
// steps 1-3 and the Fig. 3 sections.  The tile's payload offset comes from
// the decoupled look-back over `st` (one status word per tile of this field).
// Returns the payload words of tiles 0..tile (uniform).  Error bits go to
// `bad`; with STATS the tile's valid bins are added to `sums`.  Thread 0
// takes the workgroup's next ticket from `ticket` into `next`.  Contains
// barriers.
template <int SPB, bool STATS, int NT = kThreads>
__device__ __forceinline__ uint64_t compress_tile(const float* x, uint8_t* out, const Layout& g, double eb,
                                  double inv2e, float abs_ok, float abs_small, uint64_t tile, uint64_t* st, uint32_t epoch,
                                  uint32_t limit, CompressShared<NT>& sh, uint32_t& bad, BinSums& sums,
                                  uint32_t* ticket, uint32_t& next) {
  constexpr uint32_t L = SPB * 32;
  const int tid = threadIdx.x;
  const uint64_t seg = tile * NT + tid;
  const uint64_t ntiles = (g.nseg + NT - 1) / NT;
  const bool active = seg < g.nseg;
  const uint64_t blk = seg / SPB;
  const uint32_t sub = uint32_t(seg % SPB);
  uint64_t blen = 0;
  const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
  const uint64_t first = blk * L + uint64_t(32) * sub;

  uint32_t mag[32];
  uint32_t sgn = 0, mx = 0;
  int32_t outlier = 0;
  if (cnt > 0) {
    // the bin of the slot before this segment, when it is in the same block
    // (an out-of-range one is that slot's own segment's error)
    const double prevf = sub > 0 ? bin_real(x[first - 1], eb, inv2e) : 0.0;
    float v[32];
    float am;
    double ssum = 0.0, qsum = 0.0;
    if (cnt == 32) {
      const float4* src = reinterpret_cast<const float4*>(x + first);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float4 t = src[k];
        v[4 * k + 0] = t.x;
        v[4 * k + 1] = t.y;
        v[4 * k + 2] = t.z;
        v[4 * k + 3] = t.w;
      }
      am = abs_sum<true>(v, cnt);
      if (!(am <= abs_ok)) bad |= segment_errors(x + first, cnt, eb, inv2e);
      quantize_fast<true, STATS>(v, cnt, sub == 0, prevf, eb, inv2e, mag, sgn, mx, outlier, ssum,
                                 qsum);
    } else {
#pragma unroll
      for (int j = 0; j < 32; ++j) v[j] = uint32_t(j) < cnt ? x[first + j] : 0.0f;
      am = abs_sum<false>(v, cnt);
      if (!(am <= abs_ok)) bad |= segment_errors(x + first, cnt, eb, inv2e);
      quantize_fast<false, STATS>(v, cnt, sub == 0, prevf, eb, inv2e, mag, sgn, mx, outlier, ssum,
                                  qsum);
    }
    if (STATS) {
      if (am <= abs_small) {
        sums.add_segment(int32_t(ssum), uint64_t(qsum));
      } else {  // wide bins: rebuild them from the outlier or prev and the deltas
        int32_t q = sub > 0 ? cvt_i32(prevf) : 0;
        for (int j = 0; j < int(cnt); ++j) {
          if (j == 0 && sub == 0) {
            q = outlier;
          } else {
            const uint32_t m = mag[j];
            q = int32_t(((sgn >> (31 - j)) & 1u) ? uint32_t(q) - m : uint32_t(q) + m);
          }
          sums.add(q);
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 32; ++j) mag[j] = 0;
  }
  mx = block_max(mx, SPB);
  const uint32_t w = bitlen32(mx);

  uint32_t tile_words;
  const uint32_t off = wg_scan<NT>(w, tile_words, sh.tmp);
  // Publish the tile's payload size as soon as it is known, then do all work
  // that does not need the tile's offset (packing into LDS, the width,
  // outlier and sign sections) before waiting on the predecessors.
  lb_publish(st, tile, tile_words, epoch);
  const uint32_t group = pack_group(w);
  if (w > 0) pack32_grouped(&sh.pay[off], mag, w, group);
  if (active) {
    if (sub == 0) {
      out[g.off_w + blk] = uint8_t(w);
      reinterpret_cast<int32_t*>(out + g.off_o)[blk] = outlier;
    }
    reinterpret_cast<uint32_t*>(out + g.off_s)[seg] = bswap32(sgn);
  }
  const uint64_t base = lb_wait<NT>(st, tile, tile_words, epoch, sh.lb, limit, bad);
  // The next tile is requested now: its ticket is held only while this tile
  // stores, never while this tile waits on its predecessors.
  if (tid == 0) next = atomicAdd(ticket, 1u);
  __syncthreads();
  uint32_t* P = reinterpret_cast<uint32_t*>(out + g.off_p) + base;
  for (uint32_t k = tid; k < tile_words; k += NT) P[k] = bswap32(sh.pay[k]);
  if (tid == 0 && tile == ntiles - 1) write_header(out, g, 4 * (base + tile_words));
  __syncthreads();
  return base + tile_words;
}

template <int SPB, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_compress(CompressParams p) {
  __shared__ CompressShared<NT> sh;
  const int tid = threadIdx.x;
  const Layout& g = p.g;
  const uint64_t ntiles = (g.nseg + NT - 1) / NT;
  uint32_t bad = 0, next = 0;
  BinSums none;
  const uint32_t epoch = launch_epoch(p.s);
  if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
  for (;;) {
    if (tid == 0) sh.ticket = next;
    __syncthreads();
    const uint64_t tile = uni64(sh.ticket);
    if (tile >= ntiles) break;
    const uint64_t words =
        compress_tile<SPB, false, NT>(p.x, p.out, g, p.eb, p.inv2e, p.abs_ok, 0.0f, tile, p.s.st_out, epoch,
                                      p.s.wait_limit, sh,
                                  bad, none, &p.s.ctrl[C_TICKET], next);
    if (tid == 0 && tile == ntiles - 1) st_dev(&p.s.acc[A_OUT], g.off_p + 4 * words);
  }
  latch(p.s, bad);
  if (finish_arrive(&p.s.ctrl[C_DONE], &sh.flag)) {
    retire_epoch(p.s, epoch);
    publish(p.s, p.res, ld_dev(&p.s.acc[A_OUT]), 0.0);
  }
}

// mean = (S / n) 2 eps and variance = ((n Q - S^2) / n / n) (2 eps)^2 from the
// exact sums (Sec. V-B); n Q - S^2 is formed exactly in 128 bits.
__device__ __forceinline__ void mean_variance(uint64_t n, double eb, int64_t S, uint64_t ql, uint64_t qh,
                              double& mean, double& var) {
  const double two_eb = 2.0 * eb;
  mean = (double(S) / double(n)) * two_eb;
  const uint64_t nql = n * ql;
  const uint64_t nqh = n * qh + __umul64hi(n, ql);
  const uint64_t a = uint64_t(S < 0 ? -S : S);
  const uint64_t sl = a * a, sh = __umul64hi(a, a);
  const uint64_t ml = nql - sl;
  const uint64_t mh = nqh - sh - (nql < sl ? 1u : 0u);
  const double m = u128_to_double(mh, ml);
  var = ((m / double(n)) / double(n)) * (two_eb * two_eb);
}

// ------------------------------------------------------------ batched compress
//
// Many fields in one persistent launch.  The tiles of all fields form one
// work list (field order, then tile order); workgroups take tiles from one
// ticket, so within a field tiles are taken in order and each field runs its
// own look-back over its own range of status words.  Bins are summed exactly
// while they are in registers, so every field's mean and variance come out
// of the same pass.  The workgroup that finishes a field's last outstanding
// tile writes that field's result record and clears its accumulators; the
// last workgroup of the launch clears the launch counters and advances the
// status-word epoch, so the launch can be replayed (a hipGraph) with nothing
// in between.

enum { B_TICKET = 0, B_DONE = 1, B_EPOCH = 2 };
enum { F_S = 0, F_QLO = 1, F_QHI = 2, F_STATUS = 3, F_OUT = 4, F_DONE = 5, F_WORDS = kBatchAccWords };

struct BatchParams {
  const BatchField* fields;
  const uint32_t* tile_field;  // field of every work-list tile
  uint64_t total_tiles;
  uint64_t* st;                // status words, one per work-list tile
  uint32_t* ctrl;              // B_* counters
  uint64_t* facc;              // F_WORDS words per field
  hoszp_field_result* res;     // one record per field
  uint32_t wait_limit;         // look-back poll limit (see lb_wait)
};

// Adds a workgroup's sums and tile count of field f to the field's
// accumulators; the workgroup that completes the field's tile count writes
// the field's result record and clears the accumulators.  Contains barriers.
template <int NT>
__device__ __forceinline__ void batch_flush(const BatchParams& p, uint32_t f, const Layout& g,
                                            BinSums& sums, uint32_t bad, uint32_t count,
                                            CompressShared<NT>& sh) {
  const int tid = threadIdx.x;
  wg_sum_s_q<NT>(sums.s, sums.ql, sums.qh, sh.rs, sh.rl, sh.rh);
  bad = uint32_t(__ballot(bad & ST_RANGE) ? ST_RANGE : 0u) |
        uint32_t(__ballot(bad & ST_NONFINITE) ? ST_NONFINITE : 0u) |
        uint32_t(__ballot(bad & ST_TIMEOUT) ? ST_TIMEOUT : 0u);
  uint64_t* acc = p.facc + uint64_t(f) * F_WORDS;
  if ((tid & 63) == 0 && bad) atomicOr(reinterpret_cast<unsigned int*>(&acc[F_STATUS]), bad);
  if (tid == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&acc[F_S]), (unsigned long long)sums.s);
    const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&acc[F_QLO]),
                                   (unsigned long long)sums.ql);
    const uint64_t carry = (old + sums.ql < old) ? 1u : 0u;
    atomicAdd(reinterpret_cast<unsigned long long*>(&acc[F_QHI]),
              (unsigned long long)(sums.qh + carry));
  }
  if (finish_arrive_n(reinterpret_cast<uint32_t*>(&acc[F_DONE]), count, uint32_t(batch_tiles(g, NT)),
                      &sh.flag) &&
      tid == 0) {
    const uint32_t status = uint32_t(ld_dev(&acc[F_STATUS]));
    const int64_t S = int64_t(ld_dev(&acc[F_S]));
    const uint64_t ql = ld_dev(&acc[F_QLO]), qh = ld_dev(&acc[F_QHI]);
    double mean = 0.0, var = 0.0;
    if (!status) mean_variance(g.n, g.eb, S, ql, qh, mean, var);
    hoszp_field_result* r = &p.res[f];
    r->status = status;
    r->block = g.L;
    r->out_bytes = ld_dev(&acc[F_OUT]);
    r->mean = mean;
    r->variance = var;
    for (int k = 0; k < F_WORDS; ++k) acc[k] = 0;
  }
  sums = BinSums();
}

template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_batch(BatchParams p) {
  __shared__ CompressShared<NT> sh;
  const int tid = threadIdx.x;
  const uint32_t epoch = uni32(ld_dev32(&p.ctrl[B_EPOCH]));
  uint32_t next = 0;
  // sums of the tiles this workgroup has done of field cur since the last
  // flush (consecutive tickets of a workgroup mostly fall in one large field)
  uint32_t cur = kNone, count = 0, bad = 0;
  BinSums sums;
  Layout gc;
  if (tid == 0) next = atomicAdd(&p.ctrl[B_TICKET], 1u);
  for (;;) {
    if (tid == 0) sh.ticket = next;
    __syncthreads();
    const uint64_t t = uni64(sh.ticket);
    const uint32_t f = t < p.total_tiles ? uni32(p.tile_field[t]) : kNone;
    if (f != cur && cur != kNone) {
      batch_flush<NT>(p, cur, gc, sums, bad, count, sh);
      count = 0;
      bad = 0;
    }
    if (f == kNone) break;
    const BatchField fd = p.fields[f];
    Layout g;
    place(g, fd.n, fd.block, fd.eb);
    cur = f;
    gc = g;
    const uint64_t tile = t - fd.tile0;
    uint64_t words = 0;
    switch (g.spb) {
      case 1:
        words = compress_tile<1, true, NT>(fd.x, fd.out, g, fd.eb, fd.inv2e, fd.abs_ok, fd.abs_small, tile, p.st + fd.tile0,
                                       epoch, p.wait_limit, sh, bad, sums, &p.ctrl[B_TICKET], next);
        break;
      case 2:
        words = compress_tile<2, true, NT>(fd.x, fd.out, g, fd.eb, fd.inv2e, fd.abs_ok, fd.abs_small, tile, p.st + fd.tile0,
                                       epoch, p.wait_limit, sh, bad, sums, &p.ctrl[B_TICKET], next);
        break;
      default:  // 4: batches take blocks up to 128 (checked when planned)
        words = compress_tile<4, true, NT>(fd.x, fd.out, g, fd.eb, fd.inv2e, fd.abs_ok, fd.abs_small, tile, p.st + fd.tile0,
                                       epoch, p.wait_limit, sh, bad, sums, &p.ctrl[B_TICKET], next);
        break;
    }
    ++count;
    if (tid == 0 && tile == batch_tiles(g, NT) - 1)
      st_dev(&p.facc[uint64_t(f) * F_WORDS + F_OUT], g.off_p + 4 * words);
  }
  if (finish_arrive_n(&p.ctrl[B_DONE], 1u, gridDim.x, &sh.flag)) {
    const bool wrap = epoch + 1 >= kEpochLimit;  // epochs wrap: clear every status word
    if (wrap)
      for (uint64_t k = tid; k < p.total_tiles; k += NT) p.st[k] = 0;
    if (tid == 0) {
      p.ctrl[B_TICKET] = 0;
      p.ctrl[B_DONE] = 0;
      p.ctrl[B_EPOCH] = wrap ? 1u : epoch + 1;
    }
  }
}

struct DecodeParams {
  const uint8_t* c;
  uint64_t c_bytes;
  float* x;        // kDecompress: output values
  uint64_t n_cap;  // kDecompress: capacity of x; kBlockMean: capacity of means
  Scratch s;
  hoszp_result* res;
  double* means;   // kBlockMean: one mean per block
};

// sum over the set bits b of a 32-bit word of (b + 1)
__device__ __forceinline__ uint32_t weighted_popcount(uint32_t v) {
  return __popc(v) + __popc(v & 0xaaaaaaaau) + 2 * __popc(v & 0xccccccccu) +
         4 * __popc(v & 0xf0f0f0f0u) + 8 * __popc(v & 0xff00ff00u) + 16 * __popc(v & 0xffff0000u);
}

// Fast path of a full segment (32 valid slots, width 1..20) for the mean:
// E = sum_j e_j with e_j the in-segment prefix of the deltas, which equals
// sum_i (32 - i) d_i.  With x_i = m_i XOR (-s_i) = d_i - s_i (s_i the sign
// bit, slot i at bit 31 - i of `signs`):
// E = sum_i (32 - i) x_i + sum_{i: s_i} (32 - i), all in 32-bit integers.
// The same pass also yields D = the delta total (sum_i x_i + popcount(signs),
// slot 0 of a block excluded).  sum_i (32 - i) x_i is accumulated as the sum
// of the running prefixes of x, one dependent add each, so no field value
// outlives its own step.  G fields per 32-bit window (G w <= 32): one LDS
// read and funnel shift serve G fields, each then one shift or bit-field
// extract.
template <int G>
__device__ __forceinline__ int32_t mean_fast(const uint32_t* sp, uint32_t w, uint32_t signs,
                                             bool first_seg, int32_t& D) {
  const uint32_t rs = 32u - w;
  int32_t run = 0, acc = 0;
  auto step = [&](int32_t m, int j) {
    int32_t x = m ^ (int32_t(signs << j) >> 31);
    if (j == 0 && first_seg) x = 0;
    run += x;
    acc += run;
  };
#pragma unroll
  for (int j = 0; j < 32; j += G) {
    const uint32_t win = window_q(sp, field_q(w, uint32_t(j)));  // field j starts at bit j w
    step(int32_t(win >> rs), j);
#pragma unroll
    for (int k = 1; k < G; ++k)  // field j + k: bits 32 - (k+1) w .. 31 - k w of the window
      if (j + k < 32) step(int32_t(__builtin_amdgcn_ubfe(win, rs - uint32_t(k) * w, w)), j + k);
  }
  D = run + int32_t(__popc(signs));
  return acc + int32_t(weighted_popcount(signs));
}

// Fast path of a full segment (width 1..20) for the variance: E = sum e_j
// (int32), E2 = sum e_j^2 (int64), D = delta total; G as for the mean.  With
// G = 4 (w <= 8) every |e_j| <= 32 * 255 = 8160, so each square is below
// 2^26 and the 32 of them sum to at most 2 130 739 200 < 2^31: they are
// formed on the 24-bit multiplier and summed in 32 bits.
template <int G>
__device__ __forceinline__ void var_fast(const uint32_t* sp, uint32_t w, uint32_t sw,
                                         bool first_seg, int32_t& E, int64_t& E2, int32_t& D) {
  const uint32_t rs = 32u - w;
  int32_t e = 0, s1 = 0, s2n = 0;
  int64_t s2 = 0;
  auto step = [&](int32_t m, int j) {
    const int32_t neg = int32_t(sw << j) >> 31;
    int32_t d = (m ^ neg) - neg;
    if (j == 0 && first_seg) d = 0;
    e += d;
    s1 += e;
    if (G == 4)
      s2n += __mul24(e, e);
    else
      s2 += int64_t(e) * e;
  };
#pragma unroll
  for (int j = 0; j < 32; j += G) {
    const uint32_t win = window_q(sp, field_q(w, uint32_t(j)));  // field j starts at bit j w
    step(int32_t(win >> rs), j);
#pragma unroll
    for (int k = 1; k < G; ++k)
      if (j + k < 32) step(int32_t(__builtin_amdgcn_ubfe(win, rs - uint32_t(k) * w, w)), j + k);
  }
  E = s1;
  E2 = G == 4 ? int64_t(s2n) : s2;
  D = e;
}

// Fast path of a full segment (width 1..20) for decompression: the in-segment
// prefixes (modulo 2^32; the bins they lead to are int32).
template <bool PAIR, bool MAD = false>
__device__ __forceinline__ int32_t prefix_fast(const uint32_t* sp, uint32_t w, uint32_t sw,
                                               bool first_seg, int32_t* e_out) {
  const uint32_t rs = 32u - w;
  int32_t e = 0;
  auto step = [&](int32_t m, int j) {
    const int32_t neg = int32_t(sw << j) >> 31;
    int32_t d = (m ^ neg) - neg;
    if (j == 0 && first_seg) d = 0;
    e += d;
    e_out[j] = e;
  };
#pragma unroll
  for (int j = 0; j < 32; j += PAIR ? 2 : 1) {
    // field j starts at bit j w (MAD: on the 24-bit multiplier; the kernels
    // with the most registers in use keep the compiler's own form)
    const uint32_t win = MAD ? window_q(sp, field_q(w, uint32_t(j))) : window_at(sp, __umul24(w, uint32_t(j)));
    step(int32_t(win >> rs), j);
    if (PAIR) step(int32_t(__builtin_amdgcn_ubfe(win, rs - w, w)), j + 1);  // bits 32-2w .. 31-w
  }
  return e;
}

// Generic path: in-segment prefixes e_j of any segment (partial, or width up
// to 32) with 64-bit/128-bit sums; keeps e_j when KEEP.
// (Rare: kept compact rather than fast, so it does not raise the register
// count of the kernels' fast paths.)
template <bool KEEP, typename KT = int64_t>
__device__ __forceinline__ int64_t decode_generic(const uint32_t* sp, uint32_t sw, uint32_t w, uint32_t sub,
                                  uint32_t cnt, int64_t& E, unsigned __int128& E2,
                                  KT* keep) {
  int64_t e = 0;
  E = 0;
  E2 = 0;
  const uint32_t ww = w ? w : 1u;  // with w = 0 every delta is 0 (fields read, then dropped)
  auto step = [&](int j) {
    int64_t d = seg_delta(sp, sw, ww, j);
    if (w == 0 || (j == 0 && sub == 0)) d = 0;  // slot 0 of a block is the outlier
    const bool valid = uint32_t(j) < cnt;
    if (!valid) d = 0;
    e += d;
    if (valid) {
      E += e;
      const uint64_t a = uint64_t(e < 0 ? -e : e);
      E2 += (unsigned __int128)a * a;
    }
  };
  if constexpr (KEEP) {  // keep[] must stay in registers: fully unrolled
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      step(j);
      keep[j] = KT(e);
    }
  } else {
#pragma unroll 2
    for (int j = 0; j < 32; ++j) step(j);
  }
  return e;
}

// Raw loads of a wave tile's metadata, issued two tiles ahead of use: the
// lane's block width and outlier, and the tile's payload offset inputs (its
// chunk's prefix and one per-tile word count per lane).
struct MetaA {
  uint32_t w;
  int32_t outlier;
  uint32_t tw;       // tile_words[chunk * 64 + lane] when lane < tile % 64
  uint64_t chunk_off;
};

// The same tile one step later: scanned widths, sign word and the first
// payload words, issued one tile ahead of use.
// PF payload words per lane are held in registers (measured: 12 for
// decompression, whose tiles then rarely need a second round trip; 8 for the
// reductions, which run at the 128-VGPR cap and lose more to the extra
// registers than they gain).
template <int PF>
struct MetaB {
  uint32_t w, off, words, sw;
  uint32_t wmax;  // largest width of the tile (wave-uniform)
  int32_t outlier;
  uint64_t base;
  uint32_t pf[PF];
};

__device__ __forceinline__ void meta_a(const Layout& g, const uint8_t* W, const int32_t* O,
                                       const TileIndex& ix, uint64_t wt, uint64_t nwt,
                                       MetaA& m) {
  const int lane = threadIdx.x & 63;
  const uint64_t seg = wt * kWaveSegs + lane;
  const bool active = wt < nwt && seg < g.nseg;
  const uint64_t blk = (seg >> g.spb_log2);
  m.w = active ? W[blk] : 0u;
  m.outlier = active ? O[blk] : 0;
  const uint64_t chunk = wt / kChunkTiles;
  const uint32_t r = uint32_t(wt % kChunkTiles);
  m.tw = (wt < nwt && uint32_t(lane) < r) ? ix.tile_words[chunk * kChunkTiles + lane] : 0u;
  const uint64_t nch = num_chunks(g);
  if (nch <= kDirectChunks)  // every lane's chunk total, scanned in meta_b
    m.chunk_off = (wt < nwt && uint32_t(lane) < nch) ? ix.chunk_words[lane] : 0u;
  else
    m.chunk_off = wt < nwt ? ix.chunk_off[chunk] : 0u;
}

template <int PF>
__device__ __forceinline__ void meta_b(const Layout& g, const uint32_t* S, const uint32_t* P,
                                       uint64_t payload_words, uint64_t wt, uint64_t nwt,
                                       const MetaA& a, MetaB<PF>& m, uint32_t& bad) {
  const int lane = threadIdx.x & 63;
  uint32_t w = a.w;
  if (w > 32) {
    bad |= ST_FORMAT;
    w = 0;
  }
  const uint64_t seg = wt * kWaveSegs + lane;
  const uint32_t cnt = wt < nwt ? seg_valid(seg, g.n >> 5, uint32_t(g.n & 31u)) : 0u;
  const uint32_t x = wave_incl_scan(w);  // inclusive scan of the widths over the wave
  m.w = w;
  m.off = x - w;
  m.words = lane_of(x, 63);
  m.wmax = wave_max(w);
  m.outlier = a.outlier;
  uint64_t cbase = a.chunk_off;
  if (num_chunks(g) <= kDirectChunks) {
    uint32_t b2 = 0;
    cbase = direct_chunk_off(uint32_t(a.chunk_off), wt < nwt ? wt / kChunkTiles : 0u, payload_words, b2);
    if (wt < nwt) bad |= b2;
  }
  // a wave tile holds at most 64 x 32 words, so 63 of them sum below 2^17
  m.base = cbase + wave_sum32(a.tw);
  m.sw = (cnt > 0 && w > 0) ? S[seg] : 0u;
  if (m.base + m.words > payload_words) {
    bad |= ST_FORMAT;
    m.words = 0;
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const uint32_t i = uint32_t(lane) + 64u * k;
    m.pf[k] = i < m.words ? P[m.base + i] : 0u;
  }
}

// Decoders: every wave walks its own wave tiles (64 segments) with a static
// stride and stages each tile's payload in its own LDS region, so waves never
// wait on each other.  The loop is software-pipelined: widths, outliers and
// offsets are loaded two tiles ahead, sign words and the first payload words
// one tile ahead, so memory latency overlaps the current tile's arithmetic.
// Workgroup size of the decoders: decompression keeps 32 output values per
// lane (at most 168 VGPRs, 3 waves per SIMD), so 256 threads; the reductions
// fit 128 VGPRs and run one 1024-thread workgroup per CU (the same 16 waves
// per CU as four 256-thread groups, with a quarter of the end-of-kernel
// atomics).
constexpr int kReduceThreads = 1024;
__host__ __device__ constexpr int decode_threads(int mode) {
  return mode == kDecompress ? kThreads : kReduceThreads;
}

template <int MODE>
__global__ void __launch_bounds__(decode_threads(MODE))
    __attribute__((amdgpu_waves_per_eu(MODE == kDecompress ? 3 : 4))) k_decode(DecodeParams p) {
  constexpr int NT = decode_threads(MODE);
  // per-wave payload staging, reused by decompression to transpose its output
  __shared__ __align__(16) uint32_t s_pay[NT / 64][kWaveWords + 4];
  __shared__ uint32_t s_flag;
  __shared__ int64_t s_rs[NT / 64];
  __shared__ uint64_t s_rl[NT / 64], s_rh[NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  Layout g;
  uint32_t err = read_header(p.c, p.c_bytes, g);
  if (!err && MODE == kDecompress && p.n_cap < g.n) err = ST_CAPACITY;
  if (!err && MODE == kBlockMean && p.n_cap < g.nb) err = ST_CAPACITY;
  if (tid == 0 && blockIdx.x == 0) latch(p.s, err);
  const uint64_t nwt = err ? 0 : g.nwtiles;
  const uint8_t* W = p.c + g.off_w;
  const uint32_t* S = reinterpret_cast<const uint32_t*>(p.c + g.off_s);
  const int32_t* O = reinterpret_cast<const int32_t*>(p.c + g.off_o);
  const uint32_t* P = reinterpret_cast<const uint32_t*>(p.c + g.off_p);
  const uint64_t payload_words = g.payload_bytes / 4;
  uint32_t* wp = s_pay[wave];
  const double two_eb = 2.0 * g.eb;
  int64_t acc_s = 0;
  uint64_t acc_ql = 0, acc_qh = 0;
  uint32_t bad = 0, nconst = 0;
  const uint64_t stride = uint64_t(gridDim.x) * (NT / 64);
  const uint64_t wt0 = uint64_t(blockIdx.x) * (NT / 64) + wave;
  const uint64_t nfull = g.n >> 5;  // full segments; the next holds tail slots
  const uint32_t tail = uint32_t(g.n & 31u);
  MetaA a1, a2;
  constexpr int PF = MODE == kDecompress ? 12 : 8;
  MetaB<PF> b0;
  if (wt0 < nwt) {
    MetaA a0;
    meta_a(g, W, O, p.s.idx[0], wt0, nwt, a0);
    meta_a(g, W, O, p.s.idx[0], wt0 + stride, nwt, a1);
    meta_b(g, S, P, payload_words, wt0, nwt, a0, b0, bad);
  }
  for (uint64_t wt = wt0; wt < nwt; wt += stride) {
    meta_a(g, W, O, p.s.idx[0], wt + 2 * stride, nwt, a2);
    // stage this tile's payload (prefetched words first)
    const uint32_t words = b0.words;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const uint32_t i = uint32_t(lane) + 64u * k;
      if (i < words) wp[1 + i] = bswap32(b0.pf[k]);
    }
    for (uint32_t i = lane + 64u * PF; i < words; i += 64)
      wp[1 + i] = bswap32(P[b0.base + i]);
    if (lane == 0) {
      wp[0] = 0;
      wp[1 + words] = 0;
    }
    __builtin_amdgcn_wave_barrier();  // LDS operations of one wave complete in order
    const uint32_t w = b0.w, off = b0.off, sw = bswap32(b0.sw), wmax = b0.wmax;
    const int32_t outlier = b0.outlier;
    // the next tile's sign words and payload are in flight during this tile
    meta_b(g, S, P, payload_words, wt + stride, nwt, a1, b0, bad);
    a1 = a2;

    const uint64_t seg = wt * kWaveSegs + lane;
    const uint64_t blk = (seg >> g.spb_log2);
    const uint32_t sub = uint32_t(seg & (g.spb - 1));
    const uint32_t cnt = seg_valid(seg, nfull, tail);

    const uint32_t* sp = &wp[1 + off];
    const bool fast = cnt == 32 && w <= 20;
    // in-segment sums: D = delta total, E = sum of prefixes, E2 = sum of squares
    int64_t D = 0, E = 0;
    uint64_t E2 = 0;
    unsigned __int128 E2w = 0;
    // decompression keeps the in-segment prefixes modulo 2^32: every bin of a
    // valid stream is an int32, so carry + prefix wraps to the exact bin
    int32_t keep32[MODE == kDecompress ? 32 : 1];
    if (fast) {
      if (w == 0) {
        if (MODE == kDecompress) {
#pragma unroll
          for (int j = 0; j < 32; ++j) keep32[j] = 0;
        }
      } else if (MODE == kMean || MODE == kBlockMean) {
        const uint32_t signs = sub == 0 ? (sw & 0x7fffffffu) : sw;  // slot 0: the outlier
        int32_t d1;
        if (wmax <= 8)
          E = mean_fast<4>(sp, w, signs, sub == 0, d1);
        else if (wmax <= 10)
          E = mean_fast<3>(sp, w, signs, sub == 0, d1);
        else if (wmax <= 16)
          E = mean_fast<2>(sp, w, signs, sub == 0, d1);
        else
          E = mean_fast<1>(sp, w, signs, sub == 0, d1);
        D = d1;
      } else if (MODE == kVariance) {
        int32_t e1, d1;
        int64_t e2;
        if (wmax <= 8)
          var_fast<4>(sp, w, sw, sub == 0, e1, e2, d1);
        else if (wmax <= 10)
          var_fast<3>(sp, w, sw, sub == 0, e1, e2, d1);
        else if (wmax <= 16)
          var_fast<2>(sp, w, sw, sub == 0, e1, e2, d1);
        else
          var_fast<1>(sp, w, sw, sub == 0, e1, e2, d1);
        E = e1;
        E2 = uint64_t(e2);
        D = d1;
      } else {
        // one field per window here: the paired read costs the registers
        // that keep decompression at 3 waves per SIMD
        D = prefix_fast<false, true>(sp, w, sw, sub == 0, keep32);
      }
    } else if (cnt > 0) {
      D = decode_generic<MODE == kDecompress, int32_t>(sp, sw, w, sub, cnt, E, E2w, keep32);
    }
    const int64_t carry = int64_t(outlier) + block_excl(D, g.spb);
    // every bin must be a valid int32 bin (slot 0 is the outlier itself)
    if (cnt > 0 && !bins_in_range_upto(outlier, g.L, w)) {
      int64_t e = 0;
      for (int j = 0; j < int(cnt); ++j) {
        if (w && !(j == 0 && sub == 0)) e += seg_delta(sp, sw, w, j);
        const int64_t bin = carry + e;
        if (bin < -kBinMax || bin > kBinMax) bad |= ST_FORMAT;
      }
    }

    if (MODE == kDecompress) {
      // Bins -> floats, written to LDS in segment order with float4 chunks
      // XOR-swizzled by lane (conflict-free), then stored with consecutive
      // lanes on consecutive 16-byte chunks.  The payload words are no longer
      // needed: the wave has finished reading them.
      __builtin_amdgcn_wave_barrier();
      float* fl = reinterpret_cast<float*>(wp);
      if (cnt > 0) {
        const uint32_t c32 = uint32_t(carry);
        auto val = [&](int j) { return float(double(int32_t(c32 + uint32_t(keep32[j]))) * two_eb); };
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          float4 t;
          t.x = val(4 * k + 0);
          t.y = val(4 * k + 1);
          t.z = val(4 * k + 2);
          t.w = val(4 * k + 3);
          *reinterpret_cast<float4*>(&fl[lane * 32 + 4 * (k ^ (lane & 7))]) = t;
          __builtin_amdgcn_sched_barrier(0);  // convert chunk by chunk (register pressure)
        }
      }
      __builtin_amdgcn_wave_barrier();
      const uint64_t e0 = wt * (uint64_t(kWaveSegs) * 32);
      const uint64_t left = g.n - e0;
      const uint32_t valid = uint32_t(left < uint64_t(kWaveSegs) * 32 ? left : uint64_t(kWaveSegs) * 32);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t q = uint32_t(lane) + 64u * k;  // float4 chunk of the wave tile
        const uint32_t row = q >> 3, ch = q & 7u;
        const float4 v = *reinterpret_cast<const float4*>(&fl[row * 32 + 4 * (ch ^ (row & 7u))]);
        if (4 * q + 4 <= valid) {
          *reinterpret_cast<float4*>(p.x + e0 + 4 * q) = v;
        } else if (4 * q < valid) {
          const float vv[4] = {v.x, v.y, v.z, v.w};
          for (uint32_t t = 0; 4 * q + t < valid; ++t) p.x[e0 + 4 * q + t] = vv[t];
        }
      }
    } else if (MODE == kBlockMean) {
      // block sum = sum over the block's segments (consecutive lanes) of the
      // segment sums cnt * carry + E; slot 0's lane writes the block's mean
      int64_t bs = cnt > 0 ? int64_t(cnt) * carry + E : 0;
      acc_s += bs;
      for (uint32_t m = 1; m < g.spb; m <<= 1) bs += __shfl_xor(bs, int(m), 64);
      if (cnt > 0 && sub == 0) {
        const uint64_t left = g.n - blk * g.L;
        const uint64_t blen = left < g.L ? left : g.L;
        p.means[blk] = (double(bs) / double(blen)) * two_eb;
        nconst += w == 0 ? 1u : 0u;
      }
    } else if (cnt > 0) {
      // bins of the segment: carry + e_j over its cnt valid slots
      acc_s += int64_t(cnt) * carry + E;
      if (MODE == kVariance) {
        const __int128 cc = carry;
        __int128 q = __int128(cnt) * cc * cc + 2 * cc * __int128(E);
        q += fast ? __int128(E2) : __int128(E2w);
        const uint64_t ql = uint64_t(q), qh = uint64_t(q >> 64);
        const uint64_t nl = acc_ql + ql;
        acc_qh += qh + (nl < acc_ql ? 1u : 0u);
        acc_ql = nl;
      }
    }
    __builtin_amdgcn_wave_barrier();  // every lane's LDS reads precede the next staging
  }
  latch(p.s, bad);
  double value = 0.0;
  if (MODE == kBlockMean) {
    nconst = wave_sum32(nconst);
    if (lane == 0 && nconst) atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_CONST]),
                                       (unsigned long long)nconst);
  }
  if (MODE != kDecompress) {
    wg_sum_s_q<NT>(acc_s, acc_ql, acc_qh, s_rs, s_rl, s_rh);
    if (tid == 0) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_S]), (unsigned long long)acc_s);
      if (MODE == kVariance) {
        const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_QLO]),
                                       (unsigned long long)acc_ql);
        const uint64_t carry_out = (old + acc_ql < old) ? 1u : 0u;
        atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_QHI]),
                  (unsigned long long)(acc_qh + carry_out));
      }
    }
  }
  if (!finish_arrive(&p.s.ctrl[C_DONE], &s_flag)) return;
  if (tid == 0 && !err && MODE != kDecompress) {
    const int64_t S_all = int64_t(ld_dev(&p.s.acc[A_S]));
    double mean = 0.0, var = 0.0;
    mean_variance(g.n, g.eb, S_all, ld_dev(&p.s.acc[A_QLO]), ld_dev(&p.s.acc[A_QHI]), mean, var);
    value = MODE == kVariance ? var : mean;
    if (MODE == kBlockMean) p.res->count = ld_dev(&p.s.acc[A_CONST]);
  }
  publish(p.s, p.res, 0, value);
}

struct NegateParams {
  const uint8_t* c;
  uint64_t c_bytes;
  uint8_t* out;
  uint64_t out_cap;
  Scratch s;
  hoszp_result* res;
  double scalar;  // kShift: the scalar s
  int32_t sign;   // kShift: +1 adds the scalar's bin, -1 subtracts it
  int32_t pad;
};

enum { kNegate = 0, kShift = 1 };

// Smallest and largest prefix sum of block `blk`'s deltas (0 included: slot
// 0's bin is the outlier), read one field at a time from the stream's
// payload, found through the width pre-pass index.  The slow path of the
// scalar-shift range check: taken only by blocks whose outlier and width
// allow a bin to leave the range, so one lane decoding its block is enough.
// False when the widths place the block outside the payload (a malformed
// stream, which the width pre-pass also reports): nothing is read then.
__device__ __noinline__ bool block_prefix_range(const uint8_t* c, const Layout& g,
                                                const TileIndex& ix, uint64_t blk, uint32_t w,
                                                uint32_t len, int64_t& lo, int64_t& hi) {
  const uint64_t seg0 = blk << g.spb_log2;
  const uint64_t wt = seg0 / kWaveSegs, chunk = wt / kChunkTiles;
  uint64_t off = 0;
  if (num_chunks(g) <= kDirectChunks)
    for (uint64_t k = 0; k < chunk; ++k) off += ix.chunk_words[k];
  else
    off = ix.chunk_off[chunk];
  for (uint64_t t = chunk * kChunkTiles; t < wt; ++t) off += ix.tile_words[t];
  for (uint64_t b = (wt * kWaveSegs) >> g.spb_log2; b < blk; ++b)
    off += min(uint64_t(c[g.off_w + b]), uint64_t(32)) * g.spb;
  lo = 0;
  hi = 0;
  if (off + uint64_t(w) * g.spb > g.payload_bytes / 4) return false;
  const uint32_t* P = reinterpret_cast<const uint32_t*>(c + g.off_p) + off;
  const uint8_t* S = c + g.off_s + blk * (g.L / 8);
  int64_t e = 0;
  for (uint32_t k = 1; k < len; ++k) {
    const uint32_t bit = k * w, i = bit >> 5, sh = bit & 31u;
    const uint64_t win = (uint64_t(bswap32(P[i])) << 32) | (sh + w > 32 ? bswap32(P[i + 1]) : 0u);
    const uint32_t m = uint32_t((win << sh) >> (64u - w));
    e += ((S[k >> 3] >> (7u - (k & 7u))) & 1u) ? -int64_t(m) : int64_t(m);
    lo = e < lo ? e : lo;
    hi = e > hi ? e : hi;
  }
  return true;
}

// The scalar's bin by Eq. 3, evaluated as for every element (two rounded
// binary64 operations and the floor); ST_RANGE outside the bin range.
__device__ __forceinline__ int64_t scalar_bin(double s, double eb, uint32_t& bad) {
  const double inv = 1.0 / (2.0 * eb);
  const double f = floor((s + eb) * inv);
  if (!(f >= -kBinMaxD && f <= kBinMaxD)) {
    bad |= ST_RANGE;
    return 0;
  }
  return int64_t(f);
}

// Workflow 1 of Sec. V-A on the outliers, streaming the stream in 16-byte
// chunks: widths (summed and range-checked on the way), header, padding and
// payload are copied, and
//   kNegate: outliers negated, sign bits of valid slots of non-constant
//            blocks flipped (Sec. V-A negation);
//   kShift:  the scalar's bin added to (sign -1: subtracted from) every
//            outlier, signs copied (Sec. V-A scalar addition/subtraction);
//            every shifted bin must stay in range: blocks whose outlier and
//            width leave no doubt pass at once, the others are decoded
//            (block_prefix_range, via the width pre-pass index in idx[0]).
// In place (out == c) kShift touches only the width and outlier sections.
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_negate(NegateParams p) {
  __shared__ uint32_t s_flag;
  const int tid = threadIdx.x;
  Layout g;
  uint32_t err = read_header(p.c, p.c_bytes, g);
  if (!err && p.out_cap < g.total_bytes) err = ST_CAPACITY;
  uint32_t bad = 0;
  int64_t delta = 0;
  if (MODE == kShift && !err) delta = p.sign * scalar_bin(p.scalar, g.eb, err);
  if (tid == 0 && blockIdx.x == 0) latch(p.s, err);
  const bool in_place = MODE == kShift && p.out == p.c;
  const uint64_t nfull = err ? 0 : g.total_bytes / 16;  // whole 16-byte chunks
  const uint64_t kbeg = in_place ? g.off_w / 16 : 0, kend = in_place ? g.off_s / 16 : nfull;
  const uint64_t stride = uint64_t(gridDim.x) * kThreads;
  uint64_t wsum = 0;
  const uint4* src = reinterpret_cast<const uint4*>(p.c);
  uint4* dst = reinterpret_cast<uint4*>(p.out);
  const uint32_t* W32 = reinterpret_cast<const uint32_t*>(p.c + g.off_w);  // 16-byte aligned
  const uint64_t w_end = g.off_w + g.nb, o_end = g.off_o + 4 * g.nb, s_end = g.off_s + 4 * g.nseg;
  // Each thread moves kNegUnroll chunks per round, all loaded before any is
  // written (no lane condition on the loads: past the end a thread reloads the
  // last chunk and drops it), so the loads of a round are in flight together;
  // a round's loads are issued before the previous round's stores, so they
  // are in flight while that round is processed and written.
  constexpr int kNegUnroll = 4;
  // one round's chunks, and for each the aligned width word of its blocks
  auto load_round = [&](uint64_t k0, uint4* v, uint32_t* wq) {
#pragma unroll
    for (int u = 0; u < kNegUnroll; ++u) {
      const uint64_t k = min(k0 + uint64_t(u) * stride, kend - 1);
      v[u] = src[k];
      const uint64_t o = 16 * k;
      if (MODE == kNegate) {
        // a sign chunk's four segments are consecutive and start at a
        // multiple of 4, so their blocks lie in one aligned word of widths
        const uint64_t sg = (o >= g.off_s && o < s_end) ? (o - g.off_s) / 4 : 0;
        wq[u] = W32[(sg >> g.spb_log2) >> 2];
      } else {
        // an outlier chunk's four blocks start at a multiple of 4
        const uint64_t b0 = (o >= g.off_o && o < o_end) ? (o - g.off_o) / 4 : 0;
        wq[u] = W32[b0 >> 2];
      }
    }
  };
  uint4 v[kNegUnroll];
  uint32_t wq[kNegUnroll];
  uint64_t k0 = kbeg + uint64_t(blockIdx.x) * kThreads + tid;
  if (k0 < kend) load_round(k0, v, wq);
  for (; k0 < kend; k0 += kNegUnroll * stride) {
    uint4 nv[kNegUnroll];
    uint32_t nwq[kNegUnroll];
    load_round(k0 + kNegUnroll * stride, nv, nwq);  // (clamped to the last chunk past the end)
#pragma unroll
    for (int u = 0; u < kNegUnroll; ++u) {
      const uint64_t k = k0 + uint64_t(u) * stride;
      if (k >= kend) continue;
      const uint64_t o = 16 * k;
      uint32_t wd[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
      if (o >= g.off_p || o + 16 <= g.off_w) {
        // header or payload: copy
      } else if (o < g.off_o) {  // widths (and the padding after them)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint64_t b0 = o + 4 * q;
          uint32_t x = wd[q];
          if (b0 >= w_end) continue;
          if (b0 + 4 > w_end) x &= 0xffffffffu >> (8 * (b0 + 4 - w_end));
          if ((x | ((x & 0x7f7f7f7fu) + 0x5f5f5f5fu)) & 0x80808080u) bad |= ST_FORMAT;
          wsum += __builtin_amdgcn_sad_u8(x, 0u, 0u);
        }
      } else if (o < g.off_s) {  // outliers
        if (MODE == kNegate) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (o + 4 * q < o_end) wd[q] = 0u - wd[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (o + 4 * q >= o_end) continue;
            const uint64_t blk = (o - g.off_o) / 4 + q;
            const int64_t ov = int32_t(wd[q]);
            const uint32_t w = min((wq[u] >> (8 * q)) & 0xffu, 32u);
            uint64_t blen = g.L;
            if (blk == g.nb - 1) (void)seg_count(g, blk, 0, blen);
            if (!bins_surely_in_range(ov, blen, w) || !bins_surely_in_range(ov + delta, blen, w)) {
              int64_t lo = 0, hi = 0;
              if (w > 0 && !block_prefix_range(p.c, g, p.s.idx[0], blk, w, uint32_t(blen), lo, hi))
                bad |= ST_FORMAT;
              if (ov + lo < -kBinMax || ov + hi > kBinMax) bad |= ST_FORMAT;
              else if (ov + delta + lo < -kBinMax || ov + delta + hi > kBinMax) bad |= ST_RANGE;
            }
            wd[q] = uint32_t(int32_t(ov + delta));
          }
        }
      } else if (MODE == kNegate) {  // signs
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint64_t b0 = o + 4 * q;
          if (b0 >= s_end) continue;
          const uint64_t seg = (b0 - g.off_s) / 4;
          const uint64_t blk = (seg >> g.spb_log2);
          if (((wq[u] >> (8 * (blk & 3))) & 0xffu) == 0) continue;  // constant block: no signs
          uint32_t cnt = 32;
          if (blk == g.nb - 1) {
            uint64_t blen;
            cnt = seg_count(g, blk, uint32_t(seg & (g.spb - 1)), blen);
          }
          if (cnt == 0) continue;
          const uint32_t be = cnt == 32 ? 0xffffffffu : ~(0xffffffffu >> cnt);
          wd[q] ^= bswap32(be);
        }
      }
      dst[k] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
    }
#pragma unroll
    for (int u = 0; u < kNegUnroll; ++u) {
      v[u] = nv[u];
      wq[u] = nwq[u];
    }
  }
  // the last partial chunk (payload words only): one thread
  if (!err && !in_place && blockIdx.x == 0 && tid == 0)
    for (uint64_t b = 16 * nfull; b < g.total_bytes; b += 4)
      *reinterpret_cast<uint32_t*>(p.out + b) = *reinterpret_cast<const uint32_t*>(p.c + b);
  latch(p.s, bad);
  wsum = wave_sum(wsum);
  if ((tid & 63) == 0 && wsum)
    atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_WSUM]), (unsigned long long)wsum);
  if (!finish_arrive(&p.s.ctrl[C_DONE], &s_flag)) return;
  if (tid == 0 && !err && ld_dev(&p.s.acc[A_WSUM]) * (g.L / 8) != g.payload_bytes)
    atomicOr(&p.s.ctrl[C_STATUS], ST_FORMAT);
  publish(p.s, p.res, err ? 0 : g.total_bytes, 0.0);
}

struct AddParams {
  const uint8_t* a;
  uint64_t a_bytes;
  const uint8_t* b;
  uint64_t b_bytes;
  uint8_t* out;
  uint64_t out_cap;
  Scratch s;
  hoszp_result* res;
};

// Element-wise addition (Sec. V-C), one tile of NT segments per workgroup;
// SUB: element-wise subtraction A - B, the same with B's outlier negated and
// the signs of B's deltas inverted.  The two operands' payloads share one
// tile's LDS buffer: both at once when their words fit (B right after A),
// else one after the other (A's magnitudes held in registers while B's
// payload replaces A's), so the workgroup never needs two tiles of LDS.
template <int NT, bool SUB>
__global__ void __launch_bounds__(NT) k_add(AddParams p) {
  __shared__ uint32_t s_pay[NT * 32 + 2];
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint64_t s_ticket, s_base_a, s_base_b;
  __shared__ uint32_t s_flag;
  __shared__ LbShared<NT> s_lb;
  const int tid = threadIdx.x;
  Layout g, gb;
  uint32_t err = read_header(p.a, p.a_bytes, g);
  if (!err) err = read_header(p.b, p.b_bytes, gb);
  if (!err && (g.n != gb.n || g.L != gb.L ||
               __double_as_longlong(g.eb) != __double_as_longlong(gb.eb)))
    err = ST_MISMATCH;
  if (!err && p.out_cap < bound_bytes(g.n, g.L)) err = ST_CAPACITY;
  if (tid == 0 && blockIdx.x == 0) latch(p.s, err);
  const uint64_t ntiles = err ? 0 : (g.nseg + NT - 1) / NT;
  const uint32_t* Sa = reinterpret_cast<const uint32_t*>(p.a + g.off_s);
  const uint32_t* Sb = reinterpret_cast<const uint32_t*>(p.b + gb.off_s);
  const int32_t* Oa = reinterpret_cast<const int32_t*>(p.a + g.off_o);
  const int32_t* Ob = reinterpret_cast<const int32_t*>(p.b + gb.off_o);
  uint32_t next = 0;
  const uint32_t epoch = launch_epoch(p.s);
  if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
  for (;;) {
    if (tid == 0) s_ticket = next;
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= ntiles) break;
    if (tid < 64) {
      uint32_t b2 = 0;
      const uint64_t v = tile_offset(p.s.idx[0], (NT / kWaveSegs) * tile, g, b2);
      if (tid == 0) {
        s_base_a = v;
        latch(p.s, b2);
      }
    } else if (tid < 128) {
      uint32_t b2 = 0;
      const uint64_t v = tile_offset(p.s.idx[1], (NT / kWaveSegs) * tile, gb, b2);
      if (tid == 64) {
        s_base_b = v;
        latch(p.s, b2);
      }
    }
    const uint64_t seg = tile * NT + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = (seg >> g.spb_log2);
    const uint32_t sub = uint32_t(seg & (g.spb - 1));
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    // per-segment metadata: every lane loads (an inactive lane block 0's,
    // then drops it), so the loads carry no condition and overlap
    const uint64_t mblk = active ? blk : 0, mseg = active ? seg : 0;
    const int32_t oa32 = Oa[mblk], ob32 = Ob[mblk];
    const uint32_t wa8 = p.a[g.off_w + mblk], wb8 = p.b[gb.off_w + mblk];
    const uint32_t swa8 = Sa[mseg], swb8 = Sb[mseg];
    const int64_t oa = active ? oa32 : 0;
    const int64_t ob = active ? (SUB ? -int64_t(ob32) : int64_t(ob32)) : 0;
    uint32_t bad = 0;
    // widths of both operands, scanned together in the 16-bit halves of one
    // word (a tile holds at most 32 NT payload words per operand)
    static_assert(NT * 32 < 65536, "tile word counts must fit 16 bits");
    uint32_t wa = active ? wa8 : 0u, wb = active ? wb8 : 0u;
    if (wa > 32 || wb > 32) {
      bad |= ST_FORMAT;
      wa = wa > 32 ? 0u : wa;
      wb = wb > 32 ? 0u : wb;
    }
    uint32_t tw2;
    const uint32_t off2 = wg_scan<NT>(wa | (wb << 16), tw2, s_tmp);  // its barriers publish the bases
    const uint32_t off_a = off2 & 0xffffu, off_b = off2 >> 16;
    const uint32_t tw_a = tw2 & 0xffffu, tw_b = tw2 >> 16;
    const uint32_t* Pa = reinterpret_cast<const uint32_t*>(p.a + g.off_p);
    const uint32_t* Pb = reinterpret_cast<const uint32_t*>(p.b + gb.off_p);
    // both payloads in LDS at once when they fit (B right after A's guard
    // word), so their loads are in flight together; else B replaces A later
    const bool both = tw_a + tw_b + 1 <= uint32_t(NT * 32);
    const uint64_t base_a = uni64(s_base_a), base_b = uni64(s_base_b);
    const bool fits_a = base_a + tw_a <= g.payload_bytes / 4;
    const bool fits_b = base_b + tw_b <= gb.payload_bytes / 4;
    if (!fits_a || !fits_b) bad |= ST_FORMAT;  // then nothing is read
    if (both)
      stage_words<NT, false>(s_pay, Pa + base_a, fits_a && fits_b ? tw_a : 0u, Pb + base_b,
                      fits_a && fits_b ? tw_b : 0u);
    else
      stage_words<NT, false>(s_pay, Pa + base_a, fits_a ? tw_a : 0u, nullptr, 0u);
    const uint32_t swa = (cnt > 0 && wa) ? bswap32(swa8) : 0u;
    const uint32_t swb = (cnt > 0 && wb) ? (SUB ? ~bswap32(swb8) : bswap32(swb8)) : 0u;
    __syncthreads();
    // operand A's magnitudes are kept in registers
    uint32_t ma[32];
    {
      const uint32_t* sp = &s_pay[1 + off_a];
      const uint32_t rs = 32u - wa;
      uint32_t pa = 0;
      if (wa == 0) {
#pragma unroll
        for (int j = 0; j < 32; ++j) ma[j] = 0;
      } else if (wa <= 16) {  // two whole fields per 32-bit window
#pragma unroll
        for (int j = 0; j < 32; j += 2) {
          const uint32_t win = window_at(sp, pa);
          pa += 2 * wa;
          ma[j] = win >> rs;
          ma[j + 1] = __builtin_amdgcn_ubfe(win, rs - wa, wa);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          ma[j] = field_at(sp, pa, rs);
          pa += wa;
        }
      }
    }
    const uint32_t* spb = &s_pay[tw_a + 2 + off_b];
    if (!both) {
      __syncthreads();  // every lane is done reading A
      stage_words<NT, false>(s_pay, Pb + base_b, fits_b ? tw_b : 0u, nullptr, 0u);
      __syncthreads();
      spb = &s_pay[1 + off_b];
    }

    // O_{A+B} = O_A + O_B, P_{A+B} = P_A + P_B (signed), then re-encode
    const int64_t oz = oa + ob;
    uint32_t mag[32];
    uint32_t sgn = 0, mx = 0;
    int64_t D = 0;
    if (cnt == 32 && wa <= 30 && wb <= 30) {
      // |d_A + d_B| < 2^31: 32-bit arithmetic
      const uint32_t rb = 32u - wb;
      uint32_t pb = 0;
      int32_t dsum = 0;
      auto step = [&](int j, int32_t fb) {  // fb: B's magnitude of slot j
        // sign masks (0 or -1): d = (m_A ^ s_A) - s_A + (m_B ^ s_B) - s_B
        const int32_t sa = int32_t(swa << j) >> 31, sb = int32_t(swb << j) >> 31;
        int32_t d = ((int32_t(ma[j]) ^ sa) + (fb ^ sb)) - (sa + sb);
        if (j == 0 && sub == 0) d = 0;
        const uint32_t m = uint32_t(d < 0 ? -d : d);
        mag[j] = m;
        sgn = __builtin_amdgcn_alignbit(sgn, uint32_t(d), 31);  // shift in d's sign: slot j ends at bit 31 - j
        mx = max(mx, m);
        dsum += d;
      };
      if (__all(wb >= 1 && wb <= 16)) {  // wave-uniform: two B fields per window
#pragma unroll
        for (int j = 0; j < 32; j += 2) {
          const uint32_t win = window_at(spb, pb);
          pb += 2 * wb;
          step(j, int32_t(win >> rb));
          step(j + 1, int32_t(__builtin_amdgcn_ubfe(win, rb - wb, wb)));
        }
      } else {
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          int32_t fb = 0;
          if (wb) fb = int32_t(field_at(spb, pb, rb));
          pb += wb;
          step(j, fb);
        }
      }
      D = dsum;
    } else {
      bool wide = false;
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        int64_t d = ((swa >> (31 - j)) & 1u) ? -int64_t(ma[j]) : int64_t(ma[j]);
        if (wb) d += seg_delta(spb, swb, wb, j);
        if ((j == 0 && sub == 0) || uint32_t(j) >= cnt) d = 0;
        const bool neg = d < 0;
        const uint64_t a = uint64_t(neg ? -d : d);
        // |d| >= 2^32 means some bin of the sum is out of range
        wide |= (a >> 32) != 0;
        const uint32_t m = uint32_t(a);
        mag[j] = m;
        sgn |= uint32_t(neg) << (31 - j);
        mx = max(mx, m);
        D += d;
      }
      if (wide) bad |= ST_RANGE;
    }
    // every bin of the sum must stay in range (checked from the sum's own
    // deltas, so A's magnitudes need not outlive the loop above)
    const int64_t carry = oz + block_excl(D, g.spb);
    if (cnt > 0) {
      const uint64_t aa = uint64_t(oa < 0 ? -oa : oa), ab = uint64_t(ob < 0 ? -ob : ob);
      const uint64_t sa = (uint64_t(1) << wa) - 1, sb = (uint64_t(1) << wb) - 1;
      if (aa + ab + (blen - 1) * (sa + sb) > uint64_t(kBinMax)) {
        int64_t e = 0;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          e += ((sgn >> (31 - j)) & 1u) ? -int64_t(mag[j]) : int64_t(mag[j]);
          const int64_t bin = carry + e;
          if (uint32_t(j) < cnt && (bin < -kBinMax || bin > kBinMax)) bad |= ST_RANGE;
        }
      }
    }
    latch(p.s, bad);
    mx = block_max(mx, g.spb);
    const uint32_t w = bitlen32(mx);
    uint32_t tw_z;
    const uint32_t off_z = wg_scan<NT>(w, tw_z, s_tmp);  // barriers: all threads done reading B
    // publish the output tile's size, then pack and store what needs no offset
    lb_publish(p.s.st_out, tile, tw_z, epoch);
    const uint32_t group = pack_group(w);
    if (w > 0) pack32_grouped(&s_pay[off_z], mag, w, group);
    if (active) {
      if (sub == 0) {
        p.out[g.off_w + blk] = uint8_t(w);
        reinterpret_cast<int32_t*>(p.out + g.off_o)[blk] = int32_t(oz);
      }
      reinterpret_cast<uint32_t*>(p.out + g.off_s)[seg] = bswap32(sgn);
    }
    const uint64_t base_z = lb_wait<NT>(p.s.st_out, tile, tw_z, epoch, s_lb, p.s.wait_limit, bad);
    if (tid == 0) latch(p.s, bad & ST_TIMEOUT);
    if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
    __syncthreads();
    uint32_t* Pz = reinterpret_cast<uint32_t*>(p.out + g.off_p) + base_z;
    for (uint32_t k = tid; k < tw_z; k += NT) Pz[k] = bswap32(s_pay[k]);
    if (tid == 0 && tile == ntiles - 1) {
      const uint64_t payload = 4 * (base_z + tw_z);
      write_header(p.out, g, payload);
      st_dev(&p.s.acc[A_OUT], g.off_p + payload);
    }
    __syncthreads();
  }
  if (finish_arrive(&p.s.ctrl[C_DONE], &s_flag)) {
    retire_epoch(p.s, epoch);
    publish(p.s, p.res, ld_dev(&p.s.acc[A_OUT]), 0.0);
  }
}

struct MulParams {
  const uint8_t* c;
  uint64_t c_bytes;
  uint8_t* out;
  uint64_t out_cap;
  MulScalar k;
  Scratch s;
  hoszp_result* res;
};

// Scale a segment's bins front to back and turn each at once into its output
// delta's magnitude and sign, so an input bin dies as its delta is made.
// The scaled bins z_j = mul_round(s, q_j) are integers, so the delta
// z_j - z_{j-1} is exact in binary64 while both are bins (|z| <= 2^31 - 1),
// and one conversion of its absolute value and one funnel shift of its sign
// bit give the magnitude and the sign word (slot j at bit 31 - j; slot 0's
// bit is left 0).  The range test is a running maximum of |z_j|.  Slot 0's
// delta needs the previous segment's last scaled bin: its scaled bin is
// returned in z0 and its magnitude left for the caller.  FULL: every lane of
// the wave holds 32 valid slots, so no slot needs a bounds test.
template <bool FULL>
__device__ __forceinline__ void scale_deltas(const int32_t* r, uint32_t c32, uint32_t cnt, double s,
                                             uint32_t* mag, uint32_t& sgn, uint32_t& mx,
                                             int32_t& z0, int32_t& zl, uint32_t& bad) {
  double zp = (FULL || cnt > 0) ? mul_round(s, double(int32_t(c32 + uint32_t(r[0])))) : 0.0;
  double zmax = fabs(zp);
  z0 = cvt_i32(zp);
  mag[0] = 0;
#pragma unroll
  for (int j = 1; j < 32; ++j) {
    uint32_t m = 0, hi = 0;
    if (FULL || uint32_t(j) < cnt) {
      const double z = mul_round(s, double(int32_t(c32 + uint32_t(r[j]))));
      const double d = z - zp;
      m = cvt_abs_u32(d);
      hi = uint32_t(__double2hiint(d));  // d is +0 when z = zp
      zmax = fmax(zmax, fabs(z));
      zp = z;
    }
    mag[j] = m;
    sgn = __builtin_amdgcn_alignbit(sgn, hi, 31);
    mx = max(mx, m);
    __builtin_amdgcn_sched_barrier(0);  // one slot at a time (live ranges)
  }
  if (!(zmax <= kBinMaxD)) bad |= ST_RANGE;
  zl = cvt_i32(zp);
}

// Scalar multiplication, one tile of NT segments per workgroup: decode the
// bins (in-segment prefixes kept modulo 2^32: every bin of a valid stream is
// an int32, so carry + prefix wraps to the exact bin), scale them, and
// re-encode with the output look-back.
template <int NT>
__global__ void __launch_bounds__(NT) k_mul(MulParams p) {
  __shared__ uint32_t s_pay[NT * 32 + 2];
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint64_t s_ticket, s_base;
  __shared__ uint32_t s_flag;
  __shared__ LbShared<NT> s_lb;
  const int tid = threadIdx.x;
  Layout g;
  uint32_t err = read_header(p.c, p.c_bytes, g);
  if (!err && p.out_cap < bound_bytes(g.n, g.L)) err = ST_CAPACITY;
  if (tid == 0 && blockIdx.x == 0) latch(p.s, err);
  const uint64_t ntiles = err ? 0 : (g.nseg + NT - 1) / NT;
  const uint32_t* S = reinterpret_cast<const uint32_t*>(p.c + g.off_s);
  const int32_t* O = reinterpret_cast<const int32_t*>(p.c + g.off_o);
  uint32_t next = 0;
  const uint32_t epoch = launch_epoch(p.s);
  if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
  for (;;) {
    if (tid == 0) s_ticket = next;
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= ntiles) break;
    if (tid < 64) {
      uint32_t b2 = 0;
      const uint64_t v = tile_offset(p.s.idx[0], (NT / kWaveSegs) * tile, g, b2);
      if (tid == 0) {
        s_base = v;
        latch(p.s, b2);
      }
    }
    const uint64_t seg = tile * NT + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = (seg >> g.spb_log2);
    const uint32_t sub = uint32_t(seg & (g.spb - 1));
    // per-segment metadata: every lane loads (an inactive lane block 0's,
    // then drops it), so the loads carry no condition and overlap
    const uint64_t mblk = active ? blk : 0, mseg = active ? seg : 0;
    const int32_t o32 = O[mblk];
    const uint32_t w8 = p.c[g.off_w + mblk];
    const uint32_t s32 = S[mseg];
    uint32_t bad = 0;
    uint32_t w = active ? w8 : 0u;
    if (w > 32) {
      bad |= ST_FORMAT;
      w = 0;
    }
    uint32_t tile_words;
    const uint32_t off = wg_scan<NT>(w, tile_words, s_tmp);  // its barriers publish s_base
    const uint32_t* P = reinterpret_cast<const uint32_t*>(p.c + g.off_p);
    if (!stage_payload<NT>(s_pay, P, uni64(s_base), tile_words, g.payload_bytes / 4)) bad |= ST_FORMAT;
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    const int32_t outlier = active ? o32 : 0;
    const uint32_t sw = (cnt > 0 && w > 0) ? bswap32(s32) : 0u;
    __syncthreads();

    // inverse BF + inverse LZ: in-segment prefixes of the bins
    const uint32_t* sp = &s_pay[1 + off];
    int32_t r[32];
    int64_t D = 0;
    if (cnt == 32 && w <= 20) {
      if (w == 0) {
#pragma unroll
        for (int j = 0; j < 32; ++j) r[j] = 0;
      } else {
        D = w <= 16 ? prefix_fast<true>(sp, w, sw, sub == 0, r)
                    : prefix_fast<false>(sp, w, sw, sub == 0, r);
      }
    } else if (cnt > 0) {
      int64_t E = 0;
      unsigned __int128 E2w = 0;
      D = decode_generic<true, int32_t>(sp, sw, w, sub, cnt, E, E2w, r);
    } else {
#pragma unroll
      for (int j = 0; j < 32; ++j) r[j] = 0;
    }
    const int64_t carry = int64_t(outlier) + block_excl(D, g.spb);
    // every input bin must be a valid int32 bin (slot 0 is the outlier itself)
    if (cnt > 0 && !bins_surely_in_range(outlier, blen, w)) {
      int64_t e = 0;
      for (int j = 0; j < int(cnt); ++j) {
        if (w && !(j == 0 && sub == 0)) e += seg_delta(sp, sw, w, j);
        const int64_t bin = carry + e;
        if (bin < -kBinMax || bin > kBinMax) bad |= ST_FORMAT;
      }
    }
    // scaled bins and the output deltas (a zero multiplier scales by exactly 0)
    const uint32_t c32 = uint32_t(carry);
    const double sc = p.k.zero ? 0.0 : p.k.s;
    uint32_t sgn = 0, mx = 0;
    uint32_t mag[32];
    int32_t z0, zp;
    if (__all(cnt == 32))
      scale_deltas<true>(r, c32, cnt, sc, mag, sgn, mx, z0, zp, bad);
    else
      scale_deltas<false>(r, c32, cnt, sc, mag, sgn, mx, z0, zp, bad);
    // last scaled bin of the previous segment of the same block (a segment
    // with valid slots after the first always follows a full segment)
    const int32_t prev = __shfl_up(zp, 1, 64);
    int32_t outlier_z = 0;
    if (cnt > 0) {
      if (sub == 0) {
        outlier_z = z0;
      } else {
        bool neg = false;
        mag[0] = delta_mag(z0, prev, neg);
        sgn |= uint32_t(neg) << 31;
        mx = max(mx, mag[0]);
      }
    }
    latch(p.s, bad);
    mx = block_max(mx, g.spb);
    const uint32_t wz = bitlen32(mx);
    uint32_t tw_z;
    const uint32_t off_z = wg_scan<NT>(wz, tw_z, s_tmp);
    // publish the output tile's size, then pack and store what needs no offset
    lb_publish(p.s.st_out, tile, tw_z, epoch);
    if (wz > 0) pack32(&s_pay[off_z], mag, wz);
    if (active) {
      if (sub == 0) {
        p.out[g.off_w + blk] = uint8_t(wz);
        reinterpret_cast<int32_t*>(p.out + g.off_o)[blk] = outlier_z;
      }
      reinterpret_cast<uint32_t*>(p.out + g.off_s)[seg] = bswap32(sgn);
    }
    const uint64_t base_z = lb_wait<NT>(p.s.st_out, tile, tw_z, epoch, s_lb, p.s.wait_limit, bad);
    if (tid == 0) latch(p.s, bad & ST_TIMEOUT);
    if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
    __syncthreads();
    uint32_t* Pz = reinterpret_cast<uint32_t*>(p.out + g.off_p) + base_z;
    for (uint32_t k = tid; k < tw_z; k += NT) Pz[k] = bswap32(s_pay[k]);
    if (tid == 0 && tile == ntiles - 1) {
      const uint64_t payload = 4 * (base_z + tw_z);
      write_header(p.out, g, payload);
      st_dev(&p.s.acc[A_OUT], g.off_p + payload);
    }
    __syncthreads();
  }
  if (finish_arrive(&p.s.ctrl[C_DONE], &s_flag)) {
    retire_epoch(p.s, epoch);
    publish(p.s, p.res, ld_dev(&p.s.acc[A_OUT]), 0.0);
  }
}

// ------------------------------------------ bivariate: Hadamard, covariance

struct BivarParams {
  const uint8_t* a;
  uint64_t a_bytes;
  const uint8_t* b;
  uint64_t b_bytes;
  uint8_t* out;  // Hadamard only
  uint64_t out_cap;
  Scratch s;
  hoszp_result* res;
};

enum { kHadamard = 0, kCovariance = 1 };
constexpr int kBivarThreads = 512;

// floor(2 eps P + 1/2) for an integer P (|P| < 2^62) in exact integer
// arithmetic, with 2 eps = M 2^-sh (M < 2^53): the 128-bit product M |P|,
// the rounding half 2^(sh-1) (minus one for negative P, so that the shift
// rounds the magnitude towards the floor of the signed value), a shift.
// ST_RANGE when the result leaves the bin range.
__device__ __forceinline__ int32_t product_bin(int64_t P, uint64_t M, int sh, uint32_t& bad) {
  if (P == 0) return 0;
  if (sh <= 0) {  // 2 eps >= 2^52: any non-zero product is far out of range
    bad |= ST_RANGE;
    return 0;
  }
  if (sh > 120) return 0;  // |2 eps P| < 2^-5
  const bool neg = P < 0;
  const uint64_t a = neg ? 0u - uint64_t(P) : uint64_t(P);
  const unsigned __int128 t = (unsigned __int128)M * a;  // < 2^115
  const unsigned __int128 r =
      (t + ((unsigned __int128)1 << (sh - 1)) - (neg ? 1u : 0u)) >> sh;
  if (r > (unsigned __int128)kBinMax) {
    bad |= ST_RANGE;
    return 0;
  }
  return neg ? -int32_t(uint32_t(r)) : int32_t(uint32_t(r));
}

// In-segment prefixes (modulo 2^32) of a staged segment's deltas into r[32];
// returns the segment's delta total.  Also checks, when the outlier and width
// allow it, that every bin is a valid int32 bin (ST_FORMAT otherwise).
__device__ __forceinline__ int64_t segment_prefixes(const uint32_t* sp, uint32_t w, uint32_t sw,
                                                    uint32_t sub, uint32_t cnt, int32_t* r) {
  int64_t D = 0;
  if (cnt == 32 && w <= 20) {
    if (w == 0) {
#pragma unroll
      for (int j = 0; j < 32; ++j) r[j] = 0;
    } else {
      D = w <= 16 ? prefix_fast<true>(sp, w, sw, sub == 0, r) : prefix_fast<false>(sp, w, sw, sub == 0, r);
    }
  } else if (cnt > 0) {
    int64_t E = 0;
    unsigned __int128 E2w = 0;
    D = decode_generic<true, int32_t>(sp, sw, w, sub, cnt, E, E2w, r);
  } else {
#pragma unroll
    for (int j = 0; j < 32; ++j) r[j] = 0;
  }
  return D;
}

__device__ __forceinline__ void check_bins(const uint32_t* sp, uint32_t sw, uint32_t w, uint32_t sub,
                                           uint32_t cnt, int64_t outlier, int64_t carry,
                                           uint64_t blen, uint32_t& bad) {
  if (cnt > 0 && !bins_surely_in_range(outlier, blen, w)) {
    int64_t e = 0;
    for (int j = 0; j < int(cnt); ++j) {
      if (w && !(j == 0 && sub == 0)) e += seg_delta(sp, sw, w, j);
      const int64_t bin = carry + e;
      if (bin < -kBinMax || bin > kBinMax) bad |= ST_FORMAT;
    }
  }
}

// Bivariate operations on two streams of equal n and block size (Sec. V-C,
// V-D), one tile of NT segments per workgroup: both operands' bins are
// decoded (payloads staged one after the other in one LDS buffer, A's bins
// held in registers), then
//   kHadamard:   bins floor(2 eps q_A q_B + 1/2) re-encoded with the output
//                look-back, as scalar multiplication does (equal eps needed);
//   kCovariance: exact sums S_A, S_B (int64) and P = sum q_A q_B (128-bit),
//                and the last workgroup forms the population covariance.
template <int MODE, int NT>
__global__ void __launch_bounds__(NT) k_bivar(BivarParams p) {
  __shared__ uint32_t s_pay[NT * 32 + 2];
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint64_t s_ticket, s_base_a, s_base_b;
  __shared__ uint32_t s_flag;
  __shared__ LbShared<NT> s_lb;
  __shared__ int64_t s_rs[NT / 64];
  __shared__ uint64_t s_rl[NT / 64], s_rh[NT / 64];
  const int tid = threadIdx.x;
  Layout g, gb;
  uint32_t err = read_header(p.a, p.a_bytes, g);
  if (!err) err = read_header(p.b, p.b_bytes, gb);
  if (!err && (g.n != gb.n || g.L != gb.L ||
               (MODE == kHadamard && __double_as_longlong(g.eb) != __double_as_longlong(gb.eb))))
    err = ST_MISMATCH;
  if (MODE == kHadamard && !err && p.out_cap < bound_bytes(g.n, g.L)) err = ST_CAPACITY;
  if (tid == 0 && blockIdx.x == 0) latch(p.s, err);
  const uint64_t ntiles = err ? 0 : (g.nseg + NT - 1) / NT;
  // 2 eps = M 2^-sh from its binary64 fields (2 eps is finite and > 0)
  const uint64_t eb_bits = uint64_t(__double_as_longlong(2.0 * g.eb));
  const uint32_t ex = uint32_t(eb_bits >> 52) & 0x7ffu;
  const uint64_t M = (eb_bits & ((uint64_t(1) << 52) - 1)) | (ex ? uint64_t(1) << 52 : 0u);
  const int sh = ex ? 1075 - int(ex) : 1074;
  const double two_eps = 2.0 * g.eb;
  const bool fast_products = two_eps >= 0x1p-900;
  const uint32_t* Sa = reinterpret_cast<const uint32_t*>(p.a + g.off_s);
  const uint32_t* Sb = reinterpret_cast<const uint32_t*>(p.b + gb.off_s);
  const int32_t* Oa = reinterpret_cast<const int32_t*>(p.a + g.off_o);
  const int32_t* Ob = reinterpret_cast<const int32_t*>(p.b + gb.off_o);
  const uint32_t* Pa = reinterpret_cast<const uint32_t*>(p.a + g.off_p);
  const uint32_t* Pb = reinterpret_cast<const uint32_t*>(p.b + gb.off_p);
  int64_t acc_a = 0, acc_b = 0;
  uint64_t acc_pl = 0, acc_ph = 0;  // 128-bit two's complement sum of q_A q_B
  uint32_t next = 0;
  const uint32_t epoch = launch_epoch(p.s);
  if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
  for (;;) {
    if (tid == 0) s_ticket = next;
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= ntiles) break;
    if (tid < 64) {
      uint32_t b2 = 0;
      const uint64_t v = tile_offset(p.s.idx[0], (NT / kWaveSegs) * tile, g, b2);
      if (tid == 0) {
        s_base_a = v;
        latch(p.s, b2);
      }
    } else if (tid < 128) {
      uint32_t b2 = 0;
      const uint64_t v = tile_offset(p.s.idx[1], (NT / kWaveSegs) * tile, gb, b2);
      if (tid == 64) {
        s_base_b = v;
        latch(p.s, b2);
      }
    }
    const uint64_t seg = tile * NT + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = (seg >> g.spb_log2);
    const uint32_t sub = uint32_t(seg & (g.spb - 1));
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    const uint64_t mblk = active ? blk : 0, mseg = active ? seg : 0;
    const int32_t oa32 = Oa[mblk], ob32 = Ob[mblk];
    const uint32_t wa8 = p.a[g.off_w + mblk], wb8 = p.b[gb.off_w + mblk];
    const uint32_t swa8 = Sa[mseg], swb8 = Sb[mseg];
    uint32_t bad = 0;
    uint32_t wa = active ? wa8 : 0u, wb = active ? wb8 : 0u;
    if (wa > 32 || wb > 32) {
      bad |= ST_FORMAT;
      wa = wa > 32 ? 0u : wa;
      wb = wb > 32 ? 0u : wb;
    }
    static_assert(NT * 32 < 65536, "tile word counts must fit 16 bits");
    uint32_t tw2;
    const uint32_t off2 = wg_scan<NT>(wa | (wb << 16), tw2, s_tmp);  // its barriers publish the bases
    const uint32_t off_a = off2 & 0xffffu, off_b = off2 >> 16;
    const uint32_t tw_a = tw2 & 0xffffu, tw_b = tw2 >> 16;
    const uint64_t base_a = uni64(s_base_a), base_b = uni64(s_base_b);
    const bool fits_a = base_a + tw_a <= g.payload_bytes / 4;
    const bool fits_b = base_b + tw_b <= gb.payload_bytes / 4;
    if (!fits_a || !fits_b) bad |= ST_FORMAT;  // then nothing is read
    const int64_t oa = active ? oa32 : 0, ob = active ? ob32 : 0;
    const uint32_t swa = (cnt > 0 && wa) ? bswap32(swa8) : 0u;
    const uint32_t swb = (cnt > 0 && wb) ? bswap32(swb8) : 0u;
    // operand A: stage, in-segment prefixes, carry
    stage_words<NT, false>(s_pay, Pa + base_a, fits_a ? tw_a : 0u, nullptr, 0u);
    __syncthreads();
    int32_t ra[32];
    const int64_t Da = segment_prefixes(&s_pay[1 + off_a], wa, swa, sub, cnt, ra);
    const int64_t carry_a = oa + block_excl(Da, g.spb);
    check_bins(&s_pay[1 + off_a], swa, wa, sub, cnt, oa, carry_a, blen, bad);
    __syncthreads();  // every lane is done reading A
    // operand B
    stage_words<NT, false>(s_pay, Pb + base_b, fits_b ? tw_b : 0u, nullptr, 0u);
    __syncthreads();
    int32_t rb[32];
    const int64_t Db = segment_prefixes(&s_pay[1 + off_b], wb, swb, sub, cnt, rb);
    const int64_t carry_b = ob + block_excl(Db, g.spb);
    check_bins(&s_pay[1 + off_b], swb, wb, sub, cnt, ob, carry_b, blen, bad);
    const uint32_t ca = uint32_t(carry_a), cb = uint32_t(carry_b);
    if (MODE == kCovariance) {
      int64_t sa = 0, sb = 0;
      uint64_t pl = 0, ph = 0;
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        if (uint32_t(j) < cnt) {
          const int32_t qa = int32_t(ca + uint32_t(ra[j])), qb = int32_t(cb + uint32_t(rb[j]));
          const int64_t prod = int64_t(qa) * int64_t(qb);
          sa += qa;
          sb += qb;
          const uint64_t nl = pl + uint64_t(prod);
          ph += (prod < 0 ? ~uint64_t(0) : 0u) + (nl < pl ? 1u : 0u);
          pl = nl;
        }
      }
      acc_a += sa;
      acc_b += sb;
      const uint64_t nl = acc_pl + pl;
      acc_ph += ph + (nl < acc_pl ? 1u : 0u);
      acc_pl = nl;
      latch(p.s, bad);
      if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
      __syncthreads();  // every lane is done reading B before the next tile stages
      continue;
    }
    // Hadamard: product bins, their deltas, re-encode.  Fast path: while
    // |q_A q_B| < 2^53 the binary64 product P is exact and the bin is
    // mul_round(2 eps, P) (2 eps is exact in binary64; 2 eps >= 2^-900
    // keeps the rounding's error term out of the subnormal range), and the
    // output deltas come from the binary64 bins as in scalar multiplication;
    // fl(P) < 2^53 certifies |P| < 2^53, else the segment is redone on the
    // exact 128-bit path.
    uint32_t mag[32];
    uint32_t sgn = 0, mx = 0;
    int32_t z0 = 0, zp = 0;
    bool exact_path = !fast_products;
    if (fast_products) {
      double zpd = 0.0, zmax = 0.0, pmax = 0.0;
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        uint32_t m = 0, hi = 0;
        if (uint32_t(j) < cnt) {
          const int32_t qa = int32_t(ca + uint32_t(ra[j])), qb = int32_t(cb + uint32_t(rb[j]));
          const double P = double(qa) * double(qb);
          pmax = fmax(pmax, fabs(P));
          const double z = mul_round(two_eps, P);
          zmax = fmax(zmax, fabs(z));
          if (j == 0) {
            z0 = cvt_i32(z);
          } else {
            const double d = z - zpd;  // +0 when equal
            m = cvt_abs_u32(d);
            hi = uint32_t(__double2hiint(d));
          }
          zpd = z;
        }
        mag[j] = m;
        sgn = __builtin_amdgcn_alignbit(sgn, hi, 31);  // slot j at bit 31 - j
        mx = max(mx, m);
        __builtin_amdgcn_sched_barrier(0);  // one slot at a time (live ranges)
      }
      zp = cvt_i32(zpd);
      if (!(pmax < 9007199254740992.0)) {
        exact_path = true;
        sgn = 0;
        mx = 0;
      } else if (!(zmax <= kBinMaxD)) {
        bad |= ST_RANGE;
      }
    }
    if (exact_path) {
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        uint32_t m = 0;
        if (uint32_t(j) < cnt) {
          const int32_t qa = int32_t(ca + uint32_t(ra[j])), qb = int32_t(cb + uint32_t(rb[j]));
          const int32_t z = product_bin(int64_t(qa) * int64_t(qb), M, sh, bad);
          if (j == 0) {
            z0 = z;
          } else {
            bool neg = false;
            m = delta_mag(z, zp, neg);
            sgn |= uint32_t(neg) << (31 - j);
          }
          zp = z;
        }
        mag[j] = m;
        mx = max(mx, m);
      }
    }
    // slot 0's delta needs the last product bin of the previous segment of
    // the same block (a segment with valid slots after the first always
    // follows a full segment)
    const int32_t prev = __shfl_up(zp, 1, 64);
    int32_t outlier_z = 0;
    if (cnt > 0) {
      if (sub == 0) {
        outlier_z = z0;
      } else {
        bool neg = false;
        mag[0] = delta_mag(z0, prev, neg);
        sgn |= uint32_t(neg) << 31;
        mx = max(mx, mag[0]);
      }
    }
    latch(p.s, bad);
    mx = block_max(mx, g.spb);
    const uint32_t wz = bitlen32(mx);
    uint32_t tw_z;
    const uint32_t off_z = wg_scan<NT>(wz, tw_z, s_tmp);  // barriers: all threads done reading B
    lb_publish(p.s.st_out, tile, tw_z, epoch);
    const uint32_t group = pack_group(wz);
    if (wz > 0) pack32_grouped(&s_pay[off_z], mag, wz, group);
    if (active) {
      if (sub == 0) {
        p.out[g.off_w + blk] = uint8_t(wz);
        reinterpret_cast<int32_t*>(p.out + g.off_o)[blk] = outlier_z;
      }
      reinterpret_cast<uint32_t*>(p.out + g.off_s)[seg] = bswap32(sgn);
    }
    const uint64_t base_z = lb_wait<NT>(p.s.st_out, tile, tw_z, epoch, s_lb, p.s.wait_limit, bad);
    if (tid == 0) latch(p.s, bad & ST_TIMEOUT);
    if (tid == 0) next = atomicAdd(&p.s.ctrl[C_TICKET], 1u);
    __syncthreads();
    uint32_t* Pz = reinterpret_cast<uint32_t*>(p.out + g.off_p) + base_z;
    for (uint32_t k = tid; k < tw_z; k += NT) Pz[k] = bswap32(s_pay[k]);
    if (tid == 0 && tile == ntiles - 1) {
      const uint64_t payload = 4 * (base_z + tw_z);
      write_header(p.out, g, payload);
      st_dev(&p.s.acc[A_OUT], g.off_p + payload);
    }
    __syncthreads();
  }
  if (MODE == kCovariance) {
    int64_t dummy_s = acc_b;
    uint64_t zl = 0, zh = 0;
    wg_sum_s_q<NT>(acc_a, acc_pl, acc_ph, s_rs, s_rl, s_rh);
    wg_sum_s_q<NT>(dummy_s, zl, zh, s_rs, s_rl, s_rh);
    if (tid == 0) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_S]), (unsigned long long)acc_a);
      atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_SB]), (unsigned long long)dummy_s);
      const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_QLO]),
                                     (unsigned long long)acc_pl);
      const uint64_t carry_out = (old + acc_pl < old) ? 1u : 0u;
      atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[A_QHI]),
                (unsigned long long)(acc_ph + carry_out));
    }
    if (!finish_arrive(&p.s.ctrl[C_DONE], &s_flag)) return;
    double value = 0.0;
    if (tid == 0 && !err) {
      // n P - S_A S_B exactly in 128 bits (|.| < 2^126), then
      // ((double)m / n / n) (2 eps_A)(2 eps_B)
      const __int128 P = (__int128)(((unsigned __int128)ld_dev(&p.s.acc[A_QHI]) << 64) |
                                    ld_dev(&p.s.acc[A_QLO]));
      const __int128 SA = int64_t(ld_dev(&p.s.acc[A_S])), SB = int64_t(ld_dev(&p.s.acc[A_SB]));
      const __int128 m = __int128(g.n) * P - SA * SB;
      const unsigned __int128 am = m < 0 ? (unsigned __int128)(-m) : (unsigned __int128)m;
      const double mag_d = u128_to_double(uint64_t(am >> 64), uint64_t(am));
      const double md = m < 0 ? -mag_d : mag_d;
      value = ((md / double(g.n)) / double(g.n)) * ((2.0 * g.eb) * (2.0 * gb.eb));
    }
    publish(p.s, p.res, 0, value);
    return;
  }
  if (finish_arrive(&p.s.ctrl[C_DONE], &s_flag)) {
    retire_epoch(p.s, epoch);
    publish(p.s, p.res, ld_dev(&p.s.acc[A_OUT]), 0.0);
  }
}

// ---------------------------------------------------- float32 workflow ops

__global__ void __launch_bounds__(kThreads) k_f32_map(int op, const float* x, const float* y,
                                                      double s, float* out, uint64_t n) {
  const uint64_t stride = uint64_t(gridDim.x) * kThreads;
  const uint64_t gt = uint64_t(blockIdx.x) * kThreads + threadIdx.x;
  const uint64_t n4 = n / 4;
  const float4* x4 = reinterpret_cast<const float4*>(x);
  const float4* y4 = reinterpret_cast<const float4*>(y);
  float4* o4 = reinterpret_cast<float4*>(out);
  for (uint64_t k = gt; k < n4; k += stride) {
    float4 a = x4[k], r;
    if (op == 0) {
      r = make_float4(-a.x, -a.y, -a.z, -a.w);
    } else if (op == 1) {
      const float4 b = y4[k];
      r = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
    } else if (op == 2) {
      r = make_float4(float(double(a.x) * s), float(double(a.y) * s), float(double(a.z) * s),
                      float(double(a.w) * s));
    } else if (op == 3) {
      const float4 b = y4[k];
      r = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
    } else if (op == 4) {
      r = make_float4(float(double(a.x) + s), float(double(a.y) + s), float(double(a.z) + s),
                      float(double(a.w) + s));
    } else {
      const float4 b = y4[k];
      r = make_float4(a.x * b.x, a.y * b.y, a.z * b.z, a.w * b.w);
    }
    o4[k] = r;
  }
  for (uint64_t i = 4 * n4 + gt; i < n; i += stride) {
    const float a = x[i];
    float r;
    switch (op) {
      case 0: r = -a; break;
      case 1: r = a + y[i]; break;
      case 2: r = float(double(a) * s); break;
      case 3: r = a - y[i]; break;
      case 4: r = float(double(a) + s); break;
      default: r = a * y[i]; break;
    }
    out[i] = r;
  }
}

// Sum of x (pass 0) or of (x - mean)^2 (pass 1) in float64; per-workgroup
// partials in fixed order, the last workgroup adds them up in order.
__global__ void __launch_bounds__(kThreads) k_f32_sum(const float* x, uint64_t n, int pass,
                                                      Scratch s, hoszp_result* res) {
  __shared__ double s_red[kThreads];
  __shared__ uint32_t s_flag;
  const uint64_t stride = uint64_t(gridDim.x) * kThreads;
  const uint64_t gt = uint64_t(blockIdx.x) * kThreads + threadIdx.x;
  const double mean = pass ? s.part[gridDim.x] : 0.0;
  double acc = 0.0;
  const uint64_t n4 = n / 4;
  const float4* x4 = reinterpret_cast<const float4*>(x);
  for (uint64_t k = gt; k < n4; k += stride) {
    const float4 a = x4[k];
    if (pass) {
      const double d0 = double(a.x) - mean, d1 = double(a.y) - mean;
      const double d2 = double(a.z) - mean, d3 = double(a.w) - mean;
      acc += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
    } else {
      acc += double(a.x) + double(a.y) + double(a.z) + double(a.w);
    }
  }
  for (uint64_t i = 4 * n4 + gt; i < n; i += stride) {
    const double d = pass ? double(x[i]) - mean : double(x[i]);
    acc += pass ? d * d : d;
  }
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) s_red[threadIdx.x] += s_red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(&s.part[blockIdx.x], s_red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!finish_arrive(&s.ctrl[C_DONE], &s_flag)) return;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (uint32_t b = 0; b < gridDim.x; ++b)
      t += __hip_atomic_load(&s.part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double v = t / double(n);
    if (pass == 0) {
      s.part[gridDim.x] = v;  // the mean, read by pass 1
      s.ctrl[C_DONE] = 0;     // pass 1 or the next operation counts from zero
      res->status = 0;
      res->out_bytes = 0;
      res->value = v;
    } else {
      publish(s, res, 0, v);
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_reset(const Scratch& s, hoszp_result* res, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, s.ctrl, s.acc, res);
  return hipGetLastError();
}

static hipError_t launch_widths(const Scratch& s, const Grids& gr, const uint8_t* c,
                                uint64_t c_bytes, hipStream_t st) {
  WidthParams p{{c, c}, {c_bytes, c_bytes}, {s.idx[0], s.idx[0]},
                {s.ctrl + C_WIDTHS, s.ctrl + C_WIDTHS}, s, 1u};
  hipLaunchKernelGGL(k_widths, dim3(gr.widths), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}
// Both operands of a two-stream operation in one launch (index 0 and 1).
static hipError_t launch_widths2(const Scratch& s, const Grids& gr, const uint8_t* a,
                                 uint64_t a_bytes, const uint8_t* b, uint64_t b_bytes,
                                 hipStream_t st) {
  WidthParams p{{a, b}, {a_bytes, b_bytes}, {s.idx[0], s.idx[1]},
                {s.ctrl + C_WIDTHS, s.ctrl + C_WIDTHS + 1}, s, 2u};
  hipLaunchKernelGGL(k_widths, dim3(2 * gr.widths), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_compress(const Scratch& s, const Grids& gr, const float* x, const Layout& g,
                           double inv2e, uint8_t* out, hoszp_result* res, hipStream_t st) {
  CompressParams p{x, out, g, g.eb, inv2e, abs_bound(g.eb, inv2e), s, res};
  const uint32_t nt = compress_tile_segs(g.nseg, gr.cus);
  const uint64_t ntiles = (g.nseg + nt - 1) / nt;
  if (nt == uint32_t(kCompressThreads)) {
    const uint64_t grid = ntiles < uint64_t(gr.compress) ? ntiles : uint64_t(gr.compress);
    const dim3 gd = dim3(uint32_t(grid)), bd = dim3(kCompressThreads);
    switch (g.L) {
      case 32: hipLaunchKernelGGL((k_compress<1, kCompressThreads>), gd, bd, 0, st, p); break;
      case 64: hipLaunchKernelGGL((k_compress<2, kCompressThreads>), gd, bd, 0, st, p); break;
      case 128: hipLaunchKernelGGL((k_compress<4, kCompressThreads>), gd, bd, 0, st, p); break;
      case 256: hipLaunchKernelGGL((k_compress<8, kCompressThreads>), gd, bd, 0, st, p); break;
      default: return hipErrorInvalidValue;
    }
  } else {  // a small field: no more small tiles than CUs, each its own workgroup
    const dim3 gd = dim3(uint32_t(ntiles)), bd = dim3(kSmallTileSegs);
    switch (g.L) {
      case 32: hipLaunchKernelGGL((k_compress<1, kSmallTileSegs>), gd, bd, 0, st, p); break;
      case 64: hipLaunchKernelGGL((k_compress<2, kSmallTileSegs>), gd, bd, 0, st, p); break;
      case 128: hipLaunchKernelGGL((k_compress<4, kSmallTileSegs>), gd, bd, 0, st, p); break;
      case 256: hipLaunchKernelGGL((k_compress<8, kSmallTileSegs>), gd, bd, 0, st, p); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_decompress(const Scratch& s, const Grids& gr, const uint8_t* c,
                             uint64_t c_bytes, float* x, uint64_t n_cap, hoszp_result* res,
                             hipStream_t st) {
  hipError_t e = launch_widths(s, gr, c, c_bytes, st);
  if (e != hipSuccess) return e;
  DecodeParams p{c, c_bytes, x, n_cap, s, res};
  hipLaunchKernelGGL(k_decode<kDecompress>, dim3(gr.decode), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_reduce(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                         bool variance, hoszp_result* res, hipStream_t st) {
  hipError_t e = launch_widths(s, gr, c, c_bytes, st);
  if (e != hipSuccess) return e;
  DecodeParams p{c, c_bytes, nullptr, 0, s, res};
  if (variance)
    hipLaunchKernelGGL(k_decode<kVariance>, dim3(gr.reduce), dim3(kReduceThreads), 0, st, p);
  else
    hipLaunchKernelGGL(k_decode<kMean>, dim3(gr.reduce), dim3(kReduceThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_block_means(const Scratch& s, const Grids& gr, const uint8_t* c,
                              uint64_t c_bytes, double* means, uint64_t means_cap,
                              hoszp_result* res, hipStream_t st) {
  hipError_t e = launch_widths(s, gr, c, c_bytes, st);
  if (e != hipSuccess) return e;
  DecodeParams p{c, c_bytes, nullptr, means_cap, s, res, means};
  hipLaunchKernelGGL(k_decode<kBlockMean>, dim3(gr.reduce), dim3(kReduceThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_negate(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                         uint8_t* out, uint64_t out_cap, hoszp_result* res, hipStream_t st) {
  NegateParams p{c, c_bytes, out, out_cap, s, res, 0.0, 0, 0};
  hipLaunchKernelGGL(k_negate<kNegate>, dim3(gr.negate), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_shift(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                        double scalar, int sign, uint8_t* out, uint64_t out_cap,
                        hoszp_result* res, hipStream_t st) {
  hipError_t e = launch_widths(s, gr, c, c_bytes, st);
  if (e != hipSuccess) return e;
  NegateParams p{c, c_bytes, out, out_cap, s, res, scalar, sign, 0};
  hipLaunchKernelGGL(k_negate<kShift>, dim3(gr.negate), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_add(const Scratch& s, const Grids& gr, const uint8_t* a, uint64_t a_bytes,
                      const uint8_t* b, uint64_t b_bytes, uint8_t* out, uint64_t out_cap,
                      hoszp_result* res, hipStream_t st, bool sub) {
  hipError_t e = launch_widths2(s, gr, a, a_bytes, b, b_bytes, st);
  if (e != hipSuccess) return e;
  AddParams p{a, a_bytes, b, b_bytes, out, out_cap, s, res};
  if (sub)
    hipLaunchKernelGGL((k_add<kAddThreads, true>), dim3(gr.add), dim3(kAddThreads), 0, st, p);
  else
    hipLaunchKernelGGL((k_add<kAddThreads, false>), dim3(gr.add), dim3(kAddThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_mul(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                      MulScalar k, uint8_t* out, uint64_t out_cap, hoszp_result* res,
                      hipStream_t st) {
  hipError_t e = launch_widths(s, gr, c, c_bytes, st);
  if (e != hipSuccess) return e;
  MulParams p{c, c_bytes, out, out_cap, k, s, res};
  hipLaunchKernelGGL(k_mul<kMulThreads>, dim3(gr.mul), dim3(kMulThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_bivar(const Scratch& s, const Grids& gr, bool covariance, const uint8_t* a,
                        uint64_t a_bytes, const uint8_t* b, uint64_t b_bytes, uint8_t* out,
                        uint64_t out_cap, hoszp_result* res, hipStream_t st) {
  hipError_t e = launch_widths2(s, gr, a, a_bytes, b, b_bytes, st);
  if (e != hipSuccess) return e;
  BivarParams p{a, a_bytes, b, b_bytes, out, out_cap, s, res};
  if (covariance)
    hipLaunchKernelGGL((k_bivar<kCovariance, kBivarThreads>), dim3(gr.bivar), dim3(kBivarThreads), 0, st, p);
  else
    hipLaunchKernelGGL((k_bivar<kHadamard, kBivarThreads>), dim3(gr.bivar), dim3(kBivarThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_f32_unary(const Grids& gr, int op, const float* x, const float* y2, double s,
                            float* out, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_map, dim3(gr.f32), dim3(kThreads), 0, st, op, x, y2, s, out, n);
  return hipGetLastError();
}

hipError_t launch_f32_reduce(const Scratch& s, const Grids& gr, const float* x, uint64_t n,
                             bool variance, hoszp_result* res, hipStream_t st) {
  const uint32_t grid = uint32_t(gr.f32) < s.max_part - 1 ? uint32_t(gr.f32) : s.max_part - 1;
  hipLaunchKernelGGL(k_f32_sum, dim3(grid), dim3(kThreads), 0, st, x, n, 0, s, res);
  if (variance) hipLaunchKernelGGL(k_f32_sum, dim3(grid), dim3(kThreads), 0, st, x, n, 1, s, res);
  return hipGetLastError();
}

hipError_t launch_zero64(uint64_t* p, uint64_t n, hipStream_t st) {
  const uint64_t want = (n + kThreads - 1) / kThreads;
  const uint32_t grid = uint32_t(want < 4096 ? (want ? want : 1) : 4096);
  hipLaunchKernelGGL(k_zero64, dim3(grid), dim3(kThreads), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchDev& b, int grid, hipStream_t st) {
  BatchParams p{b.fields, b.tile_field, b.total_tiles, b.st, b.ctrl, b.facc, b.res, b.wait_limit};
  if (b.threads == kBatchThreadsSmall)
    hipLaunchKernelGGL(k_batch<kBatchThreadsSmall>, dim3(uint32_t(grid)), dim3(kBatchThreadsSmall),
                       0, st, p);
  else
    hipLaunchKernelGGL(k_batch<kBatchThreads>, dim3(uint32_t(grid)), dim3(kBatchThreads), 0, st, p);
  return hipGetLastError();
}

int batch_max_grid(int num_cus, uint32_t threads) {
  int occ = 0;
  const hipError_t e =
      threads == kBatchThreadsSmall
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch<kBatchThreadsSmall>,
                                                         kBatchThreadsSmall, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch<kBatchThreads>,
                                                         kBatchThreads, 0);
  if (e != hipSuccess) return num_cus;
  return num_cus * (occ < 1 ? 1 : occ);
}

hipError_t query_grids(Grids& gr, int num_cus) {
  int c = 0, d = 0, a = 0, m = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_compress<1, kCompressThreads>, kCompressThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&d, k_decode<kDecompress>, kThreads, 0);
  int r = 0;
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_decode<kMean>, kReduceThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_add<kAddThreads, false>, kAddThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, k_mul<kMulThreads>, kMulThreads, 0);
  int bv = 0;
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bv, k_bivar<kHadamard, kBivarThreads>,
                                                     kBivarThreads, 0);
  if (e != hipSuccess) return e;
  auto clampg = [&](int occ) { return num_cus * (occ < 1 ? 1 : occ); };
  gr.bivar = clampg(bv);
  gr.compress = clampg(c);
  gr.decode = clampg(d);
  gr.reduce = clampg(r);
  gr.add = clampg(a);
  gr.mul = clampg(m);
  gr.cus = num_cus;
  gr.negate = num_cus;  // one workgroup per CU: fewer end-of-kernel atomics, measured fastest
  gr.widths = num_cus;
  gr.f32 = num_cus * 4;
  return hipSuccess;
}

}  // namespace hz
