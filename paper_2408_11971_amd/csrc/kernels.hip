// kernels.hip -- gfx950 kernels of the HoSZp library (arXiv 2408.11971).
//
// Work decomposition (shared by every kernel): a block of L slots is split
// into L/32 segments of 32 slots.  One thread owns one segment, a workgroup of
// 256 threads owns a tile of 256 segments (8192 slots).  A segment of a block
// of width w owns exactly w payload words (32 slots x w bits), so payload
// offsets are a prefix sum of per-segment widths: within a tile it is a
// workgroup scan, across tiles a single-pass decoupled look-back on per-tile
// word counts (status words in the context scratch).  Tiles are taken from an
// atomic ticket so a tile only ever waits on tiles already owned by running
// workgroups; workgroups are persistent and loop until the tickets run out.
//
// Payload words are staged in LDS as big-endian values (one byte swap per
// word), so a w-bit field at bit p of a segment is one funnel shift
// (v_alignbit) of two neighbouring LDS words.

#include "hoszp_internal.h"

namespace hz {
namespace {

constexpr double kBinMaxD = 2147483647.0;
constexpr uint64_t kLbAgg = 1, kLbInc = 2;
constexpr uint64_t kLbValMask = (uint64_t(1) << 34) - 1;

enum { kMean = 0, kVariance = 1, kDecompress = 2 };

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t bswap32(uint32_t v) { return __builtin_bswap32(v); }
__device__ __forceinline__ uint32_t bitlen32(uint32_t v) { return v ? 32u - __clz(int(v)) : 0u; }

// Values every lane holds identically, moved to scalar registers so that
// branches on them (notably persistent-loop exits next to barriers) are
// compiled as uniform branches.
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return (uint64_t(uni32(uint32_t(v >> 32))) << 32) | uni32(uint32_t(v));
}

__device__ __forceinline__ void latch(hoszp_result* res, uint32_t bits) {
  if (bits) atomicOr(&res->status, bits);
}

__device__ __forceinline__ uint64_t ld_acq(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Validate a stream header and derive its section placement.
__device__ uint32_t read_header(const uint8_t* c, uint64_t c_bytes, Layout& g) {
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
__device__ void write_header(uint8_t* out, const Layout& g, uint64_t payload) {
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
__device__ uint32_t wg_scan(uint32_t v, uint32_t& total, uint32_t* tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t t = tmp[w];
    before += (w < wave) ? t : 0u;
    all += t;
  }
  __syncthreads();
  total = all;
  return before + x - v;
}

__device__ __forceinline__ uint64_t lb_word(uint32_t epoch, uint64_t flag, uint64_t v) {
  return (uint64_t(epoch) << 36) | (flag << 34) | (v & kLbValMask);
}

// Decoupled look-back: exclusive prefix over tiles of the per-tile `agg`.
// Executed by all 64 lanes of one wave; every lane gets the result.  The
// tile's aggregate is published first, so a waiting tile never blocks the
// ones before it; each window of 64 predecessors is read in parallel.
__device__ uint64_t lookback(uint64_t* st, uint64_t tile, uint64_t agg, uint32_t epoch) {
  const int lane = threadIdx.x & 63;
  if (tile == 0) {
    if (lane == 0) st_rel(&st[0], lb_word(epoch, kLbInc, agg));
    return 0;
  }
  if (lane == 0) st_rel(&st[tile], lb_word(epoch, kLbAgg, agg));
  uint64_t excl = 0;
  int64_t base = int64_t(tile);
  for (;;) {
    const int64_t idx = base - 1 - lane;
    bool ready = true, inc = true;
    uint64_t val = 0;
    if (idx >= 0) {
      const uint64_t w = ld_acq(&st[idx]);
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
    uint64_t part = ((upto >> lane) & 1u) ? val : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
    excl += part;
    if (incm) break;
    base -= 64;
  }
  if (lane == 0) st_rel(&st[tile], lb_word(epoch, kLbInc, excl + agg));
  return excl;
}

// Number of valid slots (0..32) of segment `sub` of block `blk`.
__device__ __forceinline__ uint32_t seg_count(const Layout& g, uint64_t blk, uint32_t sub,
                                              uint64_t& blen) {
  const uint64_t left = g.n - blk * g.L;
  blen = left < g.L ? left : g.L;
  const uint64_t lo = uint64_t(32) * sub;
  return blen > lo ? uint32_t(blen - lo < 32 ? blen - lo : 32) : 0u;
}

// w-bit field j of a segment whose words start at sp (sp[-1] and sp[w] must
// be readable LDS words).  w in [1, 32].
__device__ __forceinline__ uint32_t field(const uint32_t* sp, uint32_t j, uint32_t w) {
  const uint32_t p = j * w;
  const int i = int((p + 31u) >> 5);
  const uint32_t win = __builtin_amdgcn_alignbit(sp[i - 1], sp[i], 0u - p);
  return win >> (32u - w);
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

// Bins of a block stay in range if |O| + (len-1)(2^w - 1) fits.
__device__ __forceinline__ bool bins_surely_in_range(int64_t outlier, uint64_t blen, uint32_t w) {
  const uint64_t a = uint64_t(outlier < 0 ? -outlier : outlier);
  const uint64_t step = w >= 33 ? ~uint64_t(0) : ((uint64_t(1) << w) - 1);
  return a + (blen - 1) * step <= uint64_t(kBinMax);
}

// Stage payload words [base, base + words) of a stream into LDS (sp[1..]) with
// a zero guard word on each side.  Returns false when the range leaves the
// payload section.
__device__ bool stage_payload(uint32_t* sp, const uint32_t* P, uint64_t base, uint32_t words,
                              uint64_t payload_words) {
  const bool fits = base + words <= payload_words;
  if (fits)
    for (uint32_t k = threadIdx.x; k < words; k += kThreads) sp[1 + k] = bswap32(P[base + k]);
  if (threadIdx.x == 0) {
    sp[0] = 0;
    sp[1 + words] = 0;
  }
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
__device__ double u128_to_double(uint64_t hi, uint64_t lo) {
  if (hi == 0) return double(lo);
  const int lz = __clzll((long long)hi);
  const uint64_t top = lz ? (hi << lz) | (lo >> (64 - lz)) : hi;
  const uint64_t rest = lo << lz;
  const uint64_t jam = top | (rest != 0 ? 1u : 0u);  // sticky bit below the rounding bit
  return ldexp(double(jam), 64 - lz);
}

// Sum over the workgroup of an int64 and an unsigned 128-bit value (hi:lo);
// the result is valid in thread 0.
__device__ void wg_sum_s_q(int64_t& s, uint64_t& qlo, uint64_t& qhi, int64_t* ts, uint64_t* tl,
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
    for (int w = 0; w < kThreads / 64; ++w) {
      s += ts[w];
      const uint64_t nl = qlo + tl[w];
      qhi = qhi + th[w] + (nl < qlo ? 1u : 0u);
      qlo = nl;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ kernels

__global__ void k_init(uint32_t* ctrl, uint64_t* acc, hoszp_result* res) {
  const int t = threadIdx.x;
  if (t < 4) ctrl[t] = 0;
  if (t < 8) acc[t] = 0;
  if (t == 0) {
    res->status = 0;
    res->out_bytes = 0;
    res->value = 0.0;
  }
}

struct CompressParams {
  const float* x;
  uint8_t* out;
  Layout g;
  double eb, inv2e;
  Scratch s;
  uint32_t epoch;
  hoszp_result* res;
};

// Eq. 3 in binary64: floor(((double)x + eps) * (1 / (2 eps))).
__device__ __forceinline__ double bin_real(float v, double eb, double inv2e) {
  const double shifted = double(v) + eb;
  return floor(shifted * inv2e);
}

// Quantize 32 values, form Lorenzo deltas, split signs and magnitudes.
// FULL: all 32 slots valid (no padding checks).
template <bool FULL>
__device__ __forceinline__ void quantize_segment(const float* v, uint32_t cnt, bool first_seg,
                                                 int32_t prev, double eb, double inv2e,
                                                 uint32_t* mag, uint32_t& sgn, uint32_t& mx,
                                                 int32_t& outlier, uint32_t& bad) {
  int32_t qp = prev;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const float xv = v[j];
    const double f = bin_real(xv, eb, inv2e);
    const bool ok = f >= -kBinMaxD && f <= kBinMaxD;
    const int32_t q = ok ? int32_t(f) : 0;
    const bool valid = FULL || uint32_t(j) < cnt;
    if (valid && !ok) bad |= isfinite(xv) ? ST_RANGE : ST_NONFINITE;
    bool neg = false;
    uint32_t m = 0;
    if (j == 0 && first_seg) {
      outlier = q;
    } else {
      m = delta_mag(q, qp, neg);
    }
    if (!valid) {
      m = 0;
      neg = false;
    }
    mag[j] = m;
    sgn |= uint32_t(neg) << (31 - j);
    mx = max(mx, m);
    qp = q;
  }
}

template <int SPB>
__global__ void __launch_bounds__(kThreads) k_compress(CompressParams p) {
  __shared__ uint32_t s_pay[kTileWords + 2];
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint64_t s_ticket, s_base;
  constexpr uint32_t L = SPB * 32;
  const int tid = threadIdx.x;
  const Layout& g = p.g;
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&p.s.ctrl[0], 1u);
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= g.ntiles) break;
    const uint64_t seg = tile * kTileSegs + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = seg / SPB;
    const uint32_t sub = uint32_t(seg % SPB);
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    const uint64_t first = blk * L + uint64_t(32) * sub;

    uint32_t mag[32];
    uint32_t sgn = 0, mx = 0, bad = 0;
    int32_t outlier = 0;
    if (cnt > 0) {
      int32_t prev = 0;
      if (sub > 0) {  // the slot before this segment belongs to the same block
        const double f = bin_real(p.x[first - 1], p.eb, p.inv2e);
        prev = (f >= -kBinMaxD && f <= kBinMaxD) ? int32_t(f) : 0;
      }
      float v[32];
      if (cnt == 32) {
        const float4* src = reinterpret_cast<const float4*>(p.x + first);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float4 t = src[k];
          v[4 * k + 0] = t.x;
          v[4 * k + 1] = t.y;
          v[4 * k + 2] = t.z;
          v[4 * k + 3] = t.w;
        }
        quantize_segment<true>(v, cnt, sub == 0, prev, p.eb, p.inv2e, mag, sgn, mx, outlier, bad);
      } else {
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = uint32_t(j) < cnt ? p.x[first + j] : 0.0f;
        quantize_segment<false>(v, cnt, sub == 0, prev, p.eb, p.inv2e, mag, sgn, mx, outlier, bad);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 32; ++j) mag[j] = 0;
    }
    latch(p.res, bad);
    mx = block_max(mx, SPB);
    const uint32_t w = bitlen32(mx);

    uint32_t tile_words;
    const uint32_t off = wg_scan(w, tile_words, s_tmp);
    if (tid < 64) {
      const uint64_t base = lookback(p.s.st_out, tile, tile_words, p.epoch);
      if (tid == 0) s_base = base;
    }
    __syncthreads();
    const uint64_t base = s_base;
    if (w > 0) pack32(&s_pay[off], mag, w);
    __syncthreads();
    uint32_t* P = reinterpret_cast<uint32_t*>(p.out + g.off_p) + base;
    for (uint32_t k = tid; k < tile_words; k += kThreads) P[k] = bswap32(s_pay[k]);
    if (active) {
      if (sub == 0) {
        p.out[g.off_w + blk] = uint8_t(w);
        reinterpret_cast<int32_t*>(p.out + g.off_o)[blk] = outlier;
      }
      reinterpret_cast<uint32_t*>(p.out + g.off_s)[seg] = bswap32(sgn);
    }
    if (tid == 0 && tile == g.ntiles - 1) {
      const uint64_t payload = 4 * (base + tile_words);
      write_header(p.out, g, payload);
      p.res->out_bytes = g.off_p + payload;
    }
    __syncthreads();
  }
}

struct DecodeParams {
  const uint8_t* c;
  uint64_t c_bytes;
  float* x;
  uint64_t n_cap;
  Scratch s;
  uint32_t epoch;
  hoszp_result* res;
};

// Decode a segment: in-segment prefix e_j of the deltas (e_j = bin_j - bin of
// the slot before the segment, or - outlier for the first segment).
// Accumulates E = sum e_j and E2 = sum e_j^2 over valid slots, keeps e_j in
// `keep` when KEEP.  Returns the segment's delta total.
template <bool KEEP, bool WIDE>
__device__ __forceinline__ int64_t decode_segment(const uint32_t* sp, uint32_t sw, uint32_t w,
                                                  uint32_t sub, uint32_t cnt, int64_t& E,
                                                  uint64_t& E2, unsigned __int128& E2w,
                                                  int64_t* keep) {
  int64_t e = 0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    int64_t d = seg_delta(sp, sw, w, j);
    if (j == 0 && sub == 0) d = 0;  // slot 0 of a block is the outlier
    const bool valid = uint32_t(j) < cnt;
    if (!valid) d = 0;
    e += d;
    if (valid) {
      E += e;
      if (WIDE) {
        const uint64_t a = uint64_t(e < 0 ? -e : e);
        E2w += (unsigned __int128)a * a;
      } else {
        E2 += uint64_t(e * e);
      }
    }
    if (KEEP) keep[j] = e;
  }
  return e;
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_decode(DecodeParams p) {
  __shared__ uint32_t s_pay[kTileWords + 2];
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint64_t s_ticket, s_base;
  __shared__ int64_t s_rs[kThreads / 64];
  __shared__ uint64_t s_rl[kThreads / 64], s_rh[kThreads / 64];
  const int tid = threadIdx.x;
  Layout g;
  uint32_t err = read_header(p.c, p.c_bytes, g);
  if (!err && MODE == kDecompress && p.n_cap < g.n) err = ST_CAPACITY;
  if (err) {
    if (tid == 0) latch(p.res, err);
    return;
  }
  const uint64_t payload_words = g.payload_bytes / 4;
  const uint32_t* P = reinterpret_cast<const uint32_t*>(p.c + g.off_p);
  const uint32_t* S = reinterpret_cast<const uint32_t*>(p.c + g.off_s);
  const int32_t* O = reinterpret_cast<const int32_t*>(p.c + g.off_o);
  const double two_eb = 2.0 * g.eb;
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&p.s.ctrl[0], 1u);
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= g.ntiles) break;
    const uint64_t seg = tile * kTileSegs + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = seg / g.spb;
    const uint32_t sub = uint32_t(seg % g.spb);
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    uint32_t bad = 0;
    uint32_t w = active ? p.c[g.off_w + blk] : 0u;
    if (w > 32) {
      bad |= ST_FORMAT;
      w = 0;
    }
    uint32_t tile_words;
    const uint32_t off = wg_scan(w, tile_words, s_tmp);
    if (tid < 64) {
      const uint64_t base = lookback(p.s.st_a, tile, tile_words, p.epoch);
      if (tid == 0) s_base = base;
    }
    __syncthreads();
    const uint64_t base = s_base;
    if (!stage_payload(s_pay, P, base, tile_words, payload_words)) bad |= ST_FORMAT;
    if (tid == 0 && tile == g.ntiles - 1 && base + tile_words != payload_words) bad |= ST_FORMAT;
    __syncthreads();

    const int32_t outlier = active ? O[blk] : 0;
    int64_t E = 0;
    uint64_t E2 = 0;
    unsigned __int128 E2w = 0;
    int64_t keep[MODE == kDecompress ? 32 : 1];
    int64_t D = 0;
    const uint32_t* sp = &s_pay[1 + off];
    if (cnt > 0 && w > 0) {
      const uint32_t sw = bswap32(S[seg]);
      if (MODE == kDecompress) {
        D = decode_segment<true, false>(sp, sw, w, sub, cnt, E, E2, E2w, keep);
      } else if (MODE == kMean || w <= 24) {
        D = decode_segment<false, false>(sp, sw, w, sub, cnt, E, E2, E2w, keep);
      } else {
        D = decode_segment<false, true>(sp, sw, w, sub, cnt, E, E2, E2w, keep);
      }
    } else if (MODE == kDecompress) {
#pragma unroll
      for (int j = 0; j < 32; ++j) keep[j] = 0;
    }
    const int64_t carry = int64_t(outlier) + block_excl(D, g.spb);
    // every bin must be a valid int32 bin (slot 0 is the outlier itself)
    if (cnt > 0 && !bins_surely_in_range(outlier, blen, w)) {
      const uint32_t sw = w ? bswap32(S[seg]) : 0u;
      int64_t e = 0;
      for (int j = 0; j < int(cnt); ++j) {
        if (w && !(j == 0 && sub == 0)) e += seg_delta(sp, sw, w, j);
        const int64_t bin = carry + e;
        if (bin < -kBinMax || bin > kBinMax) bad |= ST_FORMAT;
      }
    }
    latch(p.res, bad);

    if (MODE == kDecompress) {
      if (cnt > 0) {
        const uint64_t first = blk * g.L + uint64_t(32) * sub;
        if (cnt == 32) {
          float4* dst = reinterpret_cast<float4*>(p.x + first);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            float4 t;
            t.x = float(double(carry + keep[4 * k + 0]) * two_eb);
            t.y = float(double(carry + keep[4 * k + 1]) * two_eb);
            t.z = float(double(carry + keep[4 * k + 2]) * two_eb);
            t.w = float(double(carry + keep[4 * k + 3]) * two_eb);
            dst[k] = t;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 32; ++j)
            if (uint32_t(j) < cnt) p.x[first + j] = float(double(carry + keep[j]) * two_eb);
        }
      }
      __syncthreads();
    } else {
      // bins of the segment: carry + e_j over its cnt valid slots
      int64_t s_seg = int64_t(cnt) * carry + E;
      uint64_t qlo = 0, qhi = 0;
      if (MODE == kVariance && cnt > 0) {
        const __int128 c = carry;
        __int128 q = __int128(cnt) * c * c + 2 * c * __int128(E);
        if (w > 24) q += __int128(E2w);
        else q += __int128(E2);
        qlo = uint64_t(q);
        qhi = uint64_t(q >> 64);
      }
      wg_sum_s_q(s_seg, qlo, qhi, s_rs, s_rl, s_rh);
      if (tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[0]), (unsigned long long)s_seg);
        if (MODE == kVariance) {
          const uint64_t old =
              atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[1]), (unsigned long long)qlo);
          const uint64_t carry_out = (old + qlo < old) ? 1u : 0u;
          atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[2]),
                    (unsigned long long)(qhi + carry_out));
        }
        __threadfence();
        const uint32_t done = atomicAdd(&p.s.ctrl[1], 1u);
        if (done == g.ntiles - 1) {
          __threadfence();
          const int64_t S_all = int64_t(ld_acq(&p.s.acc[0]));
          if (MODE == kMean) {
            p.res->value = (double(S_all) / double(g.n)) * two_eb;
          } else {
            const uint64_t ql = ld_acq(&p.s.acc[1]), qh = ld_acq(&p.s.acc[2]);
            // M = n Q - S^2 (exact, non-negative)
            const uint64_t n = g.n;
            const uint64_t nql = n * ql;
            const uint64_t nqh = n * qh + __umul64hi(n, ql);
            const uint64_t a = uint64_t(S_all < 0 ? -S_all : S_all);
            const uint64_t sl = a * a, sh = __umul64hi(a, a);
            const uint64_t ml = nql - sl;
            const uint64_t mh = nqh - sh - (nql < sl ? 1u : 0u);
            const double m = u128_to_double(mh, ml);
            p.res->value = ((m / double(n)) / double(n)) * (two_eb * two_eb);
          }
        }
      }
      __syncthreads();
    }
  }
}

struct NegateParams {
  const uint8_t* c;
  uint64_t c_bytes;
  uint8_t* out;
  uint64_t out_cap;
  Scratch s;
  hoszp_result* res;
};

// Negation of one 4-byte word of the stream at byte offset o.
__device__ __forceinline__ uint32_t negate_word(const Layout& g, const uint8_t* c, uint64_t o,
                                                uint32_t v, uint64_t& wsum, uint32_t& bad) {
  if (o >= g.off_w && o < g.off_w + g.nb) {  // widths: copied, summed and range-checked
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (o + b < g.off_w + g.nb) {
        const uint32_t w = (v >> (8 * b)) & 0xffu;
        wsum += w;
        if (w > 32) bad |= ST_FORMAT;
      }
    }
    return v;
  }
  if (o >= g.off_o && o < g.off_o + 4 * g.nb) return 0u - v;  // O -> -O
  if (o >= g.off_s && o < g.off_s + 4 * g.nseg) {              // signs of valid slots
    const uint64_t seg = (o - g.off_s) / 4;
    const uint64_t blk = seg / g.spb;
    const uint32_t sub = uint32_t(seg % g.spb);
    if (c[g.off_w + blk] == 0) return v;  // constant block: no signs
    uint64_t blen;
    const uint32_t cnt = seg_count(g, blk, sub, blen);
    if (cnt == 0) return v;
    const uint32_t be = cnt == 32 ? 0xffffffffu : ~(0xffffffffu >> cnt);
    return v ^ bswap32(be);
  }
  return v;
}

__global__ void __launch_bounds__(kThreads) k_negate(NegateParams p) {
  __shared__ uint64_t s_w[kThreads / 64];
  __shared__ uint32_t s_bad;
  const int tid = threadIdx.x;
  Layout g;
  uint32_t err = read_header(p.c, p.c_bytes, g);
  if (!err && p.out_cap < g.total_bytes) err = ST_CAPACITY;
  if (err) {
    if (tid == 0 && blockIdx.x == 0) latch(p.res, err);
    return;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  const uint64_t total = g.total_bytes;  // multiple of 4
  const uint64_t nchunk = total / 16;
  const uint64_t stride = uint64_t(gridDim.x) * kThreads;
  const uint64_t gt = uint64_t(blockIdx.x) * kThreads + tid;
  uint64_t wsum = 0;
  uint32_t bad = 0;
  const uint4* src = reinterpret_cast<const uint4*>(p.c);
  uint4* dst = reinterpret_cast<uint4*>(p.out);
  for (uint64_t k = gt; k < nchunk; k += stride) {
    uint4 v = src[k];
    const uint64_t o = 16 * k;
    v.x = negate_word(g, p.c, o + 0, v.x, wsum, bad);
    v.y = negate_word(g, p.c, o + 4, v.y, wsum, bad);
    v.z = negate_word(g, p.c, o + 8, v.z, wsum, bad);
    v.w = negate_word(g, p.c, o + 12, v.w, wsum, bad);
    dst[k] = v;
  }
  const uint64_t tail_words = (total - 16 * nchunk) / 4;
  for (uint64_t k = gt; k < tail_words; k += stride) {
    const uint64_t o = 16 * nchunk + 4 * k;
    const uint32_t v = *reinterpret_cast<const uint32_t*>(p.c + o);
    *reinterpret_cast<uint32_t*>(p.out + o) = negate_word(g, p.c, o, v, wsum, bad);
  }
  if (bad) atomicOr(&s_bad, bad);
  // width total over the grid must fill the payload
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) wsum += __shfl_xor(wsum, d, 64);
  if ((tid & 63) == 0) s_w[tid >> 6] = wsum;
  __syncthreads();
  if (tid == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
    latch(p.res, s_bad);
    atomicAdd(reinterpret_cast<unsigned long long*>(&p.s.acc[3]), (unsigned long long)t);
    __threadfence();
    const uint32_t done = atomicAdd(&p.s.ctrl[1], 1u);
    if (done == gridDim.x - 1) {
      __threadfence();
      const uint64_t all = ld_acq(&p.s.acc[3]);
      if (all * (g.L / 8) != g.payload_bytes) latch(p.res, ST_FORMAT);
      p.res->out_bytes = total;
    }
  }
}

struct AddParams {
  const uint8_t* a;
  uint64_t a_bytes;
  const uint8_t* b;
  uint64_t b_bytes;
  uint8_t* out;
  uint64_t out_cap;
  Scratch s;
  uint32_t epoch;
  hoszp_result* res;
};

__global__ void __launch_bounds__(kThreads) k_add(AddParams p) {
  __shared__ uint32_t s_a[kTileWords + 2];
  __shared__ uint32_t s_b[kTileWords + 2];
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint64_t s_ticket, s_base_a, s_base_b, s_base_z;
  const int tid = threadIdx.x;
  Layout g, gb;
  uint32_t err = read_header(p.a, p.a_bytes, g);
  if (!err) err = read_header(p.b, p.b_bytes, gb);
  if (!err && (g.n != gb.n || g.L != gb.L ||
               __double_as_longlong(g.eb) != __double_as_longlong(gb.eb)))
    err = ST_MISMATCH;
  if (!err && p.out_cap < bound_bytes(g.n, g.L)) err = ST_CAPACITY;
  if (err) {
    if (tid == 0) latch(p.res, err);
    return;
  }
  const uint64_t pw_a = g.payload_bytes / 4, pw_b = gb.payload_bytes / 4;
  const uint32_t* Pa = reinterpret_cast<const uint32_t*>(p.a + g.off_p);
  const uint32_t* Pb = reinterpret_cast<const uint32_t*>(p.b + gb.off_p);
  const uint32_t* Sa = reinterpret_cast<const uint32_t*>(p.a + g.off_s);
  const uint32_t* Sb = reinterpret_cast<const uint32_t*>(p.b + gb.off_s);
  const int32_t* Oa = reinterpret_cast<const int32_t*>(p.a + g.off_o);
  const int32_t* Ob = reinterpret_cast<const int32_t*>(p.b + gb.off_o);
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&p.s.ctrl[0], 1u);
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= g.ntiles) break;
    const uint64_t seg = tile * kTileSegs + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = seg / g.spb;
    const uint32_t sub = uint32_t(seg % g.spb);
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    uint32_t bad = 0;
    uint32_t wa = active ? p.a[g.off_w + blk] : 0u;
    uint32_t wb = active ? p.b[gb.off_w + blk] : 0u;
    if (wa > 32 || wb > 32) {
      bad |= ST_FORMAT;
      wa = wa > 32 ? 0 : wa;
      wb = wb > 32 ? 0 : wb;
    }
    uint32_t tw_a, tw_b;
    const uint32_t off_a = wg_scan(wa, tw_a, s_tmp);
    const uint32_t off_b = wg_scan(wb, tw_b, s_tmp);
    if (tid < 64) {
      const uint64_t ba = lookback(p.s.st_a, tile, tw_a, p.epoch);
      const uint64_t bb = lookback(p.s.st_b, tile, tw_b, p.epoch);
      if (tid == 0) {
        s_base_a = ba;
        s_base_b = bb;
      }
    }
    __syncthreads();
    const uint64_t base_a = s_base_a, base_b = s_base_b;
    if (!stage_payload(s_a, Pa, base_a, tw_a, pw_a)) bad |= ST_FORMAT;
    if (!stage_payload(s_b, Pb, base_b, tw_b, pw_b)) bad |= ST_FORMAT;
    if (tid == 0 && tile == g.ntiles - 1 && (base_a + tw_a != pw_a || base_b + tw_b != pw_b))
      bad |= ST_FORMAT;
    __syncthreads();

    // O_{A+B} = O_A + O_B, P_{A+B} = P_A + P_B (signed), then re-encode
    const int64_t oz = active ? int64_t(Oa[blk]) + int64_t(Ob[blk]) : 0;
    uint32_t mag[32];
    uint32_t sgn = 0, mx = 0;
    int64_t D = 0;
    const uint32_t swa = (cnt > 0 && wa) ? bswap32(Sa[seg]) : 0u;
    const uint32_t swb = (cnt > 0 && wb) ? bswap32(Sb[seg]) : 0u;
    const uint32_t* spa = &s_a[1 + off_a];
    const uint32_t* spb = &s_b[1 + off_b];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      int64_t d = 0;
      if (wa) d += seg_delta(spa, swa, wa, j);
      if (wb) d += seg_delta(spb, swb, wb, j);
      if ((j == 0 && sub == 0) || uint32_t(j) >= cnt) d = 0;
      const bool neg = d < 0;
      // |d| >= 2^32 only happens when some bin of the sum is out of range,
      // which the check below reports; the truncated field stays memory-safe
      const uint32_t m = uint32_t(neg ? -d : d);
      mag[j] = m;
      sgn |= uint32_t(neg) << (31 - j);
      mx = max(mx, m);
      D += d;
    }
    // every bin of the sum must stay in range
    const int64_t carry = oz + block_excl(D, g.spb);
    if (cnt > 0) {
      const int64_t oa = Oa[blk], ob = Ob[blk];
      const uint64_t aa = uint64_t(oa < 0 ? -oa : oa), ab = uint64_t(ob < 0 ? -ob : ob);
      const uint64_t sa = (uint64_t(1) << wa) - 1, sb = (uint64_t(1) << wb) - 1;
      if (aa + ab + (blen - 1) * (sa + sb) > uint64_t(kBinMax)) {
        int64_t e = 0;
        for (int j = 0; j < int(cnt); ++j) {
          if (j > 0 || sub > 0) {
            if (wa) e += seg_delta(spa, swa, wa, j);
            if (wb) e += seg_delta(spb, swb, wb, j);
          }
          const int64_t bin = carry + e;
          if (bin < -kBinMax || bin > kBinMax) bad |= ST_RANGE;
        }
      }
    }
    latch(p.res, bad);
    mx = block_max(mx, g.spb);
    const uint32_t w = bitlen32(mx);
    uint32_t tw_z;
    const uint32_t off_z = wg_scan(w, tw_z, s_tmp);
    if (tid < 64) {
      const uint64_t bz = lookback(p.s.st_out, tile, tw_z, p.epoch);
      if (tid == 0) s_base_z = bz;
    }
    __syncthreads();  // also: every thread is done reading s_a
    const uint64_t base_z = s_base_z;
    if (w > 0) pack32(&s_a[off_z], mag, w);
    __syncthreads();
    uint32_t* Pz = reinterpret_cast<uint32_t*>(p.out + g.off_p) + base_z;
    for (uint32_t k = tid; k < tw_z; k += kThreads) Pz[k] = bswap32(s_a[k]);
    if (active) {
      if (sub == 0) {
        p.out[g.off_w + blk] = uint8_t(w);
        reinterpret_cast<int32_t*>(p.out + g.off_o)[blk] = int32_t(oz);
      }
      reinterpret_cast<uint32_t*>(p.out + g.off_s)[seg] = bswap32(sgn);
    }
    if (tid == 0 && tile == g.ntiles - 1) {
      const uint64_t payload = 4 * (base_z + tw_z);
      write_header(p.out, g, payload);
      p.res->out_bytes = g.off_p + payload;
    }
    __syncthreads();
  }
}

struct MulParams {
  const uint8_t* c;
  uint64_t c_bytes;
  uint8_t* out;
  uint64_t out_cap;
  MulScalar k;
  Scratch s;
  uint32_t epoch;
  hoszp_result* res;
};

// floor(s q + 1/2) exactly, with s = m 2^-sh.
__device__ __forceinline__ int32_t scaled_bin(int64_t q, const MulScalar& k, uint32_t& bad) {
  if (k.big) {
    if (q != 0) bad |= ST_RANGE;
    return 0;
  }
  const __int128 prod = __int128(k.m) * __int128(q);
  const __int128 r = (prod + (__int128(1) << (k.sh - 1))) >> k.sh;
  if (r < -__int128(kBinMax) || r > __int128(kBinMax)) {
    bad |= ST_RANGE;
    return 0;
  }
  return int32_t(r);
}

__global__ void __launch_bounds__(kThreads) k_mul(MulParams p) {
  __shared__ uint32_t s_pay[kTileWords + 2];
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint64_t s_ticket, s_base, s_base_z;
  const int tid = threadIdx.x;
  Layout g;
  uint32_t err = read_header(p.c, p.c_bytes, g);
  if (!err && p.out_cap < bound_bytes(g.n, g.L)) err = ST_CAPACITY;
  if (err) {
    if (tid == 0) latch(p.res, err);
    return;
  }
  const uint64_t payload_words = g.payload_bytes / 4;
  const uint32_t* P = reinterpret_cast<const uint32_t*>(p.c + g.off_p);
  const uint32_t* S = reinterpret_cast<const uint32_t*>(p.c + g.off_s);
  const int32_t* O = reinterpret_cast<const int32_t*>(p.c + g.off_o);
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&p.s.ctrl[0], 1u);
    __syncthreads();
    const uint64_t tile = uni64(s_ticket);
    if (tile >= g.ntiles) break;
    const uint64_t seg = tile * kTileSegs + tid;
    const bool active = seg < g.nseg;
    const uint64_t blk = seg / g.spb;
    const uint32_t sub = uint32_t(seg % g.spb);
    uint64_t blen = 0;
    const uint32_t cnt = active ? seg_count(g, blk, sub, blen) : 0u;
    uint32_t bad = 0;
    uint32_t w = active ? p.c[g.off_w + blk] : 0u;
    if (w > 32) {
      bad |= ST_FORMAT;
      w = 0;
    }
    uint32_t tile_words;
    const uint32_t off = wg_scan(w, tile_words, s_tmp);
    if (tid < 64) {
      const uint64_t base = lookback(p.s.st_a, tile, tile_words, p.epoch);
      if (tid == 0) s_base = base;
    }
    __syncthreads();
    const uint64_t base = s_base;
    if (!stage_payload(s_pay, P, base, tile_words, payload_words)) bad |= ST_FORMAT;
    if (tid == 0 && tile == g.ntiles - 1 && base + tile_words != payload_words) bad |= ST_FORMAT;
    __syncthreads();

    // inverse BF + inverse LZ: bins of the segment
    const int32_t outlier = active ? O[blk] : 0;
    int64_t e_of[32];
    int64_t D = 0;
    {
      int64_t E = 0;
      uint64_t E2 = 0;
      unsigned __int128 E2w = 0;
      if (cnt > 0 && w > 0) {
        const uint32_t sw = bswap32(S[seg]);
        D = decode_segment<true, false>(&s_pay[1 + off], sw, w, sub, cnt, E, E2, E2w, e_of);
      } else {
#pragma unroll
        for (int j = 0; j < 32; ++j) e_of[j] = 0;
      }
    }
    const int64_t carry = int64_t(outlier) + block_excl(D, g.spb);
    const bool check = cnt > 0 && !bins_surely_in_range(outlier, blen, w);
    // scaled bins, then Lorenzo deltas of the result
    int32_t r[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const int64_t bin = carry + e_of[j];
      if (check && uint32_t(j) < cnt && (bin < -kBinMax || bin > kBinMax)) bad |= ST_FORMAT;
      r[j] = uint32_t(j) < cnt ? scaled_bin(bin, p.k, bad) : 0;
    }
    // last scaled bin of the previous segment of the same block (a segment
    // with valid slots after the first always follows a full segment)
    const int32_t prev = __shfl_up(r[31], 1, 64);
    uint32_t mag[32];
    uint32_t sgn = 0, mx = 0;
    int32_t outlier_z = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      bool neg = false;
      uint32_t m = 0;
      if (uint32_t(j) < cnt) {
        if (j == 0) {
          if (sub == 0) outlier_z = r[0];
          else m = delta_mag(r[0], prev, neg);
        } else {
          m = delta_mag(r[j], r[j - 1], neg);
        }
      }
      mag[j] = m;
      sgn |= uint32_t(neg) << (31 - j);
      mx = max(mx, m);
    }
    latch(p.res, bad);
    mx = block_max(mx, g.spb);
    const uint32_t wz = bitlen32(mx);
    uint32_t tw_z;
    const uint32_t off_z = wg_scan(wz, tw_z, s_tmp);
    if (tid < 64) {
      const uint64_t bz = lookback(p.s.st_out, tile, tw_z, p.epoch);
      if (tid == 0) s_base_z = bz;
    }
    __syncthreads();
    const uint64_t base_z = s_base_z;
    if (wz > 0) pack32(&s_pay[off_z], mag, wz);
    __syncthreads();
    uint32_t* Pz = reinterpret_cast<uint32_t*>(p.out + g.off_p) + base_z;
    for (uint32_t k = tid; k < tw_z; k += kThreads) Pz[k] = bswap32(s_pay[k]);
    if (active) {
      if (sub == 0) {
        p.out[g.off_w + blk] = uint8_t(wz);
        reinterpret_cast<int32_t*>(p.out + g.off_o)[blk] = outlier_z;
      }
      reinterpret_cast<uint32_t*>(p.out + g.off_s)[seg] = bswap32(sgn);
    }
    if (tid == 0 && tile == g.ntiles - 1) {
      const uint64_t payload = 4 * (base_z + tw_z);
      write_header(p.out, g, payload);
      p.res->out_bytes = g.off_p + payload;
    }
    __syncthreads();
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
    } else {
      r = make_float4(float(double(a.x) * s), float(double(a.y) * s), float(double(a.z) * s),
                      float(double(a.w) * s));
    }
    o4[k] = r;
  }
  for (uint64_t i = 4 * n4 + gt; i < n; i += stride) {
    const float a = x[i];
    out[i] = op == 0 ? -a : (op == 1 ? a + y[i] : float(double(a) * s));
  }
}

// Sum of x (pass 0) or of (x - mean)^2 (pass 1) in float64; per-workgroup
// partials in fixed order, the last workgroup adds them up in order.
__global__ void __launch_bounds__(kThreads) k_f32_sum(const float* x, uint64_t n, int pass,
                                                      double* part, uint32_t* ctrl,
                                                      hoszp_result* res) {
  __shared__ double s_red[kThreads];
  const uint64_t stride = uint64_t(gridDim.x) * kThreads;
  const uint64_t gt = uint64_t(blockIdx.x) * kThreads + threadIdx.x;
  const double mean = pass ? part[gridDim.x] : 0.0;
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
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_red[0];
    __threadfence();
    const uint32_t done = atomicAdd(&ctrl[1], 1u);
    if (done == gridDim.x - 1) {
      __threadfence();
      double t = 0.0;
      for (uint32_t b = 0; b < gridDim.x; ++b)
        t += __hip_atomic_load(&part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double v = t / double(n);
      if (pass == 0) part[gridDim.x] = v;  // mean, read by pass 1
      res->value = v;
      ctrl[1] = 0;
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_init(const Scratch& s, hoszp_result* res, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, s.ctrl, s.acc, res);
  return hipGetLastError();
}

hipError_t launch_compress(const Scratch& s, const Grids& gr, const float* x, const Layout& g,
                           double inv2e, uint8_t* out, uint32_t epoch, hoszp_result* res,
                           hipStream_t st) {
  CompressParams p{x, out, g, g.eb, inv2e, s, epoch, res};
  const uint64_t grid = g.ntiles < uint64_t(gr.compress) ? g.ntiles : uint64_t(gr.compress);
  switch (g.L) {
    case 32: hipLaunchKernelGGL(k_compress<1>, dim3(uint32_t(grid)), dim3(kThreads), 0, st, p); break;
    case 64: hipLaunchKernelGGL(k_compress<2>, dim3(uint32_t(grid)), dim3(kThreads), 0, st, p); break;
    case 128: hipLaunchKernelGGL(k_compress<4>, dim3(uint32_t(grid)), dim3(kThreads), 0, st, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_decompress(const Scratch& s, const Grids& gr, const uint8_t* c,
                             uint64_t c_bytes, float* x, uint64_t n_cap, uint32_t epoch,
                             hoszp_result* res, hipStream_t st) {
  DecodeParams p{c, c_bytes, x, n_cap, s, epoch, res};
  hipLaunchKernelGGL(k_decode<kDecompress>, dim3(gr.decode), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_reduce(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                         bool variance, uint32_t epoch, hoszp_result* res, hipStream_t st) {
  DecodeParams p{c, c_bytes, nullptr, 0, s, epoch, res};
  if (variance)
    hipLaunchKernelGGL(k_decode<kVariance>, dim3(gr.decode), dim3(kThreads), 0, st, p);
  else
    hipLaunchKernelGGL(k_decode<kMean>, dim3(gr.decode), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_negate(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                         uint8_t* out, uint64_t out_cap, hoszp_result* res, hipStream_t st) {
  NegateParams p{c, c_bytes, out, out_cap, s, res};
  hipLaunchKernelGGL(k_negate, dim3(gr.negate), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_add(const Scratch& s, const Grids& gr, const uint8_t* a, uint64_t a_bytes,
                      const uint8_t* b, uint64_t b_bytes, uint8_t* out, uint64_t out_cap,
                      uint32_t epoch, hoszp_result* res, hipStream_t st) {
  AddParams p{a, a_bytes, b, b_bytes, out, out_cap, s, epoch, res};
  hipLaunchKernelGGL(k_add, dim3(gr.add), dim3(kThreads), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_mul(const Scratch& s, const Grids& gr, const uint8_t* c, uint64_t c_bytes,
                      MulScalar k, uint8_t* out, uint64_t out_cap, uint32_t epoch,
                      hoszp_result* res, hipStream_t st) {
  MulParams p{c, c_bytes, out, out_cap, k, s, epoch, res};
  hipLaunchKernelGGL(k_mul, dim3(gr.mul), dim3(kThreads), 0, st, p);
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
  hipLaunchKernelGGL(k_f32_sum, dim3(grid), dim3(kThreads), 0, st, x, n, 0, s.part, s.ctrl, res);
  if (variance)
    hipLaunchKernelGGL(k_f32_sum, dim3(grid), dim3(kThreads), 0, st, x, n, 1, s.part, s.ctrl, res);
  return hipGetLastError();
}

hipError_t query_grids(Grids& gr, int num_cus) {
  int c = 0, d = 0, a = 0, m = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_compress<1>, kThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&d, k_decode<kVariance>, kThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_add, kThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, k_mul, kThreads, 0);
  if (e != hipSuccess) return e;
  auto clampg = [&](int occ) { return num_cus * (occ < 1 ? 1 : occ); };
  gr.compress = clampg(c);
  gr.decode = clampg(d);
  gr.add = clampg(a);
  gr.mul = clampg(m);
  gr.negate = num_cus * 8;
  gr.f32 = num_cus * 4;
  return hipSuccess;
}

}  // namespace hz
