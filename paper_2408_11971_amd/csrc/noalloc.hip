// noalloc.hip -- compression through a fixed, file-scope device scratch array,
// for callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// hoszp_compress_noalloc runs the same kernels as hoszp_compress_async.  The
// scratch those kernels need (tile ticket, finished-workgroup counter, status
// bits, the output-size accumulator and one look-back status word per
// encoder tile) lives in `scratch` below instead of a context.  Host code
// never passes `scratch` itself to a kernel (on the host that name is a
// stand-in, not a device address): once per device, at that device's first
// call, its device address is looked up with hipGetSymbolAddress and kept,
// and the kernels get that address.  Each device holds its own copy of the
// array until the process ends.

#include <math.h>

#include <mutex>

#include "hoszp_internal.h"

namespace {

// Look-back status words: one per compress tile (32 slots per segment, tiles
// of kCompressTileSegs segments, or kSmallTileSegs for fields of at most one
// small tile per compute unit); n <= 2^28 gives at most 2^23 / kCompressTileSegs
// + 1 tiles (a partial last block adds at most 8 segments).
constexpr uint64_t kLbWords = (uint64_t(1) << 23) / hz::kCompressTileSegs + 8;
constexpr uint64_t kCtrlWords = 64;  // ctrl (32 x u32) and acc (32 x u64), 256 B each
constexpr uint64_t kScratchWords = kCtrlWords + kLbWords;

__device__ __align__(256) uint64_t scratch[kScratchWords];

__global__ void k_noalloc_clear(uint64_t* p, uint64_t n) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

constexpr int kMaxDevices = 64;

struct DeviceState {
  std::once_flag once;
  int rc = HOSZP_ERR_DEVICE;
  uint64_t* ptr = nullptr;  // device address of this device's `scratch`
  hz::Grids grids{};
};

DeviceState g_dev[kMaxDevices];

// Set-up of one device (runs once, with that device current): look up the
// array's device address and size the persistent grid.  Nothing is
// launched or synchronized here, so a first call under capture still works.
void setup(int device, DeviceState& d) {
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    d.rc = HOSZP_ERR_DEVICE;
    return;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hz::query_grids(d.grids, cus) != hipSuccess) {
    (void)hipGetLastError();
    d.rc = HOSZP_ERR_DEVICE;
    return;
  }
  d.ptr = static_cast<uint64_t*>(p);
  d.rc = HOSZP_OK;
}

hz::Scratch scratch_of(uint64_t* p) {
  hz::Scratch s{};
  s.ctrl = reinterpret_cast<uint32_t*>(p);
  s.acc = p + 32;
  s.st_out = p + kCtrlWords;
  s.max_tiles = uint32_t(kLbWords);
  s.wait_limit = hz::kDefaultWaitLimit;
  return s;
}

}  // namespace

extern "C" int hoszp_compress_noalloc(const float* d_x, uint64_t n, double eb, uint32_t block,
                                      void* d_out, size_t out_cap, hoszp_result* d_res,
                                      void* stream) {
  if (!d_x || !d_out || !d_res || (reinterpret_cast<uintptr_t>(d_x) & 15u) ||
      (reinterpret_cast<uintptr_t>(d_out) & 15u) || (reinterpret_cast<uintptr_t>(d_res) & 7u))
    return HOSZP_ERR_ARG;
  if (n == 0 || !hz::block_ok(block) || !(eb > 0.0) || !isfinite(eb)) return HOSZP_ERR_ARG;
  if (n > HOSZP_NOALLOC_MAX_N) return HOSZP_ERR_LIMIT;
  if (out_cap < hz::bound_bytes(n, block)) return HOSZP_ERR_CAPACITY;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices)
    return HOSZP_ERR_DEVICE;
  DeviceState& d = g_dev[device];
  std::call_once(d.once, setup, device, std::ref(d));
  if (d.rc != HOSZP_OK) return d.rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hz::Scratch s = scratch_of(d.ptr);
  hz::Layout g;
  hz::place(g, n, block, eb);
  // Every call starts from zeroed counters and look-back status words (the
  // array keeps the previous call's contents), cleared by a kernel on the
  // caller's stream: no memset node, and a captured graph clears them again
  // on every replay, so the look-back never sees a previous call's prefixes
  // (the kernel's generation counter restarts at 1 with them).
  const uint32_t nt = hz::compress_tile_segs(g.nseg, d.grids.cus);
  const uint64_t tiles = (g.nseg + nt - 1) / nt;
  if (tiles > kLbWords) return HOSZP_ERR_LIMIT;  // (only on a GPU with over 8000 CUs)
  hipLaunchKernelGGL(k_noalloc_clear, dim3(8), dim3(256), 0, st, d.ptr, kCtrlWords + tiles);
  if (hipGetLastError() != hipSuccess) return HOSZP_ERR_DEVICE;
  const double inv2e = 1.0 / (2.0 * eb);
  if (hz::launch_compress(s, d.grids, d_x, g, inv2e, static_cast<uint8_t*>(d_out), d_res, st) !=
      hipSuccess) {
    (void)hipGetLastError();
    (void)hz::launch_reset(s, d_res, st);
    return HOSZP_ERR_DEVICE;
  }
  return HOSZP_OK;
}
